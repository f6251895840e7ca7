"""Sensitivity of the fit to Z contributions (Results, the Z null tests and the fits with Z at
a few percent): pseudo-data drawn from the ten K* alone and fitted with the ten K* + Z(4430) +
Z(4240) model must give Z fit fractions (Eq. 13) near zero; pseudo-data with both Z at fit
fractions of 3.5% and 1.2% must give them back.  Events come from the library's accept-reject
generator; fits are the FP32-adjoint MIGRAD followed by an FP64-adjoint polish with HESSE, Z
masses and widths fixed.  3e5 data and 6e5 normalisation events."""
import math

import numpy as np
import pytest

from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W

K = W.KIN
pytestmark = pytest.mark.gpu
N_DATA, N_NORM = 300_000, 600_000


@pytest.fixture(scope="module")
def setup():
    res = W.model("full2z")
    iz = [i for i, r in enumerate(res) if r.chain == 1]
    zoff = [W.coupling_offset(res, i) for i in iz]
    gen = kpsi.Engine(0, "fp64")
    gen.set_model(K, res)
    mc = gen.generate_phsp(5201, N_NORM, W.PHSP_WMAX)
    gen.load(kpsi.NORM, mc)
    scan = gen.generate_phsp(5202, 300_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    yield res, iz, zoff, gen, mc
    gen.close()


def _fit(res, data, mc, start, mask):
    x = start
    r = None
    for prec in ("fp32", "fp64"):
        e = kpsi.Engine(0, prec)
        e.set_model(K, res)
        e.load(kpsi.DATA, data)
        e.load(kpsi.NORM, mc)
        x, _, r = e.migrad(x, mask, gradient=1)
        e.close()
    return x, r


def _run(setup, point, seed):
    import torch
    res, iz, zoff, gen, mc = setup
    smax = 1.5 * float(gen.density(kpsi.DATA, point).max())
    data, _, nover = gen.generate_model(point, seed, N_DATA, W.PHSP_WMAX, smax)
    torch.cuda.synchronize()
    assert nover == 0
    ff_gen, _ = gen.fit_fractions(point)
    start = point.copy()
    for o in zoff:   # the Z couplings start small but non-zero
        start[o] = max(start[o], 0.05)
        start[o + 2] = max(start[o + 2], 0.05)
    x, r = _fit(res, data, mc, start, W.free_mask(res))
    ff, _ = gen.fit_fractions(x)
    kdiff = float(np.max(np.abs(np.delete(ff - ff_gen, iz))))
    print(f"[zsens] generated Z fractions {[f'{ff_gen[i]:.5f}' for i in iz]}, fitted {[f'{ff[i]:.5f}' for i in iz]}, "
          f"largest K* fraction change {kdiff:.4f}, fit status {r.status} edm {r.edm:.2g}", flush=True)
    return ff_gen, ff, kdiff, r


def test_kstar_only_data_gives_z_fractions_near_zero(setup):
    res, iz, zoff, gen, mc = setup
    null = W.params(res, 31)
    for o in zoff:
        null[o] = 0.0
        null[o + 2] = 0.0
    ff_gen, ff, kdiff, r = _run(setup, null, 5300)
    assert all(ff_gen[i] == 0.0 for i in iz)
    # the paper's null fits give 0.01% and below; 1e-3 is a third of the smaller positive case
    assert all(ff[i] < 1e-3 for i in iz), ff
    assert kdiff < 0.01
    # a Z coupling that fits to near zero leaves its phase flat: HESSE may then report status 3
    assert r.status in (0, 3) and r.edm < 1e-3, r.as_dict()


def test_data_with_z_at_a_few_percent_gives_them_back(setup):
    res, iz, zoff, gen, mc = setup
    truth = W.params(res, 31)
    target = {iz[0]: 0.035, iz[1]: 0.012}
    for _ in range(4):   # scale each Z's couplings to its target fraction
        ff0, _ = gen.fit_fractions(truth)
        for i, o in zip(iz, zoff):
            f = math.sqrt(target[i] / ff0[i])
            truth[o] *= f
            truth[o + 2] *= f
    ff_gen, ff, kdiff, r = _run(setup, truth, 5301)
    for i in iz:
        assert abs(ff_gen[i] - target[i]) < 2e-4
        assert abs(ff[i] - ff_gen[i]) < 0.25 * ff_gen[i], (i, ff[i], ff_gen[i])
    assert kdiff < 0.01
    assert r.status == 0, r.as_dict()

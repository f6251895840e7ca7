"""Z helicity couplings free of the parity relation (hel_free), through the C ABI, against the
FP64 oracle.

The Discussion states that the Z part can be fitted with its couplings unconstrained; with
hel_free the one Z of the model carries H'_0, H'_{+1} and H'_{-1} as independent couplings
instead of H'_{-1} = H'_{+1} (Eq. 11 for a 1+ state).  Checked here:

* per-event densities, the NLL and its gradient (every coupling, and the floating masses and
  widths of K*(1410) and the Z) at H'_{-1} != H'_{+1}, at sizes spanning several blocks with
  ragged tails, on both precisions, at the parity bars of the other tests;
* at H'_{-1} = H'_{+1} the free model is the constrained one: the same NLL, and the constrained
  gradient of H'_{+1} is the sum of the free gradients of H'_{+1} and H'_{-1} (magnitude and
  phase, by the chain rule);
* the normalisation served by the interference matrix (three Z components), with the lineshape
  derivative columns of the floating Z, and the fit fractions of Eq. 13 from it;
* the free model inside the Eq. 14 mixture, and with flavour tags (direct, and with both
  flavours' normalisations from the +phi interference matrix, which exchanges H'_{+1} and
  H'_{-1} for the -phi record);
* the accept-reject generator draws the oracle's sample from the free model;
* models the free helicities do not cover are refused.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W
from parity_bars import check_grad, check_nll

K = W.KIN
pytestmark = pytest.mark.gpu
FLOAT = ("K*(1410)", "Z(4430)")


def _sets(nd, nm, seed):
    data = W.neutral_events(nd, seed, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, seed + 1, nm, W.PHSP_WMAX)
    return data, mc


def _engine(prec, res, data, mc):
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    e.set_floating([1 if r.name in FLOAT else 0 for r in res])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    return e


def _z_offset(res):
    return W.coupling_offset(res, len(res) - 1)


@pytest.mark.parametrize("prec,tg", [("fp64", 1e-9), ("fp32", None)])
def test_free_helicity_likelihood_and_gradient_match_oracle(prec, tg):
    print(f"[case] free Z helicities {prec}: 8191 data / 24593 normalisation events", flush=True)
    res = W.model("full_zfree")
    data, mc = _sets(8191, 24593, 301)
    par = W.params(res, seed=303) + 0.04 * W.free_mask(res, FLOAT)
    z = _z_offset(res)
    assert W.n_params(res) == W.n_params(W.model("full")) + 2
    assert abs(par[z + 2] - par[z + 4]) > 0.05           # H'_{+1} and H'_{-1} differ
    e = _engine(prec, res, data, mc)
    assert e.n_params == W.n_params(res)
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    v, g = e.nll_and_grad(par)
    st, ref, gref = O.nll(K, res, par, data, mc, dirs=dirs)
    assert st == 0
    check_nll(v, ref, prec, data.shape[1], "free Z")
    check_grad(g[dirs], gref, prec, "free Z", norm=tg)
    check_nll(e.nll(par), ref, prec, data.shape[1], "free Z nll-only")
    # the three Z couplings' gradient entries, on their own
    zk = np.searchsorted(dirs, np.arange(z, z + 6))
    gz, gzr = g[dirs][zk], gref[zk]
    print(f"[parity] free Z {prec} Z-coupling gradient {gz} oracle {gzr}", flush=True)
    np.testing.assert_allclose(gz, gzr, rtol=1e-7 if prec == "fp64" else 2e-3,
                               atol=(1e-9 if prec == "fp64" else 1e-6) * np.max(np.abs(gref)))
    s = e.density(kpsi.NORM, par)[:4000]
    o = O.density(K, res, par, mc[:, :4000])
    rtol = 1e-11 if prec == "fp64" else 2e-5
    np.testing.assert_allclose(s, o, rtol=rtol, atol=rtol * 0.1 * o.max())
    e.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_helicities_at_the_parity_relation_are_the_constrained_model(prec):
    res_c, res_f = W.model("full"), W.model("full_zfree")
    data, mc = _sets(4099, 12007, 311)
    pc = W.params(res_c, seed=313)
    z = _z_offset(res_c)
    nc = sum(2 * r.n_coup for r in res_c)
    pf = np.concatenate([pc[: z + 4], pc[z + 2: z + 4], pc[nc:]])   # H'_{-1} = H'_{+1}
    ec, ef = _engine(prec, res_c, data, mc), _engine(prec, res_f, data, mc)
    vc, gc = ec.nll_and_grad(pc)
    vf, gf = ef.nll_and_grad(pf)
    tol = 1e-12 if prec == "fp64" else 1e-6
    print(f"[zfree] {prec} constrained {vc:.12g} free {vf:.12g}", flush=True)
    assert abs(vf - vc) <= tol * max(abs(vc), 2.0 * data.shape[1])
    # d/dH'_{+1} of the constrained model = d/dH'_{+1} + d/dH'_{-1} of the free one
    comb = gf[z + 2: z + 4] + gf[z + 4: z + 6]
    scale = np.max(np.abs(gc[np.isfinite(gc)]))
    gtol = 1e-9 if prec == "fp64" else 2e-6
    print(f"[zfree] {prec} H'+1 gradient constrained {gc[z + 2: z + 4]} free sum {comb}", flush=True)
    np.testing.assert_allclose(comb, gc[z + 2: z + 4], atol=gtol * scale)
    np.testing.assert_allclose(gf[: z + 2], gc[: z + 2], atol=gtol * scale)
    np.testing.assert_allclose(gf[z + 6:][np.isfinite(gc[nc:])], gc[nc:][np.isfinite(gc[nc:])], atol=gtol * scale)
    ec.close()
    ef.close()


def test_model_generator_with_free_helicities_agrees_with_oracle():
    res = W.model("full_zfree")
    e = kpsi.Engine(0, "fp64")
    e.set_model(K, res)
    par = W.params(res, seed=17)
    coef = W.acceptance_coefficients()
    ev, npr, nov = e.generate_model(par, 779, 3000, W.PHSP_WMAX, 400.0, coef)
    ref, npr_o, nov_o = O.gen_model(K, res, par, 779, 3000, W.PHSP_WMAX, 400.0, coef)
    ev = ev.cpu().numpy()
    assert npr == npr_o
    assert np.all(ev == ref, axis=0).mean() > 0.999
    e.close()


def test_models_without_free_helicity_support_are_refused():
    res = W.model("full_zfree")
    e = kpsi.Engine(0, "fp64")
    e.set_model(K, res)
    data, mc = _sets(500, 2000, 321)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    par = W.params(res, seed=5)
    # two Z with one free, and a free K*, are rejected by set_model
    z2 = dataclasses.replace(W.Z4240)
    with pytest.raises(kpsi.KpsiError):
        e.set_model(K, res + [z2])
    bad = [dataclasses.replace(W.KSTAR892, hel_free=True)]
    with pytest.raises(kpsi.KpsiError):
        e.set_model(K, bad)
    assert np.isfinite(e.nll(par))          # the context keeps its model
    e.close()


@pytest.mark.parametrize("prec,tg", [("fp64", 1e-9), ("fp32", None)])
def test_free_helicity_normalisation_from_the_interference_matrix(prec, tg):
    res = W.model("full_zfree")
    data, mc = _sets(4099, 12007, 331)
    e = _engine(prec, res, data, mc)
    e.set_norm_cache(1)
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    par = W.params(res, seed=333) + 0.03 * W.free_mask(res, FLOAT)
    z = _z_offset(res)
    p2 = par.copy()
    p2[z + 4] += 0.09          # H'_{-1} magnitude and phase: couplings only, served by the matrix
    p2[z + 5] -= 0.2
    for k, p in enumerate((par, p2)):
        st, ref, gref = O.nll(K, res, p, data, mc, dirs=dirs)
        assert st == 0
        v, g = e.nll_and_grad(p)
        check_nll(v, ref, prec, data.shape[1], f"free Z cached {k}")
        check_grad(g[dirs], gref, prec, f"free Z cached {k}", norm=tg)
        check_nll(e.nll(p), ref, prec, data.shape[1], f"free Z cached nll-only {k}")
    b, h, _ = e.norm_cache_stats()
    assert b == 1 and h >= 2
    e.close()


@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-9), ("fp32", 2e-5)])
def test_free_helicity_fit_fractions_match_oracle(prec, rtol):
    res = W.model("full_zfree")
    mc = O.gen_phsp(K, 341, 20011, W.PHSP_WMAX)
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    e.load(kpsi.NORM, mc)
    par = W.params(res, seed=343)
    ff, tot = e.fit_fractions(par)
    st, ref = O.fit_fractions(K, res, par, mc)
    assert st == 0
    print(f"[zfree] {prec} fit fractions Z {ff[-1]:.6f} oracle {ref[-1]:.6f}, sum {tot:.6f}", flush=True)
    np.testing.assert_allclose(ff, ref, rtol=rtol, atol=rtol * 1e-3)
    assert tot == pytest.approx(ref.sum(), rel=rtol)
    e.close()


@pytest.mark.parametrize("prec,tg", [("fp64", 1e-9), ("fp32", None)])
def test_free_helicities_with_the_background_mixture(prec, tg):
    """Free Z helicities inside the Eq. 14 mixture (per-event efficiency and background)."""
    res = W.model("full_zfree")
    data, mc = _sets(4099, 12007, 351)
    rng = np.random.default_rng(352)
    eps_d = O.acceptance(W.acceptance_coefficients(), W.M_LO, W.M_HI, data)
    eps_m = O.acceptance(W.acceptance_coefficients(), W.M_LO, W.M_HI, mc)
    b_d, b_m = rng.uniform(0.2, 1.5, data.shape[1]), rng.uniform(0.2, 1.5, mc.shape[1])
    e = _engine(prec, res, data, mc)
    e.set_efficiency_values(eps_m)
    e.set_background(0.8, eps_d, b_d, b_m)
    par = W.params(res, seed=353) + 0.03 * W.free_mask(res, FLOAT)
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    st, ref, gref = O.nll_mix(K, res, par, data, mc, b_d, b_m, 0.8, eps_d, eps_m, dirs)
    assert st == 0
    v, g = e.nll_and_grad(par)
    check_nll(v, ref, prec, data.shape[1], "free Z mixture")
    check_grad(g[dirs], gref, prec, "free Z mixture", norm=tg)
    e.close()


@pytest.mark.parametrize("prec,w,cached,tg", [("fp64", 0.06, False, 1e-9), ("fp32", 0.06, False, None),
                                              ("fp64", 0.04, True, 1e-9), ("fp32", 0.04, True, None)])
def test_free_helicities_with_flavour_tags(prec, w, cached, tg):
    res = W.model("full_zfree")
    data, mc = _sets(4099, 12007, 361)
    eps_m = O.acceptance(W.acceptance_coefficients(), W.M_LO, W.M_HI, mc)
    tag = np.where(np.random.default_rng(362).random(data.shape[1]) < 0.45, 1.0, -1.0)
    e = _engine(prec, res, data, mc)
    e.set_efficiency_values(eps_m)
    e.set_flavour(tag, w)
    if cached:
        e.set_norm_cache(1)
    par = W.params(res, seed=363) + 0.03 * W.free_mask(res, FLOAT)
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    z = _z_offset(res)
    pts = [par]
    if cached:
        p2 = par.copy()
        p2[z + 4] += 0.08    # H'_{-1}: a couplings-only change, served by the matrix
        p2[z + 3] -= 0.15
        pts.append(p2)
    for k, p in enumerate(pts):
        st, ref, gref = O.nll_cc(K, res, p, data, tag, mc, w, eps_m, dirs)
        assert st == 0
        v, g = e.nll_and_grad(p)
        label = f"free Z tags w={w}{' cached' if cached else ''} {k}"
        check_nll(v, ref, prec, data.shape[1], label)
        check_grad(g[dirs], gref, prec, label, norm=tg)
        check_nll(e.nll(p), ref, prec, data.shape[1], label + " nll-only")
    if cached:
        b, h, _ = e.norm_cache_stats()
        assert b == 1 and h >= 2
    e.close()

"""Entry paths the benchmark and the learned-efficiency workload use, against the FP64 oracle:

* events loaded as borrowed device arrays (kpsi_load_events_device, what the benchmark's
  GPU-generated torch tensors go through) give the same NLL and gradient, bit for bit, as the
  same events loaded from host arrays, and match the oracle;
* the likelihood with the efficiency of a trained network (kpsi_set_efficiency_mlp, Eq. 14 with
  a learned acceptance) matches the oracle's likelihood evaluated with the network's
  probabilities: exactly the device's probabilities at the ordinary bars, and the oracle's own
  FP64 network within the bound its probability differences allow.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W
from parity_bars import check_grad, check_nll, check_probabilities

K = W.KIN
pytestmark = pytest.mark.gpu
FLOAT = ("K*(1410)", "Z(4430)")


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _engine(prec, res, data, mc):
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    e.set_floating([1 if r.name in FLOAT else 0 for r in res])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    return e


@pytest.mark.parametrize("prec,tg", [("fp64", 1e-9), ("fp32", None)])
def test_device_loaded_events_match_host_loaded_and_oracle(prec, tg):
    import torch
    res = W.model("full")
    data = W.neutral_events(8191, 61, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, 62, 24593, W.PHSP_WMAX)
    par = W.params(res, seed=63) + 0.04 * W.free_mask(res, FLOAT)
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    host = _engine(prec, res, data, mc)
    dd, dm = _cuda(data), _cuda(mc)
    dev = _engine(prec, res, dd, dm)              # borrowed device pointers
    assert dev.n == [data.shape[1], mc.shape[1]]
    v0, g0 = host.nll_and_grad(par)
    v1, g1 = dev.nll_and_grad(par)
    torch.cuda.synchronize()
    assert v1 == v0 and np.array_equal(g1[dirs], g0[dirs])
    assert dev.nll(par) == host.nll(par)
    st, ref, gref = O.nll(K, res, par, data, mc, dirs=dirs)
    assert st == 0
    check_nll(v1, ref, prec, data.shape[1], "device-loaded")
    check_grad(g1[dirs], gref, prec, "device-loaded", norm=tg)
    # densities of the borrowed normalisation set, element by element
    s = dev.density(kpsi.NORM, par)[:3000]
    o = O.density(K, res, par, mc[:, :3000])
    rtol = 1e-11 if prec == "fp64" else 2e-5
    np.testing.assert_allclose(s, o, rtol=rtol, atol=rtol * 0.1 * o.max())
    host.close()
    dev.close()
    del dd, dm


@pytest.fixture(scope="module")
def trained_network():
    """A network trained on the GPU for a few epochs on labelled phase-space events of the seeded
    analytic acceptance (30-90%)."""
    e = kpsi.Engine(0, "fp32")
    e.set_model(K, W.model("full"))
    coef = W.acceptance_coefficients()
    train = e.generate_phsp(701, 400_000, W.PHSP_WMAX)
    lab, _ = e.accept_labels(702, train, coef)
    par, loss = e.mlp_train(W.mlp_init(7), train, lab, epochs=4, batch=16384, lr=3e-3)
    assert math.isfinite(loss)
    e.close()
    return par


@pytest.mark.parametrize("prec,tg", [("fp64", 1e-9), ("fp32", None)])
def test_mlp_efficiency_likelihood_matches_oracle(trained_network, prec, tg):
    par_nn = trained_network
    res = W.model("full")
    data = W.neutral_events(10007, 71, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, 72, 40009, W.PHSP_WMAX)
    e = _engine(prec, res, data, mc)
    e.set_efficiency_mlp(par_nn)
    # the network's probabilities on the normalisation events: device kernel and FP64 reference
    eps_dev = e.mlp_eval(par_nn, _cuda(mc)).cpu().numpy()
    eps_ref = O.mlp(par_nn.astype(np.float64), O.mlp_inputs(W.M_LO, W.M_HI, mc))[1]
    check_probabilities(eps_dev, eps_ref, par_nn, O.mlp_inputs(W.M_LO, W.M_HI, mc))
    assert 0.25 < eps_dev.min() and eps_dev.max() < 0.95
    par = W.params(res, seed=73) + 0.04 * W.free_mask(res, FLOAT)
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    v, g = e.nll_and_grad(par)
    nd = data.shape[1]
    # (1) the composition: the likelihood with the device's own probabilities as efficiency
    st, ref, gref = O.nll(K, res, par, data, mc, eps=eps_dev, dirs=dirs)
    assert st == 0
    check_nll(v, ref, prec, nd, "network efficiency")
    check_grad(g[dirs], gref, prec, "network efficiency", norm=tg)
    check_nll(e.nll(par), ref, prec, nd, "network efficiency nll-only")
    # (2) against the oracle's own network: N = sum eps S / N_MC moves by at most the largest
    # relative probability difference, and the NLL by 2 N_d times that
    st, ref2, _ = O.nll(K, res, par, data, mc, eps=eps_ref)
    bound = 2.0 * nd * float(np.max(np.abs(eps_dev - eps_ref) / eps_ref))
    print(f"[parity] network efficiency vs FP64 network: |dNLL| {abs(v - ref2):.3e} bound {bound:.3e}", flush=True)
    assert abs(v - ref2) <= bound + 1e-6 * max(abs(ref2), 2.0 * nd)
    e.close()


def test_time_kernel_reports_a_duration_and_leaves_results_unchanged():
    res = W.model("full")
    data = W.neutral_events(20011, 81, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, 82, 60013, W.PHSP_WMAX)
    par = W.params(res, seed=83) + 0.04 * W.free_mask(res, FLOAT)
    e = _engine("fp32", res, data, mc)
    v0, g0 = e.nll_and_grad(par)
    for grad in (True, False):
        ms = e.time_kernel(par, grad=grad, reps=50)
        assert 0.0 < ms < 50.0
    v1, g1 = e.nll_and_grad(par)
    fin = np.isfinite(g0)
    assert v1 == v0 and np.array_equal(g1[fin], g0[fin])
    st, _ = e.nll_status(par)
    assert st == kpsi.KPSI_OK
    with pytest.raises(kpsi.KpsiError):
        e.time_kernel(par, reps=0)
    e.close()


def test_call_longer_than_the_result_poll_bound_returns_the_same_results():
    """A call whose device work outlasts the 50 ms bound on polling its results (here 4000
    back-to-back launches of the per-event work over 1.2e6 events, kpsi_time_kernel) falls back
    to a stream synchronisation and still returns; later calls give the same results."""
    import torch
    res = W.model("full")
    par = W.params(res, seed=84) + 0.04 * W.free_mask(res, FLOAT)
    g = kpsi.Engine(0, "fp64")
    g.set_model(K, res)
    mc = g.generate_phsp(85, 1_000_000, W.PHSP_WMAX)
    data = g.generate_phsp(86, 200_000, W.PHSP_WMAX)
    torch.cuda.synchronize()
    g.close()
    e = _engine("fp32", res, data, mc)
    v0, g0 = e.nll_and_grad(par)
    ms = e.time_kernel(par, grad=True, reps=4000)
    print(f"[paths] 4000 launches: {ms * 4000:.1f} ms of per-event work", flush=True)
    assert 0.0 < ms < 1.0
    v1, g1 = e.nll_and_grad(par)
    fin = np.isfinite(g0)
    assert v1 == v0 and np.array_equal(g1[fin], g0[fin])
    e.close()

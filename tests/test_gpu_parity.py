"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Inputs are seeded: data-like events from the neutral generator (K*(892)-peaked mass,
uniform angles, boundary cases), normalisation events from the oracle's phase-space
generator.  Sizes span several blocks and end in ragged tails.
Tolerances: FP64 path 1e-10 relative on the NLL, FP32 path 1e-6 (paper-independent
targets of the engine); per-event densities and Z-chain observables are compared
element by element.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W
from parity_bars import check_grad, check_nll

K = W.KIN
pytestmark = pytest.mark.gpu


def _engine(model, prec, floating=()):
    res = W.model(model)
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    if floating:
        e.set_floating([1 if r.name in floating else 0 for r in res])
    return e, res


def _sets(nd, nm, seed=5, edges=True):
    data = W.neutral_events(nd, seed, peaked=True, edges=edges)
    mc = O.gen_phsp(K, seed + 1000, nm, W.PHSP_WMAX)
    return data, mc


def _interior(ev):
    """Keep the Z-chain frame well defined (away from the exact mass end points)."""
    ev = ev.copy()
    ev[0] = np.clip(ev[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    return ev


@pytest.mark.parametrize("n", [1, 255, 257, 3001])
def test_invariants_match_oracle(n):
    e, res = _engine("full", "fp64")
    ev = _interior(W.neutral_events(n, 3, edges=True))
    e.load(kpsi.DATA, ev)
    g = e.invariants(kpsi.DATA)
    o = O.z_angles(K, ev)
    np.testing.assert_allclose(g[:, 0], o[:, 0], rtol=1e-13)
    np.testing.assert_allclose(g[:, 1], np.cos(o[:, 1]), atol=1e-11)
    np.testing.assert_allclose(g[:, 2], np.cos(o[:, 2]), atol=1e-12)
    # phi~ is undefined when theta_Z or theta~ is 0 or pi (its terms then vanish, or only
    # phi~ + alpha matters); compare the angles where they are defined
    ok = (np.sin(o[:, 1]) > 1e-6) & (np.sin(o[:, 2]) > 1e-6)
    d3 = np.angle(np.exp(1j * (g[:, 3] - o[:, 3])))
    np.testing.assert_allclose(d3[ok], 0.0, atol=1e-9)
    ok4 = np.sin(o[:, 2]) > 1e-6
    d4 = np.angle(np.exp(1j * (g[:, 4] - o[:, 4])))
    np.testing.assert_allclose(d4[ok4], 0.0, atol=1e-9)


@pytest.mark.parametrize("model", ["kstar892", "kstar10", "full", "full2z"])
def test_density_fp64(model):
    e, res = _engine(model, "fp64")
    par = W.params(res, seed=13)
    ev = W.neutral_events(2053, 7, peaked=True, edges=True)
    if model in ("full", "full2z"):
        ev = _interior(ev)
    e.load(kpsi.DATA, ev)
    s = e.density(kpsi.DATA, par)
    o = O.density(K, res, par, ev)
    np.testing.assert_allclose(s, o, rtol=1e-11, atol=1e-13 * o.max())


@pytest.mark.parametrize("model", ["kstar892", "full", "full2z"])
def test_density_fp32(model):
    e, res = _engine(model, "fp32")
    par = W.params(res, seed=13)
    ev = _interior(W.neutral_events(4099, 8, peaked=True, edges=True))
    e.load(kpsi.DATA, ev)
    s = e.density(kpsi.DATA, par)
    o = O.density(K, res, par, ev)
    np.testing.assert_allclose(s, o, rtol=2e-5, atol=2e-6 * o.max())


@pytest.mark.parametrize("model,prec,rtol", [("kstar892", "fp64", 1e-10), ("full", "fp64", 1e-10),
                                             ("full2z", "fp64", 1e-10), ("kstar892", "fp32", 1e-6),
                                             ("full", "fp32", 1e-6), ("full2z", "fp32", 1e-6)])
def test_nll_matches_oracle(model, prec, rtol):
    e, res = _engine(model, prec)
    par = W.params(res, seed=17)
    # the boundary events are kept except for the single P-wave model, where the
    # threshold event has S = 0 (checked separately below)
    data, mc = _sets(20_011, 60_013, edges=(model != "kstar892"))
    if model != "kstar892":
        data = _interior(data)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    st, ref, _ = O.nll(K, res, par, data, mc)
    assert st == 0
    got = e.nll(par)
    assert got == pytest.approx(ref, rel=rtol)


@pytest.mark.parametrize("model,prec,tol", [("kstar892", "fp64", 1e-9), ("full", "fp64", 1e-9),
                                            ("kstar892", "fp32", None), ("full", "fp32", None)])
def test_gradient_matches_oracle(model, prec, tol):
    floating = ("K*(1410)", "Z(4430)") if model == "full" else ("K*(892)",)
    e, res = _engine(model, prec, floating)
    par = W.params(res, seed=19)
    par = par + 0.1 * (np.arange(par.size) % 3 == 0)   # off the generation point
    data, mc = _sets(4003, 12007, seed=9, edges=(model != "kstar892"))
    if model != "kstar892":
        data = _interior(data)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    mask = W.free_mask(res, floating)
    dirs = np.flatnonzero(mask)
    st, ref_v, ref_g = O.nll(K, res, par, data, mc, dirs=dirs)
    v, g = e.nll_and_grad(par)
    check_nll(v, ref_v, prec, data.shape[1], f"{model} 4003+12007")
    check_grad(g[dirs], ref_g, prec, f"{model} 4003+12007", norm=tol)
    # lineshape entries that are not floating are reported as NaN
    nc = sum(2 * r.n_coup for r in res)
    fixed_ls = [nc + 2 * i + k for i, r in enumerate(res) if r.name not in floating for k in (0, 1)]
    assert np.all(np.isnan(g[fixed_ls]))


def test_gradient_fp64_matches_central_differences():
    e, res = _engine("full", "fp64", ("K*(1410)", "Z(4430)"))
    par = W.params(res, seed=23)
    data, mc = _sets(3001, 9001, seed=11)
    e.load(kpsi.DATA, _interior(data))
    e.load(kpsi.NORM, mc)
    v, g = e.nll_and_grad(par)
    dirs = np.flatnonzero(W.free_mask(res, ("K*(1410)", "Z(4430)")))
    for i in dirs[:: max(1, len(dirs) // 12)].tolist() + [int(dirs[-1]), int(dirs[-2]), int(dirs[-3])]:
        h = 1e-6 * max(1.0, abs(par[i]))
        pp, pm = par.copy(), par.copy()
        pp[i] += h
        pm[i] -= h
        fd = (e.nll(pp) - e.nll(pm)) / (2 * h)
        assert g[i] == pytest.approx(fd, abs=2e-6 * max(1.0, abs(g[i])) + 40 * 1e-16 * abs(v) / h)


def test_bitwise_reproducible():
    e, res = _engine("full", "fp32", ("K*(1410)", "Z(4430)"))
    par = W.params(res)
    data, mc = _sets(50_000, 100_000)
    e.load(kpsi.DATA, _interior(data))
    e.load(kpsi.NORM, mc)
    a = e.nll_and_grad(par)
    b = e.nll_and_grad(par)
    assert a[0] == b[0]
    assert np.array_equal(np.nan_to_num(a[1], nan=7.0), np.nan_to_num(b[1], nan=7.0))


def test_nonfinite_and_state_errors():
    e, res = _engine("kstar892", "fp64")
    par = W.params(res)
    st, _ = e.nll_status(par)
    assert st == kpsi.KPSI_E_STATE
    data, mc = _sets(1000, 3000)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    p0 = par.copy()
    p0[0:6:2] = 0.0
    st, v = e.nll_status(p0)
    assert st == kpsi.KPSI_E_NONFINITE and v == math.inf
    p1 = par.copy()
    p1[1] = float("nan")
    st, _ = e.nll_status(p1)
    assert st == kpsi.KPSI_E_ARG
    bad = data.copy()
    bad[0, 5] = W.M_HI + 0.01
    with pytest.raises(kpsi.KpsiError):
        e.load(kpsi.DATA, bad)


def test_efficiency_values_and_histogram():
    e, res = _engine("full", "fp64")
    par = W.params(res)
    data, mc = _sets(2000, 8000)
    data = _interior(data)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    coef = W.acceptance_coefficients()
    eps = O.acceptance(coef, W.M_LO, W.M_HI, mc)
    e.set_efficiency_values(eps)
    st, ref, _ = O.nll(K, res, par, data, mc, eps=eps)
    assert e.nll(par) == pytest.approx(ref, rel=1e-10)
    # histogram: bin values looked up on the device equal the nearest-bin lookup
    nb = (5, 4, 3, 6)
    rng = np.random.default_rng(1)
    table = rng.uniform(0.2, 1.0, size=nb).astype(np.float32)
    lo = np.array([W.M_LO, -1, -1, -math.pi])
    hi = np.array([W.M_HI, 1, 1, math.pi])
    e.set_efficiency_hist(table, lo, hi)
    idx = [np.clip(np.floor((mc[d] - lo[d]) / (hi[d] - lo[d]) * nb[d]).astype(int), 0, nb[d] - 1) for d in range(4)]
    eps_h = table[idx[0], idx[1], idx[2], idx[3]].astype(np.float64)
    st, ref2, _ = O.nll(K, res, par, data, mc, eps=eps_h)
    assert e.nll(par) == pytest.approx(ref2, rel=1e-10)


def test_phase_space_generator_bit_exact():
    e, res = _engine("kstar892", "fp64")
    ev = e.generate_phsp(4242, 50_000, W.PHSP_WMAX).cpu().numpy()
    ref = O.gen_phsp(K, 4242, 50_000, W.PHSP_WMAX)
    assert np.array_equal(ev, ref)


def test_model_generator_agrees_with_oracle():
    e, res = _engine("full", "fp64")
    par = W.params(res)
    n = 3000
    smax = 400.0
    coef = W.acceptance_coefficients()
    ev, npr, nov = e.generate_model(par, 777, n, W.PHSP_WMAX, smax, coef)
    ref, npr_o, nov_o = O.gen_model(K, res, par, 777, n, W.PHSP_WMAX, smax, coef)
    ev = ev.cpu().numpy()
    # same proposals, same accept decisions up to rounding of S at exact ties
    same = np.all(ev == ref, axis=0)
    assert same.mean() > 0.999
    assert npr == npr_o


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_threshold_p_wave_event_is_nonfinite_on_both_sides(prec):
    # at m_Kpi = mK + mpi the P-wave amplitude has q = 0, so S = 0 and ln S diverges
    e, res = _engine("kstar892", prec)
    par = W.params(res)
    data, mc = _sets(500, 2000, edges=True)
    assert data[0, 0] == W.M_LO
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    st_o, v_o, _ = O.nll(K, res, par, data, mc)
    st, v = e.nll_status(par)
    assert st_o == -5 and st == kpsi.KPSI_E_NONFINITE and v == math.inf
    st, v = e.nll_status(par, grad=True)
    assert st == kpsi.KPSI_E_NONFINITE and v == math.inf


def test_autograd_function_returns_the_adjoint_gradient():
    # the torch.autograd.Function binding: forward = one kpsi_nll_and_grad call, backward scales
    # the stored gradient by the incoming one
    import torch
    e, res = _engine("full", "fp64", ("K*(1410)",))
    data, mc = _sets(3001, 9001, seed=21)
    data = _interior(data)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    par = W.params(res, seed=22)
    NLL = kpsi.make_nll_function(e)
    p = torch.tensor(par, dtype=torch.float64, requires_grad=True)
    v = NLL.apply(p)
    (3.0 * v).backward()
    v_ref, g_ref = e.nll_and_grad(par)
    assert float(v) == pytest.approx(v_ref, rel=1e-14)
    g = p.grad.numpy()
    fin = np.isfinite(g_ref)
    np.testing.assert_allclose(g[fin], 3.0 * g_ref[fin], rtol=1e-14)
    assert np.all(np.isnan(g[~fin]))   # lineshape entries that are not floating stay NaN


def test_kernel_timing_samples_every_kth_call_and_reports_the_median():
    e, res = _engine("kstar10", "fp32")
    data, mc = _sets(2001, 6001, seed=23)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    par = W.params(res, seed=24)
    assert math.isnan(e.timing_median())          # nothing timed yet
    e.set_timing(3)
    for _ in range(10):
        e.nll_and_grad(par)
    med = e.timing_median()
    ms, n = e.timing()
    assert n == 4                                  # calls 1, 4, 7 and 10
    assert 0.0 < med <= ms                         # a median of positive samples, below their sum
    e.nll(par)                                     # the 11th call: not a timed one
    assert e.timing()[1] == 4
    ms, n = e.timing(reset=True)
    assert math.isnan(e.timing_median()) and e.timing() == (0.0, 0)
    e.set_timing(False)
    e.nll_and_grad(par)
    assert e.timing()[1] == 0
    # more timed calls than the library keeps event pairs for between reads
    e.set_timing(1)
    for _ in range(150):
        e.nll_and_grad(par)
    ms, n = e.timing()
    assert n == 150 and 0.0 < e.timing_median() <= ms / 100


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", None)])
@pytest.mark.parametrize("nd,nm", [(1, 1), (2, 3), (255, 257), (3072, 3073)])
def test_tiny_and_block_edge_sets_match_oracle(prec, tol, nd, nm):
    """Degenerate sizes: one event per set, sets smaller than a wavefront, and sizes one past a
    whole number of 256-thread block passes; NLL and gradient of the full model with two floating
    lineshapes against the oracle."""
    floating = ("K*(1410)", "Z(4430)")
    e, res = _engine("full", prec, floating)
    par = W.params(res, seed=29) + 0.05 * W.free_mask(res, floating)
    data, mc = _sets(nd, nm, seed=31, edges=False)
    data = _interior(data)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    dirs = np.flatnonzero(W.free_mask(res, floating))
    st, ref_v, ref_g = O.nll(K, res, par, data, mc, dirs=dirs)
    assert st == 0
    v, g = e.nll_and_grad(par)
    check_nll(v, ref_v, prec, nd, f"{nd}+{nm}")
    check_grad(g[dirs], ref_g, prec, f"{nd}+{nm}", norm=tol)
    check_nll(e.nll(par), ref_v, prec, nd, f"{nd}+{nm} nll-only")


def test_empty_set_is_refused():
    e, res = _engine("full", "fp32")
    with pytest.raises(kpsi.KpsiError):
        e.load(kpsi.DATA, np.zeros((4, 0)))
    st, _ = e.nll_status(W.params(res))
    assert st == kpsi.KPSI_E_STATE                 # nothing loaded: the call reports the state

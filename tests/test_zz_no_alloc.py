"""kpsi_nll_and_grad_noalloc (block partials in the library's static device array) against
kpsi_nll_and_grad (partials in a buffer the context allocates), through the C ABI: the two
must agree bit for bit, on two calls in a row, the second over a smaller event set (the static
array then still holds the larger call's partials), in both precisions, with flavour tags (two
normalisation records), and must refuse a call whose partials exceed the array."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W

K = W.KIN
pytestmark = pytest.mark.gpu
FLOAT = ("K*(1410)", "Z(4430)")


def _engine(prec, res):
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    e.set_floating([1 if r.name in FLOAT else 0 for r in res])
    return e


def _same(e, par):
    v0, g0 = e.nll_and_grad(par)
    v1, g1 = e.nll_and_grad_noalloc(par)
    fin = np.isfinite(g0)
    assert v1 == v0
    assert np.array_equal(g1[fin], g0[fin]) and np.array_equal(np.isnan(g1), np.isnan(g0))
    return v1, g1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_allocating_entry_point(prec):
    res = W.model("full")
    par = W.params(res, seed=91) + 0.03 * W.free_mask(res, FLOAT)
    e = _engine(prec, res)
    # first call: 600k + 1.2M events
    data = W.neutral_events(600_011, 92, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, 93, 1_200_007, W.PHSP_WMAX)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    v_big, _ = _same(e, par)
    # second call, smaller: 5k + 17k events
    e.load(kpsi.DATA, data[:, :5003])
    e.load(kpsi.NORM, mc[:, :17011])
    v_small, g_small = _same(e, par)
    assert v_small != v_big
    # and the oracle on the smaller sets
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    st, ref, gref = O.nll(K, res, par, data[:, :5003], mc[:, :17011], dirs=dirs)
    assert st == 0
    tol = 1e-10 if prec == "fp64" else 1e-6
    assert abs(v_small - ref) <= tol * max(abs(ref), 2.0 * 5003 * (prec == "fp32"))
    assert np.max(np.abs(g_small[dirs] - gref)) <= (1e-9 if prec == "fp64" else 1e-6) * np.max(np.abs(gref))
    e.close()


def test_noalloc_with_flavour_tags_and_a_second_context():
    res = W.model("full")
    par = W.params(res, seed=94) + 0.03 * W.free_mask(res, FLOAT)
    data = W.neutral_events(40_009, 95, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, 96, 90_001, W.PHSP_WMAX)
    tag = np.where(np.random.default_rng(97).random(data.shape[1]) < 0.5, 1.0, -1.0)
    a = _engine("fp32", res)
    a.load(kpsi.DATA, data)
    a.load(kpsi.NORM, mc)
    a.set_flavour(tag, 0.05)
    _same(a, par)
    # another context on the same device, smaller sets, called after the first
    b = _engine("fp32", res)
    b.load(kpsi.DATA, data[:, :3001])
    b.load(kpsi.NORM, mc[:, :7001])
    _same(b, par)
    _same(a, par)
    a.close()
    b.close()


def test_noalloc_refuses_more_partials_than_the_static_array():
    res = W.model("full")
    par = W.params(res, seed=98)
    e = _engine("fp32", res)
    ev = e.generate_phsp(99, 2_200_000, W.PHSP_WMAX)
    e.load(kpsi.DATA, ev)
    e.load(kpsi.NORM, ev)
    e.set_events_per_thread(1)          # 256 events per block: 2 x 8594 block partials > 16384
    st, _ = e.nll_status(par, grad=False)
    assert st == kpsi.KPSI_OK
    g = np.empty(e.n_params)
    out = np.empty(1)
    p = np.ascontiguousarray(par, dtype=np.float64)
    st = e.L.kpsi_nll_and_grad_noalloc(e.h, p.ctypes.data, out.ctypes.data, g.ctypes.data)
    assert st == kpsi.KPSI_E_ARG
    assert "static scratch" in e.L.kpsi_last_error(e.h).decode()
    e.set_events_per_thread(0)          # the automatic grid fits again
    _same(e, par)
    e.close()

"""Flavour-tagged charge-conjugate likelihood with mistag (text after Eq. 12) in the HIP path
against the FP64 oracle: NLL and gradient for random tags with and without mistag, the
normalisation served from the interference matrix, the tag independence at w = 1/2, the
reduction to the B0 likelihood, the tags together with the Eq. 14 background mixture (direct and
cached normalisation), and the error paths of kpsi_set_flavour."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W
from parity_bars import check_grad, check_nll

K = W.KIN
pytestmark = pytest.mark.gpu


def _inputs(model, nd=5003, nm=15013, seed=81):
    res = W.model(model)
    data = W.neutral_events(nd, seed, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, seed + 1, nm, W.PHSP_WMAX)
    eps_m = O.acceptance(W.acceptance_coefficients(), W.M_LO, W.M_HI, mc)
    tag = np.where(np.random.default_rng(seed + 2).random(nd) < 0.45, 1.0, -1.0)
    return res, data, mc, eps_m, tag


def _engine(prec, res, data, mc, eps_m, floating=()):
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    if floating:
        e.set_floating([1 if r.name in floating else 0 for r in res])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    e.set_efficiency_values(eps_m)
    return e


@pytest.mark.parametrize("model,prec,w,tg", [
    ("full", "fp64", 0.0, 1e-9), ("full", "fp64", 0.06, 1e-9), ("kstar10", "fp64", 0.06, 1e-9),
    ("full", "fp32", 0.0, None), ("full", "fp32", 0.06, None), ("kstar10", "fp32", 0.06, None),
    ("lass_full2z", "fp64", 0.04, 1e-9), ("lass_full2z", "fp32", 0.04, None), ("full2z", "fp64", 0.06, 1e-9),
    ("full2z", "fp32", 0.06, None)])
def test_cc_nll_and_gradient_match_oracle(model, prec, w, tg):
    floating = ("K*(1410)", "Z(4430)") if model == "full" else ("K*(1410)",)
    res, data, mc, eps_m, tag = _inputs(model)
    e = _engine(prec, res, data, mc, eps_m, floating)
    e.set_flavour(tag, w)
    par = W.params(res, seed=83) + 0.04 * W.free_mask(res, floating)
    dirs = np.flatnonzero(W.free_mask(res, floating))
    st, ref, gref = O.nll_cc(K, res, par, data, tag, mc, w, eps_m, dirs)
    assert st == 0
    v, g = e.nll_and_grad(par)
    nd = data.shape[1]
    tag = f"cc {model} w={w}"
    check_nll(v, ref, prec, nd, tag)
    check_grad(g[dirs], gref, prec, tag, norm=tg)
    check_nll(e.nll(par), ref, prec, nd, tag + " nll-only")


@pytest.mark.parametrize("prec,tg", [("fp64", 1e-9), ("fp32", None)])
def test_cc_normalisation_from_the_interference_matrix(prec, tg):
    # the -phi normalisation comes from the +phi matrix at exchanged lambda = +-1 couplings
    floating = ("K*(1410)", "Z(4430)")
    res, data, mc, eps_m, tag = _inputs("full", 3001, 9001)
    e = _engine(prec, res, data, mc, eps_m, floating)
    e.set_flavour(tag, 0.03)
    e.set_norm_cache(1)
    dirs = np.flatnonzero(W.free_mask(res, floating))
    nd = data.shape[1]
    par = W.params(res, seed=84) + 0.03 * W.free_mask(res, floating)
    st, ref, gref = O.nll_cc(K, res, par, data, tag, mc, 0.03, eps_m, dirs)
    assert st == 0
    v, g = e.nll_and_grad(par)
    assert e.norm_cache_stats()[0] == 1
    check_nll(v, ref, prec, nd, "cc cached")
    check_grad(g[dirs], gref, prec, "cc cached", norm=tg)
    # couplings only (the lambda = -1 coupling of K*(892) among them): served from the matrix
    p2 = par.copy()
    p2[2] += 0.07
    p2[9] -= 0.05
    st, ref2, gref2 = O.nll_cc(K, res, p2, data, tag, mc, 0.03, eps_m, dirs)
    v2, g2 = e.nll_and_grad(p2)
    b, h, _ = e.norm_cache_stats()
    assert b == 1 and h >= 1
    check_nll(v2, ref2, prec, nd, "cc cached couplings-only")
    check_grad(g2[dirs], gref2, prec, "cc cached couplings-only", norm=tg)
    check_nll(e.nll(p2), ref2, prec, nd, "cc cached couplings-only nll-only")


def test_cc_tags_off_and_b0_tags_give_the_signal_likelihood():
    res, data, mc, eps_m, tag = _inputs("full", 3001, 9001)
    e = _engine("fp64", res, data, mc, eps_m, ("Z(4430)",))
    par = W.params(res, seed=85)
    v0, g0 = e.nll_and_grad(par)
    e.set_flavour(np.ones_like(tag), 0.0)
    v1, g1 = e.nll_and_grad(par)
    assert v1 == pytest.approx(v0, rel=1e-12)
    fin = np.isfinite(g0)
    np.testing.assert_allclose(g1[fin], g0[fin], rtol=1e-9, atol=1e-9 * np.abs(g0[fin]).max())
    e.set_flavour(None)
    assert e.nll(par) == pytest.approx(v0, rel=1e-14)


def test_cc_half_mistag_makes_the_tags_irrelevant():
    res, data, mc, eps_m, tag = _inputs("full", 3001, 9001)
    e = _engine("fp64", res, data, mc, eps_m)
    par = W.params(res, seed=86)
    e.set_flavour(tag, 0.5)
    v = e.nll(par)
    e.set_flavour(-tag, 0.5)
    assert e.nll(par) == pytest.approx(v, rel=1e-11)
    e.set_flavour(tag, 0.1)
    assert abs(e.nll(par) - v) > 1e-3


def test_cc_errors_and_reload():
    res, data, mc, eps_m, tag = _inputs("kstar10", 1001, 3001)
    e = _engine("fp64", res, data, mc, eps_m)
    with pytest.raises(kpsi.KpsiError):
        e.set_flavour(tag[:-1], 0.0)
    bad = tag.copy()
    bad[3] = 0.5
    with pytest.raises(kpsi.KpsiError):
        e.set_flavour(bad, 0.0)
    with pytest.raises(kpsi.KpsiError):
        e.set_flavour(tag, 0.6)
    e.set_flavour(tag, 0.02)
    par = W.params(res, seed=87)
    _, ref, _ = O.nll_cc(K, res, par, data, tag, mc, 0.02, eps_m)
    assert e.nll(par) == pytest.approx(ref, rel=1e-10)
    # loading new data events drops the tags
    e.load(kpsi.DATA, data)
    _, ref0, _ = O.nll(K, res, par, data, mc, eps=eps_m)
    assert e.nll(par) == pytest.approx(ref0, rel=1e-10)


@pytest.mark.parametrize("prec,w,cached,tg", [
    ("fp64", 0.06, False, 1e-9), ("fp32", 0.06, False, None), ("fp64", 0.0, False, 1e-9),
    ("fp64", 0.04, True, 1e-9), ("fp32", 0.04, True, None)])
def test_cc_with_background_mixture_matches_oracle(prec, w, cached, tg):
    """Tags and the Eq. 14 mixture together: one background density for both flavours, each
    flavour normalised (f = p eps S~/N_q + (1 - p) b/N_b)."""
    floating = ("K*(1410)", "Z(4430)")
    res, data, mc, eps_m, tag = _inputs("full", 5003, 15013, seed=91)
    nd, nm = data.shape[1], mc.shape[1]
    rng = np.random.default_rng(92)
    eps_d = O.acceptance(W.acceptance_coefficients(), W.M_LO, W.M_HI, data)
    b_d, b_m = rng.uniform(0.2, 1.5, nd), rng.uniform(0.2, 1.5, nm)
    e = _engine(prec, res, data, mc, eps_m, floating)
    if cached:   # the other order of the two calls
        e.set_background(0.8, eps_d, b_d, b_m)
        e.set_flavour(tag, w)
        e.set_norm_cache(1)
    else:
        e.set_flavour(tag, w)
        e.set_background(0.8, eps_d, b_d, b_m)
    par = W.params(res, seed=93) + 0.04 * W.free_mask(res, floating)
    dirs = np.flatnonzero(W.free_mask(res, floating))
    pts = [par]
    if cached:
        p2 = par.copy()
        p2[2] += 0.07
        p2[9] -= 0.05
        pts.append(p2)
    for k, p in enumerate(pts):
        st, ref, gref = O.nll_cc_mix(K, res, p, data, tag, mc, w, b_d, b_m, 0.8, eps_d, eps_m, dirs)
        assert st == 0
        v, g = e.nll_and_grad(p)
        label = f"cc+mixture w={w}{' cached' if cached else ''} point {k}"
        check_nll(v, ref, prec, nd, label)
        check_grad(g[dirs], gref, prec, label, norm=tg)
        check_nll(e.nll(p), ref, prec, nd, label + " nll-only")
    if cached:
        b, h, _ = e.norm_cache_stats()
        assert b == 1 and h >= 1
    e.close()

"""LASS S-wave (Eq. 7-8) in the HIP path against the FP64 oracle: per-event densities,
NLL and gradient (with and without the interference-matrix normalisation) and fit
fractions, for the ten-K* model with the LASS term in place of K0*(800) and K0*(1430)
and the same with the two Z states.  Edge events include the K pi threshold, where the
LASS amplitude stays finite (its effective-range term tends to m a)."""
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


def _interior(ev):
    ev = ev.copy()
    ev[0] = np.clip(ev[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    return ev


@pytest.mark.parametrize("model,prec,rtol", [("kstar_lass", "fp64", 1e-11), ("lass_full2z", "fp64", 1e-11),
                                             ("kstar_lass", "fp32", 2e-5), ("lass_full2z", "fp32", 2e-5)])
def test_lass_density_matches_oracle(model, prec, rtol):
    e, res = _engine(model, prec)
    par = W.params(res, seed=23)
    ev = W.neutral_events(3079, 29, peaked=False, edges=True)
    if model == "lass_full2z":
        ev = _interior(ev)
    else:
        assert ev[0, 0] == W.M_LO           # the threshold event is kept for the K*-only model
    e.load(kpsi.DATA, ev)
    s = e.density(kpsi.DATA, par)
    o = O.density(K, res, par, ev)
    assert np.all(o > 0)
    np.testing.assert_allclose(s, o, rtol=rtol, atol=rtol * 0.1 * o.max())


@pytest.mark.parametrize("model,prec,tg,cache", [
    ("kstar_lass", "fp64", 1e-9, 0), ("lass_full2z", "fp64", 1e-9, 0),
    ("lass_full2z", "fp64", 1e-9, 1), ("kstar_lass", "fp32", None, 0),
    ("lass_full2z", "fp32", None, 0), ("lass_full2z", "fp32", None, 1)])
def test_lass_nll_and_gradient_match_oracle(model, prec, tg, cache):
    floating = ("K*(1410)", "Z(4430)") if model == "lass_full2z" else ("K*(1410)",)
    e, res = _engine(model, prec, floating)
    par = W.params(res, seed=31) + 0.05 * W.free_mask(res, floating)
    data = _interior(W.neutral_events(6007, 37, peaked=True, edges=True))
    mc = O.gen_phsp(K, 38, 18013, W.PHSP_WMAX)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    e.set_norm_cache(cache)
    dirs = np.flatnonzero(W.free_mask(res, floating))
    st, ref_v, ref_g = O.nll(K, res, par, data, mc, dirs=dirs)
    assert st == 0
    v, g = e.nll_and_grad(par)
    nd = data.shape[1]
    tag = f"lass {model} cache={cache}"
    check_nll(v, ref_v, prec, nd, tag)
    check_grad(g[dirs], ref_g, prec, tag, norm=tg)
    check_nll(e.nll(par), ref_v, prec, nd, tag + " nll-only")
    if cache:
        assert e.norm_cache_stats()[0] >= 1


@pytest.mark.parametrize("model,prec,rtol", [("kstar_lass", "fp64", 1e-9), ("lass_full2z", "fp64", 1e-9),
                                             ("lass_full2z", "fp32", 2e-5)])
def test_lass_fit_fractions_match_oracle(model, prec, rtol):
    mc = O.gen_phsp(K, 43, 20011, W.PHSP_WMAX)
    res = W.model(model)
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    e.load(kpsi.NORM, mc)
    par = W.params(res, seed=41)
    ff, tot = e.fit_fractions(par)
    st, ref = O.fit_fractions(K, res, par, mc)
    assert st == 0
    np.testing.assert_allclose(ff, ref, rtol=rtol, atol=rtol * 1e-3)
    assert tot == pytest.approx(ref.sum(), rel=rtol)


def test_lass_lineshape_cannot_float_and_needs_valid_parameters():
    import dataclasses
    e, res = _engine("kstar_lass", "fp64")
    i = [r.name for r in res].index("LASS")
    flags = [0] * len(res)
    flags[i] = 1
    with pytest.raises(kpsi.KpsiError):
        e.set_floating(flags)
    bad = list(res)
    bad[i] = dataclasses.replace(res[i], lass_a=0.0)
    with pytest.raises(kpsi.KpsiError):
        e.set_model(K, bad)
    bad[i] = dataclasses.replace(res[i], spin=1)
    with pytest.raises(kpsi.KpsiError):
        e.set_model(K, bad)

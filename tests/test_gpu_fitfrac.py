"""Fit fractions (Eq. 13) through the FP64 matrix-core interference matrix, against the FP64
oracle's masked-density sums over the same phase-space events."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W

K = W.KIN
pytestmark = pytest.mark.gpu


def _engine(model, prec, mc, eps=None):
    res = W.model(model)
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    e.load(kpsi.NORM, mc)
    if eps is not None:
        e.set_efficiency_values(eps)
    return res, e


@pytest.mark.parametrize("model,prec,rtol", [("full", "fp64", 1e-9), ("full2z", "fp64", 1e-9),
                                             ("kstar10", "fp64", 1e-9), ("full", "fp32", 2e-5),
                                             ("full2z", "fp32", 2e-5)])
def test_fit_fractions_match_oracle(model, prec, rtol):
    mc = O.gen_phsp(K, 41, 20011, W.PHSP_WMAX)
    res, e = _engine(model, prec, mc)
    par = W.params(res, seed=8)
    ff, tot = e.fit_fractions(par)
    st, ref = O.fit_fractions(K, res, par, mc)
    assert st == 0
    np.testing.assert_allclose(ff, ref, rtol=rtol, atol=rtol * 1e-3)
    assert tot == pytest.approx(ref.sum(), rel=rtol)


def test_fit_fractions_ignore_efficiency_and_keep_the_cache():
    mc = O.gen_phsp(K, 42, 9001, W.PHSP_WMAX)
    eps = O.acceptance(W.acceptance_coefficients(), W.M_LO, W.M_HI, mc)
    res, e = _engine("full", "fp64", mc, eps)
    par = W.params(res, seed=9)
    data = W.neutral_events(3001, 43, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    e.load(kpsi.DATA, data)
    e.set_norm_cache(1)
    v0 = e.nll(par)
    b0 = e.norm_cache_stats()[0]
    ff, _ = e.fit_fractions(par)
    _, ref = O.fit_fractions(K, res, par, mc)
    np.testing.assert_allclose(ff, ref, rtol=1e-9)
    assert e.norm_cache_stats()[0] == b0          # the efficiency-weighted cache is untouched
    assert e.nll(par) == v0


def test_single_resonance_fraction_is_one():
    mc = O.gen_phsp(K, 44, 5003, W.PHSP_WMAX)
    res, e = _engine("kstar892", "fp32", mc)
    ff, tot = e.fit_fractions(W.params(res, seed=1))
    assert ff[0] == pytest.approx(1.0, rel=1e-6) and tot == pytest.approx(1.0, rel=1e-6)

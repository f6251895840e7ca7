"""Gaussian constraints on fit parameters through the C ABI: NLL and gradient against the
oracle likelihood plus the oracle penalty, a constrained fit that holds a floating mass at its
constraint, and the error paths."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W

K = W.KIN
pytestmark = pytest.mark.gpu
FLOAT = ("K*(1410)", "Z(4430)")


def _setup(prec="fp64", nd=4001, nm=12007):
    res = W.model("full")
    data = W.neutral_events(nd, 91, peaked=True)
    data[0] = np.clip(data[0], W.M_LO + 1e-6, W.M_HI - 1e-6)
    mc = O.gen_phsp(K, 92, nm, W.PHSP_WMAX)
    e = kpsi.Engine(0, prec)
    e.set_model(K, res)
    e.set_floating([1 if r.name in FLOAT else 0 for r in res])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    return res, data, mc, e


def _mass_index(res, name):
    nc = sum(2 * r.n_coup for r in res)
    return nc + 2 * [r.name for r in res].index(name)


def test_constraints_add_the_penalty_to_nll_and_gradient():
    res, data, mc, e = _setup()
    par = W.params(res, seed=93) + 0.03 * W.free_mask(res, FLOAT)
    im = _mass_index(res, "K*(1410)")
    idx = np.array([im, im + 1, 4])
    mu = par[idx] + np.array([0.01, -0.02, 0.05])
    sg = np.array([0.005, 0.03, 0.2])
    e.set_constraints(idx, mu, sg)
    dirs = np.flatnonzero(W.free_mask(res, FLOAT))
    st, ref, gref = O.nll(K, res, par, data, mc, dirs=dirs)
    assert st == 0
    pen, gpen = O.gauss_penalty(idx, mu, sg, par)
    v, g = e.nll_and_grad(par)
    assert v == pytest.approx(ref + pen, rel=1e-10)
    want = gref + gpen[dirs]
    assert np.max(np.abs(g[dirs] - want)) / np.max(np.abs(want)) < 1e-9
    assert e.nll(par) == pytest.approx(ref + pen, rel=1e-10)
    e.set_constraints()
    assert e.nll(par) == pytest.approx(ref, rel=1e-10)


def test_tight_constraint_holds_a_floating_mass_in_the_fit():
    # K*(892) pseudo-data from the oracle's generator; its mass floats with a constraint 3 MeV
    # above the generated value and 0.01 MeV wide: the fit combines the two as Gaussians, the
    # mass lands at the inverse-variance mean of the unconstrained fit and the constraint
    res = W.model("kstar892")
    truth = W.params(res, seed=11)
    scan = O.gen_phsp(K, 300, 200_000, W.PHSP_WMAX)
    smax = 1.5 * O.density(K, res, truth, scan).max()
    data, _, nover = O.gen_model(K, res, truth, 301, 10_000, W.PHSP_WMAX, smax)
    assert nover == 0
    mc = O.gen_phsp(K, 302, 100_000, W.PHSP_WMAX)
    e = kpsi.Engine(0, "fp64")
    e.set_model(K, res)
    e.set_floating([1])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    mask = W.free_mask(res, ("K*(892)",))
    im = _mass_index(res, "K*(892)")
    x0, cov0, r0 = e.migrad(truth, mask)
    assert r0.status == 0
    target = truth[im] + 0.003
    e.set_constraints([im], [target], [1e-5])
    x, cov, r = e.migrad(truth, mask)
    assert r.status == 0
    k = list(np.flatnonzero(mask)).index(im)
    free_err = np.sqrt(cov0[k, k])
    assert free_err > 1e-4                       # the data alone measure the mass much less well
    wc, wf = 1e-5 ** -2, free_err ** -2
    expect = (wc * target + wf * x0[im]) / (wc + wf)
    assert abs(x[im] - expect) < 1e-6
    assert np.sqrt(cov[k, k]) == pytest.approx((wc + wf) ** -0.5, rel=0.02)


def test_constraint_errors_and_reset_by_the_model():
    res, data, mc, e = _setup()
    n = W.n_params(res)
    with pytest.raises(kpsi.KpsiError):
        e.set_constraints([n], [0.0], [1.0])
    with pytest.raises(kpsi.KpsiError):
        e.set_constraints([0], [0.0], [0.0])
    par = W.params(res, seed=95)
    v0 = e.nll(par)
    e.set_constraints([0], [par[0] + 1.0], [0.5])
    assert e.nll(par) == pytest.approx(v0 + 4.0, rel=1e-12, abs=1e-9)
    e.set_model(K, res)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    assert e.nll(par) == pytest.approx(v0, rel=1e-12)

"""Learned efficiency: BF16 matrix-core network kernels against the FP64 reference network
(same BF16 rounding points), accept labels, histogram efficiency, and the gain of the
trained network over the 20^4 histogram against the known analytic acceptance."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14931_amd import kpsi
from paper_2007_14931_amd import workloads as W
from parity_bars import check_probabilities

K = W.KIN
pytestmark = pytest.mark.gpu


def _engine():
    e = kpsi.Engine(0, "fp32")
    e.set_model(K, W.model("full"))
    return e


def _cuda(ev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(ev)).to("cuda:0")


@pytest.mark.parametrize("n", [64, 4133])
def test_network_gradient_and_output_match_reference(n):
    import torch
    e = _engine()
    ev = W.neutral_events(n, 31)
    rng = np.random.default_rng(5)
    y = (rng.uniform(size=n) < 0.6).astype(np.uint8)
    par = W.mlp_init(3)
    par[256:320] = rng.normal(0, 0.3, 64)
    par[4416:4480] = rng.normal(0, 0.3, 64)
    g, loss = e.mlp_grad(par, _cuda(ev), torch.from_numpy(y).to("cuda:0"))
    u = O.mlp_inputs(W.M_LO, W.M_HI, ev)
    ref_loss, ref_p, ref_g = O.mlp(par.astype(np.float64), u, y.astype(np.float64), grad=True)
    assert loss == pytest.approx(ref_loss, rel=2e-5)
    assert np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g) < 1e-4
    for blk in (slice(0, 256), slice(256, 320), slice(320, 4416), slice(4416, 4480), slice(4480, 4545)):
        assert np.linalg.norm(g[blk] - ref_g[blk]) <= 1e-3 * np.linalg.norm(ref_g[blk]) + 1e-9
    p = e.mlp_eval(par, _cuda(ev)).cpu().numpy()
    check_probabilities(p, ref_p, par, u)
    # against the plain FP64 network (no BF16 rounding anywhere; its gradient is pinned by
    # differences on the CPU): the device gradient is that network's gradient up to the BF16
    # precision of the weights and 64x64 operands (8-bit significands: relative 2^-9 per rounding)
    loss64, p64, g64 = O.mlp(par.astype(np.float64), u, y.astype(np.float64), grad=True, round_bf16=False)
    eg = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    ep = float(np.max(np.abs(p - p64)))
    print(f"[parity] network n={n} vs unrounded FP64 network: gradient {eg:.2e}, loss {abs(loss - loss64) / loss64:.2e}, "
          f"max |dp| {ep:.2e}", flush=True)
    assert eg < 2e-2 and abs(loss - loss64) < 1e-4 * loss64 and ep < 3e-3


def test_labels_and_histogram():
    import torch
    e = _engine()
    coef = W.acceptance_coefficients()
    ev = e.generate_phsp(501, 300_000, W.PHSP_WMAX)
    lab, eps = e.accept_labels(502, ev, coef)
    evh = ev.cpu().numpy()
    ref = O.acceptance(coef, W.M_LO, W.M_HI, evh[:, :2000])
    np.testing.assert_allclose(eps.cpu().numpy()[:2000], ref, rtol=1e-14)
    labh = lab.cpu().numpy()
    assert abs(labh.mean() - eps.cpu().numpy().mean()) < 5 * math.sqrt(0.25 / labh.size)
    nb = (5, 4, 3, 6)
    lo = np.array([W.M_LO, -1, -1, -math.pi])
    hi = np.array([W.M_HI, 1, 1, math.pi])
    t = e.hist_efficiency(ev, lab, nb, lo, hi)
    idx = [np.clip(np.floor((evh[d] - lo[d]) / (hi[d] - lo[d]) * nb[d]).astype(int), 0, nb[d] - 1) for d in range(4)]
    flat = np.ravel_multi_index(idx, nb)
    gen = np.bincount(flat, minlength=int(np.prod(nb)))
    acc = np.bincount(flat, weights=labh, minlength=int(np.prod(nb)))
    ref_t = np.where(gen > 0, acc / np.maximum(gen, 1), labh.mean()).reshape(nb)
    np.testing.assert_allclose(t, ref_t, rtol=1e-6)


def test_trained_network_beats_histogram():
    e = _engine()
    coef = W.acceptance_coefficients()
    train = e.generate_phsp(601, 1_000_000, W.PHSP_WMAX)
    lab, _ = e.accept_labels(602, train, coef)
    par, loss = e.mlp_train(W.mlp_init(1), train, lab, epochs=12, batch=16384, lr=3e-3)
    assert math.isfinite(loss)
    val = e.generate_phsp(603, 200_000, W.PHSP_WMAX)
    _, eps_true = e.accept_labels(604, val, coef)
    eps_true = eps_true.cpu().numpy()
    eps_nn = e.mlp_eval(par, val).cpu().numpy()
    nb = (20, 20, 20, 20)
    lo = np.array([W.M_LO, -1, -1, -math.pi])
    hi = np.array([W.M_HI, 1, 1, math.pi])
    t = e.hist_efficiency(train, lab, nb, lo, hi)
    v = val.cpu().numpy()
    idx = [np.clip(np.floor((v[d] - lo[d]) / (hi[d] - lo[d]) * nb[d]).astype(int), 0, nb[d] - 1) for d in range(4)]
    eps_h = t[tuple(idx)]
    rms_nn = np.sqrt(np.mean((eps_nn - eps_true) ** 2))
    rms_h = np.sqrt(np.mean((eps_h - eps_true) ** 2))
    print(f"rms(network - truth) {rms_nn:.4f}  rms(histogram - truth) {rms_h:.4f}  loss {loss:.5f}")
    assert rms_nn < 0.5 * rms_h
    assert rms_nn < 0.03

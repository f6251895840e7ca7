"""Parity bars of the GPU tests against the FP64 oracle, in one place.

NLL: relative 1e-10 on the FP64 path and 1e-6 on the FP32 path.  The FP32 NLL is the
difference of two sums of N_d terms each (the data log-densities and the normalisation term)
and can cancel to a value far below either, so its error is measured against
max(|NLL|, 2 N_d): a relative error of 1e-6 in the per-event densities.  The FP64 bar is a
plain relative one.

Gradient: normwise, max_k |g_k - g_ref_k| / max_k |g_ref_k| (1e-6 on the FP32 path, the
test's own, tighter bar on the FP64 path), and componentwise for every component with
|g_ref_k| > 1e-3 max|g_ref|.  On the FP32 path the componentwise bar follows from the normwise
floor: the FP32 gradient carries an absolute error of 1e-7 - 3e-7 of max|g| shared by all
components, from two sources.  (i) The per-resonance constants are rounded to FP32: couplings
times the lineshape constant, P = M^2 B(z0) Gamma0/q0^(2L+1), the barrier radii.  That moves the
evaluated parameter point by about 3e-8 (relative), and at 10^4 - 10^7 events the likelihood's
curvature turns this into a gradient shift of that size.  (ii) Per-event FP32 rounding adds to it.
A component of 1e-3 max|g| therefore sees up to 1e-4 relative, which is the FP32
componentwise bar.  (The squared masses, whose rounding moved the narrow poles and dominated
before, are carried as FP32 pairs: value and rounding remainder.)

Every check prints its measured errors.
"""
from __future__ import annotations

import numpy as np

FP64_NLL = 1e-10
FP32_NLL = 1e-6
FP32_GRAD_NORM = 1e-6
FP32_GRAD_COMP = 1e-4
COMP_FLOOR = 1e-3   # components below this fraction of max|g| are covered by the normwise bar


def nll_error(v: float, ref: float, prec: str, nd: int) -> float:
    """Error of an NLL value in units of its bar's scale (see the module docstring)."""
    scale = abs(ref) if prec == "fp64" else max(abs(ref), 2.0 * nd)
    return abs(v - ref) / scale


def check_nll(v: float, ref: float, prec: str, nd: int, tag: str = "", rel: float | None = None) -> float:
    tol = rel if rel is not None else (FP64_NLL if prec == "fp64" else FP32_NLL)
    err = nll_error(v, ref, prec, nd)
    print(f"[parity] {tag} {prec} nll {v:.10g} oracle {ref:.10g} err {err:.3e} (bar {tol:.0e})", flush=True)
    assert err <= tol, (tag, prec, v, ref, err)
    return err


def grad_errors(g, ref) -> tuple[float, float]:
    """(normwise, componentwise) errors of a gradient against its reference."""
    g, ref = np.asarray(g, float), np.asarray(ref, float)
    gi = np.max(np.abs(ref))
    d = np.abs(g - ref)
    big = np.abs(ref) > COMP_FLOOR * gi
    comp = float(np.max(d[big] / np.abs(ref[big]))) if np.any(big) else 0.0
    return float(np.max(d) / gi), comp


def check_grad(g, ref, prec: str, tag: str = "", norm: float | None = None, comp: float | None = None):
    """Normwise and componentwise gradient check; FP64 bars default to the test's normwise bar
    (given as `norm`) and ten times it componentwise."""
    if prec == "fp64":
        assert norm is not None, "FP64 gradient checks state their bar"
        tn, tc = norm, (comp if comp is not None else 10.0 * norm)
    else:
        tn = norm if norm is not None else FP32_GRAD_NORM
        tc = comp if comp is not None else FP32_GRAD_COMP
    en, ec = grad_errors(g, ref)
    print(f"[parity] {tag} {prec} gradient ({len(np.atleast_1d(ref))} dirs) normwise {en:.3e} (bar {tn:.0e}) "
          f"componentwise {ec:.3e} (bar {tc:.0e})", flush=True)
    assert en <= tn and ec <= tc, (tag, prec, en, ec)
    return en, ec


def check_probabilities(p, ref_p, par, u):
    """The device rounds silu(z1) to BF16 from an FP32 value, the reference from an FP64 one.
    Where the two straddle a BF16 rounding boundary, one hidden unit differs by one BF16 ulp
    (at most 2^-8 of its value). Through the 64x64 layer (|silu'| < 1.1) and the sigmoid
    (slope <= 1/4) that moves p by at most
        (1/4) * max_i sum_o |w3_o| 1.1 |W2_oi| * 2^-8 max|h1|   per flipped unit.
    Every other event must agree to FP32 accuracy, and flips must be rare."""
    W1, b1 = par[:256].reshape(64, 4).astype(np.float64), par[256:320].astype(np.float64)
    W2, w3 = par[320:4416].reshape(64, 64).astype(np.float64), par[4480:4544].astype(np.float64)
    z1 = u @ W1.T + b1
    h1max = np.max(np.abs(z1 / (1 + np.exp(-z1))))
    one_flip = 0.25 * np.max(np.abs(w3) @ (1.1 * np.abs(W2))) * 2.0 ** -8 * h1max
    d = np.abs(p - ref_p)
    tight = d <= 1e-5 * np.abs(ref_p) + 1e-6
    assert tight.mean() >= 0.995, f"{(~tight).sum()} of {d.size} events outside FP32 agreement"
    assert d.max() <= 2 * one_flip, f"max difference {d.max():.3g} exceeds two BF16 flips ({2 * one_flip:.3g})"

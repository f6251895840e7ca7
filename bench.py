"""Benchmark: NLL+gradient evaluations per second of the full amplitude model.

Workload "full_grad_1m": ten K* + Z(4430) (Eq. 12), 1,000,000 data events drawn by
accept-reject from the model and 2,000,000 flat phase-space normalisation events (all
generated on the GPU by the library's Philox generators), masses and widths of
K*(1410) and Z(4430) floating.  One step = one kpsi_nll_and_grad call: every data and
normalisation event is evaluated, -2 ln L and its 54 free-parameter gradient are
reduced and returned to the host (what a minimiser sees per iteration).

Prints one JSON line.  `value` is host-visible evaluations/s with the events resident
in HBM; `roofline` refers to the per-event kernel, timed with HIP events on the
library's stream; `cpu_baseline` is the FP64 CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point work per event of one NLL+gradient call of this workload
# (fused multiply-add = 2, other arithmetic and reciprocal/rsqrt/log = 1), from the op count
# of the per-call formulation (bare Breit-Wigner per resonance, resonance constants in the
# couplings, barrier factors in the d functions): forward 530, adjoint 384.
TIMING_EVERY = 10     # in the timed region: HIP events on every 10th call (cross-check)
POST_CALLS = 400      # host-timed calls of each post-loop leg
KERNEL_REPS = 100     # back-to-back launches per HIP-event pair (kpsi_time_kernel)
KERNEL_BATCHES = 5
# Algorithmic bytes per event: the four observables of each event in the arithmetic's type
# (m_Kpi, cos theta_K*, cos theta_J/psi, phi), read once per call.
ALG_BYTES_PER_EVENT = {"f32": 16, "f64": 32}
FLOP_PER_EVENT = {"full_grad": 914}
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}        # MI355X published vector peaks
PEAK_TFLOPS_UNPACKED = {"f32": 78.6, "f64": 78.6}  # without packed-FP32 instructions
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}     # MI355X published dense matrix-core peaks


def measured_traffic(kernel_source: str) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None
    when the kernel source has changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "amp_kernel_traffic.json")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(os.path.join(ROOT, kernel_source), "rb").read()).hexdigest()
    except OSError:
        return None
    if not sha.startswith(rec["source_sha256_prefix"]):
        return None
    return float(rec["traffic_bytes"])


def timed_leg(e, par, grad: bool, calls: int = 0) -> dict:
    """Kernel time and host rate of NLL(+gradient) calls.  Kernel: KERNEL_BATCHES batches of
    KERNEL_REPS back-to-back launches of the per-event work between one pair of HIP events on the
    library's stream (kpsi_time_kernel); mean and median of the batches' per-launch times.  Host:
    `calls` (at least POST_CALLS) ordinary calls."""
    calls = max(calls, POST_CALLS)
    f = e.nll_and_grad if grad else e.nll
    for _ in range(20):
        f(par)
    t0 = time.perf_counter()
    for _ in range(calls):
        f(par)
    dt = time.perf_counter() - t0
    b = [e.time_kernel(par, grad=grad, reps=KERNEL_REPS) for _ in range(KERNEL_BATCHES)]
    return {"timed_launches": KERNEL_REPS * KERNEL_BATCHES, "kernel_ms_mean": float(np.mean(b)),
            "kernel_ms_median": float(np.median(b)), "host_ms_per_call": dt / calls * 1e3}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(res, par, floating, n_data: int, n_mc: int, seconds: float = 15.0) -> dict:
    """The FP64 oracle (dual-number gradient) on a bounded sample of the workload, scaled to
    evaluations/s of the full workload."""
    from oracle import oracle as O
    from paper_2007_14931_amd import workloads as W
    K = W.KIN
    dirs = np.flatnonzero(W.free_mask(res, floating))
    nd_s, nm_s = 2000, 4000
    data = W.neutral_events(nd_s, 91, peaked=True)
    mc = O.gen_phsp(K, 92, nm_s, W.PHSP_WMAX)
    scale = (n_data + n_mc) / (nd_s + nm_s)
    cores = O.max_threads()
    O.nll(K, res, par, data, mc, dirs=dirs)   # warm-up
    t0 = time.perf_counter()
    times = []
    while True:
        t1 = time.perf_counter()
        O.nll(K, res, par, data, mc, dirs=dirs)
        times.append(time.perf_counter() - t1)
        if time.perf_counter() - t0 > seconds:
            break
    dt = float(np.mean(times))
    med = float(np.median(times))
    # the same oracle on one core: one warm-up, then the median of five evaluations
    O.set_threads(1)
    try:
        O.nll(K, res, par, data, mc, dirs=dirs)
        one = []
        for _ in range(5):
            t1 = time.perf_counter()
            O.nll(K, res, par, data, mc, dirs=dirs)
            one.append(time.perf_counter() - t1)
    finally:
        O.set_threads(cores)
    one_med = float(np.median(one))
    return {"value": 1.0 / (dt * scale), "unit": "NLL+grad evals/s", "cores": cores, "kind": "oracle",
            "median_value": 1.0 / (med * scale), "one_core_value": 1.0 / (one_med * scale),
            "sample": f"{nd_s} data + {nm_s} normalisation events, {len(dirs)} gradient directions, "
                      f"{len(times)} evaluations in {sum(times):.1f} s on {cores} threads after one warm-up "
                      f"(one_core_value: median of 5 on one thread), scaled by {scale:.0f} to the full workload"}


def fit_comparison(make, truth, mask, canonical_fn) -> dict:
    """Full MIGRAD + HESSE fit of the benchmark workload from the same start point: FP32
    amplitudes with the device adjoint gradient; the same followed by an FP64 adjoint polish
    (the FP32 likelihood's rounding noise sits near the EDM target, so the FP32 fit can stop
    with a failed line search just short of it); the plain FP64 likelihood with central
    finite-difference gradients; and the same FP64 finite-difference fit with the
    interference-matrix cache in auto mode (coupling-only steps reuse the normalisation).
    Reports wall time, likelihood calls and how far apart the minima are in units of the FP64
    HESSE errors (couplings compared as magnitude >= 0, phase in (-pi, pi])."""
    rng = np.random.default_rng(7)
    x0 = truth + 0.01 * rng.standard_normal(truth.size) * mask
    free = np.flatnonzero(mask)
    runs = {}
    cache_stats = None
    for name, prec, grad, cache in (("fp32_analytic", "fp32", 1, 0), ("fp64_finite_difference", "fp64", 0, 0),
                                    ("fp64_finite_difference_cached", "fp64", 0, 2)):
        e = make(prec)
        if cache:
            e.set_norm_cache(cache)   # auto: coupling-only steps reuse the normalisation matrix
        x, cov, r = e.migrad(x0, mask, gradient=grad)
        if cache:
            b, h, ms = e.norm_cache_stats()
            cache_stats = {"builds": b, "hits": h, "last_build_ms": ms}
        e.close()
        runs[name] = (x, cov, r)
        log(f"fit {name}: status {r.status} fmin {r.fmin:.4f} edm {r.edm:.2e} wall {r.wall_seconds:.3f} s "
            f"nll calls {r.n_nll} grad calls {r.n_grad}")
        if name == "fp32_analytic":
            e = make("fp64")
            xp, cp, rp = e.migrad(x, mask, gradient=1)
            e.close()
            runs["fp32_analytic_fp64_polish"] = (xp, cp, rp)
            log(f"fit fp32_analytic + fp64 polish: status {rp.status} fmin {rp.fmin:.4f} edm {rp.edm:.2e} "
                f"wall {r.wall_seconds:.3f} + {rp.wall_seconds:.3f} s")
    xa, ca, ra = runs["fp32_analytic"]
    xf, cf, rf = runs["fp64_finite_difference"]
    xc, cc, rc = runs["fp64_finite_difference_cached"]
    xp, cp, rp = runs["fp32_analytic_fp64_polish"]
    xa, xf, xp = canonical_fn(xa), canonical_fn(xf), canonical_fn(xp)
    sig = np.sqrt(np.abs(np.diag(cf)))
    sig_a = np.sqrt(np.abs(np.diag(ca)))
    dev = np.abs(xa[free] - xf[free]) / sig
    worst = [{"index": int(free[k]), "x_fp32_analytic": float(xa[free[k]]), "x_fp64_fd": float(xf[free[k]]),
              "sigma_fp64_fd": float(sig[k]), "sigma_fp32_analytic": float(sig_a[k])}
             for k in np.argsort(dev)[-3:][::-1]]
    return {
        "largest_differences": worst,
        "fp32_analytic": ra.as_dict(),
        "fp32_analytic_fp64_polish": {**rp.as_dict(), "wall_seconds_total": ra.wall_seconds + rp.wall_seconds,
                                      "max_param_diff_sigma": float(np.max(np.abs(xp[free] - xf[free]) / sig)),
                                      "wall_ratio_fd_over_this": rf.wall_seconds / (ra.wall_seconds + rp.wall_seconds)},
        "fp64_finite_difference": rf.as_dict(),
        "fp64_finite_difference_cached": {**rc.as_dict(), "norm_cache": cache_stats,
                                          "max_param_diff_sigma_vs_uncached":
                                              float(np.max(np.abs(canonical_fn(xc)[free] - xf[free]) / sig))},
        "wall_ratio_fd_over_analytic": rf.wall_seconds / ra.wall_seconds,
        "wall_ratio_fd_over_fd_cached": rf.wall_seconds / rc.wall_seconds,
        "max_param_diff_sigma": float(dev.max()),
        "median_param_diff_sigma": float(np.median(dev)),
        "error_ratio_max_dev": float(np.max(np.abs(np.sqrt(np.abs(np.diag(ca))) / sig - 1.0))),
        "free_params": int(len(free)),
    }


def fit_far_start(make, truth, mask, canonical_fn, n_coupling_reals: int) -> dict:
    """The FP32-adjoint fit (with its FP64 polish) and the plain FP64 finite-difference fit from a
    start far from the generated point: every free coupling magnitude scaled by exp(0.3 N(0,1)),
    every free phase moved by 0.3 N(0,1) rad, the floating masses and widths by 2% N(0,1)."""
    rng = np.random.default_rng(17)
    x0 = truth.copy()
    for i in np.flatnonzero(mask):
        if i < n_coupling_reals:
            x0[i] = x0[i] * math.exp(0.3 * rng.standard_normal()) if i % 2 == 0 else x0[i] + 0.3 * rng.standard_normal()
        else:
            x0[i] *= 1.0 + 0.02 * rng.standard_normal()
    free = np.flatnonzero(mask)
    e = make("fp32")
    xa, _, ra = e.migrad(x0, mask, gradient=1)
    e.close()
    e = make("fp64")
    xp, _, rp = e.migrad(xa, mask, gradient=1)
    e.close()
    e = make("fp64")
    xf, cf, rf = e.migrad(x0, mask, gradient=0)
    e.close()
    sig = np.sqrt(np.abs(np.diag(cf)))
    dev = np.abs(canonical_fn(xp)[free] - canonical_fn(xf)[free]) / sig
    log(f"far start: fp32 adjoint {ra.wall_seconds:.3f} s (status {ra.status}, {ra.n_iter} iterations) + polish "
        f"{rp.wall_seconds:.3f} s; fp64 finite differences {rf.wall_seconds:.3f} s (status {rf.status}, "
        f"{rf.n_iter} iterations); minima {dev.max():.4f} sigma apart")
    return {"start": "couplings r exp(0.3 N), phase + 0.3 N; floating M, Gamma x (1 + 0.02 N); seed 17",
            "fp32_analytic": ra.as_dict(), "fp32_analytic_fp64_polish": rp.as_dict(),
            "fp64_finite_difference": rf.as_dict(),
            "wall_ratio_fd_over_analytic_polished": rf.wall_seconds / (ra.wall_seconds + rp.wall_seconds),
            "max_param_diff_sigma": float(dev.max()), "median_param_diff_sigma": float(np.median(dev))}


def norm_cache_leg(eng, par, res, floating, precision: str) -> dict:
    """The interference-matrix path on the benchmark engine: one build of the normalisation
    matrices at the benchmark point (matrix-core Gram product over the 2e6 normalisation events:
    FP32 products with FP64 tile sums in the FP32 context, FP64 in the FP64 context), then
    NLL+gradient calls that change only couplings, served from the matrices (only the data
    events are evaluated per call)."""
    ncomp = sum(r.n_coup for r in res)                                   # complex coupling components
    nderiv = sum(2 * r.n_coup for r in res if r.name in floating)       # d/dM and d/dGamma0 components
    # algorithmic MACs per (event, xi) row: the upper triangle of the real Gram block of the
    # components (I) and the derivative-by-component block (D)
    a, b = 2 * ncomp, 2 * nderiv
    macs_per_row = a * (a + 1) // 2 + b * a
    eng.set_norm_cache(1)
    warm = par.copy()
    warm[-1] *= 1.001                           # first build at a nearby lineshape point (kernel load)
    eng.nll_and_grad(warm)
    eng.nll_and_grad(par)                       # the timed build
    builds, _, build_ms = eng.norm_cache_stats()
    # coupling-only parameter changes: served from the matrices
    nc = sum(2 * r.n_coup for r in res)
    rng = np.random.default_rng(3)
    pts = [par.copy() for _ in range(16)]
    for q in pts:
        q[:nc] += 0.01 * rng.standard_normal(nc) * (W_free(res, floating)[:nc])
    for q in pts:
        eng.nll_and_grad(q)
    n = 2000
    t0 = time.perf_counter()
    for i in range(n):
        eng.nll_and_grad(pts[i % 16])
    ms = (time.perf_counter() - t0) / n * 1e3
    b2, hits, _ = eng.norm_cache_stats()
    eng.set_norm_cache(0)
    n_mc = eng.n[1]
    flop = 2.0 * macs_per_row * 2 * n_mc          # 2 flop per MAC, rows xi = +1, -1 per event
    mm = "f32" if precision == "fp32" else "f64"
    peak = MFMA_PEAK_TFLOPS[mm]
    return {"components": ncomp, "derivative_components": nderiv, "build_ms": build_ms,
            "kernel": "imatrix_kernel + reduce_values", "flop_per_build": flop,
            "achieved_tflops": flop / (build_ms * 1e-3) / 1e12, "mfma_dtype": mm,
            "peak_tflops_mfma": peak, "frac": flop / (build_ms * 1e-3) / 1e12 / peak,
            "cached_ms_per_step": ms, "cached_evals_per_s": 1e3 / ms, "builds": b2, "hits": hits}


def extension_legs(stream, data, mc, par, res, floating, steps: int = 1000, warmup: int = 300) -> dict:
    """Per-call NLL+gradient rate of the extensions at the benchmark sizes (same data and
    normalisation events, FP32): the signal + background mixture of Eq. 14 with per-event
    efficiency and background values, flavour-tagged events with mistag (the normalisation
    events evaluated at phi and -phi), and the LASS S-wave model (LASS + 8 K* + two Z, the
    K*(1410) and Z(4430) lineshapes floating), and the model whose Z has independent H'_{+1}
    and H'_{-1}.  The flavour-tagged and untagged calls are also timed with the
    interference-matrix cache (only the data events evaluated per call)."""
    import torch
    from paper_2007_14931_amd import kpsi
    from paper_2007_14931_amd import workloads as W
    rng = np.random.default_rng(11)
    nd, nm = data.shape[1], mc.shape[1]
    eps_d, eps_m = rng.uniform(0.3, 0.9, nd), rng.uniform(0.3, 0.9, nm)
    b_d, b_m = rng.uniform(0.2, 1.5, nd), rng.uniform(0.2, 1.5, nm)

    def timed(e, p):
        for _ in range(warmup):
            e.nll_and_grad(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            e.nll_and_grad(p)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        leg = timed_leg(e, p, grad=True)
        return {"ms_per_step": ms, "evals_per_s": 1e3 / ms, "kernel_ms": leg["kernel_ms_mean"],
                "kernel_ms_median": leg["kernel_ms_median"]}

    def cached_rate(e, p, n=1000):
        # calls at the lineshape point of the built matrices (the couplings move in a fit)
        for _ in range(100):
            e.nll_and_grad(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            e.nll_and_grad(p)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n * 1e3

    out = {}
    e = kpsi.Engine(0, "fp32", stream)
    e.set_model(W.KIN, res)
    e.set_floating([1 if r.name in floating else 0 for r in res])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    e.set_efficiency_values(eps_m)
    e.set_background(0.85, eps_d, b_d, b_m)
    out["mixture"] = {"model": "10 K* + Z(4430)", "purity": 0.85, **timed(e, par)}
    e.close()
    # flavour-tagged events (half of them the conjugate decay) with a 5% mistag fraction
    e = kpsi.Engine(0, "fp32", stream)
    e.set_model(W.KIN, res)
    e.set_floating([1 if r.name in floating else 0 for r in res])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    e.set_efficiency_values(eps_m)
    e.set_flavour(np.where(rng.random(nd) < 0.5, 1.0, -1.0), 0.05)
    out["flavour_tags"] = {"model": "10 K* + Z(4430)", "mistag": 0.05, **timed(e, par)}
    # the same with the interference-matrix cache: both flavours' normalisations come from the
    # +phi matrices, so a call evaluates only the data events (each at q phi and -q phi)
    e.set_norm_cache(1)
    e.nll_and_grad(par)
    out["flavour_tags"]["cached_ms_per_step"] = cached_rate(e, par)
    e.close()
    # the same events without tags, cached, for the ratio
    e = kpsi.Engine(0, "fp32", stream)
    e.set_model(W.KIN, res)
    e.set_floating([1 if r.name in floating else 0 for r in res])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    e.set_efficiency_values(eps_m)
    e.set_norm_cache(1)
    e.nll_and_grad(par)
    out["flavour_tags"]["untagged_cached_ms_per_step"] = cached_rate(e, par)
    e.close()
    # Z(4430) with H'_{+1} and H'_{-1} independent (no Eq. 11 relation)
    fres = W.model("full_zfree")
    fpar = W.params(fres, 37) + 0.05 * W.free_mask(fres, floating)
    e = kpsi.Engine(0, "fp32", stream)
    e.set_model(W.KIN, fres)
    e.set_floating([1 if r.name in floating else 0 for r in fres])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    out["free_z_helicities"] = {"model": "10 K* + Z(4430), H'+1 and H'-1 free", **timed(e, fpar)}
    e.close()
    lres = W.model("lass_full2z")
    lfl = ("K*(1410)", "Z(4430)")
    lpar = W.params(lres, 31) + 0.05 * W.free_mask(lres, lfl)
    e = kpsi.Engine(0, "fp32", stream)
    e.set_model(W.KIN, lres)
    e.set_floating([1 if r.name in lfl else 0 for r in lres])
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    out["lass"] = {"model": "LASS + 8 K* + Z(4430) + Z(4240)", **timed(e, lpar)}
    e.close()
    return out


def W_free(res, floating):
    from paper_2007_14931_amd import workloads as W
    return W.free_mask(res, floating).astype(float)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=10000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--ept", type=int, default=0, help="events per thread (0 = automatic)")
    ap.add_argument("--no-fit", action="store_true", help="skip the fit wall-time comparison")
    ap.add_argument("--ext-steps", type=int, default=1000,
                    help="timed calls per extension leg (mixture, flavour tags, LASS); 0 skips them")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 512 MiB device copy (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the per-call work shards by events with one small all-reduce of the reduced sums)", file=sys.stderr)
        return 2

    import torch
    from paper_2007_14931_amd import kpsi
    from paper_2007_14931_amd import workloads as W

    wl = W.WORKLOADS["full_grad_1m"]
    res = W.model(wl.model)
    truth = W.params(res, wl.coup_seed)
    floating = wl.floating
    flags = [1 if r.name in floating else 0 for r in res]
    K = W.KIN
    dev = torch.device("cuda:0")
    torch.cuda.init()
    stream = torch.cuda.current_stream(dev)

    t0 = time.perf_counter()
    gen = kpsi.Engine(0, "fp64", stream.cuda_stream)
    gen.set_model(K, res)
    mc = gen.generate_phsp(wl.mc_seed, wl.n_mc, W.PHSP_WMAX)
    # envelope for accept-reject: 1.5 x the largest density over a phase-space scan
    scan = gen.generate_phsp(wl.mc_seed + 7, 1_000_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    smax = 1.5 * float(gen.density(kpsi.DATA, truth).max())
    data, n_prop, n_over = gen.generate_model(truth, wl.data_seed, wl.n_data, W.PHSP_WMAX, smax)
    gen.close()
    del scan
    log(f"generated {wl.n_data} data events from {n_prop} proposals (over envelope: {n_over}), "
        f"{wl.n_mc} normalisation events in {time.perf_counter() - t0:.1f} s")

    def make(prec):
        e = kpsi.Engine(0, prec, stream.cuda_stream)
        e.set_model(K, res)
        e.set_floating(flags)
        e.load(kpsi.DATA, data)
        e.load(kpsi.NORM, mc)
        if args.ept:
            e.set_events_per_thread(args.ept)
        return e

    if args.copy_calib:
        a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)   # reads and writes 512 MiB once
        torch.cuda.synchronize()
        del a, b

    peaks = kpsi.measure_peaks(0)
    log(f"attainable peaks: {peaks}")
    par = truth + 0.05 * np.where(W.free_mask(res, floating), 1.0, 0.0)
    eng = make(args.precision)
    for _ in range(args.warmup):
        eng.nll_and_grad(par)
    # HIP events around the kernel on every TIMING_EVERY-th call of the timed region: the
    # kernel duration is measured live, without event records on every step
    eng.set_timing(TIMING_EVERY)
    eng.timing(reset=True)
    torch.cuda.synchronize()
    stamps = np.empty(args.steps + 1)
    t0 = time.perf_counter()
    stamps[0] = t0
    for i in range(args.steps):
        v, g = eng.nll_and_grad(par)   # returns after the call's stream synchronisation
        stamps[i + 1] = time.perf_counter()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    host_med_ms = float(np.median(np.diff(stamps))) * 1e3
    kmed_region = eng.timing_median()
    kms_region, kn_region = eng.timing(reset=True)
    ms_step = wall / args.steps * 1e3
    # kernel time: back-to-back launches of the same per-event work between HIP events on the
    # library's stream (the timed region's own every-10th-call events are kept as a cross-check)
    leg = timed_leg(eng, par, grad=True)
    kernel_ms, kmed, kn = leg["kernel_ms_mean"], leg["kernel_ms_median"], leg["timed_launches"]
    n_ev = wl.n_data + wl.n_mc
    dt = "f32" if args.precision == "fp32" else "f64"
    flops = FLOP_PER_EVENT["full_grad"] * n_ev
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    log(f"{args.precision}: {ms_step:.4f} ms/step host, kernel {kernel_ms:.4f} ms, nll {v:.6f}")

    # the other precision, for the record (same events, same parameters)
    other = "fp64" if args.precision == "fp32" else "fp32"
    e2 = make(other)
    v2, g2 = e2.nll_and_grad(par)
    leg2 = timed_leg(e2, par, grad=True)
    # likelihood-only calls (what every finite-difference step and cached data-only call runs)
    nll_legs = {}
    for prec, e_ in ((args.precision, eng), (other, e2)):
        lg = timed_leg(e_, par, grad=False)
        dtp = "f32" if prec == "fp32" else "f64"
        lg["achieved_gbs_algorithmic"] = ALG_BYTES_PER_EVENT[dtp] * n_ev / (lg["kernel_ms_mean"] * 1e-3) / 1e9
        nll_legs[prec] = lg
        log(f"{prec} likelihood-only: kernel {lg['kernel_ms_mean']:.4f} ms, host {lg['host_ms_per_call']:.4f} ms")
    e2.close()

    out = {
        "metric": "NLL+grad evals/s at 1M events, full K* model",
        "value": 1e3 / ms_step,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic: model accept-reject data and flat phase-space normalisation events from seeded "
                "Philox generators; seeded couplings",
        "config": {"workload": "full_grad_1m", "model": "10 K* + Z(4430)", "n_data": wl.n_data,
                   "n_norm": wl.n_mc, "free_params": int(W.free_mask(res, floating).sum()),
                   "floating_lineshapes": list(floating), "precision": args.precision,
                   "reductions": "f64 compensated"},
        "events_per_s": n_ev / (kernel_ms * 1e-3),
        "kernel_ms": kernel_ms,
        "kernel_ms_median": kmed,
        "kernel_timed_launches": kn,
        "kernel_ms_timed_region": kms_region / max(kn_region, 1),
        "kernel_ms_timed_region_median": kmed_region,
        "kernel_timed_calls_timed_region": kn_region,
        "host_ms_median": host_med_ms,
        "nll": v,
        "other_precision": {"precision": other, "ms_per_step": leg2["host_ms_per_call"],
                            "kernel_ms": leg2["kernel_ms_mean"], "kernel_ms_median": leg2["kernel_ms_median"],
                            "evals_per_s": 1e3 / leg2["host_ms_per_call"], "nll": v2,
                            "rel_nll_diff": abs(v2 - v) / abs(v)},
        "likelihood_only": nll_legs,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[dt],
                     "traffic": measured_traffic("paper_2007_14931_amd/csrc/kpsi_device.hip") if dt == "f32" else None,
                     "peak_unpacked": PEAK_TFLOPS_UNPACKED[dt],
                     "frac_unpacked": achieved / PEAK_TFLOPS_UNPACKED[dt],
                     "flop_per_event": FLOP_PER_EVENT["full_grad"], "events_per_launch": n_ev,
                     "kernel": "amp_kernel<GRAD>",
                     "measured_peaks": peaks,
                     "frac_measured_fma_peak": achieved / (peaks["fp32_fma_tflops"] if dt == "f32"
                                                           else peaks["fp64_fma_tflops"])},
    }
    out["norm_cache"] = norm_cache_leg(eng, par, res, floating, args.precision)
    if args.ext_steps > 0:
        out["extensions"] = extension_legs(stream.cuda_stream, data, mc, par, res, floating, args.ext_steps,
                                           max(10, args.ext_steps // 3))
    if not args.no_fit:
        out["fit"] = fit_comparison(make, truth, W.free_mask(res, floating), lambda p: W.canonical(res, p))
        out["fit_far_start"] = fit_far_start(make, truth, W.free_mask(res, floating), lambda p: W.canonical(res, p),
                                             sum(2 * r.n_coup for r in res))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(res, par, floating, wl.n_data, wl.n_mc, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    eng.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

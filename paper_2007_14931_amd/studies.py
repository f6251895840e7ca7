"""Studies of the efficiency model and the large fit, run on one GPU through libkpsi.

    python -m paper_2007_14931_amd.studies learned_eff   # learned efficiency vs 20^4 histogram
    python -m paper_2007_14931_amd.studies large_fit     # 10M + 20M events, two Z, end-to-end fit
    python -m paper_2007_14931_amd.studies pulls         # seeded pseudo-experiments of the 1M-event fit
    python -m paper_2007_14931_amd.studies z_sensitivity # Z fit fractions: null test and positive control
    python -m paper_2007_14931_amd.studies real_life     # efficiency + 15% background (Eq. 14) vs ideal fit
    python -m paper_2007_14931_amd.studies flavour_tags  # B0 + conjugate decays, 5% mistag, tagged fit
    python -m paper_2007_14931_amd.studies size_scan     # per-event kernel time against the event count
    python -m paper_2007_14931_amd.studies z_helicities  # Z couplings free of Eq. 11: likelihood-ratio test

Each prints one JSON line.  All events are synthetic, from the library's seeded generators:
flat phase space, accept labels under the seeded analytic acceptance (the paper's
efficiency templates are 2D x 2D histograms of simulated events; here the truth is known
exactly, so the efficiency models can be compared with it), and accept-reject data from
the model times the acceptance.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import kpsi
from . import workloads as W


def log(msg: str) -> None:
    print(f"[study] {msg}", file=sys.stderr, flush=True)


def _lohi():
    lo = np.array([W.M_LO, -1.0, -1.0, -math.pi])
    hi = np.array([W.M_HI, 1.0, 1.0, math.pi])
    return lo, hi


def _bins(ev: np.ndarray, nb, lo, hi):
    return tuple(np.clip(np.floor((ev[d] - lo[d]) / (hi[d] - lo[d]) * nb[d]).astype(int), 0, nb[d] - 1)
                 for d in range(4))


def train_efficiency(gen: "kpsi.Engine", coef, n_train: int, seed: int, epochs: int = 20, nb: int = 20):
    """Generate labelled phase-space events, train the network, fill the histogram."""
    t0 = time.perf_counter()
    train = gen.generate_phsp(seed, n_train, W.PHSP_WMAX)
    lab, _ = gen.accept_labels(seed + 1, train, coef)
    t1 = time.perf_counter()
    par, loss = gen.mlp_train(W.mlp_init(seed), train, lab, epochs=epochs, batch=32768, lr=3e-3)
    t2 = time.perf_counter()
    lo, hi = _lohi()
    table = gen.hist_efficiency(train, lab, (nb,) * 4, lo, hi)
    t3 = time.perf_counter()
    return par, table, {"train_events": n_train, "epochs": epochs, "final_loss": loss,
                        "accept_fraction": float(lab.float().mean().item()),
                        "generate_s": t1 - t0, "train_s": t2 - t1, "histogram_s": t3 - t2}


def efficiency_errors(gen, par, table, coef, n_val: int, seed: int):
    val = gen.generate_phsp(seed, n_val, W.PHSP_WMAX)
    _, eps_true = gen.accept_labels(seed + 1, val, coef)
    eps_true = eps_true.cpu().numpy()
    eps_nn = gen.mlp_eval(par, val).cpu().numpy()
    lo, hi = _lohi()
    eps_h = table[_bins(val.cpu().numpy(), table.shape, lo, hi)]
    return {"validation_events": n_val,
            "rms_network_minus_truth": float(np.sqrt(np.mean((eps_nn - eps_true) ** 2))),
            "rms_histogram_minus_truth": float(np.sqrt(np.mean((eps_h - eps_true) ** 2))),
            "max_abs_network_minus_truth": float(np.max(np.abs(eps_nn - eps_true)))}


def learned_eff(args) -> dict:
    import torch
    wl = W.WORKLOADS["learned_eff_1m"]
    res = W.model(wl.model)
    truth = W.params(res, wl.coup_seed)
    coef = W.acceptance_coefficients()
    stream = torch.cuda.current_stream().cuda_stream
    gen = kpsi.Engine(0, "fp64", stream)
    gen.set_model(W.KIN, res)
    par, table, train_info = train_efficiency(gen, coef, args.train, 2041, epochs=args.epochs)
    log(f"network trained: {train_info}")
    errs = efficiency_errors(gen, par, table, coef, 1_000_000, 2051)
    log(f"efficiency errors: {errs}")
    # data: accept-reject from eps_true x S; normalisation: flat phase space
    scan = gen.generate_phsp(2061, 1_000_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    smax = 1.5 * float(gen.density(kpsi.DATA, truth).max())
    data, nprop, nover = gen.generate_model(truth, wl.data_seed, wl.n_data, W.PHSP_WMAX, smax, coef)
    mc = gen.generate_phsp(wl.mc_seed, wl.n_mc, W.PHSP_WMAX)
    _, eps_mc = gen.accept_labels(2071, mc, coef)
    gen.close()
    mask = W.free_mask(res)
    fits = {}
    for name in ("true", "histogram", "network"):
        e = kpsi.Engine(0, "fp32", stream)
        e.set_model(W.KIN, res)
        e.load(kpsi.DATA, data)
        e.load(kpsi.NORM, mc)
        if name == "true":
            e.set_efficiency_values(eps_mc.cpu().numpy())
        elif name == "histogram":
            lo, hi = _lohi()
            e.set_efficiency_hist(table, lo, hi)
        else:
            e.set_efficiency_mlp(par)
        x, cov, r = e.migrad(truth, mask)
        fits[name] = (W.canonical(res, x), np.sqrt(np.abs(np.diag(cov))), r)
        log(f"fit with {name} efficiency: status {r.status} fmin {r.fmin:.3f} wall {r.wall_seconds:.3f} s")
        e.close()
    free = np.flatnonzero(mask)
    xt, st, _ = fits["true"]
    shifts = {}
    for name in ("histogram", "network"):
        d = np.abs(fits[name][0][free] - xt[free]) / st
        shifts[name] = {"mean_abs_shift_sigma": float(d.mean()), "max_abs_shift_sigma": float(d.max())}
    response = normalisation_response(res, data, mc, eps_mc.cpu().numpy(), par, table, coef, args, stream)
    return {"study": "learned_efficiency", "workload": "learned_eff_1m", "data_events": wl.n_data,
            "data_proposals": nprop, "norm_events": wl.n_mc, "free_params": int(mask.sum()),
            "training": train_info, "efficiency_errors": errs,
            "fit_status": {k: v[2].as_dict() for k, v in fits.items()},
            "fitted_parameter_shift_vs_true_efficiency": shifts,
            "normalisation_response": response}


def normalisation_response(res, data, mc, eps_true, par, table, coef, args, stream) -> dict:
    """How an efficiency estimate moves the fit, separated from the fit itself.  The data term of
    -2 ln L does not depend on the efficiency (ln eps(x_i) is dropped), so with the data fixed an
    estimate eps_X changes only the normalisation term: at the minimum x0 of the fit with the true
    efficiency the gradient changes by dg_X = g_X(x0) - g_true(x0), which moves the minimum by
    -(C/2) dg_X (C: that fit's HESSE covariance of -2 ln L), and the NLL by
    2 N_d ln(N_X / N_true).  Evaluated for the histogram and the network of the study and for a
    second histogram and network trained on an independent labelled sample: estimates whose errors
    are independent from bin to bin move the fit differently from sample to sample, while a smooth
    bias of the network moves it the same way."""
    mask = W.free_mask(res)
    free = np.flatnonzero(mask)
    e = kpsi.Engine(0, "fp64", stream)
    e.set_model(W.KIN, res)
    e.load(kpsi.DATA, data)
    e.load(kpsi.NORM, mc)
    e.set_efficiency_values(eps_true)
    x0, C, r = e.migrad(W.params(res, W.WORKLOADS["learned_eff_1m"].coup_seed), mask)
    sig = np.sqrt(np.abs(np.diag(C)))
    v_true, g_true = e.nll_and_grad(x0)
    nd = data.shape[1]
    gen = kpsi.Engine(0, "fp64", stream)
    gen.set_model(W.KIN, res)
    par2, table2, _ = train_efficiency(gen, coef, args.train, 2141, epochs=args.epochs)
    gen.close()
    lo, hi = _lohi()
    out, moved = {"fit_status": r.status}, {}
    for name, kind, obj in (("histogram", "hist", table), ("network", "mlp", par),
                            ("histogram_2", "hist", table2), ("network_2", "mlp", par2)):
        if kind == "hist":
            e.set_efficiency_hist(obj, lo, hi)
        else:
            e.set_efficiency_mlp(obj)
        v, g = e.nll_and_grad(x0)
        dg = (g - g_true)[free]
        shift = -(C @ dg) / 2.0 / sig
        moved[name] = shift
        out[name] = {"rel_normalisation_change": float(math.expm1((v - v_true) / (2.0 * nd))),
                     "rms_shift_sigma": float(np.sqrt(np.mean(shift ** 2))),
                     "max_abs_shift_sigma": float(np.max(np.abs(shift)))}
    e.close()
    corr = lambda a, b: float(np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b)))
    out["shift_correlation_histogram_vs_histogram_2"] = corr(moved["histogram"], moved["histogram_2"])
    out["shift_correlation_network_vs_network_2"] = corr(moved["network"], moved["network_2"])
    out["shift_correlation_histogram_vs_network"] = corr(moved["histogram"], moved["network"])
    log(f"normalisation response: {out}")
    return out


def large_fit(args) -> dict:
    import torch
    wl = W.WORKLOADS["large_2z_10m"]
    res = W.model(wl.model)
    truth = W.params(res, wl.coup_seed)
    floating = wl.floating
    flags = [1 if r.name in floating else 0 for r in res]
    coef = W.acceptance_coefficients()
    stream = torch.cuda.current_stream().cuda_stream
    n_data, n_mc = int(wl.n_data * args.scale), int(wl.n_mc * args.scale)
    t0 = time.perf_counter()
    gen = kpsi.Engine(0, "fp64", stream)
    gen.set_model(W.KIN, res)
    par, table, train_info = train_efficiency(gen, coef, args.train, 3041, epochs=args.epochs)
    scan = gen.generate_phsp(3061, 1_000_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    smax = 1.5 * float(gen.density(kpsi.DATA, truth).max())
    data, nprop, nover = gen.generate_model(truth, wl.data_seed, n_data, W.PHSP_WMAX, smax, coef)
    mc = gen.generate_phsp(wl.mc_seed, n_mc, W.PHSP_WMAX)
    gen.close()
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    log(f"prepared {n_data} data ({nprop} proposals) + {n_mc} normalisation events in {t_prep:.1f} s")
    mask = W.free_mask(res, floating)
    rng = np.random.default_rng(9)
    x0 = truth + 0.01 * rng.standard_normal(truth.size) * mask
    free = np.flatnonzero(mask)

    def engine(prec):
        e = kpsi.Engine(0, prec, stream)
        e.set_model(W.KIN, res)
        e.set_floating(flags)
        e.load(kpsi.DATA, data)
        e.load(kpsi.NORM, mc)
        e.set_efficiency_mlp(par)
        return e

    out = {}

    def record(name, x, cov, r, extra=None):
        out[name] = {**r.as_dict(), **(extra or {}), "x": W.canonical(res, x), "sig": np.sqrt(np.abs(np.diag(cov)))}
        log(f"{name}: status {r.status} fmin {r.fmin:.3f} edm {r.edm:.2e} migrad+hesse {r.wall_seconds:.2f} s "
            f"(nll {r.n_nll}, grad {r.n_grad})")

    # FP32 amplitudes with the device adjoint gradient
    t1 = time.perf_counter()
    e32 = engine("fp32")
    t_setup32 = time.perf_counter() - t1
    x32, cov32, r32 = e32.migrad(x0, mask)
    e32.close()
    record("fp32_analytic", x32, cov32, r32, {"setup_s": t_setup32})
    # FP64 polish: FP64 adjoint MIGRAD + HESSE from the FP32 minimum (the FP32 likelihood's
    # rounding noise at this size is above the EDM target)
    t1 = time.perf_counter()
    e64 = engine("fp64")
    t_setup64 = time.perf_counter() - t1
    xp, covp, rp = e64.migrad(x32, mask)
    record("fp64_analytic_polish", xp, covp, rp, {"setup_s": t_setup64,
                                                  "total_with_fp32_s": r32.wall_seconds + rp.wall_seconds})
    if not args.skip_fd:
        xf, covf, rf = e64.migrad(x0, mask, gradient=0)
        record("fp64_finite_difference", xf, covf, rf)
    e64.close()
    result = {"study": "large_fit", "workload": "large_2z_10m", "data_events": n_data, "norm_events": n_mc,
              "free_params": int(mask.sum()), "prepare_s": t_prep, "training": train_info}
    for k, v in out.items():
        result[k] = {kk: vv for kk, vv in v.items() if kk not in ("x", "sig")}
    if "fp64_finite_difference" in out:
        f = out["fp64_finite_difference"]
        for k in ("fp32_analytic", "fp64_analytic_polish"):
            d = np.abs(out[k]["x"][free] - f["x"][free]) / f["sig"]
            result[k]["max_param_diff_sigma_vs_fd"] = float(d.max())
            result[k]["median_param_diff_sigma_vs_fd"] = float(np.median(d))
        result["wall_ratio_fd_over_fp32_analytic"] = f["wall_seconds"] / out["fp32_analytic"]["wall_seconds"]
        result["wall_ratio_fd_over_fp32_plus_polish"] = f["wall_seconds"] / (
            out["fp32_analytic"]["wall_seconds"] + out["fp64_analytic_polish"]["wall_seconds"])
    best = out["fp64_analytic_polish"]
    pulls = (best["x"][free] - W.canonical(res, truth)[free]) / best["sig"]
    nc = W.n_params(res) - 2 * len(res)
    for k, i in enumerate(free):
        if i < nc and i % 2 == 1:
            pulls[k] = math.remainder(best["x"][i] - W.canonical(res, truth)[i], 2 * math.pi) / best["sig"][k]
    result["pull_mean"] = float(pulls.mean())
    result["pull_rms"] = float(np.sqrt(np.mean(pulls ** 2)))
    return result


def cartesian_pulls(res, x, cov, truth, mask) -> np.ndarray:
    """Pulls of the free parameters with every free coupling taken as (Re H, Im H) instead of
    (magnitude, phase): near a small magnitude the likelihood is close to quadratic in H but not
    in (r, phi).  The HESSE covariance is carried over with the Jacobian of H = r e^{i phi} at the
    fitted point (exact for the Hessian at a minimum).  cov is over the free parameters."""
    nc = W.n_params(res) - 2 * len(res)
    free = np.flatnonzero(mask)
    out = []
    k = 0
    while k < len(free):
        i = free[k]
        if i < nc and i % 2 == 0 and k + 1 < len(free) and free[k + 1] == i + 1:
            r, ph = x[i], x[i + 1]
            J = np.array([[math.cos(ph), -r * math.sin(ph)], [math.sin(ph), r * math.cos(ph)]])
            C2 = J @ cov[np.ix_([k, k + 1], [k, k + 1])] @ J.T
            h = r * complex(math.cos(ph), math.sin(ph))
            h0 = truth[i] * complex(math.cos(truth[i + 1]), math.sin(truth[i + 1]))
            out += [(h.real - h0.real) / math.sqrt(abs(C2[0, 0])), (h.imag - h0.imag) / math.sqrt(abs(C2[1, 1]))]
            k += 2
        else:
            out.append((x[i] - truth[i]) / math.sqrt(abs(cov[k, k])))
            k += 1
    return np.array(out)


def pulls(args) -> dict:
    """Pseudo-experiments of the 1M-event benchmark fit: each seed draws a new data sample at
    the truth point, fits it (FP32, device adjoint gradient, MIGRAD + HESSE) from a perturbed
    start, and records (fitted - true) / sigma for every free parameter."""
    import torch
    wl = W.WORKLOADS["full_grad_1m"]
    res = W.model(wl.model)
    truth = W.params(res, wl.coup_seed)
    flags = [1 if r.name in wl.floating else 0 for r in res]
    mask = W.free_mask(res, wl.floating)
    free = np.flatnonzero(mask)
    stream = torch.cuda.current_stream().cuda_stream
    gen = kpsi.Engine(0, "fp64", stream)
    gen.set_model(W.KIN, res)
    scan = gen.generate_phsp(4061, 1_000_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    smax = 1.5 * float(gen.density(kpsi.DATA, truth).max())
    n_mc = int(args.norm_events) if args.norm_events else wl.n_mc
    n_flat = n_mc if args.flat_fraction >= 1.0 else int(round(args.flat_fraction * n_mc))
    mc = gen.generate_phsp(wl.mc_seed, n_flat, W.PHSP_WMAX)
    if n_flat < n_mc:
        # the rest of the normalisation set drawn from the model at the truth point (importance sampling)
        mc_m, _, _ = gen.generate_model(truth, wl.mc_seed + 1, n_mc - n_flat, W.PHSP_WMAX, smax)
        mc = torch.cat([mc, mc_m], dim=1).contiguous()
        torch.cuda.synchronize()   # written on torch's stream, read on the engine's stream
        del mc_m
    e = kpsi.Engine(0, "fp32", stream)
    e.set_model(W.KIN, res)
    e.set_floating(flags)
    e.load(kpsi.NORM, mc)
    if n_flat < n_mc:
        e.set_norm_mixture(truth, n_flat)
    ct = W.canonical(res, truth)
    P, PC, statuses, walls = [], [], [], []
    n_data = int(args.data_events)
    for s in range(args.seeds):
        data, _, _ = gen.generate_model(truth, 5000 + s, n_data, W.PHSP_WMAX, smax)
        e.load(kpsi.DATA, data)
        rng = np.random.default_rng(100 + s)
        x0 = truth + 0.02 * rng.standard_normal(truth.size) * mask
        x, cov, r = e.migrad(x0, mask)
        sig = np.sqrt(np.abs(np.diag(cov)))
        d = W.canonical(res, x)[free] - ct[free]
        nc = W.n_params(res) - 2 * len(res)
        for k, i in enumerate(free):   # coupling phases are compared modulo 2 pi
            if i < nc and i % 2 == 1:
                d[k] = math.remainder(d[k], 2 * math.pi)
        P.append(d / sig)
        PC.append(cartesian_pulls(res, x, cov, truth, mask))
        if not np.all(np.isfinite(d / sig)):
            log(f"seed {s}: non-finite pulls at {free[~np.isfinite(d / sig)].tolist()}; "
                f"diag cov there {np.diag(cov)[~np.isfinite(d / sig)].tolist()}")
        statuses.append(r.status)
        walls.append(r.wall_seconds)
        log(f"seed {s}: status {r.status} wall {r.wall_seconds:.3f} s  rms pull {np.sqrt(np.mean((d / sig) ** 2)):.2f}")
        del data
    e.close()
    gen.close()
    P = np.array(P)
    PC = np.array(PC)
    mc_, sdc = PC.mean(0), PC.std(0, ddof=1)
    log(f"cartesian pulls: max |mean| {np.max(np.abs(mc_)):.2f}, rms of means {np.sqrt(np.mean(mc_ ** 2)):.2f}, "
        f"widths {sdc.min():.2f} - {sdc.max():.2f} (median {np.median(sdc):.2f}); statuses {sorted(set(statuses))}")
    m, sd = P.mean(0), P.std(0, ddof=1)
    log(f"pulls: {n_data} data, {n_mc} normalisation ({n_flat} flat): max |mean| {np.max(np.abs(m)):.2f}, "
        f"rms of means {np.sqrt(np.mean(m ** 2)):.2f} (expected {1 / math.sqrt(args.seeds):.2f}), "
        f"widths {sd.min():.2f} - {sd.max():.2f} (median {np.median(sd):.2f})")
    return {"study": "pulls", "workload": "full_grad_1m", "seeds": args.seeds, "free_params": int(mask.sum()),
            "data_events": n_data, "norm_events": n_mc, "flat_norm_events": n_flat,
            "max_abs_param_mean": float(np.max(np.abs(m))), "rms_param_mean": float(np.sqrt(np.mean(m ** 2))),
            "cartesian_per_param_mean": [float(v) for v in mc_], "cartesian_per_param_std": [float(v) for v in sdc],
            "cartesian_max_abs_mean": float(np.max(np.abs(mc_))),
            "cartesian_rms_mean": float(np.sqrt(np.mean(mc_ ** 2))), "cartesian_median_width": float(np.median(sdc)),
            "median_param_width": float(np.median(sd)),
            "fit_status": statuses, "median_fit_wall_s": float(np.median(walls)),
            "pull_mean_over_params": float(P.mean()), "pull_rms_over_params": float(np.sqrt((P ** 2).mean())),
            "per_param_mean": [float(v) for v in P.mean(0)], "per_param_std": [float(v) for v in P.std(0)],
            "frac_within_2sigma": float((np.abs(P) < 2).mean())}


def z_sensitivity(args) -> dict:
    """Sensitivity to Z contributions (Results, sensitivity of the fitter to Z contributions):
    pseudo-data from the ten K* alone are fitted with the ten K* + Z(4430) + Z(4240) model (the
    Z fit fractions should come out near zero); the same null test with the LASS S-wave (Eq. 7-8)
    in place of K0*(800) and K0*(1430) in both generation and fit; and, as a positive control,
    pseudo-data with both Z at seeded couplings fitted with the same model (the fitted Z
    fractions should match the generated ones).  Fits: FP32 adjoint MIGRAD, then an FP64 adjoint
    polish with HESSE; Z masses and widths fixed."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    n_data, n_mc = int(args.data_events), int(args.norm_events) if args.norm_events else 2_000_000
    out = {"study": "z_sensitivity", "data_events": n_data, "norm_events": n_mc}
    plan = (("full2z", "10 K* + Z(4430) + Z(4240)", ("kstar_only_data", "with_z_data")),
            ("lass_full2z", "LASS + 8 K* + Z(4430) + Z(4240)", ("lass_kstar_only_data",)))
    for model, label, cases in plan:
        res = W.model(model)
        truth = W.params(res, 31)
        iz = [i for i, r in enumerate(res) if r.chain == 1]
        zoff = [W.coupling_offset(res, i) for i in iz]
        null = truth.copy()
        for o in zoff:
            null[o] = 0.0
            null[o + 2] = 0.0
        gen = kpsi.Engine(0, "fp64", stream)
        gen.set_model(W.KIN, res)
        mc = gen.generate_phsp(5201, n_mc, W.PHSP_WMAX)
        scan = gen.generate_phsp(5202, 1_000_000, W.PHSP_WMAX)
        gen.load(kpsi.DATA, scan)
        gen.load(kpsi.NORM, mc)
        if "with_z_data" in cases:
            # positive control at the few-percent Z fractions the paper quotes for its efficiency
            # and background study (3.5% and 1.2%): scale each Z's couplings until its fraction matches
            target = {res[iz[0]].name: 0.035, res[iz[1]].name: 0.012}
            for _ in range(4):
                ff, _ = gen.fit_fractions(truth)
                for i, o in zip(iz, zoff):
                    f = math.sqrt(target[res[i].name] / ff[i])
                    truth[o] *= f
                    truth[o + 2] *= f
        mask = W.free_mask(res)
        for case in cases:
            point = truth if case == "with_z_data" else null
            smax = 1.5 * float(gen.density(kpsi.DATA, point).max())
            data, _, _ = gen.generate_model(point, 5300 + len(out), n_data, W.PHSP_WMAX, smax)
            ff_true, _ = gen.fit_fractions(point)
            start = point.copy()
            for o in zoff:   # Z couplings start small but non-zero
                start[o] = max(start[o], 0.05)
                start[o + 2] = max(start[o + 2], 0.05)
            fits = {}
            for prec in ("fp32", "fp64"):
                e = kpsi.Engine(0, prec, stream)
                e.set_model(W.KIN, res)
                e.load(kpsi.DATA, data)
                e.load(kpsi.NORM, mc)
                x, cov, r = e.migrad(start, mask)
                e.close()
                fits[prec] = (x, r)
                start = x
            x, r = fits["fp64"]
            ff, tot = gen.fit_fractions(x)
            rec = {"model": label,
                   "fit_status": {p: fits[p][1].status for p in fits},
                   "fit_wall_s": {p: fits[p][1].wall_seconds for p in fits},
                   "ff_generated": {res[i].name: float(ff_true[i]) for i in iz},
                   "ff_fitted": {res[i].name: float(ff[i]) for i in iz},
                   "ff_sum_fitted": tot,
                   "kstar_ff_max_abs_diff": float(np.max(np.abs(np.delete(ff - ff_true, iz))))}
            log(f"{case}: {rec}")
            out[case] = rec
            del data
        gen.close()
    return out


def _acceptance_templates(eng, coef, nb=(40, 40, 40, 40)):
    """2D x 2D templates of the seeded acceptance at bin centres.  The acceptance is a product
    of one-dimensional factors, so eps(m, cK, cJ, phi) = A(m, cK) B(cJ, phi) exactly, with
    A = eps(., ., cJ0, phi0) and B = eps(m0, cK0, ., .) / eps(m0, cK0, cJ0, phi0)."""
    import torch
    lo = np.array([W.M_LO, -1.0, -1.0, -math.pi])
    hi = np.array([W.M_HI, 1.0, 1.0, math.pi])
    cen = [lo[d] + (np.arange(nb[d]) + 0.5) / nb[d] * (hi[d] - lo[d]) for d in range(4)]
    ref = [0.5 * (lo[d] + hi[d]) for d in range(4)]
    g1 = np.stack(np.meshgrid(cen[0], cen[1], indexing="ij")).reshape(2, -1)
    g2 = np.stack(np.meshgrid(cen[2], cen[3], indexing="ij")).reshape(2, -1)
    ev1 = np.stack([g1[0], g1[1], np.full(g1.shape[1], ref[2]), np.full(g1.shape[1], ref[3])])
    ev2 = np.stack([np.full(g2.shape[1], ref[0]), np.full(g2.shape[1], ref[1]), g2[0], g2[1]])
    ev0 = np.array([[ref[0]], [ref[1]], [ref[2]], [ref[3]]])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    _, e1 = eng.accept_labels(1, dev(ev1), coef)
    _, e2 = eng.accept_labels(1, dev(ev2), coef)
    _, e0 = eng.accept_labels(1, dev(ev0), coef)
    t1 = e1.cpu().numpy().reshape(nb[0], nb[1])
    t2 = (e2.cpu().numpy() / float(e0.cpu().numpy()[0])).reshape(nb[2], nb[3])
    return t1.astype(np.float32), t2.astype(np.float32)


def real_life(args) -> dict:
    """The paper's real-life test (Results, applicability to real-life use cases): pseudo-data
    of ten K* + two Z with the relative efficiency applied and a 15% background, fitted with
    the Eq. 14 mixture (efficiency and background as 2D x 2D templates, purity fixed), against
    the ideal fit of signal-only pseudo-data without efficiency."""
    import torch
    res = W.model("full2z")
    truth = W.params(res, 31)
    iz = [i for i, r in enumerate(res) if r.chain == 1]
    zoff = [W.coupling_offset(res, i) for i in iz]
    coef = W.acceptance_coefficients()
    purity = 0.85
    n_data, n_mc = int(args.data_events), int(args.norm_events) if args.norm_events else 2_000_000
    stream = torch.cuda.current_stream().cuda_stream
    gen = kpsi.Engine(0, "fp64", stream)
    gen.set_model(W.KIN, res)
    mc = gen.generate_phsp(6201, n_mc, W.PHSP_WMAX)
    gen.load(kpsi.NORM, mc)
    target = {res[iz[0]].name: 0.035, res[iz[1]].name: 0.012}   # the paper's few-percent Z fractions
    for _ in range(4):
        ff, _ = gen.fit_fractions(truth)
        for i, o in zip(iz, zoff):
            f = math.sqrt(target[res[i].name] / ff[i])
            truth[o] *= f
            truth[o + 2] *= f
    scan = gen.generate_phsp(6202, 1_000_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    smax = 1.5 * float(gen.density(kpsi.DATA, truth).max())
    n_sig = int(round(purity * n_data))
    sig, _, _ = gen.generate_model(truth, 6203, n_sig, W.PHSP_WMAX, smax, coef)
    ideal, _, _ = gen.generate_model(truth, 6204, n_data, W.PHSP_WMAX, smax)
    # background: accept-reject of the template shape over flat phase space
    tb1, tb2 = W.background_templates()
    prop = gen.generate_phsp(6205, 8 * (n_data - n_sig), W.PHSP_WMAX)
    gen.load(kpsi.DATA, prop)
    bp = gen.template_values(kpsi.DATA, tb1, tb2)
    rng = np.random.Generator(np.random.PCG64(6206))
    keep = np.flatnonzero(rng.uniform(size=bp.size) * bp.max() < bp)[: n_data - n_sig]
    bkg = prop[:, torch.from_numpy(keep).to(prop.device)]
    data = torch.cat([sig, bkg], dim=1).contiguous()
    te1, te2 = _acceptance_templates(gen, coef)
    gen.load(kpsi.DATA, data)
    gen.load(kpsi.NORM, mc)
    eps_d = gen.template_values(kpsi.DATA, te1, te2)
    eps_m = gen.template_values(kpsi.NORM, te1, te2)
    b_d = gen.template_values(kpsi.DATA, tb1, tb2)
    b_m = gen.template_values(kpsi.NORM, tb1, tb2)
    gen.close()
    mask = W.free_mask(res)
    free = np.flatnonzero(mask)
    ct = W.canonical(res, truth)
    nc = W.n_params(res) - 2 * len(res)

    def fit(events, with_mixture):
        start = truth.copy()
        out = None
        for prec in ("fp32", "fp64"):
            e = kpsi.Engine(0, prec, stream)
            e.set_model(W.KIN, res)
            e.load(kpsi.DATA, events)
            e.load(kpsi.NORM, mc)
            if with_mixture:
                e.set_efficiency_values(eps_m)
                e.set_background(purity, eps_d, b_d, b_m)
            x, cov, r = e.migrad(start, mask)
            ff, _ = e.fit_fractions(x)
            e.close()
            start = x
            out = (W.canonical(res, x), np.sqrt(np.abs(np.diag(cov))), r, ff)
        return out

    x_r, s_r, r_r, ff_r = fit(data, True)
    x_i, s_i, r_i, ff_i = fit(ideal, False)

    def pulls(x, s):
        d = x[free] - ct[free]
        for k, i in enumerate(free):
            if i < nc and i % 2 == 1:
                d[k] = math.remainder(d[k], 2 * math.pi)
        return d / s
    p_r, p_i = pulls(x_r, s_r), pulls(x_i, s_i)
    return {"study": "real_life", "data_events": n_data, "signal_events": n_sig, "background_events": int(keep.size),
            "norm_events": n_mc, "purity": purity, "free_params": int(mask.sum()),
            "templates": "2D (m_Kpi, cos theta_K*) x 2D (cos theta_J/psi, phi), 40 x 40 bins each",
            "real_life_fit": {"status": r_r.status, "wall_s": r_r.wall_seconds, "pull_mean": float(p_r.mean()),
                              "pull_rms": float(np.sqrt((p_r ** 2).mean())),
                              "ff_Z": {res[i].name: float(ff_r[i]) for i in iz}},
            "ideal_fit": {"status": r_i.status, "wall_s": r_i.wall_seconds, "pull_mean": float(p_i.mean()),
                          "pull_rms": float(np.sqrt((p_i ** 2).mean())),
                          "ff_Z": {res[i].name: float(ff_i[i]) for i in iz}},
            "ff_Z_generated": target,
            "real_minus_ideal_sigma_median": float(np.median(np.abs(x_r[free] - x_i[free]) / s_r)),
            "real_minus_ideal_sigma_max": float(np.max(np.abs(x_r[free] - x_i[free]) / s_r))}


def flavour_tags(args) -> dict:
    """Flavour-tagged pseudo-data (text after Eq. 12): half of the events are B0 decays drawn
    from S, half are conjugate decays drawn from S and mirrored in phi; each tag is flipped with
    the mistag probability w = 0.05.  Fits: the tagged likelihood with w fixed (FP32 adjoint
    MIGRAD, then an FP64 polish with HESSE), and, as a control, the same events all taken as
    B0.  Reports the pulls against the generated point."""
    import torch
    res = W.model("full")
    truth = W.params(res, 31)
    w = 0.05
    n_data, n_mc = int(args.data_events), int(args.norm_events) if args.norm_events else 2_000_000
    stream = torch.cuda.current_stream().cuda_stream
    gen = kpsi.Engine(0, "fp64", stream)
    gen.set_model(W.KIN, res)
    mc = gen.generate_phsp(7101, n_mc, W.PHSP_WMAX)
    scan = gen.generate_phsp(7102, 1_000_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    smax = 1.5 * float(gen.density(kpsi.DATA, truth).max())
    n_b0 = n_data // 2
    b0, _, _ = gen.generate_model(truth, 7103, n_b0, W.PHSP_WMAX, smax)
    bb, _, _ = gen.generate_model(truth, 7104, n_data - n_b0, W.PHSP_WMAX, smax)
    bb = bb.clone()
    bb[3] = -bb[3]   # the conjugate decay's density is S(-phi)
    data = torch.cat([b0, bb], dim=1).contiguous()
    gen.close()
    flavour = np.concatenate([np.ones(n_b0), -np.ones(n_data - n_b0)])
    rng = np.random.Generator(np.random.PCG64(7105))
    mistagged = rng.uniform(size=n_data) < w
    tags = np.where(mistagged, -flavour, flavour)
    mask = W.free_mask(res)
    free = np.flatnonzero(mask)
    ct = W.canonical(res, truth)
    nc = W.n_params(res) - 2 * len(res)

    def fit(tagged):
        start = truth.copy()
        out = None
        for prec in ("fp32", "fp64"):
            e = kpsi.Engine(0, prec, stream)
            e.set_model(W.KIN, res)
            e.load(kpsi.DATA, data)
            e.load(kpsi.NORM, mc)
            if tagged:
                e.set_flavour(tags, w)
            x, cov, r = e.migrad(start, mask)
            e.close()
            start = x
            out = (W.canonical(res, x), np.sqrt(np.abs(np.diag(cov))), r)
        return out

    def pulls(x, s):
        d = x[free] - ct[free]
        for k, i in enumerate(free):
            if i < nc and i % 2 == 1:
                d[k] = math.remainder(d[k], 2 * math.pi)
        return d / s

    out = {"study": "flavour_tags", "data_events": n_data, "b0_events": n_b0, "mistag": w,
           "mistagged_events": int(mistagged.sum()), "norm_events": n_mc, "free_params": int(mask.sum()),
           "model": "10 K* + Z(4430)"}
    for name, tagged in (("tagged_fit", True), ("untagged_control_fit", False)):
        x, s, r = fit(tagged)
        p = pulls(x, s)
        out[name] = {"status": r.status, "wall_s": r.wall_seconds, "pull_mean": float(p.mean()),
                     "pull_rms": float(np.sqrt((p ** 2).mean())), "pull_max_abs": float(np.max(np.abs(p)))}
        log(f"{name}: {out[name]}")
    return out


def z_helicities(args) -> dict:
    """Z helicity couplings free of the parity relation (Eq. 11; the Discussion's unconstrained Z
    couplings).  Pseudo-data of the ten K* + Z(4430) model at 3.5% Z fit fraction, generated once
    with H'_{-1} = H'_{+1} (parity conserved in Z -> J/psi pi) and once with H'_{-1} = 0.5 H'_{+1}
    e^{i}, are fitted with the free and with the constrained model (FP32 adjoint MIGRAD, FP64
    adjoint polish, HESSE).  Reported: the fitted difference H'_{-1} - H'_{+1} and its chi^2 from
    the HESSE covariance (2 degrees of freedom), and the likelihood ratio -2 ln(L_constrained /
    L_free), chi^2 with 2 degrees of freedom when the relation holds."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    n_data = int(args.data_events)
    n_mc = int(args.norm_events) if args.norm_events else 2_000_000
    res_f, res_c = W.model("full_zfree"), W.model("full")
    iz = len(res_f) - 1
    zf = W.coupling_offset(res_f, iz)
    gen = kpsi.Engine(0, "fp64", stream)
    gen.set_model(W.KIN, res_f)
    mc = gen.generate_phsp(5601, n_mc, W.PHSP_WMAX)
    scan = gen.generate_phsp(5602, 1_000_000, W.PHSP_WMAX)
    gen.load(kpsi.DATA, scan)
    gen.load(kpsi.NORM, mc)
    base = W.params(res_f, 41)
    out = {"study": "z_helicities", "data_events": n_data, "norm_events": n_mc}

    def constrained_of(p):   # drop H'_{-1}
        return np.concatenate([p[: zf + 4], p[zf + 6:]])

    for case, (ratio, dphase) in (("parity_conserving", (1.0, 0.0)), ("parity_violating", (0.5, 1.0))):
        truth = base.copy()
        truth[zf + 4] = ratio * truth[zf + 2]
        truth[zf + 5] = truth[zf + 3] + dphase
        for _ in range(4):   # scale the Z couplings to a 3.5% fit fraction
            ff, _ = gen.fit_fractions(truth)
            f = math.sqrt(0.035 / ff[iz])
            for k in (0, 2, 4):
                truth[zf + k] *= f
        smax = 1.5 * float(gen.density(kpsi.DATA, truth).max())
        data, _, _ = gen.generate_model(truth, 5700 + len(out), n_data, W.PHSP_WMAX, smax)
        rec = {}
        for label, res, start, mask in (("free", res_f, truth.copy(), W.free_mask(res_f)),
                                        ("constrained", res_c, constrained_of(truth), W.free_mask(res_c))):
            x = start
            for prec in ("fp32", "fp64"):
                e = kpsi.Engine(0, prec, stream)
                e.set_model(W.KIN, res)
                e.load(kpsi.DATA, data)
                e.load(kpsi.NORM, mc)
                x, _, r = e.migrad(x, mask)
                if prec == "fp64":
                    cov, rh = e.hesse(x, mask)
                e.close()
            rec[label] = {"x": x, "fmin": r.fmin, "status": r.status, "hesse_status": rh.status, "cov": cov,
                          "mask": mask}
        x, cov, mask = rec["free"]["x"], rec["free"]["cov"], rec["free"]["mask"]
        free = list(np.flatnonzero(mask))
        ks = [free.index(zf + k) for k in (2, 3, 4, 5)]
        rp, pp, rm, pm = (x[zf + k] for k in (2, 3, 4, 5))
        d = np.array([rm * math.cos(pm) - rp * math.cos(pp), rm * math.sin(pm) - rp * math.sin(pp)])
        J = np.array([[-math.cos(pp), rp * math.sin(pp), math.cos(pm), -rm * math.sin(pm)],
                      [-math.sin(pp), -rp * math.cos(pp), math.sin(pm), rm * math.cos(pm)]])
        cd = J @ cov[np.ix_(ks, ks)] @ J.T
        chi2 = float(d @ np.linalg.solve(cd, d))
        dt = truth[zf + 4] * np.exp(1j * truth[zf + 5]) - truth[zf + 2] * np.exp(1j * truth[zf + 3])
        out[case] = {"generated_ratio": ratio, "generated_phase_offset": dphase,
                     "generated_difference": [float(dt.real), float(dt.imag)],
                     "fitted_difference": d.tolist(), "difference_errors": np.sqrt(np.diag(cd)).tolist(),
                     "difference_chi2_2dof": chi2,
                     "likelihood_ratio": rec["constrained"]["fmin"] - rec["free"]["fmin"],
                     "fit_status": {k: (rec[k]["status"], rec[k]["hesse_status"]) for k in rec},
                     "ff_z_generated": float(gen.fit_fractions(truth)[0][iz])}
        log(f"{case}: {out[case]}")
        del data
    gen.close()
    return out


def size_scan(args) -> dict:
    """Kernel time of the FP32 likelihood-only and gradient passes (kpsi_time_kernel: medians of
    five batches of 50 back-to-back launches) for 1/8 to 4 times the benchmark's 1e6 + 2e6 phase-
    space events of the full model, and the rate a plain torch reduction reaches over the same
    numbers of bytes (64 per event): where the record stops fitting the last-level cache."""
    import torch
    res = W.model("full")
    fl = ("K*(1410)", "Z(4430)")
    par = W.params(res, seed=11)
    rows = []
    for nd in (125_000, 250_000, 500_000, 1_000_000, 2_000_000, 4_000_000):
        e = kpsi.Engine(0, "fp32")
        e.set_model(W.KIN, res)
        e.set_floating([1 if r.name in fl else 0 for r in res])
        mc = e.generate_phsp(1234, 2 * nd, W.PHSP_WMAX)
        data = e.generate_phsp(4321, nd, W.PHSP_WMAX)
        torch.cuda.synchronize()
        e.load(kpsi.DATA, data)
        e.load(kpsi.NORM, mc)
        del mc, data
        e.nll_and_grad(par)
        t = {}
        for grad in (False, True):
            t["grad" if grad else "nll"] = float(np.median([e.time_kernel(par, grad=grad, reps=50) for _ in range(5)]))
        e.close()
        torch.cuda.empty_cache()
        nbytes = 3 * nd * 64
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        for _ in range(5):
            x.sum()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(50):
            x.sum()
        t1.record()
        torch.cuda.synchronize()
        sum_ms = t0.elapsed_time(t1) / 50
        del x
        torch.cuda.empty_cache()
        row = {"events": 3 * nd, "record_mb": nbytes / 1e6, "nll_us": 1e3 * t["nll"], "grad_us": 1e3 * t["grad"],
               "nll_tbs": nbytes / (t["nll"] * 1e-3) / 1e12, "torch_sum_us": 1e3 * sum_ms,
               "torch_sum_tbs": nbytes / (sum_ms * 1e-3) / 1e12}
        log(json.dumps(row))
        rows.append(row)
    return {"study": "size_scan", "rows": rows}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["learned_eff", "large_fit", "pulls", "z_sensitivity", "real_life",
                                      "flavour_tags", "size_scan", "z_helicities"])
    ap.add_argument("--train", type=int, default=5_000_000, help="labelled training events")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the large-fit event counts")
    ap.add_argument("--skip-fd", action="store_true")
    ap.add_argument("--seeds", type=int, default=20)
    ap.add_argument("--data-events", type=float, default=1e6)
    ap.add_argument("--norm-events", type=float, default=0, help="normalisation events of the pull study "
                    "(default: the workload's)")
    ap.add_argument("--flat-fraction", type=float, default=1.0,
                    help="fraction of the pull study's normalisation events drawn flat; the rest are drawn from "
                         "the model at the truth point and weighted back (kpsi_set_norm_mixture)")
    args = ap.parse_args()
    out = {"learned_eff": learned_eff, "large_fit": large_fit, "pulls": pulls,
           "z_sensitivity": z_sensitivity, "real_life": real_life, "flavour_tags": flavour_tags,
           "size_scan": size_scan, "z_helicities": z_helicities}[args.study](args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

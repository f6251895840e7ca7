"""Python binding of libkpsi (include/kpsi.h): argument marshalling only.

Every step of the likelihood runs in the HIP library; this module converts numpy
arrays and torch tensors to pointers, checks status codes and raises on errors.
PyTorch is used for device memory (generator outputs, borrowed event columns) and
streams.  There is no CPU fallback: if libkpsi.so is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpsi.so")

KPSI_OK, KPSI_E_ARG, KPSI_E_STATE, KPSI_E_HIP, KPSI_E_OOM, KPSI_E_NONFINITE, KPSI_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
DATA, NORM = 0, 1
_STATUS = {0: "OK", -1: "E_ARG", -2: "E_STATE", -3: "E_HIP", -4: "E_OOM", -5: "E_NONFINITE", -6: "E_UNSUPPORTED"}

# Every entry point of include/kpsi.h.
EXPORTS = [
    "kpsi_create", "kpsi_destroy", "kpsi_set_model", "kpsi_n_params", "kpsi_set_floating", "kpsi_load_events",
    "kpsi_load_events_device", "kpsi_set_efficiency_flat", "kpsi_set_efficiency_values", "kpsi_set_efficiency_hist",
    "kpsi_nll", "kpsi_nll_and_grad", "kpsi_density", "kpsi_invariants", "kpsi_generate_phsp", "kpsi_generate_model",
    "kpsi_set_timing", "kpsi_timing", "kpsi_timing_median", "kpsi_set_events_per_thread", "kpsi_last_error",
    "kpsi_fit_default_options", "kpsi_migrad", "kpsi_migrad_limited", "kpsi_hesse", "kpsi_set_norm_cache", "kpsi_norm_cache_stats",
    "kpsi_mlp_default_options", "kpsi_accept_labels", "kpsi_hist_efficiency", "kpsi_mlp_grad", "kpsi_mlp_train",
    "kpsi_mlp_eval", "kpsi_set_efficiency_mlp", "kpsi_fit_fractions", "kpsi_measure_peaks", "kpsi_set_background",
    "kpsi_template_values", "kpsi_set_flavour", "kpsi_set_constraints", "kpsi_nll_and_grad_noalloc",
    "kpsi_set_norm_mixture", "kpsi_time_kernel",
]
MLP_NP = 4545


class KpsiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Kinematics(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("m_b", "m_jpsi", "m_k", "m_pi", "r_b", "r_r")]


class Resonance(C.Structure):
    _fields_ = [("chain", C.c_int), ("spin", C.c_int), ("parity", C.c_int), ("lb", C.c_int), ("lr", C.c_int),
                ("mass", C.c_double), ("width", C.c_double), ("shape", C.c_int), ("lass_a", C.c_double),
                ("lass_b", C.c_double), ("hel_free", C.c_int)]


class FitOptions(C.Structure):
    _fields_ = [("max_calls", C.c_int64), ("tolerance", C.c_double), ("up", C.c_double), ("gradient", C.c_int),
                ("fd_rel_step", C.c_double), ("hesse", C.c_int)]


class FitResult(C.Structure):
    _fields_ = [("fmin", C.c_double), ("edm", C.c_double), ("wall_seconds", C.c_double), ("n_nll", C.c_int64),
                ("n_grad", C.c_int64), ("n_iter", C.c_int), ("status", C.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Peaks(C.Structure):
    _fields_ = [("fp32_fma_tflops", C.c_double), ("fp64_fma_tflops", C.c_double), ("fp32_rcp_tops", C.c_double),
                ("copy_gbs", C.c_double)]


def measure_peaks(device: int = 0) -> dict:
    """Attainable device rates from kpsi_measure_peaks."""
    p = Peaks()
    st = lib().kpsi_measure_peaks(device, C.byref(p))
    if st != KPSI_OK:
        raise KpsiError(st, "kpsi_measure_peaks failed")
    return {k: getattr(p, k) for k, _ in Peaks._fields_}


class MlpOptions(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int64), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libkpsi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2007_14931_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
        L.kpsi_create.argtypes = [C.c_int, vp, C.c_int, C.POINTER(vp)]
        L.kpsi_destroy.argtypes = [vp]
        L.kpsi_set_model.argtypes = [vp, C.POINTER(Kinematics), C.POINTER(Resonance), C.c_int]
        L.kpsi_n_params.argtypes = [vp, C.POINTER(C.c_int)]
        L.kpsi_set_floating.argtypes = [vp, C.POINTER(C.c_int), C.c_int]
        L.kpsi_load_events.argtypes = [vp, C.c_int, i64, dp, dp, dp, dp]
        L.kpsi_load_events_device.argtypes = [vp, C.c_int, i64, vp, vp, vp, vp]
        L.kpsi_set_efficiency_flat.argtypes = [vp]
        L.kpsi_set_efficiency_values.argtypes = [vp, dp, i64]
        L.kpsi_set_efficiency_hist.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_int), dp, dp]
        L.kpsi_set_norm_mixture.argtypes = [vp, dp, i64]
        # pointer arguments of the per-call entry points are plain addresses (the binding's fast
        # path passes ndarray.ctypes.data integers; ctypes pointer objects are accepted too)
        L.kpsi_nll.argtypes = [vp, vp, vp]
        L.kpsi_nll_and_grad.argtypes = [vp, vp, vp, vp]
        L.kpsi_nll_and_grad_noalloc.argtypes = [vp, vp, vp, vp]
        L.kpsi_density.argtypes = [vp, C.c_int, dp, dp]
        L.kpsi_invariants.argtypes = [vp, C.c_int, dp]
        L.kpsi_generate_phsp.argtypes = [vp, C.c_uint64, i64, C.c_double, vp, vp, vp, vp]
        L.kpsi_generate_model.argtypes = [vp, dp, C.c_uint64, i64, C.c_double, C.c_double, dp, vp, vp, vp, vp,
                                          C.POINTER(i64), C.POINTER(i64)]
        L.kpsi_set_timing.argtypes = [vp, C.c_int]
        L.kpsi_timing.argtypes = [vp, dp, C.POINTER(i64), C.c_int]
        L.kpsi_timing_median.argtypes = [vp, dp]
        L.kpsi_time_kernel.argtypes = [vp, dp, C.c_int, C.c_int, dp]
        L.kpsi_set_events_per_thread.argtypes = [vp, C.c_int]
        L.kpsi_fit_default_options.argtypes = [C.POINTER(FitOptions)]
        L.kpsi_migrad.argtypes = [vp, dp, C.POINTER(C.c_int), C.POINTER(FitOptions), C.POINTER(FitResult), dp]
        L.kpsi_migrad_limited.argtypes = [vp, dp, C.POINTER(C.c_int), dp, dp, C.POINTER(FitOptions),
                                          C.POINTER(FitResult), dp]
        L.kpsi_hesse.argtypes = [vp, dp, C.POINTER(C.c_int), C.POINTER(FitOptions), dp, C.POINTER(FitResult)]
        L.kpsi_set_norm_cache.argtypes = [vp, C.c_int]
        L.kpsi_norm_cache_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), dp]
        L.kpsi_fit_fractions.argtypes = [vp, dp, dp, dp]
        L.kpsi_measure_peaks.argtypes = [C.c_int, C.POINTER(Peaks)]
        L.kpsi_set_background.argtypes = [vp, C.c_double, dp, dp, dp]
        L.kpsi_template_values.argtypes = [vp, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_int),
                                           C.POINTER(C.c_float), C.POINTER(C.c_int), dp]
        fp = C.POINTER(C.c_float)
        L.kpsi_mlp_default_options.argtypes = [C.POINTER(MlpOptions)]
        L.kpsi_accept_labels.argtypes = [vp, C.c_uint64, i64, i64, vp, vp, vp, vp, dp, vp, vp]
        L.kpsi_hist_efficiency.argtypes = [vp, i64, vp, vp, vp, vp, vp, C.POINTER(C.c_int), dp, dp, fp]
        L.kpsi_mlp_grad.argtypes = [vp, fp, i64, vp, vp, vp, vp, vp, dp, dp]
        L.kpsi_mlp_train.argtypes = [vp, fp, i64, vp, vp, vp, vp, vp, C.POINTER(MlpOptions), dp]
        L.kpsi_mlp_eval.argtypes = [vp, fp, i64, vp, vp, vp, vp, vp]
        L.kpsi_set_efficiency_mlp.argtypes = [vp, fp]
        L.kpsi_last_error.argtypes = [vp]
        L.kpsi_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name != "kpsi_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def kinematics(d: dict) -> Kinematics:
    return Kinematics(d["mB"], d["mJ"], d["mK"], d["mPi"], d["rB"], d["rR"])


def resonances(res) -> C.Array:
    arr = (Resonance * len(res))()
    for i, r in enumerate(res):
        arr[i] = Resonance(r.chain, r.spin, r.parity, r.lb, r.lr, r.mass, r.width, r.shape, r.lass_a, r.lass_b,
                           int(getattr(r, "hel_free", False)))
    return arr


def create_status(device: int = 0, precision: int = FP64) -> tuple[int, str]:
    """Try kpsi_create and return (status, message) without raising (for error-path checks)."""
    L = lib()
    h = C.c_void_p()
    st = L.kpsi_create(device, None, precision, C.byref(h))
    msg = L.kpsi_last_error(None).decode()
    if st == KPSI_OK:
        L.kpsi_destroy(h)
    return st, msg


class Engine:
    """One kpsi context: model, loaded event sets and the NLL entry points."""

    def __init__(self, device: int = 0, precision: str | int = "fp64", stream=None):
        self.L = lib()
        prec = {"fp64": FP64, "fp32": FP32}.get(precision, precision)
        self.precision = prec
        self.device = device
        h = C.c_void_p()
        st = self.L.kpsi_create(device, C.c_void_p(stream) if stream else None, prec, C.byref(h))
        if st != KPSI_OK:
            raise KpsiError(st, self.L.kpsi_last_error(None).decode())
        self.h = h
        self._keep = {}
        self.n_params = 0
        self.n = [0, 0]
        self._out = C.c_double()
        self._out_addr = C.addressof(self._out)
        self._bufs(0)

    def _bufs(self, n: int) -> None:
        # parameter and gradient buffers of the per-call entry points, with their addresses taken
        # once (reading an array's address through numpy costs more than the call itself)
        self._pbuf = np.zeros(n)
        self._gbuf = np.zeros(n)
        self._pbuf_addr = self._pbuf.ctypes.data
        self._gbuf_addr = self._gbuf.ctypes.data

    def _put(self, params) -> int:
        if np.shape(params) != self._pbuf.shape:
            raise ValueError(f"expected {self._pbuf.size} parameters, got shape {np.shape(params)}")
        self._pbuf[...] = params
        return self._pbuf_addr

    def close(self):
        if getattr(self, "h", None):
            self.L.kpsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st: int):
        if st != KPSI_OK:
            raise KpsiError(st, self.L.kpsi_last_error(self.h).decode())

    def set_model(self, kin: dict, res) -> None:
        k = kinematics(kin)
        r = resonances(res)
        self._chk(self.L.kpsi_set_model(self.h, C.byref(k), r, len(res)))
        n = C.c_int()
        self._chk(self.L.kpsi_n_params(self.h, C.byref(n)))
        self.n_params = n.value
        self.n_res = len(res)
        self._bufs(self.n_params)

    def set_floating(self, flags) -> None:
        f = np.ascontiguousarray(flags, dtype=np.int32)
        self._chk(self.L.kpsi_set_floating(self.h, f.ctypes.data_as(C.POINTER(C.c_int)), len(f)))

    def load(self, which: int, events) -> None:
        """events: numpy (4, n) float64 (copied) or a CUDA float64 torch tensor (4, n) (borrowed)."""
        if hasattr(events, "is_cuda") and events.is_cuda:
            import torch
            ev = events.contiguous()
            assert ev.dtype == torch.float64 and ev.dim() == 2 and ev.shape[0] == 4
            self._keep[which] = ev
            n = ev.shape[1]
            ptrs = [C.c_void_p(ev[i].data_ptr()) for i in range(4)]
            self._chk(self.L.kpsi_load_events_device(self.h, which, n, *ptrs))
        else:
            ev = _f64(events)
            n = ev.shape[1]
            cols = [_f64(ev[i]) for i in range(4)]
            self._chk(self.L.kpsi_load_events(self.h, which, n, *(_dp(c) for c in cols)))
            self._keep.pop(which, None)
        self.n[which] = n

    def set_efficiency_flat(self) -> None:
        self._chk(self.L.kpsi_set_efficiency_flat(self.h))

    def set_efficiency_values(self, eps) -> None:
        e = _f64(eps)
        self._chk(self.L.kpsi_set_efficiency_values(self.h, _dp(e), e.size))

    def set_efficiency_hist(self, table, lo, hi) -> None:
        t = np.ascontiguousarray(table, dtype=np.float32)
        nb = np.ascontiguousarray(t.shape, dtype=np.int32)
        lo, hi = _f64(lo), _f64(hi)
        self._chk(self.L.kpsi_set_efficiency_hist(self.h, t.ctypes.data_as(C.POINTER(C.c_float)),
                                                  nb.ctypes.data_as(C.POINTER(C.c_int)), _dp(lo), _dp(hi)))

    def set_norm_mixture(self, params0, n_flat: int) -> None:
        """kpsi_set_norm_mixture: the first n_flat normalisation events are flat, the rest drawn
        from S(y; params0); the library weights them back to flat phase space."""
        p = _f64(params0)
        self._chk(self.L.kpsi_set_norm_mixture(self.h, _dp(p), int(n_flat)))

    def nll(self, params) -> float:
        st = self.L.kpsi_nll(self.h, self._put(params), self._out_addr)
        if st:
            self._chk(st)
        return self._out.value

    def nll_and_grad(self, params) -> tuple[float, np.ndarray]:
        st = self.L.kpsi_nll_and_grad(self.h, self._put(params), self._out_addr, self._gbuf_addr)
        if st:
            self._chk(st)
        return self._out.value, self._gbuf.copy()

    def nll_and_grad_noalloc(self, params) -> tuple[float, np.ndarray]:
        """kpsi_nll_and_grad_noalloc: the same pass with no device allocation (static scratch)."""
        st = self.L.kpsi_nll_and_grad_noalloc(self.h, self._put(params), self._out_addr, self._gbuf_addr)
        if st:
            self._chk(st)
        return self._out.value, self._gbuf.copy()

    def nll_status(self, params, grad: bool = False) -> tuple[int, float]:
        """Raw status and value (for error-path tests)."""
        p = _f64(params)
        out = C.c_double()
        if grad:
            g = np.empty(self.n_params)
            st = self.L.kpsi_nll_and_grad(self.h, _dp(p), C.byref(out), _dp(g))
        else:
            st = self.L.kpsi_nll(self.h, _dp(p), C.byref(out))
        return st, out.value

    def density(self, which: int, params) -> np.ndarray:
        p = _f64(params)
        out = np.empty(self.n[which])
        self._chk(self.L.kpsi_density(self.h, which, _dp(p), _dp(out)))
        return out

    def invariants(self, which: int) -> np.ndarray:
        out = np.empty((self.n[which], 5))
        self._chk(self.L.kpsi_invariants(self.h, which, _dp(out)))
        return out

    def generate_phsp(self, seed: int, n: int, wmax: float):
        import torch
        ev = torch.empty((4, n), dtype=torch.float64, device=f"cuda:{self.device}")
        ptrs = [C.c_void_p(ev[i].data_ptr()) for i in range(4)]
        self._chk(self.L.kpsi_generate_phsp(self.h, seed, n, wmax, *ptrs))
        return ev

    def generate_model(self, params, seed: int, n: int, wmax: float, smax: float, acc_coef=None):
        import torch
        p = _f64(params)
        ev = torch.empty((4, n), dtype=torch.float64, device=f"cuda:{self.device}")
        ptrs = [C.c_void_p(ev[i].data_ptr()) for i in range(4)]
        npr, nov = C.c_int64(), C.c_int64()
        co = _f64(acc_coef).reshape(-1) if acc_coef is not None else None
        self._chk(self.L.kpsi_generate_model(self.h, _dp(p), seed, n, wmax, smax, _dp(co) if co is not None else None,
                                             *ptrs, C.byref(npr), C.byref(nov)))
        return ev, npr.value, nov.value

    def set_timing(self, on: bool | int) -> None:
        """False/0: off; True: every call; an int k > 1: every k-th call."""
        every = int(on) if not isinstance(on, bool) else (1 if on else 0)
        self._chk(self.L.kpsi_set_timing(self.h, every))

    def timing(self, reset: bool = False) -> tuple[float, int]:
        ms, n = C.c_double(), C.c_int64()
        self._chk(self.L.kpsi_timing(self.h, C.byref(ms), C.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def timing_median(self) -> float:
        """Median kernel milliseconds of the timed calls since the last reset (NaN if none)."""
        ms = C.c_double()
        self._chk(self.L.kpsi_timing_median(self.h, C.byref(ms)))
        return ms.value

    def time_kernel(self, params, grad: bool = True, reps: int = 200) -> float:
        """kpsi_time_kernel: milliseconds per launch of the per-event work, `reps` launches back to
        back between one pair of HIP events."""
        p = _f64(params)
        ms = C.c_double()
        self._chk(self.L.kpsi_time_kernel(self.h, _dp(p), 1 if grad else 0, int(reps), C.byref(ms)))
        return ms.value

    def fit_options(self, **kw) -> FitOptions:
        o = FitOptions()
        self._chk(self.L.kpsi_fit_default_options(C.byref(o)))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def migrad(self, params, free_mask, lower=None, upper=None, **kw):
        """Minimise from params over the free entries, optionally within limits (arrays of
        kpsi_n_params values; non-finite entries leave that side open: kpsi_migrad_limited).
        Returns (params_at_min, covariance of the free parameters, FitResult)."""
        x = _f64(params).copy()
        m = np.ascontiguousarray(free_mask, dtype=np.int32)
        nf = int(m.sum())
        cov = np.empty((nf, nf))
        o = self.fit_options(**kw)
        r = FitResult()
        mp = m.ctypes.data_as(C.POINTER(C.c_int))
        if lower is None and upper is None:
            self._chk(self.L.kpsi_migrad(self.h, _dp(x), mp, C.byref(o), C.byref(r), _dp(cov)))
        else:
            lo = _f64(lower) if lower is not None else None
            hi = _f64(upper) if upper is not None else None
            for a in (lo, hi):
                if a is not None and a.shape != x.shape:
                    raise ValueError(f"limits need {x.size} entries, got shape {a.shape}")
            self._chk(self.L.kpsi_migrad_limited(self.h, _dp(x), mp, _dp(lo) if lo is not None else None,
                                                 _dp(hi) if hi is not None else None, C.byref(o), C.byref(r),
                                                 _dp(cov)))
        return x, cov, r

    def hesse(self, params, free_mask, **kw):
        x = _f64(params)
        m = np.ascontiguousarray(free_mask, dtype=np.int32)
        nf = int(m.sum())
        cov = np.empty((nf, nf))
        o = self.fit_options(**kw)
        r = FitResult()
        self._chk(self.L.kpsi_hesse(self.h, _dp(x), m.ctypes.data_as(C.POINTER(C.c_int)), C.byref(o), _dp(cov),
                                    C.byref(r)))
        return cov, r

    # ---- learned efficiency (event tensors: CUDA float64 (4, n); labels: CUDA uint8 (n,))
    @staticmethod
    def _ev_ptrs(ev):
        import torch
        assert ev.is_cuda and ev.dtype == torch.float64 and ev.dim() == 2 and ev.shape[0] == 4 and ev.is_contiguous()
        return [C.c_void_p(ev[i].data_ptr()) for i in range(4)]

    @staticmethod
    def _f32(params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_NP
        return p

    def accept_labels(self, seed: int, events, acc_coef, e0: int = 0):
        import torch
        n = events.shape[1]
        lab = torch.empty(n, dtype=torch.uint8, device=events.device)
        eps = torch.empty(n, dtype=torch.float64, device=events.device)
        co = _f64(acc_coef).reshape(-1)
        self._chk(self.L.kpsi_accept_labels(self.h, seed, e0, n, *self._ev_ptrs(events), _dp(co),
                                            C.c_void_p(lab.data_ptr()), C.c_void_p(eps.data_ptr())))
        return lab, eps

    def hist_efficiency(self, events, labels, nb, lo, hi) -> np.ndarray:
        nbv = np.ascontiguousarray(nb, dtype=np.int32)
        lo, hi = _f64(lo), _f64(hi)
        table = np.empty(int(np.prod(nbv)), dtype=np.float32)
        self._chk(self.L.kpsi_hist_efficiency(self.h, events.shape[1], *self._ev_ptrs(events),
                                              C.c_void_p(labels.data_ptr()), nbv.ctypes.data_as(C.POINTER(C.c_int)),
                                              _dp(lo), _dp(hi), table.ctypes.data_as(C.POINTER(C.c_float))))
        return table.reshape(tuple(nbv))

    def mlp_grad(self, params, events, labels):
        p = self._f32(params)
        g = np.empty(MLP_NP)
        loss = C.c_double()
        self._chk(self.L.kpsi_mlp_grad(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), events.shape[1],
                                       *self._ev_ptrs(events), C.c_void_p(labels.data_ptr()), _dp(g), C.byref(loss)))
        return g, loss.value

    def mlp_train(self, params, events, labels, **kw):
        p = self._f32(params).copy()
        o = MlpOptions()
        self._chk(self.L.kpsi_mlp_default_options(C.byref(o)))
        for k, v in kw.items():
            setattr(o, k, v)
        loss = C.c_double()
        self._chk(self.L.kpsi_mlp_train(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), events.shape[1],
                                        *self._ev_ptrs(events), C.c_void_p(labels.data_ptr()), C.byref(o),
                                        C.byref(loss)))
        return p, loss.value

    def mlp_eval(self, params, events):
        import torch
        p = self._f32(params)
        out = torch.empty(events.shape[1], dtype=torch.float64, device=events.device)
        self._chk(self.L.kpsi_mlp_eval(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), events.shape[1],
                                       *self._ev_ptrs(events), C.c_void_p(out.data_ptr())))
        return out

    def set_efficiency_mlp(self, params) -> None:
        p = self._f32(params)
        self._chk(self.L.kpsi_set_efficiency_mlp(self.h, p.ctypes.data_as(C.POINTER(C.c_float))))

    def set_norm_cache(self, mode: int) -> None:
        """0 off, 1 on, 2 auto (see kpsi_set_norm_cache)."""
        self._chk(self.L.kpsi_set_norm_cache(self.h, mode))

    def norm_cache_stats(self) -> tuple[int, int, float]:
        b, h, ms = C.c_int64(), C.c_int64(), C.c_double()
        self._chk(self.L.kpsi_norm_cache_stats(self.h, C.byref(b), C.byref(h), C.byref(ms)))
        return b.value, h.value, ms.value

    def fit_fractions(self, params) -> tuple[np.ndarray, float]:
        """Eq. 13 on the normalisation events: (fractions in table order, their sum)."""
        p = _f64(params)
        ff = np.empty(self.n_res)
        tot = C.c_double()
        self._chk(self.L.kpsi_fit_fractions(self.h, _dp(p), _dp(ff), C.byref(tot)))
        return ff, tot.value

    def set_flavour(self, tags, mistag: float = 0.0) -> None:
        """Flavour tags of the data events (+1 B0, -1 conjugate decay; kpsi_set_flavour) and the
        mistag fraction; tags None switches them off."""
        if tags is None:
            self._chk(self.L.kpsi_set_flavour(self.h, None, C.c_int64(0), C.c_double(0.0)))
            return
        t = _f64(tags)
        self._chk(self.L.kpsi_set_flavour(self.h, _dp(t), C.c_int64(t.size), C.c_double(mistag)))

    def set_constraints(self, index=(), mean=(), sigma=()) -> None:
        """Gaussian constraints on parameters (kpsi_set_constraints); empty removes them."""
        ix = np.ascontiguousarray(index, dtype=np.int32)
        mu, sg = _f64(mean), _f64(sigma)
        n = int(ix.size)
        if n == 0:
            self._chk(self.L.kpsi_set_constraints(self.h, 0, None, None, None))
            return
        self._chk(self.L.kpsi_set_constraints(self.h, n, ix.ctypes.data_as(C.POINTER(C.c_int)), _dp(mu), _dp(sg)))

    def set_background(self, purity: float, eps_data, b_data, b_norm) -> None:
        """Eq. 14 mixture (kpsi_set_background); b_data None switches it off."""
        arrs = [None if a is None else _f64(a) for a in (eps_data, b_data, b_norm)]
        self._chk(self.L.kpsi_set_background(self.h, purity, *(None if a is None else _dp(a) for a in arrs)))

    def template_values(self, which: int, t_mass, t_ang) -> np.ndarray:
        """Per-event product of a (m_Kpi, cos theta_K*) table and a (cos theta_J/psi, phi) table."""
        t1 = np.ascontiguousarray(t_mass, dtype=np.float32)
        t2 = np.ascontiguousarray(t_ang, dtype=np.float32)
        n1 = np.array(t1.shape, dtype=np.int32)
        n2 = np.array(t2.shape, dtype=np.int32)
        out = np.empty(self.n[which])
        fp, ip = C.POINTER(C.c_float), C.POINTER(C.c_int)
        self._chk(self.L.kpsi_template_values(self.h, which, t1.ctypes.data_as(fp), n1.ctypes.data_as(ip),
                                              t2.ctypes.data_as(fp), n2.ctypes.data_as(ip), _dp(out)))
        return out

    def set_events_per_thread(self, ept: int) -> None:
        self._chk(self.L.kpsi_set_events_per_thread(self.h, ept))


def make_nll_function(engine: Engine):
    """torch.autograd.Function over the engine: forward runs nll_and_grad once and keeps the
    gradient; backward scales it by the incoming gradient."""
    import torch

    class NLL(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params):
            v, g = engine.nll_and_grad(params.detach().cpu().numpy())
            ctx.save_for_backward(torch.from_numpy(g).to(params.device, params.dtype))
            return params.new_tensor(v)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g

    return NLL

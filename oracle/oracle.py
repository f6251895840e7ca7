"""ctypes binding of the FP64 CPU oracle (oracle/kpsi_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.  It shares no code
with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kpsi_oracle.cpp")
_LIB = os.path.join(_HERE, "libkpsi_oracle.so")
CXXFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c++17"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", *CXXFLAGS, "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Kin(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("mB", "mJ", "mK", "mPi", "rB", "rR")]


class Res(C.Structure):
    _fields_ = [("chain", C.c_int), ("spin", C.c_int), ("parity", C.c_int), ("lb", C.c_int), ("lr", C.c_int),
                ("mass", C.c_double), ("width", C.c_double), ("shape", C.c_int), ("lass_a", C.c_double),
                ("lass_b", C.c_double), ("hel_free", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # a library older than its source (say, a changed struct layout) is rebuilt, never loaded
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        kp, rp = C.POINTER(Kin), C.POINTER(Res)
        L.oracle_n_params.argtypes = [rp, C.c_int]
        L.oracle_wigner_d.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double]
        L.oracle_wigner_d.restype = C.c_double
        L.oracle_breakup.argtypes = [C.c_double] * 3
        L.oracle_breakup.restype = C.c_double
        L.oracle_lineshape.argtypes = [kp, rp, C.c_double, C.c_double, C.c_double, dp]
        L.oracle_z_angles.argtypes = [kp, C.c_int64, dp, dp, dp, dp, dp]
        L.oracle_four_vectors.argtypes = [kp, C.c_int64, dp, dp, dp, dp, dp]
        L.oracle_density.argtypes = [kp, rp, C.c_int, dp, C.c_int64, dp, dp, dp, dp, dp]
        L.oracle_nll.argtypes = [kp, rp, C.c_int, dp, C.c_int64, dp, dp, dp, dp, C.c_int64, dp, dp, dp, dp, dp,
                                 C.c_int, C.POINTER(C.c_int), dp, dp]
        L.oracle_density_grad.argtypes = [kp, rp, C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_int, C.POINTER(C.c_int), dp]
        L.oracle_density_grad.restype = C.c_double
        L.oracle_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.oracle_gen_phsp.argtypes = [kp, C.c_uint64, C.c_int64, C.c_double, dp, dp, dp, dp]
        L.oracle_gen_model.argtypes = [kp, rp, C.c_int, dp, C.c_uint64, C.c_int64, C.c_double, C.c_double, dp,
                                       C.c_int64, dp, dp, dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.oracle_acceptance.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
        L.oracle_acceptance.restype = C.c_double
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_struct_size.argtypes = [C.c_int]
        if L.oracle_struct_size(0) != C.sizeof(Kin) or L.oracle_struct_size(1) != C.sizeof(Res):
            raise RuntimeError("oracle library and binding disagree on the structure layouts")
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def kin(d: dict) -> Kin:
    return Kin(d["mB"], d["mJ"], d["mK"], d["mPi"], d["rB"], d["rR"])


def res_array(res) -> C.Array:
    arr = (Res * len(res))()
    for i, r in enumerate(res):
        arr[i] = Res(r.chain, r.spin, r.parity, r.lb, r.lr, r.mass, r.width, r.shape, r.lass_a, r.lass_b,
                     int(getattr(r, "hel_free", False)))
    return arr


def set_threads(n: int) -> None:
    lib().oracle_set_threads(n)


def max_threads() -> int:
    return lib().oracle_max_threads()


def n_params(res) -> int:
    return lib().oracle_n_params(res_array(res), len(res))


def wigner_d(j: int, mp: int, m: int, theta: float) -> float:
    return lib().oracle_wigner_d(j, mp, m, theta)


def breakup(M: float, m1: float, m2: float) -> float:
    return lib().oracle_breakup(M, m1, m2)


def lineshape(kind: dict, r, M: float, G0: float, m: float) -> complex:
    out = np.zeros(2)
    k = kin(kind)
    ra = res_array([r])
    lib().oracle_lineshape(C.byref(k), ra, M, G0, m, _dp(out))
    return complex(out[0], out[1])


def z_angles(kind: dict, ev: np.ndarray) -> np.ndarray:
    """(n, 5): m_Jpsi pi, theta_Z, theta~_J/psi, phi~, alpha."""
    ev = _f64(ev)
    n = ev.shape[1]
    out = np.zeros((n, 5))
    k = kin(kind)
    lib().oracle_z_angles(C.byref(k), n, *(_dp(_f64(ev[i])) for i in range(4)), _dp(out))
    return out


def four_vectors(kind: dict, ev: np.ndarray) -> np.ndarray:
    ev = _f64(ev)
    n = ev.shape[1]
    out = np.zeros((n, 4, 4))
    k = kin(kind)
    lib().oracle_four_vectors(C.byref(k), n, *(_dp(_f64(ev[i])) for i in range(4)), _dp(out))
    return out


def density(kind: dict, res, par, ev: np.ndarray) -> np.ndarray:
    ev = _f64(ev)
    par = _f64(par)
    n = ev.shape[1]
    out = np.zeros(n)
    k = kin(kind)
    cols = [_f64(ev[i]) for i in range(4)]
    lib().oracle_density(C.byref(k), res_array(res), len(res), _dp(par), n, *(_dp(c) for c in cols), _dp(out))
    return out


def density_grad(kind: dict, res, par, event, dirs) -> tuple[float, np.ndarray]:
    par = _f64(par)
    dirs = np.ascontiguousarray(dirs, dtype=np.int32)
    g = np.zeros(len(dirs))
    k = kin(kind)
    s = lib().oracle_density_grad(C.byref(k), res_array(res), len(res), _dp(par), *map(float, event), len(dirs),
                                  dirs.ctypes.data_as(C.POINTER(C.c_int)), _dp(g))
    return s, g


def nll(kind: dict, res, par, data: np.ndarray, mc: np.ndarray, eps=None, dirs=None):
    """-2 ln L (Eq. 14 signal part, MC-normalised).  Returns (status, nll, grad or None)."""
    par = _f64(par)
    dcols = [_f64(data[i]) for i in range(4)]
    mcols = [_f64(mc[i]) for i in range(4)]
    e = _f64(eps) if eps is not None else None
    dirs_arr = np.ascontiguousarray(dirs if dirs is not None else [], dtype=np.int32)
    out = C.c_double(0.0)
    g = np.zeros(max(1, len(dirs_arr)))
    k = kin(kind)
    st = lib().oracle_nll(C.byref(k), res_array(res), len(res), _dp(par), dcols[0].size, *(_dp(c) for c in dcols),
                          mcols[0].size, *(_dp(c) for c in mcols), _dp(e) if e is not None else None,
                          len(dirs_arr), dirs_arr.ctypes.data_as(C.POINTER(C.c_int)), C.byref(out), _dp(g))
    return st, out.value, (g[: len(dirs_arr)] if len(dirs_arr) else None)


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    P = C.POINTER(C.c_uint32)
    lib().oracle_philox(c.ctypes.data_as(P), k.ctypes.data_as(P), o.ctypes.data_as(P))
    return o


def gen_phsp(kind: dict, seed: int, n: int, wmax: float) -> np.ndarray:
    out = np.zeros((4, n))
    k = kin(kind)
    st = lib().oracle_gen_phsp(C.byref(k), seed, n, wmax, *(_dp(out[i]) for i in range(4)))
    if st != 0:
        raise RuntimeError("phase-space envelope exhausted")
    return out


def gen_model(kind: dict, res, par, seed: int, n: int, wmax: float, smax: float, acc_coef=None,
              max_prop: int = 1 << 40):
    """Accept-reject from eps*S.  Returns (events (4, n), n_proposals, n_over_envelope)."""
    par = _f64(par)
    out = np.zeros((4, n))
    npr, nov = C.c_int64(0), C.c_int64(0)
    co = _f64(acc_coef).reshape(-1) if acc_coef is not None else None
    k = kin(kind)
    st = lib().oracle_gen_model(C.byref(k), res_array(res), len(res), _dp(par), seed, n, wmax, smax,
                                _dp(co) if co is not None else None, max_prop, *(_dp(out[i]) for i in range(4)),
                                C.byref(npr), C.byref(nov))
    if st != 0:
        raise RuntimeError(f"oracle_gen_model failed ({st})")
    return out, npr.value, nov.value


def acceptance(coef, m_lo: float, m_hi: float, ev: np.ndarray) -> np.ndarray:
    co = _f64(coef).reshape(-1)
    ev = _f64(ev)
    f = lib().oracle_acceptance
    return np.array([f(_dp(co), m_lo, m_hi, *ev[:, i]) for i in range(ev.shape[1])])


def barrier(L: int, p: float, p0: float, r: float) -> float:
    f = lib().oracle_barrier
    f.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
    f.restype = C.c_double
    return f(L, p, p0, r)


def bw_poly(L: int, z: float) -> float:
    f = lib().oracle_bw_poly
    f.argtypes = [C.c_int, C.c_double]
    f.restype = C.c_double
    return f(L, z)


def mlp(par, u, y=None, grad: bool = False, round_bf16: bool = True):
    """Reference network: returns (mean loss, probabilities, gradient or None)."""
    par = _f64(par)
    u = _f64(u).reshape(-1, 4)
    n = u.shape[0]
    prob = np.zeros(n)
    g = np.zeros(4545) if grad else None
    yy = _f64(y) if y is not None else None
    f = lib().oracle_mlp
    f.argtypes = [C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int]
    f.restype = C.c_double
    loss = f(_dp(par), n, _dp(u), _dp(yy) if yy is not None else None, _dp(prob), _dp(g) if g is not None else None,
             1 if round_bf16 else 0)
    return loss, prob, g


def mlp_inputs(m_lo: float, m_hi: float, ev) -> np.ndarray:
    ev = _f64(ev)
    n = ev.shape[1]
    u = np.zeros((n, 4))
    f = lib().oracle_mlp_inputs
    f.argtypes = [C.c_double, C.c_double, C.c_int64] + [C.POINTER(C.c_double)] * 5
    f(m_lo, m_hi, n, *(_dp(_f64(ev[i])) for i in range(4)), _dp(u))
    return u


def bf16(x: float) -> float:
    f = lib().oracle_bf16
    f.argtypes = [C.c_double]
    f.restype = C.c_double
    return f(x)


def fit_fractions(kind: dict, res, par, ev, w=None):
    """Eq. 13 over the given phase-space events (optional integration weights w):
    returns (status, FF array of length len(res))."""
    ev = _f64(ev)
    par = _f64(par)
    n = ev.shape[1]
    ff = np.zeros(len(res))
    cols = [_f64(ev[i]) for i in range(4)]
    ww = _f64(w) if w is not None else None
    k = kin(kind)
    f = lib().oracle_fit_fractions
    dp = C.POINTER(C.c_double)
    f.argtypes = [C.POINTER(Kin), C.POINTER(Res), C.c_int, dp, C.c_int64, dp, dp, dp, dp, dp, dp]
    f.restype = C.c_int
    st = f(C.byref(k), res_array(res), len(res), _dp(par), n, *(_dp(c) for c in cols),
           _dp(ww) if ww is not None else None, _dp(ff))
    return st, ff


def nll_mix(kind: dict, res, par, data, mc, b_data, b_mc, purity: float, eps_data=None, eps_mc=None, dirs=None):
    """-2 ln L of the Eq. 14 mixture p eps S / N_S + (1 - p) b / N_b.
    Returns (status, nll, grad or None)."""
    par = _f64(par)
    dcols = [_f64(data[i]) for i in range(4)]
    mcols = [_f64(mc[i]) for i in range(4)]
    bd, bm = _f64(b_data), _f64(b_mc)
    ed = _f64(eps_data) if eps_data is not None else None
    em = _f64(eps_mc) if eps_mc is not None else None
    dirs_arr = np.ascontiguousarray(dirs if dirs is not None else [], dtype=np.int32)
    out = C.c_double(0.0)
    g = np.zeros(max(1, len(dirs_arr)))
    k = kin(kind)
    f = lib().oracle_nll_mix
    dp = C.POINTER(C.c_double)
    f.argtypes = [C.POINTER(Kin), C.POINTER(Res), C.c_int, dp, C.c_int64, dp, dp, dp, dp, C.c_int64, dp, dp, dp, dp,
                  dp, dp, dp, dp, C.c_double, C.c_int, C.POINTER(C.c_int), dp, dp]
    f.restype = C.c_int
    st = f(C.byref(k), res_array(res), len(res), _dp(par), dcols[0].size, *(_dp(c) for c in dcols),
           mcols[0].size, *(_dp(c) for c in mcols), _dp(ed) if ed is not None else None, _dp(bd),
           _dp(em) if em is not None else None, _dp(bm), C.c_double(purity), len(dirs_arr),
           dirs_arr.ctypes.data_as(C.POINTER(C.c_int)), C.byref(out), _dp(g))
    return st, out.value, (g[: len(dirs_arr)] if len(dirs_arr) else None)


def nll_cc(kind: dict, res, par, data, tag, mc, mistag: float, eps_mc=None, dirs=None):
    """-2 ln L of flavour-tagged events (tag +1 for B0, -1 for the conjugate decay, whose density
    is S with phi reversed) with mistag fraction w: f = [(1-w) S(x^q) + w S(x^-q)] / N_q.
    Returns (status, nll, grad or None)."""
    par = _f64(par)
    dcols = [_f64(data[i]) for i in range(4)]
    mcols = [_f64(mc[i]) for i in range(4)]
    tg = _f64(tag)
    em = _f64(eps_mc) if eps_mc is not None else None
    dirs_arr = np.ascontiguousarray(dirs if dirs is not None else [], dtype=np.int32)
    out = C.c_double(0.0)
    g = np.zeros(max(1, len(dirs_arr)))
    k = kin(kind)
    f = lib().oracle_nll_cc
    dp = C.POINTER(C.c_double)
    f.argtypes = [C.POINTER(Kin), C.POINTER(Res), C.c_int, dp, C.c_int64, dp, dp, dp, dp, dp, C.c_int64, dp, dp, dp,
                  dp, dp, C.c_double, C.c_int, C.POINTER(C.c_int), dp, dp]
    f.restype = C.c_int
    st = f(C.byref(k), res_array(res), len(res), _dp(par), dcols[0].size, *(_dp(c) for c in dcols), _dp(tg),
           mcols[0].size, *(_dp(c) for c in mcols), _dp(em) if em is not None else None, C.c_double(mistag),
           len(dirs_arr), dirs_arr.ctypes.data_as(C.POINTER(C.c_int)), C.byref(out), _dp(g))
    return st, out.value, (g[: len(dirs_arr)] if len(dirs_arr) else None)


def nll_cc_mix(kind: dict, res, par, data, tag, mc, mistag: float, b_data, b_mc, purity: float, eps_data=None,
               eps_mc=None, dirs=None):
    """-2 ln L of flavour-tagged events with the Eq. 14 background mixture:
    f = p eps [(1-w) S(x^q) + w S(x^-q)] / N_q + (1 - p) b / N_b.  Returns (status, nll, grad or None)."""
    par = _f64(par)
    dcols = [_f64(data[i]) for i in range(4)]
    mcols = [_f64(mc[i]) for i in range(4)]
    tg, bd, bm = _f64(tag), _f64(b_data), _f64(b_mc)
    ed = _f64(eps_data) if eps_data is not None else None
    em = _f64(eps_mc) if eps_mc is not None else None
    dirs_arr = np.ascontiguousarray(dirs if dirs is not None else [], dtype=np.int32)
    out = C.c_double(0.0)
    g = np.zeros(max(1, len(dirs_arr)))
    k = kin(kind)
    f = lib().oracle_nll_cc_mix
    dp = C.POINTER(C.c_double)
    f.argtypes = [C.POINTER(Kin), C.POINTER(Res), C.c_int, dp, C.c_int64, dp, dp, dp, dp, dp, C.c_int64, dp, dp, dp,
                  dp, dp, dp, dp, dp, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int), dp, dp]
    f.restype = C.c_int
    st = f(C.byref(k), res_array(res), len(res), _dp(par), dcols[0].size, *(_dp(c) for c in dcols), _dp(tg),
           mcols[0].size, *(_dp(c) for c in mcols), _dp(ed) if ed is not None else None, _dp(bd),
           _dp(em) if em is not None else None, _dp(bm), C.c_double(purity), C.c_double(mistag),
           len(dirs_arr), dirs_arr.ctypes.data_as(C.POINTER(C.c_int)), C.byref(out), _dp(g))
    return st, out.value, (g[: len(dirs_arr)] if len(dirs_arr) else None)


def gauss_penalty(idx, mean, sigma, par):
    """Gaussian constraints: (sum_k ((p[idx_k] - mean_k)/sigma_k)^2, its gradient over par)."""
    par = _f64(par)
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    mu, sg = _f64(mean), _f64(sigma)
    g = np.zeros(par.size)
    v = C.c_double(0.0)
    f = lib().oracle_gauss_penalty
    dp = C.POINTER(C.c_double)
    f.argtypes = [C.c_int, C.POINTER(C.c_int), dp, dp, C.c_int, dp, dp, dp]
    f.restype = C.c_int
    st = f(ix.size, ix.ctypes.data_as(C.POINTER(C.c_int)), _dp(mu), _dp(sg), par.size, _dp(par), C.byref(v), _dp(g))
    if st != 0:
        raise ValueError("bad constraint")
    return v.value, g

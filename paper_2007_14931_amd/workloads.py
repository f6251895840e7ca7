"""Workload definitions: decay constants, resonance tables, seeded couplings, sizes.

This module holds inputs only -- numbers and seeded draws -- and none of the
amplitude arithmetic, so both the HIP path and the CPU oracle can be fed from it.

Decay: B0 -> J/psi K+ pi-, J/psi -> mu+ mu- (paper, Methodology).  The ten K*
states are the ones the paper lists for m_Kpi up to 2.183 GeV (text after Eq. 5);
their masses and widths are world-average-like stand-ins (the paper fixes them to
world averages without printing them), except K*(892), Z(4430) and Z(4240), whose
values are the ones the workloads name.  Couplings are seeded draws (magnitude in
U[0.1, 1], phase in U[-pi, pi]); H_0 of K*(892) is fixed to 1 (Eq. 6).

Canonical parameter vector (the C ABI's layout): for each resonance in table order
its coupling (magnitude, phase) pairs -- K*: lambda = -1, 0, +1 (spin 0: lambda = 0
only); Z (1+): lambda' = 0, +1 (lambda' = -1 follows from Eq. 11), or lambda' = 0, +1, -1
for a Z whose helicity couplings are left free of that relation (hel_free) -- then
(M, Gamma0) for every resonance in table order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# GeV, GeV^-1.  r_R: barrier radius of the resonance decay; r_B: of the B decay.
KIN = dict(mB=5.27966, mJ=3.0969, mK=0.493677, mPi=0.13957, rB=5.0, rR=1.6)
M_LO = KIN["mK"] + KIN["mPi"]          # m_Kpi threshold
M_HI = KIN["mB"] - KIN["mJ"]           # m_Kpi end point (2.18276 GeV)
# envelope of the phase-space density p_B(m) q(m) (its maximum is 0.82843 GeV^2)
PHSP_WMAX = 0.85

KSTAR = 0
ZCHAIN = 1


@dataclasses.dataclass(frozen=True)
class Resonance:
    name: str
    chain: int       # 0 = K* (K pi), 1 = Z (J/psi pi)
    spin: int
    parity: int
    mass: float
    width: float
    lb: int = -1     # < 0: lowest allowed orbital momentum
    lr: int = -1
    shape: int = 0           # 0 relativistic Breit-Wigner, 1 LASS S-wave (spin-0 K* only)
    lass_a: float = 1.95     # LASS effective-range parameters (GeV^-1)
    lass_b: float = 1.76
    hel_free: bool = False   # Z only: H'_{+1} and H'_{-1} independent (no Eq. 11 relation)

    @property
    def n_coup(self) -> int:
        if self.chain == KSTAR:
            return 1 if self.spin == 0 else 3
        return 3 if self.hel_free else 2


KSTARS = [
    Resonance("K0*(800)", KSTAR, 0, +1, 0.824, 0.478),
    Resonance("K*(892)", KSTAR, 1, -1, 0.89555, 0.0473),
    Resonance("K*(1410)", KSTAR, 1, -1, 1.414, 0.232),
    Resonance("K0*(1430)", KSTAR, 0, +1, 1.425, 0.270),
    Resonance("K2*(1430)", KSTAR, 2, +1, 1.4324, 0.109),
    Resonance("K*(1680)", KSTAR, 1, -1, 1.717, 0.322),
    Resonance("K3*(1780)", KSTAR, 3, -1, 1.776, 0.159),
    Resonance("K0*(1950)", KSTAR, 0, +1, 1.945, 0.201),
    Resonance("K2*(1980)", KSTAR, 2, +1, 1.973, 0.373),
    Resonance("K4*(2045)", KSTAR, 4, +1, 2.045, 0.198),
]
Z4430 = Resonance("Z(4430)", ZCHAIN, 1, +1, 4.43, 0.18)
Z4240 = Resonance("Z(4240)", ZCHAIN, 1, +1, 4.24, 0.60)
KSTAR892 = KSTARS[1]
# The low-mass K pi S-wave in the LASS form: the effective-range term with the K0*(1430)
# resonance (mass, width of K0*(1430)); it replaces K0*(800) and K0*(1430).
LASS = Resonance("LASS", KSTAR, 0, +1, 1.425, 0.270, shape=1)


def model(name: str) -> list[Resonance]:
    """Resonance table of a named model."""
    if name == "kstar892":
        return [KSTAR892]
    if name == "kstar10":
        return list(KSTARS)
    if name == "full":
        return list(KSTARS) + [Z4430]
    if name == "full2z":
        return list(KSTARS) + [Z4430, Z4240]
    if name == "full_zfree":
        return list(KSTARS) + [dataclasses.replace(Z4430, hel_free=True)]
    if name in ("kstar_lass", "lass_full2z"):
        ks = [LASS] + [r for r in KSTARS if r.name not in ("K0*(800)", "K0*(1430)")]
        return ks if name == "kstar_lass" else ks + [Z4430, Z4240]
    raise KeyError(name)


def n_params(res: list[Resonance]) -> int:
    return sum(2 * r.n_coup for r in res) + 2 * len(res)


def coupling_offset(res: list[Resonance], i: int) -> int:
    return sum(2 * r.n_coup for r in res[:i])


def lineshape_offset(res: list[Resonance], i: int) -> int:
    return sum(2 * r.n_coup for r in res) + 2 * i


def fixed_coupling_index(res: list[Resonance]) -> int | None:
    """Index of |H_0| of K*(892) (Eq. 6); its phase is the next entry."""
    for i, r in enumerate(res):
        if r.name == "K*(892)":
            return coupling_offset(res, i) + 2 * 1   # lambda = 0 is the middle pair
    return None


def params(res: list[Resonance], seed: int = 11) -> np.ndarray:
    """Seeded truth point: magnitudes U[0.1, 1], phases U[-pi, pi]; H_0(892) = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(n_params(res))
    k = 0
    for r in res:
        for _ in range(r.n_coup):
            p[k] = rng.uniform(0.1, 1.0)
            p[k + 1] = rng.uniform(-math.pi, math.pi)
            k += 2
    for r in res:
        p[k] = r.mass
        p[k + 1] = r.width
        k += 2
    f = fixed_coupling_index(res)
    if f is not None:
        p[f] = 1.0
        p[f + 1] = 0.0
    return p


def free_mask(res: list[Resonance], floating: tuple[str, ...] = ()) -> np.ndarray:
    """Free parameters: every coupling except H_0(892); M, Gamma of the named resonances."""
    mask = np.zeros(n_params(res), dtype=bool)
    mask[: sum(2 * r.n_coup for r in res)] = True
    f = fixed_coupling_index(res)
    if f is not None:
        mask[f] = mask[f + 1] = False
    for i, r in enumerate(res):
        if r.name in floating:
            o = lineshape_offset(res, i)
            mask[o] = mask[o + 1] = True
    return mask


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    model: str
    n_data: int
    n_mc: int
    floating: tuple[str, ...] = ()
    data_seed: int = 101
    mc_seed: int = 201
    coup_seed: int = 11
    acceptance: bool = False


# The five configurations the build is measured on (sizes, models, floating lineshapes).
WORKLOADS = {
    "single_kstar_10k": Workload("single_kstar_10k", "kstar892", 10_000, 100_000, (), 101, 201),
    "full_500k": Workload("full_500k", "full", 500_000, 2_000_000, (), 102, 202),
    "full_grad_1m": Workload("full_grad_1m", "full", 1_000_000, 2_000_000, ("K*(1410)", "Z(4430)"), 103, 203),
    "learned_eff_1m": Workload("learned_eff_1m", "full", 1_000_000, 2_000_000, (), 104, 204, acceptance=True),
    "large_2z_10m": Workload("large_2z_10m", "full2z", 10_000_000, 20_000_000, ("K*(1410)", "Z(4430)"), 105, 205,
                             acceptance=True),
}


def acceptance_coefficients(seed: int = 300) -> np.ndarray:
    """a[d][l], d over (m_Kpi, cos theta_K*, cos theta_J/psi, phi), l = 1..3, from U[-1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(4, 3))


def neutral_events(n: int, seed: int, peaked: bool = False, edges: bool = False) -> np.ndarray:
    """Seeded observables (m_Kpi, cos theta_K*, cos theta_J/psi, phi), shape (4, n).

    m is uniform on the kinematic range, or (peaked=True) a 40/60 mix of a Cauchy
    peak at 0.896 GeV (half-width 0.03, truncated to the range) and the uniform
    part, mimicking data dominated by K*(892).  Angles are uniform.  With edges=True
    the first events are the boundary cases: threshold and end-point masses,
    cos = +-1 and phi = +-pi.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.uniform(M_LO, M_HI, size=n)
    if peaked:
        sel = rng.uniform(size=n) < 0.4
        c = 0.896 + 0.03 * np.tan(math.pi * (rng.uniform(size=n) - 0.5))
        c = np.where((c > M_LO) & (c < M_HI), c, m)
        m = np.where(sel, c, m)
    ck = rng.uniform(-1.0, 1.0, size=n)
    cj = rng.uniform(-1.0, 1.0, size=n)
    phi = rng.uniform(-math.pi, math.pi, size=n)
    ev = np.stack([m, ck, cj, phi])
    if edges and n >= 8:
        e = np.array([
            [M_LO, 0.3, -0.2, 1.0],
            [M_HI, -0.7, 0.4, -2.0],
            [1.0, 1.0, 0.5, 0.3],
            [1.2, -1.0, -0.5, -0.3],
            [0.9, 0.2, 1.0, 2.5],
            [0.95, -0.4, -1.0, -2.5],
            [1.5, 0.6, 0.1, math.pi],
            [1.7, -0.1, 0.9, -math.pi],
        ]).T
        ev[:, :8] = e
    return np.ascontiguousarray(ev)


def canonical(res: list[Resonance], par) -> np.ndarray:
    """Map every coupling pair to magnitude >= 0 and phase in (-pi, pi]: (r, phi) and
    (-r, phi + pi), and phases 2 pi apart, are the same point of the likelihood."""
    p = np.array(par, dtype=np.float64, copy=True)
    nc = sum(2 * r.n_coup for r in res)
    for k in range(0, nc, 2):
        if p[k] < 0:
            p[k] = -p[k]
            p[k + 1] += math.pi
        p[k + 1] = math.remainder(p[k + 1], 2 * math.pi)
    return p


# Efficiency network: 4 -> 64 -> 64 -> 1; parameter layout W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3.
MLP_NPARAMS = 4545


def mlp_init(seed: int = 0) -> np.ndarray:
    """Seeded starting point of the efficiency network (uniform Glorot ranges, zero biases,
    output bias at the logit of 0.6)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(MLP_NPARAMS, dtype=np.float32)
    a1, a2, a3 = np.sqrt(6 / (4 + 64)), np.sqrt(6 / (64 + 64)), np.sqrt(6 / (64 + 1))
    p[0:256] = rng.uniform(-a1, a1, 256) * 2.0
    p[320:4416] = rng.uniform(-a2, a2, 4096)
    p[4480:4544] = rng.uniform(-a3, a3, 64)
    p[4544] = np.log(0.6 / 0.4)
    return p


# Background shape of the signal + background study: a product of two 2D Bernstein
# polynomials of degree 3, over (m_Kpi, cos theta_K*) and (cos theta_J/psi, phi), with seeded
# positive coefficients (the paper's generic background shapes are 2D Bernstein polynomials
# passed to the fit as 2D x 2D histograms).
def background_coefficients(seed: int = 400) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.2, 1.0, size=(4, 4)), rng.uniform(0.2, 1.0, size=(4, 4))


def _bernstein2(c: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """sum_ij c[i, j] B_i^3(u) B_j^3(v) for u, v in [0, 1]."""
    def basis(t):
        return np.stack([(1 - t) ** 3, 3 * t * (1 - t) ** 2, 3 * t ** 2 * (1 - t), t ** 3])
    return np.einsum("ij,i...,j...->...", c, basis(u), basis(v))


def background_templates(nbins=(40, 40, 40, 40), seed: int = 400) -> tuple[np.ndarray, np.ndarray]:
    """The background shape at the bin centres of a (m_Kpi, cos theta_K*) table and a
    (cos theta_J/psi, phi) table, float32, row-major."""
    cm, ca = background_coefficients(seed)
    u = [(np.arange(n) + 0.5) / n for n in nbins]
    t1 = _bernstein2(cm, u[0][:, None], u[1][None, :])
    t2 = _bernstein2(ca, u[2][:, None], u[3][None, :])
    return t1.astype(np.float32), t2.astype(np.float32)


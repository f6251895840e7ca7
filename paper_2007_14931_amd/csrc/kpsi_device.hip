// Device code of the MI355X likelihood engine (gfx950).
//
//   invariants_kernel   once per event set: FP64 kinematics -> structure-of-arrays
//                       columns (breakup momenta, sines, phi as cos/sin, the Z-chain
//                       lineshape factors and angular factors of Eq. 10)
//   amp_kernel          per call: Eq. (2)-(5), (10)-(12) per event, -2 ln L terms and
//                       the adjoint of S with respect to every coupling and the
//                       floating masses/widths, reduced per block
//   reduce_final        fixed-order compensated sum of the block partials
//   phsp/accept kernels Philox4x32-10 phase-space and accept-reject generators
//
// Wavefronts are 64 lanes.  Every reduction is atomic-free and in a fixed order,
// so results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kpsi_internal.h"
#include "kpsi_math.h"

namespace kpsi {

// ------------------------------------------------------------------ math helpers
// rcp_, rsq_, fma_, the barrier polynomials and the d functions: kpsi_math.h
// natural log from the hardware base-2 logarithm, for normal inputs only: the FP32 path counts
// an event whose density is below the smallest normal float as a bad event (pos_floor)
__device__ __forceinline__ float log_(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
template <typename T> __device__ __forceinline__ constexpr T pos_floor() {
  if constexpr (std::is_same_v<T, float>) return 1.17549435e-38f;
  else return T(0);
}
__device__ __forceinline__ double log_(double x) { return log(x); }

template <typename T> __device__ __forceinline__ T ldnt(const T* p) { return __builtin_nontemporal_load(p); }
// Load at a uniform base plus a 32-bit per-lane byte offset: this maps onto the
// scalar-base + vector-offset address form, so no per-lane 64-bit address arithmetic.  The
// 32-byte FP64 column groups are loaded non-temporally; everything else with plain loads, which
// measured 3% faster than non-temporal ones in the FP32 kernel (and 1% slower in the FP64 one).
template <typename T> __device__ __forceinline__ T ldoff(const T* base, uint32_t off_bytes) {
  const T* p = (const T*)((const char*)base + off_bytes);
  if constexpr (sizeof(T) == 4 * sizeof(double)) return __builtin_nontemporal_load(p);
  else return *p;
}

// Opaque copy of a pointer to uniform kernel-argument data.  Re-deriving it inside the
// event loop keeps the compiler from hoisting every per-resonance constant out of the
// loop into vector registers: the constants are re-read with scalar loads instead.
template <typename P> using kconst_ptr = __attribute__((address_space(4))) const P*;
template <typename P> using lds_ptr = __attribute__((address_space(3))) P*;   // LDS (32-bit address)
template <typename P> __device__ __forceinline__ kconst_ptr<P> kernarg_laundered() {
  kconst_ptr<P> p = (kconst_ptr<P>)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return p;
}

// ------------------------------------------------------------------ invariants
// Columns written per event (type T, in groups of four at col_at(k, e, ld)):
//   K* chain  : m, q(m), p_B(m), cos/sin theta_K*, cos/sin theta_J/psi, cos/sin phi, and
//               q/m (column 10)
//   Z chain   : m^2_Jpsi pi (column 9), gZ = q/m_Jpsi pi (column 11), and the complex angular
//               factors Zang[l'][xi = +1] of Eq. (10) for l' = 0 (columns 12-13) and l' = +-1
//               combined through Eq. 11 (columns 14-15), each multiplied by
//               nZ = (p_B/M_B) / sqrt(1 + (r_B p_B)^2), the factor common to every Z amplitude.
//               The xi = -1 factors are (-Re, Im) of the xi = +1 ones and are not stored.
//               With free Z helicities (zfree), columns 14-15 hold F++ = Zang[+1][+1] and
//               16-17 F+- = Zang[+1][-1]; the l' = -1 factors are Zang[-1][+1] = -conj(F+-)
//               and Zang[-1][-1] = -conj(F++).
// All arithmetic in double; stored in T.
template <typename T>
__global__ __launch_bounds__(256) void invariants_kernel(InvArgs<T> a) {
  // One-time kinematics without contraction: at the threshold and end point of m_Kpi the
  // breakup momenta then round to exactly zero, as the plain double-precision definition does.
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n) return;
  const double mB = a.mB, mJ = a.mJ, mK = a.mK, mP = a.mPi;
  double m = a.obs[0][e], cK = a.obs[1][e], cJ = a.obs[2][e], ph = a.obs[3][e];
  // two-body momenta in the K pi frame and in the B frame
  const double s = m * m;
  const double q2 = (s - (mK + mP) * (mK + mP)) * (s - (mK - mP) * (mK - mP));
  const double q = q2 > 0.0 ? sqrt(q2) / (2.0 * m) : 0.0;
  const double mB2 = mB * mB;
  const double pb2 = (mB2 - (mJ + m) * (mJ + m)) * (mB2 - (mJ - m) * (mJ - m));
  const double pB = pb2 > 0.0 ? sqrt(pb2) / (2.0 * mB) : 0.0;
  const double sK = sqrt(fmax(0.0, (1.0 - cK) * (1.0 + cK)));
  const double sJ = sqrt(fmax(0.0, (1.0 - cJ) * (1.0 + cJ)));
  double sph, cph;
  sincos(ph, &sph, &cph);
  T* c = a.cols;
  const int64_t ld = a.ld;
  c[col_at(0, e, ld)] = (T)m;
  c[col_at(1, e, ld)] = (T)q;
  c[col_at(2, e, ld)] = (T)pB;
  c[col_at(3, e, ld)] = (T)cK;
  c[col_at(4, e, ld)] = (T)sK;
  c[col_at(5, e, ld)] = (T)cJ;
  c[col_at(6, e, ld)] = (T)sJ;
  c[col_at(7, e, ld)] = (T)cph;
  c[col_at(8, e, ld)] = (T)sph;
  c[col_at(10, e, ld)] = (T)(q / m);
  if (!a.with_z && !a.diag) return;

  // J/psi rest frame, reached by a boost along z from the B frame, in which the K pi
  // system moves along +z and the J/psi along -z.  The K pi system moves along +z in
  // the J/psi frame with gamma = p_Kpi.p_J/(m mJ) and gamma*beta = pB mB/(m mJ).
  const double EK = sqrt(mK * mK + q * q), EP = sqrt(mP * mP + q * q);
  const double g = (mB2 - s - mJ * mJ) / (2.0 * m * mJ);
  const double gb = pB * mB / (m * mJ);
  // K and pi momenta in the J/psi frame (x: K side of the hadron plane)
  const double kx = q * sK, kz = g * (q * cK) + gb * EK;
  const double px = -q * sK, pz = g * (-q * cK) + gb * EP;
  const double Epi = g * EP + gb * (-q * cK);
  // m^2_Jpsi pi = mJ^2 + mpi^2 + 2 mJ E_pi(J/psi frame)
  const double mz2 = mJ * mJ + mP * mP + 2.0 * mJ * Epi;
  const double mz = sqrt(mz2);
  // cos theta_Z from invariants: K and pi energies and momenta in the J/psi pi frame
  const double EKz = (mB2 - mz2 - mK * mK) / (2.0 * mz);
  const double EPz = (mz2 + mP * mP - mJ * mJ) / (2.0 * mz);
  const double pKz = sqrt(fmax(0.0, EKz * EKz - mK * mK)), pPz = sqrt(fmax(0.0, EPz * EPz - mP * mP));
  const double dotKP = EKz * EPz - 0.5 * (s - mK * mK - mP * mP);
  double cZ = (pKz * pPz > 0.0) ? dotKP / (pKz * pPz) : 1.0;
  cZ = fmin(1.0, fmax(-1.0, cZ));
  const double sZ = sqrt(fmax(0.0, (1.0 - cZ) * (1.0 + cZ)));
  // Z-chain frame in the J/psi frame: n2 = -pi direction, x2 = K side perpendicular to n2
  const double pn = sqrt(px * px + pz * pz);
  const double n2x = -px / pn, n2z = -pz / pn;       // (y component is zero: hadron plane is x-z)
  const double kd = kx * n2x + kz * n2z;
  double x2x = kx - kd * n2x, x2z = kz - kd * n2z;
  const double kn = sqrt(x2x * x2x + x2z * x2z);
  if (kn * kn > 1e-24 * (kx * kx + kz * kz)) { x2x /= kn; x2z /= kn; }
  else {  // collinear hadrons: take the K* frame's x axis projected off n2
    const double d1 = n2x;
    x2x = 1.0 - d1 * n2x; x2z = -d1 * n2z;
    const double nn = sqrt(x2x * x2x + x2z * x2z);
    x2x /= nn; x2z /= nn;
  }
  // y2 = n2 x x2 (only the y component survives for vectors in the x-z plane)
  const double y2y = n2z * x2x - n2x * x2z;
  // mu+ direction in the J/psi frame: theta_J/psi from n1 = -z, azimuth phi from x1 = +x,
  // right-handed about n1 (y1 = -y)
  const double ux = sJ * cph, uy = -sJ * sph, uz = -cJ;
  const double ct = ux * n2x + uz * n2z;                 // cos theta~
  const double ux2 = ux * x2x + uz * x2z;                 // sin theta~ cos phi~
  const double uy2 = uy * y2y;                            // sin theta~ sin phi~
  const double st = sqrt(ux2 * ux2 + uy2 * uy2);
  double cpt = 1.0, spt = 0.0;
  if (st > 0.0) { cpt = ux2 / st; spt = uy2 / st; }
  // muon helicity frame x axes: x' = cos(theta)(cos(phi) x + sin(phi) y) - sin(theta) n
  //  K* chain: x1 = +x, y1 = -y, n1 = -z
  const double xa_x = cJ * cph, xa_y = -cJ * sph, xa_z = sJ;
  //  Z chain
  const double xb_x = ct * (cpt * x2x) - st * n2x;
  const double xb_y = ct * (spt * y2y);
  const double xb_z = ct * (cpt * x2z) - st * n2z;
  // alpha: rotation about mu+ taking the Z-chain axis xb onto the K*-chain axis xa
  const double ca = xb_x * xa_x + xb_y * xa_y + xb_z * xa_z;
  const double crx = xb_y * xa_z - xb_z * xa_y, cry = xb_z * xa_x - xb_x * xa_z, crz = xb_x * xa_y - xb_y * xa_x;
  const double sa = crx * ux + cry * uy + crz * uz;
  if (a.diag) {
    double* o = a.diag + 5 * e;
    o[0] = mz; o[1] = cZ; o[2] = ct; o[3] = atan2(spt, cpt); o[4] = atan2(sa, ca);
  }
  if (!a.with_z) return;
  // Z lineshape factors (B -> Z K with L_B = 1, Z -> J/psi pi with L_R = 0)
  const double qz2 = (mz2 - (mJ + mP) * (mJ + mP)) * (mz2 - (mJ - mP) * (mJ - mP));
  const double qz = qz2 > 0.0 ? sqrt(qz2) / (2.0 * mz) : 0.0;
  const double pbz2 = (mB2 - (mz + mK) * (mz + mK)) * (mB2 - (mz - mK) * (mz - mK));
  const double pbz = pbz2 > 0.0 ? sqrt(pbz2) / (2.0 * mB) : 0.0;
  const double zb = a.rB * pbz * a.rB * pbz;
  const double nZ = (pbz / mB) / sqrt(1.0 + zb);
  c[col_at(9, e, ld)] = (T)mz2;
  c[col_at(11, e, ld)] = (T)(qz / mz);
  // Angular factors of Eq. (10): d^1_{0l'}(theta_Z) e^{i l' phi~} d^1_{l' xi}(theta~) e^{i xi alpha},
  // times nZ
  const double r2 = 0.7071067811865475244 * nZ;
  //  l' = 0:  xi = +1: cZ st/sqrt2 e^{i alpha};  xi = -1: -cZ st/sqrt2 e^{-i alpha}
  //  (xi = -1 is -z0 ca + i z0 sa: minus the real part, the same imaginary part)
  const double z0 = cZ * st * r2;
  c[col_at(12, e, ld)] = (T)(z0 * ca);
  c[col_at(13, e, ld)] = (T)(z0 * sa);
  //  l' = +-1 (H'_{-1} = H'_{+1}):  xi = +1: sZ/sqrt2 (ct cpt + i spt) e^{i alpha}
  //                                 xi = -1: sZ/sqrt2 (-ct cpt + i spt) e^{-i alpha}, again
  //                                 (-Re, Im) of the xi = +1 factor
  const double z1 = sZ * r2;
  if (a.zfree) {
    // l' = +1 alone: d^1_{0,1}(theta_Z) = sZ/sqrt2, d^1_{1,xi}(theta~) = (1 + xi ct)/2, phases
    // e^{i (phi~ + xi alpha)}
    const double up = 0.5 * z1 * (1.0 + ct), dn = 0.5 * z1 * (1.0 - ct);
    c[col_at(14, e, ld)] = (T)(up * (cpt * ca - spt * sa));
    c[col_at(15, e, ld)] = (T)(up * (spt * ca + cpt * sa));
    c[col_at(16, e, ld)] = (T)(dn * (cpt * ca + spt * sa));
    c[col_at(17, e, ld)] = (T)(dn * (spt * ca - cpt * sa));
    return;
  }
  const double pr = ct * cpt, pi_ = spt;
  c[col_at(14, e, ld)] = (T)(z1 * (pr * ca - pi_ * sa));
  c[col_at(15, e, ld)] = (T)(z1 * (pr * sa + pi_ * ca));
}

// ------------------------------------------------------------------ cross-lane exchange
// One step of a transposed butterfly at distance D = 32 or 16 on a pair of per-lane values:
// lanes whose bit log2(D) is clear end with (their lo, the partner's lo), the others with
// (the partner's hi, their hi), so lo + hi is the pair sum each lane keeps.  v_permlane32_swap
// exchanges lanes 32-63 of its first operand with lanes 0-31 of its second; v_permlane16_swap
// exchanges the odd 16-lane rows of the first with the even rows of the second.
template <int D> __device__ __forceinline__ void swap_halves(double& lo, double& hi) {
  static_assert(D == 32 || D == 16, "lane-swap distance");
  const uint64_t a = __builtin_bit_cast(uint64_t, lo), b = __builtin_bit_cast(uint64_t, hi);
  const unsigned al = (unsigned)a, ah = (unsigned)(a >> 32), bl = (unsigned)b, bh = (unsigned)(b >> 32);
  unsigned nl0, nl1, nh0, nh1;
  if constexpr (D == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
    nl0 = l[0]; nl1 = l[1]; nh0 = h[0]; nh1 = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
    nl0 = l[0]; nl1 = l[1]; nh0 = h[0]; nh1 = h[1];
  }
  lo = __builtin_bit_cast(double, ((uint64_t)nh0 << 32) | nl0);
  hi = __builtin_bit_cast(double, ((uint64_t)nh1 << 32) | nl1);
}
template <int D> __device__ __forceinline__ void swap_halves(float& lo, float& hi) {
  static_assert(D == 32 || D == 16, "lane-swap distance");
  const unsigned a = __builtin_bit_cast(unsigned, lo), b = __builtin_bit_cast(unsigned, hi);
  unsigned n0, n1;
  if constexpr (D == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    n0 = r[0]; n1 = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    n0 = r[0]; n1 = r[1];
  }
  lo = __builtin_bit_cast(float, n0);
  hi = __builtin_bit_cast(float, n1);
}
// The value of the partner lane in a butterfly step of width H = 8, 4, 2, 1 within each 16-lane
// row, by DPP: row_mirror (lane i <-> 15 - i), row_half_mirror (i <-> 7 - i in each half row),
// and the quad permutations (i <-> i ^ 2, i <-> i ^ 1).  Each pairs lanes whose bit log2(H)
// differs and whose higher bits agree, which is what the transposed butterfly needs.
template <int H> __device__ __forceinline__ unsigned dpp_partner(unsigned x) {
  static_assert(H == 8 || H == 4 || H == 2 || H == 1, "butterfly width");
  constexpr int ctrl = H == 8 ? 0x140 : (H == 4 ? 0x141 : (H == 2 ? 0x4E : 0xB1));
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, ctrl, 0xF, 0xF, false);
}
template <int H> __device__ __forceinline__ float dpp_partner(float x) {
  return __builtin_bit_cast(float, dpp_partner<H>(__builtin_bit_cast(unsigned, x)));
}
template <int H> __device__ __forceinline__ double dpp_partner(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint64_t lo = dpp_partner<H>((unsigned)b), hi = dpp_partner<H>((unsigned)(b >> 32));
  return __builtin_bit_cast(double, (hi << 32) | lo);
}

// ------------------------------------------------------------------ compensated sums
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
  s = t;
}
// Merge of two compensated sums; the two-sum error term is exact, so merging (a, b) and
// (b, a) gives the same result.
__device__ __forceinline__ void two_sum_merge(double& s, double& c, double s2, double c2) {
  const double t = s + s2;
  const double bp = t - s;
  const double err = (s - (t - bp)) + (s2 - bp);
  s = t;
  c = c + c2 + err;
}

// ------------------------------------------------------------------ per-event amplitude
template <typename T> struct Cx { T re, im; };
template <typename T> __device__ __forceinline__ void cmac(Cx<T>& acc, T ar, T ai, T br, T bi) {
  acc.re = fma_(ar, br, fma_(-ai, bi, acc.re));
  acc.im = fma_(ar, bi, fma_(ai, br, acc.im));
}

// (gr, gi) += A V: the per-event gradient contribution, fused into the accumulators
template <typename T> __device__ __forceinline__ void cacc(T& gr, T& gi, const Cx<T>& A, const Cx<T>& V) {
  gr = fma_(A.re, V.re, fma_(-A.im, V.im, gr));
  gi = fma_(A.re, V.im, fma_(A.im, V.re, gi));
}

// Lineshape-parameter derivatives of one floating resonance.  B = 1/(M^2 - m^2 - i P g) is its
// bare Breit-Wigner and Q = sum_lambda H'_lambda V'_lambda its adjoint weight, so X = B Q is
// the resonance's share of dS/dA times A.  With A = K n B (K and P depending on M, P also on
// Gamma0 = P/PoG):
//   dS/dM      = Re[X (kappa - (2M - i P' g) B)],   kappa = d ln K/dM, P' = dP/dM
//   dS/dGamma0 = Re[X i PoG g B] = -PoG g Im[X B]
// The slot's 0/1 selectors f0, f1 route the two derivatives to floating slot 0 or 1.
template <typename T, typename R>
__device__ __forceinline__ void flt_deriv(const R& rc, const Cx<T>& B, const Cx<T>& Q, T g, T& gM0, T& gG0, T& gM1,
                                          T& gG1) {
  const T Xr = B.re * Q.re - B.im * Q.im, Xi = B.re * Q.im + B.im * Q.re;
  const T pg = rc.dP * g;
  const T Yr = fma_(rc.twoM, B.re, pg * B.im), Yi = fma_(rc.twoM, B.im, -pg * B.re);
  const T dM = fma_(rc.kap, Xr, -fma_(Xr, Yr, -Xi * Yi));
  const T dG = -rc.PoG * g * fma_(Xr, B.im, Xi * B.re);
  gM0 = fma_(rc.f0, dM, gM0);
  gG0 = fma_(rc.f0, dG, gG0);
  gM1 = fma_(rc.f1, dM, gM1);
  gG1 = fma_(rc.f1, dG, gG1);
}

template <class Sh> __host__ __device__ constexpr int acc_base(int J) {   // accumulator offset of spin J
  int b = 3;
  for (int j = 0; j < J; ++j) b += Sh::N[j] * (j == 0 ? 2 : 6);
  return b;
}

// Accumulator indices (per block record of NACC doubles):
//   0, 1 : main sum and its (negated Kahan) compensation, total = [0] + [1]
//          (data: sum ln S; norm: sum eps S).  Gradient mode, flavour tags with the Eq. 14
//          mixture: data slot 0 is the whole sum and slot 1 the - flavour's sum of w S
//   2    : number of data events with S <= 0 or non-finite
//   then per K* slot (spin order) 2 (spin 0) or 6 (lambda = -1, 0, +1) values re/im of
//   sum w * dS/dH' with H' = K H (before the factor 2), then per Z slot 4 values
//   (lambda' = 0, +-1), then 2 per floating slot (d/dM, d/dGamma0).

// The gradient kernel of the large shape asks for 4 (FP32) or 2 (FP64) wavefronts per SIMD, at
// most 128 or 256 registers; its spin-1..3 accumulators live in LDS to make room (36 values x
// 256 threads: 36 KB per block in FP32, 4 blocks per compute unit; 72 KB in FP64, 2 blocks).
// The FP64 likelihood-only and density kernels of the large shape ask for 4 (128 registers).
template <typename T, class Sh, int MODE> struct AmpWaves {
  static constexpr bool lds = MODE == MODE_GRAD && Sh::LDS_HI > Sh::LDS_LO;
  static constexpr bool f32 = std::is_same<T, float>::value;
  static constexpr int v = lds ? (f32 ? 4 : 2) : (!f32 && Sh::NK > 1 ? 4 : 1);
};
// CC: flavour-tagged events (text after Eq. 12).  Data events carry a tag q = +-1 and are read
// with phi -> q phi, plus the other flavour with the mistag weight; the normalisation events run
// twice, as record 1 (phi) and record 2 (-phi), blocks [nb_data + nb_mc, nb_data + 2 nb_mc).
// ZF: one Z whose H'_{+1} and H'_{-1} are independent couplings (no Eq. 11 relation); its
// lambda' = -1 accumulators use the record slots of the second Z.
template <typename T, class Sh, int MODE, bool CC, bool ZF>
__global__ __launch_bounds__(256, (AmpWaves<T, Sh, MODE>::v)) void amp_kernel(const AmpArgs<T, Sh> a) {
  constexpr int NK = Sh::NK;
  static_assert(!ZF || Sh::NZ >= 2, "free Z helicities use the second Z's record slots");
  constexpr int NZ = ZF ? 1 : Sh::NZ;   // Z slots evaluated
  constexpr bool GRAD = (MODE == MODE_GRAD);
  using A_t = typename AccType<T>::type;   // per-thread gradient accumulator type

  const int set = (blockIdx.x < (unsigned)a.nb_data)
                      ? 0
                      : ((!CC || blockIdx.x < (unsigned)(a.nb_data + a.nb_mc)) ? 1 : 2);
  const int src = set == 0 ? 0 : 1;   // event set read by this block
  const int64_t blk = (int64_t)blockIdx.x - (set == 0 ? 0 : (set == 1 ? a.nb_data : a.nb_data + a.nb_mc));
  const int64_t n = a.n[src];
  const T* __restrict__ col = a.cols[src];
  const int64_t ld = a.ld[src];
  const int64_t e0 = blk * (int64_t)a.chunk;
  const int64_t e1 = (e0 + a.chunk < n) ? e0 + a.chunk : n;

  double ms = 0.0, mc = 0.0;   // Kahan pair
  float nbad = 0.f;   // events with a non-positive or non-finite density (exact count)
  // Eq. 14 mixture on the data set: background weight k from the reduced normalisation total
  const bool mix = (set == 0) && a.bkg_data != nullptr;
  T kb = T(0), kb2 = T(0);   // background weight k (flavour tags: of the + and - flavours)
  if (mix) {
    constexpr int NR = CC ? 2 : 1;   // normalisation records: phi (and -phi with tags)
    double tot[2] = {0.0, 0.0};
    if (a.mc_part) {
      // sum eps S over the normalisation blocks in a fixed order (the same in every block):
      // strided compensated sums per lane, a butterfly of exact two-sum merges in each
      // wavefront (both partners get the same result), then the four wavefronts in order
      __shared__ double kred[4][2 * NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double s = 0.0, c = 0.0;
        const double* mp = a.mc_part + r * a.mc_nb;
        for (int b = threadIdx.x; b < a.mc_nb; b += 256) {
          neumaier(s, c, mp[b]);
          neumaier(s, c, mp[a.pstride + b]);   // value 1: the Kahan correction
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) two_sum_merge(s, c, __shfl_xor(s, off, 64), __shfl_xor(c, off, 64));
        if ((threadIdx.x & 63) == 0) {
          kred[threadIdx.x >> 6][2 * r] = s;
          kred[threadIdx.x >> 6][2 * r + 1] = c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double s = kred[0][2 * r], c = kred[0][2 * r + 1];
        for (int w = 1; w < 4; ++w) two_sum_merge(s, c, kred[w][2 * r], kred[w][2 * r + 1]);
        tot[r] = s + c;
      }
    } else {
      tot[0] = a.norm_total[0] + a.norm_total[1];
      if (CC) tot[1] = a.norm_total[NACC] + a.norm_total[NACC + 1];
    }
    if constexpr (CC) {
      // N_q = (1 - w) I(q) + w I(-q) for the event's flavour q
      const double wm = (double)a.mistag, kp = 1.0 - wm;
      kb = (T)(a.bkg_coef * (kp * tot[0] + wm * tot[1]));
      kb2 = (T)(a.bkg_coef * (kp * tot[1] + wm * tot[0]));
    } else {
      kb = (T)(a.bkg_coef * tot[0]);
    }
  }
  A_t ws = A_t(0);    // sum_i w_i S_i (mixture, gradient mode; with tags: the + flavour's events)
  A_t ws2 = A_t(0);   // with tags: the same over the - flavour's events
  // accumulators gk[LO, HI) live in this thread's LDS column accl[.][tid] (gradient kernel)
  constexpr bool LDSACC = GRAD && (Sh::LDS_HI > Sh::LDS_LO);
  constexpr int LO = LDSACC ? Sh::LDS_LO : 0, HI = LDSACC ? Sh::LDS_HI : 0;
  __shared__ A_t accl[HI > LO ? HI - LO : 1][256];
  if constexpr (LDSACC) {
#pragma unroll
    for (int i = 0; i < HI - LO; ++i) accl[i][threadIdx.x] = A_t(0);
  }
  A_t gk[Sh::NKACC > 0 ? Sh::NKACC : 1];
  A_t gz[NZ > 0 ? 4 * Sh::NZ : 1];
  static_assert(NFL == 2, "floating accumulators are named registers for two slots");
  A_t gM0 = 0, gG0 = 0, gM1 = 0, gG1 = 0;   // d/dM, d/dGamma0 of floating slots 0 and 1
  if constexpr (GRAD) {
#pragma unroll
    for (int i = 0; i < Sh::NKACC; ++i) gk[i] = 0;
#pragma unroll
    for (int i = 0; i < 4 * Sh::NZ; ++i) gz[i] = 0;
  }

  using V4 = T __attribute__((ext_vector_type(4)));
  const V4* __restrict__ gb = (const V4*)col + e0;   // column group 0 at this block's first event
  const uint32_t n_blk = (uint32_t)(e1 > e0 ? e1 - e0 : 0);
  for (uint32_t i = threadIdx.x; i < n_blk; i += 256) {
    const int64_t e = e0 + i;
    const uint32_t ob = i * (uint32_t)sizeof(T);
    const uint32_t ob4 = i * (uint32_t)sizeof(V4);
    const auto& ka = *kernarg_laundered<AmpArgs<T, Sh>>();
    // this thread's LDS accumulator column, re-derived opaquely each event so the compiler keeps
    // the accumulators in LDS instead of promoting them back into registers across the loop
    lds_ptr<A_t> accb = (lds_ptr<A_t>)&accl[0][threadIdx.x];
    if constexpr (LDSACC) asm volatile("" : "+v"(accb));
    const V4 g0 = ldoff(gb, ob4), g1 = ldoff(gb + ld, ob4), g2 = ldoff(gb + 2 * ld, ob4);
    const T m = g0.x, q = g0.y, pB = g0.z, cK = g0.w;
    const T sK = g1.x, cJ = g1.y, sJ = g1.z, cph = g1.w;
    const T sph = g2.x, qm = g2.z;   // q/m from the event columns

    const T m2 = m * m;
    const T zR = (ka.rR * q) * (ka.rR * q);
    const T zB = (ka.rB * pB) * (ka.rB * pB);
    const T pbm = pB * ka.invMB;
    const T qq = q * q;

    // ---- K* lineshapes (Eq. 2-3) and coupling sums T_{J lambda}
    // Each resonance's amplitude is K n_J(m) B_R(m) with B_R = 1/(M^2 - m^2 - i P g_J(m)) the
    // bare Breit-Wigner, K the per-resonance constant and n_J the per-spin barrier and momentum
    // factor.  K is folded into the couplings on the host (H' = K H) and n_J into the angular
    // factors of its spin, so each resonance costs one complex reciprocal: Amp holds B_R.
    Cx<T> Amp[NK > 0 ? NK : 1];
    T gJv[5] = {T(0), T(0), T(0), T(0), T(0)};   // g_J(m) per spin (width derivative)
    T nJv[5] = {T(0), T(0), T(0), T(0), T(0)};   // n_J(m) per spin
    Cx<T> Tl[5][3];
#pragma unroll
    for (int J = 0; J < 5; ++J)
#pragma unroll
      for (int l = 0; l < 3; ++l) Tl[J][l] = Cx<T>{T(0), T(0)};

    // Every K* slot of the shape is evaluated: the host gives the slots the model leaves empty
    // zero couplings and the constants M^2 = P = 0 (a finite 1/D = -1/m^2), so they add nothing
    // and need no per-event test (the Z slots keep theirs: models often use one of the two).
    auto do_spin = [&](auto Jc) {
      constexpr int J = decltype(Jc)::value;
      if constexpr (Sh::N[J] > 0) {
        {
          constexpr int LB = LBof<J>::v;
          const T BR = bpoly<J>(zR), BB = bpoly<LB>(zB);
          const T rJ = rsq_(BR * BB);
          const T nJ = ipow<T, LB>(pbm) * ipow<T, J>(qm) * rJ;
          // 1/B_J(z_R) = rJ^2 B_LB(z_B): no second reciprocal
          T gJ = qm;
          if constexpr (J > 0) gJ = qm * ipow<T, J>(qq) * (rJ * rJ * BB);
          gJv[J] = gJ;
          nJv[J] = nJ;
          constexpr int sb = slot_base<Sh>(J);
#pragma unroll
          for (int j = 0; j < Sh::N[J]; ++j) {
            {
              const auto& rc = ka.ks[sb + j];
              const T dre = pole_gap(rc, m2);
              const T dim = rc.P * gJ;   // M Gamma(m)
              const T inv = rcp_(fma_(dre, dre, dim * dim));
              const T br = dre * inv, bi = dim * inv;
              T Ar = br, Ai = bi;
              if constexpr (J == 0) {
                if (rc.lass) {
                  // LASS (Eq. 7-8): with u = q cot(delta_B) = 1/a + b q^2/2 (finite at threshold),
                  // (m/q) sin(delta_B) e^{i delta_B} = m (u + i q)/(u^2 + q^2) and
                  // e^{2 i delta_B} = (u + i q)^2/(u^2 + q^2); the resonant term is the
                  // Breit-Wigner above times P = M^2 Gamma0/q0 and e^{2 i delta_B}
                  const T u = fma_(rc.lhb, qq, rc.lai);
                  const T dn = rcp_(fma_(u, u, qq));
                  const T er = (u * u - qq) * dn, ei = T(2) * u * q * dn;
                  const T md = m * dn;
                  Ar = fma_(md, u, rc.P * (er * br - ei * bi));
                  Ai = fma_(md, q, rc.P * (er * bi + ei * br));
                }
              }
              Amp[sb + j] = Cx<T>{Ar, Ai};
              if constexpr (J == 0) {
                cmac(Tl[0][1], rc.hr[1], rc.hi[1], Ar, Ai);
              } else {
#pragma unroll
                for (int l = 0; l < 3; ++l) cmac(Tl[J][l], rc.hr[l], rc.hi[l], Ar, Ai);
              }
            }
          }
        }
      }
    };
    do_spin(std::integral_constant<int, 0>{});
    do_spin(std::integral_constant<int, 1>{});
    do_spin(std::integral_constant<int, 2>{});
    do_spin(std::integral_constant<int, 3>{});
    do_spin(std::integral_constant<int, 4>{});

    // ---- angular sums (Eq. 4): U_lambda = sum_J d^J_{lambda 0}(theta_K) T_{J lambda}
    // (n_J times the d functions; the n_J of spins absent from the model are zero)
    T dd0[5], dd1[5];
    dd0[0] = nJv[0]; dd1[0] = T(0);
    dd0[1] = nJv[1] * d00<1>(cK); dd1[1] = nJv[1] * d10<1>(cK, sK);
    dd0[2] = nJv[2] * d00<2>(cK); dd1[2] = nJv[2] * d10<2>(cK, sK);
    dd0[3] = nJv[3] * d00<3>(cK); dd1[3] = nJv[3] * d10<3>(cK, sK);
    dd0[4] = nJv[4] * d00<4>(cK); dd1[4] = nJv[4] * d10<4>(cK, sK);
    Cx<T> U0{T(0), T(0)}, Up{T(0), T(0)}, Um{T(0), T(0)};
#pragma unroll
    for (int J = 0; J < 5; ++J) {
      if (Sh::N[J] == 0) continue;
      U0.re = fma_(dd0[J], Tl[J][1].re, U0.re);
      U0.im = fma_(dd0[J], Tl[J][1].im, U0.im);
      if (J > 0) {
        Up.re = fma_(dd1[J], Tl[J][2].re, Up.re);
        Up.im = fma_(dd1[J], Tl[J][2].im, Up.im);
        Um.re = fma_(-dd1[J], Tl[J][0].re, Um.re);
        Um.im = fma_(-dd1[J], Tl[J][0].im, Um.im);
      }
    }
    // e^{i lambda phi} d^1_{lambda xi}(theta_J):  lambda=+1: (1+c)/2, (1-c)/2;  0: s/sqrt2, -s/sqrt2;
    // lambda=-1: (1-c)/2, (1+c)/2   for xi = +1, -1
    const T hp = T(0.5) * (T(1) + cJ), hm = T(0.5) * (T(1) - cJ), s0 = sJ * T(0.70710678118654752440);
    // Amplitudes a_xi (Eq. 12) of the event read with phi -> f phi.  f = -1 is the
    // charge-conjugate decay: e^{i lambda phi} becomes e^{-i lambda phi}, and the Z-chain azimuths
    // phi~ and alpha reverse, which conjugates the Z angular factors.
    auto kstar_at = [&](T f, Cx<T>& ap_, Cx<T>& am_) {
      const T sp = f * sph;
      const Cx<T> eUp{cph * Up.re - sp * Up.im, cph * Up.im + sp * Up.re};
      const Cx<T> eUm{cph * Um.re + sp * Um.im, cph * Um.im - sp * Um.re};
      ap_ = Cx<T>{hp * eUp.re + s0 * U0.re + hm * eUm.re, hp * eUp.im + s0 * U0.im + hm * eUm.im};
      am_ = Cx<T>{hm * eUp.re - s0 * U0.re + hp * eUm.re, hm * eUp.im - s0 * U0.im + hp * eUm.im};
    };
    // Zang[l'][xi] as (re, im) pairs: l' = 0 (xi = +1, -1), l' = +-1 or +1, then (ZF) l' = -1
    T za[ZF ? 12 : 8];
    auto z_add = [&](T f, const Cx<T>& T0, const Cx<T>& T1, const Cx<T>& T2, Cx<T>& ap_, Cx<T>& am_) {
      cmac(ap_, T0.re, T0.im, za[0], f * za[1]);
      cmac(am_, T0.re, T0.im, za[2], f * za[3]);
      cmac(ap_, T1.re, T1.im, za[4], f * za[5]);
      cmac(am_, T1.re, T1.im, za[6], f * za[7]);
      if constexpr (ZF) {
        cmac(ap_, T2.re, T2.im, za[8], f * za[9]);
        cmac(am_, T2.re, T2.im, za[10], f * za[11]);
      }
    };
    // flavour of this reading: the tag of a data event, + / - for the two normalisation records
    T f1 = T(1);
    if constexpr (CC) f1 = set == 0 ? ldoff(a.tag + e0, ob) : (set == 1 ? T(1) : T(-1));
    Cx<T> ap, am;
    kstar_at(f1, ap, am);

    // ---- Z chain (Eq. 10-12)
    // (AZ holds the bare Breit-Wigner; the Z barrier factor n_Z is in the angular columns)
    Cx<T> AZ[NZ > 0 ? NZ : 1];
    T gzv = T(0);
    Cx<T> T0k{T(0), T(0)}, T1k{T(0), T(0)}, T2k{T(0), T(0)};   // Z coupling sums, kept for a second reading
    if constexpr (NZ > 0) {
      if (a.cnt[5] > 0) {
        const T mz2 = g2.y;
        gzv = g2.w;
        // Zang[l'][xi]: for l' = 0 and the combined l' = +-1, xi = -1 is (-Re, Im) of xi = +1
        const V4 g3 = ldoff(gb + 3 * ld, ob4);
        za[0] = g3.x; za[1] = g3.y; za[2] = -g3.x; za[3] = g3.y;
        if constexpr (ZF) {
          // l' = +1: F++, F+-;  l' = -1: -conj(F+-), -conj(F++)
          const V4 g4 = ldoff(gb + 4 * ld, ob4);
          za[4] = g3.z; za[5] = g3.w; za[6] = g4.x; za[7] = g4.y;
          za[8] = -g4.x; za[9] = g4.y; za[10] = -g3.z; za[11] = g3.w;
        } else {
          za[4] = g3.z; za[5] = g3.w; za[6] = -g3.z; za[7] = g3.w;
        }
        Cx<T> T0{T(0), T(0)}, T1{T(0), T(0)}, T2{T(0), T(0)};
#pragma unroll
        for (int z = 0; z < NZ; ++z) {
          if (z < a.cnt[5]) {
            const auto& rc = ka.zs[z];
            const T dre = pole_gap(rc, mz2);
            const T dim = rc.P * gzv;
            const T inv = rcp_(fma_(dre, dre, dim * dim));
            AZ[z] = Cx<T>{dre * inv, dim * inv};
            cmac(T0, rc.hr[0], rc.hi[0], AZ[z].re, AZ[z].im);
            cmac(T1, rc.hr[1], rc.hi[1], AZ[z].re, AZ[z].im);
            if constexpr (ZF) cmac(T2, rc.hr[2], rc.hi[2], AZ[z].re, AZ[z].im);
          }
        }
        z_add(f1, T0, T1, T2, ap, am);
        if constexpr (CC) {
          T0k = T0;
          T1k = T1;
          if constexpr (ZF) T2k = T2;
        }
      }
    }

    const T S = ap.re * ap.re + ap.im * ap.im + am.re * am.re + am.im * am.im;

    if constexpr (MODE == MODE_DENSITY) {
      a.s_out[set][e] = (double)S;
      continue;
    }

    // ---- likelihood terms
    T w;
    T w2 = T(0);                  // mistag: adjoint weight of the other-flavour reading
    Cx<T> ap2{T(0), T(0)}, am2{T(0), T(0)};
    if (set == 0) {
      T arg = S;   // the quantity whose logarithm is summed
      if constexpr (CC) {
        T S2 = T(0);
        if (a.mistag > T(0)) {
          // t = (1 - w) S(q phi) + w S(-q phi)
          kstar_at(-f1, ap2, am2);
          if constexpr (NZ > 0) {
            if (a.cnt[5] > 0) z_add(-f1, T0k, T1k, T2k, ap2, am2);
          }
          S2 = ap2.re * ap2.re + ap2.im * ap2.im + am2.re * am2.re + am2.im * am2.im;
          arg = fma_(a.keep, S, a.mistag * S2);
        }
        // Eq. 14 with tags: t = p eps [(1 - w) S(q phi) + w S(-q phi)] + k_q b, k_q of the
        // event's flavour; d ln t / dS = p eps (1 - w) / t
        T pe = T(1);
        if (mix) {
          pe = a.purity * (a.eps_data ? ldoff(a.eps_data + e0, ob) : T(1));
          arg = fma_(pe, arg, (f1 > T(0) ? kb : kb2) * ldoff(a.bkg_data + e0, ob));
        }
        if (!(arg > pos_floor<T>()) || !(arg < T(INFINITY))) { nbad += 1.f; continue; }
        const T r = pe * rcp_(arg);
        if (a.mistag > T(0)) {
          w = a.keep * r;
          w2 = a.mistag * r;
        } else {
          w = r;
        }
        if (mix) {
          const A_t c = (A_t)fma_(w, S, w2 * S2);
          if (f1 > T(0)) ws += c;
          else ws2 += c;
        }
      } else if (mix) {
        // Eq. 14: t = p eps S + k b; d ln t / dS = p eps / t
        const T pe = a.purity * (a.eps_data ? ldoff(a.eps_data + e0, ob) : T(1));
        arg = fma_(pe, S, kb * ldoff(a.bkg_data + e0, ob));
        if (!(arg > pos_floor<T>()) || !(arg < T(INFINITY))) { nbad += 1.f; continue; }
        w = pe * rcp_(arg);
        ws += (A_t)(w * S);
      } else {
        if (!(S > pos_floor<T>()) || !(S < T(INFINITY))) { nbad += 1.f; continue; }
        w = rcp_(S);
      }
      const double x = (double)log_(arg);
      const double y = x - mc;
      const double t = ms + y;
      mc = (t - ms) - y;
      ms = t;
    } else {
      const T eps = a.eps ? ldoff(a.eps + e0, ob) : T(1);
      const double x = (double)(eps * S);
      const double y = x - mc;
      const double t = ms + y;
      mc = (t - ms) - y;
      ms = t;
      w = eps;
    }

    if constexpr (GRAD) {
      // adjoint of S = sum_xi |a_xi|^2: b_xi = w conj(a_xi); W_lambda = sum_xi E_{lambda xi} b_xi,
      // summed over the readings of the event
      Cx<T> W0, Wp, Wm;
      Cx<T> bp, bm, bp2{T(0), T(0)}, bm2{T(0), T(0)};
      auto adj_w = [&](auto first, T wt, T f, const Cx<T>& ap_, const Cx<T>& am_, Cx<T>& bp_, Cx<T>& bm_) {
        constexpr bool F = decltype(first)::value;
        bp_ = Cx<T>{wt * ap_.re, -wt * ap_.im};
        bm_ = Cx<T>{wt * am_.re, -wt * am_.im};
        const T sp = f * sph;
        const Cx<T> Wp0{hp * bp_.re + hm * bm_.re, hp * bp_.im + hm * bm_.im};
        const Cx<T> wp{cph * Wp0.re - sp * Wp0.im, cph * Wp0.im + sp * Wp0.re};   // e^{+i f phi}
        const Cx<T> w0{s0 * (bp_.re - bm_.re), s0 * (bp_.im - bm_.im)};
        const Cx<T> Wm0{hm * bp_.re + hp * bm_.re, hm * bp_.im + hp * bm_.im};
        const Cx<T> wm{cph * Wm0.re + sp * Wm0.im, cph * Wm0.im - sp * Wm0.re};   // e^{-i f phi}
        if constexpr (F) {
          Wp = wp; W0 = w0; Wm = wm;
        } else {
          Wp.re += wp.re; Wp.im += wp.im;
          W0.re += w0.re; W0.im += w0.im;
          Wm.re += wm.re; Wm.im += wm.im;
        }
      };
      adj_w(std::true_type{}, w, f1, ap, am, bp, bm);
      const bool two = CC && set == 0 && a.mistag > T(0);
      if constexpr (CC) {
        if (two) adj_w(std::false_type{}, w2, -f1, ap2, am2, bp2, bm2);
      }

      auto grad_spin = [&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        if constexpr (Sh::N[J] > 0) {
          {
            constexpr int sb = slot_base<Sh>(J);
            constexpr int ab = acc_base<Sh>(J) - 3;
            // V_{J lambda} = d^J_{lambda 0} W_lambda
            const Cx<T> V0{dd0[J] * W0.re, dd0[J] * W0.im};
            const Cx<T> Vp{dd1[J] * Wp.re, dd1[J] * Wp.im};
            const Cx<T> Vm{-dd1[J] * Wm.re, -dd1[J] * Wm.im};
#pragma unroll
            for (int j = 0; j < Sh::N[J]; ++j) {
              {
                const Cx<T> A = Amp[sb + j];
                const auto& rc = ka.ks[sb + j];
                Cx<T> Q{T(0), T(0)};
                if constexpr (J == 0) {
                  // accumulators += A V as two fused multiply-adds per component
                  cacc(gk[ab + 2 * j], gk[ab + 2 * j + 1], A, V0);
                  if (rc.flt >= 0) cmac(Q, rc.hr[1], rc.hi[1], V0.re, V0.im);
                } else if constexpr (LDSACC && J >= 1 && J <= 3) {
                  // ab + 6 j lies in [LO, HI): read-add-write this thread's own LDS slots (no other
                  // lane touches them, so no atomics)
                  lds_ptr<A_t> g = accb + 256 * (ab + 6 * j - LO);
                  A_t v[6];
#pragma unroll
                  for (int q = 0; q < 6; ++q) v[q] = g[256 * q];
                  cacc(v[0], v[1], A, Vm);
                  cacc(v[2], v[3], A, V0);
                  cacc(v[4], v[5], A, Vp);
#pragma unroll
                  for (int q = 0; q < 6; ++q) g[256 * q] = v[q];
                  if (rc.flt >= 0) {
                    cmac(Q, rc.hr[0], rc.hi[0], Vm.re, Vm.im);
                    cmac(Q, rc.hr[1], rc.hi[1], V0.re, V0.im);
                    cmac(Q, rc.hr[2], rc.hi[2], Vp.re, Vp.im);
                  }
                } else {
                  A_t* g = gk + ab + 6 * j;
                  cacc(g[0], g[1], A, Vm);
                  cacc(g[2], g[3], A, V0);
                  cacc(g[4], g[5], A, Vp);
                  if (rc.flt >= 0) {
                    cmac(Q, rc.hr[0], rc.hi[0], Vm.re, Vm.im);
                    cmac(Q, rc.hr[1], rc.hi[1], V0.re, V0.im);
                    cmac(Q, rc.hr[2], rc.hi[2], Vp.re, Vp.im);
                  }
                }
                if (rc.flt >= 0) flt_deriv(rc, A, Q, gJv[J], gM0, gG0, gM1, gG1);
              }
            }
          }
        }
      };
      grad_spin(std::integral_constant<int, 0>{});
      grad_spin(std::integral_constant<int, 1>{});
      grad_spin(std::integral_constant<int, 2>{});
      grad_spin(std::integral_constant<int, 3>{});
      grad_spin(std::integral_constant<int, 4>{});

      if constexpr (NZ > 0) {
        if (a.cnt[5] > 0) {
          // WZ_{l'} = sum_xi Zang_{l' xi} b_xi over the readings
          auto wz = [&](T f, const Cx<T>& bp_, const Cx<T>& bm_, Cx<T>& WZ0, Cx<T>& WZ1) {
            const T z1 = f * za[1], z3 = f * za[3], z5 = f * za[5], z7 = f * za[7];
            WZ0 = Cx<T>{za[0] * bp_.re - z1 * bp_.im + za[2] * bm_.re - z3 * bm_.im,
                        za[0] * bp_.im + z1 * bp_.re + za[2] * bm_.im + z3 * bm_.re};
            WZ1 = Cx<T>{za[4] * bp_.re - z5 * bp_.im + za[6] * bm_.re - z7 * bm_.im,
                        za[4] * bp_.im + z5 * bp_.re + za[6] * bm_.im + z7 * bm_.re};
          };
          // (free helicities) WZ_{-1} from the l' = -1 factors, same form; a generic lambda, so
          // that its body exists only in the instantiations that call it (za has 12 entries there)
          auto wz2 = [&](auto f, const auto& bp_, const auto& bm_) -> Cx<T> {
            const T z9 = f * za[9], z11 = f * za[11];
            return Cx<T>{za[8] * bp_.re - z9 * bp_.im + za[10] * bm_.re - z11 * bm_.im,
                         za[8] * bp_.im + z9 * bp_.re + za[10] * bm_.im + z11 * bm_.re};
          };
          Cx<T> WZ0, WZ1, WZ2{T(0), T(0)};
          wz(f1, bp, bm, WZ0, WZ1);
          if constexpr (ZF) WZ2 = wz2(f1, bp, bm);
          if constexpr (CC) {
            if (two) {
              Cx<T> X0, X1;
              wz(-f1, bp2, bm2, X0, X1);
              WZ0.re += X0.re; WZ0.im += X0.im;
              WZ1.re += X1.re; WZ1.im += X1.im;
              if constexpr (ZF) {
                const Cx<T> X2 = wz2(-f1, bp2, bm2);
                WZ2.re += X2.re; WZ2.im += X2.im;
              }
            }
          }
#pragma unroll
          for (int z = 0; z < NZ; ++z) {
            if (z < a.cnt[5]) {
              const Cx<T> A = AZ[z];
              A_t* g = gz + 4 * z;
              cacc(g[0], g[1], A, WZ0);
              cacc(g[2], g[3], A, WZ1);
              if constexpr (ZF) cacc(g[4], g[5], A, WZ2);   // the second Z's lambda' = 0 slots
              const auto& rc = ka.zs[z];
              if (rc.flt >= 0) {
                Cx<T> Q{T(0), T(0)};
                cmac(Q, rc.hr[0], rc.hi[0], WZ0.re, WZ0.im);
                cmac(Q, rc.hr[1], rc.hi[1], WZ1.re, WZ1.im);
                if constexpr (ZF) cmac(Q, rc.hr[2], rc.hi[2], WZ2.re, WZ2.im);
                flt_deriv(rc, A, Q, gzv, gM0, gG0, gM1, gG1);
              }
            }
          }
        }
      }
    }
  }

  if constexpr (MODE == MODE_DENSITY) return;

  // ---- block reduction: wave transpose-butterfly, then the 4 waves in order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double red[4][NACC];
  if constexpr (GRAD) {
    // accumulator i >= 2 of this lane at its accumulation type (compile-time index after
    // unrolling); 0 and 1 are the FP64 likelihood sums
    auto accf = [&](int i) -> A_t {
      if (i == 2) return (A_t)nbad;
      if (LDSACC && i >= 3 + LO && i < 3 + HI) return accl[i - 3 - LO][threadIdx.x];
      if (i < 3 + Sh::NKACC) return gk[i - 3];
      if (i < 3 + Sh::NKACC + 4 * Sh::NZ) return gz[i - 3 - Sh::NKACC];
      const int f = i - 3 - Sh::NKACC - 4 * Sh::NZ;
      if (f == 0) return gM0;
      if (f == 1) return gG0;
      if (f == 2) return gM1;
      if (f == 3) return gG1;
      if (f == 4) return ws;
      return A_t(0);
    };
    // Transpose butterfly: after the step of width h, lane l keeps h values, each summed
    // with its partner lane's; after the last step lane l holds the wave sum of value l.
    // The steps of width 32 and 16 use the lane-swap instructions (swap_halves), the rest DPP
    // row permutations (dpp_partner).  Slots 0 and 1 carry the FP64 likelihood sums and every value merged into
    // them (as double); the other slots move the accumulators at their own type (FP32 sums of
    // the wave's FP32 thread accumulators in the FP32 kernel).
    if constexpr (CC) {
      // tagged mixture: slot 1 carries the - flavour's sum of w S (the Kahan correction is
      // folded into slot 0 first)
      if (mix) {
        ms = ms - mc;
        mc = -(double)ws2;
      }
    }
    double d[2];
    A_t v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      if (i < 2) {
        double lo = (i == 0) ? ms : -mc;   // Kahan: the running sum exceeds the exact one by mc
        double hi = (double)accf(i + 32);
        swap_halves<32>(lo, hi);
        d[i] = lo + hi;
      } else {
        A_t lo = accf(i), hi = accf(i + 32);
        swap_halves<32>(lo, hi);
        v[i] = lo + hi;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i < 2) {
        double lo = d[i], hi = (double)v[i + 16];
        swap_halves<16>(lo, hi);
        d[i] = lo + hi;
      } else {
        A_t lo = v[i], hi = v[i + 16];
        swap_halves<16>(lo, hi);
        v[i] = lo + hi;
      }
    }
    auto narrow = [&](auto Hc) {
      constexpr int half = decltype(Hc)::value;
      const bool up = lane & half;
#pragma unroll
      for (int i = 0; i < half; ++i) {
        if (i < 2) {
          const double hv = (i + half < 2) ? d[i + half] : (double)v[i + half];
          const double keep = up ? hv : d[i];
          const double send = up ? d[i] : hv;
          d[i] = keep + dpp_partner<half>(send);
        } else {
          // (the empty asm keeps the two slots as values, so that the selects below stay
          // selects instead of becoming a lane-dependent index into the slot array)
          A_t a0 = v[i], a1 = v[i + half];
          asm("" : "+v"(a0), "+v"(a1));
          const A_t keep = up ? a1 : a0;
          const A_t send = up ? a0 : a1;
          v[i] = keep + dpp_partner<half>(send);
        }
      }
    };
    narrow(std::integral_constant<int, 8>{});
    narrow(std::integral_constant<int, 4>{});
    narrow(std::integral_constant<int, 2>{});
    narrow(std::integral_constant<int, 1>{});
    red[wave][lane] = d[0];
  } else {
    double v0 = ms, v1 = -mc, v2 = (double)nbad;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
      v0 += __shfl_xor(v0, s, 64);
      v1 += __shfl_xor(v1, s, 64);
      v2 += __shfl_xor(v2, s, 64);
    }
    if (lane < NACC) red[wave][lane] = (lane == 0) ? v0 : (lane == 1 ? v1 : (lane == 2 ? v2 : 0.0));
  }
  __syncthreads();
  if (wave == 0) {
    const double t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    // value-major layout: value v of block b at partial[v * gridDim.x + b]
    if (GRAD || lane < 3) a.partial[(int64_t)lane * a.pstride + a.poff + blockIdx.x] = t;
  }
}

// Fixed-order compensated sum of the block partials.  Block (set, v) sums value v over the
// blocks of one set: each thread runs a Neumaier sum over a strided subset, the pairs are merged
// in a butterfly within each wavefront and the four wavefronts in order.  Output goes to
// out[set*NACC + v] (mapped pinned host memory).  The partial rows hold the data blocks, then n_mc_sets runs of
// nb_mc normalisation blocks (records 1, 2).

__global__ __launch_bounds__(256) void reduce_final(const double* __restrict__ partial, int nb_data, int nb_mc,
                                                    int n_mc_sets, int nv, double* __restrict__ out, int first_set) {
  const int set = first_set + (int)blockIdx.x / nv, v = blockIdx.x % nv;
  const int64_t nbt = nb_data + (int64_t)n_mc_sets * nb_mc;   // row stride of the partials
  const int b0 = set == 0 ? 0 : nb_data + (set - 1) * nb_mc;
  const int nb = set ? nb_mc : nb_data;
  const double* __restrict__ p = partial + (int64_t)v * nbt + b0;
  double s = 0.0, c = 0.0;
  // blocks tid, tid + 256, ... in that order; four loads are issued before their sums, so a
  // thread waits for memory once per four values rather than once per value
  for (int b0 = threadIdx.x; b0 < nb; b0 += 4 * 256) {
    double x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = b0 + k * 256 < nb ? p[b0 + k * 256] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (b0 + k * 256 < nb) neumaier(s, c, x[k]);
  }
  // butterfly of exact two-sum merges in each wavefront (every lane ends with the wavefront's
  // total), then the four wavefronts in order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) two_sum_merge(s, c, __shfl_xor(s, off, 64), __shfl_xor(c, off, 64));
  __shared__ double S[4], Cc[4];
  if ((threadIdx.x & 63) == 0) {
    S[threadIdx.x >> 6] = s;
    Cc[threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = S[0], tc = Cc[0];
    for (int w = 1; w < 4; ++w) two_sum_merge(t, tc, S[w], Cc[w]);
    out[set * NACC + v] = t + tc;
  }
}

// ------------------------------------------------------------------ efficiency histogram
__global__ __launch_bounds__(256) void hist_lookup_kernel(HistArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n) return;
  int64_t idx = 0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const double x = a.obs[d][e];
    int b = (int)floor((x - a.lo[d]) / (a.hi[d] - a.lo[d]) * a.nb[d]);
    b = b < 0 ? 0 : (b >= a.nb[d] ? a.nb[d] - 1 : b);
    idx = idx * a.nb[d] + b;
  }
  a.out_f64[e] = (double)a.table[idx];
}

// ------------------------------------------------------------------ 2D x 2D templates
__global__ __launch_bounds__(256) void template_kernel(TplArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n) return;
  int b[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const double x = a.obs[d][e];
    int k = (int)floor((x - a.lo[d]) / (a.hi[d] - a.lo[d]) * a.nb[d]);
    b[d] = k < 0 ? 0 : (k >= a.nb[d] ? a.nb[d] - 1 : k);
  }
  a.out[e] = (double)a.t1[b[0] * a.nb[1] + b[1]] * (double)a.t2[b[2] * a.nb[3] + b[3]];
}

// ------------------------------------------------------------------ generators
// Philox4x32-10 from its published definition (Salmon et al., SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}
__device__ __forceinline__ void u2(uint64_t e, uint32_t w2, uint32_t w3, uint64_t seed, double& ua, double& ub) {
  uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), w2, w3};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  ua = (double)(((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
  ub = (double)(((uint64_t)(c[2] >> 5) << 26) | (uint64_t)(c[3] >> 6)) * (1.0 / 9007199254740992.0);
}

#pragma clang fp contract(off)
// Phase-space event e: m_Kpi by accept-reject on p_B(m) q(m) < u * wmax with trial t drawn
// from counter (e, t, 0); angles from counters (e, 0, 1) and (e, 0, 2).  The acceptance
// test is evaluated without contraction so it is bit-identical to a plain FP64 host.
__device__ int phsp_event(const GenArgs& a, uint64_t e, double* ev, double* spare) {
  const double lo = a.mK + a.mPi, hi = a.mB - a.mJ;
  const double c1 = (a.mK + a.mPi) * (a.mK + a.mPi), c2 = (a.mK - a.mPi) * (a.mK - a.mPi);
  double ua, ub;
  for (int t = 0; t < 4096; ++t) {
    u2(e, (uint32_t)t, 0u, a.seed, ua, ub);
    const double m = lo + (hi - lo) * ua;
    // p_B(m) = sqrt((mB^2 - (mJ+m)^2)(mB^2 - (mJ-m)^2)) / (2 mB);  q(m) analogous
    const double s = a.mB * a.mB;
    const double pa = s - (a.mJ + m) * (a.mJ + m);
    const double pb = s - (a.mJ - m) * (a.mJ - m);
    const double px = pa * pb;
    const double pB = px <= 0.0 ? 0.0 : sqrt(px) / (2.0 * a.mB);
    const double mm = m * m;
    const double qa = mm - c1;
    const double qb = mm - c2;
    const double qx = qa * qb;
    const double q = qx <= 0.0 ? 0.0 : sqrt(qx) / (2.0 * m);
    if (ub * a.wmax < pB * q) {
      ev[0] = m;
      u2(e, 0u, 1u, a.seed, ua, ub);
      ev[1] = 2.0 * ua - 1.0;
      ev[2] = 2.0 * ub - 1.0;
      u2(e, 0u, 2u, a.seed, ua, ub);
      ev[3] = 3.14159265358979323846 * (2.0 * ua - 1.0);
      *spare = ub;
      return t + 1;
    }
  }
  return -1;
}

__global__ __launch_bounds__(256) void phsp_kernel(GenArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double ev[4], sp;
  const int t = phsp_event(a, (uint64_t)(a.e0 + i), ev, &sp);
  if (t < 0) { a.flag[i] = 0; a.out[0][i] = NAN; return; }
  a.out[0][i] = ev[0];
  a.out[1][i] = ev[1];
  a.out[2][i] = ev[2];
  a.out[3][i] = ev[3];
  if (a.spare) a.spare[i] = sp;
  a.flag[i] = 1;
}

// Seeded analytic acceptance (same definition as the generator's truth efficiency):
// eps = 0.9 prod_d (1 - delta (1 - t_d)/2), t_d = sum_l a_dl P_l(u_d) / sum_l |a_dl|.
__device__ double acceptance(const double* co, double delta, double lo, double hi, double m, double cK, double cJ,
                             double ph) {
  const double u[4] = {2.0 * (m - lo) / (hi - lo) - 1.0, cK, cJ, ph / 3.14159265358979323846};
  double eps = 0.9;
  for (int d = 0; d < 4; ++d) {
    const double x = u[d];
    const double P1 = x, P2 = 0.5 * (3.0 * x * x - 1.0), P3 = 0.5 * (5.0 * x * x * x - 3.0 * x);
    const double num = co[3 * d] * P1 + co[3 * d + 1] * P2 + co[3 * d + 2] * P3;
    const double den = fabs(co[3 * d]) + fabs(co[3 * d + 1]) + fabs(co[3 * d + 2]);
    const double t = den > 0.0 ? num / den : 0.0;
    eps *= 1.0 - delta * (1.0 - t) / 2.0;
  }
  return eps;
}
#pragma clang fp contract(on)

// Accept flags of proposals: flag = spare * smax < eps * S (S from the density kernel).
__global__ __launch_bounds__(256) void accept_kernel(AcceptArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (!a.valid[i]) { a.flag[i] = 0; return; }
  double s = a.S[i];
  if (a.acc_on) {
    s *= acceptance(a.coef, a.delta, a.lo, a.hi, a.obs[0][i], a.obs[1][i], a.obs[2][i], a.obs[3][i]);
  }
  a.over[i] = (s > a.smax) ? 1 : 0;
  a.flag[i] = (a.spare[i] * a.smax < s) ? 1 : 0;
}

// Stable compaction of accepted proposals: pos = exclusive prefix sum of flags (computed by
// the caller), write accepted events to out[base + pos] while pos < limit.
__global__ __launch_bounds__(256) void compact_kernel(CompactArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n || !a.flag[i]) return;
  const int64_t p = a.base + a.pos[i];
  if (p >= a.limit) return;
#pragma unroll
  for (int d = 0; d < 4; ++d) a.out[d][p] = a.obs[d][i];
}

// ------------------------------------------------------------------ launchers
template <typename T> hipError_t launch_invariants(const InvArgs<T>& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(invariants_kernel<T>, dim3(nb), dim3(256), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_invariants<float>(const InvArgs<float>&, hipStream_t);
template hipError_t launch_invariants<double>(const InvArgs<double>&, hipStream_t);

template <typename T, class Sh, bool ZF>
hipError_t launch_amp_zf(const AmpArgs<T, Sh>& a, int mode, int nblocks, hipStream_t st) {
  const bool cc = a.tag != nullptr && mode != MODE_DENSITY;
  if (mode == MODE_GRAD) {
    if (cc) hipLaunchKernelGGL((amp_kernel<T, Sh, MODE_GRAD, true, ZF>), dim3(nblocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((amp_kernel<T, Sh, MODE_GRAD, false, ZF>), dim3(nblocks), dim3(256), 0, st, a);
  } else if (mode == MODE_NLL) {
    if (cc) hipLaunchKernelGGL((amp_kernel<T, Sh, MODE_NLL, true, ZF>), dim3(nblocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((amp_kernel<T, Sh, MODE_NLL, false, ZF>), dim3(nblocks), dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL((amp_kernel<T, Sh, MODE_DENSITY, false, ZF>), dim3(nblocks), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}
template <typename T, class Sh>
hipError_t launch_amp(const AmpArgs<T, Sh>& a, int mode, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if constexpr (Sh::NZ >= 2) {
    if (a.zfree) {
      if (a.cnt[5] != 1) return hipErrorInvalidValue;   // refused by the host API
      return launch_amp_zf<T, Sh, true>(a, mode, nblocks, st);
    }
  } else {
    if (a.zfree) return hipErrorInvalidValue;
  }
  return launch_amp_zf<T, Sh, false>(a, mode, nblocks, st);
}
// Blocks of the per-event kernel that can be resident on one compute unit at once (from its
// register and LDS use), or 0 if the runtime cannot tell.
template <typename T, class Sh, bool ZF>
int amp_blocks_per_cu_zf(int mode, bool cc) {
  int nb = 0;
  hipError_t e;
  if (mode == MODE_GRAD)
    e = cc ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, amp_kernel<T, Sh, MODE_GRAD, true, ZF>, 256, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, amp_kernel<T, Sh, MODE_GRAD, false, ZF>, 256, 0);
  else if (mode == MODE_NLL)
    e = cc ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, amp_kernel<T, Sh, MODE_NLL, true, ZF>, 256, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, amp_kernel<T, Sh, MODE_NLL, false, ZF>, 256, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, amp_kernel<T, Sh, MODE_DENSITY, false, ZF>, 256, 0);
  return (e == hipSuccess && nb > 0) ? nb : 0;
}
template <typename T, class Sh>
int amp_blocks_per_cu(int mode, bool cc, bool zfree) {
  if constexpr (Sh::NZ >= 2) {
    if (zfree) return amp_blocks_per_cu_zf<T, Sh, true>(mode, cc);
  }
  return amp_blocks_per_cu_zf<T, Sh, false>(mode, cc);
}
template int amp_blocks_per_cu<float, ShapeSmall>(int, bool, bool);
template int amp_blocks_per_cu<double, ShapeSmall>(int, bool, bool);
template int amp_blocks_per_cu<float, ShapeFull>(int, bool, bool);
template int amp_blocks_per_cu<double, ShapeFull>(int, bool, bool);

template hipError_t launch_amp<float, ShapeSmall>(const AmpArgs<float, ShapeSmall>&, int, int, hipStream_t);
template hipError_t launch_amp<double, ShapeSmall>(const AmpArgs<double, ShapeSmall>&, int, int, hipStream_t);
template hipError_t launch_amp<float, ShapeFull>(const AmpArgs<float, ShapeFull>&, int, int, hipStream_t);
template hipError_t launch_amp<double, ShapeFull>(const AmpArgs<double, ShapeFull>&, int, int, hipStream_t);

hipError_t launch_reduce_final(const double* partial, int nb_data, int nb_mc, int n_mc_sets, int nv, double* out,
                               int first_set, int n_sets, hipStream_t st) {
  if (first_set < 0 || n_sets < 1 || n_mc_sets < 1 || n_mc_sets > 2 || first_set + n_sets > 1 + n_mc_sets)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(reduce_final, dim3(n_sets * nv), dim3(256), 0, st, partial, nb_data, nb_mc, n_mc_sets, nv, out,
                     first_set);
  return hipGetLastError();
}
hipError_t launch_hist_lookup(const HistArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(hist_lookup_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_template(const TplArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(template_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_phsp(const GenArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(phsp_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_accept(const AcceptArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(accept_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_compact(const CompactArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace kpsi

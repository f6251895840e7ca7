// FP64 CPU oracle for the four-dimensional B0 -> J/psi K pi amplitude model
// (Sur, Cristella, Di Florio, Mastrapasqua, arXiv:2007.14931).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
// this file: only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark use it.  It shares no code with the HIP path.
//
// It is the plain definition written out: per event, per resonance, per
// helicity, with no hoisting across resonances; Wigner d by Wigner's general
// factorial formula; the Z-chain angles from explicit four-vectors and boosts;
// Kahan-Neumaier sums; forward-mode dual numbers for the exact gradient.
// Build with -O2 -ffp-contract=off and no fast-math.
//
// Paper sections followed:
//   Eq. (2)  resonance lineshape A^R(m) with Blatt-Weisskopf factors
//   Eq. (3)  mass-dependent width Gamma(m)
//   Eq. (4)  K* helicity amplitude;  Eq. (5) K*-only signal density
//   Eq. (6)  H_0 of K*(892) fixed to 1 (done by the caller through the free mask)
//   Eq. (10) Z -> J/psi pi helicity amplitude, angles defined in the text below it
//   Eq. (11) parity relation of the Z helicity couplings (or, per resonance, none: Discussion)
//   Eq. (12) full signal density (K* + Z coherent sum)
//   Eq. (14) efficiency-weighted PDF (signal part), normalised by phase-space MC
//   text after Eq. (12): charge-conjugate decays (phi -> -phi) with a flavour mistag rate
// Readings where the paper is silent are listed at each place they are used.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace orc {

// ------------------------------------------------------------------ dual numbers
constexpr int KD = 96;          // maximum number of tangent directions
static int g_nd = 0;            // active directions (set before each parallel region)

struct Dual {
  double v;
  double d[KD];
  Dual() : v(0) { for (int i = 0; i < g_nd; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < g_nd; ++i) d[i] = 0; }
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r; r.v = -a.v; for (int i = 0; i < g_nd; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r; r.v = a.v * b.v; for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) { Dual r; r.v = a.v / b.v; for (int i = 0; i < g_nd; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
inline Dual operator+(const Dual& a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double a, const Dual& b) { return b + a; }
inline Dual operator-(const Dual& a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double a, const Dual& b) { return -(b - a); }
inline Dual operator*(const Dual& a, double b) { Dual r; r.v = a.v * b; for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { Dual r; r.v = a.v / b; for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] / b; return r; }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double tsqrt(double x) { return std::sqrt(x); }
inline Dual tsqrt(const Dual& x) { Dual r; r.v = std::sqrt(x.v); for (int i = 0; i < g_nd; ++i) r.d[i] = x.d[i] / (2.0 * r.v); return r; }
inline double tlog(double x) { return std::log(x); }
inline Dual tlog(const Dual& x) { Dual r; r.v = std::log(x.v); for (int i = 0; i < g_nd; ++i) r.d[i] = x.d[i] / x.v; return r; }
inline double tcos(double x) { return std::cos(x); }
inline double tsin(double x) { return std::sin(x); }
inline Dual tcos(const Dual& x) { Dual r; r.v = std::cos(x.v); double s = -std::sin(x.v); for (int i = 0; i < g_nd; ++i) r.d[i] = s * x.d[i]; return r; }
inline Dual tsin(const Dual& x) { Dual r; r.v = std::sin(x.v); double c = std::cos(x.v); for (int i = 0; i < g_nd; ++i) r.d[i] = c * x.d[i]; return r; }

template <class T> T ipow(const T& x, int n) { T r(1.0); for (int i = 0; i < n; ++i) r = r * x; return r; }

// ------------------------------------------------------------------ complex
template <class T> struct Cx { T re, im; };
template <class T> Cx<T> cadd(const Cx<T>& a, const Cx<T>& b) { return {a.re + b.re, a.im + b.im}; }
template <class T> Cx<T> cmul(const Cx<T>& a, const Cx<T>& b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
template <class T> Cx<T> cscale(const Cx<T>& a, double s) { return {a.re * s, a.im * s}; }
template <class T> Cx<T> cdiv(const Cx<T>& a, const Cx<T>& b) {
  T n = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / n, (a.im * b.re - a.re * b.im) / n};
}
template <class T> T cnorm2(const Cx<T>& a) { return a.re * a.re + a.im * a.im; }
inline Cx<double> cexpi(double x) { return {std::cos(x), std::sin(x)}; }
template <class T> Cx<T> ctoT(const Cx<double>& a) { return {T(a.re), T(a.im)}; }

// ------------------------------------------------------------------ model
struct Kin { double mB, mJ, mK, mPi, rB, rR; };
// chain: 0 = K* (K pi), 1 = Z (J/psi pi); lb/lr < 0 => lowest allowed.
// shape: 0 relativistic Breit-Wigner (Eq. 2-3); 1 LASS S-wave (Eq. 7-8) with effective-range
// parameters a, b (GeV^-1) for a spin-0 K*.
// hel_free (Z only): H'_{+1} and H'_{-1} are independent couplings instead of being tied by the
// parity relation of Eq. (11) (the Discussion states that the Z part can also be fitted with its
// couplings unconstrained).  Parameter order of such a Z: lambda' = 0, +1, -1.
struct Res { int chain, spin, parity, lb, lr; double mass, width; int shape; double lass_a, lass_b; int hel_free; };

// Lowest orbital momenta (text below Eq. 3 for the K*; angular momentum and
// parity for the Z, which decays strongly to J/psi(1-) pi(0-)).
static int res_LR(const Res& r) {
  if (r.lr >= 0) return r.lr;
  if (r.chain == 0) return r.spin;            // K* -> K pi: L = J
  return 0;                                   // Z(1+) -> J/psi pi: lowest even L
}
static int res_LB(const Res& r) {
  if (r.lb >= 0) return r.lb;
  if (r.chain == 0) return r.spin == 0 ? 1 : r.spin - 1;   // B -> J/psi K*: lowest |J-1|.., J=0 needs L=1
  return r.spin == 0 ? 0 : r.spin;                         // B -> Z K (K spinless): L = J
}
// Number of independent complex helicity couplings of a resonance.
static int res_ncoup(const Res& r) {
  if (r.chain == 0) return r.spin == 0 ? 1 : 3;   // lambda in {-1,0,1}, only 0 for spin 0 (Eq. 4)
  return r.hel_free ? 3 : 2;                     // Z: lambda' = 0, +1 (H_-1 from Eq. 11), or 0, +1, -1
}

// Two-body breakup momentum of M -> m1 m2 in the M rest frame.
template <class T> T breakup(const T& M, double m1, double m2) {
  T s = M * M;
  T a = s - (m1 + m2) * (m1 + m2);
  T b = s - (m1 - m2) * (m1 - m2);
  T x = a * b;
  if (val(x) <= 0.0) return T(0.0);
  return tsqrt(x) / (2.0 * M);
}

// Blatt-Weisskopf barrier polynomials (von Hippel and Quigg) in z = (r p)^2; the
// normalised barrier factor of Eq. (2) is F_L = sqrt(B_L(z0) / B_L(z)), so F(p0) = 1.
template <class T> T bw_poly(int L, const T& z) {
  switch (L) {
    case 0: return T(1.0);
    case 1: return 1.0 + z;
    case 2: return 9.0 + 3.0 * z + z * z;
    case 3: return 225.0 + 45.0 * z + 6.0 * z * z + z * z * z;
    case 4: return 11025.0 + 1575.0 * z + 135.0 * z * z + 10.0 * z * z * z + z * z * z * z;
    default: return T(NAN);
  }
}
template <class T> T barrier(int L, double p, const T& p0, double r) {
  T z = T(r * p * r * p);
  T z0 = (r * p0) * (r * p0);
  return tsqrt(bw_poly(L, z0) / bw_poly(L, z));
}

// Eq. (2)-(3): A^R(m) = F_B (p_B/M_B)^LB F_R (p/m)^LR / (M^2 - m^2 - i M Gamma(m)),
// Gamma(m) = Gamma0 (p/p0)^(2LR+1) (M/m) F_R^2.  The (p/m) factor uses the running
// mass m (the paper defines m_R as the running mass).
template <class T> Cx<T> lineshape(const Kin& k, const Res& r, const T& M, const T& G0, double m) {
  int LR = res_LR(r), LB = res_LB(r);
  double p, pB;
  T p0, pB0;
  if (r.chain == 0) {          // K* -> K pi, B -> J/psi K*
    p = breakup(m, k.mK, k.mPi);
    pB = breakup(k.mB, k.mJ, m);
    p0 = breakup(M, k.mK, k.mPi);
    // p_B at the pole: B -> J/psi R with the R mass set to M (M may carry tangents)
    T s = T(k.mB * k.mB);
    T a = s - (k.mJ + M) * (k.mJ + M);
    T b = s - (k.mJ - M) * (k.mJ - M);
    pB0 = tsqrt(a * b) / (2.0 * k.mB);
  } else {                     // Z -> J/psi pi, B -> Z K
    p = breakup(m, k.mJ, k.mPi);
    pB = breakup(k.mB, m, k.mK);
    p0 = breakup(M, k.mJ, k.mPi);
    T s = T(k.mB * k.mB);
    T a = s - (M + k.mK) * (M + k.mK);
    T b = s - (M - k.mK) * (M - k.mK);
    pB0 = tsqrt(a * b) / (2.0 * k.mB);
  }
  T FR = barrier(LR, p, p0, k.rR);
  T FB = barrier(LB, pB, pB0, k.rB);
  if (r.shape == 1) {
    // LASS (Eq. 7-8), written as the unitarised sum of an effective-range phase and the scalar
    // resonance (reading: the printed factor 2 of the resonant term is dropped, the B-decay
    // factor F_B (p_B/M_B)^L_B of Eq. 2 is kept):
    //   A = F_B (p_B/M_B)^L_B [ (m/q) sin dB e^{i dB} + e^{2 i dB} (M^2 G0 / q0) / (M^2 - m^2 - i M G(m)) ]
    //   cot dB = 1/(a q) + b q / 2,  G(m) = G0 (q/q0) (M/m)
    // at threshold (q = 0): dB = 0 and (m/q) sin dB e^{i dB} -> m a
    const double cot = p > 0.0 ? 1.0 / (r.lass_a * p) + 0.5 * r.lass_b * p : INFINITY;
    const double dB = std::atan2(1.0, cot);
    const Cx<T> nr = p > 0.0 ? Cx<T>{T((m / p) * std::sin(dB) * std::cos(dB)), T((m / p) * std::sin(dB) * std::sin(dB))}
                             : Cx<T>{T(m * r.lass_a), T(0.0)};
    const Cx<T> e2{T(std::cos(2.0 * dB)), T(std::sin(2.0 * dB))};
    const T Gam = G0 * (T(p) / p0) * (M / m);
    const Cx<T> res = cdiv(Cx<T>{M * M * G0 / p0, T(0.0)}, Cx<T>{M * M - m * m, -(M * Gam)});
    const T pre = FB * std::pow(pB / k.mB, LB);
    const Cx<T> t{nr.re + e2.re * res.re - e2.im * res.im, nr.im + e2.re * res.im + e2.im * res.re};
    return Cx<T>{pre * t.re, pre * t.im};
  }
  T ratio = T(p) / p0;
  T Gam = G0 * ipow(ratio, 2 * LR + 1) * (M / m) * FR * FR;
  T num = FB * std::pow(pB / k.mB, LB) * FR * std::pow(p / m, LR);
  Cx<T> den{M * M - m * m, -(M * Gam)};
  return cdiv(Cx<T>{num, T(0.0)}, den);
}

// Wigner small-d by Wigner's general formula (integer j only).
static double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
double wigner_d(int j, int mp, int m, double theta) {
  if (std::abs(mp) > j || std::abs(m) > j) return 0.0;
  double c = std::cos(0.5 * theta), s = std::sin(0.5 * theta);
  double pre = std::sqrt(fact(j + mp) * fact(j - mp) * fact(j + m) * fact(j - m));
  double sum = 0.0;
  for (int kk = 0; kk <= 2 * j; ++kk) {
    int a = j + m - kk, b = j - kk - mp, d = kk - m + mp;
    if (a < 0 || b < 0 || d < 0) continue;
    double sign = ((kk - m + mp) % 2 == 0) ? 1.0 : -1.0;
    double term = sign / (fact(a) * fact(kk) * fact(b) * fact(d));
    int pc = 2 * j - 2 * kk + m - mp, ps = 2 * kk - m + mp;
    term *= std::pow(c, pc) * std::pow(s, ps);
    sum += term;
  }
  return pre * sum;
}

// ------------------------------------------------------------------ kinematics
struct V4 { double e, x, y, z; };
static V4 boost(const V4& p, double bx, double by, double bz) {
  // Lorentz boost of p by velocity b (frame moving with -b sees ... ): returns p seen
  // in a frame that moves with velocity b relative to the current frame.
  double b2 = bx * bx + by * by + bz * bz;
  if (b2 <= 0) return p;
  double g = 1.0 / std::sqrt(1.0 - b2);
  double bp = bx * p.x + by * p.y + bz * p.z;
  double g2 = (g - 1.0) / b2;
  V4 r;
  r.e = g * (p.e - bp);
  r.x = p.x + g2 * bp * bx - g * bx * p.e;
  r.y = p.y + g2 * bp * by - g * by * p.e;
  r.z = p.z + g2 * bp * bz - g * bz * p.e;
  return r;
}
static V4 to_rest(const V4& p, const V4& frame) {
  return boost(p, frame.x / frame.e, frame.y / frame.e, frame.z / frame.e);
}
static double dot3(const V4& a, const V4& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static double norm3(const V4& a) { return std::sqrt(dot3(a, a)); }
static V4 unit3(const V4& a) { double n = norm3(a); return {0, a.x / n, a.y / n, a.z / n}; }
static V4 cross3(const V4& a, const V4& b) { return {0, a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
static V4 sub3(const V4& a, const V4& b) { return {0, a.x - b.x, a.y - b.y, a.z - b.z}; }
static V4 scale3(const V4& a, double s) { return {0, a.x * s, a.y * s, a.z * s}; }
static V4 add4(const V4& a, const V4& b) { return {a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z}; }

// Four-vectors of K, pi and the J/psi in the B rest frame, and the mu+ direction in
// the J/psi rest frame (reached by a direct boost from the B frame).  Construction:
// the K pi system flies along +z; K is emitted in the K pi frame at polar angle
// theta_K* from +z with azimuth 0, so the hadron plane is the x-z plane with K at
// x > 0.  The J/psi flies along -z.  In its rest frame mu+ has polar angle
// theta_J/psi from the J/psi flight direction n1 = -z and azimuth phi measured from
// the K side of the hadron plane (x1 = +x), right-handed about n1 (y1 = n1 x x1).
struct Frame { V4 K, Pi, Jpsi; V4 mu_dir_psi; };
static Frame build_frame(const Kin& k, double m, double cK, double cJ, double phi) {
  double q = breakup(m, k.mK, k.mPi);
  double pB = breakup(k.mB, k.mJ, m);
  double sK = std::sqrt(std::max(0.0, 1.0 - cK * cK));
  double sJ = std::sqrt(std::max(0.0, 1.0 - cJ * cJ));
  V4 Kr{std::sqrt(k.mK * k.mK + q * q), q * sK, 0.0, q * cK};
  V4 Pir{std::sqrt(k.mPi * k.mPi + q * q), -q * sK, 0.0, -q * cK};
  double EKpi = std::sqrt(m * m + pB * pB);
  // boost from the K pi rest frame to the B frame: the K pi system moves with +pB/EKpi along z
  Frame f;
  f.K = boost(Kr, 0, 0, -pB / EKpi);
  f.Pi = boost(Pir, 0, 0, -pB / EKpi);
  f.Jpsi = V4{std::sqrt(k.mJ * k.mJ + pB * pB), 0.0, 0.0, -pB};
  f.mu_dir_psi = V4{0, sJ * std::cos(phi), -sJ * std::sin(phi), -cJ};
  return f;
}

// Z-chain observables (text under Eq. 10), computed in the J/psi rest frame:
//   m_Jpsi pi; theta_Z, the Z helicity angle, the angle between K and pi in the
//   J/psi pi rest frame; theta~, the J/psi helicity angle in the Z chain: the angle of
//   mu+ from the J/psi direction in the Z frame, which in the J/psi frame is the
//   direction opposite to the pi (equivalently the angle between mu- and pi);
//   phi~, the azimuth of mu+ about that axis measured from the K side of the (K, pi)
//   plane; alpha, the rotation about the mu+ direction that carries the (mu+, pi)
//   plane onto the (mu+, K pi) plane (the two chains' muon helicity frames).
struct ZAng { double mJpi, thZ, thJ, phiZ, alpha; };
ZAng z_angles(const Kin& k, double m, double cK, double cJ, double phi) {
  Frame f = build_frame(k, m, cK, cJ, phi);
  ZAng z;
  V4 Zp = add4(f.Jpsi, f.Pi);
  z.mJpi = std::sqrt(Zp.e * Zp.e - dot3(Zp, Zp));
  // theta_Z in the J/psi pi rest frame
  V4 KZ = to_rest(f.K, Zp), PiZ = to_rest(f.Pi, Zp);
  double cz = dot3(KZ, PiZ) / (norm3(KZ) * norm3(PiZ));
  z.thZ = std::acos(std::max(-1.0, std::min(1.0, cz)));
  // J/psi rest frame (direct boost from the B frame along z).  K* chain frame:
  // n1 = -z (the J/psi flight direction, unchanged by a boost along z), x1 = +x (K side).
  V4 Kp = to_rest(f.K, f.Jpsi), Pip = to_rest(f.Pi, f.Jpsi);
  V4 mu = f.mu_dir_psi;
  V4 n1{0, 0, 0, -1}, x1{0, 1, 0, 0};
  V4 y1 = cross3(n1, x1);
  // Z chain frame: n2 = -pi direction (J/psi flight direction in the J/psi pi frame),
  // x2 = K side of the (K, pi) plane, perpendicular to n2.  For collinear hadrons the
  // plane is undefined; every lambda' = +-1 term then carries sin(theta_Z) = 0, and x2 is
  // taken from x1.
  V4 n2 = scale3(unit3(Pip), -1.0);
  V4 kperp = sub3(Kp, scale3(n2, dot3(Kp, n2)));
  V4 x2;
  if (dot3(kperp, kperp) > 1e-24 * dot3(Kp, Kp)) x2 = unit3(kperp);
  else x2 = unit3(sub3(x1, scale3(n2, dot3(x1, n2))));
  V4 y2 = cross3(n2, x2);
  double ct = dot3(mu, n2);
  z.thJ = std::acos(std::max(-1.0, std::min(1.0, ct)));
  z.phiZ = std::atan2(dot3(mu, y2), dot3(mu, x2));
  // Muon helicity frames of the two chains: the x axis of R(phi, theta, 0) applied to
  // each chain's frame, x' = cos(theta) (cos(phi) x + sin(phi) y) - sin(theta) n.  In the
  // K* chain (theta, phi) are the event's theta_J/psi and phi themselves (Eq. 4), which
  // stay meaningful when sin(theta_J/psi) = 0.
  double th1 = std::acos(std::max(-1.0, std::min(1.0, cJ)));
  double ph1 = phi;
  V4 xa = sub3(scale3(add4(scale3(x1, std::cos(ph1)), scale3(y1, std::sin(ph1))), std::cos(th1)),
               scale3(n1, std::sin(th1)));
  V4 xb = sub3(scale3(add4(scale3(x2, std::cos(z.phiZ)), scale3(y2, std::sin(z.phiZ))), std::cos(z.thJ)),
               scale3(n2, std::sin(z.thJ)));
  V4 cr = cross3(xb, xa);
  z.alpha = std::atan2(dot3(cr, mu), dot3(xb, xa));
  return z;
}

// ------------------------------------------------------------------ parameters
// Canonical full parameter vector: for each resonance in table order its coupling
// (magnitude, phase) pairs -- K*: lambda = -1, 0, +1 (spin 0: lambda = 0 only); Z:
// lambda' = 0, +1 -- then (M, Gamma0) for every resonance in table order.
static int n_coupling_reals(const std::vector<Res>& rs) { int n = 0; for (auto& r : rs) n += 2 * res_ncoup(r); return n; }
int n_full_params(const std::vector<Res>& rs) { return n_coupling_reals(rs) + 2 * (int)rs.size(); }

struct Event { double m, cK, cJ, phi; };

// Signal density S of Eq. (12) (Eq. (5) when no Z is present) for one event.
template <class T>
T density(const Kin& k, const std::vector<Res>& rs, const T* par, const Event& ev, const ZAng& za) {
  Cx<T> a[2] = {{T(0.0), T(0.0)}, {T(0.0), T(0.0)}};   // xi = +1, -1
  const int xis[2] = {+1, -1};
  const int nc = n_coupling_reals(rs);
  double thK = std::acos(ev.cK), thJ = std::acos(ev.cJ);
  int ip = 0;
  for (size_t ir = 0; ir < rs.size(); ++ir) {
    const Res& r = rs[ir];
    const T& M = par[nc + 2 * ir];
    const T& G = par[nc + 2 * ir + 1];
    if (r.chain == 0) {
      // Eq. (4): H_lambda A(m_Kpi) d^J_{lambda 0}(theta_K*) e^{i lambda phi} d^1_{lambda xi}(theta_J/psi)
      Cx<T> A = lineshape(k, r, M, G, ev.m);
      int nl = res_ncoup(r);
      for (int il = 0; il < nl; ++il) {
        int lam = (nl == 1) ? 0 : il - 1;
        const T& mag = par[ip + 2 * il];
        const T& ph = par[ip + 2 * il + 1];
        Cx<T> H{mag * tcos(ph), mag * tsin(ph)};
        double dk = wigner_d(r.spin, lam, 0, thK);
        Cx<T> HA = cmul(H, A);
        for (int x = 0; x < 2; ++x) {
          double dj = wigner_d(1, lam, xis[x], thJ);
          Cx<double> e = cexpi(lam * ev.phi);
          Cx<T> term = cmul(HA, ctoT<T>(cscale(e, dk * dj)));
          a[x] = cadd(a[x], term);
        }
      }
      ip += 2 * nl;
    } else {
      // Eq. (10): H'_l A^Z(m_Jpsi pi) d^J_{0 l}(theta_Z) e^{i l phi~} d^1_{l xi}(theta~) e^{i xi alpha}
      Cx<T> A = lineshape(k, r, M, G, za.mJpi);
      // Eq. (11): H'_{-l} = -P (-1)^J H'_{l}, unless the resonance leaves H'_{-1} free
      double eta = -(double)r.parity * ((r.spin % 2 == 0) ? 1.0 : -1.0);
      Cx<T> H0{par[ip] * tcos(par[ip + 1]), par[ip] * tsin(par[ip + 1])};
      Cx<T> H1{par[ip + 2] * tcos(par[ip + 3]), par[ip + 2] * tsin(par[ip + 3])};
      Cx<T> Hm1 = r.hel_free ? Cx<T>{par[ip + 4] * tcos(par[ip + 5]), par[ip + 4] * tsin(par[ip + 5])}
                             : Cx<T>{H1.re * eta, H1.im * eta};
      for (int lam = -1; lam <= 1; ++lam) {
        Cx<T> H = (lam == 0) ? H0 : (lam == 1 ? H1 : Hm1);
        double dz = wigner_d(r.spin, 0, lam, za.thZ);
        Cx<T> HA = cmul(H, A);
        for (int x = 0; x < 2; ++x) {
          double dj = wigner_d(1, lam, xis[x], za.thJ);
          Cx<double> e = cexpi(lam * za.phiZ + xis[x] * za.alpha);
          a[x] = cadd(a[x], cmul(HA, ctoT<T>(cscale(e, dz * dj))));
        }
      }
      ip += 2 * res_ncoup(r);
    }
  }
  return cnorm2(a[0]) + cnorm2(a[1]);
}

// Kahan-Neumaier accumulator
struct KSum {
  double s = 0, c = 0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  double get() const { return s + c; }
};

}  // namespace orc

using namespace orc;

// ================================================================== C API
extern "C" {

struct oracle_kin { double mB, mJ, mK, mPi, rB, rR; };
struct oracle_res { int chain, spin, parity, lb, lr; double mass, width; int shape; double lass_a, lass_b; int hel_free; };

static std::vector<Res> to_res(const oracle_res* r, int n) {
  std::vector<Res> v;
  for (int i = 0; i < n; ++i)
    v.push_back(Res{r[i].chain, r[i].spin, r[i].parity, r[i].lb, r[i].lr, r[i].mass, r[i].width, r[i].shape,
                    r[i].lass_a, r[i].lass_b, r[i].chain == 1 ? r[i].hel_free : 0});
  return v;
}
static Kin to_kin(const oracle_kin* k) { return Kin{k->mB, k->mJ, k->mK, k->mPi, k->rB, k->rR}; }

int oracle_n_params(const oracle_res* res, int n_res) { return n_full_params(to_res(res, n_res)); }
// Sizes of the structures the binding passes (a mismatched binding is refused at load).
int oracle_struct_size(int which) { return which == 0 ? (int)sizeof(oracle_kin) : (int)sizeof(oracle_res); }

double oracle_wigner_d(int j, int mp, int m, double theta) { return wigner_d(j, mp, m, theta); }
double oracle_breakup(double M, double m1, double m2) { return breakup(M, m1, m2); }

// Lineshape of resonance ir at running mass m (Eq. 2-3); M and Gamma0 given explicitly.
void oracle_lineshape(const oracle_kin* kin, const oracle_res* res, double M, double G0, double m, double* out_re_im) {
  Kin k = to_kin(kin);
  Res r{res->chain, res->spin, res->parity, res->lb, res->lr, res->mass, res->width, res->shape, res->lass_a,
        res->lass_b, 0};
  Cx<double> a = lineshape<double>(k, r, M, G0, m);
  out_re_im[0] = a.re; out_re_im[1] = a.im;
}

// Per-event Z-chain observables: out[5*i + {0..4}] = (m_Jpsi pi, theta_Z, theta~, phi~, alpha).
void oracle_z_angles(const oracle_kin* kin, int64_t n, const double* m, const double* cK, const double* cJ,
                     const double* phi, double* out) {
  Kin k = to_kin(kin);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    ZAng z = z_angles(k, m[i], cK[i], cJ[i], phi[i]);
    out[5 * i + 0] = z.mJpi; out[5 * i + 1] = z.thZ; out[5 * i + 2] = z.thJ;
    out[5 * i + 3] = z.phiZ; out[5 * i + 4] = z.alpha;
  }
}

// Four-vectors used for the Z-chain observables (for kinematic identity tests):
// out[16*i ..] = K(e,x,y,z), pi(e,x,y,z), J/psi(e,x,y,z), mu+ direction in J/psi frame (0,x,y,z).
void oracle_four_vectors(const oracle_kin* kin, int64_t n, const double* m, const double* cK, const double* cJ,
                         const double* phi, double* out) {
  Kin k = to_kin(kin);
  for (int64_t i = 0; i < n; ++i) {
    Frame f = build_frame(k, m[i], cK[i], cJ[i], phi[i]);
    const V4* vs[4] = {&f.K, &f.Pi, &f.Jpsi, &f.mu_dir_psi};
    for (int j = 0; j < 4; ++j) {
      out[16 * i + 4 * j + 0] = vs[j]->e; out[16 * i + 4 * j + 1] = vs[j]->x;
      out[16 * i + 4 * j + 2] = vs[j]->y; out[16 * i + 4 * j + 3] = vs[j]->z;
    }
  }
}

// Per-event signal density S (Eq. 12).
void oracle_density(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, int64_t n,
                    const double* m, const double* cK, const double* cJ, const double* phi, double* out) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Event ev{m[i], cK[i], cJ[i], phi[i]};
    ZAng za{0, 0, 0, 0, 0};
    if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
    out[i] = density<double>(k, rs, par, ev, za);
  }
}

// Fit fractions (Eq. 13): FF_j = sum_e w_e S_j(x_e) / sum_e w_e S(x_e), where S_j is the
// density with every helicity coupling outside resonance j set to zero (masses and widths as
// given) and the sums run over phase-space events (flat measure; w = NULL means unit weights,
// otherwise w carries integration weights).  The integral in Eq. 13 is read as the phase-space
// integral of S.  Returns 0, or -5 when sum w S is not positive.
int oracle_fit_fractions(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, int64_t n,
                         const double* m, const double* cK, const double* cJ, const double* phi, const double* w,
                         double* ff) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  const int np = n_full_params(rs);
  // weighted phase-space sum of the density at parameter vector q
  auto integral = [&](const std::vector<double>& q) {
    int nt = omp_get_max_threads();
    std::vector<KSum> part(nt);
#pragma omp parallel
    {
      int t = omp_get_thread_num();
#pragma omp for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        Event ev{m[i], cK[i], cJ[i], phi[i]};
        ZAng za{0, 0, 0, 0, 0};
        if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
        const double s = density<double>(k, rs, q.data(), ev, za);
        part[t].add(w ? w[i] * s : s);
      }
    }
    KSum tot;
    for (int t = 0; t < nt; ++t) { tot.add(part[t].s); tot.add(part[t].c); }
    return tot.get();
  };
  std::vector<double> full(par, par + np);
  const double den = integral(full);
  if (!(den > 0.0)) return -5;
  for (int j = 0; j < n_res; ++j) {
    std::vector<double> q(full);
    int o2 = 0;
    for (int i = 0; i < n_res; ++i) {
      const int nl = res_ncoup(rs[i]);
      if (i != j)
        for (int l = 0; l < nl; ++l) q[o2 + 2 * l] = 0.0;   // magnitude of coupling l of resonance i
      o2 += 2 * nl;
    }
    ff[j] = integral(q) / den;
  }
  return 0;
}

// -2 ln L of the mixture PDF of Eq. 14,  f = p eps S / N_S + (1 - p) b / N_b,  where
// N_S = (1/N_MC) sum_j eps_j S(y_j) and N_b = (1/N_MC) sum_j b_j over the phase-space
// normalisation events, so that both terms are normalised over phase space (the constant
// phase-space volume is dropped).  NLL = -2 sum_i ln f(x_i).  eps_d / eps_m may be NULL
// (efficiency 1); b_d, b_m are the background density at the data and normalisation events;
// 0 < purity <= 1.  Gradient (forward-mode duals) along dirs[] when n_dir > 0.  Returns 0, -1
// for bad arguments, or -5 when some f(x_i) <= 0 or a normalisation is not positive.
int oracle_nll_mix(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, int64_t nd,
                   const double* dm, const double* dck, const double* dcj, const double* dphi, int64_t nm,
                   const double* mm, const double* mck, const double* mcj, const double* mphi, const double* eps_d,
                   const double* b_d, const double* eps_m, const double* b_m, double purity, int n_dir,
                   const int* dirs, double* nll, double* grad) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  const int np = n_full_params(rs);
  if (nd <= 0 || nm <= 0 || !b_d || !b_m || !(purity > 0.0 && purity <= 1.0)) return -1;
  if (n_dir < 0 || n_dir > KD) return -1;
  for (int d = 0; d < n_dir; ++d) if (dirs[d] < 0 || dirs[d] >= np) return -1;
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  g_nd = n_dir;
  std::vector<Dual> P(np);
  for (int i = 0; i < np; ++i) P[i] = Dual(par[i]);
  for (int d = 0; d < n_dir; ++d) P[dirs[d]].d[d] = 1.0;
  auto dens = [&](double m, double cK, double cJ, double ph) {
    Event ev{m, cK, cJ, ph};
    ZAng za{0, 0, 0, 0, 0};
    if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
    return density<Dual>(k, rs, P.data(), ev, za);
  };
  // normalisations over the phase-space events
  KSum sS, sB;
  std::vector<double> gS(n_dir, 0.0);
  for (int64_t j = 0; j < nm; ++j) {
    const Dual s = dens(mm[j], mck[j], mcj[j], mphi[j]);
    const double e = eps_m ? eps_m[j] : 1.0;
    sS.add(e * s.v);
    for (int d = 0; d < n_dir; ++d) gS[d] += e * s.d[d];
    sB.add(b_m[j]);
  }
  const double NS = sS.get() / (double)nm, NB = sB.get() / (double)nm;
  if (!(NS > 0.0) || !(NB > 0.0)) { *nll = INFINITY; return -5; }
  std::vector<double> dNS(n_dir);
  for (int d = 0; d < n_dir; ++d) dNS[d] = gS[d] / (double)nm;
  // data: f_i = p eps_i S_i / N_S + (1 - p) b_i / N_b
  KSum L;
  std::vector<double> gL(n_dir, 0.0);
  for (int64_t i = 0; i < nd; ++i) {
    const Dual s = dens(dm[i], dck[i], dcj[i], dphi[i]);
    const double e = eps_d ? eps_d[i] : 1.0;
    const double f = purity * e * s.v / NS + (1.0 - purity) * b_d[i] / NB;
    if (!(f > 0.0) || !std::isfinite(f)) { *nll = INFINITY; return -5; }
    L.add(std::log(f));
    for (int d = 0; d < n_dir; ++d) {
      const double df = purity * e * (s.d[d] / NS - s.v * dNS[d] / (NS * NS));
      gL[d] += df / f;
    }
  }
  *nll = -2.0 * L.get();
  for (int d = 0; d < n_dir; ++d) grad[d] = -2.0 * gL[d];
  return 0;
}

// Charge-conjugate decays with a per-event flavour tag (text after Eq. 12): the density of the
// conjugate decay is S with the sign of phi reversed.  Reading (the paper states only that the
// sign flips and that mis-tagging is allowed for): an event tagged q = +1 (B0) or -1 (B0bar) is
// of the other flavour with probability w, both flavours equally produced, so
//   f(x, q) = [(1 - w) S(x^(q)) + w S(x^(-q))] / N_q,   x^(s) = (m, cos K, cos J, s phi),
//   N_q = (1 - w) I(q) + w I(-q),   I(s) = (1/N_MC) sum_j eps_j S(y_j^(s)),
// and NLL = -2 sum_i ln f(x_i, q_i) (the data efficiencies dropped as for the signal NLL).
// The Z-chain angles of x^(s) are recomputed from the flipped event.  tag[i] is +1 or -1.
// Returns 0, -1 on bad arguments, or -5 when a data term or a normalisation is not positive.
int oracle_nll_cc(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, int64_t nd,
                  const double* dm, const double* dck, const double* dcj, const double* dphi, const double* tag,
                  int64_t nm, const double* mm, const double* mck, const double* mcj, const double* mphi,
                  const double* eps_m, double mistag, int n_dir, const int* dirs, double* nll, double* grad) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  const int np = n_full_params(rs);
  if (nd <= 0 || nm <= 0 || !tag || !(mistag >= 0.0 && mistag <= 0.5)) return -1;
  if (n_dir < 0 || n_dir > KD) return -1;
  for (int d = 0; d < n_dir; ++d) if (dirs[d] < 0 || dirs[d] >= np) return -1;
  for (int64_t i = 0; i < nd; ++i) if (tag[i] != 1.0 && tag[i] != -1.0) return -1;
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  g_nd = n_dir;
  std::vector<Dual> P(np);
  for (int i = 0; i < np; ++i) P[i] = Dual(par[i]);
  for (int d = 0; d < n_dir; ++d) P[dirs[d]].d[d] = 1.0;
  auto dens = [&](double m, double cK, double cJ, double ph) {
    Event ev{m, cK, cJ, ph};
    ZAng za{0, 0, 0, 0, 0};
    if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
    return density<Dual>(k, rs, P.data(), ev, za);
  };
  // I(+1), I(-1) over the phase-space events
  KSum sI[2];
  std::vector<double> gI[2] = {std::vector<double>(n_dir, 0.0), std::vector<double>(n_dir, 0.0)};
  for (int64_t j = 0; j < nm; ++j) {
    const double e = eps_m ? eps_m[j] : 1.0;
    for (int f = 0; f < 2; ++f) {
      const Dual s = dens(mm[j], mck[j], mcj[j], f == 0 ? mphi[j] : -mphi[j]);
      sI[f].add(e * s.v);
      for (int d = 0; d < n_dir; ++d) gI[f][d] += e * s.d[d];
    }
  }
  double I[2], dI[2][KD];
  for (int f = 0; f < 2; ++f) {
    I[f] = sI[f].get() / (double)nm;
    for (int d = 0; d < n_dir; ++d) dI[f][d] = gI[f][d] / (double)nm;
  }
  // N_q for q = +1 (index 0) and q = -1 (index 1)
  double N[2], dN[2][KD];
  for (int f = 0; f < 2; ++f) {
    N[f] = (1.0 - mistag) * I[f] + mistag * I[1 - f];
    for (int d = 0; d < n_dir; ++d) dN[f][d] = (1.0 - mistag) * dI[f][d] + mistag * dI[1 - f][d];
    if (!(N[f] > 0.0)) { *nll = INFINITY; return -5; }
  }
  KSum L;
  std::vector<double> gL(n_dir, 0.0);
  for (int64_t i = 0; i < nd; ++i) {
    const int f = tag[i] > 0.0 ? 0 : 1;
    const double ph = dphi[i];
    const Dual s_same = dens(dm[i], dck[i], dcj[i], f == 0 ? ph : -ph);
    const Dual s_other = dens(dm[i], dck[i], dcj[i], f == 0 ? -ph : ph);
    const double t = (1.0 - mistag) * s_same.v + mistag * s_other.v;
    if (!(t > 0.0) || !std::isfinite(t)) { *nll = INFINITY; return -5; }
    L.add(std::log(t) - std::log(N[f]));
    for (int d = 0; d < n_dir; ++d) {
      const double dt = (1.0 - mistag) * s_same.d[d] + mistag * s_other.d[d];
      gL[d] += dt / t - dN[f][d] / N[f];
    }
  }
  *nll = -2.0 * L.get();
  for (int d = 0; d < n_dir; ++d) grad[d] = -2.0 * gL[d];
  return 0;
}

// Flavour-tagged events with the signal + background mixture of Eq. 14.  Reading: the
// background density b is the same for both flavours, and each flavour's PDF is normalised, so
//   f(x, q) = p eps(x) [(1 - w) S(x^(q)) + w S(x^(-q))] / N_q + (1 - p) b(x) / N_b,
// with N_q = (1 - w) I(q) + w I(-q), I(s) = (1/N_MC) sum_j eps_j S(y_j^(s)), N_b = (1/N_MC) sum_j b_j
// (the mixture above for the signal part, the tagged form above for the flavours), and
// NLL = -2 sum_i ln f(x_i, q_i).  eps_d / eps_m may be NULL (efficiency 1).  Returns 0, -1 on bad
// arguments, or -5 when some f(x_i) <= 0 or a normalisation is not positive.
int oracle_nll_cc_mix(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, int64_t nd,
                      const double* dm, const double* dck, const double* dcj, const double* dphi, const double* tag,
                      int64_t nm, const double* mm, const double* mck, const double* mcj, const double* mphi,
                      const double* eps_d, const double* b_d, const double* eps_m, const double* b_m, double purity,
                      double mistag, int n_dir, const int* dirs, double* nll, double* grad) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  const int np = n_full_params(rs);
  if (nd <= 0 || nm <= 0 || !tag || !b_d || !b_m) return -1;
  if (!(purity > 0.0 && purity <= 1.0) || !(mistag >= 0.0 && mistag <= 0.5)) return -1;
  if (n_dir < 0 || n_dir > KD) return -1;
  for (int d = 0; d < n_dir; ++d) if (dirs[d] < 0 || dirs[d] >= np) return -1;
  for (int64_t i = 0; i < nd; ++i) if (tag[i] != 1.0 && tag[i] != -1.0) return -1;
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  g_nd = n_dir;
  std::vector<Dual> P(np);
  for (int i = 0; i < np; ++i) P[i] = Dual(par[i]);
  for (int d = 0; d < n_dir; ++d) P[dirs[d]].d[d] = 1.0;
  auto dens = [&](double m, double cK, double cJ, double ph) {
    Event ev{m, cK, cJ, ph};
    ZAng za{0, 0, 0, 0, 0};
    if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
    return density<Dual>(k, rs, P.data(), ev, za);
  };
  // I(+1), I(-1) and N_b over the phase-space events
  KSum sI[2], sB;
  std::vector<double> gI[2] = {std::vector<double>(n_dir, 0.0), std::vector<double>(n_dir, 0.0)};
  for (int64_t j = 0; j < nm; ++j) {
    const double e = eps_m ? eps_m[j] : 1.0;
    for (int f = 0; f < 2; ++f) {
      const Dual s = dens(mm[j], mck[j], mcj[j], f == 0 ? mphi[j] : -mphi[j]);
      sI[f].add(e * s.v);
      for (int d = 0; d < n_dir; ++d) gI[f][d] += e * s.d[d];
    }
    sB.add(b_m[j]);
  }
  const double NB = sB.get() / (double)nm;
  if (!(NB > 0.0)) { *nll = INFINITY; return -5; }
  double N[2], dN[2][KD];
  for (int f = 0; f < 2; ++f) {
    const double Iq = sI[f].get() / (double)nm, Io = sI[1 - f].get() / (double)nm;
    N[f] = (1.0 - mistag) * Iq + mistag * Io;
    for (int d = 0; d < n_dir; ++d) dN[f][d] = ((1.0 - mistag) * gI[f][d] + mistag * gI[1 - f][d]) / (double)nm;
    if (!(N[f] > 0.0)) { *nll = INFINITY; return -5; }
  }
  KSum L;
  std::vector<double> gL(n_dir, 0.0);
  for (int64_t i = 0; i < nd; ++i) {
    const int f = tag[i] > 0.0 ? 0 : 1;
    const double ph = dphi[i];
    const Dual s_same = dens(dm[i], dck[i], dcj[i], f == 0 ? ph : -ph);
    const Dual s_other = dens(dm[i], dck[i], dcj[i], f == 0 ? -ph : ph);
    const double e = eps_d ? eps_d[i] : 1.0;
    const double sig = (1.0 - mistag) * s_same.v + mistag * s_other.v;
    const double fi = purity * e * sig / N[f] + (1.0 - purity) * b_d[i] / NB;
    if (!(fi > 0.0) || !std::isfinite(fi)) { *nll = INFINITY; return -5; }
    L.add(std::log(fi));
    for (int d = 0; d < n_dir; ++d) {
      const double dsig = (1.0 - mistag) * s_same.d[d] + mistag * s_other.d[d];
      gL[d] += purity * e * (dsig / N[f] - sig * dN[f][d] / (N[f] * N[f])) / fi;
    }
  }
  *nll = -2.0 * L.get();
  for (int d = 0; d < n_dir; ++d) grad[d] = -2.0 * gL[d];
  return 0;
}

// -2 ln L of the signal PDF eps*S normalised by the phase-space MC sum (Eq. 14 with
// purity 1):  NLL = -2 sum_i ln S(x_i) + 2 N_d ln( (1/N_MC) sum_j eps_j S(y_j) ).
// Parameter-independent terms (ln eps(x_i), phase-space factor, volume) are dropped.
// eps may be NULL (flat efficiency).  Returns 0, or -5 when a data S <= 0 or the
// normalisation is not positive (nll is then +inf).
// When n_dir > 0 the gradient with respect to the parameters listed in dirs[] is
// returned in grad[] (forward-mode dual numbers, exact to rounding).
static int nll_impl_double(const Kin& k, const std::vector<Res>& rs, const double* par, int64_t nd,
                           const double* const* D, int64_t nm, const double* const* Mc, const double* eps,
                           double* nll) {
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  int nt = omp_get_max_threads();
  std::vector<KSum> sd(nt), sm(nt);
  std::vector<int> bad(nt, 0);
#pragma omp parallel
  {
    int t = omp_get_thread_num();
#pragma omp for schedule(static)
    for (int64_t i = 0; i < nd; ++i) {
      Event ev{D[0][i], D[1][i], D[2][i], D[3][i]};
      ZAng za{0, 0, 0, 0, 0};
      if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
      double s = density<double>(k, rs, par, ev, za);
      if (!(s > 0.0) || !std::isfinite(s)) { bad[t]++; continue; }
      sd[t].add(std::log(s));
    }
#pragma omp for schedule(static)
    for (int64_t j = 0; j < nm; ++j) {
      Event ev{Mc[0][j], Mc[1][j], Mc[2][j], Mc[3][j]};
      ZAng za{0, 0, 0, 0, 0};
      if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
      double s = density<double>(k, rs, par, ev, za);
      sm[t].add(eps ? eps[j] * s : s);
    }
  }
  KSum SD, SM;
  int nbad = 0;
  for (int t = 0; t < nt; ++t) { SD.add(sd[t].s); SD.add(sd[t].c); SM.add(sm[t].s); SM.add(sm[t].c); nbad += bad[t]; }
  double norm = SM.get() / (double)nm;
  if (nbad > 0 || !(norm > 0.0)) { *nll = INFINITY; return -5; }
  *nll = -2.0 * SD.get() + 2.0 * (double)nd * std::log(norm);
  return 0;
}

static int nll_impl_dual(const Kin& k, const std::vector<Res>& rs, const double* par, int np, const int* dirs,
                         int n_dir, int64_t nd, const double* const* D, int64_t nm, const double* const* Mc,
                         const double* eps, double* nll, double* grad) {
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  g_nd = n_dir;
  std::vector<Dual> P(np);
  for (int i = 0; i < np; ++i) { P[i] = Dual(par[i]); }
  for (int d = 0; d < n_dir; ++d) P[dirs[d]].d[d] = 1.0;
  int nt = omp_get_max_threads();
  std::vector<KSum> sd(nt), sm(nt);
  std::vector<std::vector<double>> gd(nt, std::vector<double>(n_dir, 0.0)), gm(nt, std::vector<double>(n_dir, 0.0));
  std::vector<int> bad(nt, 0);
#pragma omp parallel
  {
    int t = omp_get_thread_num();
#pragma omp for schedule(static)
    for (int64_t i = 0; i < nd; ++i) {
      Event ev{D[0][i], D[1][i], D[2][i], D[3][i]};
      ZAng za{0, 0, 0, 0, 0};
      if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
      Dual s = density<Dual>(k, rs, P.data(), ev, za);
      if (!(s.v > 0.0) || !std::isfinite(s.v)) { bad[t]++; continue; }
      sd[t].add(std::log(s.v));
      for (int d = 0; d < n_dir; ++d) gd[t][d] += s.d[d] / s.v;
    }
#pragma omp for schedule(static)
    for (int64_t j = 0; j < nm; ++j) {
      Event ev{Mc[0][j], Mc[1][j], Mc[2][j], Mc[3][j]};
      ZAng za{0, 0, 0, 0, 0};
      if (hasZ) za = z_angles(k, ev.m, ev.cK, ev.cJ, ev.phi);
      Dual s = density<Dual>(k, rs, P.data(), ev, za);
      double e = eps ? eps[j] : 1.0;
      sm[t].add(e * s.v);
      for (int d = 0; d < n_dir; ++d) gm[t][d] += e * s.d[d];
    }
  }
  KSum SD, SM;
  int nbad = 0;
  std::vector<double> GD(n_dir, 0.0), GM(n_dir, 0.0);
  for (int t = 0; t < nt; ++t) {
    SD.add(sd[t].s); SD.add(sd[t].c); SM.add(sm[t].s); SM.add(sm[t].c); nbad += bad[t];
    for (int d = 0; d < n_dir; ++d) { GD[d] += gd[t][d]; GM[d] += gm[t][d]; }
  }
  double sumM = SM.get();
  double norm = sumM / (double)nm;
  if (nbad > 0 || !(norm > 0.0)) { *nll = INFINITY; return -5; }
  *nll = -2.0 * SD.get() + 2.0 * (double)nd * std::log(norm);
  for (int d = 0; d < n_dir; ++d) grad[d] = -2.0 * GD[d] + 2.0 * (double)nd * GM[d] / sumM;
  return 0;
}

int oracle_nll(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, int64_t nd,
               const double* dm, const double* dck, const double* dcj, const double* dphi, int64_t nm,
               const double* mm, const double* mck, const double* mcj, const double* mphi, const double* eps,
               int n_dir, const int* dirs, double* nll, double* grad) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  int np = n_full_params(rs);
  if (nd <= 0 || nm <= 0) return -1;
  if (n_dir < 0 || n_dir > KD) return -1;
  for (int d = 0; d < n_dir; ++d) if (dirs[d] < 0 || dirs[d] >= np) return -1;
  const double* D[4] = {dm, dck, dcj, dphi};
  const double* Mc[4] = {mm, mck, mcj, mphi};
  if (n_dir == 0) return nll_impl_double(k, rs, par, nd, D, nm, Mc, eps, nll);
  return nll_impl_dual(k, rs, par, np, dirs, n_dir, nd, D, nm, Mc, eps, nll, grad);
}

// Gradient of S itself at one event, with respect to the listed directions (for tests).
double oracle_density_grad(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, double m,
                           double cK, double cJ, double phi, int n_dir, const int* dirs, double* grad) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  int np = n_full_params(rs);
  g_nd = n_dir;
  std::vector<Dual> P(np);
  for (int i = 0; i < np; ++i) P[i] = Dual(par[i]);
  for (int d = 0; d < n_dir; ++d) P[dirs[d]].d[d] = 1.0;
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  Event ev{m, cK, cJ, phi};
  ZAng za{0, 0, 0, 0, 0};
  if (hasZ) za = z_angles(k, m, cK, cJ, phi);
  Dual s = density<Dual>(k, rs, P.data(), ev, za);
  for (int d = 0; d < n_dir; ++d) grad[d] = s.d[d];
  return s.v;
}

// ------------------------------------------------------------------ generators
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its published
// definition: ten rounds of two 32x32->64 multiplies with key bumps by the Weyl
// constants between rounds.
void oracle_philox(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}
static double u53(uint32_t a, uint32_t b) {
  uint64_t x = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
  return (double)x * (1.0 / 9007199254740992.0);
}
static void philox_u2(uint64_t e, uint32_t w2, uint32_t w3, uint64_t seed, double* u) {
  uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), w2, w3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  oracle_philox(ctr, key, o);
  u[0] = u53(o[0], o[1]);
  u[1] = u53(o[2], o[3]);
}

// Flat four-body phase-space event number e: m_Kpi distributed as p_B(m) q(m) on
// [mK + mpi, mB - mJ] by accept-reject with envelope wmax (trial t uses counter
// (e, t, 0)); cos theta_K*, cos theta_J/psi uniform in [-1, 1) from counter (e, 0, 1);
// phi uniform in [-pi, pi) and one spare uniform from counter (e, 0, 2).
// Returns the number of trials, or -1 if 4096 trials were not enough.
static int phsp_event(const Kin& k, uint64_t seed, uint64_t e, double wmax, double* ev, double* spare) {
  double lo = k.mK + k.mPi, hi = k.mB - k.mJ;
  double u[2];
  for (int t = 0; t < 4096; ++t) {
    philox_u2(e, (uint32_t)t, 0u, seed, u);
    double m = lo + (hi - lo) * u[0];
    double w = breakup(k.mB, k.mJ, m) * breakup(m, k.mK, k.mPi);
    if (u[1] * wmax < w) {
      ev[0] = m;
      philox_u2(e, 0u, 1u, seed, u);
      ev[1] = 2.0 * u[0] - 1.0;
      ev[2] = 2.0 * u[1] - 1.0;
      philox_u2(e, 0u, 2u, seed, u);
      ev[3] = M_PI * (2.0 * u[0] - 1.0);
      *spare = u[1];
      return t + 1;
    }
  }
  return -1;
}

int oracle_gen_phsp(const oracle_kin* kin, uint64_t seed, int64_t n, double wmax, double* m, double* cK,
                    double* cJ, double* phi) {
  Kin k = to_kin(kin);
  int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
  for (int64_t i = 0; i < n; ++i) {
    double ev[4], sp;
    if (phsp_event(k, seed, (uint64_t)i, wmax, ev, &sp) < 0) { err |= 1; continue; }
    m[i] = ev[0]; cK[i] = ev[1]; cJ[i] = ev[2]; phi[i] = ev[3];
  }
  return err ? -1 : 0;
}

// Accept-reject of phase-space proposals e = 0, 1, 2, ... against S (times an optional
// efficiency given as a callback-free analytic acceptance, see oracle_acceptance):
// proposal e is kept when spare_u(e) * smax < eff(x) S(x).  Accepted events are written
// in proposal order until n are kept.  *n_prop receives the number of proposals used;
// *n_over the number of proposals with eff*S > smax (the envelope was too low).
double oracle_acceptance(const double* coef, double m_lo, double m_hi, double m, double cK, double cJ, double phi);
int oracle_gen_model(const oracle_kin* kin, const oracle_res* res, int n_res, const double* par, uint64_t seed,
                     int64_t n, double wmax, double smax, const double* acc_coef, int64_t max_prop, double* m,
                     double* cK, double* cJ, double* phi, int64_t* n_prop, int64_t* n_over) {
  Kin k = to_kin(kin);
  std::vector<Res> rs = to_res(res, n_res);
  bool hasZ = false;
  for (auto& r : rs) hasZ |= (r.chain == 1);
  double lo = k.mK + k.mPi, hi = k.mB - k.mJ;
  int64_t kept = 0, e0 = 0, over = 0;
  const int64_t B = 65536;
  std::vector<double> ev(4 * B), sp(B);
  std::vector<char> acc(B);
  int err = 0;
  while (kept < n) {
    if (e0 >= max_prop) { err = -2; break; }
    int64_t nb = std::min<int64_t>(B, max_prop - e0);
#pragma omp parallel for schedule(static) reduction(+ : over) reduction(| : err)
    for (int64_t i = 0; i < nb; ++i) {
      double* x = &ev[4 * i];
      if (phsp_event(k, seed, (uint64_t)(e0 + i), wmax, x, &sp[i]) < 0) { err |= 1; acc[i] = 0; continue; }
      Event e{x[0], x[1], x[2], x[3]};
      ZAng za{0, 0, 0, 0, 0};
      if (hasZ) za = z_angles(k, e.m, e.cK, e.cJ, e.phi);
      double s = density<double>(k, rs, par, e, za);
      if (acc_coef) s *= oracle_acceptance(acc_coef, lo, hi, e.m, e.cK, e.cJ, e.phi);
      if (s > smax) over++;
      acc[i] = (sp[i] * smax < s) ? 1 : 0;
    }
    for (int64_t i = 0; i < nb && kept < n; ++i) {
      if (!acc[i]) continue;
      m[kept] = ev[4 * i]; cK[kept] = ev[4 * i + 1]; cJ[kept] = ev[4 * i + 2]; phi[kept] = ev[4 * i + 3];
      kept++;
      if (kept == n) { e0 += i + 1; nb = 0; break; }
    }
    e0 += nb;
  }
  *n_prop = e0;
  *n_over = over;
  return err ? (err < 0 ? err : -1) : 0;
}

// Seeded smooth four-dimensional acceptance: eps = 0.9 prod_d f_d with
// f_d = 1 - delta (1 - t_d) / 2, t_d = sum_{l=1..3} a_{d,l} P_l(u_d) / sum_l |a_{d,l}|,
// delta = 1 - 3^(-1/4), and u = (mapped m_Kpi, cos theta_K*, cos theta_J/psi, phi/pi),
// so eps lies in [0.3, 0.9].  coef holds a[4][3].
double oracle_acceptance(const double* coef, double m_lo, double m_hi, double m, double cK, double cJ, double phi) {
  double u[4] = {2.0 * (m - m_lo) / (m_hi - m_lo) - 1.0, cK, cJ, phi / M_PI};
  double delta = 1.0 - std::pow(3.0, -0.25);
  double eps = 0.9;
  for (int d = 0; d < 4; ++d) {
    double x = u[d];
    double P[3] = {x, 0.5 * (3 * x * x - 1), 0.5 * (5 * x * x * x - 3 * x)};
    double num = 0, den = 0;
    for (int l = 0; l < 3; ++l) { num += coef[3 * d + l] * P[l]; den += std::fabs(coef[3 * d + l]); }
    double t = den > 0 ? num / den : 0.0;
    eps *= 1.0 - delta * (1.0 - t) / 2.0;
  }
  return eps;
}

// Gaussian constraints on fit parameters (Conclusion: applied to fit parameters when required):
// a factor prod_k N(p[idx_k]; mean_k, sigma_k) in the likelihood adds
//   sum_k ((p[idx_k] - mean_k) / sigma_k)^2
// to -2 ln L (up to a constant).  grad (length n_par, may be NULL) receives its gradient
// 2 (p - mean) / sigma^2 at the constrained positions and 0 elsewhere.  Returns -1 on a bad
// index or a non-positive sigma.
int oracle_gauss_penalty(int n, const int* idx, const double* mean, const double* sigma, int n_par, const double* par,
                         double* value, double* grad) {
  double v = 0.0;
  if (grad) for (int i = 0; i < n_par; ++i) grad[i] = 0.0;
  for (int k = 0; k < n; ++k) {
    if (idx[k] < 0 || idx[k] >= n_par || !(sigma[k] > 0.0)) return -1;
    const double z = (par[idx[k]] - mean[k]) / sigma[k];
    v += z * z;
    if (grad) grad[idx[k]] += 2.0 * z / sigma[k];
  }
  *value = v;
  return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

}  // extern "C"

extern "C" {
// Normalised Blatt-Weisskopf factor F_L(p; p0, r) = sqrt(B_L((r p0)^2) / B_L((r p)^2)) and
// the bare polynomial B_L(z), exported for the barrier-factor pins.
double oracle_barrier(int L, double p, double p0, double r) { return barrier<double>(L, p, p0, r); }
double oracle_bw_poly(int L, double z) { return bw_poly<double>(L, z); }
}

// ================================================================== learned efficiency
// Reference of the efficiency network: inputs u = (2 (m - lo)/(hi - lo) - 1, cos theta_K*,
// cos theta_J/psi, phi/pi); z1 = W1 u + b1, h1 = silu(z1); z2 = W2 h1 + b2, h2 = silu(z2);
// p = sigmoid(w3 . h2 + b3); loss = mean binary cross-entropy against accept labels.
// The network is defined with BF16 weights and BF16 operands of the 64x64 layer (its
// matrix-core form): W1, W2, w3, h1 and the 64x64 layer's back-propagated z2 gradient
// (per event, before the 1/n of the mean) are rounded to BF16 (round to nearest even) where the device rounds them; everything
// else is FP64 (round_bf16 = 0 gives the plain FP64 network, whose gradient is exact).  The
// gradient treats the roundings as identity, as the device does.  Parameter layout (4545 floats): W1[64][4], b1[64], W2[64][64], b2[64],
// w3[64], b3.
namespace {
double bf16_round(double x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;   // inf / nan unchanged
  const uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7fffu + lsb) & 0xffff0000u;
  std::memcpy(&f, &u, 4);
  return (double)f;
}
double silu(double z) { return z / (1.0 + std::exp(-z)); }
double dsilu(double z) { double s = 1.0 / (1.0 + std::exp(-z)); return s * (1.0 + z * (1.0 - s)); }
}  // namespace

extern "C" {

double oracle_bf16(double x) { return bf16_round(x); }

// Forward (probabilities) and, when grad != NULL, the gradient of the mean BCE over the n
// events with respect to the 4545 parameters.  Returns the mean loss.
double oracle_mlp(const double* par, int64_t n, const double* u, const double* y, double* prob, double* grad,
                  int round_bf16) {
  auto bf16_round = [round_bf16](double x) { return round_bf16 ? ::bf16_round(x) : x; };
  const double* W1 = par;
  const double* b1 = par + 256;
  const double* W2 = par + 320;
  const double* b2 = par + 4416;
  const double* w3 = par + 4480;
  const double b3 = par[4544];
  std::vector<double> W1r(256), W2r(4096), w3r(64);
  for (int i = 0; i < 256; ++i) W1r[i] = bf16_round(W1[i]);
  for (int i = 0; i < 4096; ++i) W2r[i] = bf16_round(W2[i]);
  for (int i = 0; i < 64; ++i) w3r[i] = bf16_round(w3[i]);
  if (grad) std::fill(grad, grad + 4545, 0.0);
  double loss = 0.0;
  for (int64_t e = 0; e < n; ++e) {
    double x[4], z1[64], h1[64], z2[64], h2[64];
    for (int k = 0; k < 4; ++k) x[k] = u[4 * e + k];
    for (int j = 0; j < 64; ++j) {
      double s = b1[j];
      for (int k = 0; k < 4; ++k) s += W1r[4 * j + k] * x[k];
      z1[j] = s;
      h1[j] = bf16_round(silu(s));
    }
    for (int o = 0; o < 64; ++o) {
      double s = b2[o];
      for (int i = 0; i < 64; ++i) s += W2r[64 * o + i] * h1[i];
      z2[o] = s;
      h2[o] = silu(s);
    }
    double z3 = b3;
    for (int o = 0; o < 64; ++o) z3 += w3r[o] * h2[o];
    const double p = 1.0 / (1.0 + std::exp(-z3));
    if (prob) prob[e] = p;
    if (y) {
      const double pc = std::min(std::max(p, 1e-12), 1.0 - 1e-12);
      loss += -(y[e] * std::log(pc) + (1.0 - y[e]) * std::log(1.0 - pc));
    }
    if (!grad) continue;
    const double dz3 = (p - y[e]) / (double)n;
    grad[4544] += dz3;
    double dz2[64];
    for (int o = 0; o < 64; ++o) {
      grad[4480 + o] += dz3 * h2[o];
      dz2[o] = dz3 * w3r[o] * dsilu(z2[o]);
      grad[4416 + o] += dz2[o];
    }
    double dz2r[64];
    for (int o = 0; o < 64; ++o) dz2r[o] = bf16_round(dz2[o] * (double)n) / (double)n;
    for (int o = 0; o < 64; ++o)
      for (int i = 0; i < 64; ++i) grad[320 + 64 * o + i] += dz2r[o] * h1[i];
    for (int i = 0; i < 64; ++i) {
      double dh1 = 0.0;
      for (int o = 0; o < 64; ++o) dh1 += dz2r[o] * W2r[64 * o + i];
      const double dz1 = dh1 * dsilu(z1[i]);
      grad[256 + i] += dz1;
      for (int k = 0; k < 4; ++k) grad[4 * i + k] += dz1 * x[k];
    }
  }
  return y ? loss / (double)n : 0.0;
}

// Network input of an event.
void oracle_mlp_inputs(double m_lo, double m_hi, int64_t n, const double* m, const double* cK, const double* cJ,
                       const double* phi, double* u) {
  for (int64_t e = 0; e < n; ++e) {
    u[4 * e + 0] = 2.0 * (m[e] - m_lo) / (m_hi - m_lo) - 1.0;
    u[4 * e + 1] = cK[e];
    u[4 * e + 2] = cJ[e];
    u[4 * e + 3] = phi[e] / M_PI;
  }
}

}  // extern "C"

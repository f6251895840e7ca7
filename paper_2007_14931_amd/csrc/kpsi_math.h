// Device arithmetic shared by the per-event kernel and the interference-matrix kernel: the
// hardware reciprocal and reciprocal square root (refined by Newton steps in FP64), the
// normalised Blatt-Weisskopf polynomials, and the small-d functions d^J_{00}, d^J_{10} of the
// K* helicity angle (Eq. 4).  One copy, so both kernels evaluate the same lineshape and
// angular polynomials.
#pragma once

#include <hip/hip_runtime.h>

namespace kpsi {

// 1/x and 1/sqrt(x): the FP32 forms are the hardware instructions (about 1 ulp); the FP64
// forms refine the hardware estimate with two Newton steps to full double precision.
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  double e = __builtin_fma(-h * r, r, 0.5);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-h * r, r, 0.5);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float sqrt_(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// M^2 - s, the real part of a Breit-Wigner denominator (Eq. 2).  In FP32 the squared mass is
// carried as M2 plus its rounding remainder M2lo: near a narrow pole M^2 - s is far smaller than
// M^2, and the rounding of M^2 alone would move the pole of every event by the same amount (a
// shift of 0.5 ulp of M^2 is 1e-3 of the statistical error of a K*(892) mass at 3e6 events).
template <typename T, typename R> __device__ __forceinline__ T pole_gap(const R& rc, T s) {
  if constexpr (sizeof(T) == sizeof(float)) return (rc.M2 - s) + rc.M2lo;
  else return rc.M2 - s;
}

// Blatt-Weisskopf polynomial B_L(z), z = (r p)^2, in Horner form: the barrier factor of
// Eq. 2-3 is F_L = sqrt(B_L(z0) / B_L(z)).
template <int L, typename T> __device__ __forceinline__ T bpoly(T z) {
  if constexpr (L == 0) return T(1);
  else if constexpr (L == 1) return T(1) + z;
  else if constexpr (L == 2) return T(9) + z * (T(3) + z);
  else if constexpr (L == 3) return T(225) + z * (T(45) + z * (T(6) + z));
  else return T(11025) + z * (T(1575) + z * (T(135) + z * (T(10) + z)));
}
// Lowest orbital momentum of B -> J/psi K* for a K* of spin J (text below Eq. 3).
template <int J> struct LBof { static constexpr int v = (J == 0) ? 1 : J - 1; };

template <typename T, int n> __device__ __forceinline__ T ipow(T x) {
  T r = T(1);
#pragma unroll
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

// d^J_{00}(theta_K) and d^J_{10}(theta_K) (d^J_{-1,0} = -d^J_{10}) as polynomials in cos and sin.
template <int J, typename T> __device__ __forceinline__ T d00(T c) {
  if constexpr (J == 0) return T(1);
  else if constexpr (J == 1) return c;
  else if constexpr (J == 2) return T(1.5) * c * c - T(0.5);
  else if constexpr (J == 3) return c * (T(2.5) * c * c - T(1.5));
  else { T c2 = c * c; return (T(35) * c2 * c2 - T(30) * c2 + T(3)) * T(0.125); }
}
template <int J, typename T> __device__ __forceinline__ T d10(T c, T s) {
  // -sin * P_J'(cos) / sqrt(J (J+1))
  if constexpr (J == 1) return -s * T(0.70710678118654752440);
  else if constexpr (J == 2) return -s * c * T(1.22474487139158904910);
  else if constexpr (J == 3) return -s * (T(15) * c * c - T(3)) * T(0.14433756729740644113);
  else if constexpr (J == 4) return -s * c * (T(35) * c * c - T(15)) * T(0.11180339887498948482);
  else return T(0);
}

// First K* slot of spin J in a compiled kernel shape (slots are ordered by spin).
template <class Sh> __host__ __device__ constexpr int slot_base(int J) {
  int b = 0;
  for (int j = 0; j < J; ++j) b += Sh::N[j];
  return b;
}

}  // namespace kpsi

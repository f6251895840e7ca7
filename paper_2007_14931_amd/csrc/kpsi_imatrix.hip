// Interference matrix of the normalisation integral (gfx950 matrix cores).
//
// With a_xi = sum_k c_k B_k,xi (complex couplings c_k, per-event component amplitudes
// B_k,xi = A_R(m) x angular factor of Eq. 4 or Eq. 10), the MC normalisation sum is
//   sum_j eps_j S(y_j) = sum_kl c_k conj(c_l) I_kl,   I_kl = sum_j eps_j sum_xi B_k,xi conj(B_l,xi),
// and its derivative with respect to a lineshape parameter p of resonance R needs
//   D^p_kl = sum_j eps_j sum_xi dB_k,xi/dp conj(B_l,xi)   (k in R).
// Both are blocks of the real Gram matrix G = X^T X of the matrix X whose rows are
// (event, xi), each scaled by sqrt(eps) of its event, and whose columns are the real and
// imaginary parts of the components followed by the derivative components.  G is accumulated
// over 16x16 tiles of its upper triangle on the matrix cores: v_mfma_f32_16x16x4f32 for FP32
// rows (FP32 sums over one 64-row tile, then FP64 sums), v_mfma_f64_16x16x4f64 for FP64 rows.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kpsi_internal.h"
#include "kpsi_math.h"

namespace kpsi {

namespace im {

template <class Sh> __host__ __device__ constexpr int comp_base(int J) {   // first component of spin J
  int b = 0;
  for (int j = 0; j < J; ++j) b += Sh::N[j] * (j == 0 ? 1 : 3);
  return b;
}

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

}  // namespace im

// One wavefront per block.  Each tile holds 32 events (64 rows: xi = +1, -1).
// ZF: one Z whose H'_{+1} and H'_{-1} are independent couplings: three Z components
// (lambda' = 0, +1, -1), the third in the component position of the second Z.
template <typename T, class Sh, int C, bool ZF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void imatrix_kernel(const ImArgs<T, Sh> a) {
  using namespace im;
  constexpr int NT = C / 16;
  constexpr int NTILE = NT * (NT + 1) / 2;
  static_assert(!ZF || Sh::NZ >= 2, "free Z helicities use the second Z's component position");
  constexpr int NZ = ZF ? 1 : Sh::NZ;   // Z slots evaluated
  // Rows are staged at the context precision in dynamic LDS sized for the columns in use (the
  // padded width C is only the MFMA tiling): FP32 rows of the 76-column benchmark model take
  // 19.5 KB, so eight one-wavefront blocks fit per compute unit (two per SIMD), and one wave's
  // row building overlaps the other's matrix work.  The row stride LDX = ncols + 1 is odd:
  // the 32 lanes writing rows l (and l + 32) hit 32 different banks.  Column ncols of every
  // row is never written and stays zero; the matrix phase reads it in place of the padded
  // columns ncols .. C - 1.  Each row is scaled by sqrt(eps) of its event, so the Gram product
  // of the rows with themselves carries the weight eps once.
  extern __shared__ double im_smem[];
  T* X = reinterpret_cast<T*>(im_smem);
  const int LDX = a.ncols + 1;
  const int lane = threadIdx.x;
  d4_t acc[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int64_t ntiles = (a.n + 31) / 32;
  // Every tile writes the same row positions (the columns of the model's components and
  // derivatives), so the rows are cleared once: the padding and unused columns stay zero.
  for (int i = lane; i < 64 * LDX; i += 64) X[i] = T(0);

  // The event columns of this lane's event in the next tile are fetched before the matrix phase
  // of the current one, so their latency hides behind it.  Column groups of four (K* chain:
  // 0-11; Z angular factors: 12-15, present when the model has Z states; with free Z
  // helicities 16-17 as well).
  using V4 = T __attribute__((ext_vector_type(4)));
  const V4* __restrict__ gcol = reinterpret_cast<const V4*>(a.cols);
  const int64_t ld = a.ld;
  const bool zon = NZ > 0 && a.cnt[5] > 0;
  V4 g0{}, g1{}, g2{}, g3{}, g4{};
  T wv = T(0);
  auto fetch = [&](int64_t tile) {
    const int64_t e = tile * 32 + (lane & 31);
    if (tile < ntiles && e < a.n) {
      g0 = gcol[e];
      g1 = gcol[ld + e];
      g2 = gcol[2 * ld + e];
      if (zon) g3 = gcol[3 * ld + e];
      if (ZF && zon) g4 = gcol[4 * ld + e];
      wv = a.eps ? a.eps[e] : T(1);
    }
  };
  fetch(blockIdx.x);

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // ---- rows of this tile: lane l fills row l, event l % 32 at xi = +1 (l < 32) or -1.  The
    //      two lanes of an event both evaluate its amplitudes (the same instructions), and each
    //      writes one row with its own angular factors.
    const int64_t e = tile * 32 + (lane & 31);
    const bool xm = lane >= 32;   // xi = -1
    T* rr = X + lane * LDX;
    if (e < a.n) {
      const T m = g0.x, q = g0.y, pB = g0.z, cK = g0.w;
      const T sK = g1.x, cJ = g1.y, sJ = g1.z, cph = g1.w;
      const T sph = g2.x, qm = g2.z;   // column 10: q/m
      const T sw = sqrt_(wv);
      const T m2 = m * m;
      const T zR = (a.rR * q) * (a.rR * q), zB = (a.rB * pB) * (a.rB * pB);
      const T pbm = pB * a.invMB, qq = q * q;
      const T hp = T(0.5) * (T(1) + cJ), hm = T(0.5) * (T(1) - cJ), s0 = sJ * T(0.70710678118654752440);
      // write a component (or derivative) column: value A times this row's angular factor g
      auto put = [&](int c, T Ar, T Ai, T gr, T gi) {
        rr[2 * c] = Ar * gr - Ai * gi;
        rr[2 * c + 1] = Ar * gi + Ai * gr;
      };
      // e^{i lambda phi} d^1_{lambda xi}(theta_J) of this row for lambda = +1, 0, -1
      // (xi = +1: (1+c)/2, s/sqrt2, (1-c)/2;  xi = -1: (1-c)/2, -s/sqrt2, (1+c)/2)
      const T h1 = xm ? hm : hp, h2 = xm ? hp : hm, sx = xm ? -s0 : s0;
      const T ep_r = cph * h1, ep_i = sph * h1;     // lambda = +1
      const T fp_r = cph * h2, fp_i = -sph * h2;    // lambda = -1
      auto do_spin = [&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        if constexpr (Sh::N[J] > 0) {
          constexpr int LB = LBof<J>::v;
          const T BR = bpoly<J>(zR), BB = bpoly<LB>(zB);
          // n_J with the row weight sqrt(eps) folded in
          const T nJ = ipow<T, LB>(pbm) * ipow<T, J>(qm) * rsq_(BR * BB) * sw;
          const T gJ = qm * ipow<T, J>(qq) * rcp_(BR);
          const T a0 = d00<J>(cK), a1 = d10<J>(cK, sK);
#pragma unroll
          for (int j = 0; j < Sh::N[J]; ++j) {
            if (j >= a.cnt[J]) continue;
            const auto& rc = a.ks[slot_base<Sh>(J) + j];
            const T dre = pole_gap(rc, m2), dim = -rc.P * gJ;
            const T inv = rcp_(dre * dre + dim * dim);
            const T sc = rc.K * nJ * inv;
            const T br = sc * dre, bi = -sc * dim;
            T Ar = br, Ai = bi;
            if constexpr (J == 0) {
              if (rc.lass) {
                // LASS (Eq. 7-8): u = q cot(delta_B) = 1/a + b q^2/2; the non-resonant term is
                // m (u + i q)/(u^2 + q^2), the resonant one P e^{2 i delta_B} times the Breit-Wigner
                const T u = rc.lhb * qq + rc.lai;
                const T dn = rcp_(u * u + qq);
                const T er = (u * u - qq) * dn, ei = T(2) * u * q * dn;
                const T md = m * dn * (rc.K * nJ);
                Ar = md * u + rc.P * (er * br - ei * bi);
                Ai = md * q + rc.P * (er * bi + ei * br);
              }
            }
            const int c0 = comp_base<Sh>(J) + (J == 0 ? j : 3 * j);
            // derivative factors: dA/dM = A (kappa - Y), dA/dGamma0 = A i (P/Gamma0) g conj(den)/|den|^2
            T dMr = 0, dMi = 0, dGr = 0, dGi = 0;
            if (rc.flt >= 0) {
              const T pr = rc.twoM, pim = -rc.dP * gJ;
              const T Yr = (pr * dre + pim * dim) * inv, Yi = (pim * dre - pr * dim) * inv;
              const T kr = rc.kap - Yr, ki = -Yi;
              dMr = Ar * kr - Ai * ki;
              dMi = Ar * ki + Ai * kr;
              const T zf = rc.PoG * gJ * inv;
              const T zr = zf * dim, zi = zf * dre;
              dGr = Ar * zr - Ai * zi;
              dGi = Ar * zi + Ai * zr;
            }
            if constexpr (J == 0) {
              put(c0, Ar, Ai, sx, T(0));
              if (rc.flt >= 0) {
                const int dc = a.dcol[rc.flt];
                put(dc, dMr, dMi, sx, T(0));
                put(dc + 1, dGr, dGi, sx, T(0));
              }
            } else {
              // lambda = -1: -d10 e^{-i phi} h2; 0: d00 (+-s0); +1: d10 e^{+i phi} h1
              const T g1r = -a1 * fp_r, g1i = -a1 * fp_i;
              const T h0 = a0 * sx;
              const T k1r = a1 * ep_r, k1i = a1 * ep_i;
              put(c0, Ar, Ai, g1r, g1i);
              put(c0 + 1, Ar, Ai, h0, T(0));
              put(c0 + 2, Ar, Ai, k1r, k1i);
              if (rc.flt >= 0) {
                const int dc = a.dcol[rc.flt];
                put(dc, dMr, dMi, g1r, g1i);
                put(dc + 1, dMr, dMi, h0, T(0));
                put(dc + 2, dMr, dMi, k1r, k1i);
                put(dc + 3, dGr, dGi, g1r, g1i);
                put(dc + 4, dGr, dGi, h0, T(0));
                put(dc + 5, dGr, dGi, k1r, k1i);
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
      if constexpr (NZ > 0) {
        if (zon) {
          // (the angular columns za carry the Z barrier factor n_Z)
          const T mz2 = g2.y, gz = g2.w;
          // this row's Zang[l'][xi]: xi = +1 columns 12-13 (l' = 0) and 14-15 (l' = 1); xi = -1 is
          // (-Re, Im) of xi = +1
          const T z0r = xm ? -g3.x : g3.x, z0i = g3.y;
          T z1r = xm ? -g3.z : g3.z, z1i = g3.w;
          T z2r = T(0), z2i = T(0);
          if constexpr (ZF) {
            // lambda' = +1: F++ (xi = +1, columns 14-15) or F+- (xi = -1, columns 16-17);
            // lambda' = -1: -conj(F+-) (xi = +1) or -conj(F++) (xi = -1)
            z1r = xm ? g4.x : g3.z;
            z1i = xm ? g4.y : g3.w;
            z2r = xm ? -g3.z : -g4.x;
            z2i = xm ? g3.w : g4.y;
          }
          constexpr int zc0 = comp_base<Sh>(5);
          constexpr int ZN = ZF ? 3 : 2;   // components per Z slot
#pragma unroll
          for (int z = 0; z < NZ; ++z) {
            if (z >= a.cnt[5]) continue;
            const auto& rc = a.zs[z];
            const T dre = pole_gap(rc, mz2), dim = -rc.P * gz;
            const T inv = rcp_(dre * dre + dim * dim);
            const T sc = rc.K * inv * sw;
            const T Ar = sc * dre, Ai = -sc * dim;
            put(zc0 + 2 * z, Ar, Ai, z0r, z0i);
            put(zc0 + 2 * z + 1, Ar, Ai, z1r, z1i);
            if constexpr (ZF) put(zc0 + 2, Ar, Ai, z2r, z2i);
            if (rc.flt >= 0) {
              const T pr = rc.twoM, pim = -rc.dP * gz;
              const T Yr = (pr * dre + pim * dim) * inv, Yi = (pim * dre - pr * dim) * inv;
              const T kr = rc.kap - Yr, ki = -Yi;
              const T dMr = Ar * kr - Ai * ki, dMi = Ar * ki + Ai * kr;
              const T zf = rc.PoG * gz * inv;
              const T zr = zf * dim, zi = zf * dre;
              const T dGr = Ar * zr - Ai * zi, dGi = Ar * zi + Ai * zr;
              const int dc = a.dcol[rc.flt];
              put(dc, dMr, dMi, z0r, z0i);
              put(dc + 1, dMr, dMi, z1r, z1i);
              put(dc + ZN, dGr, dGi, z0r, z0i);
              put(dc + ZN + 1, dGr, dGi, z1r, z1i);
              if constexpr (ZF) {
                put(dc + 2, dMr, dMi, z2r, z2i);
                put(dc + 5, dGr, dGi, z2r, z2i);
              }
            }
          }
        }
      }
    } else {
      // past the last event (the final tile only): a zero row
      for (int c = 0; c < a.ncols; ++c) rr[c] = T(0);
    }
    fetch(tile + gridDim.x);
    __syncthreads();
    // ---- Gram tiles: A[i][k] = X[row][16 ti + i], B[k][j] = X[row][16 tj + j], row = 4 s + k;
    //      lane = i + 16 k provides A[i][k] and B[k][j = i].  The A and B operands of a row group
    //      are the same LDS elements, so each group loads NT values per lane and feeds all
    //      NT(NT+1)/2 tiles; consecutive MFMAs accumulate into different tiles.  The next
    //      group's values are read from LDS before the current group's MFMAs are issued.
    const int r16 = lane & 15, k4 = lane >> 4;
    int cofs[NT];   // this lane's column of each tile, padded columns mapped to the zero column
#pragma unroll
    for (int t = 0; t < NT; ++t) cofs[t] = min(16 * t + r16, a.ncols);
    T nx[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) nx[t] = X[k4 * LDX + cofs[t]];
    if constexpr (std::is_same_v<T, float>) {
      // FP32 rows: FP32 matrix cores (each product of two FP32 values, summed in FP32 over the
      // tile's 64 rows), then the tile's sums are added into the FP64 accumulators.  Accumulator
      // layout of the 32-bit form: lane l, register r hold row 4 (l / 16) + r, column l % 16.
      f4_t a32[NTILE];
#pragma unroll
      for (int t = 0; t < NTILE; ++t) a32[t] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
      for (int s = 0; s < 16; ++s) {
        float v[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) v[t] = nx[t];
        if (s + 1 < 16) {
          const int row = 4 * (s + 1) + k4;
#pragma unroll
          for (int t = 0; t < NT; ++t) nx[t] = X[row * LDX + cofs[t]];
        }
        // keep those reads ahead of the MFMAs in the instruction stream
        __builtin_amdgcn_sched_barrier(0);
        int t = 0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
#pragma unroll
          for (int tj = ti; tj < NT; ++tj, ++t) {
            if (ti == NT - 1 && tj == NT - 1 && a.skip_last) continue;
            a32[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[ti], v[tj], a32[t], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NTILE; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] += (double)a32[t][r];
      }
    } else {
      // FP64 rows: FP64 matrix cores.  Accumulator layout of the FP64 form: lane l, register r
      // hold row l / 16 + 4 r, column l % 16.
#pragma unroll 2
      for (int s = 0; s < 16; ++s) {
        double v[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) v[t] = (double)nx[t];
        if (s + 1 < 16) {
          const int row = 4 * (s + 1) + k4;
#pragma unroll
          for (int t = 0; t < NT; ++t) nx[t] = X[row * LDX + cofs[t]];
        }
        __builtin_amdgcn_sched_barrier(0);
        int t = 0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
#pragma unroll
          for (int tj = ti; tj < NT; ++tj, ++t) {
            // the last diagonal tile holds only derivative x derivative products when the
            // derivative columns fill it: nothing reads them, so it is left at zero
            if (ti == NT - 1 && tj == NT - 1 && a.skip_last) continue;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[ti], v[tj], acc[t], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  // ---- block partial: the four accumulator registers of (tile t, lane) are values
  //      v = (t*64 + lane)*4 + r, stored as one 32-byte record per (t, lane) and block at
  //      record (t*64 + lane) * nb + block (blocks of one record group adjacent)
  const int nb = gridDim.x;
  d4_t* P = reinterpret_cast<d4_t*>(a.partial);
#pragma unroll
  for (int t = 0; t < NTILE; ++t) P[((int64_t)t * 64 + lane) * nb + blockIdx.x] = acc[t];
}

// Fixed-order compensated sums over blocks of the 32-byte partial records: block g sums record
// group g (values 4g .. 4g+3) over the nb blocks into out[4g + r].
__global__ __launch_bounds__(256) void reduce_values(const double* __restrict__ partial, int nb, double* out) {
  using im::d4_t;
  const int g = blockIdx.x;
  const d4_t* p = reinterpret_cast<const d4_t*>(partial) + (int64_t)g * nb;
  double s[4] = {0.0, 0.0, 0.0, 0.0}, c[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += 256) {
    const d4_t x4 = p[b];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double x = x4[r];
      const double t = s[r] + x;
      c[r] += (fabs(s[r]) >= fabs(x)) ? (s[r] - t) + x : (x - t) + s[r];
      s[r] = t;
    }
  }
  __shared__ double S[4][256], Cc[4][256];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    S[r][threadIdx.x] = s[r];
    Cc[r][threadIdx.x] = c[r];
  }
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double a = S[r][threadIdx.x], b = S[r][threadIdx.x + w];
        const double tt = a + b, bp = tt - a;
        const double err = (a - (tt - bp)) + (b - bp);
        S[r][threadIdx.x] = tt;
        Cc[r][threadIdx.x] = Cc[r][threadIdx.x] + Cc[r][threadIdx.x + w] + err;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[4 * g + threadIdx.x] = S[threadIdx.x][0] + Cc[threadIdx.x][0];
}

// dynamic LDS of a block: 64 rows of ncols + 1 values
template <typename T> size_t imatrix_smem(int ncols) { return 64 * (size_t)(ncols + 1) * sizeof(T); }

template <typename T, class Sh, int C>
hipError_t launch_imatrix_c(const ImArgs<T, Sh>& a, int nb, double* out, hipStream_t st) {
  if (a.ncols <= 0 || a.ncols > C || (a.ncols & 1)) return hipErrorInvalidValue;
  if constexpr (Sh::NZ >= 2) {
    if (a.zfree) {
      if (a.cnt[5] != 1) return hipErrorInvalidValue;   // refused by the host API
      hipLaunchKernelGGL((imatrix_kernel<T, Sh, C, true>), dim3(nb), dim3(64), imatrix_smem<T>(a.ncols), st, a);
    } else {
      hipLaunchKernelGGL((imatrix_kernel<T, Sh, C, false>), dim3(nb), dim3(64), imatrix_smem<T>(a.ncols), st, a);
    }
  } else {
    if (a.zfree) return hipErrorInvalidValue;
    hipLaunchKernelGGL((imatrix_kernel<T, Sh, C, false>), dim3(nb), dim3(64), imatrix_smem<T>(a.ncols), st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int NT = C / 16;
  const int nv = NT * (NT + 1) / 2 * 256;
  hipLaunchKernelGGL(reduce_values, dim3(nv / 4), dim3(256), 0, st, a.partial, nb, out);
  return hipGetLastError();
}

template <typename T, class Sh, int C> int imatrix_blocks_per_cu_c(int ncols) {
  int nb = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, imatrix_kernel<T, Sh, C, false>, 64, imatrix_smem<T>(ncols));
  return (e == hipSuccess && nb > 0) ? nb : 0;
}
// Blocks (one wavefront each) of the interference-matrix kernel resident per compute unit.
template <typename T, class Sh> int imatrix_blocks_per_cu(int ncols) {
  if (ncols <= 16) return imatrix_blocks_per_cu_c<T, Sh, 16>(ncols);
  if (ncols <= 32) return imatrix_blocks_per_cu_c<T, Sh, 32>(ncols);
  if (ncols <= 64) return imatrix_blocks_per_cu_c<T, Sh, 64>(ncols);
  return imatrix_blocks_per_cu_c<T, Sh, 80>(ncols);
}
template int imatrix_blocks_per_cu<float, ShapeSmall>(int);
template int imatrix_blocks_per_cu<double, ShapeSmall>(int);
template int imatrix_blocks_per_cu<float, ShapeFull>(int);
template int imatrix_blocks_per_cu<double, ShapeFull>(int);

template <typename T, class Sh>
hipError_t launch_imatrix(const ImArgs<T, Sh>& a, int ncols, int nb, double* out, hipStream_t st) {
  if (ncols <= 16) return launch_imatrix_c<T, Sh, 16>(a, nb, out, st);
  if (ncols <= 32) return launch_imatrix_c<T, Sh, 32>(a, nb, out, st);
  if (ncols <= 64) return launch_imatrix_c<T, Sh, 64>(a, nb, out, st);
  if (ncols <= 80) return launch_imatrix_c<T, Sh, 80>(a, nb, out, st);
  return hipErrorInvalidValue;
}
template hipError_t launch_imatrix<float, ShapeSmall>(const ImArgs<float, ShapeSmall>&, int, int, double*, hipStream_t);
template hipError_t launch_imatrix<double, ShapeSmall>(const ImArgs<double, ShapeSmall>&, int, int, double*, hipStream_t);
template hipError_t launch_imatrix<float, ShapeFull>(const ImArgs<float, ShapeFull>&, int, int, double*, hipStream_t);
template hipError_t launch_imatrix<double, ShapeFull>(const ImArgs<double, ShapeFull>&, int, int, double*, hipStream_t);

}  // namespace kpsi

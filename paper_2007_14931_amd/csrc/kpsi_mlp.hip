// Learned efficiency: a 4 -> 64 -> 64 -> 1 network (SiLU, SiLU, sigmoid) trained on accept
// labels with binary cross-entropy and Adam, and evaluated once per normalisation event.
// The 64x64 layer (forward, weight gradient and input gradient) runs on BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16: 16x16 outputs, 32-deep products, 8 operands per lane) with FP32
// accumulation; the 4-wide input layer and the output layer run on the vector ALUs in FP32.
// Master weights are FP32; a small kernel writes the BF16 copies of the 64x64 layer in both
// layouts once per parameter update, and blocks stage them into LDS with 16-byte copies.
//
// Parameter layout (4545 floats): W1[64][4], b1[64], W2[64][64] (row = output), b2[64],
// w3[64], b3.  Network input: u = (2 (m - lo)/(hi - lo) - 1, cos theta_K*, cos theta_J/psi,
// phi/pi).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpsi_internal.h"

namespace kpsi {

namespace nn {

constexpr int P_W1 = 0, P_B1 = 256, P_W2 = 320, P_B2 = 4416, P_W3 = 4480, P_B3 = 4544;
constexpr int TE = 64;   // events per tile

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

struct __align__(16) Smem {
  unsigned short W2[64 * 64];    // [o][i] bf16 (W2 and W2T adjacent: staged as one copy)
  unsigned short W2T[64 * 64];   // [i][o] bf16
  unsigned short H1[TE * 64];    // [e][i]
  unsigned short H1T[64 * TE];   // [i][e]
  unsigned short DZ[TE * 64];    // [e][o]
  unsigned short DZT[64 * TE];   // [o][e]
  float U[TE * 4];
  float Y[TE];
  float W1[256], B1[64], B2[64], W3[64];
  float red[256];
};

// eight consecutive bf16 of an LDS row (16-byte aligned) as an MFMA operand: one 16-byte read
__device__ __forceinline__ bf8_t ld8(const unsigned short* p) { return *reinterpret_cast<const bf8_t*>(p); }

// One 64 x 64 x (64 deep) product tile row for the wave: acc += A[16 rows][64] B[64][16 cols], with
// A's rows at a + 64 * (lane % 16) and B's columns at b + 64 * (lane % 16) (both row-major in k).
// Lane l supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] for each 32-deep half.
__device__ __forceinline__ f4_t mm16x64(const unsigned short* a, const unsigned short* b, int l16, int lg) {
  f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const bf8_t av = ld8(a + 64 * l16 + 32 * kk + 8 * lg);
    const bf8_t bv = ld8(b + 64 * l16 + 32 * kk + 8 * lg);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ float input_of(const MlpArgs& a, int k, int64_t e) {
  const double x = a.obs[k][e];
  if (k == 0) return (float)(2.0 * (x - a.lo) / (a.hi - a.lo) - 1.0);
  if (k == 3) return (float)(x * 0.31830988618379067154);
  return (float)x;
}

// Stage weights into LDS: the BF16 copies of W2 in both layouts (8192 values, from w2h), and the
// FP32 small layers (W1 and w3 rounded to BF16 like W2).
__device__ void stage_weights(const MlpArgs& a, Smem& s) {
  const uint4* src = reinterpret_cast<const uint4*>(a.w2h);
  uint4* dst = reinterpret_cast<uint4*>(s.W2);
  for (int i = threadIdx.x; i < 2 * 4096 * 2 / 16; i += 256) dst[i] = src[i];
  for (int i = threadIdx.x; i < 256; i += 256) s.W1[i] = from_bf16(bf16(a.params[P_W1 + i]));
  if (threadIdx.x < 64) {
    s.B1[threadIdx.x] = a.params[P_B1 + threadIdx.x];
    s.B2[threadIdx.x] = a.params[P_B2 + threadIdx.x];
    s.W3[threadIdx.x] = from_bf16(bf16(a.params[P_W3 + threadIdx.x]));
  }
}

// Forward over one tile of 64 events starting at e0 (rows past n are zero-filled).
// Leaves the inputs and h1 (both layouts) in LDS, returns in z2[nt][r] this lane's 16 values of
// z2 for events 16 w + 4 (lane/16) + r and outputs 16 nt + lane % 16.
__device__ void forward_tile(const MlpArgs& a, Smem& s, int64_t e0, f4_t z2[4]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // inputs and labels
  if (t < TE) {
    const int64_t e = e0 + t;
    const bool ok = e < a.n;
#pragma unroll
    for (int k = 0; k < 4; ++k) s.U[t * 4 + k] = ok ? input_of(a, k, e) : 0.0f;
    s.Y[t] = (ok && a.label) ? (float)a.label[e] : 0.0f;
  }
  __syncthreads();
  // layer 1 (VALU): thread t -> event t % 64, features 16 (t / 64) .. + 15
  {
    const int e = t & 63, j0 = (t >> 6) * 16;
    const float u0 = s.U[e * 4], u1 = s.U[e * 4 + 1], u2 = s.U[e * 4 + 2], u3 = s.U[e * 4 + 3];
#pragma unroll
    for (int j = j0; j < j0 + 16; ++j) {
      const float z = s.B1[j] + s.W1[4 * j] * u0 + s.W1[4 * j + 1] * u1 + s.W1[4 * j + 2] * u2 + s.W1[4 * j + 3] * u3;
      const unsigned short h = bf16(silu(z));
      s.H1[e * 64 + j] = h;
      s.H1T[j * TE + e] = h;
    }
  }
  __syncthreads();
  // layer 2 (MFMA): wave w computes events 16 w .. 16 w + 15 for all 64 outputs:
  // A[m = event][k = input] = h1 (rows of H1), B[k = input][n = output] = W2[output][input]
  const int l16 = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) z2[nt] = mm16x64(&s.H1[(16 * w) * 64], &s.W2[(16 * nt) * 64], l16, lg);
}

}  // namespace nn

// Per-block gradient of the summed BCE (no 1/n) over the events [blk*per, (blk+1)*per),
// written block-major to partial[block * 4546 + v] (one contiguous record per block, so the
// writes are coalesced); v = 4545 is the loss.
__global__ __launch_bounds__(256) void mlp_grad_kernel(MlpArgs a) {
  using namespace nn;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Smem& s = *reinterpret_cast<Smem*>(smem_raw);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, l16 = lane & 15, lg = lane >> 4;
  stage_weights(a, s);
  const float b3 = a.params[P_B3];
  float gW2[4][4];        // dW2[o = 16 w + 4 lg + r][i = 16 nt + l16]
  float gb2[4], gw3[4];   // outputs 16 nt + l16 (this lane's events)
  float gb1[4], gW1[4][4];
  float gb3 = 0.f, loss = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gb2[i] = gw3[i] = gb1[i] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) { gW2[i][k] = 0.f; gW1[i][k] = 0.f; }
  }
  __syncthreads();
  const int64_t begin = (int64_t)blockIdx.x * a.per_block;
  const int64_t end = begin + a.per_block < a.n ? begin + a.per_block : a.n;
  for (int64_t e0 = begin; e0 < end; e0 += TE) {
    f4_t z2[4];
    forward_tile(a, s, e0, z2);
    // output layer: z3 for events 16 w + 4 lg + r
    float z3p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int o = 16 * nt + l16;
      const float bb = s.B2[o], ww = s.W3[o];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        z2[nt][r] += bb;
        z3p[r] += ww * silu(z2[nt][r]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) z3p[r] += __shfl_xor(z3p[r], off, 64);
    }
    float dz3[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = 16 * w + 4 * lg + r;
      const bool ok = e0 + e < end;
      const float p = 1.0f / (1.0f + __expf(-(z3p[r] + b3)));
      const float y = s.Y[e];
      dz3[r] = ok ? p - y : 0.0f;
      if (ok && l16 == 0) {
        const float pc = fminf(fmaxf(p, 1e-12f), 1.0f - 1e-12f);
        loss += -(y * __logf(pc) + (1.0f - y) * __logf(1.0f - pc));
        gb3 += dz3[r];
      }
    }
    // back-propagate to z2: dz2 = dz3 w3 silu'(z2); bias and w3 gradients
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int o = 16 * nt + l16;
      const float ww = s.W3[o];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = 16 * w + 4 * lg + r;
        const float z = z2[nt][r];
        gw3[nt] += dz3[r] * silu(z);
        const float d = dz3[r] * ww * dsilu(z);
        gb2[nt] += d;
        const unsigned short h = bf16(d);
        s.DZ[e * 64 + o] = h;
        s.DZT[o * TE + e] = h;
      }
    }
    __syncthreads();
    // dW2[o][i] += sum_e dz2[e][o] h1[e][i]: wave w owns o-tile w;
    // A[m = o][k = e] = dz2[e][o] (rows of DZT), B[k = e][n = i] = h1[e][i] (rows of H1T)
    static_assert(TE == 64, "tile rows are 64 deep");
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f4_t acc = nn::mm16x64(&s.DZT[(16 * w) * TE], &s.H1T[(16 * nt) * TE], l16, lg);
#pragma unroll
      for (int r = 0; r < 4; ++r) gW2[nt][r] += acc[r];
    }
    // dh1[e][i] = sum_o dz2[e][o] W2[o][i]: wave w owns events 16 w ..;
    // A[m = e][k = o] = dz2 (rows of DZ), B[k = o][n = i] = W2[o][i] (rows of W2T)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f4_t acc = nn::mm16x64(&s.DZ[(16 * w) * 64], &s.W2T[(16 * nt) * 64], l16, lg);
      const int i = 16 * nt + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = 16 * w + 4 * lg + r;
        const float z1 = s.B1[i] + s.W1[4 * i] * s.U[e * 4] + s.W1[4 * i + 1] * s.U[e * 4 + 1] +
                         s.W1[4 * i + 2] * s.U[e * 4 + 2] + s.W1[4 * i + 3] * s.U[e * 4 + 3];
        const float dz1 = acc[r] * nn::dsilu(z1);
        gb1[nt] += dz1;
#pragma unroll
        for (int k = 0; k < 4; ++k) gW1[nt][k] += dz1 * s.U[e * 4 + k];
      }
    }
    __syncthreads();
  }
  // ---- block partials (value-major).  dW2 entries have a unique owner lane.
  float* rec = a.partial + (int64_t)blockIdx.x * (MLP_NV);
  auto put = [&](int v, float x) { rec[v] = x; };
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) put(P_W2 + (16 * w + 4 * lg + r) * 64 + 16 * nt + l16, gW2[nt][r]);
  // per-output sums: combine the 4 lane groups of a wave, then the 4 waves, in fixed order
  auto reduce_out = [&](float x, int v) {
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    if (lg == 0) s.red[w * 64 + l16 + 0] = x;   // 16 values per wave at [w*64 + l16]
    __syncthreads();
    if (t < 16) put(v + t, ((s.red[t] + s.red[64 + t]) + s.red[128 + t]) + s.red[192 + t]);
    __syncthreads();
  };
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    reduce_out(gb2[nt], P_B2 + 16 * nt);
    reduce_out(gw3[nt], P_W3 + 16 * nt);
    reduce_out(gb1[nt], P_B1 + 16 * nt);
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float x = gW1[nt][k];
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      if (lg == 0) s.red[w * 64 + l16] = x;
      __syncthreads();
      if (t < 16) put(P_W1 + 4 * (16 * nt + t) + k, ((s.red[t] + s.red[64 + t]) + s.red[128 + t]) + s.red[192 + t]);
      __syncthreads();
    }
  // b3 and loss: a butterfly in each wavefront, then the four wavefronts in order
  auto block_sum = [&](float x) -> float {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) s.red[w] = x;
    __syncthreads();
    const float r = ((s.red[0] + s.red[1]) + s.red[2]) + s.red[3];
    __syncthreads();
    return r;
  };
  const float sb3 = block_sum(gb3), sloss = block_sum(loss);
  if (t == 0) {
    put(P_B3, sb3);
    put(4545, sloss);
  }
}

// Sum of block-major partials in FP64, fixed order: out[v] = scale * sum_b partial[b * nv + v].
// A workgroup takes 64 consecutive values; its four wavefronts take the blocks b = s mod 4
// (s = 0..3), each lane keeping four sums (blocks 16 k + s, + 4, + 8, + 12) so four reads are in
// flight, and the 4 x 4 sums are combined in a fixed order.  A wavefront reads 64 consecutive
// values of one block record: every read is coalesced.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial, int nb, int nv,
                                                         double scale, double* __restrict__ out) {
  __shared__ double red[4][64];
  const int vl = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const int v = blockIdx.x * 64 + vl;
  double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
  if (v < nv) {
    int b = seg;
    for (; b + 12 < nb; b += 16) {
      x0 += (double)partial[(int64_t)b * nv + v];
      x1 += (double)partial[(int64_t)(b + 4) * nv + v];
      x2 += (double)partial[(int64_t)(b + 8) * nv + v];
      x3 += (double)partial[(int64_t)(b + 12) * nv + v];
    }
    for (; b < nb; b += 4) x0 += (double)partial[(int64_t)b * nv + v];
  }
  red[seg][vl] = (x0 + x1) + (x2 + x3);
  __syncthreads();
  if (seg == 0 && v < nv) out[v] = scale * (((red[0][vl] + red[1][vl]) + red[2][vl]) + red[3][vl]);
}

// Adam step on the FP32 master parameters; with w2h, also the BF16 copies of the updated 64x64
// layer in both layouts (as launch_mlp_bf16 writes them).
__global__ __launch_bounds__(256) void adam_kernel(float* p, float* m, float* v, const double* g, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2,
                                                   unsigned short* w2h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = (float)g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  const int k = i - nn::P_W2;
  if (w2h && k >= 0 && k < 4096) {
    const unsigned short h = nn::bf16(pi);
    w2h[k] = h;
    w2h[4096 + (k & 63) * 64 + (k >> 6)] = h;
  }
}

// Probabilities of the network for n events.
__global__ __launch_bounds__(256) void mlp_eval_kernel(MlpArgs a) {
  using namespace nn;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Smem& s = *reinterpret_cast<Smem*>(smem_raw);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, l16 = lane & 15, lg = lane >> 4;
  stage_weights(a, s);
  const float b3 = a.params[P_B3];
  __syncthreads();
  const int64_t begin = (int64_t)blockIdx.x * a.per_block;
  const int64_t end = begin + a.per_block < a.n ? begin + a.per_block : a.n;
  for (int64_t e0 = begin; e0 < end; e0 += TE) {
    f4_t z2[4];
    forward_tile(a, s, e0, z2);
    float z3p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int o = 16 * nt + l16;
      const float bb = s.B2[o], ww = s.W3[o];
#pragma unroll
      for (int r = 0; r < 4; ++r) z3p[r] += ww * silu(z2[nt][r] + bb);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) z3p[r] += __shfl_xor(z3p[r], off, 64);
      const int64_t e = e0 + 16 * w + 4 * lg + r;
      if (l16 == 0 && e < end) a.out[e] = 1.0 / (1.0 + exp(-(double)(z3p[r] + b3)));
    }
    __syncthreads();
  }
}

// Accept labels: label_e = [u_e < eps_true(x_e)], u_e from Philox counter (e, 0, 3).
__device__ __forceinline__ void philox_c(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void label_kernel(LabelArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n) return;
  uint32_t c[4] = {(uint32_t)(a.e0 + e), (uint32_t)((uint64_t)(a.e0 + e) >> 32), 0u, 3u};
  philox_c(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  const double u = (double)(((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
  const double x[4] = {2.0 * (a.obs[0][e] - a.lo) / (a.hi - a.lo) - 1.0, a.obs[1][e], a.obs[2][e],
                       a.obs[3][e] / 3.14159265358979323846};
  double eps = 0.9;
  for (int d = 0; d < 4; ++d) {
    const double v = x[d];
    const double P1 = v, P2 = 0.5 * (3.0 * v * v - 1.0), P3 = 0.5 * (5.0 * v * v * v - 3.0 * v);
    const double num = a.coef[3 * d] * P1 + a.coef[3 * d + 1] * P2 + a.coef[3 * d + 2] * P3;
    const double den = fabs(a.coef[3 * d]) + fabs(a.coef[3 * d + 1]) + fabs(a.coef[3 * d + 2]);
    const double tt = den > 0.0 ? num / den : 0.0;
    eps *= 1.0 - a.delta * (1.0 - tt) / 2.0;
  }
  if (a.eps_out) a.eps_out[e] = eps;
  a.label[e] = (u < eps) ? 1 : 0;
}
#pragma clang fp contract(on)

// Histogram counts: generated and accepted events per bin of a 4D grid (integer atomics,
// so the counts are exact and order-independent).
__global__ __launch_bounds__(256) void hist_count_kernel(HistCountArgs a) {
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
  atomicAdd(&a.gen[idx], 1u);
  if (a.label[e]) atomicAdd(&a.acc[idx], 1u);
}

// BF16 copies of the 64x64 layer's weights: w2h[0, 4096) = W2[o][i], w2h[4096, 8192) = W2[o][i] at [i][o].
__global__ __launch_bounds__(256) void mlp_bf16_kernel(const float* __restrict__ params, unsigned short* __restrict__ w2h) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= 4096) return;
  const unsigned short h = nn::bf16(params[nn::P_W2 + i]);
  w2h[i] = h;
  w2h[4096 + (i & 63) * 64 + (i >> 6)] = h;
}

size_t mlp_smem_bytes() { return sizeof(nn::Smem); }

hipError_t launch_mlp_bf16(const float* params, unsigned short* w2h, hipStream_t st) {
  hipLaunchKernelGGL(mlp_bf16_kernel, dim3(16), dim3(256), 0, st, params, w2h);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpArgs& a, int nb, hipStream_t st) {
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb), dim3(256), sizeof(nn::Smem), st, a);
  return hipGetLastError();
}
hipError_t launch_mlp_reduce(const float* partial, int nb, int nv, double scale, double* out, hipStream_t st) {
  if (nv != MLP_NV) return hipErrorInvalidValue;   // the block records are MLP_NV values long
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((nv + 63) / 64), dim3(256), 0, st, partial, nb, nv, scale, out);
  return hipGetLastError();
}
hipError_t launch_adam(float* p, float* m, float* v, const double* g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, unsigned short* w2h, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, m, v, g, n, lr, b1, b2, eps, c1, c2,
                     w2h);
  return hipGetLastError();
}
hipError_t launch_mlp_eval(const MlpArgs& a, int nb, hipStream_t st) {
  hipLaunchKernelGGL(mlp_eval_kernel, dim3(nb), dim3(256), sizeof(nn::Smem), st, a);
  return hipGetLastError();
}
hipError_t launch_labels(const LabelArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(label_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_hist_count(const HistCountArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(hist_count_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace kpsi

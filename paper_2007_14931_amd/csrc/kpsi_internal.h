// Internal declarations shared by the device code and the host runtime of libkpsi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpsi.h"

namespace kpsi {

constexpr int BLOCK = 256;      // threads per block (4 wavefronts of 64)
constexpr int NACC = 64;        // doubles per block partial (one per lane of a wavefront)
constexpr int NFL = 2;          // floating (M, Gamma0) slots in the adjoint
constexpr int NCOL_KSTAR = 9;   // per-event columns of the K* chain
constexpr int NCOL_Z = 7;       // extra per-event columns of the Z chain
constexpr int NCOL_ZFREE = 2;   // and of a Z whose H'_{+1}, H'_{-1} are independent
constexpr int NCOL_MAX = 4 * ((NCOL_KSTAR + NCOL_Z + NCOL_ZFREE + 3) / 4);   // whole column groups
// Per-event columns are stored in groups of four: column k of event e sits at element
// ((k / 4) * ld + e) * 4 + k % 4, so one 16-byte (FP32) or 32-byte (FP64) load per lane
// reads four columns of an event, and a wavefront's load is one contiguous span.
__host__ __device__ constexpr int col_groups(int ncol) { return (ncol + 3) / 4; }
__host__ __device__ constexpr int64_t col_at(int k, int64_t e, int64_t ld) {
  return ((int64_t)(k >> 2) * ld + e) * 4 + (k & 3);
}

enum { MODE_DENSITY = 0, MODE_NLL = 1, MODE_GRAD = 2 };

// Per-resonance constants of one call (host-computed in double, stored as T).
//   den(m) = M2 - m^2 - i P g(m),  A(m) = K n(m) / den(m)
template <typename T> struct RC {
  T M2, P, K;
  T M2lo;             // M^2 - M2 (FP32 constants: the rounding remainder of M^2; FP64: 0)
  T hr[3], hi[3];     // K*: lambda = -1, 0, +1; Z: [0] lambda' = 0, [1] lambda' = +-1 (Eq. 11)
                      // or, free helicities, [1] lambda' = +1 and [2] lambda' = -1
  T kap, twoM, dP, PoG;   // d ln K/dM, 2M, dP/dM, P/Gamma0
  int flt;            // floating slot or -1
  T f0, f1;           // 1 where flt is 0 (1), else 0
  int lass;           // 1: LASS S-wave (spin-0 K* only), 0: Breit-Wigner
  T lai, lhb;         // LASS 1/a and b/2: q cot(delta_B) = lai + lhb q^2
};

// Compile-time capacity of a kernel instantiation: K* slots per spin 0..4 and Z slots.
template <int N0, int N1, int N2, int N3, int N4, int NZ_> struct Shape {
  static constexpr int N[5] = {N0, N1, N2, N3, N4};
  static constexpr int NK = N0 + N1 + N2 + N3 + N4;
  static constexpr int NZ = NZ_;
  static constexpr int NKACC = 2 * N0 + 6 * (N1 + N2 + N3 + N4);
  // Coupling accumulators [LDS_LO, LDS_HI) (spins 1..3) that the per-event gradient kernel
  // keeps in per-thread LDS slots instead of registers, for the large shape only: 36 values x
  // 256 threads per block (36 KB in FP32, 4 blocks per compute unit; 72 KB in FP64, 2 blocks),
  // and the freed registers allow 4 (FP32) or 2 (FP64) wavefronts per SIMD.
  static constexpr int LDS_LO = (NK >= 8) ? 2 * N0 : 0;
  static constexpr int LDS_HI = (NK >= 8) ? 2 * N0 + 6 * (N1 + N2 + N3) : 0;
  static_assert(3 + NKACC + 4 * NZ_ + 2 * NFL + 1 <= NACC, "accumulators exceed the block record");
};
using ShapeSmall = Shape<0, 1, 0, 0, 0, 0>;   // one spin-1 K*
using ShapeFull = Shape<3, 3, 2, 1, 1, 2>;    // the ten K* of the paper and two Z

template <typename T> struct AccType { using type = T; };

template <typename T, class Sh> struct AmpArgs {
  const T* cols[2];     // data, normalisation column bases
  int64_t ld[2];        // column strides (elements)
  int64_t n[2];         // events per set
  const T* eps;         // per-normalisation-event efficiency, or null (flat)
  double* partial;      // value-major: value v of block b at [v * pstride + poff + b]
  int64_t pstride;      // row stride of the partials (blocks of both sets)
  int poff;             // block offset of this launch in the partial rows
  double* s_out[2];     // density mode: per-event S of each set
  int nb_data;          // blocks of the data set; the rest cover the normalisation set
  int chunk;            // events per block
  int cnt[6];           // slots in use per spin 0..4 and Z
  T rR, rB, invMB;
  RC<T> ks[Sh::NK > 0 ? Sh::NK : 1];
  RC<T> zs[Sh::NZ > 0 ? Sh::NZ : 1];
  // Signal + background mixture (Eq. 14) on the data set, active when bkg_data != null:
  // each data event contributes ln t with t = purity eps_i S_i + k b_i, where
  // k = bkg_coef * sum eps S over the normalisation events (bkg_coef = (1 - p) / (N_b N_MC)).
  // The sum comes from the normalisation launch's block partials (mc_part: values 0 and 1 of
  // mc_nb blocks, rows pstride apart), or, when mc_part is null, from norm_total (a reduced
  // record in device memory: the interference-matrix normalisation).
  // Flavour-tagged events (text after Eq. 12), active when tag != null: data event i is read
  // with phi -> tag[i] phi (weight keep = 1 - mistag) and, when mistag > 0, with -tag[i] phi
  // (weight mistag); the normalisation events give record 1 (phi) and record 2 (-phi) from
  // nb_mc blocks each.
  const T* tag;
  T mistag, keep;
  int nb_mc;
  const T* eps_data;    // per-data-event efficiency, or null (1)
  const T* bkg_data;    // per-data-event background density, or null (signal only)
  const double* mc_part;
  int mc_nb;
  const double* norm_total;
  double bkg_coef;
  T purity;
  // Free Z helicities (one Z, H'_{+1} and H'_{-1} independent): selects the kernel
  // instantiation that reads the extra angular columns; its lambda' = -1 accumulators take the
  // record slots of the (then unused) second Z.
  int zfree;
};
// Record slot of sum_i w_i S_i over the data events of the mixture (gradient mode).
template <class Sh> constexpr int ws_slot() { return 3 + Sh::NKACC + 4 * Sh::NZ + 2 * NFL; }

template <typename T> struct InvArgs {
  const double* obs[4];   // m_Kpi, cos theta_K*, cos theta_J/psi, phi
  T* cols;
  int64_t ld, n;
  double mB, mJ, mK, mPi, rB, rR;
  int with_z;
  int zfree;              // with_z and free Z helicities: columns 14-17 hold the separate factors
  double* diag;           // optional (n, 5) output: m_Jpsi pi, cos theta_Z, cos theta~, phi~, alpha
};

struct HistArgs {
  const double* obs[4];
  const float* table;
  int nb[4];
  double lo[4], hi[4];
  int64_t n;
  double* out_f64;
};

// Product of a 2D table over (m_Kpi, cos theta_K*) and a 2D table over (cos theta_J/psi, phi),
// looked up per event (bins [lo, hi), clamped into the edge bins), written as FP64.
struct TplArgs {
  const double* obs[4];
  const float* t1;      // nb[0] x nb[1], row-major
  const float* t2;      // nb[2] x nb[3], row-major
  int nb[4];
  double lo[4], hi[4];
  int64_t n;
  double* out;
};

struct GenArgs {
  uint64_t seed;
  int64_t e0, n;
  double wmax, mB, mJ, mK, mPi;
  double* out[4];
  double* spare;
  int* flag;
};

struct AcceptArgs {
  const double* obs[4];
  const double* S;
  const double* spare;
  const int* valid;
  int acc_on;
  double coef[12];
  double delta, lo, hi, smax;
  int64_t n;
  int* flag;
  int* over;
};

struct CompactArgs {
  const double* obs[4];
  const int* flag;
  const int* pos;
  int64_t n, base, limit;
  double* out[4];
};

// Interference-matrix build: per-event component amplitudes of the normalisation set.
template <typename T, class Sh> struct ImArgs {
  const T* cols;
  int64_t ld, n;
  const T* eps;         // per-event efficiency or null
  double* partial;      // block partials of the Gram tiles, in 32-byte records (four values)
  int ncols;            // real columns in use (even; at most the kernel's padded width)
  int skip_last;        // 1: the last diagonal 16 x 16 tile has derivative columns only; skip it
  int cnt[6];
  int dcol[NFL];        // first derivative component of floating slot f
  T rR, rB, invMB;
  RC<T> ks[Sh::NK > 0 ? Sh::NK : 1];
  RC<T> zs[Sh::NZ > 0 ? Sh::NZ : 1];
  int zfree;            // one Z with independent H'_{+1}, H'_{-1}: three Z components (0, +1, -1)
};

constexpr int MLP_NV = 4546;     // values per block record of the network gradient: 4545 parameters and the loss
struct MlpArgs {
  const double* obs[4];
  const uint8_t* label;   // accept labels (training) or null
  const float* params;    // FP32 master parameters (4545)
  const unsigned short* w2h;   // BF16 W2 [o][i] then [i][o] (8192, 16-byte aligned; launch_mlp_bf16)
  float* partial;         // value-major block gradients (4546 values x blocks)
  double* out;            // probabilities (evaluation)
  double lo, hi;          // m_Kpi range of the input map
  int64_t n, per_block;
};

struct LabelArgs {
  const double* obs[4];
  uint64_t seed;
  int64_t e0, n;
  double coef[12];
  double delta, lo, hi;
  uint8_t* label;
  double* eps_out;        // optional true efficiency per event
};

struct HistCountArgs {
  const double* obs[4];
  const uint8_t* label;
  int nb[4];
  double lo[4], hi[4];
  int64_t n;
  unsigned int* gen;
  unsigned int* acc;
};

size_t mlp_smem_bytes();
hipError_t launch_mlp_bf16(const float* params, unsigned short* w2h, hipStream_t st);
hipError_t launch_mlp_grad(const MlpArgs& a, int nb, hipStream_t st);
hipError_t launch_mlp_reduce(const float* partial, int nb, int nv, double scale, double* out, hipStream_t st);
hipError_t launch_adam(float* p, float* m, float* v, const double* g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, unsigned short* w2h, hipStream_t st);
hipError_t launch_mlp_eval(const MlpArgs& a, int nb, hipStream_t st);
hipError_t launch_labels(const LabelArgs& a, hipStream_t st);
hipError_t launch_hist_count(const HistCountArgs& a, hipStream_t st);

template <typename T> hipError_t launch_invariants(const InvArgs<T>& a, hipStream_t st);
template <typename T, class Sh>
hipError_t launch_imatrix(const ImArgs<T, Sh>& a, int ncols, int nb, double* out, hipStream_t st);
template <typename T, class Sh> int imatrix_blocks_per_cu(int ncols);
template <typename T, class Sh> hipError_t launch_amp(const AmpArgs<T, Sh>& a, int mode, int nblocks, hipStream_t st);
template <typename T, class Sh> int amp_blocks_per_cu(int mode, bool cc, bool zfree);
// Fixed-order sums of the block partials of records first_set .. first_set + n_sets - 1 into
// out[set * NACC + v] (record 0: data blocks; records 1 .. n_mc_sets: runs of nb_mc
// normalisation blocks).
hipError_t launch_reduce_final(const double* partial, int nb_data, int nb_mc, int n_mc_sets, int nv, double* out,
                               int first_set, int n_sets, hipStream_t st);
hipError_t launch_hist_lookup(const HistArgs& a, hipStream_t st);
hipError_t launch_template(const TplArgs& a, hipStream_t st);
hipError_t launch_phsp(const GenArgs& a, hipStream_t st);
hipError_t launch_accept(const AcceptArgs& a, hipStream_t st);
hipError_t launch_compact(const CompactArgs& a, hipStream_t st);
hipError_t exclusive_scan_int(const int* in, int* out, int64_t n, void* tmp, size_t* tmp_bytes, hipStream_t st);

// Record an error message on a context (the host runtime's kpsi_last_error) and return s.
kpsi_status set_error(kpsi_ctx* c, kpsi_status s, const char* msg);

}  // namespace kpsi

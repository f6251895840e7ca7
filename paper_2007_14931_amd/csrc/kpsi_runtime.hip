// Host runtime of libkpsi: the C ABI of include/kpsi.h.
//
// Owns the device buffers of a context (event columns, efficiency, block partials,
// pinned result staging), packs the fit parameters into per-resonance constants,
// launches the per-event kernel and the final reduction on the context stream, and
// assembles -2 ln L and its gradient from the reduced sums.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kpsi.h"
#include "kpsi_internal.h"

using namespace kpsi;

// Block partials of kpsi_nll_and_grad_noalloc: a fixed device array in place of the buffer a
// context allocates (16384 block partials of NACC doubles, 8 MiB).  Each device holds its own
// copy for the life of the process; host code reaches it only through the address looked up
// per device (scratch_ptr), never through the array's name.
constexpr size_t kScratchDoubles = (size_t)16384 * NACC;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_looked_up[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with that device current
// (kpsi_create); null when the lookup failed or the device index is beyond the table.
void lookup_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_looked_up[device]) return;
  g_scratch_looked_up[device] = true;
  double* ptr = nullptr;
  if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[device] = ptr;
  else (void)hipGetLastError();
}
double* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

struct DevSet {
  int64_t n = 0;
  const double* obs[4] = {nullptr, nullptr, nullptr, nullptr};
  double* owned = nullptr;      // owned FP64 copy (4 columns)
  void* cols = nullptr;         // derived columns (T)
  int64_t ld = 0;
  size_t cols_cap = 0;
};

std::string g_create_error;
constexpr size_t kTimingSamples = 65536;   // timed kernel durations kept for the median
constexpr int kTimingPairs = 64;            // timed calls whose events are read together

}  // namespace

struct kpsi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  kpsi_precision prec = KPSI_FP64;
  bool has_model = false;
  kpsi_kinematics kin{};
  std::vector<kpsi_resonance> res;
  int shape = 0;                // 0: ShapeSmall, 1: ShapeFull
  std::vector<int> slot;        // table index -> K* slot index, or Z index
  std::vector<int> coff;        // table index -> coupling offset in the parameter vector
  int cnt[6] = {0, 0, 0, 0, 0, 0};
  int nparams = 0;
  bool has_z = false;
  bool zfree = false;   // the model's one Z has independent H'_{+1}, H'_{-1}
  std::vector<int> fslot;       // table index -> floating slot or -1
  DevSet set[2];
  void* eps = nullptr;          // T array over the normalisation set, or null (flat): the
                                // efficiency times the importance weight of each event
  double* eps_f64 = nullptr;    // FP64 efficiency over the normalisation set, or null (flat)
  // importance weights of a mixed normalisation set (kpsi_set_norm_mixture), or null (flat set)
  double* norm_w = nullptr;     // FP64, device
  void* wcol = nullptr;         // the same as a T column (efficiency-free integrals)
  std::vector<double> norm_w_host;
  double* partial = nullptr;
  size_t partial_cap = 0;       // in doubles
  double* red = nullptr;        // device view of red_host
  double* red_host = nullptr;   // [3][NACC], mapped pinned host memory (fine-grained, so the
                                // reduction's stores reach it as they are made): data,
                                // normalisation, and the normalisation read with phi reversed
                                // (flavour tags).  A call marks the values its reduction writes
                                // with kPending and polls them (wait_results).
  double* red_dev = nullptr;    // [3][NACC] device copy of the normalisation records 1, 2 (mixture)
  // Gaussian constraints on parameters (kpsi_set_constraints): position, mean, sigma
  std::vector<int> con_idx;
  std::vector<double> con_mean, con_sigma;
  // flavour-tagged events (kpsi_set_flavour)
  bool cc_on = false;
  void* tag = nullptr;          // T array over the data set, +1 / -1
  double mistag = 0.0;
  int64_t ntag[2] = {0, 0};     // data events tagged +1, -1
  // signal + background mixture of Eq. 14 (kpsi_set_background)
  bool bkg_on = false;
  double purity = 1.0;
  double bkg_coef = 0.0;        // (1 - p) / (N_b N_MC)
  void* eps_data = nullptr;     // T per data event, or null (efficiency 1)
  void* bkg_data = nullptr;     // T per data event
  std::string err;
  bool timing = false;           // this call records timing events
  int timing_every = 0;          // time every k-th call (0: off)
  int64_t timing_calls = 0;      // calls since timing was set
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // event pairs of the timed calls (kpsi_set_timing), read when all are used or when the
  // timings are asked for, so that a timed call does not wait for its events
  std::vector<hipEvent_t> tev;
  int t_pend = 0;                // recorded pairs not yet read
  double t_ms = 0.0;
  int64_t t_n = 0;
  std::vector<float> t_samples;  // the first kTimingSamples timed durations since the last reset
  int64_t t_dropped = 0;         // timed calls whose duration could not be read
  unsigned short* mlp_w2h = nullptr;   // BF16 copies of the network's 64x64 layer (8192 values)
  int bench_reps = 0;             // kpsi_time_kernel: back-to-back launches of the per-event work
  double bench_ms = 0.0;          // their duration per launch
  int ept_override = 0;
  int n_cu = 0;                                                   // compute units of the device
  int blocks_per_cu[2][3][4] = {{{-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}},
                                {{-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}}};   // [shape][mode][cc + 2 zfree]
  // interference-matrix cache of the normalisation sum (mode 0 off, 1 on, 2 auto)
  int cache_mode = 0;
  bool cache_valid = false;
  std::vector<double> cache_ls;           // lineshape parameters the cache was built at
  std::vector<double> last_ls;            // lineshape parameters of the previous call (auto mode)
  int ls_streak = 0;                      // consecutive calls at last_ls
  int cache_ncomp = 0, cache_ncols = 0;   // complex components, derivative components
  std::vector<double> cache_I;            // ncomp x ncomp complex (re, im), sums over the set
  std::vector<double> cache_D;            // (ncols - ncomp) x ncomp complex
  int cache_dcol[NFL] = {0, 0};
  double* cache_partial = nullptr;
  size_t cache_partial_cap = 0;
  double* cache_out = nullptr;
  size_t cache_out_cap = 0;
  int64_t cache_builds = 0, cache_hits = 0;
  double cache_build_ms = 0.0;
};

namespace {

kpsi_status fail(kpsi_ctx* c, kpsi_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else g_create_error = buf;
  return s;
}

}  // namespace

kpsi_status kpsi::set_error(kpsi_ctx* c, kpsi_status s, const char* msg) { return fail(c, s, "%s", msg); }

namespace {

#define HIPCHECK(c, call)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail((c), KPSI_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t tsize(const kpsi_ctx* c) { return c->prec == KPSI_FP32 ? sizeof(float) : sizeof(double); }

int lowest_lb(const kpsi_resonance& r) { return r.chain == 0 ? (r.spin == 0 ? 1 : r.spin - 1) : 1; }
int lowest_lr(const kpsi_resonance& r) { return r.chain == 0 ? r.spin : 0; }
int ncoup(const kpsi_resonance& r) { return r.chain == 0 ? (r.spin == 0 ? 1 : 3) : (r.hel_free ? 3 : 2); }

// ---------------------------------------------------------------- lineshape constants
// A(m) = K n(m) / (M^2 - m^2 - i P g(m)) reproduces Eq. (2)-(3) with the per-event
// factors n(m) = (p_B/M_B)^LB (q/m)^LR / sqrt(B_LB(z_B) B_LR(z_R)) and
// g(m) = q^(2LR+1) / (m B_LR(z_R)); here K = sqrt(B_LB(z_B0) B_LR(z_R0)) and
// P = Gamma0 M^2 B_LR(z_R0) / q0^(2LR+1), plus their M derivatives.
struct LsConst { double M2, P, K, kap, twoM, dP, PoG; };

double bpoly(int L, double z) {
  switch (L) {
    case 0: return 1.0;
    case 1: return 1.0 + z;
    case 2: return 9.0 + z * (3.0 + z);
    case 3: return 225.0 + z * (45.0 + z * (6.0 + z));
    default: return 11025.0 + z * (1575.0 + z * (135.0 + z * (10.0 + z)));
  }
}
double dbpoly(int L, double z) {
  switch (L) {
    case 0: return 0.0;
    case 1: return 1.0;
    case 2: return 3.0 + 2.0 * z;
    case 3: return 45.0 + z * (12.0 + 3.0 * z);
    default: return 1575.0 + z * (270.0 + z * (30.0 + 4.0 * z));
  }
}

LsConst lineshape_consts(const kpsi_kinematics& k, const kpsi_resonance& r, double M, double G0) {
  const int LR = lowest_lr(r), LB = lowest_lb(r);
  double m1, m2, mp;
  if (r.chain == 0) { m1 = k.m_k; m2 = k.m_pi; mp = k.m_jpsi; }
  else { m1 = k.m_jpsi; m2 = k.m_pi; mp = k.m_k; }
  const double a2 = (m1 + m2) * (m1 + m2), b2 = (m1 - m2) * (m1 - m2);
  const double f = (M * M - a2) * (M * M - b2);
  const double sf = std::sqrt(std::fmax(f, 0.0));
  const double q0 = sf / (2.0 * M);
  const double dq0 = (2.0 * M * M - a2 - b2) / (2.0 * sf) - q0 / M;
  const double mB2 = k.m_b * k.m_b;
  const double u = mB2 - (mp + M) * (mp + M), v = mB2 - (mp - M) * (mp - M);
  const double h = u * v;
  const double sh = std::sqrt(std::fmax(h, 0.0));
  const double pB0 = sh / (2.0 * k.m_b);
  const double dh = -2.0 * (mp + M) * v + 2.0 * (mp - M) * u;
  const double dpB0 = dh / (4.0 * k.m_b * sh);
  const double zR0 = (k.r_r * q0) * (k.r_r * q0), dzR0 = 2.0 * k.r_r * k.r_r * q0 * dq0;
  const double zB0 = (k.r_b * pB0) * (k.r_b * pB0), dzB0 = 2.0 * k.r_b * k.r_b * pB0 * dpB0;
  const double BR0 = bpoly(LR, zR0), dBR0 = dbpoly(LR, zR0);
  const double BB0 = bpoly(LB, zB0), dBB0 = dbpoly(LB, zB0);
  LsConst c;
  c.M2 = M * M;
  c.twoM = 2.0 * M;
  c.K = std::sqrt(BB0 * BR0);
  c.kap = 0.5 * (dBB0 * dzB0 / BB0 + dBR0 * dzR0 / BR0);
  double q0p = 1.0;
  for (int i = 0; i < 2 * LR + 1; ++i) q0p *= q0;
  c.PoG = M * M * BR0 / q0p;
  c.P = G0 * c.PoG;
  c.dP = c.P * (2.0 / M + dBR0 * dzR0 / BR0 - (2 * LR + 1) * dq0 / q0);
  return c;
}

// The couplings are stored multiplied by the resonance constant K (H' = K H): the per-event
// kernel evaluates the bare Breit-Wigner and leaves K to the couplings, so its coupling
// accumulators come out divided by K (undone in kpsi_nll_and_grad).
template <typename T> void fill_rc(RC<T>& rc, const LsConst& c, const double* hr, const double* hi, int nl, int flt) {
  rc.M2 = (T)c.M2; rc.P = (T)c.P; rc.K = (T)c.K;
  rc.M2lo = (T)(c.M2 - (double)rc.M2);
  for (int l = 0; l < 3; ++l) {
    rc.hr[l] = (T)(l < nl ? c.K * hr[l] : 0.0);
    rc.hi[l] = (T)(l < nl ? c.K * hi[l] : 0.0);
  }
  rc.kap = (T)c.kap; rc.twoM = (T)c.twoM; rc.dP = (T)c.dP; rc.PoG = (T)c.PoG;
  rc.flt = flt;
  rc.f0 = (T)(flt == 0 ? 1 : 0);
  rc.f1 = (T)(flt == 1 ? 1 : 0);
  rc.lass = 0;
  rc.lai = rc.lhb = T(0);
}

// Pack the canonical parameter vector into kernel arguments.
template <typename T, class Sh> void pack(const kpsi_ctx* c, const double* par, AmpArgs<T, Sh>& a) {
  const int ncr = c->nparams - 2 * (int)c->res.size();
  // K* slots the model leaves empty are still evaluated by the kernel: zero couplings, M^2 = P = 0
  // (a finite Breit-Wigner), not floating
  for (int k = 0; k < Sh::NK; ++k) {
    a.ks[k] = RC<T>{};
    a.ks[k].flt = -1;
  }
  for (size_t i = 0; i < c->res.size(); ++i) {
    const kpsi_resonance& r = c->res[i];
    const double M = par[ncr + 2 * i], G = par[ncr + 2 * i + 1];
    LsConst lc = lineshape_consts(c->kin, r, M, G);
    const double* p = par + c->coff[i];
    double hr[3], hi[3];
    int nl;
    if (r.chain == 0) {
      if (r.spin == 0) {   // only lambda = 0, stored in the middle slot
        hr[0] = hi[0] = hr[2] = hi[2] = 0.0;
        hr[1] = p[0] * std::cos(p[1]); hi[1] = p[0] * std::sin(p[1]);
      } else {
        for (int l = 0; l < 3; ++l) { hr[l] = p[2 * l] * std::cos(p[2 * l + 1]); hi[l] = p[2 * l] * std::sin(p[2 * l + 1]); }
      }
      nl = 3;
      fill_rc(a.ks[c->slot[i]], lc, hr, hi, nl, c->fslot[i]);
      if (r.shape == 1) {
        RC<T>& rc = a.ks[c->slot[i]];
        rc.lass = 1;
        rc.lai = (T)(1.0 / r.lass_a);
        rc.lhb = (T)(0.5 * r.lass_b);
      }
    } else {
      // lambda' = 0, +1 (standing for +-1 through Eq. 11), and -1 when the helicities are free
      nl = ncoup(r);
      for (int l = 0; l < nl; ++l) { hr[l] = p[2 * l] * std::cos(p[2 * l + 1]); hi[l] = p[2 * l] * std::sin(p[2 * l + 1]); }
      fill_rc(a.zs[c->slot[i]], lc, hr, hi, nl, c->fslot[i]);
    }
  }
  a.zfree = c->zfree ? 1 : 0;
  for (int j = 0; j < 6; ++j) a.cnt[j] = c->cnt[j];
  a.rR = (T)c->kin.r_r;
  a.rB = (T)c->kin.r_b;
  a.invMB = (T)(1.0 / c->kin.m_b);
}

// Accumulator offset of the couplings of table resonance i inside the block record.
int acc_offset(const kpsi_ctx* c, size_t i, const int* N) {
  const kpsi_resonance& r = c->res[i];
  int nkacc = 0;
  for (int j = 0; j < 5; ++j) nkacc += N[j] * (j == 0 ? 2 : 6);
  if (r.chain == 1) return 3 + nkacc + 4 * c->slot[i];
  int off = 3, base = 0;
  for (int j = 0; j < r.spin; ++j) { off += N[j] * (j == 0 ? 2 : 6); base += N[j]; }
  return off + (c->slot[i] - base) * (r.spin == 0 ? 2 : 6);
}

int shape_counts(int shape, int* N, int* NZ) {
  if (shape == 0) { int n[5] = {0, 1, 0, 0, 0}; for (int j = 0; j < 5; ++j) N[j] = n[j]; *NZ = 0; }
  else { int n[5] = {3, 3, 2, 1, 1}; for (int j = 0; j < 5; ++j) N[j] = n[j]; *NZ = 2; }
  return 0;
}

kpsi_status ensure_partial(kpsi_ctx* c, size_t nblocks) {
  const size_t need = nblocks * NACC;
  if (need <= c->partial_cap) return KPSI_OK;
  if (c->partial) hipFree(c->partial);
  c->partial = nullptr;
  c->partial_cap = 0;
  if (hipMalloc(&c->partial, need * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "partial buffer");
  c->partial_cap = need;
  return KPSI_OK;
}

// Events per thread of the per-event kernel.  The grid is sized to one resident round: the
// smallest ept whose data and normalisation blocks together fit in the blocks the device can
// hold at once (compute units x resident blocks per unit for this kernel).  A grid slightly
// larger than that would run a nearly empty second round; a much larger one pays the
// per-thread reduction tail more often.  Capped at 64 (then the grid runs several full rounds).
template <typename T, class Sh>
int pick_ept(kpsi_ctx* c, int mode, int64_t nd, int64_t nm) {
  if (c->ept_override > 0) return c->ept_override;
  const bool cc = c->cc_on && mode != MODE_DENSITY;
  int& bpc = c->blocks_per_cu[c->shape][mode][(cc ? 1 : 0) + (c->zfree ? 2 : 0)];
  if (bpc < 0) bpc = amp_blocks_per_cu<T, Sh>(mode, cc, c->zfree);
  const int64_t cap = (int64_t)(c->n_cu > 0 ? c->n_cu : 256) * (bpc > 0 ? bpc : 3);
  auto blocks = [&](int64_t ept) {
    const int64_t ch = (int64_t)BLOCK * ept;
    return (nd + ch - 1) / ch + (nm + ch - 1) / ch;
  };
  int64_t ept = (nd + nm + (int64_t)BLOCK * cap - 1) / ((int64_t)BLOCK * cap);
  if (ept < 1) ept = 1;
  while (ept < 64 && blocks(ept) > cap) ++ept;
  return (int)(ept > 64 ? 64 : ept);
}

kpsi_status derive_columns(kpsi_ctx* c, int s) {
  DevSet& d = c->set[s];
  if (d.n == 0 || !c->has_model) return KPSI_OK;
  const int ncol = NCOL_KSTAR + (c->has_z ? NCOL_Z : 0) + (c->zfree ? NCOL_ZFREE : 0);
  const int64_t ld = (d.n + 63) / 64 * 64;
  const size_t bytes = (size_t)ld * col_groups(ncol) * 4 * tsize(c);
  if (bytes > d.cols_cap) {
    if (d.cols) hipFree(d.cols);
    d.cols = nullptr;
    d.cols_cap = 0;
    if (hipMalloc(&d.cols, bytes) != hipSuccess) return fail(c, KPSI_E_OOM, "event columns (%zu bytes)", bytes);
    d.cols_cap = bytes;
  }
  d.ld = ld;
  auto go = [&](auto tag) -> hipError_t {
    using T = decltype(tag);
    InvArgs<T> a{};
    for (int j = 0; j < 4; ++j) a.obs[j] = d.obs[j];
    a.cols = (T*)d.cols;
    a.ld = ld;
    a.n = d.n;
    a.mB = c->kin.m_b; a.mJ = c->kin.m_jpsi; a.mK = c->kin.m_k; a.mPi = c->kin.m_pi;
    a.rB = c->kin.r_b; a.rR = c->kin.r_r;
    a.with_z = c->has_z ? 1 : 0;
    a.zfree = c->zfree ? 1 : 0;
    a.diag = nullptr;
    return launch_invariants<T>(a, c->stream);
  };
  hipError_t e = c->prec == KPSI_FP32 ? go(float{}) : go(double{});
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "invariants kernel: %s", hipGetErrorString(e));
  return KPSI_OK;
}

__global__ void validate_kernel(const double* m, const double* ck, const double* cj, const double* ph, int64_t n,
                                double lo, double hi, unsigned int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double tol = 1e-12;
  const bool ok = (m[i] >= lo - tol) && (m[i] <= hi + tol) && (fabs(ck[i]) <= 1.0 + tol) &&
                  (fabs(cj[i]) <= 1.0 + tol) && (fabs(ph[i]) <= 3.14159265358979323846 + tol);
  if (!ok) atomicOr(bad, 1u);
}

template <typename T> __global__ void to_t_kernel(const double* in, T* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}
// out = a * b elementwise (a or b null: 1), as T
template <typename T> __global__ void prod_t_kernel(const double* a, const double* b, T* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)((a ? a[i] : 1.0) * (b ? b[i] : 1.0));
}

// A T column a * b over the normalisation set (either factor may be null), replacing *col.
kpsi_status product_column(kpsi_ctx* c, const double* a, const double* b, void** col) {
  const int64_t n = c->set[1].n;
  void* e = nullptr;
  if (hipMalloc(&e, (size_t)n * tsize(c)) != hipSuccess) return fail(c, KPSI_E_OOM, "per-event column");
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (c->prec == KPSI_FP32) hipLaunchKernelGGL(prod_t_kernel<float>, dim3(nb), dim3(256), 0, c->stream, a, b, (float*)e, n);
  else hipLaunchKernelGGL(prod_t_kernel<double>, dim3(nb), dim3(256), 0, c->stream, a, b, (double*)e, n);
  hipError_t er = hipStreamSynchronize(c->stream);
  if (er != hipSuccess) { hipFree(e); return fail(c, KPSI_E_HIP, "column product: %s", hipGetErrorString(er)); }
  if (*col) hipFree(*col);
  *col = e;
  return KPSI_OK;
}

kpsi_status validate(kpsi_ctx* c, int64_t n, const double* const* obs) {
  if (n == 0) return KPSI_OK;
  unsigned int* bad = nullptr;
  HIPCHECK(c, hipMalloc(&bad, sizeof(unsigned int)));
  hipMemsetAsync(bad, 0, sizeof(unsigned int), c->stream);
  const double lo = c->kin.m_k + c->kin.m_pi, hi = c->kin.m_b - c->kin.m_jpsi;
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, obs[0], obs[1],
                     obs[2], obs[3], n, lo, hi, bad);
  unsigned int h = 0;
  hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, c->stream);
  hipError_t e = hipStreamSynchronize(c->stream);
  hipFree(bad);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "validation: %s", hipGetErrorString(e));
  if (h) return fail(c, KPSI_E_ARG, "event outside the physical region (m in [%.6f, %.6f], |cos| <= 1, |phi| <= pi)",
                     lo, hi);
  return KPSI_OK;
}

// ---------------------------------------------------------------- interference-matrix cache
void invalidate_cache(kpsi_ctx* c) { c->cache_valid = false; c->last_ls.clear(); c->ls_streak = 0; }

// Complex components in accumulator order: K* slots by spin (1 or 3 each), then Z slots (2; a
// single Z with free helicities uses 3, the third in the second slot's first position).
int n_components(int shape) {
  int N[5], NZ;
  shape_counts(shape, N, &NZ);
  int n = 0;
  for (int j = 0; j < 5; ++j) n += N[j] * (j == 0 ? 1 : 3);
  return n + 2 * NZ;
}
// First component and component count of table resonance i.
void components_of(const kpsi_ctx* c, size_t i, int* first, int* count) {
  int N[5], NZ;
  shape_counts(c->shape, N, &NZ);
  const kpsi_resonance& r = c->res[i];
  if (r.chain == 1) {
    int nk = 0;
    for (int j = 0; j < 5; ++j) nk += N[j] * (j == 0 ? 1 : 3);
    *first = nk + 2 * c->slot[i];
    *count = ncoup(r);   // 2, or 3 with free helicities (one Z: the third takes the next slot's first)
    return;
  }
  int base = 0, slot0 = 0;
  for (int j = 0; j < r.spin; ++j) { base += N[j] * (j == 0 ? 1 : 3); slot0 += N[j]; }
  *first = base + (c->slot[i] - slot0) * (r.spin == 0 ? 1 : 3);
  *count = r.spin == 0 ? 1 : 3;
}
// Complex couplings in component order.
std::vector<double> component_couplings(const kpsi_ctx* c, const double* par) {
  std::vector<double> cv(2 * n_components(c->shape), 0.0);
  for (size_t i = 0; i < c->res.size(); ++i) {
    int k0, nk;
    components_of(c, i, &k0, &nk);
    const double* p = par + c->coff[i];
    for (int l = 0; l < nk; ++l) {
      cv[2 * (k0 + l)] = p[2 * l] * std::cos(p[2 * l + 1]);
      cv[2 * (k0 + l) + 1] = p[2 * l] * std::sin(p[2 * l + 1]);
    }
  }
  return cv;
}
std::vector<double> lineshape_params(const kpsi_ctx* c, const double* par) {
  const int ncr = c->nparams - 2 * (int)c->res.size();
  return std::vector<double>(par + ncr, par + c->nparams);
}

// Gram build over the normalisation set at the lineshape point of par: the complex
// component matrix I (ncomp x ncomp) and, when with_deriv, the lineshape-derivative rows D
// (nderiv x ncomp) with dcol[] the first derivative component of each floating slot.
// with_eps weights each event by the context's efficiency column.
struct Gram {
  int ncomp = 0, nderiv = 0;
  int dcol[NFL] = {0, 0};
  std::vector<double> I, D;
  float ms = 0.f;
};
template <typename T, class Sh>
kpsi_status gram_build_t(kpsi_ctx* c, const double* par, bool with_eps, bool with_deriv, Gram& g) {
  const DevSet& d = c->set[1];
  const int ncomp = n_components(c->shape);
  int nderiv = 0;
  int dcol[NFL] = {0, 0};
  if (with_deriv) {
    for (size_t i = 0; i < c->res.size(); ++i) {
      if (c->fslot[i] < 0) continue;
      int k0, nk;
      components_of(c, i, &k0, &nk);
      dcol[c->fslot[i]] = ncomp + nderiv;
      nderiv += 2 * nk;
    }
  }
  const int ncx = ncomp + nderiv;
  const int ncols = 2 * ncx;
  const int C = ncols <= 16 ? 16 : ncols <= 32 ? 32 : ncols <= 64 ? 64 : ncols <= 80 ? 80 : 0;
  if (!C) return fail(c, KPSI_E_UNSUPPORTED, "interference matrix of %d columns exceeds the compiled 80", ncols);
  const int NT = C / 16, NTILE = NT * (NT + 1) / 2, nv = NTILE * 256;
  const int64_t ntiles = (d.n + 31) / 32;
  // one resident round of one-wavefront blocks (their LDS rows limit them per compute unit)
  const int bpc = imatrix_blocks_per_cu<T, Sh>(ncols);
  const int64_t cap = (int64_t)(c->n_cu > 0 ? c->n_cu : 256) * (bpc > 0 ? bpc : 4);
  const int nb = (int)std::min<int64_t>(ntiles, cap);
  const size_t need = (size_t)nv * nb;
  if (need > c->cache_partial_cap) {
    if (c->cache_partial) hipFree(c->cache_partial);
    c->cache_partial = nullptr;
    c->cache_partial_cap = 0;
    if (hipMalloc(&c->cache_partial, need * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "cache partials");
    c->cache_partial_cap = need;
  }
  if ((size_t)nv > c->cache_out_cap) {
    if (c->cache_out) hipFree(c->cache_out);
    c->cache_out = nullptr;
    c->cache_out_cap = 0;
    if (hipMalloc(&c->cache_out, nv * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "cache output");
    c->cache_out_cap = nv;
  }
  AmpArgs<T, Sh> pa{};
  pack<T, Sh>(c, par, pa);
  ImArgs<T, Sh> a{};
  a.cols = (const T*)d.cols;
  a.ld = d.ld;
  a.n = d.n;
  a.eps = with_eps ? (const T*)c->eps : (const T*)c->wcol;   // wcol: importance weights or null
  a.partial = c->cache_partial;
  a.ncols = ncols;
  a.zfree = c->zfree ? 1 : 0;
  a.skip_last = (NT > 1 && 16 * (NT - 1) >= 2 * ncomp) ? 1 : 0;
  for (int j = 0; j < 6; ++j) a.cnt[j] = pa.cnt[j];
  for (int f = 0; f < NFL; ++f) a.dcol[f] = dcol[f];
  a.rR = pa.rR; a.rB = pa.rB; a.invMB = pa.invMB;
  for (int k = 0; k < (Sh::NK > 0 ? Sh::NK : 1); ++k) a.ks[k] = pa.ks[k];
  for (int k = 0; k < (Sh::NZ > 0 ? Sh::NZ : 1); ++k) {
    a.zs[k] = pa.zs[k];
  }
  if (!with_deriv) {   // no derivative columns: every lineshape counts as fixed in this matrix
    for (int k = 0; k < (Sh::NK > 0 ? Sh::NK : 1); ++k) a.ks[k].flt = -1;
    for (int k = 0; k < (Sh::NZ > 0 ? Sh::NZ : 1); ++k) a.zs[k].flt = -1;
  }
  hipEvent_t e0 = c->ev0, e1 = c->ev1;
  hipEventRecord(e0, c->stream);
  hipError_t e = launch_imatrix<T, Sh>(a, ncols, nb, c->cache_out, c->stream);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "interference matrix: %s", hipGetErrorString(e));
  hipEventRecord(e1, c->stream);
  std::vector<double> out(nv);
  HIPCHECK(c, hipMemcpyAsync(out.data(), c->cache_out, nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  g.ms = 0.f;
  hipEventElapsedTime(&g.ms, e0, e1);
  // real Gram matrix G from its upper 16x16 tiles.  The FP64 16x16x4 MFMA accumulator (FP64
  // context) holds, in lane l and register r, row l/16 + 4 r and column l % 16 of the tile (rows
  // interleaved across the four registers); the FP32 16x16x4 form (FP32 context) holds row
  // 4 (l/16) + r, column l % 16
  std::vector<double> G((size_t)C * C, 0.0);
  int t = 0;
  for (int ti = 0; ti < NT; ++ti)
    for (int tj = ti; tj < NT; ++tj, ++t)
      for (int lane = 0; lane < 64; ++lane)
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * ti + (std::is_same<T, float>::value ? 4 * (lane / 16) + r : lane / 16 + 4 * r);
          const int col = 16 * tj + lane % 16;
          const double v = out[((size_t)t * 64 + lane) * 4 + r];
          G[(size_t)row * C + col] = v;
          G[(size_t)col * C + row] = v;
        }
  // complex blocks: sum B_k conj(B_l) = (G[2k][2l] + G[2k+1][2l+1]) + i (G[2k+1][2l] - G[2k][2l+1])
  auto cre = [&](int k, int l) { return G[(size_t)(2 * k) * C + 2 * l] + G[(size_t)(2 * k + 1) * C + 2 * l + 1]; };
  auto cim = [&](int k, int l) { return G[(size_t)(2 * k + 1) * C + 2 * l] - G[(size_t)(2 * k) * C + 2 * l + 1]; };
  g.I.assign(2 * (size_t)ncomp * ncomp, 0.0);
  for (int k = 0; k < ncomp; ++k)
    for (int l = 0; l < ncomp; ++l) {
      g.I[2 * ((size_t)k * ncomp + l)] = cre(k, l);
      g.I[2 * ((size_t)k * ncomp + l) + 1] = cim(k, l);
    }
  g.D.assign(2 * (size_t)nderiv * ncomp, 0.0);
  for (int dd = 0; dd < nderiv; ++dd)
    for (int l = 0; l < ncomp; ++l) {
      g.D[2 * ((size_t)dd * ncomp + l)] = cre(ncomp + dd, l);
      g.D[2 * ((size_t)dd * ncomp + l) + 1] = cim(ncomp + dd, l);
    }
  g.ncomp = ncomp;
  g.nderiv = nderiv;
  for (int f = 0; f < NFL; ++f) g.dcol[f] = dcol[f];
  return KPSI_OK;
}

kpsi_status gram_build(kpsi_ctx* c, const double* par, bool with_eps, bool with_deriv, Gram& g) {
  if (c->prec == KPSI_FP32)
    return c->shape == 0 ? gram_build_t<float, ShapeSmall>(c, par, with_eps, with_deriv, g)
                         : gram_build_t<float, ShapeFull>(c, par, with_eps, with_deriv, g);
  return c->shape == 0 ? gram_build_t<double, ShapeSmall>(c, par, with_eps, with_deriv, g)
                       : gram_build_t<double, ShapeFull>(c, par, with_eps, with_deriv, g);
}

kpsi_status build_cache(kpsi_ctx* c, const double* par) {
  Gram g;
  kpsi_status st = gram_build(c, par, true, true, g);
  if (st) return st;
  c->cache_build_ms = g.ms;
  c->cache_I = std::move(g.I);
  c->cache_D = std::move(g.D);
  c->cache_ncomp = g.ncomp;
  c->cache_ncols = g.ncomp + g.nderiv;
  for (int f = 0; f < NFL; ++f) c->cache_dcol[f] = g.dcol[f];
  c->cache_ls = lineshape_params(c, par);
  c->cache_valid = true;
  c->cache_builds++;
  return KPSI_OK;
}


// Normalisation record (what the per-event kernel accumulates over the normalisation set)
// from the cached matrices: sum eps S = c^T I conj(c), coupling sensitivities (I conj(c))_k,
// and Re sum_{k in R} c_k (D^p conj(c))_k for the floating lineshapes.
void cached_norm_record(const kpsi_ctx* c, const double* par, double* rm) {
  const int n = c->cache_ncomp;
  const std::vector<double> cv = component_couplings(c, par);
  for (int v = 0; v < NACC; ++v) rm[v] = 0.0;
  double smr = 0.0;
  for (int k = 0; k < n; ++k) {
    double gr = 0.0, gi = 0.0;   // (I conj(c))_k
    for (int l = 0; l < n; ++l) {
      const double ir = c->cache_I[2 * ((size_t)k * n + l)], ii = c->cache_I[2 * ((size_t)k * n + l) + 1];
      const double cr = cv[2 * l], ci = -cv[2 * l + 1];
      gr += ir * cr - ii * ci;
      gi += ir * ci + ii * cr;
    }
    rm[3 + 2 * k] = gr;
    rm[3 + 2 * k + 1] = gi;
    smr += cv[2 * k] * gr - cv[2 * k + 1] * gi;   // Re(c_k g_k)
  }
  rm[0] = smr;
  int N[5], NZ;
  shape_counts(c->shape, N, &NZ);
  int nkacc = 0;
  for (int j = 0; j < 5; ++j) nkacc += N[j] * (j == 0 ? 2 : 6);
  for (size_t i = 0; i < c->res.size(); ++i) {
    const int f = c->fslot[i];
    if (f < 0) continue;
    int k0, nk;
    components_of(c, i, &k0, &nk);
    for (int p = 0; p < 2; ++p) {
      double val = 0.0;
      for (int q = 0; q < nk; ++q) {
        const int dd = c->cache_dcol[f] - n + p * nk + q;
        double gr = 0.0, gi = 0.0;
        for (int l = 0; l < n; ++l) {
          const double dr = c->cache_D[2 * ((size_t)dd * n + l)], di = c->cache_D[2 * ((size_t)dd * n + l) + 1];
          const double cr = cv[2 * l], ci = -cv[2 * l + 1];
          gr += dr * cr - di * ci;
          gi += dr * ci + di * cr;
        }
        const double ckr = cv[2 * (k0 + q)], cki = cv[2 * (k0 + q) + 1];
        val += ckr * gr - cki * gi;
      }
      rm[3 + nkacc + 4 * NZ + 2 * f + p] = val;
    }
  }
}

// Decide whether this call uses the cache (building it when the policy says so).
kpsi_status use_cache(kpsi_ctx* c, const double* par, bool* use) {
  *use = false;
  if (c->cache_mode == 0) return KPSI_OK;
  const std::vector<double> ls = lineshape_params(c, par);
  if (c->cache_valid && ls == c->cache_ls) { *use = true; c->cache_hits++; return KPSI_OK; }
  if (ls == c->last_ls) {
    ++c->ls_streak;
  } else {
    c->last_ls = ls;
    c->ls_streak = 1;
  }
  const bool build = c->cache_mode == 1 || (c->cache_mode == 2 && c->ls_streak >= KPSI_CACHE_AUTO_STREAK);
  if (!build) return KPSI_OK;
  kpsi_status st = build_cache(c, par);
  if (st) return st;
  *use = true;
  return KPSI_OK;
}

// Normalisation record from the interference matrix into the host record; with the Eq. 14
// mixture also into the device copy that the data pass reads.
//
// With flavour tags the second record is the normalisation at -phi.  Reversing phi of an event
// gives the density of the original event with the lambda = -1 and lambda = +1 couplings of
// every K* of spin >= 1 exchanged (the d^1_{lambda xi} symmetry takes e^{-i lambda phi} to the
// opposite helicities; the Z-chain terms of the two xi swap, with a common sign: the Z angular
// factors conjugate, Zang[l'][xi] -> -Zang[-l'][-xi], which leaves Eq. 11 couplings as they are
// and exchanges free H'_{+1} and H'_{-1}), so
// I(-phi; H) = I(+phi; H') with H' the exchanged couplings, and the +phi matrix serves both
// records: record 2 is the +phi record at H', its coupling entries mapped back through the
// same exchange (its lineshape-derivative entries need no mapping).
kpsi_status put_cached_record(kpsi_ctx* c, const double* params) {
  cached_norm_record(c, params, c->red_host + NACC);
  if (c->cc_on) {
    std::vector<double> sw(params, params + c->nparams);
    int off = 0;
    for (const kpsi_resonance& r : c->res) {
      if (r.chain == 0 && r.spin > 0) {
        std::swap(sw[off], sw[off + 4]);
        std::swap(sw[off + 1], sw[off + 5]);
      } else if (r.chain == 1 && r.hel_free) {   // lambda' = +1 and -1 (order 0, +1, -1)
        std::swap(sw[off + 2], sw[off + 4]);
        std::swap(sw[off + 3], sw[off + 5]);
      }
      off += 2 * ncoup(r);
    }
    double* r2 = c->red_host + 2 * NACC;
    cached_norm_record(c, sw.data(), r2);
    for (size_t i = 0; i < c->res.size(); ++i) {
      const kpsi_resonance& r = c->res[i];
      const bool kst = r.chain == 0 && r.spin > 0, zf = r.chain == 1 && r.hel_free;
      if (!kst && !zf) continue;
      int k0, nk;
      components_of(c, i, &k0, &nk);
      const int ka = kst ? k0 : k0 + 1;   // the exchanged components: k0 + {0, 2} or k0 + {1, 2}
      std::swap(r2[3 + 2 * ka], r2[3 + 2 * (k0 + 2)]);
      std::swap(r2[3 + 2 * ka + 1], r2[3 + 2 * (k0 + 2) + 1]);
    }
  }
  if (c->bkg_on) {
    HIPCHECK(c, hipMemcpyAsync(c->red_dev + NACC, c->red_host + NACC, 2 * sizeof(double), hipMemcpyHostToDevice,
                               c->stream));
    if (c->cc_on)
      HIPCHECK(c, hipMemcpyAsync(c->red_dev + 2 * NACC, c->red_host + 2 * NACC, 2 * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
  }
  return KPSI_OK;
}

// Read the recorded event pairs of timed calls (each waits on its end event first: the runtime
// can mark an event complete after the call that recorded it has seen its results).
static void drain_timing(kpsi_ctx* c) {
  for (int i = 0; i < c->t_pend; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(c->tev[2 * i + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, c->tev[2 * i], c->tev[2 * i + 1]) == hipSuccess) {
      c->t_ms += ms;
      c->t_n += 1;
      if (c->t_samples.size() < kTimingSamples) c->t_samples.push_back(ms);
    } else {
      c->t_dropped += 1;
    }
  }
  c->t_pend = 0;
}

// ---------------------------------------------------------------- per-call driver
// Bit pattern of a result value not yet written: a NaN payload that no arithmetic produces
// (operations on NaN inputs return them with their payload, and the inputs here are computed).
constexpr uint64_t kPending = 0x7ff4c0de5e9d0001ull;

static uint64_t* result_word(kpsi_ctx* c, int k) { return reinterpret_cast<uint64_t*>(c->red_host) + k; }

// Mark the values the final reduction of this call will write: sets [first, first + nsets) of
// nv values each.  Called before the reduction is enqueued; the previous call's reduction has
// written all its values by then (its wait saw them), so nothing else writes these words.
static void mark_pending(kpsi_ctx* c, int first, int nsets, int nv) {
  for (int s = first; s < first + nsets; ++s)
    for (int v = 0; v < nv; ++v) __atomic_store_n(result_word(c, s * NACC + v), kPending, __ATOMIC_RELAXED);
}

// Wait for a call: the final reduction's blocks each store one value into the fine-grained
// mapped result buffer, and the call is complete when every marked value has been replaced.
// Each is one aligned 8-byte store, read here as one 8-byte load, so a value is either pending
// or whole.  The poll is bounded (50 ms; a long call or a faulted kernel): past it the stream
// is synchronized, which also reports any error of the call's kernels.
kpsi_status wait_results(kpsi_ctx* c, int first, int nsets, int nv) {
  const auto t0 = std::chrono::steady_clock::now();
  int s = first, v = 0;
  for (unsigned k = 1;; ++k) {
    while (s < first + nsets && __atomic_load_n(result_word(c, s * NACC + v), __ATOMIC_ACQUIRE) != kPending) {
      if (++v == nv) {
        v = 0;
        ++s;
      }
    }
    if (s == first + nsets) {
      // a launch error of this call's kernels (their asynchronous faults stop the stream, so the
      // values never arrive and the synchronisation below reports them)
      const hipError_t le = hipGetLastError();
      if (le != hipSuccess) return fail(c, KPSI_E_HIP, "kernel launch: %s", hipGetErrorString(le));
      return KPSI_OK;
    }
    if ((k & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) break;
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return KPSI_OK;
}

// `fixed` (may be null): a caller-provided block-partial buffer of `fixed_cap` doubles used in place
// of the context's own (which may grow by allocation); calls that would need more fail.
template <typename T, class Sh>
kpsi_status run_amp(kpsi_ctx* c, int mode, const double* par, int which /*-1: both*/, double** dens_out,
                    double* fixed, size_t fixed_cap) {
  AmpArgs<T, Sh> a{};
  for (int s = 0; s < 2; ++s) {
    a.cols[s] = (const T*)c->set[s].cols;
    a.ld[s] = c->set[s].ld;
    a.n[s] = c->set[s].n;
    a.s_out[s] = dens_out ? dens_out[s] : nullptr;
  }
  a.eps = (const T*)c->eps;
  pack<T, Sh>(c, par, a);
  const int nv = mode == MODE_GRAD ? NACC : 3;
  const bool mix = c->bkg_on && mode != MODE_DENSITY;
  if (mix) {
    a.eps_data = (const T*)c->eps_data;
    a.bkg_data = (const T*)c->bkg_data;
    a.norm_total = c->red_dev + NACC;
    a.bkg_coef = c->bkg_coef;
    a.purity = (T)c->purity;
  }
  c->timing = !fixed && c->bench_reps == 0 && mode != MODE_DENSITY && c->timing_every > 0 &&
              (c->timing_calls++ % c->timing_every) == 0;
  if (c->timing) {
    if (c->t_pend == kTimingPairs) drain_timing(c);
    hipEventRecord(c->tev[2 * c->t_pend], c->stream);
  }
  // Launches over the events of [nd data, nm normalisation] write block partials (rows of
  // nbd + nbm blocks, data first); one reduction then writes the record of each set covered
  // (by the GPU straight into mapped pinned host memory).
  const int64_t nd = (which == 1) ? 0 : c->set[0].n, nm = (which == 0) ? 0 : c->set[1].n;
  // flavour tags: the normalisation events run twice (records 1 and 2: phi and -phi)
  const bool cc = c->cc_on && mode != MODE_DENSITY;
  const int nmsets = cc ? 2 : 1;
  if (cc) {
    a.tag = (const T*)c->tag;
    a.mistag = (T)c->mistag;
    a.keep = (T)(1.0 - c->mistag);
  }
  int chunk_d, chunk_m;
  if (!mix) {
    chunk_d = chunk_m = BLOCK * pick_ept<T, Sh>(c, mode, nd, nmsets * nm);
  } else {
    // Eq. 14: the data terms need the normalisation total, so the normalisation events run in
    // a launch of their own first, and the data launch sums their block partials (unless the
    // normalisation record comes from the interference matrix and is already in red_dev)
    chunk_m = BLOCK * pick_ept<T, Sh>(c, mode, 0, nmsets * nm);
    chunk_d = BLOCK * pick_ept<T, Sh>(c, mode, nd, 0);
  }
  const int nbd = (int)((nd + chunk_d - 1) / chunk_d), nbm = (int)((nm + chunk_m - 1) / chunk_m);
  double* part = c->partial;
  if (mode != MODE_DENSITY) {
    const size_t rows = (size_t)(nbd + nmsets * nbm);
    if (fixed) {
      if (rows * NACC > fixed_cap)
        return fail(c, KPSI_E_ARG, "%zu block partials of %d doubles exceed the static scratch of %zu doubles "
                    "(at most %zu blocks)", rows, NACC, fixed_cap, fixed_cap / NACC);
      part = fixed;
    } else {
      kpsi_status st = ensure_partial(c, rows);
      if (st) return st;
      part = c->partial;
    }
  }
  a.partial = part;
  a.pstride = nbd + nmsets * nbm;
  a.nb_mc = nbm;
  auto launch = [&](const AmpArgs<T, Sh>& b, int nblocks) -> kpsi_status {
    hipError_t e = launch_amp<T, Sh>(b, mode, nblocks, c->stream);
    if (e != hipSuccess) return fail(c, KPSI_E_HIP, "amplitude kernel: %s", hipGetErrorString(e));
    return KPSI_OK;
  };
  kpsi_status st = KPSI_OK;
  // kpsi_time_kernel: the per-event launches repeated back to back between one pair of events
  const int reps = (c->bench_reps > 0 && mode != MODE_DENSITY) ? c->bench_reps : 1;
  if (reps > 1 || c->bench_reps > 0) hipEventRecord(c->ev0, c->stream);
  for (int rep = 0; rep < reps && !st; ++rep) {
  if (!mix) {
    AmpArgs<T, Sh> b = a;
    b.chunk = chunk_d;
    b.nb_data = nbd;
    b.poff = 0;
    st = launch(b, nbd + nmsets * nbm);
  } else {
    if (nm > 0) {
      AmpArgs<T, Sh> b = a;
      b.chunk = chunk_m;
      b.nb_data = 0;
      b.poff = nbd;
      st = launch(b, nmsets * nbm);   // with tags: records 1 (phi) and 2 (-phi)
    }
    if (!st && nd > 0) {
      AmpArgs<T, Sh> b = a;
      b.chunk = chunk_d;
      b.nb_data = nbd;
      b.poff = 0;
      if (nm > 0) {
        b.mc_part = part + nbd;
        b.mc_nb = nbm;
      }
      st = launch(b, nbd);
    }
  }
  }
  if (st) return st;
  // end of the per-event work
  if (c->bench_reps > 0) hipEventRecord(c->ev1, c->stream);
  else if (c->timing) hipEventRecord(c->tev[2 * c->t_pend + 1], c->stream);
  if (mode == MODE_DENSITY) return KPSI_OK;
  const int first_set = nd > 0 ? 0 : 1, nsets = (nd > 0) + (nm > 0) * nmsets;
  mark_pending(c, first_set, nsets, nv);
  hipError_t e = launch_reduce_final(part, nbd, nbm, nmsets, nv, c->red, first_set, nsets, c->stream);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "reduction kernel: %s", hipGetErrorString(e));
  if (kpsi_status ws = wait_results(c, first_set, nsets, nv)) return ws;
  if (c->bench_reps > 0) {
    float ms = 0.f;
    if (hipEventSynchronize(c->ev1) != hipSuccess || hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess)
      return fail(c, KPSI_E_HIP, "kernel timing events");
    c->bench_ms = (double)ms / reps;
    return KPSI_OK;
  }
  if (c->timing) ++c->t_pend;   // read later (drain_timing)
  return KPSI_OK;
}

kpsi_status dispatch(kpsi_ctx* c, int mode, const double* par, int which, double** dens, double* fixed = nullptr,
                     size_t fixed_cap = 0) {
  if (c->prec == KPSI_FP32) {
    return c->shape == 0 ? run_amp<float, ShapeSmall>(c, mode, par, which, dens, fixed, fixed_cap)
                         : run_amp<float, ShapeFull>(c, mode, par, which, dens, fixed, fixed_cap);
  }
  return c->shape == 0 ? run_amp<double, ShapeSmall>(c, mode, par, which, dens, fixed, fixed_cap)
                       : run_amp<double, ShapeFull>(c, mode, par, which, dens, fixed, fixed_cap);
}

kpsi_status check_ready(kpsi_ctx* c, const double* params) {
  if (!c) return KPSI_E_ARG;
  if (!params) return fail(c, KPSI_E_ARG, "params is NULL");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  if (c->set[0].n <= 0) return fail(c, KPSI_E_STATE, "no data events loaded");
  if (c->set[1].n <= 0) return fail(c, KPSI_E_STATE, "no normalisation events loaded");
  for (int i = 0; i < c->nparams; ++i)
    if (!std::isfinite(params[i])) return fail(c, KPSI_E_ARG, "parameter %d is not finite", i);
  const int ncr = c->nparams - 2 * (int)c->res.size();
  for (size_t i = 0; i < c->res.size(); ++i) {
    const double M = params[ncr + 2 * i], G = params[ncr + 2 * i + 1];
    const kpsi_resonance& r = c->res[i];
    const double thr = r.chain == 0 ? c->kin.m_k + c->kin.m_pi : c->kin.m_jpsi + c->kin.m_pi;
    const double top = r.chain == 0 ? c->kin.m_b - c->kin.m_jpsi : c->kin.m_b - c->kin.m_k;
    if (!(M > thr) || !(M < top)) return fail(c, KPSI_E_ARG, "mass of resonance %zu outside (%.5f, %.5f)", i, thr, top);
    if (!(G > 0.0)) return fail(c, KPSI_E_ARG, "width of resonance %zu not positive", i);
  }
  return KPSI_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

kpsi_status kpsi_create(int device, void* stream, kpsi_precision prec, kpsi_ctx** out) {
  if (!out) return fail(nullptr, KPSI_E_ARG, "out is NULL");
  *out = nullptr;
  if (prec != KPSI_FP64 && prec != KPSI_FP32) return fail(nullptr, KPSI_E_ARG, "unknown precision %d", (int)prec);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(nullptr, KPSI_E_HIP, "no HIP device");
  if (device < 0 || device >= ndev) return fail(nullptr, KPSI_E_ARG, "device %d out of range", device);
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, KPSI_E_HIP, "hipSetDevice failed");
  lookup_scratch(device);
  kpsi_ctx* c = new kpsi_ctx();
  c->device = device;
  c->prec = prec;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) c->n_cu = 0;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(nullptr, KPSI_E_HIP, "stream creation failed");
    }
    c->own_stream = true;
  }
  // fine-grained where the system has it (each value is seen as the reduction stores it);
  // otherwise the values appear when the reduction kernel ends, and the poll still works
  if (hipHostMalloc(&c->red_host, 3 * NACC * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    (void)hipGetLastError();
    c->red_host = nullptr;
    if (hipHostMalloc(&c->red_host, 3 * NACC * sizeof(double), hipHostMallocMapped) != hipSuccess) c->red_host = nullptr;
  }
  if (!c->red_host || hipHostGetDevicePointer((void**)&c->red, c->red_host, 0) != hipSuccess ||
      hipMalloc(&c->red_dev, 3 * NACC * sizeof(double)) != hipSuccess) {
    kpsi_destroy(c);
    return fail(nullptr, KPSI_E_OOM, "result buffers");
  }
  hipEventCreate(&c->ev0);
  hipEventCreate(&c->ev1);
  *out = c;
  return KPSI_OK;
}

kpsi_status kpsi_destroy(kpsi_ctx* c) {
  if (!c) return KPSI_E_ARG;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  for (int s = 0; s < 2; ++s) {
    if (c->set[s].owned) hipFree(c->set[s].owned);
    if (c->set[s].cols) hipFree(c->set[s].cols);
  }
  if (c->eps) hipFree(c->eps);
  if (c->mlp_w2h) hipFree(c->mlp_w2h);
  if (c->eps_f64) hipFree(c->eps_f64);
  if (c->norm_w) hipFree(c->norm_w);
  if (c->wcol) hipFree(c->wcol);
  if (c->partial) hipFree(c->partial);
  if (c->cache_partial) hipFree(c->cache_partial);
  if (c->cache_out) hipFree(c->cache_out);
  if (c->red_host) hipHostFree(c->red_host);
  if (c->red_dev) hipFree(c->red_dev);
  if (c->eps_data) hipFree(c->eps_data);
  if (c->bkg_data) hipFree(c->bkg_data);
  if (c->tag) hipFree(c->tag);
  for (hipEvent_t e : c->tev)
    if (e) hipEventDestroy(e);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  delete c;
  return KPSI_OK;
}

kpsi_status kpsi_set_model(kpsi_ctx* c, const kpsi_kinematics* kin, const kpsi_resonance* res, int n_res) {
  if (!c) return KPSI_E_ARG;
  if (!kin || !res || n_res <= 0) return fail(c, KPSI_E_ARG, "kinematics/resonances missing");
  const kpsi_kinematics& k = *kin;
  if (!(k.m_b > k.m_jpsi + k.m_k + k.m_pi) || !(k.m_k > 0) || !(k.m_pi > 0) || !(k.m_jpsi > 0) || !(k.r_b >= 0) ||
      !(k.r_r >= 0))
    return fail(c, KPSI_E_ARG, "unphysical kinematics");
  int counts[5] = {0, 0, 0, 0, 0}, nz = 0, nfree = 0;
  for (int i = 0; i < n_res; ++i) {
    const kpsi_resonance& r = res[i];
    if (r.hel_free != 0 && r.hel_free != 1) return fail(c, KPSI_E_ARG, "resonance %d: hel_free must be 0 or 1", i);
    if (r.chain == 0 && r.hel_free) return fail(c, KPSI_E_ARG, "resonance %d: hel_free applies to a Z only", i);
    if (r.chain == 0) {
      if (r.spin < 0 || r.spin > 4) return fail(c, KPSI_E_UNSUPPORTED, "K* spin %d not in 0..4", r.spin);
      counts[r.spin]++;
    } else if (r.chain == 1) {
      if (r.spin != 1 || r.parity != 1) return fail(c, KPSI_E_UNSUPPORTED, "only 1+ Z states are supported");
      nz++;
      if (r.hel_free) nfree++;
    } else {
      return fail(c, KPSI_E_ARG, "resonance %d: chain must be 0 or 1", i);
    }
    if ((r.lb >= 0 && r.lb != lowest_lb(r)) || (r.lr >= 0 && r.lr != lowest_lr(r)))
      return fail(c, KPSI_E_UNSUPPORTED, "resonance %d: only the lowest orbital momenta are supported", i);
    if (r.shape == 1) {
      if (r.chain != 0 || r.spin != 0)
        return fail(c, KPSI_E_UNSUPPORTED, "resonance %d: the LASS lineshape is defined for spin-0 K* only", i);
      if (!(r.lass_a > 0) || !std::isfinite(r.lass_a) || !std::isfinite(r.lass_b))
        return fail(c, KPSI_E_ARG, "resonance %d: LASS needs a > 0 and a finite b", i);
    } else if (r.shape != 0) {
      return fail(c, KPSI_E_ARG, "resonance %d: shape must be 0 (Breit-Wigner) or 1 (LASS)", i);
    }
  }
  if (nfree && nz != 1)
    return fail(c, KPSI_E_UNSUPPORTED, "free Z helicity couplings need a model with exactly one Z (it has %d)", nz);
  int shape = -1;
  const int small[5] = {0, 1, 0, 0, 0}, full[5] = {3, 3, 2, 1, 1};
  bool fits_small = nz == 0, fits_full = nz <= 2;
  for (int j = 0; j < 5; ++j) { fits_small &= counts[j] <= small[j]; fits_full &= counts[j] <= full[j]; }
  if (fits_small) shape = 0;
  else if (fits_full) shape = 1;
  else return fail(c, KPSI_E_UNSUPPORTED, "model exceeds the compiled capacity (K* per spin 3,3,2,1,1; 2 Z)");
  c->kin = k;
  c->res.assign(res, res + n_res);
  c->shape = shape;
  c->slot.assign(n_res, 0);
  c->coff.assign(n_res, 0);
  c->fslot.assign(n_res, -1);
  int N[5], NZ;
  shape_counts(shape, N, &NZ);
  int used[5] = {0, 0, 0, 0, 0}, zused = 0, off = 0;
  c->has_z = false;
  c->zfree = nfree > 0;
  for (int i = 0; i < n_res; ++i) {
    const kpsi_resonance& r = res[i];
    c->coff[i] = off;
    off += 2 * ncoup(r);
    if (r.chain == 0) {
      int base = 0;
      for (int j = 0; j < r.spin; ++j) base += N[j];
      c->slot[i] = base + used[r.spin]++;
    } else {
      c->slot[i] = zused++;
      c->has_z = true;
    }
  }
  for (int j = 0; j < 5; ++j) c->cnt[j] = counts[j];
  c->cnt[5] = nz;
  c->nparams = off + 2 * n_res;
  c->con_idx.clear();   // constraint positions refer to the previous parameter vector
  c->con_mean.clear();
  c->con_sigma.clear();
  c->has_model = true;
  invalidate_cache(c);
  hipSetDevice(c->device);
  for (int s = 0; s < 2; ++s) {
    kpsi_status st = derive_columns(c, s);
    if (st) return st;
  }
  return KPSI_OK;
}

kpsi_status kpsi_n_params(const kpsi_ctx* c, int* n) {
  if (!c || !n) return KPSI_E_ARG;
  if (!c->has_model) return KPSI_E_STATE;
  *n = c->nparams;
  return KPSI_OK;
}

kpsi_status kpsi_set_floating(kpsi_ctx* c, const int* flags, int n_res) {
  if (!c) return KPSI_E_ARG;
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  if (n_res != (int)c->res.size()) return fail(c, KPSI_E_ARG, "expected %zu flags", c->res.size());
  int k = 0;
  std::vector<int> fs(n_res, -1);
  for (int i = 0; i < n_res; ++i) {
    if (flags && flags[i]) {
      if (k >= NFL) return fail(c, KPSI_E_UNSUPPORTED, "at most %d floating lineshapes", NFL);
      if (c->res[i].shape == 1)
        return fail(c, KPSI_E_UNSUPPORTED, "resonance %d: a LASS lineshape cannot float", i);
      fs[i] = k++;
    }
  }
  c->fslot = fs;
  invalidate_cache(c);
  return KPSI_OK;
}

static void drop_background(kpsi_ctx* c) {
  if (c->eps_data) hipFree(c->eps_data);
  if (c->bkg_data) hipFree(c->bkg_data);
  c->eps_data = c->bkg_data = nullptr;
  c->bkg_on = false;
}

static void drop_flavour(kpsi_ctx* c) {
  if (c->tag) hipFree(c->tag);
  c->tag = nullptr;
  c->cc_on = false;
  c->mistag = 0.0;
  c->ntag[0] = c->ntag[1] = 0;
}

static kpsi_status load_common(kpsi_ctx* c, kpsi_set set, int64_t n) {
  if (!c) return KPSI_E_ARG;
  if (set != KPSI_DATA && set != KPSI_NORM) return fail(c, KPSI_E_ARG, "unknown set");
  if (n <= 0) return fail(c, KPSI_E_ARG, "n must be positive");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "set the model before loading events");
  drop_background(c);   // its per-event values belong to the previous events
  if (set == KPSI_DATA) drop_flavour(c);
  return KPSI_OK;
}

// Per-event values of a host array into a new device array of the context precision.
static kpsi_status upload_values(kpsi_ctx* c, const double* v, int64_t n, void** out) {
  const size_t ts = tsize(c);
  if (hipMalloc(out, (size_t)n * ts) != hipSuccess) return fail(c, KPSI_E_OOM, "per-event values");
  std::vector<unsigned char> buf((size_t)n * ts);
  if (c->prec == KPSI_FP32) {
    float* f = reinterpret_cast<float*>(buf.data());
    for (int64_t i = 0; i < n; ++i) f[i] = (float)v[i];
  } else {
    std::memcpy(buf.data(), v, (size_t)n * sizeof(double));
  }
  HIPCHECK(c, hipMemcpy(*out, buf.data(), buf.size(), hipMemcpyHostToDevice));
  return KPSI_OK;
}

kpsi_status kpsi_set_background(kpsi_ctx* c, double purity, const double* eps_data, const double* b_data,
                                const double* b_norm) {
  if (!c) return KPSI_E_ARG;
  hipSetDevice(c->device);
  drop_background(c);
  if (!b_data) return KPSI_OK;   // signal-only likelihood
  if (!b_norm) return fail(c, KPSI_E_ARG, "b_norm is NULL");
  if (!(purity > 0.0 && purity <= 1.0)) return fail(c, KPSI_E_ARG, "purity %g outside (0, 1]", purity);
  const int64_t nd = c->set[0].n, nm = c->set[1].n;
  if (nd <= 0 || nm <= 0) return fail(c, KPSI_E_STATE, "load both event sets before the background");
  for (int64_t i = 0; i < nd; ++i) {
    if (!(b_data[i] >= 0.0) || !std::isfinite(b_data[i])) return fail(c, KPSI_E_ARG, "b_data[%lld] invalid", (long long)i);
    if (eps_data && (!(eps_data[i] >= 0.0) || !std::isfinite(eps_data[i])))
      return fail(c, KPSI_E_ARG, "eps_data[%lld] invalid", (long long)i);
  }
  // Neumaier sum of b over the normalisation events (times their importance weights, if any)
  double s = 0.0, comp = 0.0;
  const bool wtd = !c->norm_w_host.empty();
  for (int64_t j = 0; j < nm; ++j) {
    if (!(b_norm[j] >= 0.0) || !std::isfinite(b_norm[j])) return fail(c, KPSI_E_ARG, "b_norm[%lld] invalid", (long long)j);
    const double x = wtd ? b_norm[j] * c->norm_w_host[j] : b_norm[j];
    const double t = s + x;
    comp += (std::fabs(s) >= std::fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  const double nb = (s + comp) / (double)nm;
  if (!(nb > 0.0)) return fail(c, KPSI_E_ARG, "background integral over the normalisation events is %g", nb);
  kpsi_status st = upload_values(c, b_data, nd, &c->bkg_data);
  if (!st && eps_data) st = upload_values(c, eps_data, nd, &c->eps_data);
  if (st) { drop_background(c); return st; }
  c->purity = purity;
  c->bkg_coef = (1.0 - purity) / (nb * (double)nm);
  c->bkg_on = true;
  return KPSI_OK;
}

kpsi_status kpsi_set_flavour(kpsi_ctx* c, const double* tags, int64_t n, double mistag) {
  if (!c) return KPSI_E_ARG;
  hipSetDevice(c->device);
  drop_flavour(c);
  invalidate_cache(c);
  if (!tags) return KPSI_OK;   // B0 only
  if (n != c->set[0].n || n <= 0) return fail(c, KPSI_E_ARG, "expected %lld tags (one per data event)", (long long)c->set[0].n);
  if (!(mistag >= 0.0 && mistag <= 0.5)) return fail(c, KPSI_E_ARG, "mistag %g outside [0, 1/2]", mistag);
  int64_t np = 0, nn = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (tags[i] == 1.0) ++np;
    else if (tags[i] == -1.0) ++nn;
    else return fail(c, KPSI_E_ARG, "tags[%lld] = %g is not +1 or -1", (long long)i, tags[i]);
  }
  kpsi_status st = upload_values(c, tags, n, &c->tag);
  if (st) { drop_flavour(c); return st; }
  c->mistag = mistag;
  c->ntag[0] = np;
  c->ntag[1] = nn;
  c->cc_on = true;
  return KPSI_OK;
}

kpsi_status kpsi_template_values(kpsi_ctx* c, kpsi_set set, const float* t_mass, const int n_mass[2],
                                 const float* t_ang, const int n_ang[2], double* out) {
  if (!c) return KPSI_E_ARG;
  if (set != KPSI_DATA && set != KPSI_NORM) return fail(c, KPSI_E_ARG, "unknown set");
  if (!t_mass || !n_mass || !t_ang || !n_ang || !out) return fail(c, KPSI_E_ARG, "NULL argument");
  if (n_mass[0] <= 0 || n_mass[1] <= 0 || n_ang[0] <= 0 || n_ang[1] <= 0) return fail(c, KPSI_E_ARG, "bad bin counts");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set (kinematics needed)");
  const DevSet& d = c->set[set];
  if (d.n <= 0) return fail(c, KPSI_E_STATE, "set not loaded");
  hipSetDevice(c->device);
  const size_t n1 = (size_t)n_mass[0] * n_mass[1], n2 = (size_t)n_ang[0] * n_ang[1];
  float *d1 = nullptr, *d2 = nullptr;
  double* dout = nullptr;
  auto cleanup = [&]() { if (d1) hipFree(d1); if (d2) hipFree(d2); if (dout) hipFree(dout); };
  if (hipMalloc(&d1, n1 * sizeof(float)) || hipMalloc(&d2, n2 * sizeof(float)) ||
      hipMalloc(&dout, (size_t)d.n * sizeof(double))) {
    cleanup();
    return fail(c, KPSI_E_OOM, "template buffers");
  }
  TplArgs a{};
  for (int j = 0; j < 4; ++j) a.obs[j] = d.obs[j];
  a.t1 = d1;
  a.t2 = d2;
  a.nb[0] = n_mass[0]; a.nb[1] = n_mass[1]; a.nb[2] = n_ang[0]; a.nb[3] = n_ang[1];
  a.lo[0] = c->kin.m_k + c->kin.m_pi; a.hi[0] = c->kin.m_b - c->kin.m_jpsi;
  a.lo[1] = -1.0; a.hi[1] = 1.0;
  a.lo[2] = -1.0; a.hi[2] = 1.0;
  a.lo[3] = -M_PI; a.hi[3] = M_PI;
  a.n = d.n;
  a.out = dout;
  hipError_t e = hipMemcpyAsync(d1, t_mass, n1 * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d2, t_ang, n2 * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_template(a, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, (size_t)d.n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  cleanup();
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "template lookup: %s", hipGetErrorString(e));
  return KPSI_OK;
}

// The efficiency, importance weights and their columns belong to the loaded normalisation set.
static void drop_norm_columns(kpsi_ctx* c) {
  for (void** p : {&c->eps, (void**)&c->eps_f64, (void**)&c->norm_w, &c->wcol}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  c->norm_w_host.clear();
}

kpsi_status kpsi_load_events(kpsi_ctx* c, kpsi_set set, int64_t n, const double* m, const double* ck,
                             const double* cj, const double* phi) {
  kpsi_status st = load_common(c, set, n);
  if (st) return st;
  if (!m || !ck || !cj || !phi) return fail(c, KPSI_E_ARG, "NULL event array");
  hipSetDevice(c->device);
  DevSet& d = c->set[set];
  if (d.owned) hipFree(d.owned);
  d.owned = nullptr;
  d.n = 0;
  if (hipMalloc(&d.owned, 4 * (size_t)n * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "event copy");
  const double* src[4] = {m, ck, cj, phi};
  for (int j = 0; j < 4; ++j) {
    d.obs[j] = d.owned + (size_t)j * n;
    HIPCHECK(c, hipMemcpyAsync((void*)d.obs[j], src[j], n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  st = validate(c, n, d.obs);
  if (st) return st;
  d.n = n;
  if (set == KPSI_NORM) drop_norm_columns(c);
  if (set == KPSI_NORM) invalidate_cache(c);
  st = derive_columns(c, set);
  if (st) return st;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return KPSI_OK;
}

kpsi_status kpsi_load_events_device(kpsi_ctx* c, kpsi_set set, int64_t n, const double* m, const double* ck,
                                    const double* cj, const double* phi) {
  kpsi_status st = load_common(c, set, n);
  if (st) return st;
  if (!m || !ck || !cj || !phi) return fail(c, KPSI_E_ARG, "NULL event array");
  hipSetDevice(c->device);
  DevSet& d = c->set[set];
  if (d.owned) hipFree(d.owned);
  d.owned = nullptr;
  d.n = 0;
  const double* src[4] = {m, ck, cj, phi};
  st = validate(c, n, src);
  if (st) return st;
  for (int j = 0; j < 4; ++j) d.obs[j] = src[j];
  d.n = n;
  if (set == KPSI_NORM) drop_norm_columns(c);
  if (set == KPSI_NORM) invalidate_cache(c);
  st = derive_columns(c, set);
  if (st) return st;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return KPSI_OK;
}

// The per-event column the kernels read: efficiency times importance weight (null when both are 1).
static kpsi_status rebuild_eps(kpsi_ctx* c) {
  invalidate_cache(c);
  if (!c->eps_f64 && !c->norm_w) {
    if (c->eps) hipFree(c->eps);
    c->eps = nullptr;
    return KPSI_OK;
  }
  return product_column(c, c->eps_f64, c->norm_w, &c->eps);
}

kpsi_status kpsi_set_efficiency_flat(kpsi_ctx* c) {
  if (!c) return KPSI_E_ARG;
  hipSetDevice(c->device);
  if (c->eps_f64) hipFree(c->eps_f64);
  c->eps_f64 = nullptr;
  return rebuild_eps(c);
}

static kpsi_status eps_from_device_f64(kpsi_ctx* c, const double* d_eps, int64_t n) {
  double* e = nullptr;
  if (hipMalloc(&e, (size_t)n * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "efficiency column");
  hipError_t er = hipMemcpyAsync(e, d_eps, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (er != hipSuccess) { hipFree(e); return fail(c, KPSI_E_HIP, "efficiency copy: %s", hipGetErrorString(er)); }
  if (c->eps_f64) hipFree(c->eps_f64);
  c->eps_f64 = e;
  return rebuild_eps(c);
}

kpsi_status kpsi_set_efficiency_values(kpsi_ctx* c, const double* eps, int64_t n) {
  if (!c) return KPSI_E_ARG;
  if (!eps) return fail(c, KPSI_E_ARG, "eps is NULL");
  if (c->set[1].n <= 0) return fail(c, KPSI_E_STATE, "load the normalisation set first");
  if (n != c->set[1].n) return fail(c, KPSI_E_ARG, "expected %lld efficiency values", (long long)c->set[1].n);
  for (int64_t i = 0; i < n; ++i)
    if (!(eps[i] >= 0.0 && eps[i] <= 1.0)) return fail(c, KPSI_E_ARG, "efficiency %lld outside [0, 1]", (long long)i);
  hipSetDevice(c->device);
  double* d = nullptr;
  if (hipMalloc(&d, (size_t)n * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "efficiency staging");
  hipError_t er = hipMemcpyAsync(d, eps, (size_t)n * sizeof(double), hipMemcpyHostToDevice, c->stream);
  kpsi_status st = er == hipSuccess ? eps_from_device_f64(c, d, n) : fail(c, KPSI_E_HIP, "efficiency upload");
  hipFree(d);
  return st;
}

kpsi_status kpsi_set_efficiency_hist(kpsi_ctx* c, const float* eff, const int nb[4], const double lo[4],
                                     const double hi[4]) {
  if (!c) return KPSI_E_ARG;
  if (!eff || !nb || !lo || !hi) return fail(c, KPSI_E_ARG, "NULL histogram argument");
  if (c->set[1].n <= 0) return fail(c, KPSI_E_STATE, "load the normalisation set first");
  int64_t nbins = 1;
  for (int d = 0; d < 4; ++d) {
    if (nb[d] <= 0 || !(hi[d] > lo[d])) return fail(c, KPSI_E_ARG, "bad histogram axis %d", d);
    nbins *= nb[d];
  }
  for (int64_t i = 0; i < nbins; ++i)
    if (!(eff[i] >= 0.0f && eff[i] <= 1.0f)) return fail(c, KPSI_E_ARG, "bin %lld outside [0, 1]", (long long)i);
  hipSetDevice(c->device);
  float* table = nullptr;
  double* vals = nullptr;
  const int64_t n = c->set[1].n;
  if (hipMalloc(&table, nbins * sizeof(float)) != hipSuccess || hipMalloc(&vals, n * sizeof(double)) != hipSuccess) {
    if (table) hipFree(table);
    return fail(c, KPSI_E_OOM, "histogram");
  }
  HistArgs a{};
  for (int d = 0; d < 4; ++d) { a.obs[d] = c->set[1].obs[d]; a.nb[d] = nb[d]; a.lo[d] = lo[d]; a.hi[d] = hi[d]; }
  a.table = table;
  a.n = n;
  a.out_f64 = vals;
  hipError_t er = hipMemcpyAsync(table, eff, nbins * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (er == hipSuccess) er = launch_hist_lookup(a, c->stream);
  kpsi_status st = er == hipSuccess ? eps_from_device_f64(c, vals, n) : fail(c, KPSI_E_HIP, "histogram lookup");
  hipFree(table);
  hipFree(vals);
  return st;
}

kpsi_status kpsi_set_norm_mixture(kpsi_ctx* c, const double* params0, int64_t n_flat) {
  if (!c) return KPSI_E_ARG;
  if (!params0) return fail(c, KPSI_E_ARG, "params0 is NULL");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  const int64_t n = c->set[1].n;
  if (n <= 0) return fail(c, KPSI_E_STATE, "load the normalisation set first");
  if (n_flat < 1 || n_flat > n) return fail(c, KPSI_E_ARG, "n_flat %lld outside [1, %lld]", (long long)n_flat, (long long)n);
  if (c->bkg_on) return fail(c, KPSI_E_STATE, "set the normalisation mixture before the background");
  for (int i = 0; i < c->nparams; ++i)
    if (!std::isfinite(params0[i])) return fail(c, KPSI_E_ARG, "params0[%d] is not finite", i);
  hipSetDevice(c->device);
  auto drop = [&]() {
    for (void** p : {(void**)&c->norm_w, &c->wcol}) {
      if (*p) hipFree(*p);
      *p = nullptr;
    }
    c->norm_w_host.clear();
  };
  drop();
  if (n_flat == n) return rebuild_eps(c);   // a flat set: no weights
  // S(y; params0) of every normalisation event
  double* d = nullptr;
  if (hipMalloc(&d, (size_t)n * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "density output");
  double* outs[2] = {nullptr, d};
  std::vector<double> s0((size_t)n);
  kpsi_status st = dispatch(c, MODE_DENSITY, params0, 1, outs);
  if (!st) {
    hipError_t e = hipMemcpyAsync(s0.data(), d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = fail(c, KPSI_E_HIP, "density copy: %s", hipGetErrorString(e));
  }
  hipFree(d);
  if (st) return st;
  // Z0: the flat events' mean of S0 (compensated sum)
  double sum = 0.0, comp = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (!(s0[j] >= 0.0) || !std::isfinite(s0[j])) return fail(c, KPSI_E_ARG, "density of normalisation event %lld is %g",
                                                          (long long)j, s0[j]);
    if (j >= n_flat) continue;
    const double t = sum + s0[j];
    comp += (std::fabs(sum) >= std::fabs(s0[j])) ? (sum - t) + s0[j] : (s0[j] - t) + sum;
    sum = t;
  }
  const double z0 = (sum + comp) / (double)n_flat;
  if (!(z0 > 0.0)) return fail(c, KPSI_E_ARG, "mean density of the flat events is %g", z0);
  // density of the mixture relative to flat phase space: alpha + (1 - alpha) S0 / Z0
  const double alpha = (double)n_flat / (double)n;
  c->norm_w_host.resize((size_t)n);
  for (int64_t j = 0; j < n; ++j) c->norm_w_host[j] = 1.0 / (alpha + (1.0 - alpha) * (s0[j] / z0));
  if (hipMalloc(&c->norm_w, (size_t)n * sizeof(double)) != hipSuccess) {
    c->norm_w = nullptr;
    drop();
    return fail(c, KPSI_E_OOM, "importance weights");
  }
  hipError_t e = hipMemcpyAsync(c->norm_w, c->norm_w_host.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                                c->stream);
  if (e != hipSuccess) { drop(); return fail(c, KPSI_E_HIP, "weight upload: %s", hipGetErrorString(e)); }
  st = product_column(c, c->norm_w, nullptr, &c->wcol);
  if (!st) st = rebuild_eps(c);
  if (st) { drop(); rebuild_eps(c); }
  return st;
}

// Normalisation term of the NLL from the normalisation records, and the factors that weight
// their gradient accumulators.  Signal and mixture: 2 N_d ln(sum eps S / N_MC) from record 1,
// gradient factor 2 W / sum eps S (W = N_d, or sum_i w_i S_i with the mixture).  Flavour
// tags: 2 sum_q n_q ln N_q with N_q = (1 - w) I(q) + w I(-q), I(+) and I(-) from records 1
// and 2.  Returns false when a normalisation is not positive (value then holds it).
// wp, wn: the weights W of the data events (per flavour with tags): their count, or with the
// Eq. 14 mixture sum_i w_i S_i over them.
static bool norm_term(const kpsi_ctx* c, double wp, double wn, double* value, double* c1, double* c2) {
  const double* r1 = c->red_host + NACC;
  const double nd = (double)c->set[0].n, nm = (double)c->set[1].n;
  const double s1 = r1[0] + r1[1];
  if (!c->cc_on) {
    *value = s1;
    if (!(s1 > 0.0)) return false;
    *value = 2.0 * nd * std::log(s1 / nm);
    *c1 = 2.0 * wp / s1;
    *c2 = 0.0;
    return true;
  }
  const double* r2 = c->red_host + 2 * NACC;
  const double ip = s1 / nm, im = (r2[0] + r2[1]) / nm, w = c->mistag;
  const double np = (double)c->ntag[0], nn = (double)c->ntag[1];
  const double Np = (1.0 - w) * ip + w * im, Nn = (1.0 - w) * im + w * ip;
  *value = Np < Nn ? Np : Nn;
  if (!(Np > 0.0) || !(Nn > 0.0)) return false;
  *value = 2.0 * ((np > 0.0 ? np * std::log(Np) : 0.0) + (nn > 0.0 ? nn * std::log(Nn) : 0.0));
  *c1 = 2.0 / nm * (wp * (1.0 - w) / Np + wn * w / Nn);
  *c2 = 2.0 / nm * (wp * w / Np + wn * (1.0 - w) / Nn);
  return true;
}

kpsi_status kpsi_set_constraints(kpsi_ctx* c, int n, const int* index, const double* mean, const double* sigma) {
  if (!c) return KPSI_E_ARG;
  if (n < 0) return fail(c, KPSI_E_ARG, "negative constraint count");
  if (n > 0 && (!index || !mean || !sigma)) return fail(c, KPSI_E_ARG, "NULL constraint arrays");
  if (n > 0 && !c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  for (int k = 0; k < n; ++k) {
    if (index[k] < 0 || index[k] >= c->nparams) return fail(c, KPSI_E_ARG, "constraint %d: index %d out of range", k, index[k]);
    if (!(sigma[k] > 0.0) || !std::isfinite(sigma[k]) || !std::isfinite(mean[k]))
      return fail(c, KPSI_E_ARG, "constraint %d: needs a finite mean and sigma > 0", k);
  }
  c->con_idx.assign(index, index + n);
  c->con_mean.assign(mean, mean + n);
  c->con_sigma.assign(sigma, sigma + n);
  return KPSI_OK;
}

// Gaussian constraints: sum_k ((p - mean)/sigma)^2 added to -2 ln L, and 2 (p - mean)/sigma^2
// to the gradient (grad may be null).
static double add_constraints(const kpsi_ctx* c, const double* params, double* grad) {
  double v = 0.0;
  for (size_t k = 0; k < c->con_idx.size(); ++k) {
    const double z = (params[c->con_idx[k]] - c->con_mean[k]) / c->con_sigma[k];
    v += z * z;
    if (grad) grad[c->con_idx[k]] += 2.0 * z / c->con_sigma[k];
  }
  return v;
}

kpsi_status kpsi_nll(kpsi_ctx* c, const double* params, double* nll) {
  kpsi_status st = check_ready(c, params);
  if (st) return st;
  if (!nll) return fail(c, KPSI_E_ARG, "nll is NULL");
  hipSetDevice(c->device);
  bool cached = false;
  st = use_cache(c, params, &cached);
  if (st) return st;
  if (cached) {
    st = put_cached_record(c, params);
    if (st) return st;
  }
  st = dispatch(c, MODE_NLL, params, cached ? 0 : -1, nullptr);
  if (st) return st;
  const double* rd = c->red_host;
  const double nd = (double)c->set[0].n;
  double nt, c1, c2;
  const bool ok = norm_term(c, (double)c->ntag[0], (double)c->ntag[1], &nt, &c1, &c2);   // (value only)
  if (rd[2] > 0.0 || !ok) {
    *nll = INFINITY;
    return fail(c, KPSI_E_NONFINITE, "%.0f data events with non-positive density; normalisation %g", rd[2],
                ok ? 1.0 : nt);
  }
  *nll = -2.0 * (rd[0] + rd[1]) + nt + add_constraints(c, params, nullptr);
  return KPSI_OK;
}

// -2 ln L and its gradient from the reduced records of a gradient-mode pass (the normalisation
// record from the interference matrix when `cached`).
static kpsi_status assemble_grad(kpsi_ctx* c, const double* params, bool cached, double* nll, double* grad) {
  const double* rd = c->red_host;
  const double* rm = c->red_host + NACC;
  const double* rm2 = c->red_host + 2 * NACC;
  const double nd = (double)c->set[0].n;
  for (int i = 0; i < c->nparams; ++i) grad[i] = NAN;
  // combined complex sensitivity G = -2 G_data + c1 G_norm1 (+ c2 G_norm2 with flavour tags):
  // c1 = 2 W / sum(eps S), W = N_d (signal only) or sum_i w_i S_i (Eq. 14 mixture,
  // w_i = p eps_i / t_i); dNLL/dr = 2 Re(e^{i phi} G), dNLL/dphi = -2 Im(H G)
  int N[5], NZ;
  shape_counts(c->shape, N, &NZ);
  int nkacc = 0;
  for (int j = 0; j < 5; ++j) nkacc += N[j] * (j == 0 ? 2 : 6);
  // W per flavour: the data counts, or with the mixture sum_i w_i S_i (the - flavour's in slot 1
  // of the data record, whose log sum is then slot 0 alone)
  const bool tagmix = c->bkg_on && c->cc_on;
  double wp = c->cc_on ? (double)c->ntag[0] : nd, wn = (double)c->ntag[1];
  if (c->bkg_on) wp = rd[3 + nkacc + 4 * NZ + 2 * NFL];
  if (tagmix) wn = rd[1];
  double nt, fm, fm2;
  const bool ok = norm_term(c, wp, wn, &nt, &fm, &fm2);
  if (rd[2] > 0.0 || !ok) {
    *nll = INFINITY;
    return fail(c, KPSI_E_NONFINITE, "%.0f data events with non-positive density; normalisation %g", rd[2],
                ok ? 1.0 : nt);
  }
  *nll = -2.0 * (tagmix ? rd[0] : rd[0] + rd[1]) + nt;
  const int ncr = c->nparams - 2 * (int)c->res.size();
  for (size_t i = 0; i < c->res.size(); ++i) {
    const kpsi_resonance& r = c->res[i];
    const int ao = acc_offset(c, i, N);
    const int nl = ncoup(r);
    const double* p = params + c->coff[i];
    // the kernel's coupling accumulators are d/dH' with H' = K H: multiply by K (the
    // interference-matrix record is already in terms of H)
    const double kr = lineshape_consts(c->kin, r, params[ncr + 2 * i], params[ncr + 2 * i + 1]).K;
    const double km = cached ? 1.0 : kr;
    for (int l = 0; l < nl; ++l) {
      // K* spin >= 1 accumulators are lambda = -1, 0, +1; spin 0 has lambda = 0 only; Z has 0, +-1
      const int a = ao + 2 * l;
      const double gr = -2.0 * kr * rd[a] + km * (fm * rm[a] + fm2 * rm2[a]);
      const double gi = -2.0 * kr * rd[a + 1] + km * (fm * rm[a + 1] + fm2 * rm2[a + 1]);
      const double mag = p[2 * l], ph = p[2 * l + 1];
      const double cph = std::cos(ph), sph = std::sin(ph);
      grad[c->coff[i] + 2 * l] = 2.0 * (cph * gr - sph * gi);
      grad[c->coff[i] + 2 * l + 1] = -2.0 * mag * (cph * gi + sph * gr);
    }
    if (c->fslot[i] >= 0) {
      const int a = 3 + nkacc + 4 * NZ + 2 * c->fslot[i];
      grad[ncr + 2 * i] = 2.0 * (-2.0 * rd[a] + fm * rm[a] + fm2 * rm2[a]);
      grad[ncr + 2 * i + 1] = 2.0 * (-2.0 * rd[a + 1] + fm * rm[a + 1] + fm2 * rm2[a + 1]);
    }
  }
  *nll += add_constraints(c, params, grad);
  return KPSI_OK;
}

kpsi_status kpsi_nll_and_grad(kpsi_ctx* c, const double* params, double* nll, double* grad) {
  kpsi_status st = check_ready(c, params);
  if (st) return st;
  if (!nll || !grad) return fail(c, KPSI_E_ARG, "nll/grad is NULL");
  hipSetDevice(c->device);
  bool cached = false;
  st = use_cache(c, params, &cached);
  if (st) return st;
  if (cached) {
    st = put_cached_record(c, params);
    if (st) return st;
  }
  st = dispatch(c, MODE_GRAD, params, cached ? 0 : -1, nullptr);
  if (st) return st;
  return assemble_grad(c, params, cached, nll, grad);
}

// The same pass with its block partials in the static device array: nothing is allocated.  Every
// partial the final reduction reads is written by the per-event launch of the same call, so the
// array needs no clearing between calls.
kpsi_status kpsi_nll_and_grad_noalloc(kpsi_ctx* c, const double* params, double* nll, double* grad) {
  kpsi_status st = check_ready(c, params);
  if (st) return st;
  if (!nll || !grad) return fail(c, KPSI_E_ARG, "nll/grad is NULL");
  double* scr = scratch_ptr(c->device);
  if (!scr) return fail(c, KPSI_E_HIP, "the static scratch array has no address on device %d", c->device);
  hipSetDevice(c->device);
  st = dispatch(c, MODE_GRAD, params, -1, nullptr, scr, kScratchDoubles);
  if (st) return st;
  return assemble_grad(c, params, false, nll, grad);
}

kpsi_status kpsi_density(kpsi_ctx* c, kpsi_set set, const double* params, double* out) {
  if (!c) return KPSI_E_ARG;
  if (!params || !out) return fail(c, KPSI_E_ARG, "NULL argument");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  if (set != KPSI_DATA && set != KPSI_NORM) return fail(c, KPSI_E_ARG, "unknown set");
  const int64_t n = c->set[set].n;
  if (n <= 0) return fail(c, KPSI_E_STATE, "set not loaded");
  hipSetDevice(c->device);
  double* d = nullptr;
  if (hipMalloc(&d, n * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "density output");
  double* outs[2] = {set == 0 ? d : nullptr, set == 1 ? d : nullptr};
  kpsi_status st = dispatch(c, MODE_DENSITY, params, (int)set, outs);
  if (!st) {
    hipError_t e = hipMemcpyAsync(out, d, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = fail(c, KPSI_E_HIP, "density copy: %s", hipGetErrorString(e));
  }
  hipFree(d);
  return st;
}

kpsi_status kpsi_invariants(kpsi_ctx* c, kpsi_set set, double* out) {
  if (!c) return KPSI_E_ARG;
  if (!out) return fail(c, KPSI_E_ARG, "out is NULL");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  if (set != KPSI_DATA && set != KPSI_NORM) return fail(c, KPSI_E_ARG, "unknown set");
  DevSet& s = c->set[set];
  if (s.n <= 0) return fail(c, KPSI_E_STATE, "set not loaded");
  hipSetDevice(c->device);
  double *diag = nullptr, *cols = nullptr;
  const int64_t ld = (s.n + 63) / 64 * 64;
  if (hipMalloc(&diag, 5 * s.n * sizeof(double)) != hipSuccess ||
      hipMalloc(&cols, (size_t)ld * NCOL_MAX * sizeof(double)) != hipSuccess) {
    if (diag) hipFree(diag);
    return fail(c, KPSI_E_OOM, "diagnostic buffers");
  }
  InvArgs<double> a{};
  for (int j = 0; j < 4; ++j) a.obs[j] = s.obs[j];
  a.cols = cols;
  a.ld = ld;
  a.n = s.n;
  a.mB = c->kin.m_b; a.mJ = c->kin.m_jpsi; a.mK = c->kin.m_k; a.mPi = c->kin.m_pi;
  a.rB = c->kin.r_b; a.rR = c->kin.r_r;
  a.with_z = 1;
  a.diag = diag;
  hipError_t e = launch_invariants<double>(a, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, diag, 5 * s.n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(diag);
  hipFree(cols);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "invariants: %s", hipGetErrorString(e));
  return KPSI_OK;
}

kpsi_status kpsi_generate_phsp(kpsi_ctx* c, uint64_t seed, int64_t n, double wmax, double* m, double* ck,
                               double* cj, double* phi) {
  if (!c) return KPSI_E_ARG;
  if (n <= 0 || !m || !ck || !cj || !phi || !(wmax > 0.0)) return fail(c, KPSI_E_ARG, "bad generator arguments");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set (kinematics needed)");
  hipSetDevice(c->device);
  int* flag = nullptr;
  if (hipMalloc(&flag, n * sizeof(int)) != hipSuccess) return fail(c, KPSI_E_OOM, "generator flags");
  GenArgs g{};
  g.seed = seed; g.e0 = 0; g.n = n; g.wmax = wmax;
  g.mB = c->kin.m_b; g.mJ = c->kin.m_jpsi; g.mK = c->kin.m_k; g.mPi = c->kin.m_pi;
  g.out[0] = m; g.out[1] = ck; g.out[2] = cj; g.out[3] = phi;
  g.spare = nullptr;
  g.flag = flag;
  hipError_t e = launch_phsp(g, c->stream);
  // every event must have been produced within the trial budget
  int* dsum = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  int last_pos = 0, last_flag = 0;
  if (e == hipSuccess) e = hipMalloc(&dsum, n * sizeof(int));
  if (e == hipSuccess) e = exclusive_scan_int(flag, dsum, n, nullptr, &tb, c->stream);
  if (e == hipSuccess) e = hipMalloc(&tmp, tb);
  if (e == hipSuccess) e = exclusive_scan_int(flag, dsum, n, tmp, &tb, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&last_pos, dsum + n - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&last_flag, flag + n - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(flag);
  if (dsum) hipFree(dsum);
  if (tmp) hipFree(tmp);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "phase-space generator: %s", hipGetErrorString(e));
  if (last_pos + last_flag != n) return fail(c, KPSI_E_ARG, "envelope wmax too small: trial budget exhausted");
  return KPSI_OK;
}

kpsi_status kpsi_generate_model(kpsi_ctx* c, const double* params, uint64_t seed, int64_t n, double wmax,
                                double smax, const double* acc_coef, double* m, double* ck, double* cj,
                                double* phi, int64_t* n_prop, int64_t* n_over) {
  if (!c) return KPSI_E_ARG;
  if (!params || n <= 0 || !m || !ck || !cj || !phi || !(wmax > 0.0) || !(smax > 0.0) || !n_prop || !n_over)
    return fail(c, KPSI_E_ARG, "bad generator arguments");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  hipSetDevice(c->device);
  const int64_t B = 1 << 20;
  const int64_t ld = B;
  double *obs = nullptr, *spare = nullptr, *S = nullptr, *cols = nullptr;
  int *valid = nullptr, *flag = nullptr, *over = nullptr, *pos = nullptr, *opos = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  auto cleanup = [&]() {
    for (void* p : {(void*)obs, (void*)spare, (void*)S, (void*)cols, (void*)valid, (void*)flag, (void*)over,
                    (void*)pos, (void*)opos, tmp})
      if (p) hipFree(p);
  };
  if (hipMalloc(&obs, 4 * B * sizeof(double)) || hipMalloc(&spare, B * sizeof(double)) ||
      hipMalloc(&S, B * sizeof(double)) || hipMalloc(&cols, (size_t)ld * NCOL_MAX * sizeof(double)) ||
      hipMalloc(&valid, B * sizeof(int)) || hipMalloc(&flag, B * sizeof(int)) || hipMalloc(&over, B * sizeof(int)) ||
      hipMalloc(&pos, B * sizeof(int)) || hipMalloc(&opos, B * sizeof(int))) {
    cleanup();
    return fail(c, KPSI_E_OOM, "generator buffers");
  }
  exclusive_scan_int(flag, pos, B, nullptr, &tb, c->stream);
  if (hipMalloc(&tmp, tb)) { cleanup(); return fail(c, KPSI_E_OOM, "scan scratch"); }
  const double delta = 1.0 - std::pow(3.0, -0.25);
  int64_t kept = 0, e0 = 0, novr = 0;
  kpsi_status st = KPSI_OK;
  std::vector<int> hpos, hflag;
  while (kept < n) {
    GenArgs g{};
    g.seed = seed; g.e0 = e0; g.n = B; g.wmax = wmax;
    g.mB = c->kin.m_b; g.mJ = c->kin.m_jpsi; g.mK = c->kin.m_k; g.mPi = c->kin.m_pi;
    for (int j = 0; j < 4; ++j) g.out[j] = obs + j * B;
    g.spare = spare;
    g.flag = valid;
    hipError_t e = launch_phsp(g, c->stream);
    InvArgs<double> ia{};
    for (int j = 0; j < 4; ++j) ia.obs[j] = obs + j * B;
    ia.cols = cols; ia.ld = ld; ia.n = B;
    ia.mB = c->kin.m_b; ia.mJ = c->kin.m_jpsi; ia.mK = c->kin.m_k; ia.mPi = c->kin.m_pi;
    ia.rB = c->kin.r_b; ia.rR = c->kin.r_r;
    ia.with_z = c->has_z ? 1 : 0;
    ia.zfree = c->zfree ? 1 : 0;
    if (e == hipSuccess) e = launch_invariants<double>(ia, c->stream);
    if (e != hipSuccess) { st = fail(c, KPSI_E_HIP, "generator: %s", hipGetErrorString(e)); break; }
    // density of the proposals through the FP64 amplitude kernel
    {
      auto dens = [&](auto shtag) -> hipError_t {
        using Sh = decltype(shtag);
        AmpArgs<double, Sh> a{};
        a.cols[0] = cols; a.ld[0] = ld; a.n[0] = B;
        a.cols[1] = cols; a.ld[1] = ld; a.n[1] = 0;
        a.s_out[0] = S; a.s_out[1] = nullptr;
        a.eps = nullptr;
        pack<double, Sh>(c, params, a);
        a.chunk = BLOCK * 4;
        a.nb_data = (int)((B + a.chunk - 1) / a.chunk);
        a.partial = nullptr;
        return launch_amp<double, Sh>(a, MODE_DENSITY, a.nb_data, c->stream);
      };
      e = c->shape == 0 ? dens(ShapeSmall{}) : dens(ShapeFull{});
    }
    AcceptArgs aa{};
    for (int j = 0; j < 4; ++j) aa.obs[j] = obs + j * B;
    aa.S = S; aa.spare = spare; aa.valid = valid;
    aa.acc_on = acc_coef ? 1 : 0;
    for (int j = 0; j < 12; ++j) aa.coef[j] = acc_coef ? acc_coef[j] : 0.0;
    aa.delta = delta;
    aa.lo = c->kin.m_k + c->kin.m_pi; aa.hi = c->kin.m_b - c->kin.m_jpsi;
    aa.smax = smax; aa.n = B; aa.flag = flag; aa.over = over;
    if (e == hipSuccess) e = launch_accept(aa, c->stream);
    if (e == hipSuccess) e = exclusive_scan_int(flag, pos, B, tmp, &tb, c->stream);
    if (e == hipSuccess) e = exclusive_scan_int(over, opos, B, tmp, &tb, c->stream);
    CompactArgs ca{};
    for (int j = 0; j < 4; ++j) { ca.obs[j] = obs + j * B; }
    ca.out[0] = m; ca.out[1] = ck; ca.out[2] = cj; ca.out[3] = phi;
    ca.flag = flag; ca.pos = pos; ca.n = B; ca.base = kept; ca.limit = n;
    if (e == hipSuccess) e = launch_compact(ca, c->stream);
    int tail[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(&tail[0], pos + B - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&tail[1], flag + B - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&tail[2], opos + B - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&tail[3], over + B - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { st = fail(c, KPSI_E_HIP, "generator: %s", hipGetErrorString(e)); break; }
    const int64_t acc = tail[0] + tail[1];
    novr += tail[2] + tail[3];
    if (kept + acc >= n) {
      // locate the proposal that completes the sample
      hpos.resize(B);
      hflag.resize(B);
      e = hipMemcpy(hpos.data(), pos, B * sizeof(int), hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(hflag.data(), flag, B * sizeof(int), hipMemcpyDeviceToHost);
      if (e != hipSuccess) { st = fail(c, KPSI_E_HIP, "generator: %s", hipGetErrorString(e)); break; }
      const int64_t need = n - kept;
      int64_t last = B - 1;
      for (int64_t i = 0; i < B; ++i)
        if (hflag[i] && hpos[i] == need - 1) { last = i; break; }
      e0 += last + 1;
      kept = n;
      break;
    }
    kept += acc;
    e0 += B;
    if (e0 > ((int64_t)1 << 40)) { st = fail(c, KPSI_E_ARG, "proposal budget exhausted"); break; }
  }
  cleanup();
  *n_prop = e0;
  *n_over = novr;
  return st;
}

kpsi_status kpsi_time_kernel(kpsi_ctx* c, const double* params, int grad, int reps, double* ms_per_launch) {
  kpsi_status st = check_ready(c, params);
  if (st) return st;
  if (!ms_per_launch) return fail(c, KPSI_E_ARG, "ms_per_launch is NULL");
  if (reps < 1 || reps > 100000) return fail(c, KPSI_E_ARG, "reps %d outside [1, 100000]", reps);
  hipSetDevice(c->device);
  c->bench_reps = reps;
  st = dispatch(c, grad ? MODE_GRAD : MODE_NLL, params, -1, nullptr);
  c->bench_reps = 0;
  if (st) return st;
  *ms_per_launch = c->bench_ms;
  return KPSI_OK;
}

kpsi_status kpsi_set_timing(kpsi_ctx* c, int every) {
  if (!c) return KPSI_E_ARG;
  if (every < 0) return fail(c, KPSI_E_ARG, "timing interval %d < 0", every);
  drain_timing(c);
  if (every > 0 && c->tev.empty()) {
    std::vector<hipEvent_t> ev(2 * kTimingPairs, nullptr);
    for (hipEvent_t& e : ev) {
      if (hipEventCreate(&e) != hipSuccess) {
        for (hipEvent_t x : ev)
          if (x) hipEventDestroy(x);
        return fail(c, KPSI_E_HIP, "timing events");
      }
    }
    c->tev = std::move(ev);
  }
  c->timing_every = every;
  c->timing_calls = 0;
  c->timing = false;
  return KPSI_OK;
}

kpsi_status kpsi_timing(kpsi_ctx* c, double* ms, int64_t* n, int reset) {
  if (!c) return KPSI_E_ARG;
  drain_timing(c);
  if (ms) *ms = c->t_ms;
  if (n) *n = c->t_n;
  if (reset) { c->t_ms = 0.0; c->t_n = 0; c->t_dropped = 0; c->t_samples.clear(); }
  return KPSI_OK;
}

kpsi_status kpsi_timing_median(kpsi_ctx* c, double* ms) {
  if (!c || !ms) return KPSI_E_ARG;
  drain_timing(c);
  std::vector<float> v = c->t_samples;
  if (v.empty()) { *ms = NAN; return KPSI_OK; }
  std::sort(v.begin(), v.end());
  const size_t h = v.size() / 2;
  *ms = (v.size() & 1) ? v[h] : 0.5 * ((double)v[h - 1] + (double)v[h]);
  return KPSI_OK;
}

const char* kpsi_last_error(const kpsi_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

// ---------------------------------------------------------------- learned efficiency
static const int MLP_NP = 4545;

kpsi_status kpsi_mlp_default_options(kpsi_mlp_options* o) {
  if (!o) return KPSI_E_ARG;
  o->epochs = 20;
  o->batch = 32768;
  o->lr = 2e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->eps = 1e-8;
  return KPSI_OK;
}

static bool mlp_obs_ok(const double* m, const double* ck, const double* cj, const double* phi) {
  return m && ck && cj && phi;
}

static MlpArgs mlp_args(const kpsi_ctx* c, int64_t n, const double* m, const double* ck, const double* cj,
                        const double* phi) {
  MlpArgs a{};
  a.obs[0] = m; a.obs[1] = ck; a.obs[2] = cj; a.obs[3] = phi;
  a.lo = c->kin.m_k + c->kin.m_pi;
  a.hi = c->kin.m_b - c->kin.m_jpsi;
  a.n = n;
  return a;
}

kpsi_status kpsi_accept_labels(kpsi_ctx* c, uint64_t seed, int64_t e0, int64_t n, const double* m, const double* ck,
                               const double* cj, const double* phi, const double* acc_coef, uint8_t* label,
                               double* eps_true) {
  if (!c) return KPSI_E_ARG;
  if (n <= 0 || e0 < 0 || !mlp_obs_ok(m, ck, cj, phi) || !acc_coef || !label) return fail(c, KPSI_E_ARG, "bad arguments");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set (kinematics needed)");
  hipSetDevice(c->device);
  LabelArgs a{};
  a.obs[0] = m; a.obs[1] = ck; a.obs[2] = cj; a.obs[3] = phi;
  a.seed = seed; a.e0 = e0; a.n = n;
  for (int j = 0; j < 12; ++j) a.coef[j] = acc_coef[j];
  a.delta = 1.0 - std::pow(3.0, -0.25);
  a.lo = c->kin.m_k + c->kin.m_pi;
  a.hi = c->kin.m_b - c->kin.m_jpsi;
  a.label = label;
  a.eps_out = eps_true;
  hipError_t e = launch_labels(a, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "labels: %s", hipGetErrorString(e));
  return KPSI_OK;
}

kpsi_status kpsi_hist_efficiency(kpsi_ctx* c, int64_t n, const double* m, const double* ck, const double* cj,
                                 const double* phi, const uint8_t* label, const int nb[4], const double lo[4],
                                 const double hi[4], float* table) {
  if (!c) return KPSI_E_ARG;
  if (n <= 0 || !mlp_obs_ok(m, ck, cj, phi) || !label || !nb || !lo || !hi || !table)
    return fail(c, KPSI_E_ARG, "bad arguments");
  int64_t nbins = 1;
  for (int d = 0; d < 4; ++d) {
    if (nb[d] <= 0 || !(hi[d] > lo[d])) return fail(c, KPSI_E_ARG, "bad histogram axis %d", d);
    nbins *= nb[d];
  }
  hipSetDevice(c->device);
  unsigned int* cnt = nullptr;
  if (hipMalloc(&cnt, 2 * nbins * sizeof(unsigned int)) != hipSuccess) return fail(c, KPSI_E_OOM, "histogram counts");
  HistCountArgs a{};
  a.obs[0] = m; a.obs[1] = ck; a.obs[2] = cj; a.obs[3] = phi;
  a.label = label;
  for (int d = 0; d < 4; ++d) { a.nb[d] = nb[d]; a.lo[d] = lo[d]; a.hi[d] = hi[d]; }
  a.n = n;
  a.gen = cnt;
  a.acc = cnt + nbins;
  std::vector<unsigned int> h(2 * nbins);
  hipError_t e = hipMemsetAsync(cnt, 0, 2 * nbins * sizeof(unsigned int), c->stream);
  if (e == hipSuccess) e = launch_hist_count(a, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), cnt, 2 * nbins * sizeof(unsigned int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(cnt);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "histogram: %s", hipGetErrorString(e));
  uint64_t tg = 0, ta = 0;
  for (int64_t i = 0; i < nbins; ++i) { tg += h[i]; ta += h[nbins + i]; }
  const float mean = tg ? (float)((double)ta / (double)tg) : 0.0f;
  for (int64_t i = 0; i < nbins; ++i) table[i] = h[i] ? (float)((double)h[nbins + i] / (double)h[i]) : mean;
  return KPSI_OK;
}

// Mean BCE gradient over events [0, n) into the device array g (MLP_NP doubles) and the mean
// loss into g[MLP_NP].
// BF16 copies of the 64x64 layer of the parameters at dparams (device), for the network kernels.
static hipError_t prep_w2h(kpsi_ctx* c, const float* dparams) {
  if (!c->mlp_w2h) {
    hipError_t e = hipMalloc(&c->mlp_w2h, 8192 * sizeof(unsigned short));
    if (e != hipSuccess) { c->mlp_w2h = nullptr; return e; }
  }
  return launch_mlp_bf16(dparams, c->mlp_w2h, c->stream);
}

// w2h_current: the BF16 copies already match dparams (the Adam kernel of the previous step wrote them)
static hipError_t mlp_grad_device(kpsi_ctx* c, const float* dparams, int64_t n, const double* m, const double* ck,
                                  const double* cj, const double* phi, const uint8_t* label, float* partial,
                                  int nbmax, double* g, bool w2h_current = false) {
  MlpArgs a = mlp_args(c, n, m, ck, cj, phi);
  a.label = label;
  a.params = dparams;
  if (!w2h_current || !c->mlp_w2h)
    if (hipError_t e = prep_w2h(c, dparams)) return e;
  a.w2h = c->mlp_w2h;
  a.partial = partial;
  const int64_t tiles = (n + 63) / 64;
  const int nb = (int)std::min<int64_t>(tiles, nbmax);
  a.per_block = (tiles + nb - 1) / nb * 64;
  hipError_t e = launch_mlp_grad(a, nb, c->stream);
  if (e != hipSuccess) return e;
  return launch_mlp_reduce(partial, nb, MLP_NV, 1.0 / (double)n, g, c->stream);
}

kpsi_status kpsi_mlp_grad(kpsi_ctx* c, const float* params, int64_t n, const double* m, const double* ck,
                          const double* cj, const double* phi, const uint8_t* label, double* grad, double* loss) {
  if (!c) return KPSI_E_ARG;
  if (!params || n <= 0 || !mlp_obs_ok(m, ck, cj, phi) || !label || !grad) return fail(c, KPSI_E_ARG, "bad arguments");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set (kinematics needed)");
  hipSetDevice(c->device);
  const int nbmax = 512;
  float *dp = nullptr, *part = nullptr;
  double* g = nullptr;
  auto cleanup = [&]() { if (dp) hipFree(dp); if (part) hipFree(part); if (g) hipFree(g); };
  if (hipMalloc(&dp, MLP_NP * sizeof(float)) || hipMalloc(&part, (size_t)(MLP_NP + 1) * nbmax * sizeof(float)) ||
      hipMalloc(&g, (MLP_NP + 1) * sizeof(double))) {
    cleanup();
    return fail(c, KPSI_E_OOM, "network buffers");
  }
  std::vector<double> h(MLP_NP + 1);
  hipError_t e = hipMemcpyAsync(dp, params, MLP_NP * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = mlp_grad_device(c, dp, n, m, ck, cj, phi, label, part, nbmax, g);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), g, (MLP_NP + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  cleanup();
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "network gradient: %s", hipGetErrorString(e));
  for (int i = 0; i < MLP_NP; ++i) grad[i] = h[i];
  if (loss) *loss = h[MLP_NP];
  return KPSI_OK;
}

kpsi_status kpsi_mlp_train(kpsi_ctx* c, float* params, int64_t n, const double* m, const double* ck,
                           const double* cj, const double* phi, const uint8_t* label, const kpsi_mlp_options* o,
                           double* loss) {
  if (!c) return KPSI_E_ARG;
  if (!params || n <= 0 || !mlp_obs_ok(m, ck, cj, phi) || !label || !o || o->epochs < 0 || o->batch < 64)
    return fail(c, KPSI_E_ARG, "bad arguments");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set (kinematics needed)");
  hipSetDevice(c->device);
  // at most one block per compute unit: a batch of 32768 events then runs two 64-event tiles per
  // block, which halves the weight staging and the block records against one tile per block
  // (38.4 against 42.8 us per training step; four tiles per block, on half the units: 47.5 us)
  const int nbmax = c->n_cu > 0 ? c->n_cu : 256;
  float *dp = nullptr, *mm = nullptr, *vv = nullptr, *part = nullptr;
  double* g = nullptr;
  auto cleanup = [&]() {
    for (void* p : {(void*)dp, (void*)mm, (void*)vv, (void*)part, (void*)g}) if (p) hipFree(p);
  };
  if (hipMalloc(&dp, MLP_NP * sizeof(float)) || hipMalloc(&mm, MLP_NP * sizeof(float)) ||
      hipMalloc(&vv, MLP_NP * sizeof(float)) || hipMalloc(&part, (size_t)(MLP_NP + 1) * nbmax * sizeof(float)) ||
      hipMalloc(&g, (MLP_NP + 1) * sizeof(double))) {
    cleanup();
    return fail(c, KPSI_E_OOM, "network buffers");
  }
  hipError_t e = hipMemcpyAsync(dp, params, MLP_NP * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(mm, 0, MLP_NP * sizeof(float), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(vv, 0, MLP_NP * sizeof(float), c->stream);
  const int64_t B = o->batch;
  const int64_t nbatch = (n + B - 1) / B;
  int64_t step = 0;
  double last_loss = 0.0;
  for (int ep = 0; ep < o->epochs && e == hipSuccess; ++ep) {
    double eloss = 0.0;
    for (int64_t b = 0; b < nbatch && e == hipSuccess; ++b) {
      const int64_t off = b * B, cnt = std::min(B, n - off);
      e = mlp_grad_device(c, dp, cnt, m + off, ck + off, cj + off, phi + off, label + off, part, nbmax, g, step > 0);
      ++step;
      const float c1 = (float)(1.0 / (1.0 - std::pow(o->beta1, (double)step)));
      const float c2 = (float)(1.0 / (1.0 - std::pow(o->beta2, (double)step)));
      if (e == hipSuccess)
        e = launch_adam(dp, mm, vv, g, MLP_NP, (float)o->lr, (float)o->beta1, (float)o->beta2, (float)o->eps, c1, c2,
                        c->mlp_w2h, c->stream);
      if (ep == o->epochs - 1 && e == hipSuccess) {
        double lb = 0.0;
        e = hipMemcpyAsync(&lb, g + MLP_NP, sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        eloss += lb * (double)cnt;
      }
    }
    if (ep == o->epochs - 1) last_loss = eloss / (double)n;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(params, dp, MLP_NP * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  cleanup();
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "network training: %s", hipGetErrorString(e));
  if (loss) *loss = last_loss;
  return KPSI_OK;
}

static hipError_t mlp_eval_device(kpsi_ctx* c, const float* dparams, int64_t n, const double* m, const double* ck,
                                  const double* cj, const double* phi, double* out) {
  MlpArgs a = mlp_args(c, n, m, ck, cj, phi);
  a.params = dparams;
  a.out = out;
  if (hipError_t e = prep_w2h(c, dparams)) return e;
  a.w2h = c->mlp_w2h;
  const int64_t tiles = (n + 63) / 64;
  const int nb = (int)std::min<int64_t>(tiles, 2048);
  a.per_block = (tiles + nb - 1) / nb * 64;
  return launch_mlp_eval(a, nb, c->stream);
}

kpsi_status kpsi_mlp_eval(kpsi_ctx* c, const float* params, int64_t n, const double* m, const double* ck,
                          const double* cj, const double* phi, double* out) {
  if (!c) return KPSI_E_ARG;
  if (!params || n <= 0 || !mlp_obs_ok(m, ck, cj, phi) || !out) return fail(c, KPSI_E_ARG, "bad arguments");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set (kinematics needed)");
  hipSetDevice(c->device);
  float* dp = nullptr;
  if (hipMalloc(&dp, MLP_NP * sizeof(float)) != hipSuccess) return fail(c, KPSI_E_OOM, "network parameters");
  hipError_t e = hipMemcpyAsync(dp, params, MLP_NP * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = mlp_eval_device(c, dp, n, m, ck, cj, phi, out);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(dp);
  if (e != hipSuccess) return fail(c, KPSI_E_HIP, "network evaluation: %s", hipGetErrorString(e));
  return KPSI_OK;
}

kpsi_status kpsi_set_efficiency_mlp(kpsi_ctx* c, const float* params) {
  if (!c) return KPSI_E_ARG;
  if (!params) return fail(c, KPSI_E_ARG, "params is NULL");
  if (c->set[1].n <= 0) return fail(c, KPSI_E_STATE, "load the normalisation set first");
  hipSetDevice(c->device);
  const int64_t n = c->set[1].n;
  double* vals = nullptr;
  if (hipMalloc(&vals, n * sizeof(double)) != hipSuccess) return fail(c, KPSI_E_OOM, "efficiency values");
  kpsi_status st = kpsi_mlp_eval(c, params, n, c->set[1].obs[0], c->set[1].obs[1], c->set[1].obs[2],
                                 c->set[1].obs[3], vals);
  if (!st) st = eps_from_device_f64(c, vals, n);
  hipFree(vals);
  return st;
}

kpsi_status kpsi_set_norm_cache(kpsi_ctx* c, int mode) {
  if (!c) return KPSI_E_ARG;
  if (mode < 0 || mode > 2) return fail(c, KPSI_E_ARG, "cache mode must be 0, 1 or 2");
  c->cache_mode = mode;
  invalidate_cache(c);
  return KPSI_OK;
}

kpsi_status kpsi_norm_cache_stats(const kpsi_ctx* c, int64_t* builds, int64_t* hits, double* last_build_ms) {
  if (!c) return KPSI_E_ARG;
  if (builds) *builds = c->cache_builds;
  if (hits) *hits = c->cache_hits;
  if (last_build_ms) *last_build_ms = c->cache_build_ms;
  return KPSI_OK;
}

kpsi_status kpsi_fit_fractions(kpsi_ctx* c, const double* params, double* ff, double* ff_sum) {
  if (!c) return KPSI_E_ARG;
  if (!params || !ff) return fail(c, KPSI_E_ARG, "NULL argument");
  if (!c->has_model) return fail(c, KPSI_E_STATE, "no model set");
  if (c->set[1].n <= 0) return fail(c, KPSI_E_STATE, "no normalisation events loaded");
  for (int i = 0; i < c->nparams; ++i)
    if (!std::isfinite(params[i])) return fail(c, KPSI_E_ARG, "parameter %d is not finite", i);
  hipSetDevice(c->device);
  Gram g;
  kpsi_status st = gram_build(c, params, false, false, g);
  if (st) return st;
  const std::vector<double> cv = component_couplings(c, params);
  const int n = g.ncomp;
  // Re sum_{k,l in K} c_k conj(c_l) I_kl over a component set K
  auto quad = [&](int k0, int k1) {
    double v = 0.0;
    for (int k = k0; k < k1; ++k)
      for (int l = k0; l < k1; ++l) {
        const double ir = g.I[2 * ((size_t)k * n + l)], ii = g.I[2 * ((size_t)k * n + l) + 1];
        const double pr = cv[2 * k] * cv[2 * l] + cv[2 * k + 1] * cv[2 * l + 1];   // c_k conj(c_l)
        const double pi = cv[2 * k + 1] * cv[2 * l] - cv[2 * k] * cv[2 * l + 1];
        v += pr * ir - pi * ii;
      }
    return v;
  };
  const double den = quad(0, n);
  if (!(den > 0.0)) return fail(c, KPSI_E_NONFINITE, "phase-space integral of the density is %g", den);
  double tot = 0.0;
  for (size_t i = 0; i < c->res.size(); ++i) {
    int k0, nk;
    components_of(c, i, &k0, &nk);
    ff[i] = quad(k0, k0 + nk) / den;
    tot += ff[i];
  }
  if (ff_sum) *ff_sum = tot;
  return KPSI_OK;
}

kpsi_status kpsi_set_events_per_thread(kpsi_ctx* c, int ept) {
  if (!c || ept < 0 || ept > 1024) return KPSI_E_ARG;
  c->ept_override = ept;
  return KPSI_OK;
}

}  // extern "C"

namespace kpsi {
hipError_t exclusive_scan_int(const int* in, int* out, int64_t n, void* tmp, size_t* tmp_bytes, hipStream_t st) {
  return hipcub::DeviceScan::ExclusiveSum(tmp, *tmp_bytes, in, out, (int)n, st);
}
}  // namespace kpsi

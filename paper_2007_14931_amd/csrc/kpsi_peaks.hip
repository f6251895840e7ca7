// Attainable-peak microbenchmarks of the device the library runs on: the rates that bound the
// likelihood kernels (FP32 and FP64 fused multiply-add issue without packed instructions, the
// FP32 reciprocal unit, and device-memory streaming).  Each kernel is a register-resident loop
// of independent chains; the result is stored only under a data-dependent condition that never
// holds, so the loop is not removed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpsi.h"

namespace {

constexpr int CHAINS = 8;
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__global__ __launch_bounds__(256) void fma_loop(T a, T b, int iters, T* sink) {
  T x[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) x[c] = a + T(c) * b + T(threadIdx.x) * T(1e-7);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = fma_(x[c], a, b);
  }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += x[c];
  if (s == T(-12345.0)) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void rcp_loop(float a, int iters, float* sink) {
  float x[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) x[c] = a + 0.01f * c + 1e-6f * threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = __builtin_amdgcn_rcpf(x[c]);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += x[c];
  if (s == -12345.0f) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void copy_kernel(const f4_t* __restrict__ src, f4_t* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Milliseconds of the second of two launches of f on stream st.
template <typename F>
hipError_t time_launch(F f, hipStream_t st, float* ms) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) { (void)hipEventDestroy(e0); return e; }
  f();
  (void)hipEventRecord(e0, st);
  f();
  (void)hipEventRecord(e1, st);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

extern "C" kpsi_status kpsi_measure_peaks(int device, kpsi_peaks* out) {
  if (!out) return KPSI_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || device < 0 || device >= ndev) return KPSI_E_HIP;
  if (hipSetDevice(device) != hipSuccess) return KPSI_E_HIP;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    return KPSI_E_HIP;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return KPSI_E_HIP;
  const int blocks = cus * 16, threads = 256;
  const int iters = 4096;
  const double lanes = (double)blocks * threads;
  double* sink = nullptr;
  f4_t *src = nullptr, *dst = nullptr;
  const int64_t n4 = (int64_t)1 << 26;   // 1 GiB per buffer
  kpsi_status rc = KPSI_OK;
  float ms = 0.f;
  if (hipMalloc(&sink, (size_t)blocks * threads * sizeof(double)) != hipSuccess ||
      hipMalloc(&src, (size_t)n4 * sizeof(f4_t)) != hipSuccess ||
      hipMalloc(&dst, (size_t)n4 * sizeof(f4_t)) != hipSuccess) {
    rc = KPSI_E_OOM;
  }
  if (!rc && time_launch([&] { hipLaunchKernelGGL(fma_loop<float>, dim3(blocks), dim3(threads), 0, st, 0.999f, 1e-3f,
                                                  iters, (float*)sink); }, st, &ms) != hipSuccess)
    rc = KPSI_E_HIP;
  if (!rc) out->fp32_fma_tflops = 2.0 * CHAINS * iters * lanes / (ms * 1e-3) / 1e12;
  if (!rc && time_launch([&] { hipLaunchKernelGGL(fma_loop<double>, dim3(blocks), dim3(threads), 0, st, 0.999, 1e-3,
                                                  iters, sink); }, st, &ms) != hipSuccess)
    rc = KPSI_E_HIP;
  if (!rc) out->fp64_fma_tflops = 2.0 * CHAINS * iters * lanes / (ms * 1e-3) / 1e12;
  if (!rc && time_launch([&] { hipLaunchKernelGGL(rcp_loop, dim3(blocks), dim3(threads), 0, st, 1.5f, iters / 4,
                                                  (float*)sink); }, st, &ms) != hipSuccess)
    rc = KPSI_E_HIP;
  if (!rc) out->fp32_rcp_tops = (double)CHAINS * (iters / 4) * lanes / (ms * 1e-3) / 1e12;
  if (!rc && hipMemsetAsync(src, 0, (size_t)n4 * sizeof(f4_t), st) != hipSuccess) rc = KPSI_E_HIP;
  if (!rc && time_launch([&] { hipLaunchKernelGGL(copy_kernel, dim3(cus * 32), dim3(256), 0, st, src, dst, n4); }, st,
                         &ms) != hipSuccess)
    rc = KPSI_E_HIP;
  if (!rc) out->copy_gbs = 2.0 * (double)n4 * sizeof(f4_t) / (ms * 1e-3) / 1e9;
  (void)hipStreamSynchronize(st);
  if (sink) (void)hipFree(sink);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  (void)hipStreamDestroy(st);
  return rc;
}

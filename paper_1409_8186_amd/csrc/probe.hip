// Device throughput probes: the FP64 rates the vector ALUs and the matrix
// cores reach on this device, and the device-to-device copy bandwidth, so that
// kernel rates can be reported against measured as well as published peaks.
// Nothing here is part of the scattering method.
#include "common.h"

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int FMA_CHAINS = 16;    // independent FMA chains per thread
constexpr int FMA_ITERS = 4096;
constexpr int MFMA_CHAINS = 8;    // independent accumulators per wave
constexpr int MFMA_ITERS = 1024;
constexpr int BLOCKS_PER_CU = 8;

__global__ __launch_bounds__(PROBE_THREADS) void k_probe_fma(double* out, double b, double c) {
  double acc[FMA_CHAINS];
#pragma unroll
  for (int k = 0; k < FMA_CHAINS; ++k) acc[k] = 1.0 + 1e-3 * (threadIdx.x + k);
  for (int it = 0; it < FMA_ITERS; ++it) {
#pragma unroll
    for (int k = 0; k < FMA_CHAINS; ++k) acc[k] = fma(acc[k], b, c);
  }
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < FMA_CHAINS; ++k) t += acc[k];
  out[(int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = t;
}

typedef double probe_d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(PROBE_THREADS) void k_probe_mfma(double* out, double a0, double b0) {
  probe_d4 acc[MFMA_CHAINS];
#pragma unroll
  for (int k = 0; k < MFMA_CHAINS; ++k) acc[k] = probe_d4{0.0, 0.0, 0.0, 0.0};
  const double a = a0 * (1.0 + 1e-3 * threadIdx.x), b = b0;
  for (int it = 0; it < MFMA_ITERS; ++it) {
#pragma unroll
    for (int k = 0; k < MFMA_CHAINS; ++k)
      acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  }
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < MFMA_CHAINS; ++k) t += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = t;
}

__global__ __launch_bounds__(PROBE_THREADS) void k_probe_copy(const double2* __restrict__ src,
                                                              double2* __restrict__ dst,
                                                              int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * PROBE_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

int n_compute_units() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return ncu;
}

}  // namespace

extern "C" size_t mudiff_probe_workspace_size(int kind, size_t bytes) {
  const int ncu = n_compute_units();
  if (ncu <= 0) return 0;
  const size_t per_thread = (size_t)ncu * BLOCKS_PER_CU * PROBE_THREADS * sizeof(double);
  if (kind == MUDIFF_PROBE_FP64_FMA || kind == MUDIFF_PROBE_FP64_MFMA) return align256(per_thread);
  if (kind == MUDIFF_PROBE_COPY) return 2 * align256(bytes / 16 * 16);
  return 0;
}

extern "C" int mudiff_probe(int kind, size_t bytes, void* workspace, size_t ws_bytes, double* rate,
                            void* stream) {
  if (!workspace || !rate) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (kind < MUDIFF_PROBE_FP64_FMA || kind > MUDIFF_PROBE_COPY)
    return fail(MUDIFF_ERR_INVALID, "unknown probe kind");
  if (kind == MUDIFF_PROBE_COPY && bytes < 16) return fail(MUDIFF_ERR_INVALID, "copy probe needs bytes >= 16");
  const size_t need = mudiff_probe_workspace_size(kind, bytes);
  if (need == 0) return fail(MUDIFF_ERR_DEVICE, "no device");
  if (ws_bytes < need) return fail(MUDIFF_ERR_NOMEM, "probe workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int ncu = n_compute_units();
  const unsigned blocks = (unsigned)(ncu * BLOCKS_PER_CU);
  double* out = (double*)workspace;
  const int64_t n16 = (int64_t)(bytes / 16);
  const double2* src = (const double2*)workspace;
  double2* dst = (double2*)((char*)workspace + align256(n16 * 16));
  auto launch = [&]() {
    if (kind == MUDIFF_PROBE_FP64_FMA)
      hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(PROBE_THREADS), 0, s, out, 0.999, 1e-3);
    else if (kind == MUDIFF_PROBE_FP64_MFMA)
      hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(PROBE_THREADS), 0, s, out, 1e-3, 0.5);
    else
      hipLaunchKernelGGL(k_probe_copy, dim3(blocks * 4), dim3(PROBE_THREADS), 0, s, src, dst, n16);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MUDIFF_ERR_DEVICE, "hipEventCreate");
  }
  constexpr int REPS = 3;
  launch();  // warm-up
  hipError_t e = hipEventRecord(e0, s);
  for (int r = 0; r < REPS && e == hipSuccess; ++r) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(MUDIFF_ERR_DEVICE, std::string("probe: ") + hipGetErrorString(e));
  const double sec = ms * 1e-3 / REPS;
  const double threads = (double)blocks * PROBE_THREADS;
  if (kind == MUDIFF_PROBE_FP64_FMA) {
    *rate = threads * FMA_ITERS * FMA_CHAINS * 2.0 / sec / 1e12;
  } else if (kind == MUDIFF_PROBE_FP64_MFMA) {
    const double waves = threads / 64.0;
    *rate = waves * MFMA_ITERS * MFMA_CHAINS * (16.0 * 16.0 * 4.0 * 2.0) / sec / 1e12;
  } else {
    *rate = 2.0 * (double)n16 * 16.0 / sec / 1e9;
  }
  return MUDIFF_OK;
}

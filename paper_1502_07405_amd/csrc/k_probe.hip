// Machine-peak probes that the roofline figures are checked against: a
// device-to-device copy (HBM), a loop of independent FP64 fused
// multiply-adds (vector ALU) and a loop of FP64 matrix-core instructions
// (16 x 16 x 4), each timed with HIP events, best of several runs.
#include "kernels.hpp"

namespace hssmf {

namespace {
typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kProbeChains = 8;   // independent FMA chains per thread
constexpr int kProbeAcc = 4;      // independent matrix-core accumulators per wavefront

// one 16-byte element per thread; the grid covers n exactly
__global__ __launch_bounds__(256) void probe_copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst,
                                                         int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// a <- a * m + c on kProbeChains independent values; m and c arrive at run
// time so the loop cannot be folded, and the result is stored
__global__ __launch_bounds__(256) void probe_fma_kernel(double* __restrict__ out, int iters, double m, double c) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double a[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = 1e-3 * (double)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = fma(a[k], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += a[k];
  out[g] = s;
}

// kProbeAcc independent 16 x 16 x 4 FP64 matrix-core products per step
__global__ __launch_bounds__(256) void probe_mfma_kernel(double* __restrict__ out, int iters, double x) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double a = x * (double)(threadIdx.x & 63), b = x / (1.0 + (double)(threadIdx.x & 63));
  dbl4 acc[kProbeAcc];
#pragma unroll
  for (int k = 0; k < kProbeAcc; ++k) acc[k] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kProbeAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[g] = s;
}

// best (shortest) of reps timed launches, in ms
template <class F>
float best_ms(hipStream_t s, int reps, F launch) {
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  float best = 0.0f;
  launch();   // warm-up
  for (int r = 0; r < reps; ++r) {
    HIP_CHECK(hipEventRecord(e0, s));
    launch();
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (r == 0 || ms < best) best = ms;
  }
  HIP_CHECK(hipEventDestroy(e0));
  HIP_CHECK(hipEventDestroy(e1));
  return best;
}

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) { HIP_CHECK(hipMalloc(&p, bytes)); }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

void measure_peaks(hipStream_t s, double* hbm_gbps, double* valu_tflops, double* mfma_tflops) {
  int dev = 0, cus = 0;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int reps = 5;
  // copy: 512 MiB each way, larger than the last-level cache
  const int64_t n = (int64_t)1 << 25;   // 16-byte elements
  DevBuf src(n * sizeof(double2)), dst(n * sizeof(double2));
  HIP_CHECK(hipMemsetAsync(src.p, 0, n * sizeof(double2), s));
  const unsigned cblocks = (unsigned)((n + 255) / 256);
  const float cms = best_ms(s, reps, [&]() {
    hipLaunchKernelGGL(probe_copy_kernel, dim3(cblocks), dim3(256), 0, s, (const double2*)src.p, (double2*)dst.p, n);
    HIP_CHECK(hipGetLastError());
  });
  *hbm_gbps = 2.0 * (double)n * sizeof(double2) / (cms * 1e-3) / 1e9;
  // compute loops: eight workgroups of 256 threads per compute unit
  const unsigned blocks = (unsigned)std::max(cus, 1) * 8;
  DevBuf out((size_t)blocks * 256 * sizeof(double));
  const int fiters = 1 << 14;
  const float fms = best_ms(s, reps, [&]() {
    hipLaunchKernelGGL(probe_fma_kernel, dim3(blocks), dim3(256), 0, s, (double*)out.p, fiters, 0.999999, 1e-7);
    HIP_CHECK(hipGetLastError());
  });
  *valu_tflops = 2.0 * kProbeChains * (double)fiters * blocks * 256 / (fms * 1e-3) / 1e12;
  const int miters = 1 << 12;
  const float mms = best_ms(s, reps, [&]() {
    hipLaunchKernelGGL(probe_mfma_kernel, dim3(blocks), dim3(256), 0, s, (double*)out.p, miters, 1e-3);
    HIP_CHECK(hipGetLastError());
  });
  // 2 x 16 x 16 x 4 flops per wavefront instruction, four wavefronts per workgroup
  *mfma_tflops = 2.0 * 16 * 16 * 4 * kProbeAcc * (double)miters * blocks * 4 / (mms * 1e-3) / 1e12;
  HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace hssmf

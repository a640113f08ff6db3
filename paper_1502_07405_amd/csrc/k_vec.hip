// Vector kernels of the outer solvers: CSR sparse matrix-vector product,
// dot products with device-resident results, axpy with device scalars, the
// adjoint's entrywise gradient.
#include "kernels.hpp"
#include "vec.hpp"

namespace hssmf {

// y = alpha A x + beta y (one row per thread, CSR of the caller's matrix)
__global__ void spmv_kernel(const int64_t* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                            const int64_t* __restrict__ vidx, const double* __restrict__ x, double* y, int n,
                            double alpha, double beta) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc += v[vidx ? vidx[e] : e] * x[ci[e]];
  y[i] = alpha * acc + (beta == 0.0 ? 0.0 : beta * y[i]);
}

void launch_spmv(const int64_t* rp, const int* ci, const double* v, const int64_t* vidx, const double* x, double* y,
                 int n, double alpha, double beta, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(spmv_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rp, ci, v, vidx, x, y, n, alpha, beta);
  HIP_CHECK(hipGetLastError());
}

// two-pass dot product: 512 partial sums, then one workgroup adds them in a
// fixed order (bitwise repeatable)
__global__ __launch_bounds__(256) void dot_partial_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                          int n, double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) acc += a[i] * b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void dot_final_kernel(const double* __restrict__ part, int np, double* out,
                                                        int sqrt_out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt_out ? sqrt(red[0]) : red[0];
}

void launch_dot(const double* a, const double* b, int n, double* part, double* out, int sqrt_out, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotParts), dim3(256), 0, s, a, b, n, part);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, part, kDotParts, out, sqrt_out);
  HIP_CHECK(hipGetLastError());
}

// y = y + sgn * (*alpha) * x   (alpha may be null: 1), or y = x * (1 / *alpha) when inv
__global__ void axpy_kernel(double* y, const double* __restrict__ x, int n, const double* alpha, double sgn, int inv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = alpha ? *alpha : 1.0;
  if (inv) y[i] = x[i] / a;
  else y[i] += sgn * a * x[i];
}

void launch_axpy(double* y, const double* x, int n, const double* alpha, double sgn, int inv, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpy_kernel, dim3((n + 255) / 256), dim3(256), 0, s, y, x, n, alpha, sgn, inv);
  HIP_CHECK(hipGetLastError());
}

// gather y[i] = x[map[i]]
__global__ void gather_kernel(double* y, const double* __restrict__ x, const int* __restrict__ map, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[map[i]];
}

void launch_gather(double* y, const double* x, const int* map, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_kernel, dim3((n + 255) / 256), dim3(256), 0, s, y, x, map, n);
  HIP_CHECK(hipGetLastError());
}

// dL/dval[e] = -lambda[row(e)] * x[col(e)]
// sum of squares of each segment [off[s], off[s+1]) of x: one workgroup per
// segment, fixed reduction order
__global__ __launch_bounds__(256) void seg_sumsq_kernel(const double* __restrict__ x,
                                                        const int64_t* __restrict__ off, double* out) {
  __shared__ double red[256];
  const int64_t b = off[blockIdx.x], e = off[blockIdx.x + 1];
  double acc = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) acc += x[i] * x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

void launch_seg_sumsq(const double* x, const int64_t* off, int nseg, double* out, hipStream_t s) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(seg_sumsq_kernel, dim3(nseg), dim3(256), 0, s, x, off, out);
  HIP_CHECK(hipGetLastError());
}

__global__ void adjoint_grad_kernel(const int* __restrict__ row, const int* __restrict__ col,
                                    const double* __restrict__ lam, const double* __restrict__ x, double* g,
                                    int64_t nnz) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    g[e] = -lam[row[e]] * x[col[e]];
}

void launch_adjoint_grad(const int* row, const int* col, const double* lam, const double* x, double* g, int64_t nnz,
                         hipStream_t s) {
  if (nnz <= 0) return;
  int64_t b = (nnz + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(adjoint_grad_kernel, dim3((unsigned)b), dim3(256), 0, s, row, col, lam, x, g, nnz);
  HIP_CHECK(hipGetLastError());
}

}  // namespace hssmf

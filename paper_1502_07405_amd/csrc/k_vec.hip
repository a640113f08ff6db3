// Vector kernels of the outer solvers: CSR sparse matrix-vector product,
// dot products with device-resident results, axpy with device scalars, the
// Arnoldi and Givens steps of GMRES, the adjoint's entrywise gradient.
#include <algorithm>

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

// complex values (re, im pairs, complex CSR order) into the real-equivalent
// matrix's values: row i's entries a + ib give [a, -b] in row 2i and [b, a]
// in row 2i + 1, each row of the real form holding two values per complex
// entry; one thread per complex row
__global__ void zexpand_kernel(double* __restrict__ out, const double* __restrict__ z,
                               const int64_t* __restrict__ zrow, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t e0 = zrow[i], len = zrow[i + 1] - e0;
  double* r0 = out + 4 * e0;        // row 2i
  double* r1 = r0 + 2 * len;        // row 2i + 1
  for (int64_t t = 0; t < len; ++t) {
    const double re = z[2 * (e0 + t)], im = z[2 * (e0 + t) + 1];
    r0[2 * t] = re;
    r0[2 * t + 1] = -im;
    r1[2 * t] = im;
    r1[2 * t + 1] = re;
  }
}

void launch_zexpand(double* out, const double* z, const int64_t* zrow, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zexpand_kernel, dim3((n + 255) / 256), dim3(256), 0, s, out, z, zrow, n);
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------- GMRES ------

GmDev gm_dev(double* base) {
  GmDev d;
  d.H = base;
  base += (int64_t)(kGmMaxRestart + 1) * kGmMaxRestart;
  d.cs = base;
  base += kGmMaxRestart + 2;
  d.sn = base;
  base += kGmMaxRestart + 2;
  d.g = base;
  base += kGmMaxRestart + 2;
  d.y = base;
  base += kGmMaxRestart + 2;
  d.hcol = base;
  return d;
}

__global__ void gm_start_kernel(double* v0, const double* __restrict__ w, int n, double beta, GmDev d, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v0[i] = w[i] / beta;
  if (i <= m) d.g[i] = i == 0 ? beta : 0.0;
}

void launch_gm_start(double* v0, const double* w, int n, double beta, GmDev d, int m, hipStream_t s) {
  const int cnt = std::max(n, m + 1);
  hipLaunchKernelGGL(gm_start_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, v0, w, n, beta, d, m);
  HIP_CHECK(hipGetLastError());
}

// the Givens step of GMRES for Hessenberg column j (h[0..j+1]): rotations
// 0..j-1 applied in order, the new rotation zeroing h[j+1], the column stored
// to H, g rotated; then the estimate |g[j+1]| and the tag to the host
__device__ void givens_step(double* h, int j, GmDev d, GmStatus* status, int tag) {
  for (int i = 0; i < j; ++i) {
    const double t = d.cs[i] * h[i] + d.sn[i] * h[i + 1];
    h[i + 1] = -d.sn[i] * h[i] + d.cs[i] * h[i + 1];
    h[i] = t;
  }
  const double den = hypot(h[j], h[j + 1]);
  d.cs[j] = h[j] / den;
  d.sn[j] = h[j + 1] / den;
  h[j] = den;
  h[j + 1] = 0.0;
  for (int i = 0; i <= j; ++i) d.H[i + (int64_t)j * (kGmMaxRestart + 1)] = h[i];
  const double gj = d.g[j];
  d.g[j + 1] = -d.sn[j] * gj;
  d.g[j] = d.cs[j] * gj;
  __hip_atomic_store(&status->est, fabs(d.g[j + 1]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&status->tag, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// sum over a 1024-thread workgroup, the same bits in every thread: butterfly
// inside each wavefront, then every thread adds the 16 wavefront sums in
// order.  red alternates between two buffers, so one barrier per call
// suffices.
__device__ double block_sum(double v, double (*red)[16], int& par) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[par][threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < 16; ++w) s += red[par][w];
  par ^= 1;
  return s;
}

template <int PER>
__global__ __launch_bounds__(1024) void arnoldi_kernel(const double* __restrict__ win, double* V, int n, int j,
                                                        GmDev d, GmStatus* status, int tag) {
  __shared__ double red[2][16];
  __shared__ double hl[kGmMaxRestart + 2];
  int par = 0;
  const int tid = threadIdx.x;
  double w[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = tid + 1024 * q;
    w[q] = i < n ? win[i] : 0.0;
  }
  // modified Gram-Schmidt: h_i = <w, v_i>, then w -= h_i v_i, i = 0..j
  for (int k = 0; k <= j; ++k) {
    const double* vk = V + (int64_t)k * n;
    double v[PER];
    double p = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tid + 1024 * q;
      v[q] = i < n ? vk[i] : 0.0;
      p += w[q] * v[q];
    }
    const double hk = block_sum(p, red, par);
#pragma unroll
    for (int q = 0; q < PER; ++q) w[q] -= hk * v[q];
    if (tid == 0) hl[k] = hk;
  }
  double p = 0.0;
#pragma unroll
  for (int q = 0; q < PER; ++q) p += w[q] * w[q];
  const double hn = sqrt(block_sum(p, red, par));
  double* vn = V + (int64_t)(j + 1) * n;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = tid + 1024 * q;
    if (i < n) vn[i] = w[q] / hn;
  }
  if (tid == 0) {
    hl[j + 1] = hn;
    givens_step(hl, j, d, status, tag);
  }
}

void launch_arnoldi(const double* w, double* V, int n, int j, GmDev d, GmStatus* status, int tag, hipStream_t s) {
  REQUIRE(n <= kArnoldiMaxN && j < kGmMaxRestart, HSSMF_EINVAL, "arnoldi: problem too large for one workgroup");
  const int per = (n + 1023) / 1024;
  if (per <= 4) hipLaunchKernelGGL(arnoldi_kernel<4>, dim3(1), dim3(1024), 0, s, w, V, n, j, d, status, tag);
  else if (per <= 8) hipLaunchKernelGGL(arnoldi_kernel<8>, dim3(1), dim3(1024), 0, s, w, V, n, j, d, status, tag);
  else hipLaunchKernelGGL(arnoldi_kernel<16>, dim3(1), dim3(1024), 0, s, w, V, n, j, d, status, tag);
  HIP_CHECK(hipGetLastError());
}

__global__ void givens_kernel(int j, GmDev d, GmStatus* status, int tag) {
  if (threadIdx.x == 0) givens_step(d.hcol, j, d, status, tag);
}

void launch_givens(int j, GmDev d, GmStatus* status, int tag, hipStream_t s) {
  REQUIRE(j < kGmMaxRestart, HSSMF_EINVAL, "givens: restart too large");
  hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, s, j, d, status, tag);
  HIP_CHECK(hipGetLastError());
}

// back substitution with the rotated Hessenberg matrix (one thread: k is at
// most the restart length)
__global__ void gm_solve_kernel(GmDev d, int k) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = d.g[i];
    for (int l = i + 1; l < k; ++l) s -= d.H[i + (int64_t)l * (kGmMaxRestart + 1)] * d.y[l];
    d.y[i] = s / d.H[i + (int64_t)i * (kGmMaxRestart + 1)];
  }
}

// out = x + sum_l y_l V(:, l), terms added in order of l
__global__ void gm_combine_kernel(double* out, const double* __restrict__ x, const double* __restrict__ V, int n, int k,
                                  GmDev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int l = 0; l < k; ++l) acc += d.y[l] * V[i + (int64_t)l * n];
  out[i] = acc;
}

void launch_gm_update(double* out, const double* x, const double* V, int n, int k, GmDev d, hipStream_t s) {
  hipLaunchKernelGGL(gm_solve_kernel, dim3(1), dim3(64), 0, s, d, k);
  if (n > 0) hipLaunchKernelGGL(gm_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, s, out, x, V, n, k, d);
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

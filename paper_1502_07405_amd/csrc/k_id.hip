// Column-pivoted Householder QR for the interpolative decomposition of
// Sec. 2.2, with the stopping rule of Sec. 5.4, for many problems at once.
//
// A problem is Y = S^T (d x m): the m candidates (rows of the node samples)
// are the columns.  Each problem is split over P workgroups that own 32
// candidates each, and every pivot step is one kernel launch, so the launch
// boundary is the only synchronization between the workgroups of a problem
// (no in-kernel grid barrier, nothing to spin on).  In step t every
// workgroup reads the partial maxima written by step t-1, picks the pivot
// (largest remaining 2-norm, ties to the lowest candidate index), forms the
// reflector from the pivot column in LDS, applies it to its own active
// candidates and recomputes their remaining norms from the updated columns.
// Columns never move: perm / ipos record the pivot order with the same
// interchanges a column-swapping QR would make, so R(i, j) of the
// factorization sits in row i of candidate perm[j].
#include "kernels.hpp"

namespace hssmf {

namespace {

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ int find_prob(const IDProb* __restrict__ p, int np, int wg) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (p[mid].wg0 <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// partial maximum of the active candidates' norms of one workgroup
__device__ void write_partial(const IDProb& q, int b, int parity, double* red, int* redi) {
  const int tid = threadIdx.x;
  double best = -1.0;
  int bi = 0x7fffffff;
  const int j = b * kIDCols + tid;
  if (tid < kIDCols && j < q.m && q.active[j]) { best = q.norms[j]; bi = j; }
  red[tid] = best;
  redi[tid] = bi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      double o = red[tid + off];
      int oi = redi[tid + off];
      if (o > red[tid] || (o == red[tid] && oi < redi[tid])) { red[tid] = o; redi[tid] = oi; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* sl = q.slots + ((size_t)parity * q.P + b) * 2;
    sl[0] = red[0];
    sl[1] = (double)redi[0];
  }
}

}  // namespace

__global__ __launch_bounds__(256) void id_init_kernel(const IDProb* __restrict__ probs, int np) {
  __shared__ double red[256];
  __shared__ int redi[256];
  const int pi = find_prob(probs, np, blockIdx.x);
  const IDProb q = probs[pi];
  const int b = blockIdx.x - q.wg0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j0 = b * kIDCols, j1 = min(q.m, j0 + kIDCols);
  // stage Y = S^T for this workgroup's candidates (reads coalesced along j)
  const int nj = j1 - j0;
  for (int64_t e = tid; e < (int64_t)nj * q.d; e += 256) {
    int jj = (int)(e % nj), kk = (int)(e / nj);
    q.W[kk + (int64_t)(j0 + jj) * q.d] = q.S[(j0 + jj) + (int64_t)kk * q.lds];
  }
  for (int j = j0 + tid; j < j1; j += 256) {
    q.perm[j] = j;
    q.ipos[j] = j;
    q.active[j] = 1;
  }
  __syncthreads();
  for (int j = j0 + wave; j < j1; j += 4) {
    const double* col = q.W + (int64_t)j * q.d;
    double ss = 0.0;
    for (int i = lane; i < q.d; i += 64) ss += col[i] * col[i];
    ss = wsum(ss);
    if (lane == 0) q.norms[j] = sqrt(ss);
  }
  if (b == 0 && tid == 0) {
    q.state[0] = (q.m == 0 || q.d == 0) ? 1 : 0;
    q.state[1] = 0;
    q.first[0] = 0.0;
  }
  __syncthreads();
  write_partial(q, b, 0, red, redi);
}

// NR: entries of a column each lane keeps in registers between the dot
// product and the update (columns up to 64 NR rows; longer columns are read
// twice)
template <int NR>
__global__ __launch_bounds__(256) void id_step_kernel(const IDProb* __restrict__ probs, const int* __restrict__ wgmap,
                                                      int t) {
  extern __shared__ double x[];           // pivot column, rows t..d-1
  __shared__ double red[256];
  __shared__ int redi[256];
  __shared__ double nloc[kIDCols];
  __shared__ double bc[1];
  const IDProb& q = probs[wgmap[blockIdx.x]];
  const int b = blockIdx.x - q.wg0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (q.state[0]) return;
  const int m = q.m, d = q.d;
  const int kmax = min(m, d);
  // pivot from the partial maxima of step t-1 (parallel reduction)
  {
    const double* sl = q.slots + (size_t)(t & 1) * q.P * 2;
    double v = -1.0;
    int c = 0x7fffffff;
    for (int w = tid; w < q.P; w += 256) {
      double vw = sl[2 * w];
      int cw = (int)sl[2 * w + 1];
      if (vw > v || (vw == v && cw < c)) { v = vw; c = cw; }
    }
    red[tid] = v;
    redi[tid] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) {
        double o = red[tid + off];
        int oi = redi[tid + off];
        if (o > red[tid] || (o == red[tid] && oi < redi[tid])) { red[tid] = o; redi[tid] = oi; }
      }
      __syncthreads();
    }
  }
  const double best = red[0];
  const int p = redi[0];
  const double first = (t == 0) ? best : q.first[0];
  const bool stop = (t >= kmax) || (t == 0 ? best <= 0.0 : best <= q.eps * first);
  if (stop) {
    if (b == 0 && tid == 0) {
      q.state[1] = (t == 0 && best <= 0.0) ? 0 : t;
      q.state[0] = 1;
    }
    return;
  }
  const double* colp = q.W + (int64_t)p * d;
  const double x0 = colp[t];
  const double alpha = (x0 >= 0.0) ? -best : best;
  if (b == 0 && tid == 0) {
    if (t == 0) q.first[0] = best;
    int qpos = q.ipos[p];
    int ct = q.perm[t];
    q.perm[t] = p;
    q.perm[qpos] = ct;
    q.ipos[p] = t;
    q.ipos[ct] = qpos;
  }
  if (tid == 0 && p / kIDCols == b) {
    q.active[p] = 0;
    q.alpha[t] = alpha;
  }
  const int len = d - t;
  for (int i = tid; i < len; i += 256) x[i] = colp[t + i];
  if (tid < kIDCols) nloc[tid] = -1.0;
  __syncthreads();
  if (tid == 0) {
    double v0 = x0 - alpha;
    double vtv = v0 * v0 + (best * best - x0 * x0);
    bc[0] = (vtv > 0.0 && best > 0.0) ? 2.0 / vtv : 0.0;
    x[0] = v0;
  }
  __syncthreads();
  const double tau = bc[0];
  const int j0 = b * kIDCols;
  for (int jj = wave; jj < kIDCols; jj += 4) {
    const int j = j0 + jj;
    if (j >= m || j == p || !q.active[j]) continue;
    double* col = q.W + (int64_t)j * d + t;
    double rc[NR];
    double dot = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = lane + 64 * r;
      rc[r] = (i < len) ? col[i] : 0.0;
      if (i < len) dot += x[i] * rc[r];
    }
    for (int i = lane + 64 * NR; i < len; i += 64) dot += x[i] * col[i];
    dot = wsum(dot) * tau;
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = lane + 64 * r;
      if (i < len) {
        const double y = rc[r] - dot * x[i];
        col[i] = y;
        if (i > 0) ss += y * y;
      }
    }
    for (int i = lane + 64 * NR; i < len; i += 64) {
      const double y = col[i] - dot * x[i];
      col[i] = y;
      ss += y * y;
    }
    ss = wsum(ss);
    if (lane == 0) nloc[jj] = sqrt(ss);   // exact recomputation, no downdating
  }
  __syncthreads();
  // partial maximum over this workgroup's candidates for step t+1
  if (tid == 0) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int jj = 0; jj < kIDCols; ++jj) {
      const int j = j0 + jj;
      if (j < m && j != p && q.active[j] && nloc[jj] > bv) { bv = nloc[jj]; bi = j; }
    }
    double* sl = q.slots + ((size_t)((t + 1) & 1) * q.P + b) * 2;
    sl[0] = bv;
    sl[1] = (double)bi;
  }
}

// R1 (k x k upper, pivot order) gathered from the untouched columns
__global__ void id_r1_kernel(const IDProb* __restrict__ probs) {
  const IDProb q = probs[blockIdx.y];
  const int k = q.state[1];
  const int64_t kk = (int64_t)k * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kk; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e % k), l = (int)(e / k);
    double v = 0.0;
    if (i == l) v = q.alpha[i];
    else if (i < l) v = q.W[i + (int64_t)q.perm[l] * q.d];
    q.R1[i + (int64_t)l * k] = v;
  }
}

// R2 (k x (m-k)) gathered into E's storage as a k x (m-k) block; the host
// then solves R1 X = R2 in place with the batched blocked triangular solve
// and transposes X into E
__global__ void id_r2_kernel(const IDProb* __restrict__ probs) {
  const IDProb q = probs[blockIdx.y];
  const int k = q.state[1];
  const int nrest = q.m - k;
  const int64_t tot = (int64_t)k * nrest;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e % k), c = (int)(e / k);
    q.W2[i + (int64_t)c * k] = q.W[i + (int64_t)q.perm[k + c] * q.d];
  }
}

void launch_id_init(const IDProb* p, int np, int total_wg, int max_d, hipStream_t s) {
  if (np <= 0 || total_wg <= 0) return;
  (void)max_d;
  hipLaunchKernelGGL(id_init_kernel, dim3(total_wg), dim3(256), 0, s, p, np);
  HIP_CHECK(hipGetLastError());
}

void launch_id_step(const IDProb* p, const int* wgmap, int total_wg, int t, int max_d, hipStream_t s) {
  if (total_wg <= 0) return;
  size_t lds = (size_t)std::max(max_d, 1) * sizeof(double);
  REQUIRE(lds <= 48 * 1024, HSSMF_ERANK, "interpolative decomposition: more than 6144 samples");
  if (max_d <= 64 * 4)
    hipLaunchKernelGGL(id_step_kernel<4>, dim3(total_wg), dim3(256), lds, s, p, wgmap, t);
  else if (max_d <= 64 * 10)
    hipLaunchKernelGGL(id_step_kernel<10>, dim3(total_wg), dim3(256), lds, s, p, wgmap, t);
  else
    hipLaunchKernelGGL(id_step_kernel<16>, dim3(total_wg), dim3(256), lds, s, p, wgmap, t);
  HIP_CHECK(hipGetLastError());
}

void launch_id_finish(const IDProb* p, int np, int max_m, hipStream_t s) {
  if (np <= 0 || max_m <= 0) return;
  int64_t kk = (int64_t)max_m * max_m;
  int64_t bx = (kk + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(id_r1_kernel, dim3((unsigned)bx, np), dim3(256), 0, s, p);
  hipLaunchKernelGGL(id_r2_kernel, dim3((unsigned)bx, np), dim3(256), 0, s, p);
  HIP_CHECK(hipGetLastError());
}

}  // namespace hssmf

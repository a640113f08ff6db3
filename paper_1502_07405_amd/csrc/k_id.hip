// Column-pivoted Householder QR for the interpolative decomposition of
// Sec. 2.2, with the stopping rule of Sec. 5.3, for many problems at once.
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

// H = I - tau v v^T applied to one candidate column (rows t.. in rc, the
// first NR * 64 of them, the rest streamed from col); writes the column back
// and the 2-norm of its rows t+1.. to *norm
template <int NR>
__device__ __forceinline__ void reflect(double (&rc)[NR], double* __restrict__ col, const double* __restrict__ x,
                                        double v0, double tau, int len, int lane, double* norm) {
  double dot = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    if (i < len) dot += ((i == 0) ? v0 : x[i]) * rc[r];
  }
  for (int i = lane + 64 * NR; i < len; i += 64) dot += x[i] * col[i];
  dot = wsum(dot) * tau;
  double ss = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    if (i < len) {
      const double y = rc[r] - dot * ((i == 0) ? v0 : x[i]);
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
  if (lane == 0) *norm = sqrt(ss);   // exact recomputation, no downdating
}

// One pivot step.  Each of the four wavefronts owns two of the workgroup's
// candidates and keeps rows t.. of both in registers (NR entries per lane;
// rows beyond 64 NR are streamed).  Every global load that does not depend
// on the pivot (state, partial maxima, first norm, the own columns) is
// issued at entry, so a step costs two dependent memory round trips: the
// partial maxima, then the pivot column.
template <int NR>
__global__ __launch_bounds__(256) void id_step_kernel(const IDProb* __restrict__ probs, const int2* __restrict__ wgmap,
                                                      int t) {
  extern __shared__ double x[];           // pivot column, rows t..d-1
  __shared__ double wred[4];
  __shared__ int wredi[4];
  __shared__ double nloc[kIDCols];
  const int2 wm = wgmap[blockIdx.x];
  const IDProb& q = probs[wm.x];
  const int b = wm.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = q.m, d = q.d;
  const int kmax = min(m, d);
  const int len = d - t;
  const int j0 = b * kIDCols;
  const int ja = j0 + wave, jb = j0 + wave + 4;
  // independent loads first
  const int done = q.state[0];
  double first = (t == 0) ? 0.0 : q.first[0];
  double sv = -1.0;
  int sc = 0x7fffffff;
  if (wave == 0) {
    const double* sl = q.slots + (size_t)(t & 1) * q.P * 2;
    for (int w = lane; w < q.P; w += 64) {
      const double vw = sl[2 * w];
      const int cw = (int)sl[2 * w + 1];
      if (vw > sv || (vw == sv && cw < sc)) { sv = vw; sc = cw; }
    }
  }
  double ra[NR], rb[NR];
  const bool hasa = ja < m, hasb = jb < m;
  const double* ca = q.W + (int64_t)ja * d + t;
  const double* cb = q.W + (int64_t)jb * d + t;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    ra[r] = (hasa && i < len) ? ca[i] : 0.0;
    rb[r] = (hasb && i < len) ? cb[i] : 0.0;
  }
  const bool acta = hasa && q.active[ja];
  const bool actb = hasb && q.active[jb];
  if (done) return;
  // pivot: largest partial maximum, ties to the lowest candidate index
  if (wave == 0) {
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(sv, off);
      const int oi = __shfl_xor(sc, off);
      if (o > sv || (o == sv && oi < sc)) { sv = o; sc = oi; }
    }
    if (lane == 0) { wred[0] = sv; wredi[0] = sc; }
  }
  __syncthreads();
  const double best = wred[0];
  const int p = wredi[0];
  if (t == 0) first = best;
  const bool stop = (t >= kmax) || (t == 0 ? best <= 0.0 : best <= q.eps * first);
  if (stop) {
    if (b == 0 && tid == 0) {
      q.state[1] = (t == 0 && best <= 0.0) ? 0 : t;
      q.state[0] = 1;
    }
    return;
  }
  const double* colp = q.W + (int64_t)p * d + t;
  for (int i = tid; i < len; i += 256) x[i] = colp[i];
  if (tid < kIDCols) nloc[tid] = -1.0;
  __syncthreads();
  const double x0 = x[0];
  const double alpha = (x0 >= 0.0) ? -best : best;
  const double v0 = x0 - alpha;
  const double vtv = v0 * v0 + (best * best - x0 * x0);
  const double tau = (vtv > 0.0 && best > 0.0) ? 2.0 / vtv : 0.0;
  if (tid == 0) {
    if (b == 0) {
      if (t == 0) q.first[0] = best;
      const int qpos = q.ipos[p];
      const int ct = q.perm[t];
      q.perm[t] = p;
      q.perm[qpos] = ct;
      q.ipos[p] = t;
      q.ipos[ct] = qpos;
    }
    if (p / kIDCols == b) {
      q.active[p] = 0;
      q.alpha[t] = alpha;
    }
  }
  // apply the reflector (v = x with v[0] = v0) to the own active candidates
  if (acta && ja != p) reflect<NR>(ra, q.W + (int64_t)ja * d + t, x, v0, tau, len, lane, &nloc[wave]);
  if (actb && jb != p) reflect<NR>(rb, q.W + (int64_t)jb * d + t, x, v0, tau, len, lane, &nloc[wave + 4]);
  __syncthreads();
  // partial maximum over this workgroup's candidates for step t+1
  if (tid == 0) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int jj = 0; jj < kIDCols; ++jj) {
      if (nloc[jj] > bv) { bv = nloc[jj]; bi = j0 + jj; }
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

void launch_id_step(const IDProb* p, const int2* wgmap, int total_wg, int t, int max_d, hipStream_t s) {
  if (total_wg <= 0) return;
  size_t lds = (size_t)std::max(max_d, 1) * sizeof(double);
  REQUIRE(lds <= 48 * 1024, HSSMF_ERANK, "interpolative decomposition: more than 6144 samples");
  hipEvent_t e0, e1;
  prof::ext(0, 0.0, &e0, &e1);   // timing hook (no-op when off); work is added per pass
  if (max_d <= 64 * 4)
    hipExtLaunchKernelGGL(id_step_kernel<4>, dim3(total_wg), dim3(256), lds, s, e0, e1, 0, p, wgmap, t);
  else if (max_d <= 64 * 10)
    hipExtLaunchKernelGGL(id_step_kernel<10>, dim3(total_wg), dim3(256), lds, s, e0, e1, 0, p, wgmap, t);
  else
    hipExtLaunchKernelGGL(id_step_kernel<16>, dim3(total_wg), dim3(256), lds, s, e0, e1, 0, p, wgmap, t);
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

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
  // own columns: only the active ones are read (a pivoted column is never
  // touched again); these loads wait for the flags, as the pivot column's
  // load waits for the partial maxima, so the chain gets no longer
  const bool acta = ja < m && q.active[ja];
  const bool actb = jb < m && q.active[jb];
  double ra[NR], rb[NR];
  const double* ca = q.W + (int64_t)ja * d + t;
  const double* cb = q.W + (int64_t)jb * d + t;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    ra[r] = (acta && i < len) ? ca[i] : 0.0;
    rb[r] = (actb && i < len) ? cb[i] : 0.0;
  }
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
  const bool stop = (t >= kmax) || (t == 0 ? best <= q.atol : best <= fmax(q.eps * first, q.atol));
  if (stop) {
    if (b == 0 && tid == 0) {
      q.state[1] = (t == 0 && best <= 0.0) ? 0 : t;
      q.state[0] = 1;
      // tell the host without a copy back: a plain store, visible system-wide
      if (q.hdone) __hip_atomic_store(q.hdone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
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

// ---------------------------------------------------------------------------
// Cooperative variant.  The whole grid is resident (cooperative launch), so
// the workgroups of one problem can wait for each other: each keeps its
// eight candidates in registers for the whole factorization (rows by
// absolute index, row = lane + 64 r), publishes only its best remaining
// candidate column and partial maximum per step (double-buffered by step
// parity), and waits for the step tags of the problem's other workgroups.
// A wait is bounded: after kSpinLimit polls it sets *err and the problem's
// workgroups leave, so the launch always ends.  Workgroup 0 of a
// problem alone keeps the pivot order (perm / ipos).
namespace {
constexpr unsigned kSpinLimit = 1u << 22;

// Only the partial maxima and the published candidate columns cross
// workgroups inside the launch.  They are written and read with agent-scope
// atomic accesses (coherent across the chip's L2 caches, no cache-wide
// writeback).  A workgroup publishes its candidate column, waits for those
// stores to complete, then writes its slot (norm, index) and last the step
// tag; readers poll the tags.
__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// reflector on a register-resident column: rows t..d-1 take part, v[t] = v0
template <int NR>
__device__ __forceinline__ void reflect_abs(double (&rc)[NR], const double* __restrict__ x, double v0, double tau,
                                            int t, int d, int lane, double* norm) {
  double dot = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    if (i >= t && i < d) dot += ((i == t) ? v0 : x[i]) * rc[r];
  }
  dot = wsum(dot) * tau;
  double ss = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    if (i >= t && i < d) {
      rc[r] -= dot * ((i == t) ? v0 : x[i]);
      if (i > t) ss += rc[r] * rc[r];
    }
  }
  ss = wsum(ss);
  if (lane == 0) *norm = sqrt(ss);
}

template <int NR, bool COH>
__device__ __forceinline__ void store_col(const double (&rc)[NR], double* __restrict__ dst, int r0, int d, int lane) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    if (i >= r0 && i < d) {
      if (COH) st_coh(dst + i, rc[r]);
      else dst[i] = rc[r];
    }
  }
}
}  // namespace

template <int NR>
__global__ __launch_bounds__(256) void id_coop_kernel(const IDProb* __restrict__ probs,
                                                      const int2* __restrict__ wgmap, int* err) {
  extern __shared__ double x[];   // pivot column by absolute row
  __shared__ double tile[kIDCols * 64];
  __shared__ double nloc[kIDCols];
  __shared__ double pbest;
  __shared__ int pidx, win, flag;
  const int2 wm = wgmap[blockIdx.x];
  const IDProb& q = probs[wm.x];
  const int b = wm.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = q.m, d = q.d, P = q.P;
  const int kmax = min(m, d);
  const int j0 = b * kIDCols;
  const int ja = j0 + wave, jb = ja + 4;
  bool acta = ja < m, actb = jb < m;
  // stage the eight candidates (rows j0.. of S) 64 samples at a time
  double ra[NR], rb[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    for (int e = tid; e < kIDCols * 64; e += 256) {
      const int jj = e & 7, kk = e >> 3;
      const int j = j0 + jj, k = 64 * r + kk;
      tile[jj * 64 + kk] = (j < m && k < d) ? q.S[j + (int64_t)k * q.lds] : 0.0;
    }
    __syncthreads();
    ra[r] = tile[wave * 64 + lane];
    rb[r] = tile[(wave + 4) * 64 + lane];
    __syncthreads();
  }
  {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) { sa += ra[r] * ra[r]; sb += rb[r] * rb[r]; }
    sa = wsum(sa);
    sb = wsum(sb);
    if (lane == 0) {
      nloc[wave] = acta ? sqrt(sa) : -1.0;
      nloc[wave + 4] = actb ? sqrt(sb) : -1.0;
    }
  }
  if (b == 0) {   // the pivot order is kept by workgroup 0 alone
    for (int j = tid; j < m; j += 256) {
      q.perm[j] = j;
      q.ipos[j] = j;
    }
    if (tid == 0) {
      q.state[0] = 0;
      q.state[1] = 0;
    }
  }
  double first = 0.0;
  for (int t = 0;; ++t) {
    // publish this workgroup's best remaining candidate for step t: the
    // column first, then (after it has completed) the slot with its step tag
    __syncthreads();
    if (tid == 0) {
      double bv = -1.0;
      int bi = 0x7fffffff, bw = -1;
      for (int jj = 0; jj < kIDCols; ++jj)
        if (nloc[jj] > bv) { bv = nloc[jj]; bi = j0 + jj; bw = jj; }
      pbest = bv;
      pidx = bi;
      win = bw;
    }
    __syncthreads();
    if (win >= 0 && (win & 3) == wave) {
      double* dst = q.cand + ((size_t)(t & 1) * P + b) * d;
      if (win < 4) store_col<NR, true>(ra, dst, t, d, lane);
      else store_col<NR, true>(rb, dst, t, d, lane);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      double* sl = q.slots + ((size_t)(t & 1) * P + b) * 4;
      st_coh(sl, pbest);
      st_coh(sl + 1, (double)pidx);
      __builtin_amdgcn_s_waitcnt(0);
      st_coh(sl + 2, (double)t);
    }
    // pivot: wait for every workgroup's step-t slot, then the largest
    // partial maximum, ties to the lowest candidate index
    if (wave == 0) {
      const double* sl = q.slots + (size_t)(t & 1) * P * 4;
      double sv = -1.0;
      int sc = 0x7fffffff;
      bool ok = true;
      for (int w0 = 0; w0 < P; w0 += 64) {
        const int w = w0 + lane;
        unsigned spins = 0;
        bool ready = w >= P;
        while (true) {
          if (!ready) ready = ld_coh(sl + 4 * w + 2) == (double)t;
          if (__all(ready)) break;
          if (++spins > kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) break;
        if (w < P) {
          const double vw = ld_coh(sl + 4 * w);
          const int cw = (int)ld_coh(sl + 4 * w + 1);
          if (vw > sv || (vw == sv && cw < sc)) { sv = vw; sc = cw; }
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(sv, off);
        const int oi = __shfl_xor(sc, off);
        if (o > sv || (o == sv && oi < sc)) { sv = o; sc = oi; }
      }
      if (lane == 0) {
        if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        flag = ok;
        pbest = sv;
        pidx = sc;
      }
    }
    __syncthreads();
    if (!flag) return;
    const double best = pbest;
    const int p = pidx;
    if (t == 0) first = best;
    const bool stop = (t >= kmax) || (t == 0 ? best <= q.atol : best <= fmax(q.eps * first, q.atol));
    if (stop) {
      if (b == 0 && tid == 0) {
        q.first[0] = first;
        q.state[1] = (t == 0 && best <= 0.0) ? 0 : t;
        q.state[0] = 1;
      }
      break;
    }
    const double* pc = q.cand + ((size_t)(t & 1) * P + p / kIDCols) * d;
    for (int i = t + tid; i < d; i += 256) x[i] = ld_coh(pc + i);
    if (tid < kIDCols) nloc[tid] = -1.0;
    __syncthreads();
    const double x0 = x[t];
    const double alpha = (x0 >= 0.0) ? -best : best;
    const double v0 = x0 - alpha;
    const double vtv = v0 * v0 + (best * best - x0 * x0);
    const double tau = (vtv > 0.0 && best > 0.0) ? 2.0 / vtv : 0.0;
    if (tid == 0) {
      if (b == 0) {
        const int qpos = q.ipos[p];
        const int ct = q.perm[t];
        q.perm[t] = p;
        q.perm[qpos] = ct;
        q.ipos[p] = t;
        q.ipos[ct] = qpos;
      }
      if (p / kIDCols == b) q.alpha[t] = alpha;
    }
    if (p == ja) acta = false;
    if (p == jb) actb = false;
    if (acta) reflect_abs<NR>(ra, x, v0, tau, t, d, lane, &nloc[wave]);
    if (actb) reflect_abs<NR>(rb, x, v0, tau, t, d, lane, &nloc[wave + 4]);
  }
  // the factored columns (R in rows < k) for the R1 / R2 gathers
  if (ja < m) store_col<NR, false>(ra, q.W + (int64_t)ja * d, 0, d, lane);
  if (jb < m) store_col<NR, false>(rb, q.W + (int64_t)jb * d, 0, d, lane);
}

namespace {
template <int NR>
int coop_capacity_nr(int max_d) {
  int dev = 0, cus = 0, coop = 0, nb = 0;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return 0;
  HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, id_coop_kernel<NR>, 256,
                                                         (size_t)std::max(max_d, 1) * sizeof(double)));
  return nb * cus;
}
}  // namespace

int id_coop_capacity(int max_d) {
  if (max_d <= 64 * 4) return coop_capacity_nr<4>(max_d);
  if (max_d <= 64 * 10) return coop_capacity_nr<10>(max_d);
  if (max_d <= 64 * 16) return coop_capacity_nr<16>(max_d);
  return 0;
}

void launch_id_coop(const IDProb* p, const int2* wgmap, int total_wg, int max_d, int* err, hipStream_t s) {
  if (total_wg <= 0) return;
  REQUIRE(max_d <= 64 * 16, HSSMF_EINVAL, "cooperative interpolative decomposition: more than 1024 samples");
  const size_t lds = (size_t)std::max(max_d, 1) * sizeof(double);
  void* args[] = {(void*)&p, (void*)&wgmap, (void*)&err};
  const void* fn = max_d <= 64 * 4    ? (const void*)id_coop_kernel<4>
                   : max_d <= 64 * 10 ? (const void*)id_coop_kernel<10>
                                      : (const void*)id_coop_kernel<16>;
  const int tok = prof::begin(0, s);   // timing hook (no-op when off)
  HIP_CHECK(hipLaunchCooperativeKernel(fn, dim3(total_wg), dim3(256), args, lds, s));
  prof::end(tok, s);
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

// the k x k identity into columns [m-k, m) of W2 (k x m, ld k), for the
// strong-RRQR test's solve with R1
__global__ void srrqr_eye_kernel(const IDProb* __restrict__ probs, const int* __restrict__ idx) {
  const IDProb q = probs[idx[blockIdx.y]];
  const int k = q.state[1];
  const int64_t kk = (int64_t)k * k;
  double* Z = q.W2 + (int64_t)(q.m - k) * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kk; e += (int64_t)gridDim.x * blockDim.x)
    Z[e] = (e % k == e / k) ? 1.0 : 0.0;
}

// Per problem (one workgroup): gamma_j^2 over the remaining columns and the
// squared row norms of Z = R1^{-1} into LDS, then the largest
// rho = X_ij^2 + gamma_j^2 |Z_i|^2 over e = i + k j, ties to the lowest e
__global__ __launch_bounds__(256) void srrqr_test_kernel(const IDProb* __restrict__ probs, const int* __restrict__ idx,
                                                         double* __restrict__ rho_out, int* __restrict__ e_out) {
  extern __shared__ double sm[];
  __shared__ double wv[4];
  __shared__ int wi[4];
  const IDProb q = probs[idx[blockIdx.x]];
  const int k = q.state[1], m = q.m, d = q.d, nr = m - k;
  const int tid = threadIdx.x;
  double* gam2 = sm;        // nr
  double* zr2 = sm + nr;    // k
  for (int j = tid; j < nr; j += 256) {
    const double* c = q.W + (int64_t)q.perm[k + j] * d;
    double ss = 0.0;
    for (int i = k; i < d; ++i) ss += c[i] * c[i];
    gam2[j] = ss;
  }
  const double* X = q.W2;
  const double* Z = q.W2 + (int64_t)nr * k;
  for (int i = tid; i < k; i += 256) {
    double ss = 0.0;
    for (int l = i; l < k; ++l) ss += Z[i + (int64_t)l * k] * Z[i + (int64_t)l * k];
    zr2[i] = ss;
  }
  __syncthreads();
  double bv = -1.0;
  int bi = 0x7fffffff;
  const int64_t tot = (int64_t)k * nr;
  for (int64_t e = tid; e < tot; e += 256) {
    const int i = (int)(e % k), j = (int)(e / k);
    const double x = X[e];
    const double v = x * x + gam2[j] * zr2[i];
    if (v > bv) { bv = v; bi = (int)e; }   // each thread's e ascend: the first of equals stays
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(bv, off);
    const int oi = __shfl_xor(bi, off);
    if (o > bv || (o == bv && oi < bi)) { bv = o; bi = oi; }
  }
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) { wv[wave] = bv; wi[wave] = bi; }
  __syncthreads();
  if (tid == 0) {
    bv = wv[0];
    bi = wi[0];
    for (int w = 1; w < 4; ++w)
      if (wv[w] > bv || (wv[w] == bv && wi[w] < bi)) { bv = wv[w]; bi = wi[w]; }
    rho_out[blockIdx.x] = bv;
    e_out[blockIdx.x] = bi;
  }
}

void launch_srrqr_eye(const IDProb* p, const int* idx, int n, int max_k, hipStream_t s) {
  if (n <= 0 || max_k <= 0) return;
  int64_t bx = ((int64_t)max_k * max_k + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(srrqr_eye_kernel, dim3((unsigned)bx, n), dim3(256), 0, s, p, idx);
  HIP_CHECK(hipGetLastError());
}

void launch_srrqr_test(const IDProb* p, const int* idx, int n, int max_m, double* rho, int* e, hipStream_t s) {
  if (n <= 0) return;
  const size_t lds = (size_t)std::max(max_m, 1) * sizeof(double);
  REQUIRE(lds <= 64 * 1024, HSSMF_EINVAL, "strong RRQR: more than 8192 rows in one ID");
  hipLaunchKernelGGL(srrqr_test_kernel, dim3(n), dim3(256), lds, s, p, idx, rho, e);
  HIP_CHECK(hipGetLastError());
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
  auto fn = max_d <= 64 * 4 ? id_step_kernel<4> : max_d <= 64 * 10 ? id_step_kernel<10> : id_step_kernel<16>;
  if (prof::enabled()) {
    hipEvent_t e0, e1;
    prof::ext(0, 0.0, &e0, &e1);   // timing hook; the work is added per pass
    hipExtLaunchKernelGGL(fn, dim3(total_wg), dim3(256), lds, s, e0, e1, 0, p, wgmap, t);
  } else {
    hipLaunchKernelGGL(fn, dim3(total_wg), dim3(256), lds, s, p, wgmap, t);
  }
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

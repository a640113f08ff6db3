// Column-pivoted Householder QR for the interpolative decomposition of
// Sec. 2.2, stopped at the epsilon-rank of Sec. 5.3, with every pivot step
// of a problem inside one launch and its candidates resident in registers.
//
// A problem is Y = S^T (d x m): its m candidates (rows of the node samples)
// are the columns, each of length d.  A 512-thread workgroup (one per CU,
// two wavefronts per SIMD, so each may hold 256 registers) holds C
// candidates: each of its 8 wavefronts owns CW of them, and lane l keeps
// rows l, l + 64, ..., l + 64 (NR - 1) of each in registers.  Problems of at
// most C candidates (the leaves and most lower nodes) run on one workgroup,
// so a pivot step costs two workgroup barriers: the remaining norms are
// published in LDS and every wavefront takes the pivot (largest remaining
// norm, ties to the lowest candidate index); the owner copies the pivot
// column to LDS; every wavefront forms the reflector and applies it to its
// active candidates, recomputing their remaining norms from the updated
// entries (no downdating).  Larger problems are spread over P workgroups of
// one cooperative launch (all resident at once): per step each workgroup
// publishes its best candidate's column and then its (norm, index) with a
// step tag through agent-coherent memory, waits (bounded) for the other
// workgroups' tags of that step, and takes the pivot column from the
// winner's published copy.  Columns never move: perm / ipos record the
// interchanges a swapping QR would make, and the factored columns are
// written back to W (d x m) at the end for the R1 / R2 gathers.
#include "kernels.hpp"

namespace hssmf {

namespace {

constexpr int kResThreads = 512;
constexpr int kResWaves = kResThreads / 64;
constexpr unsigned kResSpinLimit = 1u << 22;

__device__ __forceinline__ double rsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double rdlane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sums over the wavefront of N values per lane at once (N a power of two
// up to 64).  The first log2(N) exchange levels halve the values each lane
// carries (a lane keeps the half its offset bit selects and adds the
// partner's copy of it), so they take N - 1 exchanges in all instead of
// N log2(N); the remaining levels are plain butterflies.  Value c's sum
// ends up in lanes (64 / N) c ..; it is returned to every lane (wave
// uniform) in v[c].
template <int N>
__device__ __forceinline__ void msum(double (&v)[N], int lane) {
#pragma unroll
  for (int o = 32, cnt = N; cnt > 1; o >>= 1, cnt >>= 1) {
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < cnt / 2; ++i) {
      const double keep = up ? v[i + cnt / 2] : v[i];
      const double send = up ? v[i] : v[i + cnt / 2];
      v[i] = keep + __shfl_xor(send, o);
    }
  }
#pragma unroll
  for (int o = 32 / N; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o);
  const double w = v[0];
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] = rdlane(w, (64 / N) * c);
}

// (value, index) maximum over the wavefront: larger value wins, ties to the
// lower index
__device__ __forceinline__ void wargmax(double& v, int& i) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off);
    const int oi = __shfl_xor(i, off);
    if (o > v || (o == v && oi < i)) { v = o; i = oi; }
  }
}

}  // namespace

template <int NR, int CW>
__global__ __launch_bounds__(kResThreads) void id_res_kernel(const IDProb* __restrict__ probs,
                                                             const int2* __restrict__ wgmap, int* err) {
  constexpr int C = kResWaves * CW;          // candidates per workgroup
  constexpr int TLD = 65;                     // staging tile: candidate-major, padded
  constexpr int kStage = C * TLD;
  constexpr int kV = 64 * NR;
  constexpr int kLds = kStage > kV ? kStage : kV;
  __shared__ double sh[kLds];                 // staging tile, then the pivot column (absolute rows)
  __shared__ double nrm[C];
  __shared__ double gbest;
  __shared__ int gidx, gok;
  double* v = sh;

  const int2 wm = wgmap[blockIdx.x];
  const IDProb& q = probs[wm.x];
  const int b = wm.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = q.m, d = q.d, P = q.P;
  const int kmax = min(m, d);
  const int j0 = b * C;
  const int jw = j0 + wave * CW;              // this wavefront's first candidate

  // stage the workgroup's candidates: rows j0.. of S (m x d, ld lds), 64
  // samples at a time, read coalesced along the candidates and turned
  // around in LDS
  double col[CW][NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (64 * r < d) {
      for (int e = tid; e < C * 64; e += kResThreads) {
        const int jj = e % C, kk = e / C;
        const int j = j0 + jj, k = 64 * r + kk;
        sh[jj * TLD + kk] = (j < m && k < d) ? q.S[j + (int64_t)k * q.lds] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < CW; ++c) col[c][r] = sh[(wave * CW + c) * TLD + lane];
      __syncthreads();
    } else {
#pragma unroll
      for (int c = 0; c < CW; ++c) col[c][r] = 0.0;
    }
  }
  // the pivot column buffer is zero past row d for the whole run
  for (int i = d + tid; i < 64 * NR; i += kResThreads) v[i] = 0.0;
  // active candidates of this wavefront (bit c: candidate jw + c), and
  // their remaining norms in LDS (-1 once pivoted or past m)
  unsigned act = 0;
  {
    double ss[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      if (jw + c < m) act |= 1u << c;
      ss[c] = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) ss[c] += col[c][r] * col[c][r];
    }
    msum<CW>(ss, lane);
#pragma unroll
    for (int c = 0; c < CW; ++c)
      if (lane == c) nrm[wave * CW + c] = (act >> c & 1u) ? sqrt(ss[c]) : -1.0;
  }
  if (b == 0) {   // the pivot order is kept by workgroup 0 alone
    for (int j = tid; j < m; j += kResThreads) {
      q.perm[j] = j;
      q.ipos[j] = j;
    }
  }
  double first = 0.0;
  bool failed = false;
  int t = 0;
  for (;; ++t) {
    __syncthreads();
    // this workgroup's best remaining candidate
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int e = lane; e < C; e += 64) {
      const double x = nrm[e];
      if (x > bv) { bv = x; bi = j0 + e; }
    }
    wargmax(bv, bi);
    double best = bv;
    int p = bi;
    bool local = true;
    if (P > 1) {
      // publish the best column (rows t..), then (norm, index), then the tag
      const int bl = bi - j0;
      if (bv >= 0.0 && bl / CW == wave) {
        double* dst = q.cand + ((size_t)(t & 1) * P + b) * d;
#pragma unroll
        for (int c = 0; c < CW; ++c)
          if (c == bl % CW) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
              const int i = lane + 64 * r;
              if (i >= t && i < d) st_coh(dst + i, col[c][r]);
            }
          }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) {
        double* sl = q.slots + ((size_t)(t & 1) * P + b) * 4;
        st_coh(sl, bv);
        st_coh(sl + 1, (double)bi);
        __builtin_amdgcn_s_waitcnt(0);
        st_coh(sl + 2, (double)t);
      }
      if (wave == 0) {
        const double* sl = q.slots + (size_t)(t & 1) * P * 4;
        double sv = -1.0;
        int sc = 0x7fffffff;
        bool ok = true;
        for (int w0 = 0; w0 < P && ok; w0 += 64) {
          const int w = w0 + lane;
          unsigned spins = 0;
          bool ready = w >= P;
          while (true) {
            if (!ready) ready = ld_coh(sl + 4 * w + 2) == (double)t;
            if (__all(ready)) break;
            if (++spins > kResSpinLimit ||
                __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
              ok = false;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          if (ok && w < P) {
            const double vw = ld_coh(sl + 4 * w);
            const int cw = (int)ld_coh(sl + 4 * w + 1);
            if (vw > sv || (vw == sv && cw < sc)) { sv = vw; sc = cw; }
          }
        }
        wargmax(sv, sc);
        if (lane == 0) {
          if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          gok = ok;
          gbest = sv;
          gidx = sc;
        }
      }
      __syncthreads();
      if (!gok) { failed = true; break; }
      best = gbest;
      p = gidx;
      local = p >= j0 && p < j0 + C;
    }
    if (t == 0) first = best;
    const bool stop = (t >= kmax) || (t == 0 ? best <= q.atol : best <= fmax(q.eps * first, q.atol));
    if (stop) break;
    // the pivot column, rows t.., into LDS
    if (local) {
      const int pl = p - j0;
      if (pl / CW == wave) {
#pragma unroll
        for (int c = 0; c < CW; ++c)
          if (c == pl % CW) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
              const int i = lane + 64 * r;
              if (i >= t && i < d) v[i] = col[c][r];
            }
            act &= ~(1u << c);
          }
      }
    } else {
      const double* src = q.cand + ((size_t)(t & 1) * P + p / C) * d;
      for (int i = t + tid; i < d; i += kResThreads) v[i] = ld_coh(src + i);
    }
    __syncthreads();
    const double x0 = v[t];
    const double alpha = (x0 >= 0.0) ? -best : best;
    const double v0 = x0 - alpha;
    const double vtv = v0 * v0 + (best * best - x0 * x0);
    const double tau = (vtv > 0.0 && best > 0.0) ? 2.0 / vtv : 0.0;
    if (b == 0 && tid == 0) {
      const int qpos = q.ipos[p];
      const int ct = q.perm[t];
      q.perm[t] = p;
      q.perm[qpos] = ct;
      q.ipos[p] = t;
      q.ipos[ct] = qpos;
      q.alpha[t] = alpha;
    }
    // the reflector (v with v[t] = v0) on every candidate of the wavefront.
    // Rows below t are finished: the reflector is zero there, so a block of
    // 64 rows entirely below t is skipped, and only the block holding row t
    // needs per-row masks (v is zero past d, as are the columns).  Pivoted
    // candidates are updated too: their rows above their own pivot step (R
    // entries) are left unchanged by every later reflector.
    // Candidates go through in chunks of CH (fewer live registers); each
    // chunk reads the reflector from LDS twice.
    const int r0 = t >> 6;
    constexpr int CH = (NR <= 4 ? 8 : 4) < CW ? (NR <= 4 ? 8 : 4) : CW;
#pragma unroll
    for (int cb = 0; cb < CW; cb += CH) {
      double dot[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) dot[c] = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < r0) continue;
        const int i = lane + 64 * r;
        double vi = v[i];
        if (r == r0) vi = (i == t) ? v0 : (i > t ? vi : 0.0);
#pragma unroll
        for (int c = 0; c < CH; ++c) dot[c] += vi * col[cb + c][r];
      }
      msum<CH>(dot, lane);
#pragma unroll
      for (int c = 0; c < CH; ++c) dot[c] *= tau;
      double ss[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) ss[c] = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < r0) continue;
        const int i = lane + 64 * r;
        double vi = v[i];
        if (r == r0) vi = (i == t) ? v0 : (i > t ? vi : 0.0);
        const double keep = (r == r0 && i <= t) ? 0.0 : 1.0;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const double y = col[cb + c][r] - dot[c] * vi;
          col[cb + c][r] = y;
          ss[c] += keep * (y * y);
        }
      }
      msum<CH>(ss, lane);
      // lane c publishes candidate cb + c's remaining norm (v is next
      // rewritten after the next step's first barrier, when every
      // wavefront is done with it)
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (lane == c) nrm[wave * CW + cb + c] = (act >> (cb + c) & 1u) ? sqrt(ss[c]) : -1.0;
    }
  }
  if (b == 0 && tid == 0) {
    q.first[0] = first;
    q.state[1] = failed ? 0 : t;
    q.state[0] = 1;
  }
  if (failed) return;
  // the factored columns (R in rows < k) for the R1 / R2 gathers
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int j = jw + c;
    if (j < m) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int i = lane + 64 * r;
        if (i < d) q.W[i + (int64_t)j * d] = col[c][r];
      }
    }
  }
}

namespace {

// template for a pass whose largest sample count is max_d: rows per lane
// and candidates per wavefront, at most 80 register-resident entries per
// lane
struct ResShape {
  int nr, cw;
};
ResShape res_shape(int max_d) {
  if (max_d <= 128) return {2, 16};
  if (max_d <= 256) return {4, 16};
  if (max_d <= 640) return {10, 8};
  if (max_d <= 1280) return {20, 4};
  if (max_d <= 2560) return {40, 2};
  return {0, 0};
}

template <int NR, int CW>
const void* res_fn() {
  return (const void*)id_res_kernel<NR, CW>;
}

const void* res_kernel(int max_d) {
  const ResShape s = res_shape(max_d);
  if (s.nr == 2) return res_fn<2, 16>();
  if (s.nr == 4) return res_fn<4, 16>();
  if (s.nr == 10) return res_fn<10, 8>();
  if (s.nr == 20) return res_fn<20, 4>();
  if (s.nr == 40) return res_fn<40, 2>();
  return nullptr;
}

}  // namespace

int id_res_candidates(int max_d) {
  const ResShape s = res_shape(max_d);
  return s.nr ? kResWaves * s.cw : 0;
}

int id_res_capacity(int max_d) {
  const void* fn = res_kernel(max_d);
  if (!fn) return 0;
  int dev = 0, cus = 0, coop = 0, nb = 0;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return 0;
  HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kResThreads, 0));
  return nb * cus;
}

void launch_id_res(const IDProb* p, const int2* wgmap, int total_wg, int max_d, bool coop, int* err,
                   hipStream_t s) {
  if (total_wg <= 0) return;
  const void* fn = res_kernel(max_d);
  REQUIRE(fn != nullptr, HSSMF_ERANK, "interpolative decomposition: more than 2560 samples");
  void* args[] = {(void*)&p, (void*)&wgmap, (void*)&err};
  const int tok = prof::begin(0, s);   // timing hook (no-op when off)
  if (coop) HIP_CHECK(hipLaunchCooperativeKernel(fn, dim3(total_wg), dim3(kResThreads), args, 0, s));
  else HIP_CHECK(hipLaunchKernel(fn, dim3(total_wg), dim3(kResThreads), args, 0, s));
  prof::end(tok, s);
}

}  // namespace hssmf

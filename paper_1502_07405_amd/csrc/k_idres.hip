// Column-pivoted Householder QR for the interpolative decomposition of
// Sec. 2.2, stopped at the epsilon-rank of Sec. 5.3, with every pivot step
// of a problem inside one launch and its candidates resident in registers.
//
// A problem is Y = S^T (d x m): its m candidates (rows of the node samples)
// are the columns, each of length d.  A 512-thread workgroup (one per CU,
// two wavefronts per SIMD, so each may hold 256 registers) holds C
// candidates.  Each candidate lives in one group of LPC = 16 lanes of a
// wavefront (a DPP row), lane e of the group keeping rows
// e, e + LPC, ..., so the sums over a candidate's rows (its dot product
// with the reflector, its remaining norm) are butterflies inside the group:
// data-parallel-primitive moves within a row, bitwise the same result in
// every lane of the group (each level adds a and b in one lane and b and a
// in its partner).  A wavefront holds SL candidates per group.
//
// Problems of at most C candidates (the leaves and most lower nodes) run on
// one workgroup, with one workgroup barrier per pivot step: each wavefront
// publishes its best remaining candidate (norm, index) and that candidate's
// column, already in reflector form, in LDS; after the barrier every
// wavefront takes the pivot (largest remaining norm, ties to the lowest
// candidate index) and applies its reflector to its own candidates,
// recomputing their remaining norms from the updated entries (no
// downdating).  Larger problems are spread over P workgroups of one
// cooperative launch (all resident at once): per step each workgroup also
// publishes its best column and then its (norm, index) through
// agent-coherent memory, in records that are empty (NaN) until written and
// rotate over three buffers, waits (bounded) until the other workgroups'
// records of that step are filled, and takes the pivot column from the
// winner's published copy.  Columns never move: perm / ipos record the interchanges a swapping
// QR would make, and the factored columns are written back to W (d x m) at
// the end for the R1 / R2 gathers.  A problem may instead bring a pivot
// order to follow (the re-factorizations of the strong rank-revealing QR):
// then only that step's candidate competes, and the steps end with the
// order.
#include "kernels.hpp"

namespace hssmf {

namespace {

constexpr int kResThreads = 512;
constexpr int kResWaves = kResThreads / 64;
constexpr unsigned kResSpinLimit = 1u << 22;
constexpr double kEmpty = __builtin_nan("");   // an exchange record not yet written

__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a double moved between lanes of a 16-lane row by a data-parallel
// primitive (CTRL: quad permutation, half-row mirror or row rotation)
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over each group of 16 lanes (a row), the same bits in every lane of
// the group: partners 1 and 2 apart (quad permutations), then the other
// quad of the half-row (its mirror: all lanes of a quad already agree),
// then the other half-row (rotation by 8).
template <int LPC>
__device__ __forceinline__ double gsum(double x) {
  static_assert(LPC == 16, "a candidate spans one 16-lane row");
  x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp<0x141>(x);  // row_half_mirror
  x += dpp<0x128>(x);  // row_ror:8
  return x;
}

// per-wavefront record of a pivot step: its best candidate's remaining norm
// and index, and that column's entry in the pivot row
struct alignas(16) WRec {
  double v, x0;
  int i, pad[3];
};

// (v, i) <- the larger of (v, i) and (o, oi), ties to the lower index, by
// selects
__device__ __forceinline__ void amax(double& v, int& i, double o, int oi) {
  const bool tk = (o > v) | ((o == v) & (oi < i));
  v = tk ? o : v;
  i = tk ? oi : i;
}

// y * y rounded on its own (never fused into a following sum)
__device__ __forceinline__ double sq_rn(double y) {
#pragma clang fp contract(off)
  return y * y;
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

// LPC lanes per candidate, RL rows per lane (d <= LPC RL), SL candidates per
// lane group; FORCED: every problem of the launch follows its forced order
template <int LPC, int RL, int SL, bool FORCED>
__global__ __launch_bounds__(kResThreads) void id_res_kernel(const IDProb* __restrict__ probs,
                                                             const int2* __restrict__ wgmap, int* err) {
  constexpr int G = 64 / LPC;                 // lane groups per wavefront
  constexpr int CW = G * SL;                  // candidates per wavefront
  constexpr int NW = kResWaves;
  constexpr int C = NW * CW;                  // candidates per workgroup
  constexpr int TLD = 65;                     // staging tile: candidate-major, padded
  constexpr int kStage = C * TLD;
  constexpr int kV = LPC * RL;
  constexpr int kBuf = 2 * NW * kV + kV;      // per-wavefront columns by step parity, remote pivot
  constexpr int kLds = kStage > kBuf ? kStage : kBuf;
  constexpr int kMaxM = 2 * LPC * RL;         // a node's rows: at most twice the samples
  constexpr int RPC = 64 / LPC;               // r-slots per 64-row staging chunk
  constexpr int RB = RL % 8 == 0 ? 8 : RL;    // r-blocks per chunk of rows
  constexpr int NCH = RL / RB;
  __shared__ double sh[kLds];                 // staging tile, then the column buffers
  __shared__ WRec wrec[2][NW];
  __shared__ int lperm[kMaxM], lipos[kMaxM];  // pivot order (workgroup 0 of a problem)
  __shared__ double lalpha[kV];               // R diagonal, written out at the end
  __shared__ int lforce[kV];                  // a forced pivot order
  __shared__ double gbest, gx0;
  __shared__ int gidx, gok;

  const int2 wm = wgmap[blockIdx.x];
  const int b = wm.y;
  // the problem's fields, read once: stores through the output pointers
  // below must not make the compiler fetch them again
  const IDProb& qr = probs[wm.x];
  const double* __restrict__ S = qr.S;
  double* __restrict__ W = qr.W;
  double* __restrict__ alpha_out = qr.alpha;
  double* __restrict__ slots = qr.slots;
  double* __restrict__ cand = qr.cand;
  int* __restrict__ perm_out = qr.perm;
  int* __restrict__ ipos_out = qr.ipos;
  int* __restrict__ state = qr.state;
  double* __restrict__ first_out = qr.first;
  const int m = qr.m, d = qr.d, P = qr.P, lds = qr.lds;
  const double eps = qr.eps, atol = qr.atol;
  constexpr bool forced = FORCED;
  const int* __restrict__ force = FORCED ? qr.force : nullptr;
  const int kf = FORCED ? qr.kf : 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane / LPC, e = lane % LPC;   // lane group, row offset in it
  const int kmax = min(m, d);
  const int j0 = b * C;
  const int jw = j0 + wave * CW;              // this wavefront's first candidate
  const bool keeper = b == 0;                 // keeps the pivot order
  const int dc = (d + LPC * RB - 1) / (LPC * RB);   // chunks holding rows < d
  // candidate of slot s in this lane's group: jw + s G + g

  if (forced)
    for (int j = tid; j < kf; j += kResThreads) lforce[j] = force[j];
  // stage the workgroup's candidates: rows j0.. of S (m x d, ld lds), 64
  // samples at a time, read coalesced along the candidates and turned
  // around in LDS
  double col[SL][RL];
#pragma unroll
  for (int k = 0; k < (RL + RPC - 1) / RPC; ++k) {
    if (64 * k < d) {
      for (int x = tid; x < C * 64; x += kResThreads) {
        const int jj = x % C, kk = x / C;
        const int j = j0 + jj, i = 64 * k + kk;
        sh[jj * TLD + kk] = (j < m && i < d) ? S[j + (int64_t)i * lds] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < RPC; ++rr) {
        const int r = k * RPC + rr;
        if (r < RL) {
#pragma unroll
          for (int s = 0; s < SL; ++s) col[s][r] = sh[(wave * CW + s * G + g) * TLD + e + LPC * rr];
        }
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int rr = 0; rr < RPC; ++rr) {
        const int r = k * RPC + rr;
        if (r < RL) {
#pragma unroll
          for (int s = 0; s < SL; ++s) col[s][r] = 0.0;
        }
      }
    }
  }
  if (keeper)
    for (int j = tid; j < m; j += kResThreads) {
      lperm[j] = j;
      lipos[j] = j;
    }
  // active slots of this lane's group (bit s) and their remaining norms
  // (the same in every lane of the group)
  unsigned act = 0;
  double nv[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    if (jw + s * G + g < m) act |= 1u << s;
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < RL; ++r) ss += col[s][r] * col[s][r];
    nv[s] = sqrt(gsum<LPC>(ss));
  }
  double first = 0.0;
  bool failed = false;
  int t = 0;
  // One workgroup barrier per pivot step: every wavefront publishes its best
  // remaining candidate (norm, index) and that candidate's column, already
  // in reflector form for step t (rows below t zero, row t holding
  // x0 - alpha), in its own buffer; after the barrier all wavefronts take
  // the largest (ties to the lowest index) and apply that buffer.  Buffers
  // alternate with the step's parity, so a wavefront that runs ahead to
  // step t + 1 never overwrites what the others still read for step t.
  for (;; ++t) {
    const int par = t & 1;
    const int tc = t / (LPC * RB);            // the chunk holding row t
    // this wavefront's best active candidate (inactive slots never win;
    // with a forced order only the slot holding the step's candidate may)
    unsigned sel = act;
    if (forced && t < kf) {
      const int qf = lforce[t] - jw;
      sel = (qf >= 0 && qf < CW && qf % G == g) ? (act & (1u << (qf / G))) : 0u;
    }
    double bv = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const bool on = (sel >> s) & 1u;
      amax(bv, bi, on ? nv[s] : -1.0, on ? jw + s * G + g : 0x7fffffff);
    }
#pragma unroll
    for (int off = LPC; off < 64; off <<= 1) {
      const double o = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      amax(bv, bi, o, oi);
    }
    // the lanes of the group holding it write its column, in reflector form
    // for step t, to this wavefront's buffer (one uniform branch per chunk
    // of rows; the slot is the same in every lane of the group)
    if ((bv >= 0.0) & ((bi - jw) % G == g)) {
      const int sb = __builtin_amdgcn_readfirstlane((bi - jw) / G);
      double* dst = sh + (size_t)(par * NW + wave) * kV;
      const double al = bv;
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        if (s != sb) continue;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          if (ch < tc || ch >= dc) continue;
          if (ch == tc) {
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
              const int r = ch * RB + rr;
              const int i = e + LPC * r;
              const double x = col[s][r];
              double w = i > t ? x : 0.0;
              if (i == t) {
                w = x - ((x >= 0.0) ? -al : al);
                wrec[par][wave].x0 = x;
              }
              dst[i] = w;
            }
          } else {
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
              const int r = ch * RB + rr;
              dst[e + LPC * r] = col[s][r];
            }
          }
        }
      }
    }
    if (lane == 0) {
      wrec[par][wave].v = bv;
      wrec[par][wave].i = bi;
    }
    __syncthreads();
    // the workgroup's best: all (norm, index) records read at once, then
    // compared; the pivot-row entry of the winner's column after that
    double rv[NW];
    int ri[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      rv[w] = wrec[par][w].v;
      ri[w] = wrec[par][w].i;
    }
    double best = rv[0];
    int p = ri[0], pw = 0;
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const bool tk = (rv[w] > best) | ((rv[w] == best) & (ri[w] < p));
      best = tk ? rv[w] : best;
      p = tk ? ri[w] : p;
      pw = tk ? w : pw;
    }
    double x0 = wrec[par][pw].x0;
    const double* vp = sh + (size_t)(par * NW + pw) * kV;
    bool local = true;
    if (P > 1) {
      // Exchange with the problem's other workgroups through three rotating
      // buffers of agent-coherent records (norm, index), NaN when empty:
      // publish this workgroup's best column (rows t.., raw) and clear its
      // record for step t + 1 (last used at step t - 2, which every
      // workgroup has finished reading: each has published step t - 1
      // since); once those stores are complete, publish (norm, index) of
      // step t, then wait (bounded) until every record of step t is filled.
      const int u = t % 3;
      if (best >= 0.0) {
        double* dst = cand + ((size_t)u * P + b) * d;
        for (int i = t + tid; i < d; i += kResThreads) st_coh(dst + i, i == t ? x0 : vp[i]);
      }
      if (tid == 0) {
        double* nx = slots + ((size_t)((t + 1) % 3) * P + b) * 2;
        st_coh(nx, kEmpty);
        st_coh(nx + 1, kEmpty);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) {
        double* sl = slots + ((size_t)u * P + b) * 2;
        st_coh(sl, best);
        st_coh(sl + 1, (double)p);
      }
      if (wave == 0) {
        const double* sl = slots + (size_t)u * P * 2;
        double sv = -1.0;
        int sc = 0x7fffffff;
        bool ok = true;
        for (int w0 = 0; w0 < P && ok; w0 += 64) {
          const int w = w0 + lane;
          double vw = -1.0, cw = 0.0;
          bool ready = w >= P;
          unsigned spins = 0;
          while (true) {
            if (!ready) {
              vw = ld_coh(sl + 2 * w);
              cw = ld_coh(sl + 2 * w + 1);
              ready = !__builtin_isnan(vw) && !__builtin_isnan(cw);
            }
            if (__all(ready)) break;
            if (++spins > kResSpinLimit ||
                __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
              ok = false;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          if (ok && w < P) amax(sv, sc, vw, (int)cw);
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
      if (local) {
        pw = (p - j0) / CW;
        vp = sh + (size_t)(par * NW + pw) * kV;
        x0 = wrec[par][pw].x0;
      } else if (best >= 0.0 && t < kmax) {
        // another workgroup's column, rows from the chunk holding t
        double* gv = sh + (size_t)2 * NW * kV;
        const double* src = cand + ((size_t)u * P + p / C) * d;
        const double al = best;
        for (int i = tc * RB * LPC + tid; i < dc * RB * LPC; i += kResThreads) {
          const double x = (i >= t && i < d) ? ld_coh(src + i) : 0.0;
          double w = i > t ? x : 0.0;
          if (i == t) {
            w = x - ((x >= 0.0) ? -al : al);
            gx0 = x;
          }
          gv[i] = w;
        }
        __syncthreads();
        vp = gv;
        x0 = gx0;
      }
    }
    if (t == 0) first = best;
    const bool stop = (t >= kmax) || (forced ? t >= kf : t == 0 ? best <= atol : best <= fmax(eps * first, atol));
    if (stop) break;
    const double alpha = (x0 >= 0.0) ? -best : best;
    const double v0 = x0 - alpha;   // row t of the reflector
    const double vtv = v0 * v0 + (best * best - x0 * x0);
    const double tau = (vtv > 0.0 && best > 0.0) ? 2.0 / vtv : 0.0;
    if (local && wave == pw) {
      const int q = p - jw;
      act &= (q % G == g) ? ~(1u << (q / G)) : ~0u;
    }
    if (keeper && tid == kResThreads - 1) {   // the interchange of step t
      const int qpos = lipos[p];
      const int ct = lperm[t];
      lperm[t] = p;
      lperm[qpos] = ct;
      lipos[p] = t;
      lipos[ct] = qpos;
    }
    if (tid == 0) lalpha[t] = alpha;
    // the reflector on every candidate of the group.  Pivoted candidates
    // are updated too: their rows above their own pivot step (R entries)
    // are left unchanged by every later reflector.  Chunks below the one
    // holding row t are finished and skipped, as are chunks past d (the
    // reflector and the columns are zero there); the remaining norms leave
    // out rows up to t, which only that chunk masks.
    double dot[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) dot[s] = 0.0;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      if (ch < tc || ch >= dc) continue;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const int r = ch * RB + rr;
        const double vi = vp[e + LPC * r];
#pragma unroll
        for (int s = 0; s < SL; ++s) dot[s] += vi * col[s][r];
      }
    }
#pragma unroll
    for (int s = 0; s < SL; ++s) dot[s] = gsum<LPC>(dot[s]) * tau;
    double ss[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) ss[s] = 0.0;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      if (ch < tc || ch >= dc) continue;
      const bool tchunk = ch == tc;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const int r = ch * RB + rr;
        const int i = e + LPC * r;
        const double vi = vp[i];
        const double keep = (!tchunk || i > t) ? 1.0 : 0.0;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const double y = col[s][r] - dot[s] * vi;
          col[s][r] = y;
          ss[s] += keep * sq_rn(y);   // exactly ss + y^2 or ss
        }
      }
    }
#pragma unroll
    for (int s = 0; s < SL; ++s) nv[s] = sqrt(gsum<LPC>(ss[s]));
  }
  __syncthreads();
  if (keeper) {
    for (int j = tid; j < m; j += kResThreads) {
      perm_out[j] = lperm[j];
      ipos_out[j] = lipos[j];
    }
    for (int j = tid; j < t; j += kResThreads) alpha_out[j] = lalpha[j];
    if (tid == 0) {
      if (!forced) first_out[0] = first;
      state[1] = failed ? 0 : t;
      state[0] = 1;
    }
  }
  if (failed) return;
  // the factored columns (R in rows < k) for the R1 / R2 gathers
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int j = jw + s * G + g;
    if (j < m) {
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int i = e + LPC * r;
        if (i < d) W[i + (int64_t)j * d] = col[s][r];
      }
    }
  }
}

namespace {

// Templates: lanes per candidate, rows per lane (samples up to 16 rl) and
// candidates per lane group (32 sl candidates per workgroup), each without
// register spills.  A launch takes the fewest rows per lane that hold its
// largest sample count and then the fewest candidates per group that hold
// its largest problem (every wavefront runs every slot, so spare slots cost
// time), or the most if none does (fewest workgroups per problem).
struct ResShape {
  int lpc, rl, sl;
  const void* fn;    // pivots by the largest remaining norm
  const void* fnf;   // pivots in a forced order
};
const ResShape kShapes[] = {
    {16, 8, 2, (const void*)id_res_kernel<16, 8, 2, false>, (const void*)id_res_kernel<16, 8, 2, true>},
    {16, 8, 4, (const void*)id_res_kernel<16, 8, 4, false>, (const void*)id_res_kernel<16, 8, 4, true>},
    {16, 8, 8, (const void*)id_res_kernel<16, 8, 8, false>, (const void*)id_res_kernel<16, 8, 8, true>},
    {16, 16, 2, (const void*)id_res_kernel<16, 16, 2, false>, (const void*)id_res_kernel<16, 16, 2, true>},
    {16, 16, 4, (const void*)id_res_kernel<16, 16, 4, false>, (const void*)id_res_kernel<16, 16, 4, true>},
    {16, 16, 5, (const void*)id_res_kernel<16, 16, 5, false>, (const void*)id_res_kernel<16, 16, 5, true>},
    {16, 24, 2, (const void*)id_res_kernel<16, 24, 2, false>, (const void*)id_res_kernel<16, 24, 2, true>},
    {16, 24, 3, (const void*)id_res_kernel<16, 24, 3, false>, (const void*)id_res_kernel<16, 24, 3, true>},
    {16, 32, 2, (const void*)id_res_kernel<16, 32, 2, false>, (const void*)id_res_kernel<16, 32, 2, true>},
    {16, 40, 2, (const void*)id_res_kernel<16, 40, 2, false>, (const void*)id_res_kernel<16, 40, 2, true>},
};

const ResShape* res_shape(int max_d, int max_m) {
  int rl = 0;
  for (const ResShape& r : kShapes)
    if (16 * r.rl >= max_d && (rl == 0 || r.rl < rl)) rl = r.rl;
  if (rl == 0 || max_m > 2 * 16 * rl) return nullptr;   // the pivot order is kept in LDS
  const ResShape* pick = nullptr;
  for (const ResShape& r : kShapes) {
    if (r.rl != rl) continue;
    const int c = kResWaves * (64 / r.lpc) * r.sl;
    if (c >= max_m) {
      if (!pick || r.sl < pick->sl || kResWaves * (64 / pick->lpc) * pick->sl < max_m) pick = &r;
    } else if (!pick || (kResWaves * (64 / pick->lpc) * pick->sl < max_m && r.sl > pick->sl)) {
      pick = &r;
    }
  }
  return pick;
}

int capacity_of(const ResShape* s) {
  if (!s) return 0;
  int dev = 0, cus = 0, coop = 0, nb = 0;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return 0;
  HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, s->fn, kResThreads, 0));
  int nbf = 0;
  HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nbf, s->fnf, kResThreads, 0));
  return std::min(nb, nbf) * cus;
}

void launch_shape(const ResShape* sh, const IDProb* p, const int2* wgmap, int total_wg, bool coop, int* err,
                  hipStream_t s, bool forced) {
  if (total_wg <= 0) return;
  REQUIRE(sh != nullptr, HSSMF_ERANK, "interpolative decomposition: more than 640 samples");
  void* args[] = {(void*)&p, (void*)&wgmap, (void*)&err};
  const void* fn = forced ? sh->fnf : sh->fn;
  const int tok = prof::begin(4, s);   // timing hook (no-op when off)
  if (coop) HIP_CHECK(hipLaunchCooperativeKernel(fn, dim3(total_wg), dim3(kResThreads), args, 0, s));
  else HIP_CHECK(hipLaunchKernel(fn, dim3(total_wg), dim3(kResThreads), args, 0, s));
  prof::end(tok, s);
}

}  // namespace

int id_res_candidates(int max_d, int max_m) {
  const ResShape* s = res_shape(max_d, max_m);
  return s ? kResWaves * (64 / s->lpc) * s->sl : 0;
}

int id_res_capacity(int max_d, int max_m) { return capacity_of(res_shape(max_d, max_m)); }

void launch_id_res(const IDProb* p, const int2* wgmap, int total_wg, int max_d, int max_m, bool coop, int* err,
                   hipStream_t s) {
  launch_shape(res_shape(max_d, max_m), p, wgmap, total_wg, coop, err, s, false);
}

int id_res_template(int d, int m) {
  // rows per lane for d samples, or more when the pivot order of m rows
  // needs a larger template
  const ResShape* s = res_shape(std::max(d, (m + 1) / 2), m);
  return s ? (int)(s - kShapes) : -1;
}

int id_res_template_candidates(int tpl) {
  const ResShape& s = kShapes[tpl];
  return kResWaves * (64 / s.lpc) * s.sl;
}

int id_res_template_capacity(int tpl) { return capacity_of(&kShapes[tpl]); }

void launch_id_res_template(int tpl, const IDProb* p, const int2* wgmap, int total_wg, bool coop, int* err,
                            hipStream_t s, bool forced) {
  launch_shape(&kShapes[tpl], p, wgmap, total_wg, coop, err, s, forced);
}

}  // namespace hssmf

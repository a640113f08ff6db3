// Variable-size batched GEMM on CDNA4 matrix cores.
//
// One launch covers a list of independent products C = alpha op(A) op(B) +
// beta C (column major) of arbitrary shapes; every workgroup owns one 64x64
// tile of one product (found by binary search over the tile prefix sums).
// Four 64-lane wavefronts each own a 32x32 quadrant built from 16x16 MFMA
// blocks.  FP64 uses v_mfma_f64_16x16x4; FP32 and BF16 inputs accumulate in
// FP32 with v_mfma_f32_16x16x4_f32 / v_mfma_f32_16x16x32_bf16.
// Optional row maps fuse the gathers / scatters of the multifrontal
// extend-add into the product.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <type_traits>
#include <mutex>
#include <tuple>

#include "common.hpp"

namespace hssmf {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 64;

__device__ __forceinline__ int find_desc(const GemmDesc* __restrict__ d, int nd, int64_t tile) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The descriptors of one launch.  A batch of up to kGemmInline products
// travels in the kernel arguments themselves, so launching it costs no
// upload; larger batches are staged in device memory.
constexpr int kGemmInline = 24;
struct GemmBatch {
  const GemmDesc* descs;   // staged array, or nullptr: the inline copies
  int nd, pad;
  GemmDesc inl[kGemmInline];
};

__device__ __forceinline__ GemmDesc batch_desc(const GemmBatch& b, int64_t tile) {
  GemmDesc g = b.descs ? b.descs[find_desc(b.descs, b.nd, tile)] : b.inl[find_desc(b.inl, b.nd, tile)];
  // the descriptor is uniform: keep it in scalar registers
  static_assert(sizeof(GemmDesc) % 4 == 0, "descriptor of whole words");
  int w[sizeof(GemmDesc) / 4];
  __builtin_memcpy(w, &g, sizeof(g));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(GemmDesc) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  __builtin_memcpy(&g, w, sizeof(g));
  return g;
}

// Operand loads of one thread for the k-tiles of one product.  Element q of
// a k-tile is e = tid + 256 q: (i, kk) of op(A) and (kk, j) of op(B), ordered
// so that consecutive threads read consecutive addresses.  Indices past the
// edge are clamped to the last row / column / k and the value is zeroed when
// it is stored to LDS, so no load sits behind a branch and all of a thread's
// loads are in flight together.  A's row map does not depend on k and is
// resolved once; the entries of B's row map for the next k-tile are loaded
// together with the current tile, so no tile waits on a map lookup.
template <class T, int PER, int TK, int BM, int BN>
struct TileLoader {
  int64_t abase[PER], bbase[PER];
  int bnx[PER];
  unsigned arow_ok, bcol_ok, am, bm;
  T ra[PER], rb[PER];
  int tid;
  bool tA, tB;

  __device__ __forceinline__ void a_idx(int q, int& i, int& kk) const {
    const int e = tid + 256 * q;
    if (tA) { kk = e % TK; i = e / TK; } else { i = e % BM; kk = e / BM; }
  }
  __device__ __forceinline__ void b_idx(int q, int& kk, int& j) const {
    const int e = tid + 256 * q;
    if (tB) { j = e % BN; kk = e / BN; } else { kk = e % TK; j = e / TK; }
  }
  __device__ __forceinline__ void map_ahead(const GemmDesc& g, int k0) {
    const auto bmap = (gptr<const int>)g.bmap;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int kk, j;
      b_idx(q, kk, j);
      bnx[q] = bmap[min(k0 + kk, g.k - 1)];
    }
  }
  __device__ __forceinline__ void init(const GemmDesc& g, int row0, int col0) {
    tid = threadIdx.x;
    tA = g.transA;
    tB = g.transB;
    arow_ok = bcol_ok = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, kk, j, kb;
      a_idx(q, i, kk);
      b_idx(q, kb, j);
      const int ig = row0 + i, jg = col0 + j;
      arow_ok |= (unsigned)(ig < g.m) << q;
      bcol_ok |= (unsigned)(jg < g.n) << q;
      const int ic = min(ig, g.m - 1), jc = min(jg, g.n - 1);
      abase[q] = tA ? (int64_t)ic * g.lda : (int64_t)ic;
      bbase[q] = tB ? (int64_t)jc : (int64_t)jc * g.ldb;
    }
    if (!tA && g.amap) {
      const auto amap = (gptr<const int>)g.amap;
#pragma unroll
      for (int q = 0; q < PER; ++q) abase[q] = amap[(int)abase[q]];
    }
    if (!tB && g.bmap) map_ahead(g, 0);
  }
  // tile k0 into registers; B's map entries of tile knext behind it
  __device__ __forceinline__ void fetch(const GemmDesc& g, int k0, int knext) {
    const auto A = (gptr<const T>)g.A;
    const auto B = (gptr<const T>)g.B;
    const bool bmapped = !tB && g.bmap;
    am = bm = 0;
    int64_t ao[PER], bo[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, kk, j, kb;
      a_idx(q, i, kk);
      b_idx(q, kb, j);
      const int ka = k0 + kk, kca = min(ka, g.k - 1);
      const int kb2 = k0 + kb, kcb = min(kb2, g.k - 1);
      am |= (unsigned)(ka < g.k) << q;
      bm |= (unsigned)(kb2 < g.k) << q;
      ao[q] = abase[q] + (tA ? (int64_t)kca : (int64_t)kca * g.lda);
      bo[q] = bbase[q] + (tB ? (int64_t)kcb * g.ldb : (int64_t)(bmapped ? bnx[q] : kcb));
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) ra[q] = A[ao[q]];
#pragma unroll
    for (int q = 0; q < PER; ++q) rb[q] = B[bo[q]];
    if (bmapped && knext < g.k) map_ahead(g, knext);
  }
  template <class TO>
  __device__ __forceinline__ TO a(int q) const { return ((am & arow_ok) >> q & 1u) ? (TO)ra[q] : TO(0); }
  template <class TO>
  __device__ __forceinline__ TO b(int q) const { return ((bm & bcol_ok) >> q & 1u) ? (TO)rb[q] : TO(0); }
};

// C(cmap(i), j) = alpha * acc + beta * C(cmap(i), j) for the NR x NC values a
// thread holds (rows r[], columns c[]); map entries and old values of C are
// loaded in one batch each before any store.  TA is the accumulator type.
template <class TC, class TA, int NR, int NC>
__device__ __forceinline__ void store_c(const GemmDesc& g, const int* r, const int* c, const TA (*acc)[NC]) {
  const auto C = (gptr<TC>)g.C;
  int rr[NR], cc[NC];
#pragma unroll
  for (int x = 0; x < NR; ++x) rr[x] = min(r[x], g.m - 1);
#pragma unroll
  for (int y = 0; y < NC; ++y) cc[y] = min(c[y], g.n - 1);
  if (g.cmap) {
    const auto cmap = (gptr<const int>)g.cmap;
#pragma unroll
    for (int x = 0; x < NR; ++x) rr[x] = cmap[rr[x]];
  }
  TC val[NR][NC];
#pragma unroll
  for (int x = 0; x < NR; ++x)
#pragma unroll
    for (int y = 0; y < NC; ++y) val[x][y] = (TC)(g.alpha * (double)acc[x][y]);
  if (g.beta != 0.0) {
    TC old[NR][NC];
#pragma unroll
    for (int x = 0; x < NR; ++x)
#pragma unroll
      for (int y = 0; y < NC; ++y) old[x][y] = C[rr[x] + (int64_t)cc[y] * g.ldc];
#pragma unroll
    for (int x = 0; x < NR; ++x)
#pragma unroll
      for (int y = 0; y < NC; ++y) {
        // pin the loads here, ahead of the guarded stores below
        asm volatile("" : "+v"(old[x][y]));
        val[x][y] = (TC)(val[x][y] + (TC)g.beta * old[x][y]);
      }
  }
#pragma unroll
  for (int x = 0; x < NR; ++x)
#pragma unroll
    for (int y = 0; y < NC; ++y)
      if (r[x] < g.m && c[y] < g.n) C[rr[x] + (int64_t)cc[y] * g.ldc] = val[x][y];
}

// ---------------------------------------------------------------- FP64 -----
// k-tiles of TK (16 or 32) double-buffered in LDS: while the matrix cores
// work on tile k0, every thread already holds its share of tile k0+TK in
// registers and stores it into the other buffer afterwards (one barrier per
// k-tile).  Each output accumulates over k in the same order for either TK.
template <int TK>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmBatch batch) {
  constexpr int PER = TM * TK / 256;   // elements of A (and of B) per thread per k-tile
  __shared__ double As[2][TK][TM + 1];
  __shared__ double Bs[2][TK][TN + 1];
  const GemmDesc g = batch_desc(batch, blockIdx.x);
  const int64_t t = blockIdx.x - g.tile_base;
  if (t >= (int64_t)g.tiles_m * g.tiles_n) return;
  const int row0 = (int)(t % g.tiles_m) * TM;
  const int col0 = (int)(t / g.tiles_m) * TN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  TileLoader<double, PER, TK, TM, TN> ld;
  ld.init(g, row0, col0);
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, kk, j, kb;
      ld.a_idx(q, i, kk);
      As[buf][kk][i] = ld.template a<double>(q);
      ld.b_idx(q, kb, j);
      Bs[buf][kb][j] = ld.template b<double>(q);
    }
  };
  dbl4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0, 0, 0, 0};
  int buf = 0;
  if (g.k > 0) {
    ld.fetch(g, 0, TK);
    store(0);
  }
  __syncthreads();
  for (int k0 = 0; k0 < g.k; k0 += TK) {
    const bool more = k0 + TK < g.k;
    if (more) ld.fetch(g, k0 + TK, k0 + 2 * TK);   // in flight while the matrix cores run
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kk = ks + (lane >> 4);
      const double a0 = As[buf][kk][wr + (lane & 15)];
      const double a1 = As[buf][kk][wr + 16 + (lane & 15)];
      const double b0 = Bs[buf][kk][wc + (lane & 15)];
      const double b1 = Bs[buf][kk][wc + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) store(buf ^ 1);   // the other buffer was last read before the previous barrier
    __syncthreads();
    buf ^= 1;
  }
  // FP64 16x16x4 result layout: lane l, slot v holds (row l/16 + 4v, col l%16)
  int r[8], c[2];
  double out[8][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      r[4 * a + v] = row0 + wr + a * 16 + (lane >> 4) + 4 * v;
#pragma unroll
      for (int b = 0; b < 2; ++b) out[4 * a + v][b] = acc[a][b][v];
    }
#pragma unroll
  for (int b = 0; b < 2; ++b) c[b] = col0 + wc + b * 16 + (lane & 15);
  store_c<double, double, 8, 2>(g, r, c, out);
}

// 128 x 128 tiles for large products: four wavefronts each own a 64 x 64
// quadrant (4 x 4 MFMA blocks).  Every output accumulates over k in the same
// order as gemm_f64_kernel (k-tiles of 16, one 16x16x4 MFMA per 4), so the
// two kernels give identical results; the choice between them is speed only.
__global__ __launch_bounds__(256) void gemm_f64_128_kernel(const GemmBatch batch) {
  constexpr int BM = 128, BN = 128, TK = 16, PER = BM * TK / 256;
  __shared__ double As[2][TK][BM + 1];
  __shared__ double Bs[2][TK][BN + 1];
  const GemmDesc g = batch_desc(batch, blockIdx.x);
  const int64_t t = blockIdx.x - g.tile_base;
  if (t >= (int64_t)g.tiles_m * g.tiles_n) return;
  const int row0 = (int)(t % g.tiles_m) * BM;
  const int col0 = (int)(t / g.tiles_m) * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;
  TileLoader<double, PER, TK, BM, BN> ld;
  ld.init(g, row0, col0);
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, kk, j, kb;
      ld.a_idx(q, i, kk);
      As[buf][kk][i] = ld.template a<double>(q);
      ld.b_idx(q, kb, j);
      Bs[buf][kb][j] = ld.template b<double>(q);
    }
  };
  dbl4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = dbl4{0, 0, 0, 0};
  int buf = 0;
  if (g.k > 0) {
    ld.fetch(g, 0, TK);
    store(0);
  }
  __syncthreads();
  for (int k0 = 0; k0 < g.k; k0 += TK) {
    const bool more = k0 + TK < g.k;
    if (more) ld.fetch(g, k0 + TK, k0 + 2 * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kk = ks + (lane >> 4);
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[buf][kk][wr + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[buf][kk][wc + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // two passes of 32 values keep the epilogue's registers in bounds
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int r[8], c[4];
    double out[8][4];
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 2 * h + a2;
        r[4 * a2 + v] = row0 + wr + a * 16 + (lane >> 4) + 4 * v;
#pragma unroll
        for (int b = 0; b < 4; ++b) out[4 * a2 + v][b] = acc[a][b][v];
      }
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] = col0 + wc + b * 16 + (lane & 15);
    store_c<double, double, 8, 4>(g, r, c, out);
  }
}

// ------------------------------------------------- FP32 / BF16 inputs -----
// A, B stored in float (FP32 path) or __bf16 (BF16 path); products
// accumulate in FP32; C is stored as TOut (float, or double when a low
// precision product is added into an FP64 result).
template <class TIn, class TOut>
__global__ __launch_bounds__(256) void gemm_lp_kernel(const GemmBatch batch) {
  constexpr int TK = 32;
  constexpr int PER = TM * TK / 256;
  __shared__ float As[2][TK][TM + 1];
  __shared__ float Bs[2][TK][TN + 1];
  const GemmDesc g = batch_desc(batch, blockIdx.x);
  const int64_t t = blockIdx.x - g.tile_base;
  if (t >= (int64_t)g.tiles_m * g.tiles_n) return;
  const int row0 = (int)(t % g.tiles_m) * TM;
  const int col0 = (int)(t / g.tiles_m) * TN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  TileLoader<TIn, PER, TK, TM, TN> ld;
  ld.init(g, row0, col0);
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, kk, j, kb;
      ld.a_idx(q, i, kk);
      As[buf][kk][i] = ld.template a<float>(q);
      ld.b_idx(q, kb, j);
      Bs[buf][kb][j] = ld.template b<float>(q);
    }
  };
  flt4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0, 0, 0, 0};
  // FP32 products with an FP64 result: each k-tile's FP32 sum (32 terms)
  // is added into FP64 accumulators, so the accumulated rounding stays at
  // the level of one 32-term FP32 sum instead of growing with k
  constexpr bool acc64 = sizeof(TOut) == 8 && sizeof(TIn) != 2;
  double acc_d[2][2][4];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) acc_d[a][b][v] = 0.0;
  int buf = 0;
  if (g.k > 0) {
    ld.fetch(g, 0, TK);
    store(0);
  }
  __syncthreads();
  for (int k0 = 0; k0 < g.k; k0 += TK) {
    const bool more = k0 + TK < g.k;
    if (more) ld.fetch(g, k0 + TK, k0 + 2 * TK);   // in flight while the matrix cores run
    if constexpr (sizeof(TIn) != 2) {   // FP32 inputs, or FP64 inputs rounded to FP32
#pragma unroll
      for (int ks = 0; ks < TK; ks += 4) {
        const int kk = ks + (lane >> 4);
        float a0 = As[buf][kk][wr + (lane & 15)], a1 = As[buf][kk][wr + 16 + (lane & 15)];
        float b0 = Bs[buf][kk][wc + (lane & 15)], b1 = Bs[buf][kk][wc + 16 + (lane & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    } else {
      // one 16x16x32 BF16 step: lane l holds k = 8*(l/16) .. +7
      bf16x8 a0, a1, b0, b1;
      const int kb = 8 * (lane >> 4);
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        a0[v] = (__bf16)As[buf][kb + v][wr + (lane & 15)];
        a1[v] = (__bf16)As[buf][kb + v][wr + 16 + (lane & 15)];
        b0[v] = (__bf16)Bs[buf][kb + v][wc + (lane & 15)];
        b1[v] = (__bf16)Bs[buf][kb + v][wc + 16 + (lane & 15)];
      }
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    if constexpr (acc64) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc_d[a][b][v] += (double)acc[a][b][v];
          acc[a][b] = flt4{0, 0, 0, 0};
        }
    }
    if (more) store(buf ^ 1);   // the other buffer was last read before the previous barrier
    __syncthreads();
    buf ^= 1;
  }
  // FP32 16x16 result layout: lane l, slot v holds (row 4(l/16) + v, col l%16)
  int r[8], c[2];
  using TAcc = std::conditional_t<acc64, double, float>;
  TAcc out[8][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      r[4 * a + v] = row0 + wr + a * 16 + 4 * (lane >> 4) + v;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if constexpr (acc64) out[4 * a + v][b] = acc_d[a][b][v];
        else out[4 * a + v][b] = acc[a][b][v];
      }
    }
#pragma unroll
  for (int b = 0; b < 2; ++b) c[b] = col0 + wc + b * 16 + (lane & 15);
  store_c<TOut, TAcc, 8, 2>(g, r, c, out);
}

// 128 x 128 tiles for large FP32-input products: eight wavefronts (512
// threads) each own a 64 x 32 block (4 x 2 MFMA blocks), k-tiles of 32 as in
// gemm_lp_kernel, so each output accumulates over k in exactly the same
// order and the two kernels give identical results.  Each thread loads 8
// entries of A and of B per k-tile at fixed offsets from one row (or
// column, or k) it owns, with addresses formed as it goes instead of held
// per entry, which keeps the registers of both operands, the FP32 block
// accumulators and the FP64 sums of the FP64-result forms within budget.
template <class TIn, class TOut>
__global__ __launch_bounds__(512) void gemm_lp_128_kernel(const GemmBatch batch) {
  constexpr int BM = 128, BN = 128, TK = 32, NT = 512, PER = BM * TK / NT;   // 8
  __shared__ float As[2][TK][BM + 1];
  __shared__ float Bs[2][TK][BN + 1];
  const GemmDesc g = batch_desc(batch, blockIdx.x);
  const int64_t t = blockIdx.x - g.tile_base;
  if (t >= (int64_t)g.tiles_m * g.tiles_n) return;
  const int row0 = (int)(t % g.tiles_m) * BM;
  const int col0 = (int)(t / g.tiles_m) * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 64, wc = (wave >> 1) * 32;
  const auto A = (gptr<const TIn>)g.A;
  const auto B = (gptr<const TIn>)g.B;
  const bool tA = g.transA, tB = g.transB;
  // entry q of a k-tile: op(A)(ia + sa q, ka + ta q), op(B)(kb + tb q, jb + sb q)
  const int ia = tA ? tid >> 5 : tid & 127, ka = tA ? tid & 31 : tid >> 7;
  const int kb = tB ? tid >> 7 : tid & 31, jb = tB ? tid & 127 : tid >> 5;
  // the fixed row of A (!tA, through the row map) and column of B (tB)
  int64_t arow = 0, bcol = 0;
  if (!tA) {
    const int ic = min(row0 + ia, g.m - 1);
    arow = g.amap ? ((gptr<const int>)g.amap)[ic] : ic;
  }
  if (tB) bcol = min(col0 + jb, g.n - 1);
  TIn ra[PER], rb[PER];
  unsigned aok = 0, bok = 0;
  auto fetch = [&](int k0) {
    aok = bok = 0;
    int64_t ao[PER], bo[PER];
    // B's k row through the map (!tB): one lookup per k-tile
    int64_t bk = 0;
    if (!tB) {
      const int kc = min(k0 + kb, g.k - 1);
      bk = g.bmap ? ((gptr<const int>)g.bmap)[kc] : kc;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      if (tA) {
        const int ig = row0 + ia + 16 * q, k = k0 + ka;
        aok |= (unsigned)(ig < g.m && k < g.k) << q;
        ao[q] = (int64_t)min(k, g.k - 1) + (int64_t)min(ig, g.m - 1) * g.lda;
      } else {
        const int k = k0 + ka + 4 * q;
        aok |= (unsigned)(row0 + ia < g.m && k < g.k) << q;
        ao[q] = arow + (int64_t)min(k, g.k - 1) * g.lda;
      }
      if (tB) {
        const int k = k0 + kb + 4 * q;
        bok |= (unsigned)(col0 + jb < g.n && k < g.k) << q;
        bo[q] = bcol + (int64_t)min(k, g.k - 1) * g.ldb;
      } else {
        const int jg = col0 + jb + 16 * q, k = k0 + kb;
        bok |= (unsigned)(jg < g.n && k < g.k) << q;
        bo[q] = bk + (int64_t)min(jg, g.n - 1) * g.ldb;
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) ra[q] = A[ao[q]];
#pragma unroll
    for (int q = 0; q < PER; ++q) rb[q] = B[bo[q]];
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tA ? ia + 16 * q : ia, kk = tA ? ka : ka + 4 * q;
      As[buf][kk][i] = (aok >> q & 1u) ? (float)ra[q] : 0.0f;
      const int j = tB ? jb : jb + 16 * q, kq = tB ? kb + 4 * q : kb;
      Bs[buf][kq][j] = (bok >> q & 1u) ? (float)rb[q] : 0.0f;
    }
  };
  flt4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0, 0, 0, 0};
  // FP64-result forms: each k-tile's FP32 sum is added into FP64 sums, as
  // in gemm_lp_kernel
  constexpr bool acc64 = sizeof(TOut) == 8;
  double acc_d[4][2][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc_d[a][b][v] = 0.0;
  int buf = 0;
  if (g.k > 0) {
    fetch(0);
    store(0);
  }
  __syncthreads();
  for (int k0 = 0; k0 < g.k; k0 += TK) {
    const bool more = k0 + TK < g.k;
    if (more) fetch(k0 + TK);   // in flight while the matrix cores run
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kk = ks + (lane >> 4);
      float av[4], bv[2];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[buf][kk][wr + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[buf][kk][wc + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if constexpr (acc64) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc_d[a][b][v] += (double)acc[a][b][v];
          acc[a][b] = flt4{0, 0, 0, 0};
        }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // FP32 16x16 result layout: lane l, slot v holds (row 4(l/16) + v, col
  // l%16); two passes of 16 values keep the epilogue's registers in bounds
  using TAcc = std::conditional_t<acc64, double, float>;
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {
    int r[8], c[2];
    TAcc out[8][2];
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 2 * h2 + a2;
        r[4 * a2 + v] = row0 + wr + 16 * a + 4 * (lane >> 4) + v;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if constexpr (acc64) out[4 * a2 + v][b] = acc_d[a][b][v];
          else out[4 * a2 + v][b] = acc[a][b][v];
        }
      }
#pragma unroll
    for (int b = 0; b < 2; ++b) c[b] = col0 + wc + 16 * b + (lane & 15);
    store_c<TOut, TAcc, 8, 2>(g, r, c, out);
  }
}

// C(cmap(i), j) = alpha * sum_c P_c(i, j) + beta * C(cmap(i), j): the
// fixed-order reduction of split-K partial products (no atomics)
struct SplitRed {
  const double* P;   // nsplit partial m x n blocks, ld m
  void* C;
  const int* cmap;
  int m, n, ldc, nsplit;
  double alpha, beta;
};

template <class TOut>
__global__ void splitk_reduce_kernel(const SplitRed* __restrict__ rs) {
  const SplitRed r = rs[blockIdx.y];
  const int64_t mn = (int64_t)r.m * r.n;
  TOut* C = static_cast<TOut*>(r.C);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % r.m), j = (int)(e / r.m);
    double acc = 0.0;
    for (int c = 0; c < r.nsplit; ++c) acc += r.P[e + c * mn];
    const int ri = r.cmap ? r.cmap[i] : i;
    TOut* o = C + ri + (int64_t)j * r.ldc;
    const double v = r.alpha * acc;
    *o = (TOut)(r.beta == 0.0 ? v : v + r.beta * (double)*o);
  }
}

namespace {
// element size of the A / B operands of a GEMM type
size_t in_bytes(GemmType t) {
  return (t == GEMM_F64 || t == GEMM_D_F32) ? 8 : (t == GEMM_F32 || t == GEMM_F32_D) ? 4 : 2;
}

void launch_tiles(const std::vector<GemmDesc>& d, int64_t tiles, GemmType type, Stager& st, hipStream_t s,
                  double flops, int tile) {
  GemmBatch b;
  b.nd = (int)d.size();
  b.pad = 0;
  if (d.size() <= (size_t)kGemmInline) {
    b.descs = nullptr;
    std::copy(d.begin(), d.end(), b.inl);
  } else {
    b.descs = st.put_vec(d, s);
  }
  // the 128 x 128 FP32-input kernel runs 512 threads, the others 256
  const bool lp128 = tile == 128 && (type == GEMM_F32 || type == GEMM_F32_D || type == GEMM_D_F32);
  dim3 grid((unsigned)tiles), blk(lp128 ? 512 : 256);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof::enabled()) prof::ext(type == GEMM_F64 ? 1 : 2, flops, &e0, &e1);   // timing hook
#define HSSMF_GEMM_LAUNCH(K)                                                      \
  if (e0) hipExtLaunchKernelGGL(K, grid, blk, 0, s, e0, e1, 0, b);                \
  else hipLaunchKernelGGL(K, grid, blk, 0, s, b);
  switch (type) {
    case GEMM_F64:
      if (tile == 128) { HSSMF_GEMM_LAUNCH(gemm_f64_128_kernel) }
      else if (tile == 65) { HSSMF_GEMM_LAUNCH(gemm_f64_kernel<32>) }
      else { HSSMF_GEMM_LAUNCH(gemm_f64_kernel<16>) }
      break;
    case GEMM_F32:
      if (lp128) { HSSMF_GEMM_LAUNCH((gemm_lp_128_kernel<float, float>)) }
      else { HSSMF_GEMM_LAUNCH((gemm_lp_kernel<float, float>)) }
      break;
    case GEMM_F32_D:
      if (lp128) { HSSMF_GEMM_LAUNCH((gemm_lp_128_kernel<float, double>)) }
      else { HSSMF_GEMM_LAUNCH((gemm_lp_kernel<float, double>)) }
      break;
    case GEMM_D_F32:
      if (lp128) { HSSMF_GEMM_LAUNCH((gemm_lp_128_kernel<double, double>)) }
      else { HSSMF_GEMM_LAUNCH((gemm_lp_kernel<double, double>)) }
      break;
    case GEMM_BF16: HSSMF_GEMM_LAUNCH((gemm_lp_kernel<__bf16, float>)) break;
    case GEMM_BF16_D: HSSMF_GEMM_LAUNCH((gemm_lp_kernel<__bf16, double>)) break;
  }
#undef HSSMF_GEMM_LAUNCH
  HIP_CHECK(hipGetLastError());
}

// tile counts and prefix offsets of a batch for square tiles of side T
int64_t set_tiles(std::vector<GemmDesc>& d, int T) {
  if (T == 65) T = 64;   // 64 x 64 tiles, k-tiles of 32
  int64_t t = 0;
  for (auto& g : d) {
    g.tiles_m = (g.m + T - 1) / T;
    g.tiles_n = (g.n + T - 1) / T;
    g.tile_base = t;
    t += (int64_t)g.tiles_m * g.tiles_n;
  }
  return t;
}

// Tile autotuner: the first time a batch of a given type and shape class
// (log2 of its largest k, log2 of its 64 x 64 tile count) is large enough to
// matter, the kernel variants of that type (FP64: 64 x 64 tiles with k-tiles
// of 16 or 32, 128 x 128 tiles; FP32 inputs: 64 x 64 or 128 x 128 tiles)
// are timed on the same operands with the products written to the
// workspace, and the fastest is kept for that class for the rest of the
// process.  The results do not depend on the choice.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int>& tune_table() {
  static std::map<std::tuple<int, int, int>, int> t;
  return t;
}

int tuned_tile(const std::vector<GemmDesc>& d, GemmType type, int64_t tiles64, int64_t kmax, double flops,
               Stager& st, hipStream_t s) {
  if (flops < 2e8 || tiles64 < 16) return 64;
  auto lg = [](int64_t v) { int b = 0; while ((int64_t(1) << (b + 1)) <= v) ++b; return b; };
  const std::tuple<int, int, int> key{(int)type, lg(std::max<int64_t>(kmax, 1)), lg(tiles64)};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = tune_table().find(key);
    if (it != tune_table().end()) return it->second;
  }
  int64_t mn = 0;
  for (auto& g : d) mn += (int64_t)g.m * g.n;
  int choice = 64;
  if ((size_t)mn <= st.ws_elems) {
    std::vector<GemmDesc> tr = d;
    int64_t off = 0;
    for (auto& g : tr) {
      g.C = st.ws + off;
      g.ldc = g.m;
      g.cmap = nullptr;
      g.beta = 0.0;
      off += (int64_t)g.m * g.n;
    }
    // FP64 variants: 64 x 64 with k-tiles of 16 (64), of 32 (65), 128 x 128
    // (128); FP32 inputs: 64 x 64 (64), 128 x 128 (128).  Two rounds, the
    // second one timed
    const bool f64 = type == GEMM_F64;
    const int nv = f64 ? 3 : 2;
    const int var64[3] = {64, 65, 128}, varlp[2] = {64, 128};
    const int* var = f64 ? var64 : varlp;
    hipEvent_t ev[7];
    for (auto& e : ev) HIP_CHECK(hipEventCreate(&e));
    HIP_CHECK(hipEventRecord(ev[0], s));
    for (int rep = 0; rep < 2; ++rep)
      for (int vi = 0; vi < nv; ++vi) {
        const int64_t nt = set_tiles(tr, var[vi]);
        launch_tiles(tr, nt, type, st, s, 0.0, var[vi]);
        HIP_CHECK(hipEventRecord(ev[1 + nv * rep + vi], s));
      }
    HIP_CHECK(hipEventSynchronize(ev[2 * nv]));
    float best = 0.0f;
    for (int vi = 0; vi < nv; ++vi) {
      float ms = 0.0f;
      HIP_CHECK(hipEventElapsedTime(&ms, ev[nv + vi], ev[nv + 1 + vi]));
      if (vi == 0 || ms < best) { best = ms; choice = var[vi]; }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_table()[key] = choice;
  return choice;
}
}  // namespace

namespace {
// shape census of the batched GEMMs (diagnostics, HSSMF_GEMM_CENSUS=1):
// every call is timed with a synchronizing event pair and binned by its
// largest k and its tile count
struct CensusBin {
  int64_t calls = 0, tiles = 0;
  double flops = 0, ms = 0;
};
bool census_on() {
  static int on = -1;
  if (on < 0) {
    const char* e = std::getenv("HSSMF_GEMM_CENSUS");
    on = (e && *e == '1') ? 1 : 0;
  }
  return on == 1;
}
std::map<std::pair<int, int>, CensusBin>& census() {
  static std::map<std::pair<int, int>, CensusBin> c;
  return c;
}
int log2bin(int64_t v) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= v) ++b;
  return b;
}
}  // namespace

void gemm_census_print() {
  if (!census_on()) return;
  std::fprintf(stderr, "gemm census: kmax-bin tiles-bin calls tiles GFLOP ms TFLOP/s\n");
  for (auto& kv : census())
    std::fprintf(stderr, "  k<2^%d tiles<2^%d %8lld %10lld %9.2f %9.2f %6.2f\n", kv.first.first + 1,
                 kv.first.second + 1, (long long)kv.second.calls, (long long)kv.second.tiles, kv.second.flops / 1e9,
                 kv.second.ms, kv.second.ms > 0 ? kv.second.flops / kv.second.ms / 1e9 : 0.0);
  census().clear();
}

void gemm_batched(const std::vector<GemmDesc>& in, GemmType type, Stager& st, hipStream_t s, int tile_pref) {
  std::vector<GemmDesc> d;
  d.reserve(in.size());
  int64_t tiles = 0;
  double flops = 0.0;
  for (const GemmDesc& g0 : in) {
    if (g0.m <= 0 || g0.n <= 0) continue;
    GemmDesc g = g0;
    if (g.k <= 0) {
      if (g.beta == 1.0) continue;
      g.k = 0;  // alpha * 0 + beta * C: still launched to scale C
    }
    g.tiles_m = (g.m + TM - 1) / TM;
    g.tiles_n = (g.n + TN - 1) / TN;
    tiles += (int64_t)g.tiles_m * g.tiles_n;
    flops += 2.0 * g.m * g.n * (double)g.k;
    d.push_back(g);
  }
  if (d.empty()) return;
  REQUIRE(tiles < (1LL << 31), HSSMF_EINVAL, "gemm batch too large");
  hipEvent_t ce0 = nullptr, ce1 = nullptr;
  if (census_on()) {
    HIP_CHECK(hipEventCreate(&ce0));
    HIP_CHECK(hipEventCreate(&ce1));
    HIP_CHECK(hipEventRecord(ce0, s));
  }
  // split-K when the batch has too few output tiles to fill the chip and
  // the reductions are long: partial products into the workspace, then a
  // fixed-order reduction (the result is bitwise reproducible)
  int64_t kmax = 0, mnsum = 0;
  for (auto& g : d) { kmax = std::max<int64_t>(kmax, g.k); mnsum += (int64_t)g.m * g.n; }
  int nsplit = 1;
  while (nsplit < 16 && tiles * nsplit < 1024 && kmax / (2 * nsplit) >= 256) nsplit *= 2;
  const bool split = nsplit > 1 && (size_t)(mnsum * nsplit) <= st.ws_elems;
  // tile size (FP64 only): forced, or from the autotuner (the split-K
  // decision above uses the 64 x 64 tile count either way)
  int tile = 64;
  if (type == GEMM_F64) {
    if (tile_pref == 64 || tile_pref == 65 || tile_pref == 128) tile = tile_pref;
    else if (!split) tile = tuned_tile(d, type, tiles, kmax, flops, st, s);
  } else if (type != GEMM_BF16 && type != GEMM_BF16_D) {
    if (tile_pref == 64 || tile_pref == 65 || tile_pref == 128) tile = tile_pref == 65 ? 64 : tile_pref;
    else if (!split) tile = tuned_tile(d, type, tiles, kmax, flops, st, s);
  }
  if (split) {
    std::vector<GemmDesc> parts;
    std::vector<SplitRed> red;
    int64_t wsoff = 0, ptiles = 0;
    for (auto& g : d) {
      const int64_t mn = (int64_t)g.m * g.n;
      SplitRed r{st.ws + wsoff, g.C, g.cmap, g.m, g.n, g.ldc, nsplit, g.alpha, g.beta};
      const int kc = (g.k + nsplit - 1) / nsplit;
      const size_t eb = in_bytes(type);
      for (int c = 0; c < nsplit; ++c) {
        GemmDesc p = g;
        const int k0 = c * kc;
        p.k = std::max(0, std::min(g.k, k0 + kc) - k0);
        const char* A = static_cast<const char*>(g.A);
        const char* B = static_cast<const char*>(g.B);
        if (g.transA) A += (size_t)k0 * eb; else A += (size_t)k0 * g.lda * eb;
        if (g.transB) B += (size_t)k0 * g.ldb * eb;
        else if (g.bmap) p.bmap = g.bmap + k0;
        else B += (size_t)k0 * eb;
        p.A = A;
        p.B = B;
        p.C = st.ws + wsoff + c * mn;
        p.ldc = g.m;
        p.cmap = nullptr;
        p.alpha = 1.0;
        p.beta = 0.0;
        p.tile_base = ptiles;
        ptiles += (int64_t)p.tiles_m * p.tiles_n;
        parts.push_back(p);
      }
      red.push_back(r);
      wsoff += mn * nsplit;
    }
    // partial products are always accumulated and stored in FP64 here
    GemmType pt = type;
    if (type == GEMM_F32) pt = GEMM_F32_D;
    if (type == GEMM_BF16) pt = GEMM_BF16_D;
    if (tile != 64) ptiles = set_tiles(parts, tile);
    launch_tiles(parts, ptiles, pt, st, s, flops, tile);
    int64_t mx = 0;
    for (auto& r : red) mx = std::max<int64_t>(mx, (int64_t)r.m * r.n);
    int64_t bx = std::min<int64_t>((mx + 255) / 256, 2048);
    SplitRed* dr = st.put_vec(red, s);
    if (type == GEMM_F32 || type == GEMM_BF16)
      hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3((unsigned)bx, (unsigned)red.size()), dim3(256), 0, s, dr);
    else
      hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3((unsigned)bx, (unsigned)red.size()), dim3(256), 0, s, dr);
    HIP_CHECK(hipGetLastError());
  } else {
    const int64_t nt = set_tiles(d, tile);
    launch_tiles(d, nt, type, st, s, flops, tile);
  }
  if (ce0) {
    HIP_CHECK(hipEventRecord(ce1, s));
    HIP_CHECK(hipEventSynchronize(ce1));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, ce0, ce1));
    (void)hipEventDestroy(ce0);
    (void)hipEventDestroy(ce1);
    int64_t km = 0;
    for (auto& g : d) km = std::max<int64_t>(km, g.k);
    CensusBin& b = census()[{log2bin(std::max<int64_t>(km, 1)), log2bin(tiles)}];
    b.calls++;
    b.tiles += tiles;
    b.flops += flops;
    b.ms += ms;
  }
}

}  // namespace hssmf

// Kernels of the HSS fronts (Sec. 2.2, Sec. 4): keyed Gaussian random
// matrix, sparse products with the original entries of a front, batched
// gathers / copies, element extraction from F_i = A_i (+) U_children, the
// column-pivoted QR behind the interpolative decomposition, plain
// Householder QR for the ULV step, and blocked triangular solves.
#include "kernels.hpp"

namespace hssmf {

// ---------------------------------------------------------------- RNG ----
// Philox4x32-10 (Salmon et al., SC'11) keyed by (row id, seed low word),
// counter (column, seed high word, 0, 0); Box-Muller on 53-bit uniforms.
// Entry (row, c) depends only on (seed, original row id, c), so fronts that
// share a row agree on it (the extend-merge of the random vectors).
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void rng_kernel(double* R, int ldr, const int* __restrict__ orig, int nrows, int c0, int nc,
                           uint32_t seed_lo, uint32_t seed_hi) {
  const int64_t total = (int64_t)nrows * nc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e % nrows), c = c0 + (int)(e / nrows);
    uint32_t x[4] = {(uint32_t)c, seed_hi, 0u, 0u};
    philox10(x, (uint32_t)orig[i], seed_lo);
    double a = (double)(x[0] >> 5), b = (double)(x[1] >> 6);
    double u1 = (a * 67108864.0 + b + 1.0) * (1.0 / 9007199254740992.0);
    double a2 = (double)(x[2] >> 5), b2 = (double)(x[3] >> 6);
    double u2 = (a2 * 67108864.0 + b2) * (1.0 / 9007199254740992.0);
    R[i + (int64_t)c * ldr] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

void launch_rng(double* R, int ldr, const int* orig, int nrows, int c0, int nc, uint64_t seed, hipStream_t s) {
  int64_t total = (int64_t)nrows * nc;
  if (total <= 0) return;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(rng_kernel, dim3((unsigned)blocks), dim3(256), 0, s, R, ldr, orig, nrows, c0, nc,
                     (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32));
  HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------- SpMM ---
// A_i R for the original entries of a front (first term of Eq. FtimesR)
__global__ void spmm_kernel(const SpmmDesc* __restrict__ descs) {
  const SpmmDesc d = descs[blockIdx.z];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= d.nrows || c >= d.ncols) return;
  double acc = 0.0;
  for (int e = d.A.rowptr[i]; e < d.A.rowptr[i + 1]; ++e)
    acc += d.val[d.A.vidx[e]] * d.X[d.A.col[e] + (int64_t)c * d.ldx];
  d.Y[i + (int64_t)c * d.ldy] = acc;
}

void launch_spmm(const SpmmDesc* d, int nd, int max_rows, int max_cols, hipStream_t s) {
  if (nd <= 0 || max_rows <= 0 || max_cols <= 0) return;
  hipLaunchKernelGGL(spmm_kernel, dim3((max_rows + 255) / 256, max_cols, nd), dim3(256), 0, s, d);
  HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------- copy ---
// dst(i, j) [+]= alpha * src(rmap(i), cmap(j)) (trans: src(cmap(j), rmap(i))).
// A plain copy runs over tiles of copy_tile_rows(m) rows, one destination row
// per thread and eight columns per thread; a transposed one over 64 x 64 tiles read along
// the source's contiguous dimension and turned around in LDS, so both sides
// stay coalesced.  Column indices past the edge are clamped to the last
// column, so every load is unconditional and a thread's loads are in flight
// together.  A clamped lane holds exactly the value of the last column; an
// overwriting copy stores it there again (the same value twice), an
// accumulating one skips it.
template <class TD, int U>
__device__ inline void store_batch(gptr<TD> D, int64_t ldd, int i, const int* j, int n, const double* v, int acc) {
  if (acc) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j[u] < n) D[i + (int64_t)j[u] * ldd] = (TD)((double)D[i + (int64_t)j[u] * ldd] + v[u]);
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) D[i + (int64_t)min(j[u], n - 1) * ldd] = (TD)v[u];
  }
}

template <class TD>
__global__ __launch_bounds__(256) void copy_kernel(const CopyBatch batch) {
  __shared__ double tile[64][65];
  const CopyDesc d = batch_get(batch, blockIdx.y);
  if (d.m <= 0 || d.n <= 0) return;
  const auto S = (gptr<const double>)d.src;
  const auto D = (gptr<TD>)d.dst;
  const auto rmap = (gptr<const int>)d.rmap;
  const auto cmap = (gptr<const int>)d.cmap;
  if (!d.trans) {
    const int TR = copy_tile_rows(d.m), G = 256 / TR, TC = 8 * G;
    const int r = (int)threadIdx.x % TR, c0 = (int)threadIdx.x / TR, cs = G;
    const int tm = (d.m + TR - 1) / TR, tn = (d.n + TC - 1) / TC;
    for (int t = blockIdx.x; t < tm * tn; t += gridDim.x) {
      const int i = (t % tm) * TR + r, jb = (t / tm) * TC + c0;
      if (i >= d.m) continue;
      const int si = rmap ? rmap[i] : i;
      int jj[8], sj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        jj[u] = jb + u * cs;
        sj[u] = min(jj[u], d.n - 1);
      }
      if (cmap) {
#pragma unroll
        for (int u = 0; u < 8; ++u) sj[u] = cmap[sj[u]];
      }
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = d.alpha * S[si + (int64_t)sj[u] * d.lds];
      store_batch<TD, 8>(D, d.ldd, i, jj, d.n, v, d.accumulate);
    }
    return;
  }
  const int tm = (d.m + 63) / 64, tn = (d.n + 63) / 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < tm * tn; t += gridDim.x) {
    const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
    // read src(cmap(j), rmap(i)) with j along the lanes; rows past the edge
    // are clamped as well (they are never stored)
    const int jr = min(j0 + tx, d.n - 1);
    const int sj = cmap ? cmap[jr] : jr;
    int si[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) si[u] = min(i0 + ty + 4 * u, d.m - 1);
    if (rmap) {
#pragma unroll
      for (int u = 0; u < 16; ++u) si[u] = rmap[si[u]];
    }
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = S[sj + (int64_t)si[u] * d.lds];
    __syncthreads();   // the previous tile has been read out
#pragma unroll
    for (int u = 0; u < 16; ++u) tile[ty + 4 * u][tx] = v[u];
    __syncthreads();
    const int i = i0 + tx;
    if (i < d.m) {
      int jj[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        jj[u] = j0 + ty + 4 * u;
        v[u] = d.alpha * tile[tx][ty + 4 * u];
      }
      store_batch<TD, 16>(D, d.ldd, i, jj, d.n, v, d.accumulate);
    }
  }
}

void launch_copy(const CopyBatch& d, int nd, int64_t max_tiles, int f32, hipStream_t s) {
  if (nd <= 0 || max_tiles <= 0) return;
  // one workgroup per tile of the largest copy (grid-stride beyond)
  const int64_t blocks = max_tiles < 4096 ? max_tiles : 4096;
  if (f32)
    hipLaunchKernelGGL(copy_kernel<float>, dim3((unsigned)blocks, nd), dim3(256), 0, s, d);
  else
    hipLaunchKernelGGL(copy_kernel<double>, dim3((unsigned)blocks, nd), dim3(256), 0, s, d);
  HIP_CHECK(hipGetLastError());
}

__global__ void convert_kernel(const double* __restrict__ src, void* dst, int64_t n, int to_bf16) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (to_bf16) static_cast<__bf16*>(dst)[i] = (__bf16)(float)src[i];
    else static_cast<float*>(dst)[i] = (float)src[i];
  }
}

void launch_convert(const double* src, void* dst, int64_t n, int to_bf16, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, to_bf16);
  HIP_CHECK(hipGetLastError());
}

__global__ void round_lp_kernel(double* x, void* lp, int64_t n, int to_bf16) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (to_bf16) {
      __bf16 v = (__bf16)(float)x[i];
      static_cast<__bf16*>(lp)[i] = v;
      x[i] = (double)(float)v;
    } else {
      float v = (float)x[i];
      static_cast<float*>(lp)[i] = v;
      x[i] = (double)v;
    }
  }
}

void launch_round_lp(double* x, void* lp, int64_t n, int to_bf16, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(round_lp_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, lp, n, to_bf16);
  HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------- extraction ---
// F_i(I, J) = A_i(I, J) + sum over children of U_child(inv(I), inv(J))
// (the element access that Alg. 1 needs for D and B, Sec. 4.5)
// entry (a, b) of a child's update matrix F22 - Theta^* Phi in low-rank
// form, by one wavefront: F22 from a leaf block or from Ubig of the lowest
// common ancestor's row-side child times B Vbig^T of the column side, minus
// row a of Theta^* times column b of Phi; the dot products are split over
// the lanes and summed by a butterfly (the same value in every lane)
__device__ double hss_kid_entry(const HssKidDev& K, int a, int b, int lane) {
  const HssKidNode* N = K.nodes;
  int x = K.leaf_of[a], y = K.leaf_of[b];
  double v = 0.0;
  if (x == y) {
    const HssKidNode& L = N[x];
    if (lane == 0) v = L.D[(a - L.lo) + (int64_t)(b - L.lo) * L.m];
  } else {
    while (N[x].depth > N[y].depth) x = N[x].parent;
    while (N[y].depth > N[x].depth) y = N[y].parent;
    while (N[x].parent != N[y].parent) {
      x = N[x].parent;
      y = N[y].parent;
    }
    const HssKidNode& P = N[N[x].parent];
    const HssKidNode& X = N[x];
    const HssKidNode& Y = N[y];
    const int ld = X.r > 1 ? X.r : 1;
    const double* T = (x == P.kid0 ? P.T12 : P.T21) + (int64_t)(b - Y.lo) * ld;
    const double* U = X.UT + (int64_t)(a - X.lo) * ld;
    for (int l = lane; l < X.r; l += 64) v += U[l] * T[l];
  }
  const double* th = K.ThT + (int64_t)a * K.mk;
  const double* ph = K.Phi + (int64_t)b * K.mk;
  for (int l = lane; l < K.mk; l += 64) v -= th[l] * ph[l];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ void extract_kernel(const ExtractDesc* __restrict__ descs, const FrontOpDev* __restrict__ fops) {
  const ExtractDesc d = descs[blockIdx.y];
  const FrontOpDev& f = fops[d.fop];
  const int64_t total = (int64_t)d.m * d.n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int r = (int)(e % d.m), c = (int)(e / d.m);
    int i = d.I[r], j = d.J[c];
    double v = 0.0;
    int lo = f.A.rowptr[i], hi = f.A.rowptr[i + 1] - 1;
    while (lo <= hi) {
      int mid = (lo + hi) >> 1;
      int cm = f.A.col[mid];
      if (cm == j) { v = f.val[f.A.vidx[mid]]; break; }
      if (cm < j) lo = mid + 1; else hi = mid - 1;
    }
    for (int k = 0; k < f.nkids; ++k) {
      if (f.hk[k]) continue;   // low-rank children: the second pass
      int a = f.inv[k][i], b = f.inv[k][j];
      if (a >= 0 && b >= 0) v += f.U[k][a + (int64_t)b * f.ldu[k]];
    }
    d.dst[r + (int64_t)c * d.ldd] = v;
  }
}

// the low-rank children's entries, added to what extract_kernel wrote: one
// wavefront per entry
__global__ __launch_bounds__(256) void extract_lowrank_kernel(const ExtractDesc* __restrict__ descs,
                                                              const FrontOpDev* __restrict__ fops) {
  const ExtractDesc d = descs[blockIdx.y];
  const FrontOpDev& f = fops[d.fop];
  bool any = false;
  for (int k = 0; k < f.nkids; ++k) any = any || f.hk[k] != nullptr;
  if (!any) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t total = (int64_t)d.m * d.n;
  for (int64_t e = blockIdx.x * 4 + w; e < total; e += (int64_t)gridDim.x * 4) {
    const int r = (int)(e % d.m), c = (int)(e / d.m);
    const int i = d.I[r], j = d.J[c];
    double v = 0.0;
    bool hit = false;
    for (int k = 0; k < f.nkids; ++k) {
      if (!f.hk[k]) continue;
      const int a = f.inv[k][i], b = f.inv[k][j];
      if (a >= 0 && b >= 0) {
        v += hss_kid_entry(*f.hk[k], a, b, lane);
        hit = true;
      }
    }
    if (hit && lane == 0) d.dst[r + (int64_t)c * d.ldd] += v;
  }
}

void launch_extract(const ExtractDesc* d, int nd, const FrontOpDev* fops, int64_t max_elems, bool lowrank,
                    hipStream_t s) {
  if (nd <= 0 || max_elems <= 0) return;
  int64_t blocks = (max_elems + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(extract_kernel, dim3((unsigned)blocks, nd), dim3(256), 0, s, d, fops);
  if (lowrank) {
    int64_t b2 = (max_elems + 3) / 4;
    if (b2 > 4096) b2 = 4096;
    hipLaunchKernelGGL(extract_lowrank_kernel, dim3((unsigned)b2, nd), dim3(256), 0, s, d, fops);
  }
  HIP_CHECK(hipGetLastError());
}

// --------------------------------------------------- interpolative basis --
__global__ void interp_kernel(const InterpDesc* __restrict__ descs) {
  const InterpDesc d = descs[blockIdx.y];
  const int64_t total = (int64_t)d.m * d.k;
  const int nr = d.m - d.k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e % d.m), j = (int)(e / d.m);
    double v = (i < d.k) ? (i == j ? 1.0 : 0.0) : d.E[(i - d.k) + (int64_t)j * nr];
    d.dst[d.perm[i] + (int64_t)j * d.ldd] = v;
  }
}

void launch_interp_dense(const InterpDesc* d, int nd, int64_t max_elems, hipStream_t s) {
  if (nd <= 0 || max_elems <= 0) return;
  int64_t blocks = (max_elems + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(interp_kernel, dim3((unsigned)blocks, nd), dim3(256), 0, s, d);
  HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------- row interchanges ---
// Row interchanges ipiv[0..k) (LAPACK order; reverse = undo them) applied to
// every column of M.  The interchange sequence is first folded into a
// permutation (one workgroup, in LDS), then every column is permuted through
// LDS: row i of the result is row perm[i] of the input.
__global__ __launch_bounds__(256) void perm_from_ipiv_kernel(const int* __restrict__ ipiv, int k, int* perm,
                                                             int reverse) {
  extern __shared__ int pm[];   // 2k ints: permutation, then the interchanges
  int* iv = pm + k;
  for (int i = threadIdx.x; i < k; i += 256) {
    pm[i] = i;
    iv[i] = ipiv[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!reverse)
      for (int i = 0; i < k; ++i) { const int p = iv[i]; const int t = pm[i]; pm[i] = pm[p]; pm[p] = t; }
    else
      for (int i = k - 1; i >= 0; --i) { const int p = iv[i]; const int t = pm[i]; pm[i] = pm[p]; pm[p] = t; }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += 256) perm[i] = pm[i];
}

__global__ __launch_bounds__(256) void permute_rows_kernel(double* M, int ld, int k, const int* __restrict__ perm) {
  extern __shared__ double cv[];
  double* col = M + (int64_t)blockIdx.x * ld;
  for (int i = threadIdx.x; i < k; i += 256) cv[i] = col[i];
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += 256) col[i] = cv[perm[i]];
}

void launch_pivots(double* M, int ld, int ncols, const int* ipiv, int k, int reverse, int* perm_ws, hipStream_t s) {
  if (ncols <= 0 || k <= 0) return;
  REQUIRE((size_t)k * 8 <= 64 * 1024, HSSMF_EINVAL, "row interchanges: more than 8192 rows");
  hipLaunchKernelGGL(perm_from_ipiv_kernel, dim3(1), dim3(256), (size_t)k * 2 * sizeof(int), s, ipiv, k, perm_ws,
                     reverse);
  hipLaunchKernelGGL(permute_rows_kernel, dim3(ncols), dim3(256), (size_t)k * sizeof(double), s, M, ld, k, perm_ws);
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------ blocked triangular solve --
// one diagonal block (rows [b0, b0+bs), bs <= 64) of T X = B: one
// wavefront per right-hand-side column, lane i holding row b0 + i, the
// substitution carried out with lane shuffles; the caller applies the
// off-diagonal updates with GEMMs between blocks
template <int LOWER, int UNIT, int TRANS>
__global__ __launch_bounds__(256) void trsm_block_kernel(const TrsmBatch batch) {
  const TrsmDesc d = batch_get(batch, blockIdx.y);
  __shared__ double Tb[64][65];
  const int bs = d.bs;
  if (bs <= 0) return;
  {
    // the diagonal block, read along the stored columns: all sixteen loads
    // of a thread unconditional (indices clamped into the block) and in
    // flight together, then stored to LDS where they belong to the block
    const auto T = (gptr<const double>)d.T;
    const int fast = threadIdx.x & 63, slow0 = threadIdx.x >> 6;
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int f = d.b0 + min(fast, bs - 1), sl = d.b0 + min(slow0 + 4 * u, bs - 1);
      v[u] = T[f + (int64_t)sl * d.ldt];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int sl = slow0 + 4 * u;
      if (fast < bs && sl < bs) {
        if (TRANS) Tb[sl][fast] = v[u];   // T(gi, gj) = stored (gj, gi)
        else Tb[fast][sl] = v[u];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int c = blockIdx.x * 4 + wave; c < d.ncols; c += gridDim.x * 4) {
    double* x = d.X + (int64_t)c * d.ldx + d.b0;
    double v = (lane < bs) ? x[lane] : 0.0;
    if (LOWER) {
      for (int j = 0; j < bs; ++j) {
        if (!UNIT && lane == j) v /= Tb[j][j];
        const double xj = __shfl(v, j);
        if (lane > j && lane < bs) v -= Tb[lane][j] * xj;
      }
    } else {
      for (int j = bs - 1; j >= 0; --j) {
        if (!UNIT && lane == j) v /= Tb[j][j];
        const double xj = __shfl(v, j);
        if (lane < j) v -= Tb[lane][j] * xj;
      }
    }
    if (lane < bs) x[lane] = v;
  }
}

void launch_trsm_block(const TrsmBatch& d, int nd, int lower, int unit, int trans, int max_cols, hipStream_t s) {
  if (nd <= 0 || max_cols <= 0) return;
  int gx = (max_cols + 3) / 4;
  if (gx > 512) gx = 512;
  dim3 g(gx, nd), b(256);
  int code = lower * 4 + unit * 2 + trans;
  switch (code) {
    case 0: hipLaunchKernelGGL((trsm_block_kernel<0, 0, 0>), g, b, 0, s, d); break;
    case 1: hipLaunchKernelGGL((trsm_block_kernel<0, 0, 1>), g, b, 0, s, d); break;
    case 2: hipLaunchKernelGGL((trsm_block_kernel<0, 1, 0>), g, b, 0, s, d); break;
    case 3: hipLaunchKernelGGL((trsm_block_kernel<0, 1, 1>), g, b, 0, s, d); break;
    case 4: hipLaunchKernelGGL((trsm_block_kernel<1, 0, 0>), g, b, 0, s, d); break;
    case 5: hipLaunchKernelGGL((trsm_block_kernel<1, 0, 1>), g, b, 0, s, d); break;
    case 6: hipLaunchKernelGGL((trsm_block_kernel<1, 1, 0>), g, b, 0, s, d); break;
    default: hipLaunchKernelGGL((trsm_block_kernel<1, 1, 1>), g, b, 0, s, d); break;
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace hssmf

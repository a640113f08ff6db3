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
template <class TD>
__global__ void copy_kernel(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.y];
  const int64_t total = (int64_t)d.m * d.n;
  const double* S = static_cast<const double*>(d.src);
  TD* D = static_cast<TD*>(d.dst);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e % d.m), j = (int)(e / d.m);
    int si = d.rmap ? d.rmap[i] : i;
    int sj = d.cmap ? d.cmap[j] : j;
    double v = d.trans ? S[sj + (int64_t)si * d.lds] : S[si + (int64_t)sj * d.lds];
    v *= d.alpha;
    TD* o = D + i + (int64_t)j * d.ldd;
    if (d.accumulate) *o = (TD)((double)*o + v); else *o = (TD)v;
  }
}

void launch_copy(const CopyDesc* d, int nd, int64_t max_elems, int f32, hipStream_t s) {
  if (nd <= 0 || max_elems <= 0) return;
  int64_t blocks = (max_elems + 255) / 256;
  if (blocks > 4096) blocks = 4096;
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

// ---------------------------------------------------------- extraction ---
// F_i(I, J) = A_i(I, J) + sum over children of U_child(inv(I), inv(J))
// (the element access that Alg. 1 needs for D and B, Sec. 4.3)
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
      int a = f.inv[k][i], b = f.inv[k][j];
      if (a >= 0 && b >= 0) v += f.U[k][a + (int64_t)b * f.ldu[k]];
    }
    d.dst[r + (int64_t)c * d.ldd] = v;
  }
}

void launch_extract(const ExtractDesc* d, int nd, const FrontOpDev* fops, int64_t max_elems, hipStream_t s) {
  if (nd <= 0 || max_elems <= 0) return;
  int64_t blocks = (max_elems + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(extract_kernel, dim3((unsigned)blocks, nd), dim3(256), 0, s, d, fops);
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------ Householder QR ---
// Y = S^T (d x m) is staged column by column (column j = row j of S), so
// every candidate is a contiguous vector.  One workgroup per problem; four
// wavefronts take the trailing columns round robin, each doing its dot
// product and update with a lane-stride loop and a shuffle reduction.
//
// PIVOT = true (interpolative decomposition, Sec. 2.2 and Sec. 5.4): the
// pivot is the column with the largest remaining 2-norm, recomputed from
// the updated column after every step (ties to the lowest index); stop
// before step i+1 when that norm <= eps * (first pivot norm).  Then
// X = R1^{-1} R2 and E = X^T.
// PIVOT = false: plain QR of all min(d, m) columns; writes L = R^T and the
// explicit d x d orthogonal factor Q (Y = Q R).
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <bool PIVOT>
__global__ __launch_bounds__(256) void qr_kernel(const QRDesc* __restrict__ descs) {
  extern __shared__ char lds_raw[];
  const QRDesc q = descs[blockIdx.x];
  const int m = q.m, d = q.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* nrm = reinterpret_cast<double*>(lds_raw);          // m
  double* tau = nrm + m;                                     // min(d, m)
  double* rv = tau + ((m < d) ? m : d);                      // 256 reduction values
  int* ri = reinterpret_cast<int*>(rv + 256);                // 256 reduction indices
  int* perm = ri + 256;                                      // m
  __shared__ double bcast[4];
  __shared__ int kout;
  double* W = q.W;
  // stage Y = S^T
  for (int64_t e = tid; e < (int64_t)m * d; e += 256) {
    int j = (int)(e / d), kk = (int)(e % d);
    W[kk + (int64_t)j * d] = q.S[j + (int64_t)kk * q.lds];
  }
  for (int j = tid; j < m; j += 256) perm[j] = j;
  __syncthreads();
  for (int j = wave; j < m; j += 4) {
    double acc = 0.0;
    for (int i = lane; i < d; i += 64) { double x = W[i + (int64_t)j * d]; acc += x * x; }
    acc = wave_sum(acc);
    if (lane == 0) nrm[j] = sqrt(acc);
  }
  __syncthreads();
  const int kmax = (m < d) ? m : d;
  double first = 0.0;
  int k = kmax;
  for (int t = 0; t < kmax; ++t) {
    int p = t;
    double best = nrm[t];
    if (PIVOT) {
      best = -1.0;
      for (int j = t + tid; j < m; j += 256)
        if (nrm[j] > best) { best = nrm[j]; p = j; }
      rv[tid] = best;
      ri[tid] = p;
      __syncthreads();
      for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
          double o = rv[tid + off];
          int oi = ri[tid + off];
          if (o > rv[tid] || (o == rv[tid] && oi < ri[tid])) { rv[tid] = o; ri[tid] = oi; }
        }
        __syncthreads();
      }
      best = rv[0];
      p = ri[0];
      __syncthreads();
      if (t == 0) {
        first = best;
        if (first == 0.0) { k = 0; break; }
      } else if (best <= q.eps * first) {
        k = t;
        break;
      }
      if (p != t) {
        for (int i = tid; i < d; i += 256) {
          double a = W[i + (int64_t)t * d];
          W[i + (int64_t)t * d] = W[i + (int64_t)p * d];
          W[i + (int64_t)p * d] = a;
        }
        if (tid == 0) {
          double x = nrm[t]; nrm[t] = nrm[p]; nrm[p] = x;
          int y = perm[t]; perm[t] = perm[p]; perm[p] = y;
        }
      }
      __syncthreads();
    }
    // Householder reflector for W[t:, t]; best = its 2-norm
    if (tid == 0) {
      double x0 = W[t + (int64_t)t * d];
      double alpha = (x0 >= 0.0) ? -best : best;
      double v0 = x0 - alpha;
      double vtv = v0 * v0 + (best * best - x0 * x0);
      double tv = (vtv > 0.0 && best > 0.0) ? 2.0 / vtv : 0.0;
      bcast[0] = v0;
      bcast[1] = tv;
      bcast[2] = alpha;
      tau[t] = tv;
      W[t + (int64_t)t * d] = v0;
    }
    __syncthreads();
    {
      const double tv = bcast[1];
      const double* v = W + (int64_t)t * d;
      for (int j = t + 1 + wave; j < m; j += 4) {
        double* col = W + (int64_t)j * d;
        double dot = 0.0;
        if (tv != 0.0) {
          for (int i = t + lane; i < d; i += 64) dot += v[i] * col[i];
          dot = wave_sum(dot) * tv;
        }
        double ss = 0.0;
        for (int i = t + lane; i < d; i += 64) {
          double x = col[i] - dot * v[i];
          col[i] = x;
          if (i > t) ss += x * x;
        }
        ss = wave_sum(ss);
        if (lane == 0) nrm[j] = sqrt(ss);   // exact recomputation, no downdating
      }
    }
    __syncthreads();
    if (tid == 0) {
      nrm[t] = bcast[0];                    // keep v0 (needed to form Q)
      W[t + (int64_t)t * d] = bcast[2];     // R_tt
    }
    __syncthreads();
  }
  if (tid == 0) kout = k;
  __syncthreads();
  k = kout;
  if (PIVOT) {
    if (tid == 0) *q.rank = k;
    for (int j = tid; j < m; j += 256) q.perm[j] = perm[j];
    // X = R1^{-1} R2, one column per thread, then E = X^T
    const int nrest = m - k;
    for (int j = k + tid; j < m; j += 256) {
      double* col = W + (int64_t)j * d;
      for (int i = k - 1; i >= 0; --i) {
        double acc = col[i];
        for (int l = i + 1; l < k; ++l) acc -= W[i + (int64_t)l * d] * col[l];
        col[i] = acc / W[i + (int64_t)i * d];
      }
      for (int l = 0; l < k; ++l) q.E[(j - k) + (int64_t)l * nrest] = col[l];
    }
  } else {
    if (tid == 0) *q.rank = k;
    // L = R^T (k x k)
    for (int64_t e = tid; e < (int64_t)k * k; e += 256) {
      int i = (int)(e % k), j = (int)(e / k);
      q.L[i + (int64_t)j * k] = (i >= j) ? W[j + (int64_t)i * d] : 0.0;
    }
    // Q = H_0 H_1 ... H_{k-1}: apply the reflectors in reverse order to I
    if (q.Q) {
      double* Q = q.Q;
      for (int64_t e = tid; e < (int64_t)d * d; e += 256) {
        int i = (int)(e % d), j = (int)(e / d);
        Q[i + (int64_t)j * d] = (i == j) ? 1.0 : 0.0;
      }
      __syncthreads();
      for (int t = k - 1; t >= 0; --t) {
        const double tv = tau[t];
        if (tv == 0.0) continue;
        const double v0 = nrm[t];
        const double* v = W + (int64_t)t * d;  // v[i] for i > t; v[t] = v0
        for (int j = wave; j < d; j += 4) {
          double* col = Q + (int64_t)j * d;
          double dot = 0.0;
          for (int i = t + lane; i < d; i += 64) dot += ((i == t) ? v0 : v[i]) * col[i];
          dot = wave_sum(dot) * tv;
          for (int i = t + lane; i < d; i += 64) col[i] -= dot * ((i == t) ? v0 : v[i]);
        }
        __syncthreads();
      }
    }
  }
}

void launch_qr(const QRDesc* d, int nd, int pivot, int max_m, hipStream_t s) {
  if (nd <= 0) return;
  size_t lds = (size_t)max_m * 8 * 2 + 256 * 8 + 256 * 4 + (size_t)max_m * 4;
  REQUIRE(lds <= 64 * 1024, HSSMF_ERANK, "interpolative decomposition: node too large for one workgroup");
  if (pivot)
    hipLaunchKernelGGL(qr_kernel<true>, dim3(nd), dim3(256), lds, s, d);
  else
    hipLaunchKernelGGL(qr_kernel<false>, dim3(nd), dim3(256), lds, s, d);
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
__global__ void pivots_kernel(double* M, int ld, int ncols, const int* ipiv, int k, int reverse) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  double* col = M + (int64_t)c * ld;
  if (!reverse) {
    for (int i = 0; i < k; ++i) { int p = ipiv[i]; if (p != i) { double t = col[i]; col[i] = col[p]; col[p] = t; } }
  } else {
    for (int i = k - 1; i >= 0; --i) { int p = ipiv[i]; if (p != i) { double t = col[i]; col[i] = col[p]; col[p] = t; } }
  }
}

void launch_pivots(double* M, int ld, int ncols, const int* ipiv, int k, int reverse, hipStream_t s) {
  if (ncols <= 0 || k <= 0) return;
  hipLaunchKernelGGL(pivots_kernel, dim3((ncols + 255) / 256), dim3(256), 0, s, M, ld, ncols, ipiv, k, reverse);
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------ blocked triangular solve --
// one diagonal block (rows [b0, b0+bs), bs <= 64) of T X = B: one
// wavefront per right-hand-side column, lane i holding row b0 + i, the
// substitution carried out with lane shuffles; the caller applies the
// off-diagonal updates with GEMMs between blocks
template <int LOWER, int UNIT, int TRANS>
__global__ __launch_bounds__(256) void trsm_block_kernel(const TrsmDesc* __restrict__ descs) {
  const TrsmDesc d = descs[blockIdx.y];
  __shared__ double Tb[64][65];
  const int bs = d.bs;
  for (int e = threadIdx.x; e < bs * bs; e += 256) {
    int i = e % bs, j = e / bs;
    int gi = d.b0 + i, gj = d.b0 + j;
    Tb[i][j] = TRANS ? d.T[gj + (int64_t)gi * d.ldt] : d.T[gi + (int64_t)gj * d.ldt];
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

void launch_trsm_block(const TrsmDesc* d, int nd, int lower, int unit, int trans, int max_cols, hipStream_t s) {
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

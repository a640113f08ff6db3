// Dense-front kernels of the multifrontal method (Sec. 3.2, Sec. 3.3):
// assembly of original entries, extend-add of children's update matrices,
// the pieces of a batched right-looking blocked partial LU with pivoting
// restricted to F11, and the per-front triangular solves / products of the
// forward and backward sweeps.  All fronts of one elimination-tree level go
// through each launch together.
#include <type_traits>

#include <cstdlib>

#include "kernels.hpp"

namespace hssmf {

// ------------------------------------------------------------- utilities --
__global__ void fill_kernel(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  HIP_CHECK(hipGetLastError());
}

// assembly: front entries from the CSR values (Eq. frontal_1); each front
// position receives exactly one entry, so the scatter has no conflicts
__global__ void assemble_kernel(double* base, const int64_t* __restrict__ dst, const int64_t* __restrict__ src,
                                const double* __restrict__ val, int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    base[dst[e]] = val[src[e]];
}

void launch_assemble(double* base, const int64_t* dst, const int64_t* src, const double* val, int64_t count,
                     hipStream_t s) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)blocks), dim3(256), 0, s, base, dst, src, val, count);
  HIP_CHECK(hipGetLastError());
}

// extend-add (Eq. extend-add) as an owner-computes update: one launch per
// child slot, so two children of a parent never race and the summation
// order is fixed (no floating-point atomics)
__global__ void extend_add_kernel(const EADesc* __restrict__ descs) {
  const EADesc d = descs[blockIdx.y];
  const int64_t uu = (int64_t)d.u * d.u;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < uu; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e % d.u), j = (int)(e / d.u);
    d.F[d.map[i] + (int64_t)d.map[j] * d.ldf] += d.U[i + (int64_t)j * d.ldu];
  }
}

void launch_extend_add(const EADesc* d, int nd, int max_u, hipStream_t s) {
  if (nd <= 0 || max_u <= 0) return;
  int64_t blocks = ((int64_t)max_u * max_u + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(extend_add_kernel, dim3((unsigned)blocks, nd), dim3(256), 0, s, d);
  HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------- blocked LU ---
// Panel: columns [jb, jb+w) over rows [jb, n) of each front; pivot search
// over rows [col, s) only (partial pivoting inside F11, Sec. 3.2).  Rows
// below s are eliminated with the same multipliers, which yields
// L21 = F21 U11^{-1}.
// Panel of a front whose F11 rows do not fit in LDS, worked on in place in
// global memory by one workgroup of NT threads per front: for each column,
// the pivot search (largest |value| over the remaining F11 rows, ties to
// the lowest row), the interchange inside the panel, and the scaling and
// rank-1 update of every row below.  A thread's loads are issued together
// (indices clamped into the front, values past the edge unused); the row
// update loads a row's panel entries before storing any, and it also takes
// each thread's running maximum for the next column's pivot search from
// the values it has just computed, so a column costs two dependent rounds
// of memory traffic (the interchange, the update) instead of four.
template <int NT>
__global__ __launch_bounds__(NT) void lu_panel_kernel(const LUFront* __restrict__ fr, int jb, int nb, int* info) {
  constexpr int NW = NT / 64;
  const LUFront f = fr[blockIdx.x];
  if (jb >= f.s) return;
  const int w = min(nb, f.s - jb);   // <= 32
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double wv[NW];
  __shared__ int wi[NW];
  __shared__ double prow[32];
  const auto F = (gptr<double>)f.F;
  const int64_t ld = f.ld;
  // this thread's candidate for the first column's pivot
  double best = -1.0;
  int bi = jb;
  for (int i0 = jb + tid; i0 < f.s; i0 += 4 * NT) {
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = fabs(F[min(i0 + NT * u, f.s - 1) + jb * ld]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + NT * u < f.s && a[u] > best) { best = a[u]; bi = i0 + NT * u; }
  }
  for (int c = 0; c < w; ++c) {
    const int col = jb + c;
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (o > best || (o == best && oi < bi)) { best = o; bi = oi; }
    }
    if (lane == 0) { wv[wave] = best; wi[wave] = bi; }
    __syncthreads();
    best = wv[0];
    bi = wi[0];
#pragma unroll
    for (int k = 1; k < NW; ++k)
      if (wv[k] > best || (wv[k] == best && wi[k] < bi)) { best = wv[k]; bi = wi[k]; }
    const int p = bi;
    if (tid == 0) {
      f.ipiv[col] = p;
      if (best == 0.0) atomicCAS(info, 0, f.id + 1);
    }
    // the interchange inside the panel; the pivot row goes to LDS directly
    if (tid < w) {
      const double a = F[col + (int64_t)(jb + tid) * ld];
      const double b = F[p + (int64_t)(jb + tid) * ld];
      if (p != col) {
        F[col + (int64_t)(jb + tid) * ld] = b;
        F[p + (int64_t)(jb + tid) * ld] = a;
      }
      prow[tid] = (p != col) ? b : a;
    }
    __syncthreads();
    const double piv = prow[c];
    const double rp = (piv != 0.0) ? 1.0 / piv : 0.0;
    best = -1.0;
    bi = col + 1;
    for (int i = col + 1 + tid; i < f.n; i += NT) {
      const double lraw = F[i + col * ld];
      double v[32];
#pragma unroll
      for (int cc = 0; cc < 32; ++cc) v[cc] = F[i + (int64_t)(jb + min(cc, w - 1)) * ld];
      const double l = lraw * rp;
      F[i + col * ld] = l;
      double nxt = 0.0;
#pragma unroll
      for (int cc = 0; cc < 32; ++cc)
        if (cc > c && cc < w) {
          const double y = v[cc] - l * prow[cc];
          F[i + (int64_t)(jb + cc) * ld] = y;
          if (cc == c + 1) nxt = y;
        }
      if (c + 1 < w && i < f.s && fabs(nxt) > best) { best = fabs(nxt); bi = i; }
    }
    __syncthreads();
  }
}

// a double moved between lanes of a 16-lane row by a data-parallel
// primitive (CTRL: quad permutation, half-row mirror or row rotation)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, false);
}

// (v, i) <- the larger of (v, i) and (o, oi), ties to the lower index
__device__ __forceinline__ void amax_pair(double& v, int& i, double o, int oi) {
  const bool tk = (o > v) | ((o == v) & (oi < i));
  v = tk ? o : v;
  i = tk ? oi : i;
}

// (value, index) maximum over the wavefront, larger value first, ties to the
// lower index, the same in every lane: inside each 16-lane row by quad
// permutations, half-row mirror and rotation by 8, then over the four rows'
// results read as scalars.  The maximum with that tie rule does not depend
// on the order it is taken in.
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  amax_pair(v, i, dpp_d<0xB1>(v), dpp_i<0xB1>(i));     // quad_perm [1,0,3,2]
  amax_pair(v, i, dpp_d<0x4E>(v), dpp_i<0x4E>(i));     // quad_perm [2,3,0,1]
  amax_pair(v, i, dpp_d<0x141>(v), dpp_i<0x141>(i));   // row_half_mirror
  amax_pair(v, i, dpp_d<0x128>(v), dpp_i<0x128>(i));   // row_ror:8
  double rv = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(__double_as_longlong(v) >> 32), 0) << 32) |
                                   (unsigned)__builtin_amdgcn_readlane((int)(__double_as_longlong(v) & 0xffffffffll), 0));
  int ri = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const long long u = __double_as_longlong(v);
    const double o = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(u >> 32), 16 * r) << 32) |
                                          (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffll), 16 * r));
    amax_pair(rv, ri, o, __builtin_amdgcn_readlane(i, 16 * r));
  }
  v = rv;
  i = ri;
}

// Panel of the F11 rows only, resident in LDS: rows [jb, s) x columns
// [jb, jb+w) of each front (m1 = s - jb rows, column major with ld m1).
// Same pivot rule and the same operations per element as lu_panel_kernel;
// the F21 rows of the panel are done afterwards by lu_panel21_kernel.  Two
// workgroup barriers per column: the next column's pivot candidates are
// found while the rows are updated, and every thread combines the
// wavefronts' records itself.
__global__ __launch_bounds__(256) void lu_panel11_kernel(const LUFront* __restrict__ fr, int jb, int nb, int* info) {
  extern __shared__ double P[];
  __shared__ double wv[4];
  __shared__ int wi[4];
  __shared__ double prow[32];
  const LUFront f = fr[blockIdx.x];
  if (jb >= f.s) return;
  const int w = min(nb, f.s - jb), m1 = f.s - jb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* F = f.F;
  const int64_t ld = f.ld;
  {
    // stage the panel: a thread takes one row per 256-row chunk and loads
    // its 32 panel entries at once (column indices clamped to the panel),
    // so the loads are in flight together rather than one per round trip
    const auto G = (gptr<const double>)F;
    for (int r = tid; r < m1; r += 256) {
      double v[32];
#pragma unroll
      for (int c = 0; c < 32; ++c) v[c] = G[(jb + r) + (int64_t)(jb + min(c, w - 1)) * ld];
#pragma unroll
      for (int c = 0; c < 32; ++c)
        if (c < w) P[r + c * m1] = v[c];
    }
  }
  __syncthreads();
  // this thread's candidate for the first column's pivot: largest |value|
  // in column 0 over its rows, ties to the lowest row
  double best = -1.0;
  int bi = 0;
  for (int r = tid; r < m1; r += 256) {
    const double a = fabs(P[r]);
    if (a > best) { best = a; bi = r; }
  }
  for (int c = 0; c < w; ++c) {
    wave_argmax(best, bi);
    if (lane == 0) { wv[wave] = best; wi[wave] = bi; }
    __syncthreads();
    best = wv[0];
    bi = wi[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) amax_pair(best, bi, wv[q], wi[q]);
    const int p = bi;
    if (tid == 0) {
      f.ipiv[jb + c] = jb + p;
      if (best == 0.0) atomicCAS(info, 0, f.id + 1);
    }
    // the interchange inside the panel; the pivot row also goes to prow
    if (tid < w) {
      const double a = P[c + tid * m1];
      const double b = P[p + tid * m1];
      if (p != c) {
        P[c + tid * m1] = b;
        P[p + tid * m1] = a;
      }
      prow[tid] = (p != c) ? b : a;
    }
    __syncthreads();
    const double piv = prow[c];
    const double rp = (piv != 0.0) ? 1.0 / piv : 0.0;
    best = -1.0;
    bi = c + 1;
    for (int r = c + 1 + tid; r < m1; r += 256) {
      const double l = P[r + c * m1] * rp;
      P[r + c * m1] = l;
      for (int cc = c + 1; cc < w; ++cc) {
        const double y = P[r + cc * m1] - l * prow[cc];
        P[r + cc * m1] = y;
        if (cc == c + 1 && fabs(y) > best) { best = fabs(y); bi = r; }
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < m1 * w; e += 256) {
    const int r = e % m1, c = e / m1;
    F[(jb + r) + (int64_t)(jb + c) * ld] = P[e];
  }
}

// F21 rows of the panel: every row x of F[s:n, jb:jb+w) becomes x U^{-1}
// with the panel's w x w upper block, which is what the column-by-column
// elimination does to those rows (same operations, same order).  One thread
// per row, the row in registers.
template <int NB>
__global__ __launch_bounds__(256) void lu_panel21_kernel(const LUFront* __restrict__ fr, int jb) {
  __shared__ double U[NB][NB + 1];
  const LUFront f = fr[blockIdx.y];
  if (jb >= f.s) return;
  const int w = min(NB, f.s - jb);
  const int tid = threadIdx.x;
  double* F = f.F;
  const int64_t ld = f.ld;
  if ((int64_t)blockIdx.x * 256 >= f.n - f.s) return;
  // loads with indices clamped into the panel are unconditional, so all of
  // a thread's loads are in flight together; entries past w are zeroed in
  // U and never used in x
  const auto G = (gptr<const double>)F;
  {
    constexpr int Q = NB * NB / 256;
    double uv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q, r = e % NB, c = e / NB;
      uv[q] = G[(jb + min(r, w - 1)) + (int64_t)(jb + min(c, w - 1)) * ld];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q, r = e % NB, c = e / NB;
      U[r][c] = (r < w && c < w) ? uv[q] : 0.0;
    }
  }
  __syncthreads();
  const int i = f.s + blockIdx.x * 256 + tid;
  if (i >= f.n) return;
  double x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = G[i + (int64_t)(jb + min(c, w - 1)) * ld];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < w) {
      const double piv = U[c][c];
      const double rp = (piv != 0.0) ? 1.0 / piv : 0.0;
      const double l = x[c] * rp;
      x[c] = l;
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc)
        if (cc < w) x[cc] -= l * U[c][cc];
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < w) F[i + (int64_t)(jb + c) * ld] = x[c];
}

// dynamic LDS a workgroup may take on this device, less what the kernels
// hold statically
size_t lds_budget(size_t static_bytes) {
  static size_t limit = 0;
  if (!limit) {
    int dev = 0, v = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    limit = (size_t)v;
  }
  return limit > static_bytes ? limit - static_bytes : 0;
}

bool lu_panel_split_fits(int max_m1, int nb) {
  return (size_t)max_m1 * nb * sizeof(double) <= std::min<size_t>(144 * 1024, lds_budget(1024));
}

void launch_lu_panel_split(const LUFront* fr, int nf, int jb, int nb, int max_m1, int max_u, int* info, hipStream_t s,
                           double flops) {
  if (nf <= 0) return;
  REQUIRE(nb == 32, HSSMF_EINVAL, "panel width");
  REQUIRE(lu_panel_split_fits(max_m1, nb), HSSMF_EINVAL, "panel too tall for LDS");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof::enabled()) prof::ext(3, flops, &e0, &e1);   // timing hook
  const size_t lds = (size_t)std::max(max_m1, 1) * nb * sizeof(double);
  if (e0) hipExtLaunchKernelGGL(lu_panel11_kernel, dim3(nf), dim3(256), lds, s, e0, e1, 0, fr, jb, nb, info);
  else hipLaunchKernelGGL(lu_panel11_kernel, dim3(nf), dim3(256), lds, s, fr, jb, nb, info);
  HIP_CHECK(hipGetLastError());
  if (max_u > 0) {
    hipLaunchKernelGGL(lu_panel21_kernel<32>, dim3((max_u + 255) / 256, nf), dim3(256), 0, s, fr, jb);
    HIP_CHECK(hipGetLastError());
  }
}

void launch_lu_panel(const LUFront* fr, int nf, int jb, int nb, int* info, hipStream_t s, double flops) {
  if (nf <= 0) return;
  REQUIRE(nb <= 32, HSSMF_EINVAL, "panel width");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof::enabled()) prof::ext(3, flops, &e0, &e1);   // timing hook
  // fronts this tall are few: one 512-thread workgroup each
  if (e0) hipExtLaunchKernelGGL(lu_panel_kernel<512>, dim3(nf), dim3(512), 0, s, e0, e1, 0, fr, jb, nb, info);
  else hipLaunchKernelGGL(lu_panel_kernel<512>, dim3(nf), dim3(512), 0, s, fr, jb, nb, info);
  HIP_CHECK(hipGetLastError());
}

// apply the panel's interchanges to the columns outside the panel
// The interchanges (p0 + t, ipiv[p0 + t]), t < w = min(np, s - p0), in order,
// applied to the columns [c0, c1) of each front (c1 < 0: up to n; else
// clamped to s) other than the pivot columns [p0, p0 + w) themselves.
__global__ void laswp_kernel(const LUFront* __restrict__ fr, int p0, int np, int c0, int c1) {
  const LUFront f = fr[blockIdx.y];
  if (p0 >= f.s) return;
  const int w = min(np, f.s - p0);
  const int cend = c1 < 0 ? f.n : min(c1, f.s);
  const int col = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= cend || (col >= p0 && col < p0 + w)) return;
  double* c = f.F + (int64_t)col * f.ld;
  for (int t = 0; t < w; ++t) {
    int r1 = p0 + t, r2 = f.ipiv[r1];
    if (r1 != r2) { double x = c[r1]; c[r1] = c[r2]; c[r2] = x; }
  }
}

void launch_laswp(const LUFront* fr, int nf, int p0, int np, int c0, int c1, int max_n, hipStream_t s) {
  const int span = (c1 < 0 ? max_n : std::min(c1, max_n)) - c0;
  if (nf <= 0 || span <= 0) return;
  hipLaunchKernelGGL(laswp_kernel, dim3((span + 255) / 256, nf), dim3(256), 0, s, fr, p0, np, c0, c1);
  HIP_CHECK(hipGetLastError());
}

// U12 block row: X = L_pp^{-1} X for rows [jb, jb+w), w = min(nb, s - jb)
// <= 64, and the columns [c0, c1) (c0 < 0: from jb + w; c1 < 0: up to n;
// explicit bounds clamped to s)
__global__ __launch_bounds__(256) void trsm_u12_kernel(const LUFront* __restrict__ fr, int jb, int nb, int c0,
                                                       int c1) {
  const LUFront f = fr[blockIdx.y];
  if (jb >= f.s) return;
  const int w = min(nb, f.s - jb);
  const int cbeg = c0 < 0 ? jb + w : min(c0, f.s);
  const int cend = c1 < 0 ? f.n : min(c1, f.s);
  if (cbeg >= cend) return;
  __shared__ double Lp[64][65];
  // the diagonal block: unconditional loads (indices clamped into the
  // block) in flight together, then stored to LDS; a 32 x 32 footprint for
  // panels up to 32 wide, 64 x 64 beyond
  auto stage = [&](auto tw) {
    constexpr int TW = decltype(tw)::value, U = TW * TW / 256;
    const auto F = (gptr<const double>)f.F;
    const int i = threadIdx.x % TW, j0 = threadIdx.x / TW;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = F[(jb + min(i, w - 1)) + (int64_t)(jb + min(j0 + (256 / TW) * u, w - 1)) * f.ld];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i < w && j0 + (256 / TW) * u < w) Lp[i][j0 + (256 / TW) * u] = v[u];
  };
  if (w <= 32) stage(std::integral_constant<int, 32>{});
  else stage(std::integral_constant<int, 64>{});
  __syncthreads();
  // one wavefront per column, lane i holding row jb + i (unit lower solve)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int col = cbeg + blockIdx.x * 4 + wave; col < cend; col += gridDim.x * 4) {
    double* c = f.F + (int64_t)col * f.ld + jb;
    double v = (lane < w) ? c[lane] : 0.0;
    for (int j = 0; j < w; ++j) {
      const double xj = __shfl(v, j);
      if (lane > j && lane < w) v -= Lp[lane][j] * xj;
    }
    if (lane < w) c[lane] = v;
  }
}

void launch_trsm_u12(const LUFront* fr, int nf, int jb, int nb, int c0, int c1, int max_n, hipStream_t s) {
  if (nf <= 0 || max_n <= 0) return;
  REQUIRE(nb <= 64, HSSMF_EINVAL, "U12 solve: more than 64 rows at once");
  int gx = (max_n + 3) / 4;
  if (gx > 256) gx = 256;
  hipLaunchKernelGGL(trsm_u12_kernel, dim3(gx, nf), dim3(256), 0, s, fr, jb, nb, c0, c1);
  HIP_CHECK(hipGetLastError());
}

// -------------------------------------------------------------- solves ---
// batched GEMV: each workgroup owns 16 outputs (non-transposed: 16 column
// phases per row, eight loads in flight per thread, partial sums added in
// phase order) or 4 outputs (transposed: one wavefront per column dot
// product)
__global__ __launch_bounds__(256) void gemv_kernel(const GemvDesc* __restrict__ descs) {
  const GemvDesc d = descs[blockIdx.y];
  const int tid = threadIdx.x;
  if (!d.trans) {
    if (blockIdx.x * 16 >= d.rows) return;
    const int r = blockIdx.x * 16 + (tid & 15);
    const int ph = tid >> 4;
    __shared__ double red[16][17];
    double acc = 0.0;
    if (r < d.rows && d.alpha != 0.0) {
      // indices clamped into the matrix, so every load is unconditional:
      // the map entries of a round go out together, then all matrix and
      // vector entries; only the accumulation is guarded
      const auto M = (gptr<const double>)d.M;
      const auto X = (gptr<const double>)d.x;
      for (int j0 = ph; j0 < d.cols; j0 += 128) {
        int jc[8], xj[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) jc[u] = xj[u] = min(j0 + 16 * u, d.cols - 1);
        if (d.xmap) {
          const auto xmap = (gptr<const int>)d.xmap;
#pragma unroll
          for (int u = 0; u < 8; ++u) xj[u] = xmap[jc[u]];
        }
        double mv[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          mv[u] = M[r + (int64_t)jc[u] * d.ld];
          xv[u] = X[xj[u]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (j0 + 16 * u < d.cols) acc += mv[u] * xv[u];
      }
    }
    red[ph][tid & 15] = acc;
    __syncthreads();
    if (ph == 0 && r < d.rows) {
      double v = 0.0;
      for (int q = 0; q < 16; ++q) v += red[q][tid];
      const int yr = d.ymap ? d.ymap[r] : r;
      d.y[yr] = d.overwrite ? d.alpha * v : d.y[yr] + d.alpha * v;
    }
  } else {
    const int c = blockIdx.x * 4 + (tid >> 6);
    const int lane = tid & 63;
    if (c >= d.cols) return;
    double acc = 0.0;
    const auto col = (gptr<const double>)d.M + (int64_t)c * d.ld;
    const auto X = (gptr<const double>)d.x;
    if (d.alpha != 0.0)
      for (int i0 = lane; i0 < d.rows; i0 += 512) {
        int ic[8], xi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ic[u] = xi[u] = min(i0 + 64 * u, d.rows - 1);
        if (d.xmap) {
          const auto xmap = (gptr<const int>)d.xmap;
#pragma unroll
          for (int u = 0; u < 8; ++u) xi[u] = xmap[ic[u]];
        }
        double mv[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          mv[u] = col[ic[u]];
          xv[u] = X[xi[u]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (i0 + 64 * u < d.rows) acc += mv[u] * xv[u];
      }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) {
      int yc = d.ymap ? d.ymap[c] : c;
      d.y[yc] = d.overwrite ? d.alpha * acc : d.y[yc] + d.alpha * acc;
    }
  }
}

// gx: workgroups along x, the largest of ceil(rows / 16) (non-transposed)
// and ceil(cols / 4) (transposed) over the batch
void launch_gemv(const GemvDesc* d, int nd, int gx, hipStream_t s) {
  if (nd <= 0 || gx <= 0) return;
  hipLaunchKernelGGL(gemv_kernel, dim3(gx, nd), dim3(256), 0, s, d);
  HIP_CHECK(hipGetLastError());
}

// lane j's copy of a double, for every lane (j uniform): two scalar lane
// reads, no trip through LDS
__device__ __forceinline__ double lane_bcast(double v, int j) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), j);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The row interchanges of rows [c0, c1) (their pivot indices staged in
// pv[i - c0]) applied to v in order (FWD) or in reverse order, by wavefront
// 0: each group of 64 indices is read once into registers and taken lane
// by lane as scalars, and lane 0 makes the swaps in sequence.
template <bool FWD>
__device__ __forceinline__ void swap_rows(double* v, const int* pv, int c0, int c1, int lane) {
  for (int g = 0; g < c1 - c0; g += 64) {
    const int i0 = FWD ? c0 + g : max(c0, c1 - g - 64);
    const int n = FWD ? min(64, c1 - i0) : c1 - g - i0;
    const int pl = lane < n ? pv[i0 - c0 + lane] : i0 + lane;
    for (int k = 0; k < n; ++k) {
      const int u = FWD ? k : n - 1 - k;
      const int p = __builtin_amdgcn_readlane(pl, u);
      const int i = i0 + u;
      if (p != i && lane == 0) {
        const double t = v[i];
        v[i] = v[p];
        v[p] = t;
      }
    }
  }
}

// Triangular solves with the F11 factors, one workgroup per front, the
// right-hand side staged in LDS.  Blocks of 64: the diagonal block is staged
// in LDS with coalesced loads, one wavefront solves it (each new entry read
// out of its lane into scalar registers for the others), then all threads
// update the rest of the right-hand side.  Row interchanges are applied in
// their sequential order, and only when a chunk of 256 holds any.
template <int KIND, bool STAGE, int NT>
__global__ __launch_bounds__(NT) void trsv_kernel(const TrsvDesc* __restrict__ descs) {
  extern __shared__ double xs[];   // s entries, then (STAGE) the 64 x 65 block
  const TrsvDesc d = descs[blockIdx.x];
  double (*Tb)[65] = reinterpret_cast<double (*)[65]>(xs + ((d.s + 1) & ~1));
  const int s = d.s, tid = threadIdx.x, lane = tid & 63;
  const int64_t ld = d.ld;
  __shared__ int pv[256];   // pivot indices, staged 256 at a time for the sequential swaps
  for (int i = tid; i < s; i += NT) xs[i] = d.x[i];
  __syncthreads();
  if (KIND == 0 && d.ipiv)
    for (int c0 = 0; c0 < s; c0 += 256) {
      bool sw = false;
      if (tid < 256 && c0 + tid < s) {
        const int p = d.ipiv[c0 + tid];
        pv[tid] = p;
        sw = p != c0 + tid;
      }
      if (__syncthreads_or(sw) && tid < 64) swap_rows<true>(xs, pv, c0, min(s, c0 + 256), lane);
      __syncthreads();
    }
  // logical matrix T: KIND 0: L (unit lower), 1: U (upper), 2: U^T (lower),
  // 3: L^T (unit upper), 4: L (non-unit lower), 5: L^T (non-unit upper)
  constexpr bool trans = (KIND == 2 || KIND == 3 || KIND == 5);
  auto T = [&](int i, int j) -> double {
    return trans ? d.F[j + (int64_t)i * ld] : d.F[i + (int64_t)j * ld];
  };
  // Tb[r][c] = T(b0 + r, b0 + c) for r, c < bs, read along the stored columns
  auto stage = [&](int b0, int bs) {
    if (!STAGE) return;
    for (int e = tid; e < 64 * 64; e += NT) {
      const int fast = e & 63, slow = e >> 6;
      const int r = trans ? slow : fast, c = trans ? fast : slow;
      if (r < bs && c < bs) Tb[r][c] = T(b0 + r, b0 + c);
    }
  };
  // sum over the block's columns of T(i, b0 + j) x(b0 + j), in column order,
  // thirty-two loads in flight at a time
  auto row_dot = [&](int i, int b0, int bs) {
    double acc = 0.0;
    for (int j0 = 0; j0 < bs; j0 += 32) {
      double tv[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) tv[u] = (j0 + u < bs) ? T(i, b0 + j0 + u) : 0.0;
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (j0 + u < bs) acc += tv[u] * xs[b0 + j0 + u];
    }
    return acc;
  };
  constexpr bool lower = (KIND == 0 || KIND == 2 || KIND == 4);
  constexpr bool unit = (KIND == 0 || KIND == 3);
  if (lower) {
    for (int b0 = 0; b0 < s; b0 += 64) {
      const int bs = min(64, s - b0);
      stage(b0, bs);
      __syncthreads();
      if (tid < 64) {
        double v = (lane < bs) ? xs[b0 + lane] : 0.0;
        for (int j = 0; j < bs; ++j) {
          const double t = (STAGE ? Tb[lane][j] : T(b0 + lane, b0 + j));
          if (!unit && lane == j) v /= STAGE ? Tb[j][j] : T(b0 + j, b0 + j);
          const double vj = lane_bcast(v, j);
          if (lane > j && lane < bs) v -= t * vj;
        }
        if (lane < bs) xs[b0 + lane] = v;
      }
      __syncthreads();
      for (int i = b0 + bs + tid; i < s; i += NT) xs[i] -= row_dot(i, b0, bs);
      __syncthreads();
    }
  } else {
    for (int b1 = s; b1 > 0; b1 -= 64) {
      const int b0 = max(0, b1 - 64), bs = b1 - b0;
      stage(b0, bs);
      __syncthreads();
      if (tid < 64) {
        double v = (lane < bs) ? xs[b0 + lane] : 0.0;
        for (int j = bs - 1; j >= 0; --j) {
          const double t = (STAGE ? Tb[lane][j] : T(b0 + lane, b0 + j));
          if (!unit && lane == j) v /= STAGE ? Tb[j][j] : T(b0 + j, b0 + j);
          const double vj = lane_bcast(v, j);
          if (lane < j) v -= t * vj;
        }
        if (lane < bs) xs[b0 + lane] = v;
      }
      __syncthreads();
      for (int i = tid; i < b0; i += NT) xs[i] -= row_dot(i, b0, bs);
      __syncthreads();
    }
  }
  if (KIND == 3 && d.ipiv)
    for (int c1 = s; c1 > 0; c1 -= 256) {
      const int c0 = max(0, c1 - 256);
      __syncthreads();
      bool sw = false;
      if (tid < 256 && c0 + tid < c1) {
        const int p = d.ipiv[c0 + tid];
        pv[tid] = p;
        sw = p != c0 + tid;
      }
      if (__syncthreads_or(sw) && tid < 64) swap_rows<false>(xs, pv, c0, c1, lane);
    }
  __syncthreads();
  for (int i = tid; i < s; i += NT) d.x[i] = xs[i];
}

// The same triangular solves with one workgroup per block of 64 entries
// (the blocks the one-workgroup kernel steps through, in the same order).
// The workgroup of block q subtracts every earlier block from its own as
// each is published, in block order, then solves its block and publishes
// its entries in x through agent-coherent stores and then its flag; each
// entry takes exactly the operations of the one-workgroup kernel in the
// same order, so both give identical results.  Workgroups take their
// (system, block) from a ticket drawn when they start, blocks in order
// across the systems, so a workgroup only ever waits for workgroups that
// started before it: no co-residency is needed and an ordinary launch (also
// inside a graph) is safe.  Flags hold the number of the launch that set
// them (ws[0] counts launches; the last workgroup to finish advances it and
// resets the ticket and finish counters), so no reset is needed between
// launches; every wait is bounded and gives up once any workgroup has set
// *err (host-visible memory, polled every 256 spins).
constexpr unsigned kTrsvSpinLimit = 1u << 22;

__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int KIND>
__global__ __launch_bounds__(256) void trsv_multi_kernel(const TrsvDesc* __restrict__ descs, int nd, int maxnb,
                                                         int* __restrict__ ws, int* __restrict__ err) {
  constexpr int NT = 256;
  constexpr bool trans = (KIND == 2 || KIND == 3 || KIND == 5);
  constexpr bool lower = (KIND == 0 || KIND == 2 || KIND == 4);
  constexpr bool unit = (KIND == 0 || KIND == 3);
  extern __shared__ double sm[];
  // LDS: this block's diagonal block and the block being subtracted (each
  // staged ahead of the wait for the block it holds the columns of), the
  // published block being applied, this block's entries, and (pivoted
  // kinds) the whole vector for the sequential interchanges
  double (*Td)[65] = reinterpret_cast<double (*)[65]>(sm);
  double (*To)[65] = reinterpret_cast<double (*)[65]>(sm + 64 * 65);
  double* xq = sm + 2 * 64 * 65;
  double* own = xq + 64;
  double* xall = own + 64;
  __shared__ int pv[256];
  __shared__ int sh_i;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid == 0) sh_i = __hip_atomic_fetch_add(ws + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int ticket = sh_i;
  const int f = ticket % nd, t = ticket / nd;   // system, block
  const TrsvDesc d = descs[f];
  const int s = d.s;
  const int64_t ld = d.ld;
  const int nb = (s + 63) / 64;
  int* flags = ws + 3 + (size_t)f * (maxnb + 1);   // [q]: block q published, [nb]: interchanges applied
  const int target = __hip_atomic_load(ws, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
  auto T = [&](int i, int j) -> double {
    return trans ? d.F[j + (int64_t)i * ld] : d.F[i + (int64_t)j * ld];
  };
  auto blk = [&](int q, int& b0, int& bs) {
    if (lower) {
      b0 = 64 * q;
      bs = min(64, s - b0);
    } else {
      const int b1 = s - 64 * q;
      b0 = max(0, b1 - 64);
      bs = b1 - b0;
    }
  };
  // D[r][c] = T(r0 + r, c0 + c), read along the stored columns
  auto stage = [&](double (*D)[65], int r0, int rs, int c0, int cs) {
    for (int e = tid; e < 64 * 64; e += NT) {
      const int fast = e & 63, slow = e >> 6;
      const int r = trans ? slow : fast, c = trans ? fast : slow;
      if (r < rs && c < cs) D[r][c] = T(r0 + r, c0 + c);
    }
  };
  // bounded wait (thread 0, agent-coherent polls) until *fl holds this
  // launch's number, then one acquire fence
  auto wait_flag = [&](const int* fl) {
    if (tid == 0) {
      unsigned spins = 0;
      int ok = 1;
      while (__hip_atomic_load(const_cast<int*>(fl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
        if (++spins > kTrsvSpinLimit ||
            ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      sh_i = ok;
    }
    __syncthreads();
    return sh_i != 0;
  };
  // every (agent-coherent) store of the workgroup complete, then the flag
  auto publish = [&](int* fl) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(fl, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  bool alive = t < nb;
  int b0 = 0, bs = 0;
  if (alive) blk(t, b0, bs);
  // interchanges before the solve (KIND 0): applied to the whole vector by
  // the workgroup of block 0 (the first of its system), only when there are
  // any
  bool swaps = false;
  if ((KIND == 0 || KIND == 3) && d.ipiv && alive) {
    bool any = false;
    for (int i = tid; i < s; i += NT) any |= d.ipiv[i] != i;
    swaps = __syncthreads_or(any);
  }
  if (KIND == 0 && swaps) {
    if (t == 0) {
      for (int i = tid; i < s; i += NT) xall[i] = d.x[i];
      for (int c0 = 0; c0 < s; c0 += 256) {
        __syncthreads();
        if (tid < 256 && c0 + tid < s) pv[tid] = d.ipiv[c0 + tid];
        __syncthreads();
        if (tid < 64) swap_rows<true>(xall, pv, c0, min(s, c0 + 256), lane);
      }
      __syncthreads();
      for (int i = tid; i < s; i += NT) st_agent(d.x + i, xall[i]);
      publish(flags + nb);
    } else {
      alive = wait_flag(flags + nb);
    }
  }
  if (alive) {
    // this block's right-hand side and diagonal block
    if (tid < bs) own[tid] = (KIND == 0 && swaps) ? ld_agent(d.x + b0 + tid) : d.x[b0 + tid];
    stage(Td, b0, bs, b0, bs);
    // every earlier block, in order: its block in this block's rows is read
    // before the wait for it
    for (int q = 0; q < t; ++q) {
      int c0, cs;
      blk(q, c0, cs);
      __syncthreads();   // To and xq may still be read by the previous step
      stage(To, b0, bs, c0, cs);
      if (!wait_flag(flags + q)) { alive = false; break; }
      if (tid < cs) xq[tid] = ld_agent(d.x + c0 + tid);
      __syncthreads();
      if (tid < bs) {
        double acc = 0.0;
        if (cs == 64) {
          double tv[64];
#pragma unroll
          for (int c = 0; c < 64; ++c) tv[c] = To[tid][c];
#pragma unroll
          for (int c = 0; c < 64; ++c) acc += tv[c] * xq[c];
        } else {
          for (int c = 0; c < cs; ++c) acc += To[tid][c] * xq[c];
        }
        own[tid] -= acc;
      }
    }
  }
  if (alive) {
    // solve the block, publish it
    __syncthreads();
    if (tid < 64) {
      double v = (lane < bs) ? own[lane] : 0.0;
      if (bs == 64) {
        // a whole block: the lane's row in registers, every step unrolled
        double tr[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) tr[j] = Td[lane][j];
        const double dl = Td[lane][lane];
        if (lower) {
#pragma unroll
          for (int j = 0; j < 64; ++j) {
            if (!unit && lane == j) v /= dl;
            const double vj = lane_bcast(v, j);
            if (lane > j) v -= tr[j] * vj;
          }
        } else {
#pragma unroll
          for (int j = 63; j >= 0; --j) {
            if (!unit && lane == j) v /= dl;
            const double vj = lane_bcast(v, j);
            if (lane < j) v -= tr[j] * vj;
          }
        }
      } else if (lower) {
        for (int j = 0; j < bs; ++j) {
          const double tj = Td[lane][j];
          if (!unit && lane == j) v /= Td[j][j];
          const double vj = lane_bcast(v, j);
          if (lane > j && lane < bs) v -= tj * vj;
        }
      } else {
        for (int j = bs - 1; j >= 0; --j) {
          const double tj = Td[lane][j];
          if (!unit && lane == j) v /= Td[j][j];
          const double vj = lane_bcast(v, j);
          if (lane < j) v -= tj * vj;
        }
      }
      if (lane < bs) st_agent(d.x + b0 + lane, v);
    }
    publish(flags + t);
  }
  // interchanges after the solve (KIND 3): by the workgroup of the last
  // block, the last of its system, once every block is published
  if (KIND == 3 && swaps && alive && t == nb - 1) {
    for (int q = 0; q < nb - 1 && alive; ++q) alive = wait_flag(flags + q);
    if (alive) {
      for (int i = tid; i < s; i += NT) xall[i] = ld_agent(d.x + i);
      for (int c1 = s; c1 > 0; c1 -= 256) {
        const int c0 = max(0, c1 - 256);
        __syncthreads();
        if (tid < 256 && c0 + tid < c1) pv[tid] = d.ipiv[c0 + tid];
        __syncthreads();
        if (tid < 64) swap_rows<false>(xall, pv, c0, c1, lane);
      }
      __syncthreads();
      for (int i = tid; i < s; i += NT) d.x[i] = xall[i];
    }
  }
  // the last workgroup of the launch advances the launch count and resets
  // the ticket and finish counters
  __syncthreads();
  if (tid == 0) {
    const int done = __hip_atomic_fetch_add(ws + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done == (int)gridDim.x - 1) {
      __hip_atomic_store(ws + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ws + 2, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ws, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

void launch_trsv(const TrsvDesc* d, int nd, int kind, int max_s, hipStream_t s) {
  if (nd <= 0) return;
  // LDS holds the whole right-hand side and, when it fits, the 64 x 64
  // diagonal block being solved.  A batch of few fronts (each on its own
  // CU) takes 1024 threads per front, so the row updates keep four times as
  // many loads in flight.
  const size_t xs = (size_t)(std::max(max_s, 1) + 1) / 2 * 2 * sizeof(double);
  const size_t blk = 64 * 65 * sizeof(double);
  const size_t budget = lds_budget(256 * sizeof(int));
  REQUIRE(xs <= budget, HSSMF_EINVAL, "triangular solve: right-hand side too long for LDS");
  const bool stage = xs + blk <= budget;
  const size_t lds = stage ? xs + blk : xs;
  const bool wide = nd <= 128 && max_s >= 256;
#define HSSMF_TRSV(K)                                                                                     \
  if (wide) {                                                                                             \
    if (stage) hipLaunchKernelGGL((trsv_kernel<K, true, 1024>), dim3(nd), dim3(1024), lds, s, d);         \
    else hipLaunchKernelGGL((trsv_kernel<K, false, 1024>), dim3(nd), dim3(1024), lds, s, d);              \
  } else {                                                                                                \
    if (stage) hipLaunchKernelGGL((trsv_kernel<K, true, 256>), dim3(nd), dim3(256), lds, s, d);           \
    else hipLaunchKernelGGL((trsv_kernel<K, false, 256>), dim3(nd), dim3(256), lds, s, d);                \
  }
  switch (kind) {
    case 0: HSSMF_TRSV(0) break;
    case 1: HSSMF_TRSV(1) break;
    case 2: HSSMF_TRSV(2) break;
    case 3: HSSMF_TRSV(3) break;
    case 4: HSSMF_TRSV(4) break;
    default: HSSMF_TRSV(5) break;
  }
#undef HSSMF_TRSV
  HIP_CHECK(hipGetLastError());
}

size_t trsv_multi_lds(int kind, int max_s) {
  size_t b = (size_t)(2 * 64 * 65 + 128) * sizeof(double);
  if (kind == 0 || kind == 3) b += (size_t)max_s * sizeof(double);
  return b;
}

// Systems of at least 256 entries.  Along the stored columns (L, U) the
// one-workgroup kernel reads coalesced and many systems keep the chip busy
// by themselves, so beyond 32 systems it stays; the transposed kinds read
// across the stored columns there and always take the per-block kernel.
bool trsv_multi_use(int nd, int kind, int max_s) {
  // diagnostics: HSSMF_TRSV_ONE_WG=1 keeps every solve on one workgroup
  static const bool one_wg = std::getenv("HSSMF_TRSV_ONE_WG") != nullptr;
  const bool trans = kind == 2 || kind == 3 || kind == 5;
  return !one_wg && nd > 0 && max_s >= 256 && (trans || nd <= 32) &&
         trsv_multi_lds(kind, max_s) <= lds_budget(256 * sizeof(int) + 64);
}

void launch_trsv_multi(const TrsvDesc* d, int nd, int kind, int max_s, int* ws, int* err, hipStream_t s) {
  if (nd <= 0) return;
  const int maxnb = (max_s + 63) / 64;
  const size_t lds = trsv_multi_lds(kind, max_s);
  const dim3 grid((unsigned)(nd * maxnb)), blk(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(trsv_multi_kernel<0>, grid, blk, lds, s, d, nd, maxnb, ws, err); break;
    case 1: hipLaunchKernelGGL(trsv_multi_kernel<1>, grid, blk, lds, s, d, nd, maxnb, ws, err); break;
    case 2: hipLaunchKernelGGL(trsv_multi_kernel<2>, grid, blk, lds, s, d, nd, maxnb, ws, err); break;
    case 3: hipLaunchKernelGGL(trsv_multi_kernel<3>, grid, blk, lds, s, d, nd, maxnb, ws, err); break;
    case 4: hipLaunchKernelGGL(trsv_multi_kernel<4>, grid, blk, lds, s, d, nd, maxnb, ws, err); break;
    default: hipLaunchKernelGGL(trsv_multi_kernel<5>, grid, blk, lds, s, d, nd, maxnb, ws, err); break;
  }
  HIP_CHECK(hipGetLastError());
}

// forward-sweep right-hand side of a front: own separator entries plus the
// children's update vectors, gathered through parent-to-child index maps
__global__ void rhs_gather_kernel(const RhsDesc* __restrict__ descs) {
  const RhsDesc d = descs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  double v = (i < d.s) ? d.y[d.sep_lo + i] : 0.0;
  for (int c = 0; c < d.nkids; ++c) {
    int k = d.inv[c][i];
    if (k >= 0) v += d.wc[c][k];
  }
  if (i < d.s) d.y[d.sep_lo + i] = v; else d.w[i - d.s] = v;
}

void launch_rhs_gather(const RhsDesc* d, int nd, int max_n, hipStream_t s) {
  if (nd <= 0 || max_n <= 0) return;
  hipLaunchKernelGGL(rhs_gather_kernel, dim3((max_n + 255) / 256, nd), dim3(256), 0, s, d);
  HIP_CHECK(hipGetLastError());
}

}  // namespace hssmf

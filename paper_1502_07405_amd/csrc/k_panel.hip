// Panel factorization of the blocked Householder QR used by the ULV step
// (the LQ of Sec. 2.3 computed as a QR of the transposed block): one
// workgroup per panel of at most 32 columns, then the compact WY factor T.
#include "kernels.hpp"

namespace hssmf {

namespace {
__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
}  // namespace

// LDS = true: the panel (rows j0..m-1 of its nb columns) is staged in LDS
// for the column loop and written back; false: the loop works on global
// memory (panels too tall for LDS).  The Gram matrix Y^T Y is accumulated
// from 64-row chunks by all threads, and T column by column in parallel.
// NT threads: each trailing column of a step is one wavefront's work, so
// wider workgroups (for batches of few panels, one per CU) take more
// columns at once; every sum keeps its order whatever NT is.
template <bool LDS, int NT>
__global__ __launch_bounds__(NT) void qr_panel_kernel(const PanelDesc* __restrict__ descs) {
  constexpr int NW = NT / 64;
  extern __shared__ double Pl[];
  __shared__ double tau[kPanel], v0s[kPanel], G[kPanel][kPanel + 1], Ts[kPanel][kPanel + 1];
  __shared__ double Yc[64][kPanel + 1];
  __shared__ double bc[3];
  const PanelDesc pd = descs[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = pd.m, j0 = pd.j0, nb = pd.nb, mp = m - j0;
  double* C = pd.C;
  // element (absolute row i >= j0, panel column l)
  auto el = [&](int l, int i) -> double& {
    if (LDS) return Pl[(i - j0) + (int64_t)l * mp];
    return C[i + (int64_t)(j0 + l) * m];
  };
  if (LDS) {
    // stage the panel: a thread takes one row per NT-row chunk and loads its
    // kPanel entries at once (column indices clamped to the panel), so the
    // loads are in flight together rather than one per round trip
    const auto G = (gptr<const double>)C;
    for (int r = tid; r < mp; r += NT) {
      double v[kPanel];
#pragma unroll
      for (int l = 0; l < kPanel; ++l) v[l] = G[(j0 + r) + (int64_t)(j0 + min(l, nb - 1)) * m];
#pragma unroll
      for (int l = 0; l < kPanel; ++l)
        if (l < nb) Pl[r + (int64_t)l * mp] = v[l];
    }
    __syncthreads();
  }
  for (int l = 0; l < nb; ++l) {
    const int t = j0 + l;
    // norm of column l, rows t..m-1
    if (wave == 0) {
      double ss = 0.0;
      for (int i = t + lane; i < m; i += 64) {
        const double v = el(l, i);
        ss += v * v;
      }
      ss = wsum(ss);
      if (lane == 0) {
        const double nrm = sqrt(ss);
        const double x0 = el(l, t);
        const double alpha = (x0 >= 0.0) ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double vtv = v0 * v0 + (ss - x0 * x0);
        bc[0] = (vtv > 0.0 && nrm > 0.0) ? 2.0 / vtv : 0.0;
        bc[1] = v0;
        bc[2] = alpha;
      }
    }
    __syncthreads();
    const double tv = bc[0], v0 = bc[1];
    // apply H_t to the remaining panel columns
    for (int c = l + 1 + wave; c < nb; c += NW) {
      double dot = 0.0;
      for (int i = t + lane; i < m; i += 64) dot += ((i == t) ? v0 : el(l, i)) * el(c, i);
      dot = wsum(dot) * tv;
      for (int i = t + lane; i < m; i += 64) el(c, i) -= dot * ((i == t) ? v0 : el(l, i));
    }
    __syncthreads();
    if (tid == 0) {
      tau[l] = tv;
      v0s[l] = v0;
      el(l, t) = bc[2];  // R_tt
    }
    __syncthreads();
  }
  // Y (m x nb): column l = [0 ... 0, v0, rows t+1.. of panel column l]
  auto yv = [&](int i, int l) -> double {
    const int t = j0 + l;
    if (i < t) return 0.0;
    if (i == t) return v0s[l];
    return el(l, i);
  };
  for (int64_t e = tid; e < (int64_t)m * nb; e += NT) {
    const int i = (int)(e % m), l = (int)(e / m);
    pd.Y[i + (int64_t)l * m] = (i < j0) ? 0.0 : yv(i, l);
  }
  if (LDS) {
    for (int64_t e = tid; e < (int64_t)mp * nb; e += NT) {
      const int r = (int)(e % mp), l = (int)(e / mp);
      C[(j0 + r) + (int64_t)(j0 + l) * m] = Pl[e];
    }
  }
  // Gram matrix G = Y^T Y over rows j0..m-1 (pairs a <= b, Q per thread)
  constexpr int Q = (kPanel * (kPanel + 1) / 2 + NT - 1) / NT;
  double g[Q];
  int pa[Q], pb[Q];
  for (int q = 0; q < Q; ++q) {
    g[q] = 0.0;
    int p = tid + NT * q, a = 0;
    if (p >= kPanel * (kPanel + 1) / 2) {   // no pair for this slot
      pa[q] = pb[q] = kPanel;
      continue;
    }
    while (p >= kPanel - a) { p -= kPanel - a; ++a; }   // row a of the upper triangle
    pa[q] = a;
    pb[q] = a + p;
  }
  for (int r0 = j0; r0 < m; r0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * kPanel; e += NT) {
      const int r = e % 64, l = e / 64;
      Yc[r][l] = (r0 + r < m && l < nb) ? yv(r0 + r, l) : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < Q; ++q) {
      if (pa[q] >= nb || pb[q] >= nb) continue;
      double acc = 0.0;
      for (int r = 0; r < 64; ++r) acc += Yc[r][pa[q]] * Yc[r][pb[q]];
      g[q] += acc;
    }
  }
  for (int q = 0; q < Q; ++q)
    if (pa[q] < nb && pb[q] < nb) G[pa[q]][pb[q]] = g[q];
  __syncthreads();
  // T: T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) G(0:i, i)
  for (int i = 0; i < nb; ++i) {
    if (tid < i) {
      double sacc = 0.0;
      for (int c = tid; c < i; ++c) sacc += Ts[tid][c] * G[c][i];
      Ts[tid][i] = -tau[i] * sacc;
    } else if (tid == i) {
      Ts[i][i] = tau[i];
    }
    __syncthreads();
  }
  for (int e = tid; e < kPanel * kPanel; e += NT) {
    const int r = e % kPanel, i = e / kPanel;
    pd.T[r + i * kPanel] = (r <= i && i < nb) ? Ts[r][i] : 0.0;
  }
}

size_t qr_panel_lds_budget() {
  static size_t b = 0;
  if (!b) {
    int dev = 0, v = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t fixed = sizeof(double) * (2 * kPanel + 2 * kPanel * (kPanel + 1) + 64 * (kPanel + 1) + 3) + 512;
    b = (size_t)v > fixed ? (size_t)v - fixed : 0;
  }
  return b;
}

void launch_qr_panel(const PanelDesc* d, int nd, int max_mp, hipStream_t s) {
  if (nd <= 0) return;
  const size_t lds = (size_t)std::max(max_mp, 1) * kPanel * sizeof(double);
  // a batch of few panels has a CU per panel: 1024 threads each
  const bool wide = nd <= 128;
  if (lds <= qr_panel_lds_budget()) {
    if (wide) hipLaunchKernelGGL((qr_panel_kernel<true, 1024>), dim3(nd), dim3(1024), lds, s, d);
    else hipLaunchKernelGGL((qr_panel_kernel<true, 256>), dim3(nd), dim3(256), lds, s, d);
  } else {
    if (wide) hipLaunchKernelGGL((qr_panel_kernel<false, 1024>), dim3(nd), dim3(1024), 0, s, d);
    else hipLaunchKernelGGL((qr_panel_kernel<false, 256>), dim3(nd), dim3(256), 0, s, d);
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace hssmf

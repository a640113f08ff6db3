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

__global__ __launch_bounds__(256) void qr_panel_kernel(const PanelDesc* __restrict__ descs) {
  const PanelDesc pd = descs[blockIdx.x];
  __shared__ double tau[kPanel], v0s[kPanel], G[kPanel][kPanel + 1];
  __shared__ double bc[3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = pd.m, j0 = pd.j0, nb = pd.nb;
  double* C = pd.C;
  for (int l = 0; l < nb; ++l) {
    const int t = j0 + l;
    double* col = C + (int64_t)t * m;
    // norm of col[t:m]
    if (wave == 0) {
      double ss = 0.0;
      for (int i = t + lane; i < m; i += 64) ss += col[i] * col[i];
      ss = wsum(ss);
      if (lane == 0) {
        const double nrm = sqrt(ss);
        const double x0 = col[t];
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
    for (int c = l + 1 + wave; c < nb; c += 4) {
      double* cc = C + (int64_t)(j0 + c) * m;
      double dot = 0.0;
      for (int i = t + lane; i < m; i += 64) dot += ((i == t) ? v0 : col[i]) * cc[i];
      dot = wsum(dot) * tv;
      for (int i = t + lane; i < m; i += 64) cc[i] -= dot * ((i == t) ? v0 : col[i]);
    }
    __syncthreads();
    if (tid == 0) {
      tau[l] = tv;
      v0s[l] = v0;
      col[t] = bc[2];  // R_tt
    }
    __syncthreads();
  }
  // Y (m x nb): column l = [0 ... 0, v0, C[t+1:m, t]]
  for (int64_t e = tid; e < (int64_t)m * nb; e += 256) {
    const int i = (int)(e % m), l = (int)(e / m);
    const int t = j0 + l;
    double v = 0.0;
    if (i == t) v = v0s[l];
    else if (i > t) v = C[i + (int64_t)t * m];
    pd.Y[i + (int64_t)l * m] = v;
  }
  __syncthreads();
  // Gram matrix G = Y^T Y over rows j0..m-1
  for (int pidx = wave; pidx < nb * nb; pidx += 4) {
    const int a = pidx % nb, b = pidx / nb;
    if (a > b) continue;
    const double* ya = pd.Y + (int64_t)a * m;
    const double* yb = pd.Y + (int64_t)b * m;
    double s = 0.0;
    for (int i = j0 + lane; i < m; i += 64) s += ya[i] * yb[i];
    s = wsum(s);
    if (lane == 0) G[a][b] = s;
  }
  __syncthreads();
  // T: T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) G(0:i, i)
  if (tid == 0) {
    double* T = pd.T;
    for (int i = 0; i < nb; ++i) {
      for (int r = 0; r < nb; ++r) T[r + i * kPanel] = 0.0;
      T[i + i * kPanel] = tau[i];
      for (int r = 0; r < i; ++r) {
        double s = 0.0;
        for (int c = r; c < i; ++c) s += T[r + c * kPanel] * G[c][i];
        T[r + i * kPanel] = -tau[i] * s;
      }
    }
  }
}

void launch_qr_panel(const PanelDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(qr_panel_kernel, dim3(nd), dim3(256), 0, s, d);
  HIP_CHECK(hipGetLastError());
}

}  // namespace hssmf

// Launchers of the vector kernels used by the outer solvers.
#pragma once
#include "common.hpp"

namespace hssmf {

constexpr int kDotParts = 512;

// Device state of GMRES(m) (Sec. 4.6): the Hessenberg matrix after the
// Givens rotations (upper triangular, (kGmMaxRestart + 1) x kGmMaxRestart,
// column-major), the rotations, the rotated right-hand side g and the
// least-squares solution y.  One per handle.
constexpr int kGmMaxRestart = 200;
struct GmDev {
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* y;
  double* hcol;   // the current Hessenberg column before rotation (j + 2 entries)
};
constexpr int64_t kGmDevDoubles = (int64_t)(kGmMaxRestart + 1) * kGmMaxRestart + 6 * (kGmMaxRestart + 2);
GmDev gm_dev(double* base);   // carve a GmDev out of kGmDevDoubles doubles
// what an Arnoldi step reports to the host through mapped memory: the
// estimated residual |g[j+1]| and the step's tag, stored last
struct GmStatus {
  double est;
  int tag;
  int pad;
};

// g = (beta, 0, ..., 0) of length m + 1, v0 = w / beta
void launch_gm_start(double* v0, const double* w, int n, double beta, GmDev d, int m, hipStream_t s);
// One Arnoldi step j of GMRES on the device: modified Gram-Schmidt of w
// against V[:, 0..j] (ld n), the new basis vector V[:, j+1] = w / ||w||, the
// previous Givens rotations applied to the new Hessenberg column, the new
// rotation, the updated g, and the estimate |g[j+1]| with `tag` stored to
// *status.  n at most kArnoldiMaxN: one workgroup, w in registers.
constexpr int kArnoldiMaxN = 16384;
void launch_arnoldi(const double* w, double* V, int n, int j, GmDev d, GmStatus* status, int tag, hipStream_t s);
// the rotation part alone, for a Hessenberg column already in d.hcol
void launch_givens(int j, GmDev d, GmStatus* status, int tag, hipStream_t s);
// y = H(0:k, 0:k)^{-1} g(0:k), then out = x + V(:, 0:k) y
void launch_gm_update(double* out, const double* x, const double* V, int n, int k, GmDev d, hipStream_t s);

void launch_spmv(const int64_t* rp, const int* ci, const double* v, const int64_t* vidx, const double* x, double* y,
                 int n, double alpha, double beta, hipStream_t s);
void launch_dot(const double* a, const double* b, int n, double* part, double* out, int sqrt_out, hipStream_t s);
void launch_axpy(double* y, const double* x, int n, const double* alpha, double sgn, int inv, hipStream_t s);
void launch_gather(double* y, const double* x, const int* map, int n, hipStream_t s);
// the real-equivalent matrix's values (out, 4 zrow[n] doubles) from complex
// values z ((re, im) pairs in complex CSR order), zrow the complex row
// pointers (base 0, n + 1 entries)
void launch_zexpand(double* out, const double* z, const int64_t* zrow, int n, hipStream_t s);
// out[s] = sum of x[i]^2 over [off[s], off[s+1]), s < nseg (off on the device)
void launch_seg_sumsq(const double* x, const int64_t* off, int nseg, double* out, hipStream_t s);
void launch_adjoint_grad(const int* row, const int* col, const double* lam, const double* x, double* g, int64_t nnz,
                         hipStream_t s);

}  // namespace hssmf

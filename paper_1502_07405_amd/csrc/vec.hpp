// Launchers of the vector kernels used by the outer solvers.
#pragma once
#include "common.hpp"

namespace hssmf {

constexpr int kDotParts = 512;

void launch_spmv(const int64_t* rp, const int* ci, const double* v, const int64_t* vidx, const double* x, double* y,
                 int n, double alpha, double beta, hipStream_t s);
void launch_dot(const double* a, const double* b, int n, double* part, double* out, int sqrt_out, hipStream_t s);
void launch_axpy(double* y, const double* x, int n, const double* alpha, double sgn, int inv, hipStream_t s);
void launch_gather(double* y, const double* x, const int* map, int n, hipStream_t s);
// out[s] = sum of x[i]^2 over [off[s], off[s+1]), s < nseg (off on the device)
void launch_seg_sumsq(const double* x, const int64_t* off, int nseg, double* out, hipStream_t s);
void launch_adjoint_grad(const int* row, const int* col, const double* lam, const double* x, double* g, int64_t nnz,
                         hipStream_t s);

}  // namespace hssmf

// FP64 small dense linear algebra for the factorization step of the two-site
// update: Cholesky-QR of the sketch, and the symmetric eigenproblem that gives
// the truncated SVD.  Every kernel takes a device array of per-problem
// descriptors so one launch serves all bonds of a batched half-step.
#pragma once

#include "common.hpp"

namespace mpofit {

// Cholesky G = R^T R (R upper triangular, R_jj > 0); R is written row-major
// into `R` (ldr), its strictly lower part zeroed.  G is only read.
struct CholDesc {
  const double* G;
  int ldg;
  double* R;
  int ldr;
  int k;
  int* flag;  // FLAG_CHOL on a non-positive pivot
};

// X <- X R^{-1} for an n x k row-major X (ldx) and upper triangular R (ldr).
struct TrsmDesc {
  double* X;
  int ldx;
  const double* R;
  int ldr;
  int n, k;
};

// Top-r eigenpairs of a symmetric k x k matrix H (row-major, ldh, only the
// lower triangle is read): eigenvalues descending in `evals`, eigenvectors as
// the columns of the k x r row-major Z (ldz).
struct EigDesc {
  const double* H;
  int ldh;
  int k, r;
  double* evals;
  double* Z;
  int ldz;
  double* work;  // >= eig_work_doubles(k, r) doubles
  int* flag;
};

size_t eig_work_doubles(int k, int r);
// Offsets inside the eigen work area: Q^T (k x k, row-major) of the
// register path, and the k x r eigenvectors of the tridiagonal matrix.
double* eig_work_qt(double* w, int k, int r);
double* eig_work_x(double* w, int k, int r);

// Largest k handled by the register-resident kernels.
constexpr int kRegMax = 160;

// Cholesky of G.  inverse = 0: R (upper, R^T R = G) into d.R.
// inverse = 1 (needs every k <= kRegMax): R^{-1} (upper) into d.R instead.
void launch_chol(const CholDesc* d, int n, int max_k, int inverse, hipStream_t s);
void launch_trsm(const TrsmDesc* d, int n, int max_rows, hipStream_t s);
// Runs the eigen pipeline: tridiagonalization (stage 0), bisection (1),
// twisted-factorization eigenvectors (2), back-transformation (3, not with
// `reg`); stage < 0 runs all of them.  With `reg` (every k <= kRegMax) the
// reduction keeps the matrix in registers and leaves Q^T in the work area;
// the caller then forms Z = Q X with a GEMM.  `h_descs` is the host copy of `d`.
void launch_eig(const EigDesc* d, const EigDesc* h_descs, int n, int reg, int stage, hipStream_t s);

}  // namespace mpofit

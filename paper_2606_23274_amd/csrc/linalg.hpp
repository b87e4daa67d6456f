// FP64 small dense linear algebra for the factorization step of the two-site
// update: Cholesky-QR of the sketch, and the symmetric eigenproblem that gives
// the truncated SVD.  Every kernel takes a device array of per-problem
// descriptors so one launch serves all bonds of a batched half-step.
#pragma once

#include "common.hpp"

namespace mpofit {

// Cholesky G = R^T R (R upper triangular, R_jj > 0); R is written row-major
// into `R` (ldr), its strictly lower part zeroed.  G is only read.
//
// keep (nullable, k entries): a column j with keep[j] == 0 is known to be
// zero in the matrix whose Gram G is; G(j, j) is taken as 1 so that R has a
// unit row and column there and X R^{-1} keeps the column zero.
// eta > 0 (rank-revealing): a pivot at or below eta times the column's own
// diagonal G(j, j) means the column lies in the span of the previous ones;
// its row of R (and of R^{-1}) becomes zero, without a flag, so X R^{-1} has
// a zero column there.
struct CholDesc {
  const double* G;
  int ldg;
  double* R;
  int ldr;
  int k;
  int* flag;  // FLAG_CHOL on a non-positive pivot (eta = 0) or a non-finite one
  double shift = 0;  // > 0: factor G + shift * trace(G) I instead (general kernel)
  const double* keep = nullptr;
  double eta = 0;
};

// X <- X R^{-1} for an n x k row-major X (ldx) and upper triangular R (ldr);
// a zero diagonal entry of R gives a zero column.
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

// One-sided Jacobi SVD (Hestenes) of a q x q row-major matrix R: columns are
// rotated pairwise (round-robin order) until every pair is orthogonal to
// 1e-15 relative, then the column norms S (descending) and the unit columns
// Ur (row-major q x q, ldu, same order) are written, so that R V = Ur diag(S)
// for an orthogonal V that is not formed.  Small singular values keep high
// relative accuracy (no Gram matrix is formed).  work: q*q doubles, used
// when q > kJacobiLds.  Singular values S_j <= trunc S_0 are truncated (S_j
// and column j of Ur set to zero) and counted in *count.
struct JacobiDesc {
  const double* R;
  int ldr, q;
  double* Ur;
  int ldu;
  double* S;
  double* work;
  double trunc;
  int* count;
};
constexpr int kJacobiLds = 128;
void launch_jacobi(const JacobiDesc* d, int n, int max_q, hipStream_t s);

// Householder QR of an m x n row-major X (ldx), overwritten: writes the
// upper-trapezoidal R (min(m, n) x n, row-major, ldr, zeros below the
// diagonal) of X = Q R; Q is not formed.  Backward stable (no Gram matrix),
// so a norm carried through a sweep of such factorizations keeps an absolute
// accuracy of a few units of rounding of the input's norm.
struct GeqrDesc {
  double* X;
  int m, n, ldx;
  double* R;
  int ldr;
  double* tau;  // nullable: the reflector coefficients, for orgqr_kernel
};
// Q (m x n, m >= n) from the reflectors geqr_kernel left in X and tau, with
// the signs normalized so that diag(R) >= 0 (column c of Q and row c of R
// negated where R(c, c) < 0).
struct OrgqrDesc {
  const double* X;
  int m, n, ldx;
  const double* tau;
  double* Q;
  int ldq;
  double* R;
  int ldr;
};
void launch_geqr(const GeqrDesc* d, int n, hipStream_t s);
void launch_orgqr(const OrgqrDesc* d, int n, hipStream_t s);
// Both in one kernel with X resident in LDS (when hhqr_fits_lds(m, n) for
// every problem of the launch; max_m, max_n size the LDS): R (diag >= 0),
// tau (nullable) and Q out, X left unchanged.
struct HhqrDesc {
  const double* X;
  int m, n, ldx;
  double* tau;
  double* Q;
  int ldq;
  double* R;
  int ldr;
};
bool hhqr_fits_lds(int m, int n);
void launch_hhqr(const HhqrDesc* d, int n, int max_m, int max_n, hipStream_t s);

size_t eig_work_doubles(int k, int r);
// Panel reduction of the global-memory path: widest panel, the panel width
// for a launch (0: use the unblocked kernel), the stage code of the panel
// starting at column j0 (kEigPanelStage + j0), and the work-array pieces the
// trailing-update GEMM reads and writes: the full symmetric matrix (k x k)
// and the panel operands P1 = [V W], P2 = P1 + 2 kPanel k (k rows of 2 nb).
constexpr int kPanel = 32;
constexpr int kEigPanelStage = 1 << 20;
int eig_panel_width(int max_k);
__host__ __device__ inline double* eig_work_h(double* w, int k, int r) {
  return w + 3 * (size_t)k + (size_t)k * k + (size_t)k * r;
}
__host__ __device__ inline double* eig_work_panel(double* w, int k, int r) {
  return w + 3 * (size_t)k + 2 * (size_t)k * k + (size_t)k * r;
}

// Largest k handled by the register-resident kernels.
constexpr int kRegMax = 176;

// Cholesky of G.  inverse = 0: R (upper, R^T R = G) into d.R.
// inverse = 1 (needs every k <= kRegMax): R^{-1} (upper) into d.R instead.
void launch_chol(const CholDesc* d, int n, int max_k, int inverse, hipStream_t s);
void launch_trsm(const TrsmDesc* d, int n, int max_rows, hipStream_t s);
// Runs the eigen pipeline: tridiagonalization (stage 0), bisection (1),
// twisted-factorization eigenvectors (2), back-transformation (3); stage < 0
// runs all of them.  With `reg` (every k <= kRegMax) the reduction keeps the
// matrix in registers and stage 3 applies the reflectors to the rows of X^T
// (Z^T = X^T Q^T).  `h_descs` is the host copy of `d`.
void launch_eig(const EigDesc* d, const EigDesc* h_descs, int n, int reg, int stage, hipStream_t s);

}  // namespace mpofit

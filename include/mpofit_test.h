/*
 * Test hooks of libmpofit: direct entry points to some of its kernels so the
 * test suite can check them in isolation against NumPy.  Not part of the fit
 * API.  Same conventions as mpofit.h (device pointers, caller-owned
 * workspace of at least 64 MiB, 256-byte aligned, work on `stream`, the call
 * synchronizes the stream before returning).
 */
#ifndef MPOFIT_TEST_H
#define MPOFIT_TEST_H

#include "mpofit.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C[M x N] = alpha * op(A) op(B) (+ C if beta), through the grouped MFMA GEMM.
   mode: 0 FP64, 1 FP32, 2 BF16; ta/tb/tc: 0 FP64, 1 FP32 element types;
   a_kcontig: A(m,k) at m*lda+k (1) or k*lda+m (0); b_kcontig: B(k,n) at
   n*ldb+k (1) or k*ldb+n (0); C(m,n) at m*ldc+n; tile 0 (64x64), 1
   (128x128, FP32/BF16), 2 (64x64 with half-depth K slabs, FP32/BF16), 3
   (32x32), 4 (32x32 with deep K slabs) or 5 (16x16 with the
   K range split over the workgroup's waves, FP64, splits = 1); splits >= 1
   forces that many K chunks.  Another tile returns MPO_ERR_INVALID_ARG. */
mpo_status mpo_test_gemm(int mode, int ta, int tb, int tc, int a_kcontig, int b_kcontig, int tile,
                         int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                         void* Cm, int ldc, double alpha, int beta, int splits, void* workspace,
                         size_t ws_bytes, void* stream);

/* Top r eigenpairs of the symmetric k x k FP64 matrix H (row-major, lower
   triangle read): evals descending, Z k x r row-major. */
mpo_status mpo_test_eig(const double* H, int k, int r, double* evals, double* Z, void* workspace,
                        size_t ws_bytes, void* stream);

/* The same for n independent problems in one launch of each eigen kernel
   (the batched schedules' configuration): H is n consecutive k x k
   matrices, evals n x r, Z n consecutive k x r matrices. */
mpo_status mpo_test_eig_batch(const double* H, int n, int k, int r, double* evals, double* Z,
                              void* workspace, size_t ws_bytes, void* stream);

/* Q = CholeskyQR2 of the n x k FP64 matrix X (row-major, in place). */
mpo_status mpo_test_cholqr(double* X, int n, int k, void* workspace, size_t ws_bytes, void* stream);

/* One-sided Jacobi SVD (the kernel of the inverse canonical form's
   initialization): W is q x q row-major (1 <= q <= 512); on return the
   columns of Ur (q x q row-major) are the left singular vectors of W and S
   its singular values, both in descending order of S, with no truncation. */
mpo_status mpo_test_jacobi(const double* W, int q, double* Ur, double* S, void* workspace,
                           size_t ws_bytes, void* stream);

/* The range finder's QR: one rank-revealing Cholesky-QR pass (a column in
   the span of the previous ones, pivot at or below 1e-12 of its own squared
   norm, becomes a zero column of Q instead of a failure), then one
   Newton-Schulz step Q <- Q (3 I - Q^T Q) / 2. */
mpo_status mpo_test_cholqr_rr(double* X, int n, int k, void* workspace, size_t ws_bytes, void* stream);

/* Gaussian test matrix of one bond (same definition as the fit's): out is
   m x k FP64 row-major with rows in (c'', su) order, m = chi * dd. */
mpo_status mpo_test_omega(double* out, int chi, int dd, int k, int bond, int stream_idx, int pair,
                          uint64_t seed, void* workspace, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MPOFIT_TEST_H */

// Element-wise and small kernels of the two-site update (gfx950).
#pragma once

#include "common.hpp"

namespace mpofit {

// Gaussian test matrix Omega of one bond (Sec. 3.1, Fig. rsvd (b1)), m x k,
// FP64, stored row-major with row p = c''*dd + su for the two-site matrix's
// column (c'', su) (su = s2*d + u2).  Element value: Philox4x64-10 at
// counter (e/4, bond, stream, pair), key (seed, 0), Box-Muller of words
// (2q, 2q+1) with q = (e%4)/2, cosine for even e and sine for odd e, where
// e = i*k + j and i = su*chi + c'' is the column index in (s2, u2, c'')
// row-major order.  stream = (*stream_base) * stream_mul + stream_add.
struct OmegaDesc {
  double* out;
  int m, k;        // m = chi * dd
  int chi, dd;     // chi'' and d*d
  int bond, pair;
  int stream_mul, stream_add;
  const int* stream_base;
  unsigned long long seed;
  // with rk (the current bond dims of the train, indexed by bond: the
  // tolerance rule of Sec. 2.3.4 changes them during a sweep) the matrix
  // has the bond's actual shape, chi = rk[bond + 1] and
  // k = min(kk, cap, rk[bond - 1] * dd, dd * chi), drawn as above into rows
  // with c'' < chi and columns j < k of the buffer (ld k), which the caller
  // zeroes first
  const int* rk = nullptr;
  int kk = 0, cap = 0;  // chi_max + p and the rank cap chi^A chi^B of the bond
};
void launch_omega(const OmegaDesc* d, int n, int max_elems, hipStream_t s);

// Column signs of U (n x r, ld): largest-magnitude entry of each column made
// positive (first index on ties); U scaled in place, signs written (+-1).
// Also records max |U| into *amax (float bits) when amax is non-null.
struct SignDesc {
  double* U;
  int n, r, ld;
  double* sign;
  unsigned* amax;
};
void launch_signfix(const SignDesc* d, int n, int max_r, hipStream_t s);

// out(i, j) = in(i, j) * (row ? row[i] : 1) * (col ? col[j] : 1) for an
// n x r matrix; `out` may alias `in`.  row_inv/col_inv = 1 invert the scale
// vector (pseudo-inverse: a zero entry gives zero); col_inv = 2 uses col as
// a mask (out = col[j] != 0 ? in : 0).
struct ScaleDesc {
  const double* in;
  double* out;
  int n, r, ldi, ldo;
  const double* row;
  const double* col;
  int row_inv, col_inv;
};
void launch_scale(const ScaleDesc* d, int n, int max_elems, hipStream_t s);

// 4-D copy with permutation and type conversion: out[o] = in[i] where the
// input index is (i0, i1, i2, i3) with extents n[] and strides si[], and the
// output index uses strides so[] for the same (i0..i3).  Types: 0 = FP64,
// 1 = FP32.  Scale multiplies every element.
// Strided copy / permutation of up to 6 axes (axis 5 fastest), with type
// conversion (0 = FP64, 1 = FP32) and a scale.
struct PermDesc {
  const void* in;
  void* out;
  int n[6];
  long long si[6], so[6];
  int tin, tout;
  double scale;
  unsigned* amax;  // nullable: atomic max of |out| (float bits)
};
void launch_perm(const PermDesc* d, int n, long long max_elems, hipStream_t s);

// Singular values of the top r eigenvalues of a Gram matrix, S_j =
// sqrt(max(lambda_j, 0)), with the drop rule of the update: keep[j] = 1 if
// S_j > kDrop S_0, else 0, and then S_j = 0 (the triplet is dropped; in the
// inverse gauge this is the truncation before inversion).  Dropped values
// are counted in *count (nullable); NaN/Inf raise FLAG_NONFINITE.
struct SvalDesc {
  const double* evals;
  double* S;
  int r;
  int unused;
  int* flag;
  double* keep = nullptr;
  int* count = nullptr;
};
// Relative cut of singular values: an FP64 SVD fixes the vectors of values
// above it to about 1e-10, and 1 / sigma amplifies rounding by at most 1e6
// (the Gram eigenproblem itself resolves sigma down to about 1e-8 sigma_1).
constexpr double kDrop = 1e-6;
void launch_svals(const SvalDesc* d, int n, int max_r, hipStream_t s);

// Tolerance truncation of Sec. 2.3.4 for one bond, after launch_svals: with
// lambda_j (descending, j < r) the computed top eigenvalues of a Gram matrix
// whose diagonal (kd entries) is `diag`, so that the sum of all sigma^2 is
// its trace T, the kept count is the smallest c >= 1 with
// T - sum_{j<c} max(lambda_j, 0) <= thr T (thr = (tau / L)^2), capped at
// min(chi_max, cap, rk[bond - 1] dd, dd rk[bond + 1], r).  S_j and keep_j
// are zeroed for j >= c, rk[bond] = c, and the drop rule's zeros among the
// kept values are counted into *count (nullable).  One workgroup per bond.
struct TruncDesc {
  const double* diag;
  int kd;
  int r;
  const double* evals;
  double* S;
  double* keep;
  int* rk;
  int bond, dd, chi_max, cap;
  double thr;
  int* count;
};
void launch_trunc(const TruncDesc* d, int n, hipStream_t s);

// Zero `n_words` 32-bit words at each pointer; when eye_rows > 0 write an
// eye_rows x eye_cols identity (row-major, FP64 if eye_f64 else FP32) instead.
struct FillDesc {
  void* p;
  long long n_words;
  int eye_rows, eye_cols, eye_f64;
};

// nu = ||x||_F of n doubles (one workgroup), x /= nu, *nu_out = nu.
struct NormDesc {
  double* x;
  long long n;
  double* nu_out;
};
void launch_norm(const NormDesc* d, int n, hipStream_t s);
// The same for one large array, over many workgroups: partial sums of
// squares into `part` (>= 1024 doubles), then nu, then the division.
void launch_norm_big(double* x, long long n, double* part, double* nu_out, hipStream_t s);
void launch_fill(const FillDesc* d, int n, long long max_words, hipStream_t s);

// Alg. 1 (naive product) for one site: P[(ia, ib), s, u, (ja, jb)] =
// sum_t A[ia, s, t, ja] B[ib, t, u, jb], all FP64 row-major, the left and
// right bonds of P grouped with A's index major.
struct NaiveDesc {
  const double* A;
  const double* B;
  double* P;
  int a0, a1, b0, b1, d;
};
void launch_naive(const NaiveDesc* d, int n, long long max_elems, hipStream_t s);

// One Newton-Schulz step towards the orthonormal polar factor: with
// G = X^T X (k x k, row-major), G <- (3 I - G) / 2; then X G has
// ||(X G)^T (X G) - I|| <= (3/4) ||X^T X - I||^2 + rounding.  Zero columns of
// X stay zero and do not touch the others.
struct PolishDesc {
  double* G;
  int k;
};
void launch_polish(const PolishDesc* d, int n, int max_k, hipStream_t s);

// *counter += 1 (one thread); used to advance the sweep index inside a graph.
void launch_bump(int* counter, int by, hipStream_t s);

}  // namespace mpofit

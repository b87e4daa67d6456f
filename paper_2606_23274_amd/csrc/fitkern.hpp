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
// n x r matrix; `out` may alias `in`.  rinv/cinv invert the scale vector.
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

// Singular values S_j = sqrt(max(lambda_j, 0)) of r eigenvalues; raises
// FLAG_NONFINITE on NaN/Inf.
// S = sqrt(max(lambda, 0)).  With `guard` (inverse gauge) keep[j] = 1 if
// S_j > kInvTrunc S_0 else 0 (the value is then truncated before inversion,
// and counted in *count).
struct SvalDesc {
  const double* evals;
  double* S;
  int r;
  int guard;
  int* flag;
  double* keep = nullptr;
  int* count = nullptr;
};
constexpr double kInvTrunc = 1e-12;
void launch_svals(const SvalDesc* d, int n, int max_r, hipStream_t s);

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

// *counter += 1 (one thread); used to advance the sweep index inside a graph.
void launch_bump(int* counter, int by, hipStream_t s);

}  // namespace mpofit

// Grouped, batched, split-K GEMM on the gfx950 matrix cores.
//
// One launch runs a list of problems ("descriptors"); each problem is
// C[b] = alpha * op(A[b]) op(B[b]) (+ C[b] if beta), with a three-level batch
// index b = (b0, b1, b2) whose strides are given per operand.  Every tensor
// contraction of the fit is one such problem: the leg orders of the stored
// tensors are chosen so that each contracted and each free index group has a
// single stride (see the layout notes in runtime.hip).
#pragma once

#include "common.hpp"

namespace mpofit {

struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  long long sA[3], sB[3], sC[3];  // batch strides (elements) for b0, b1, b2
  int nb[3];                      // batch extents
  int M, N, K;
  int lda;      // A(m,k) at m*lda + k (K-contiguous) or k*lda + m (M-contiguous)
  int ldb;      // B(k,n) at n*ldb + k (K-contiguous) or k*ldb + n (N-contiguous)
  int ldc;      // C(m,n) at m*ldc + n
  int splits;   // K split into `splits` chunks of `kchunk` (multiple of BK)
  int kchunk;
  int tiles_m, tiles_n;
  int wg_begin;  // first workgroup of this problem within the launch
  int beta;      // 1: accumulate into C
  int vec_a, vec_b;  // 4-wide vector loads are in bounds and aligned
  double alpha;
  const unsigned* amax_a;  // BF16 mode: |A| maximum (float bits) for the scale
  const unsigned* amax_b;
  unsigned* amax_c;        // nullable: atomic max of |C| (float bits)
  void* partials;          // split-K partial tiles (accumulator type)
  int* counters;           // split-K arrival counters, zero between launches
};

// Compile-time shape of a launch.
struct GemmKind {
  Mode mode;
  DType ta, tb, tc;
  bool a_kcontig, b_kcontig;
  int tile;  // 0: 64x64 tile, 1: 128x128 tile (FP32/BF16 modes only)
  bool operator<(const GemmKind& o) const {
    return std::tie(mode, ta, tb, tc, a_kcontig, b_kcontig, tile) <
           std::tie(o.mode, o.ta, o.tb, o.tc, o.a_kcontig, o.b_kcontig, o.tile);
  }
};

int gemm_bm(int tile);
int gemm_bn(int tile);
int gemm_bk(Mode mode, int tile);
size_t gemm_acc_bytes(Mode mode);

// Launches one grouped GEMM: `d_descs` is a device array of `n_desc`
// descriptors whose wg_begin fields are the prefix sums of their workgroup
// counts; `total_wgs` is the grand total.
void launch_gemm(const GemmKind& kind, const GemmDesc* d_descs, int n_desc, int total_wgs,
                 hipStream_t stream);

}  // namespace mpofit

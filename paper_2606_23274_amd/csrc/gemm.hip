// Grouped MFMA GEMM for gfx950 (see gemm.hpp).
//
// Workgroup = 256 threads = 4 wave64s in a 2x2 grid; each wave owns a
// (BM/2) x (BN/2) block of the tile made of 16x16 MFMA blocks.
//   FP64: v_mfma_f64_16x16x4f64
//   FP32: v_mfma_f32_16x16x4f32
//   BF16: v_mfma_f32_16x16x32_bf16, FP32 accumulation
//   BF16X3: each operand x = hi + lo with hi = bf16(x), lo = bf16(x - hi);
//         three BF16 MFMAs per product (lo*hi + hi*lo + hi*hi), FP32 accumulation
// Both operand tiles sit in LDS as [row][BK + pad] with K contiguous, so each
// lane fetches its fragment with one wide LDS read.  Within each 16-wide
// (FP32/FP64) or 32-wide (BF16) sub-slab, lane group g = lane/16 feeds
// k = 4g + s (k = 8g + s) to MFMA step s: a permutation of the summation order
// that lets those values be one vector read.  The LDS is double-buffered: the
// global loads of slab t+1 are in flight while slab t is multiplied.  The
// slab depth BK is chosen so that one slab's MFMA work (about 2000 cycles per
// wave) covers the latency of the next slab's global loads; the two LDS
// buffers then take about 70 KB, two workgroups per CU.
#include <tuple>

#include "gemm.hpp"

namespace mpofit {

namespace {

constexpr int kThreads = 256;

template <int TILE> struct TileShape;
template <> struct TileShape<0> { static constexpr int BM = 64, BN = 64; };
template <> struct TileShape<1> { static constexpr int BM = 128, BN = 128; };
template <> struct TileShape<2> { static constexpr int BM = 64, BN = 64; };  // half-depth slabs
// For products with few 64 x 64 tiles, where those leave most of the chip
// idle and split-K pays a device-scope fence per tile (FP64: the small
// factorization products, k x k Gram matrices and n x k applications; FP32:
// the serial sweep's two-site product, 64 tiles of 64 x 64; BF16 modes
// likewise):
//   3: 32 x 32, one 16 x 16 MFMA block per wave, 32-deep slabs (BF16: 64,
//      split BF16: 32);
//   4: the same with 128-deep slabs (fewer global-load round trips; split
//      BF16: 64);
// FP64 only:
//   5: 16 x 16, the four waves take interleaved quarters of each 128-deep
//      slab and sum their blocks through LDS at the end (a quarter of the
//      MFMA chain per wave, no global split-K).
template <> struct TileShape<3> { static constexpr int BM = 32, BN = 32; };
template <> struct TileShape<4> { static constexpr int BM = 32, BN = 32; };
template <> struct TileShape<5> { static constexpr int BM = 16, BN = 16; };

template <Mode M> struct ModeT;
template <> struct ModeT<Mode::F64> {
  using acc_t = double;
  using lds_t = double;
  using accv_t = doublex4;
  static constexpr int KSUB = 16;  // K per sub-slab (4 MFMA steps of 4)
  static constexpr int PAD = 2;
  static constexpr int PADT = 2;   // row pad of the k-major staging
};
template <> struct ModeT<Mode::F32> {
  using acc_t = float;
  using lds_t = float;
  using accv_t = floatx4;
  static constexpr int KSUB = 16;
  static constexpr int PAD = 4;
  static constexpr int PADT = 4;
};
template <> struct ModeT<Mode::BF16> {
  using acc_t = float;
  using lds_t = unsigned short;
  using accv_t = floatx4;
  static constexpr int KSUB = 32;  // one MFMA step
  static constexpr int PAD = 8;
  static constexpr int PADT = 0;  // (BF16 operands are always staged row-major)
};
template <> struct ModeT<Mode::BF16X3> : ModeT<Mode::BF16> {};

// Slab depth per (mode, tile); must agree with gemm_bk() below.  Tile 2 is
// the 64 x 64 tile with half-depth slabs: half the LDS, so twice the
// workgroups per CU, which pays when K is short and every tile's first
// loads are exposed.
constexpr int slab_k(Mode m, int tile) {
  return m == Mode::F64 ? (tile >= 4 ? 128 : 32)
         : m == Mode::F32 ? (tile == 0 ? 64 : tile == 4 ? 128 : 32)
         : m == Mode::BF16 ? (tile == 0 || tile == 4 ? 128 : 64)
                           : (tile == 0 || tile == 4 ? 64 : 32);
}

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <DType T> struct DT;
template <> struct DT<DType::F64> { using type = double; };
template <> struct DT<DType::F32> { using type = float; };

// FP32 -> BF16 bits, round to nearest even: the hardware conversion
// (v_cvt_pk_bf16_f32 on gfx950), two values per instruction.
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned short f2bf(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
__device__ __forceinline__ unsigned f2bf2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2v{a, b}, bf16x2v));
}

// Exponent e with 2^e <= amax < 2^(e+1); 0 for amax == 0.
__device__ __forceinline__ int scale_exp(const unsigned* amax) {
  if (!amax) return 0;
  float a = __uint_as_float(*amax);
  if (!(a > 0.f)) return 0;
  int e;
  frexpf(a, &e);
  return e - 1;
}

template <Mode MODE, typename T>
__device__ __forceinline__ typename ModeT<MODE>::lds_t to_lds(T v, float inv_scale) {
  if constexpr (MODE == Mode::F64) return (double)v;
  else if constexpr (MODE == Mode::F32) return (float)v;
  else return f2bf((float)v * inv_scale);
}

// Loads a (ROWS x BK) operand tile into registers in the stored type; the
// conversion to the LDS type (and the BF16 scale) happens at the LDS store.
// RT (BF16 modes, operand rows contiguous in memory): each thread loads four
// consecutive k of one row (lanes take consecutive rows, so every load is
// coalesced across the wave) and stores them as one packed 8-byte LDS write
// into the row-major [row][k] tile the BF16 MFMA reads.
template <typename T, bool KCONTIG, int ROWS, int BK, bool RT = false>
struct TileLoader {
  static constexpr int NV = ROWS * BK / 4 / kThreads;  // 4-wide loads per thread
  static_assert(NV >= 1, "tile too small");
  T v[NV][4];

  __device__ __forceinline__ void load(const T* base, int ld, int rows_valid, int k0, int kend,
                                       bool vec_ok) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int idx = threadIdx.x + kThreads * i;
      int r, k;
      if constexpr (RT) {
        r = idx % ROWS;
        k = k0 + 4 * (idx / ROWS);
        const GAS T* g = gload_ptr(base + (long long)k * ld + r);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          v[i][j] = (r < rows_valid && k + j < kend) ? g[(long long)j * ld] : T(0);
        continue;
      } else if constexpr (KCONTIG) {
        r = idx / (BK / 4);
        k = k0 + 4 * (idx % (BK / 4));
      } else {
        k = k0 + idx / (ROWS / 4);
        r = 4 * (idx % (ROWS / 4));
      }
      const T* p = KCONTIG ? base + (long long)r * ld + k : base + (long long)k * ld + r;
      const bool full = KCONTIG ? (r < rows_valid && k + 3 < kend) : (r + 3 < rows_valid && k < kend);
      if (vec_ok && full) {
        if constexpr (sizeof(T) == 4) {
          const floatx4 q = *reinterpret_cast<const GAS floatx4*>(gload_ptr(p));
          v[i][0] = q[0]; v[i][1] = q[1]; v[i][2] = q[2]; v[i][3] = q[3];
        } else {
          const doublex2 q0 = *reinterpret_cast<const GAS doublex2*>(gload_ptr(p));
          const doublex2 q1 = *reinterpret_cast<const GAS doublex2*>(gload_ptr(p + 2));
          v[i][0] = q0[0]; v[i][1] = q0[1]; v[i][2] = q1[0]; v[i][3] = q1[1];
        }
      } else {
        const GAS T* g = gload_ptr(p);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool ok = KCONTIG ? (r < rows_valid && k + j < kend) : (r + j < rows_valid && k < kend);
          v[i][j] = ok ? g[j] : T(0);
        }
      }
    }
  }

  // Row-major staging ([row][k], pitch ldl) or, with KMAJOR (an operand
  // whose rows are contiguous in memory, FP32/FP64 only), k-major staging
  // ([k][row], pitch ldl): the four rows a thread loaded go out as one
  // 16-byte-aligned vector store, free of bank conflicts.
  template <Mode MODE, bool KMAJOR = false, typename L>
  __device__ __forceinline__ void store(L* lds, L* lds_lo, int ldl, float inv_scale) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int idx = threadIdx.x + kThreads * i;
      if constexpr (KMAJOR) {
        static_assert(!KCONTIG, "k-major staging is for row-contiguous operands");
        const int k = idx / (ROWS / 4);
        const int r = 4 * (idx % (ROWS / 4));
        L* q = lds + k * ldl + r;
        if constexpr (sizeof(L) == 4) {
          *reinterpret_cast<floatx4*>(q) =
              floatx4{to_lds<MODE>(v[i][0], inv_scale), to_lds<MODE>(v[i][1], inv_scale),
                      to_lds<MODE>(v[i][2], inv_scale), to_lds<MODE>(v[i][3], inv_scale)};
        } else {
          *reinterpret_cast<doublex2*>(q) =
              doublex2{to_lds<MODE>(v[i][0], inv_scale), to_lds<MODE>(v[i][1], inv_scale)};
          *reinterpret_cast<doublex2*>(q + 2) =
              doublex2{to_lds<MODE>(v[i][2], inv_scale), to_lds<MODE>(v[i][3], inv_scale)};
        }
      } else if constexpr (MODE == Mode::BF16 || MODE == Mode::BF16X3) {
        static_assert(KCONTIG || RT, "BF16 operands are staged row-major");
        const int r = RT ? idx % ROWS : idx / (BK / 4);
        const int k = RT ? 4 * (idx / ROWS) : 4 * (idx % (BK / 4));
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = (float)v[i][j] * inv_scale;
        const unsigned h0 = f2bf2(x[0], x[1]), h1 = f2bf2(x[2], x[3]);
        *reinterpret_cast<uint2*>(lds + r * ldl + k) = uint2{h0, h1};
        if constexpr (MODE == Mode::BF16X3) {  // lo = bf16(x - hi)
          const float l0 = x[0] - __uint_as_float(h0 << 16), l1 = x[1] - __uint_as_float(h0 & 0xffff0000u);
          const float l2 = x[2] - __uint_as_float(h1 << 16), l3 = x[3] - __uint_as_float(h1 & 0xffff0000u);
          *reinterpret_cast<uint2*>(lds_lo + r * ldl + k) = uint2{f2bf2(l0, l1), f2bf2(l2, l3)};
        }
      } else if constexpr (KCONTIG) {
        int r = idx / (BK / 4);
        int k = 4 * (idx % (BK / 4));
        L* q = lds + r * ldl + k;
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] = to_lds<MODE>(v[i][j], inv_scale);
      } else {
        static_assert(KCONTIG, "row-contiguous FP32 / FP64 operands are staged k-major");
      }
    }
  }
};

template <Mode MODE, typename TA, typename TB, typename TC, bool AK, bool BKC, int TILE>
__global__ void __launch_bounds__(kThreads)
gemm_kernel(const GemmDesc* __restrict__ descs, int n_desc) {
  using MT = ModeT<MODE>;
  using acc_t = typename MT::acc_t;
  using lds_t = typename MT::lds_t;
  using accv_t = typename MT::accv_t;
  constexpr int BM = TileShape<TILE>::BM, BN = TileShape<TILE>::BN;
  constexpr int BK = slab_k(MODE, TILE), LDL = BK + MT::PAD;
  constexpr int NSUB = BK / MT::KSUB;
  constexpr bool KW = TILE == 5;                // waves split K (one output block)
  constexpr int WM = KW ? BM : BM / 2, WN = KW ? BN : BN / 2;  // wave tile
  constexpr int FM = WM / 16, FN = WN / 16;     // MFMA blocks per wave

  constexpr int NLO = MODE == Mode::BF16X3 ? 2 : 1;  // hi (and lo) tiles
  // row-contiguous FP32 / FP64 operands are staged k-major (pitch BM + PADT)
  constexpr bool AT = !AK && (MODE == Mode::F32 || MODE == Mode::F64);
  constexpr bool BT = !BKC && (MODE == Mode::F32 || MODE == Mode::F64);
  constexpr int LDMA = BM + MT::PADT, LDMB = BN + MT::PADT;
  constexpr int SZA = AT ? BK * LDMA : BM * LDL, SZB = BT ? BK * LDMB : BN * LDL;
  __shared__ __align__(16) lds_t sA[NLO][2][SZA];
  __shared__ __align__(16) lds_t sB[NLO][2][SZB];
  __shared__ int s_last;

  // locate this workgroup's problem
  const int wg = blockIdx.x;
  int lo = 0, hi = n_desc - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (descs[mid].wg_begin <= wg) lo = mid; else hi = mid - 1;
  }
  const GemmDesc& d = descs[lo];
  int local = wg - d.wg_begin;
  const int tn = local % d.tiles_n; local /= d.tiles_n;
  const int tm = local % d.tiles_m; local /= d.tiles_m;
  const int split = local % d.splits;
  const int bidx = local / d.splits;
  const int b2 = bidx % d.nb[2];
  const int b1 = (bidx / d.nb[2]) % d.nb[1];
  const int b0 = bidx / (d.nb[2] * d.nb[1]);

  const TA* Ab = reinterpret_cast<const TA*>(d.A) + b0 * d.sA[0] + b1 * d.sA[1] + b2 * d.sA[2];
  const TB* Bb = reinterpret_cast<const TB*>(d.B) + b0 * d.sB[0] + b1 * d.sB[1] + b2 * d.sB[2];
  TC* Cb = reinterpret_cast<TC*>(d.C) + b0 * d.sC[0] + b1 * d.sC[1] + b2 * d.sC[2];

  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = split * d.kchunk;
  const int kend = min(d.K, kbeg + d.kchunk);
  // operand origins: A(m0, .), B(., n0)
  const TA* Ap = AK ? Ab + (long long)m0 * d.lda : Ab + m0;
  const TB* Bp = BKC ? Bb + (long long)n0 * d.ldb : Bb + n0;
  const int rows_a = d.M - m0, rows_b = d.N - n0;

  float inv_sa = 1.f, inv_sb = 1.f, out_scale = 1.f;
  if constexpr (MODE == Mode::BF16 || MODE == Mode::BF16X3) {
    int ea = scale_exp(d.amax_a), eb = scale_exp(d.amax_b);
    inv_sa = ldexpf(1.f, -ea);
    inv_sb = ldexpf(1.f, -eb);
    out_scale = ldexpf(1.f, ea + eb);
  }

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = KW ? 0 : (wave >> 1) * WM, wn = KW ? 0 : (wave & 1) * WN;
  const int lrow = lane & 15, lgrp = lane >> 4;

  accv_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = accv_t{0, 0, 0, 0};
  // FP32 32 x 32 tiles run unsplit over long K (4096 in the serial two-site
  // product): sub-slab ks accumulates into partial sum ks % NACC, which
  // shortens each FP32 accumulation chain NACC times; the partial sums are
  // added in a fixed order after the last slab
  constexpr int NACC = (MODE == Mode::F32 && (TILE == 3 || TILE == 4)) ? 4 : 1;
  accv_t accp[NACC > 1 ? NACC - 1 : 1][FM][FN];
#pragma unroll
  for (int q = 0; q < (NACC > 1 ? NACC - 1 : 1); ++q)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) accp[q][i][j] = accv_t{0, 0, 0, 0};

  constexpr bool BF = MODE == Mode::BF16 || MODE == Mode::BF16X3;
  TileLoader<TA, AK, BM, BK, BF && !AK> la;
  TileLoader<TB, BKC, BN, BK, BF && !BKC> lb;
  const int nslab = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;

  if (nslab > 0) {
    la.load(Ap, d.lda, rows_a, kbeg, kend, d.vec_a);
    lb.load(Bp, d.ldb, rows_b, kbeg, kend, d.vec_b);
    la.template store<MODE, AT>(sA[0][0], sA[NLO - 1][0], AT ? LDMA : LDL, inv_sa);
    lb.template store<MODE, BT>(sB[0][0], sB[NLO - 1][0], BT ? LDMB : LDL, inv_sb);
  }
  __syncthreads();

  for (int t = 0; t < nslab; ++t) {
    const int cur = t & 1;
    const bool more = t + 1 < nslab;
    if (more) {
      la.load(Ap, d.lda, rows_a, kbeg + (t + 1) * BK, kend, d.vec_a);
      lb.load(Bp, d.ldb, rows_b, kbeg + (t + 1) * BK, kend, d.vec_b);
    }
#pragma unroll
    for (int ks = 0; ks < NSUB; ++ks) {
    if (KW && (ks & 3) != wave) continue;  // wave-uniform
    const lds_t* As = sA[0][cur] + ks * MT::KSUB;
    const lds_t* Bs = sB[0][cur] + ks * MT::KSUB;
    if constexpr (MODE == Mode::BF16X3) {
      const lds_t* Al = sA[NLO - 1][cur] + ks * MT::KSUB;
      const lds_t* Bl = sB[NLO - 1][cur] + ks * MT::KSUB;
      bf16x8 af[FM], bfr[FN], afl[FM], bfl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        af[i] = *reinterpret_cast<const bf16x8*>(As + (wm + 16 * i + lrow) * LDL + 8 * lgrp);
        afl[i] = *reinterpret_cast<const bf16x8*>(Al + (wm + 16 * i + lrow) * LDL + 8 * lgrp);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        bfr[j] = *reinterpret_cast<const bf16x8*>(Bs + (wn + 16 * j + lrow) * LDL + 8 * lgrp);
        bfl[j] = *reinterpret_cast<const bf16x8*>(Bl + (wn + 16 * j + lrow) * LDL + 8 * lgrp);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afl[i], bfr[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
    } else if constexpr (MODE == Mode::BF16) {
      bf16x8 af[FM], bfr[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        af[i] = *reinterpret_cast<const bf16x8*>(As + (wm + 16 * i + lrow) * LDL + 8 * lgrp);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bfr[j] = *reinterpret_cast<const bf16x8*>(Bs + (wn + 16 * j + lrow) * LDL + 8 * lgrp);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    } else {
      lds_t af[FM][4], bfr[FN][4];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        if constexpr (AT) {  // k-major: rows of one k are adjacent
          const lds_t* p = sA[0][cur] + (ks * MT::KSUB + 4 * lgrp) * LDMA + wm + 16 * i + lrow;
#pragma unroll
          for (int s = 0; s < 4; ++s) af[i][s] = p[s * LDMA];
        } else {
          const lds_t* p = As + (wm + 16 * i + lrow) * LDL + 4 * lgrp;
#pragma unroll
          for (int s = 0; s < 4; ++s) af[i][s] = p[s];
        }
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if constexpr (BT) {
          const lds_t* p = sB[0][cur] + (ks * MT::KSUB + 4 * lgrp) * LDMB + wn + 16 * j + lrow;
#pragma unroll
          for (int s = 0; s < 4; ++s) bfr[j][s] = p[s * LDMB];
        } else {
          const lds_t* p = Bs + (wn + 16 * j + lrow) * LDL + 4 * lgrp;
#pragma unroll
          for (int s = 0; s < 4; ++s) bfr[j][s] = p[s];
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (MODE == Mode::F64)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][s], bfr[j][s], acc[i][j], 0, 0, 0);
            else if (NACC > 1 && ks % NACC != 0)
              accp[ks % NACC - 1][i][j] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s], bfr[j][s], accp[ks % NACC - 1][i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s], bfr[j][s], acc[i][j], 0, 0, 0);
          }
    }
    }  // sub-slab
    if (more) {
      la.template store<MODE, AT>(sA[0][cur ^ 1], sA[NLO - 1][cur ^ 1], AT ? LDMA : LDL, inv_sa);
      lb.template store<MODE, BT>(sB[0][cur ^ 1], sB[NLO - 1][cur ^ 1], BT ? LDMB : LDL, inv_sb);
    }
    __syncthreads();
  }
  if constexpr (NACC > 1) {
#pragma unroll
    for (int q = 0; q < NACC - 1; ++q)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[i][j][e] += accp[q][i][j][e];
  }

  if constexpr (KW) {  // the four partial blocks, summed in wave order
    __shared__ acc_t red[3][4][64];
    if (wave > 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) red[wave - 1][e][lane] = acc[0][0][e];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[0][0][e] += red[w][e][lane];
  }
  // split-K: every split stores its partial tile; the last to arrive sums
  // them in split order (deterministic) and runs the epilogue.
  if (!KW && d.splits > 1) {
    const long long tile_id = ((long long)bidx * d.tiles_m + tm) * d.tiles_n + tn;
    acc_t* part = reinterpret_cast<acc_t*>(d.partials) +
                  (tile_id * d.splits) * (long long)(BM * BN);
    acc_t* mine = part + (long long)split * (BM * BN);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          gstore_ptr(mine)[(((wave * FM + i) * FN + j) * 4 + e) * 64 + lane] = acc[i][j][e];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      int prev = atomicAdd(d.counters + tile_id, 1);
      s_last = (prev == d.splits - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // sum in split order; the loop is unrolled so that the loads of several
    // partial tiles are in flight together
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = accv_t{0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < d.splits; ++s) {
      const GAS acc_t* ps = gload_ptr(part + (long long)s * (BM * BN) + lane);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[i][j][e] += ps[(((wave * FM + i) * FN + j) * 4 + e) * 64];
    }
    if (threadIdx.x == 0) d.counters[tile_id] = 0;
  }

  // epilogue: lane holds column lrow of each 16x16 block; result register e
  // is row 4*lgrp + e for the FP32/BF16 instructions and row lgrp + 4*e for
  // the FP64 one (four one-row groups per block)
  const double alpha = d.alpha * (double)out_scale;
  float amax = 0.f;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn + 16 * j + lrow;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm + 16 * i + (MODE == Mode::F64 ? lgrp + 4 * e : 4 * lgrp + e);
        if (row < d.M && col < d.N) {
          GAS TC* p = gstore_ptr(Cb + (long long)row * d.ldc + col);
          double v = alpha * (double)acc[i][j][e];
          if (d.beta) v += (double)*p;
          *p = (TC)v;
          amax = fmaxf(amax, fabsf((float)v));
        }
      }
    }
  if (d.amax_c) {
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    if (lane == 0) atomicMax(d.amax_c, __float_as_uint(amax));
  }
}

template <Mode MODE, typename TA, typename TB, typename TC, bool AK, bool BKC>
void launch_tile(int tile, const GemmDesc* d, int n, int wgs, hipStream_t s) {
  if constexpr (MODE == Mode::F64) {
    if (tile == 3) gemm_kernel<MODE, TA, TB, TC, AK, BKC, 3><<<wgs, kThreads, 0, s>>>(d, n);
    else if (tile == 4) gemm_kernel<MODE, TA, TB, TC, AK, BKC, 4><<<wgs, kThreads, 0, s>>>(d, n);
    else if (tile == 5) gemm_kernel<MODE, TA, TB, TC, AK, BKC, 5><<<wgs, kThreads, 0, s>>>(d, n);
    else gemm_kernel<MODE, TA, TB, TC, AK, BKC, 0><<<wgs, kThreads, 0, s>>>(d, n);
  } else {
    if (tile == 1) gemm_kernel<MODE, TA, TB, TC, AK, BKC, 1><<<wgs, kThreads, 0, s>>>(d, n);
    else if (tile == 2) gemm_kernel<MODE, TA, TB, TC, AK, BKC, 2><<<wgs, kThreads, 0, s>>>(d, n);
    // the 32 x 32 tiles, for products with few 64 x 64 tiles
    else if (tile == 3) gemm_kernel<MODE, TA, TB, TC, AK, BKC, 3><<<wgs, kThreads, 0, s>>>(d, n);
    else if (tile == 4) gemm_kernel<MODE, TA, TB, TC, AK, BKC, 4><<<wgs, kThreads, 0, s>>>(d, n);
    else gemm_kernel<MODE, TA, TB, TC, AK, BKC, 0><<<wgs, kThreads, 0, s>>>(d, n);
  }
}

template <Mode MODE, typename TA, typename TB, typename TC>
void launch_layout(const GemmKind& k, const GemmDesc* d, int n, int wgs, hipStream_t s) {
  if (k.a_kcontig && k.b_kcontig) launch_tile<MODE, TA, TB, TC, true, true>(k.tile, d, n, wgs, s);
  else if (k.a_kcontig) launch_tile<MODE, TA, TB, TC, true, false>(k.tile, d, n, wgs, s);
  else if (k.b_kcontig) launch_tile<MODE, TA, TB, TC, false, true>(k.tile, d, n, wgs, s);
  else launch_tile<MODE, TA, TB, TC, false, false>(k.tile, d, n, wgs, s);
}

// Instantiated combinations: FP64 mode takes FP64 or FP32 operands and writes
// FP64; FP32 and BF16 modes take an FP32 or FP64 first
// operand, an FP32 second operand, and write FP32.
template <Mode MODE>
void launch_types(const GemmKind& k, const GemmDesc* d, int n, int wgs, hipStream_t s) {
  if constexpr (MODE == Mode::F64) {
    if (k.tc != DType::F64) throw Error{6, "FP64 GEMM writes FP64"};
    if (k.ta == DType::F64 && k.tb == DType::F64) launch_layout<MODE, double, double, double>(k, d, n, wgs, s);
    else if (k.ta == DType::F64) launch_layout<MODE, double, float, double>(k, d, n, wgs, s);
    else if (k.tb == DType::F64) launch_layout<MODE, float, double, double>(k, d, n, wgs, s);
    else launch_layout<MODE, float, float, double>(k, d, n, wgs, s);
  } else {
    if (k.tc != DType::F32 || k.tb != DType::F32) throw Error{6, "FP32/BF16 GEMM operand types"};
    if (k.ta == DType::F64) launch_layout<MODE, double, float, float>(k, d, n, wgs, s);
    else launch_layout<MODE, float, float, float>(k, d, n, wgs, s);
  }
}

}  // namespace

int gemm_bm(int tile) { return tile == 1 ? 128 : tile == 5 ? 16 : tile >= 3 ? 32 : 64; }
int gemm_bn(int tile) { return gemm_bm(tile); }
int gemm_bk(Mode mode, int tile) { return slab_k(mode, mode == Mode::F64 ? (tile >= 3 ? tile : 0) : tile); }
size_t gemm_acc_bytes(Mode mode) { return mode == Mode::F64 ? 8 : 4; }

void launch_gemm(const GemmKind& kind, const GemmDesc* d_descs, int n_desc, int total_wgs,
                 hipStream_t stream) {
  if (total_wgs <= 0) return;
  switch (kind.mode) {
    case Mode::F64: launch_types<Mode::F64>(kind, d_descs, n_desc, total_wgs, stream); break;
    case Mode::F32: launch_types<Mode::F32>(kind, d_descs, n_desc, total_wgs, stream); break;
    case Mode::BF16: launch_types<Mode::BF16>(kind, d_descs, n_desc, total_wgs, stream); break;
    case Mode::BF16X3: launch_types<Mode::BF16X3>(kind, d_descs, n_desc, total_wgs, stream); break;
  }
}

}  // namespace mpofit

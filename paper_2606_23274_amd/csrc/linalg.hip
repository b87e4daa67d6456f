// FP64 small dense linear algebra of the two-site update (see linalg.hpp).
//
// Cholesky:   one workgroup per matrix; up to k = 176 the matrix and its
//             inverse stay in registers (blocked, right-looking), beyond that
//             the working copy is packed (lower triangle) in LDS when it fits,
//             else kept in the output buffer.
// TRSM:       one wave per row of X; the row lives in registers and the
//             right-looking substitution needs one broadcast per column.
// Eigenpairs: Householder tridiagonalization in one workgroup (in registers
//             up to k = 176; in panels with
//             GPU-wide GEMM updates beyond), then per eigenvalue: bisection on
//             Sturm counts (a workgroup evaluates 256 shifts per round, or
//             eight lanes 8 when there are many eigenvalues), an eigenvector
//             of the tridiagonal from its twisted factorization (one wave per
//             eigenvalue), and the reflectors applied back in column blocks
//             (on the register path row by row, one wave per four
//             eigenvectors).
#include <type_traits>
#include <algorithm>
#include <cfloat>

#include "linalg.hpp"

namespace mpofit {

namespace {

constexpr int kBig = 1024;           // threads of the one-workgroup kernels
constexpr int kPackedMax = 176;      // packed lower triangle in LDS up to this k
constexpr int kTwistWaveMax = 1600;  // one wave per eigenvector up to this k (6 k doubles of LDS)

__device__ __forceinline__ long long pidx(int i, int j) { return (long long)i * (i + 1) / 2 + j; }

// Symmetric matrix, lower triangle (i >= j): packed in LDS, or full
// row-major in global memory.
template <bool GLOBAL> struct SymT;
template <> struct SymT<false> {
  double* p;
  __device__ __forceinline__ double& at(int i, int j) const { return p[pidx(i, j)]; }
};
template <> struct SymT<true> {
  GAS double* p;
  int ld;
  __device__ __forceinline__ GAS double& at(int i, int j) const { return p[(long long)i * ld + j]; }
};

template <int NW>
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------- Cholesky
template <bool GLOBAL>
__global__ void __launch_bounds__(kBig) chol_kernel(const CholDesc* __restrict__ descs) {
  extern __shared__ double lds[];
  __shared__ double s_piv;
  const CholDesc d = descs[blockIdx.x];
  const int k = d.k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  SymT<GLOBAL> A;
  if constexpr (GLOBAL) A = SymT<true>{gstore_ptr(d.R), d.ldr};
  else A = SymT<false>{lds};
  const GAS double* G = gload_ptr(d.G);
  GAS double* Rg = gstore_ptr(d.R);
  for (int i = wave; i < k; i += kBig / 64)
    for (int j = lane; j <= i; j += 64)
      A.at(i, j) = G[(long long)i * d.ldg + j] + ((i == j && d.keep && d.keep[i] == 0.0) ? 1.0 : 0.0);
  if (d.shift > 0.0) {  // G + shift * trace(G) I
    __syncthreads();
    if (threadIdx.x == 0) {
      double tr = 0.0;
      for (int j = 0; j < k; ++j) tr += A.at(j, j);
      s_piv = d.shift * tr;
    }
    __syncthreads();
    const double sh = s_piv;
    for (int j = threadIdx.x; j < k; j += kBig) A.at(j, j) += sh;
  }
  bool bad = false;
  for (int j = 0; j < k; ++j) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = A.at(j, j);
      if (d.eta > 0.0) {  // rank-revealing: a dependent column gives a zero row of R
        const double g0 = G[(long long)j * d.ldg + j] + ((d.keep && d.keep[j] == 0.0) ? 1.0 : 0.0);
        if (v <= d.eta * g0) v = 0.0;
        if (!isfinite(v)) bad = true;
        s_piv = v > 0.0 ? sqrt(v) : 0.0;
      } else {
        if (!(v > 0.0) || !isfinite(v)) { bad = true; v = DBL_MIN; }
        s_piv = sqrt(v);
      }
      A.at(j, j) = s_piv;
    }
    __syncthreads();
    const double inv = s_piv > 0.0 ? 1.0 / s_piv : 0.0;
    for (int i = j + 1 + threadIdx.x; i < k; i += kBig) A.at(i, j) *= inv;
    __syncthreads();
    const int t = k - j - 1;
    for (int il = wave; il < t; il += kBig / 64) {
      const int i = j + 1 + il;
      const double aij = A.at(i, j);
      for (int cl = lane; cl <= il; cl += 64) {
        const int c = j + 1 + cl;
        A.at(i, c) -= aij * A.at(c, j);
      }
    }
  }
  __syncthreads();
  if (bad && d.flag) atomicOr(d.flag, FLAG_CHOL);
  // R = L^T, row-major upper triangle; zero below
  if constexpr (!GLOBAL) {
    for (int i = wave; i < k; i += kBig / 64)
      for (int j = lane; j < k; j += 64)
        Rg[(long long)i * d.ldr + j] = (j >= i) ? A.at(j, i) : 0.0;
  } else {
    for (int i = wave; i < k; i += kBig / 64)
      for (int j = lane; j < i; j += 64) {
        double lo = Rg[(long long)i * d.ldr + j];  // L(i, j)
        Rg[(long long)j * d.ldr + i] = lo;
        Rg[(long long)i * d.ldr + j] = 0.0;
      }
  }
}

// ---------------------------------------------------------------- TRSM
template <int NS>
__global__ void __launch_bounds__(kBig) trsm_kernel(const TrsmDesc* __restrict__ descs) {
  __shared__ double s_inv[64 * NS];
  const TrsmDesc d = descs[blockIdx.y];
  const int k = d.k;
  const GAS double* Rg = gload_ptr(d.R);
  for (int j = threadIdx.x; j < k; j += kBig) {
    const double rjj = Rg[(long long)j * d.ldr + j];
    s_inv[j] = rjj != 0.0 ? 1.0 / rjj : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (kBig / 64) + (threadIdx.x >> 6);
  if (row >= d.n) return;
  GAS double* x = gstore_ptr(d.X + (long long)row * d.ldx);
  double y[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    int c = 64 * s + lane;
    y[s] = c < k ? x[c] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    for (int jj = 0; jj < 64; ++jj) {
      const int j = 64 * s + jj;
      if (j >= k) break;
      const double xj = __shfl(y[s], jj) * s_inv[j];
      if (lane == jj) y[s] = xj;
      const GAS double* rj = Rg + (long long)j * d.ldr;
#pragma unroll
      for (int s2 = s; s2 < NS; ++s2) {
        const int c = 64 * s2 + lane;
        if (c > j && c < k) y[s2] -= xj * rj[c];
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    int c = 64 * s + lane;
    if (c < k) x[c] = y[s];
  }
}

// ---------------------------------------------------------------- eigen
// One DPP move of a double (both 32-bit halves) with a row_ror control.  A
// rotation inside a 16-lane row reads a valid lane everywhere, so no "old"
// value is needed (and none has to be materialised).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over the G lanes of a thread row, returned to all of them: rotations
// by 8, 4, 2, 1 inside each 16-lane DPP row, then (G = 32) one exchange
// between the two rows.
template <int G>
__device__ __forceinline__ double row_reduce(double v) {
  v += dpp_d<0x128>(v);  // row_ror:8
  v += dpp_d<0x124>(v);  // row_ror:4
  v += dpp_d<0x122>(v);  // row_ror:2
  v += dpp_d<0x121>(v);  // row_ror:1
  if constexpr (G == 32) v += __shfl_xor(v, 16);
  return v;
}

// Row sums for every row of a register block, level by level so that the
// NB independent chains interleave.
template <int G, int I0, int NB>
__device__ __forceinline__ void row_reduce_all(double (&p)[NB]) {
#pragma unroll
  for (int i = I0; i < NB; ++i) p[i] += dpp_d<0x128>(p[i]);
#pragma unroll
  for (int i = I0; i < NB; ++i) p[i] += dpp_d<0x124>(p[i]);
#pragma unroll
  for (int i = I0; i < NB; ++i) p[i] += dpp_d<0x122>(p[i]);
#pragma unroll
  for (int i = I0; i < NB; ++i) p[i] += dpp_d<0x121>(p[i]);
  if constexpr (G == 32) {
#pragma unroll
    for (int i = I0; i < NB; ++i) p[i] += __shfl_xor(p[i], 16);
  }
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (all lanes active), returned to all of
// them: row sums by DPP, then the four rows read out as (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0x128>(v);
  v += dpp_d<0x124>(v);
  v += dpp_d<0x122>(v);
  v += dpp_d<0x121>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// 1/x and 1/sqrt(x) for x != 0 (and finite): the hardware estimate refined by two Newton
// steps (about 1 ulp), a shorter dependency chain than the IEEE division.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// work layout (doubles): d[k] e[k] tau[k] V[k*k] X[k*r] Hfull[k*k]
struct EigWork {
  GAS double *d, *e, *tau, *V, *X, *H;
  __device__ EigWork(double* w, int k, int r)
      : d(gstore_ptr(w)), e(gstore_ptr(w + k)), tau(gstore_ptr(w + 2 * k)), V(gstore_ptr(w + 3 * k)),
        X(gstore_ptr(w + 3 * k + (long long)k * k)),
        H(gstore_ptr(w + 3 * k + (long long)k * k + (long long)k * r)) {}
};

// Householder reduction of the symmetric H to tridiagonal T = Q^T H Q with
// Q = H_0 H_1 ... H_{k-3}, H_j = I - tau_j v_j v_j^T, v_j(j+1) = 1 (LAPACK's
// dsytrd convention, lower triangle).
template <bool GLOBAL>
__global__ void __launch_bounds__(kBig) sytrd_kernel(const EigDesc* __restrict__ descs) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  __shared__ double s_tau, s_scal;
  const EigDesc dd = descs[blockIdx.x];
  const int k = dd.k;
  EigWork W(dd.work, k, dd.r);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* sv = lds;          // k
  double* sp = lds + k;      // k
  SymT<GLOBAL> A;
  if constexpr (GLOBAL) A = SymT<true>{W.H, k};
  else A = SymT<false>{lds + 2 * k};
  const GAS double* Hin = gload_ptr(dd.H);
  for (int i = wave; i < k; i += 16)
    for (int j = lane; j <= i; j += 64) A.at(i, j) = Hin[(long long)i * dd.ldh + j];
  for (int j = threadIdx.x; j < k * k; j += kBig) W.V[j] = 0.0;
  __syncthreads();
  for (int j = 0; j + 2 < k; ++j) {
    const int t = k - j - 1;
    for (int i = threadIdx.x; i < t; i += kBig) sv[i] = A.at(j + 1 + i, j);
    __syncthreads();
    double part = 0.0;
    for (int i = threadIdx.x + 1; i < t; i += kBig) part += sv[i] * sv[i];
    const double xnorm2 = block_sum<16>(part, red);
    if (threadIdx.x == 0) {
      const double alpha = sv[0];
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      W.e[j] = beta;
      W.tau[j] = tau;
      W.d[j] = A.at(j, j);
      s_tau = tau;
      s_scal = scal;
    }
    __syncthreads();
    const double tau = s_tau;
    if (tau == 0.0) continue;  // uniform
    for (int i = threadIdx.x; i < t; i += kBig) {
      const double v = (i == 0) ? 1.0 : sv[i] * s_scal;
      sv[i] = v;
      W.V[(long long)j * k + j + 1 + i] = v;
    }
    __syncthreads();
    // p = tau * A22 v
    for (int il = wave; il < t; il += 16) {
      double acc = 0.0;
      for (int cl = lane; cl < t; cl += 64) {
        const double a = (cl <= il) ? A.at(j + 1 + il, j + 1 + cl) : A.at(j + 1 + cl, j + 1 + il);
        acc += a * sv[cl];
      }
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) sp[il] = tau * acc;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = threadIdx.x; i < t; i += kBig) pv += sp[i] * sv[i];
    const double K = -0.5 * tau * block_sum<16>(pv, red);
    for (int i = threadIdx.x; i < t; i += kBig) sp[i] += K * sv[i];
    __syncthreads();
    for (int il = wave; il < t; il += 16) {
      const double vi = sv[il], wi = sp[il];
      for (int cl = lane; cl <= il; cl += 64)
        A.at(j + 1 + il, j + 1 + cl) -= vi * sp[cl] + wi * sv[cl];
    }
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (k >= 2) {
      W.d[k - 2] = A.at(k - 2, k - 2);
      W.e[k - 2] = A.at(k - 1, k - 2);
      W.tau[k - 2] = 0.0;
    }
    W.d[k - 1] = A.at(k - 1, k - 1);
    W.e[k - 1] = 0.0;
    W.tau[k - 1] = 0.0;
  }
}

// Sum over the workgroup (all threads active): wave sums through DPP, one
// barrier.  `red` (16 doubles) must not be read by any thread since the
// previous barrier; callers alternate buffers.
__device__ __forceinline__ double block_sum1(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kBig / 64; ++w) s += red[w];
  return s;
}

// Panel form of the same reduction (the delayed-update scheme of LAPACK's
// dlatrd): the full symmetric matrix lives in W.H and is current at the
// panel start j0; step jj = j0 + cur works with
//   A_cur = A_j0 - V W^T - W V^T   (V, W: the panel's first cur vectors)
// without forming it: column jj and the product A_cur v come from the
// panel-start matrix plus the corrections, so each step reads the trailing
// block once, row by row (coalesced; both triangles are kept).  The panel
// vectors stay in LDS ([p][row]) and leave as P1 = [V W], P2 = [W V] (rows of
// 2 NBP); a batched GEMM then applies A -= P1 P2^T to the trailing block
// before the next panel.  Reflectors, tau, d and e as in sytrd_kernel.
template <int NBP>
__global__ void __launch_bounds__(kBig) sytrd_panel_kernel(const EigDesc* __restrict__ descs, int j0) {
  // column chunks per row (k <= 64 QM for each panel width) and rows per group
  constexpr int QM = NBP == 32 ? 3 : NBP == 16 ? 5 : 9;  // chunks of 128 columns
  constexpr int RW = NBP == 32 ? 4 : 1;
  extern __shared__ double lds[];
  __shared__ double redA[16], redB[16];
  __shared__ double s_y1[NBP], s_y2[NBP];
  const EigDesc dd = descs[blockIdx.x];
  const int k = dd.k;
  EigWork W(dd.work, k, dd.r);
  GAS double* A = W.H;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (j0 == 0) {  // the full symmetric copy (the lower triangle of H is read); zero reflectors
    const GAS double* Hin = gload_ptr(dd.H);
    for (int idx = threadIdx.x; idx < k * k; idx += kBig) {
      const int i = idx / k, j = idx % k;
      A[idx] = Hin[(long long)max(i, j) * dd.ldh + min(i, j)];
      W.V[idx] = 0.0;
    }
    __syncthreads();
    if (k <= 2) {
      if (threadIdx.x == 0) {
        W.d[0] = A[0];
        W.e[0] = 0.0;
        W.tau[0] = 0.0;
        if (k == 2) { W.d[1] = A[3]; W.e[0] = A[2]; W.e[1] = 0.0; W.tau[1] = 0.0; }
      }
      return;
    }
  }
  if (j0 >= k - 2) return;  // uniform: this problem's panels are done
  const int pend = min(j0 + NBP, k - 2), nbp = pend - j0;
  double* Vs = lds;                             // [NBP][k]
  double* Ws = lds + (long long)NBP * k;        // [NBP][k]
  double* sv = lds + 2 * (long long)NBP * k;    // k
  double* sp = sv + k;                          // k
  for (int cur = 0; cur < nbp; ++cur) {
    const int jj = j0 + cur;
    // column jj (rows >= jj) of A_cur: row jj of the panel-start matrix
    // (symmetric storage) minus the corrections
    double sq = 0.0;
    for (int r = jj + threadIdx.x; r < k; r += kBig) {
      // four independent partial sums so that the LDS reads overlap
      double c0 = A[(long long)jj * k + r], c1 = 0.0, c2 = 0.0, c3 = 0.0;
      int p = 0;
      for (; p + 4 <= cur; p += 4) {
        c0 -= Vs[p * k + r] * Ws[p * k + jj] + Ws[p * k + r] * Vs[p * k + jj];
        c1 -= Vs[(p + 1) * k + r] * Ws[(p + 1) * k + jj] + Ws[(p + 1) * k + r] * Vs[(p + 1) * k + jj];
        c2 -= Vs[(p + 2) * k + r] * Ws[(p + 2) * k + jj] + Ws[(p + 2) * k + r] * Vs[(p + 2) * k + jj];
        c3 -= Vs[(p + 3) * k + r] * Ws[(p + 3) * k + jj] + Ws[(p + 3) * k + r] * Vs[(p + 3) * k + jj];
      }
      for (; p < cur; ++p) c0 -= Vs[p * k + r] * Ws[p * k + jj] + Ws[p * k + r] * Vs[p * k + jj];
      const double c = (c0 + c1) + (c2 + c3);
      if (r == jj) W.d[jj] = c;
      else sv[r] = c;
      sq += r >= jj + 2 ? c * c : 0.0;
    }
    const double xnorm2 = block_sum1(sq, redA);
    const double alpha = sv[jj + 1];
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (xnorm2 > 0.0) {
      const double n2 = fma(alpha, alpha, xnorm2);
      const double rs = rsq_nr(n2), nrm = n2 * rs;
      const double sg = alpha < 0.0 ? -1.0 : 1.0;
      beta = -sg * nrm;
      tau = fma(fabs(alpha), rs, 1.0);
      scal = sg * rcp_nr(fabs(alpha) + nrm);
    }
    if (threadIdx.x == 0) {
      W.e[jj] = beta;
      W.tau[jj] = tau;
    }
    double* v = Vs + (long long)cur * k;
    for (int r = threadIdx.x; r < k; r += kBig) {
      const double x = r == jj + 1 ? 1.0 : (r > jj + 1 ? sv[r] * scal : 0.0);
      const double vr = tau != 0.0 ? x : 0.0;
      v[r] = vr;
      W.V[(long long)jj * k + r] = vr;
    }
    __syncthreads();
    if (tau == 0.0) {  // uniform: H_jj = I, nothing to correct with
      for (int r = threadIdx.x; r < k; r += kBig) Ws[(long long)cur * k + r] = 0.0;
      __syncthreads();
      continue;
    }
    // p = A_j0 v on rows > jj: a wave per row, RW rows at a time with every
    // chunk's load issued before the first product, so a row group costs one
    // L2 round trip.  A lane reads two adjacent columns (16 bytes; rows are
    // 16-byte aligned when k is even, else 8-byte loads), chunks of 128
    // columns from the even column c0 <= jj + 1 cover the row.
    const int c0 = (jj + 1) & ~1;
    double vq[QM][2];
#pragma unroll
    for (int q = 0; q < QM; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = c0 + 2 * lane + 128 * q + h;
        const double x = v[min(c, k - 1)];  // in-bounds read, masked: no branch per load
        vq[q][h] = (c > jj && c < k) ? x : 0.0;
      }
    const bool even = (k & 1) == 0;
    for (int r0 = jj + 1 + wave; r0 < k; r0 += RW * (kBig / 64)) {
      double x[RW][QM][2];
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        const int r = min(r0 + u * (kBig / 64), k - 1);
#pragma unroll
        for (int q = 0; q < QM; ++q) {  // clamped columns meet vq = 0
          const int c = c0 + 2 * lane + 128 * q;
          const GAS double* row = A + (long long)r * k;
          if (even) {  // c and k even: c < k implies c + 1 < k
            const doublex2 t2 = *reinterpret_cast<const GAS doublex2*>(row + min(c, k - 2));
            x[u][q][0] = t2[0];
            x[u][q][1] = t2[1];
          } else {
            x[u][q][0] = row[min(c, k - 1)];
            x[u][q][1] = row[min(c + 1, k - 1)];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < QM; ++q) acc = fma(x[u][q][1], vq[q][1], fma(x[u][q][0], vq[q][0], acc));
        const int r = r0 + u * (kBig / 64);
        const double sum = wave_sum(acc);
        if (lane == 0 && r < k) sp[r] = sum;
      }
    }
    // y1 = W^T v, y2 = V^T v over rows > jj (the correction's small factors)
    for (int p = wave; p < cur; p += kBig / 64) {
      double a1 = 0.0, a2 = 0.0;
#pragma unroll 4
      for (int r = jj + 1 + lane; r < k; r += 64) {
        const double vr = v[r];
        a1 = fma(Ws[p * k + r], vr, a1);
        a2 = fma(Vs[p * k + r], vr, a2);
      }
      a1 = wave_sum(a1);
      a2 = wave_sum(a2);
      if (lane == 0) { s_y1[p] = a1; s_y2[p] = a2; }
    }
    __syncthreads();
    // p = tau (A_j0 v - V y1 - W y2); w = p - (tau/2)(p.v) v
    double pvp = 0.0;
    for (int r = jj + 1 + threadIdx.x; r < k; r += kBig) {
      double p0 = sp[r], p1 = 0.0, p2 = 0.0, p3 = 0.0;
      int p = 0;
      for (; p + 4 <= cur; p += 4) {
        p0 -= Vs[p * k + r] * s_y1[p] + Ws[p * k + r] * s_y2[p];
        p1 -= Vs[(p + 1) * k + r] * s_y1[p + 1] + Ws[(p + 1) * k + r] * s_y2[p + 1];
        p2 -= Vs[(p + 2) * k + r] * s_y1[p + 2] + Ws[(p + 2) * k + r] * s_y2[p + 2];
        p3 -= Vs[(p + 3) * k + r] * s_y1[p + 3] + Ws[(p + 3) * k + r] * s_y2[p + 3];
      }
      for (; p < cur; ++p) p0 -= Vs[p * k + r] * s_y1[p] + Ws[p * k + r] * s_y2[p];
      double pr = (p0 + p1) + (p2 + p3);
      pr *= tau;
      sp[r] = pr;
      pvp = fma(pr, v[r], pvp);
    }
    const double K = -0.5 * tau * block_sum1(pvp, redB);
    for (int r = threadIdx.x; r < k; r += kBig)
      Ws[(long long)cur * k + r] = r > jj ? fma(K, v[r], sp[r]) : 0.0;
    __syncthreads();
  }
  // the panel as GEMM operands (zero columns past nbp)
  GAS double* P1 = gstore_ptr(eig_work_panel(dd.work, k, dd.r));
  GAS double* P2 = P1 + 2 * (long long)kPanel * k;
  for (int idx = threadIdx.x; idx < k * NBP; idx += kBig) {
    const int r = idx / NBP, p = idx % NBP;
    const double vv = p < nbp ? Vs[p * k + r] : 0.0, ww = p < nbp ? Ws[p * k + r] : 0.0;
    P1[(long long)r * 2 * NBP + p] = vv;
    P1[(long long)r * 2 * NBP + NBP + p] = ww;
    P2[(long long)r * 2 * NBP + p] = ww;
    P2[(long long)r * 2 * NBP + NBP + p] = vv;
  }
  if (pend == k - 2 && threadIdx.x == 0) {  // the trailing 2 x 2 block of the last panel
    auto at = [&](int r, int c) {
      double x = A[(long long)r * k + c];
      for (int p = 0; p < nbp; ++p) x -= Vs[p * k + r] * Ws[p * k + c] + Ws[p * k + r] * Vs[p * k + c];
      return x;
    };
    W.d[k - 2] = at(k - 2, k - 2);
    W.d[k - 1] = at(k - 1, k - 1);
    W.e[k - 2] = at(k - 1, k - 2);
    W.e[k - 1] = 0.0;
    W.tau[k - 2] = 0.0;
    W.tau[k - 1] = 0.0;
  }
}

// Number of eigenvalues of T strictly below x: the signs of the pivots q_i
// of the LDL^T factorization of T - x I, with LAPACK's pivmin guard.
// de[i] = (d_i, e_{i-1}^2) with e_{-1} = 0.  The guard keeps |q| >= pivmin =
// DBL_MIN max(1, max e^2), so e^2 / q cannot overflow; the quotient uses the
// refined reciprocal (a perturbation of e^2 by about an ulp, well inside the
// backward error of the recurrence).
__device__ __forceinline__ int sturm_count(const double2* de, int k, double x, double pivmin) {
  double q = de[0].x - x;
  q = fabs(q) < pivmin ? -pivmin : q;
  int cnt = q < 0.0 ? 1 : 0;
  for (int i = 1; i < k; ++i) {
    const double2 p = de[i];
    q = fma(-p.y, rcp_nr(q), p.x - x);
    q = fabs(q) < pivmin ? -pivmin : q;
    cnt += q < 0.0 ? 1 : 0;
  }
  return cnt;
}

constexpr int kBisect = 256;

// log2(WL + 1) bits per multisection round; the rounds give a bracket about
// 2^-96 of the Gerschgorin interval unless the relative criterion stops first.
constexpr int bisect_rounds(int WL) {
  return WL == 8 ? 31 : WL == 16 ? 24 : WL == 32 ? 20 : WL == 64 ? 16 : 12;
}

// Eigenvalue jj (0 = largest) of T by multisection: a group of WL lanes
// evaluates WL shifts spread over the current bracket and keeps the
// sub-bracket holding it.  WL = 256 is the whole workgroup (counts through a
// barrier), for few eigenvalues; WL <= 64 packs 256 / WL eigenvalues per
// workgroup, each group counting through a wave ballot with no barrier.
template <int WL>
__global__ void __launch_bounds__(kBisect) bisect_kernel(const EigDesc* __restrict__ descs) {
  extern __shared__ double2 lds_de[];  // 16-byte aligned pairs
  __shared__ double s_lo[4], s_hi[4], s_em[4];
  __shared__ double s_a, s_b;
  constexpr int PER = kBisect / WL;
  const EigDesc dd = descs[blockIdx.y];
  const int k = dd.k;
  if (blockIdx.x * PER >= dd.r) return;  // uniform
  EigWork W(dd.work, k, dd.r);
  double2* de = lds_de;
  double lo = DBL_MAX, hi = -DBL_MAX, emax2 = 0.0;
  for (int i = threadIdx.x; i < k; i += kBisect) {
    const double di = W.d[i];
    const double em = i > 0 ? fabs(W.e[i - 1]) : 0.0;
    const double ep = i + 1 < k ? fabs(W.e[i]) : 0.0;
    de[i] = make_double2(di, em * em);
    lo = fmin(lo, di - em - ep);
    hi = fmax(hi, di + em + ep);
    emax2 = fmax(emax2, ep * ep);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    emax2 = fmax(emax2, __shfl_xor(emax2, off));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { s_lo[wave] = lo; s_hi[wave] = hi; s_em[wave] = emax2; }
  __syncthreads();
  lo = fmin(fmin(s_lo[0], s_lo[1]), fmin(s_lo[2], s_lo[3]));
  hi = fmax(fmax(s_hi[0], s_hi[1]), fmax(s_hi[2], s_hi[3]));
  emax2 = fmax(fmax(s_em[0], s_em[1]), fmax(s_em[2], s_em[3]));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double span = fmax(hi - lo, DBL_MIN);
  double a = lo - 2.0 * DBL_EPSILON * span - pivmin;
  double b = hi + 2.0 * DBL_EPSILON * span + pivmin;
  const int g = threadIdx.x / WL, t = threadIdx.x % WL;
  const int jj = blockIdx.x * PER + g;
  const bool active = jj < dd.r;
  const int m = k - 1 - jj;  // ascending index
  if constexpr (WL == kBisect) {
    // With a positive upper bound the first round uses the points
    // hi 2^(t - WL + 1) (the lowest replaced by 0 when lo < 0): the bracket
    // then holds the eigenvalue to a factor of 2 whatever its size, and the
    // uniform rounds after it gain relative accuracy at the same rate for
    // small eigenvalues as for large ones.
    const bool geo = hi > 0.0;
    auto gpt = [&](int u) { return (u == 0 && lo < 0.0) ? 0.0 : ldexp(hi, u - (WL - 1)); };
    for (int round = 0; round < bisect_rounds(WL); ++round) {
      const bool g0 = geo && round == 0;
      const double x = g0 ? gpt(t) : a + (b - a) * (double)(t + 1) / (double)(WL + 1);
      const int c = sturm_count(de, k, x, pivmin);
      const int below = __syncthreads_count(c <= m);
      if (threadIdx.x == 0) {
        double na = a, nb = b;
        if (g0) {
          if (below > 0) na = fmax(a, gpt(below - 1));
          if (below < WL) nb = fmin(b, gpt(below));
        } else {
          if (below > 0) na = a + (b - a) * (double)below / (double)(WL + 1);
          if (below < WL) nb = a + (b - a) * (double)(below + 1) / (double)(WL + 1);
        }
        s_a = na;
        s_b = nb;
      }
      __syncthreads();
      a = s_a;
      b = s_b;
      if (b - a <= 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + pivmin) break;
    }
  } else {
    const int sh = (lane / WL) * WL;  // the group's first lane in the wave
    const unsigned long long gmask = WL == 64 ? ~0ull : ((1ull << (WL & 63)) - 1ull);
    for (int round = 0; round < bisect_rounds(WL); ++round) {
      const bool done = !active || b - a <= 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + pivmin;
      if (__ballot(!done) == 0ull) break;  // wave-uniform
      const double x = a + (b - a) * (double)(t + 1) / (double)(WL + 1);
      const int c = done ? 0 : sturm_count(de, k, x, pivmin);
      const unsigned long long bal = __ballot(c <= m);
      const int below = __popcll((bal >> sh) & gmask);
      if (!done) {
        double na = a, nb = b;
        if (below > 0) na = a + (b - a) * (double)below / (double)(WL + 1);
        if (below < WL) nb = a + (b - a) * (double)(below + 1) / (double)(WL + 1);
        a = na;
        b = nb;
      }
    }
  }
  if (active && t == 0) dd.evals[jj] = 0.5 * (a + b);
}

// Eigenvector of T for eigenvalue evals[j] from the twisted factorization
// T - lambda I = N_g Delta_g N_g^T at the twist index g minimizing |gamma_g|
// (Dhillon-Parlett): z_g = 1, z_i = -(e_i / D+_i) z_{i+1} above g and
// z_{i+1} = -(e_i / D-_{i+1}) z_i below g.  One thread per eigenvalue; the
// D+ and D- sequences are kept in LDS (interleaved by thread).
__global__ void twisted_kernel(const EigDesc* __restrict__ descs) {
  extern __shared__ double lds[];
  const EigDesc dd = descs[blockIdx.y];
  const int k = dd.k;
  const int T = blockDim.x;
  EigWork W(dd.work, k, dd.r);
  double* sd = lds;                          // k
  double* se = lds + k;                      // k
  double* Dp = lds + 2 * k;                  // [i*T + tid]
  double* Dm = Dp + (long long)k * T;
  for (int i = threadIdx.x; i < k; i += T) {
    sd[i] = W.d[i];
    se[i] = i + 1 < k ? W.e[i] : 0.0;
  }
  __syncthreads();
  const int j = blockIdx.x * T + threadIdx.x;
  if (j >= dd.r) return;
  const int tid = threadIdx.x;
  const double lam = dd.evals[j];
  double emax2 = 0.0;
  for (int i = 0; i + 1 < k; ++i) emax2 = fmax(emax2, se[i] * se[i]);
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  // |q| >= pivmin after the guard, so the quotients below cannot overflow;
  // they use the refined reciprocal (about an ulp of e^2 / q)
  auto guard = [pivmin](double q) { return fabs(q) < pivmin ? (q < 0 ? -pivmin : pivmin) : q; };
  // bottom-up D-
  double q = guard(sd[k - 1] - lam);
  Dm[(long long)(k - 1) * T + tid] = q;
  for (int i = k - 2; i >= 0; --i) {
    const double ei = se[i];
    q = guard(fma(-ei * ei, rcp_nr(q), sd[i] - lam));
    Dm[(long long)i * T + tid] = q;
  }
  // top-down D+ and the twist gamma_i = (d_i - lam) - e_{i-1}^2/D+_{i-1} - e_i^2/D-_{i+1}
  double best = DBL_MAX;
  int g = 0;
  double p = 1.0;
  for (int i = 0; i < k; ++i) {
    const double di = sd[i] - lam;
    const double em2 = i > 0 ? se[i - 1] * se[i - 1] : 0.0;
    const double top = (i == 0) ? di : fma(-em2, rcp_nr(p), di);
    const double gam = i + 1 < k ? fma(-se[i] * se[i], rcp_nr(Dm[(long long)(i + 1) * T + tid]), top) : top;
    p = guard(top);
    Dp[(long long)i * T + tid] = p;
    if (fabs(gam) < best) { best = fabs(gam); g = i; }
  }
  // vector, written over D+ (above g) and D- (below g)
  double nrm2 = 1.0;
  double z = 1.0;
  for (int i = g - 1; i >= 0; --i) {
    z = -(se[i] * rcp_nr(Dp[(long long)i * T + tid])) * z;
    Dp[(long long)i * T + tid] = z;
    nrm2 += z * z;
  }
  z = 1.0;
  for (int i = g + 1; i < k; ++i) {
    z = -(se[i - 1] * rcp_nr(Dm[(long long)i * T + tid])) * z;
    Dm[(long long)i * T + tid] = z;
    nrm2 += z * z;
  }
  const double inv = rsq_nr(nrm2);
  for (int i = 0; i < k; ++i) {
    const double zi = (i < g) ? Dp[(long long)i * T + tid] : (i == g ? 1.0 : Dm[(long long)i * T + tid]);
    W.X[(long long)i * dd.r + j] = zi * inv;
  }
}

// The same eigenvector as twisted_kernel, one wave per eigenvalue.  Lane 0
// runs the bottom-up D- recurrence while lane 1 runs the top-down D+ one
// (the same instructions on mirrored indices); all lanes then form the twist
// values gamma_i and their first minimum.  Each side of the twist is a
// product of ratios (z_i = prod_{l=i}^{g-1} f_l above g, prod_{l=g+1}^{i} f_l
// below), taken as a prefix / suffix product scan over the wave: lane l owns
// the rows [l C, l C + C), C = ceil(k / 64), and partial products are kept as
// mantissa / exponent pairs so that no intermediate can overflow or underflow
// before the final scaling.  LDS: 6 k doubles.
struct MantExp {
  double m;
  int e;
};
__device__ __forceinline__ MantExp me_mul(MantExp a, MantExp b) {
  int x;
  const double m = frexp(a.m * b.m, &x);
  return MantExp{m, a.e + b.e + x};
}
__device__ __forceinline__ MantExp me_of(double v) {
  int x;
  const double m = frexp(v, &x);
  return MantExp{m, x};
}

__global__ void __launch_bounds__(64) twisted_wave_kernel(const EigDesc* __restrict__ descs) {
  extern __shared__ double lds[];
  const EigDesc dd = descs[blockIdx.y];
  const int k = dd.k, j = blockIdx.x;
  if (j >= dd.r) return;  // uniform
  EigWork W(dd.work, k, dd.r);
  double* sd = lds;          // d_i - lambda
  double* se = lds + k;      // e_i, e_{k-1} = 0
  double* Dm = lds + 2 * k;  // D-_i
  double* Dp = lds + 3 * k;  // D+_i
  double* tf = lds + 4 * k;  // D+_i before the guard, then the ratios f_i (2 k)
  const int lane = threadIdx.x;
  const double lam = dd.evals[j];
  double emax2 = 0.0;
  for (int i = lane; i < k; i += 64) {
    sd[i] = W.d[i] - lam;
    const double ei = i + 1 < k ? W.e[i] : 0.0;
    se[i] = ei;
    emax2 = fmax(emax2, ei * ei);
  }
  for (int off = 32; off > 0; off >>= 1) emax2 = fmax(emax2, __shfl_xor(emax2, off));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  auto guard = [pivmin](double q) { return fabs(q) < pivmin ? (q < 0 ? -pivmin : pivmin) : q; };
  __syncthreads();
  if (lane < 2) {
    // step t works on row i(t) = t (lane 1, D+) or k - 1 - t (lane 0, D-),
    // with the off-diagonal entry e_{i-1} or e_i; both are read two steps
    // ahead, before the stores of the steps in between
    const bool down = lane == 1;
    double* dst = down ? Dp : Dm;
    double* tops = down ? tf : tf + k;  // lane 0 stores its tops past tf (unused)
    auto row = [&](int t) { return down ? t : k - 1 - t; };
    auto ecol = [&](int t) { return se[down ? max(t - 1, 0) : k - 1 - t]; };
    double d0 = sd[row(0)], c0 = 0.0;
    double d1 = k > 1 ? sd[row(1)] : 0.0, c1 = k > 1 ? ecol(1) : 0.0;
    double q = 1.0;
    for (int t = 0; t < k; ++t) {
      const double di = d0, ci = c0;
      d0 = d1;
      c0 = c1;
      if (t + 2 < k) {
        d1 = sd[row(t + 2)];
        c1 = ecol(t + 2);
      }
      const double top = t == 0 ? di : fma(-ci * ci, rcp_nr(q), di);
      const double gq = top < 0.0 ? -pivmin : pivmin;
      q = fabs(top) < pivmin ? gq : top;
      const int i = row(t);
      dst[i] = q;
      tops[i] = top;
    }
  }
  __syncthreads();
  // twist: first i minimizing |gamma_i|, gamma_i = top_i - e_i^2 / D-_{i+1}
  double best = DBL_MAX;
  int g = 0;
  for (int i = lane; i < k; i += 64) {
    const double top = tf[i];
    const double gam = i + 1 < k ? fma(-se[i] * se[i], rcp_nr(Dm[i + 1]), top) : top;
    if (fabs(gam) < best) { best = fabs(gam); g = i; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int og = __shfl_xor(g, off);
    if (ob < best || (ob == best && og < g)) { best = ob; g = og; }
  }
  __syncthreads();  // every lane has read tf
  // ratios: f_i = -e_i / D+_i above the twist, -e_{i-1} / D-_i below it
  const int C = (k + 63) / 64;
  const int i0 = min(lane * C, k), i1 = min(i0 + C, k);
  MantExp pf{0.5, 1}, pu{0.5, 1};  // chunk products below / above the twist (1 = 0.5 * 2^1)
  for (int i = i0; i < i1; ++i) {
    double f = 1.0;
    if (i < g) f = -(se[i] * rcp_nr(Dp[i]));
    else if (i > g) f = -(se[i - 1] * rcp_nr(Dm[i]));
    tf[i] = f;
    if (i > g) pf = me_mul(pf, me_of(f));
    if (i < g) pu = me_mul(pu, me_of(f));
  }
  // exclusive prefix product of pf over lower lanes, suffix product of pu over higher ones
  MantExp xf = pf, xu = pu;
  for (int off = 1; off < 64; off <<= 1) {
    const double fm = __shfl_up(xf.m, off);
    const int fe = __shfl_up(xf.e, off);
    const double um = __shfl_down(xu.m, off);
    const int ue = __shfl_down(xu.e, off);
    if (lane >= off) xf = me_mul(xf, MantExp{fm, fe});
    if (lane + off < 64) xu = me_mul(xu, MantExp{um, ue});
  }
  MantExp ef{__shfl_up(xf.m, 1), __shfl_up(xf.e, 1)};
  MantExp eu{__shfl_down(xu.m, 1), __shfl_down(xu.e, 1)};
  if (lane == 0) ef = MantExp{0.5, 1};
  if (lane == 63) eu = MantExp{0.5, 1};
  double nrm2 = 0.0;
  for (int i = i0; i < i1; ++i) {  // below the twist and the twist itself, ascending
    if (i > g) ef = me_mul(ef, me_of(tf[i]));
    if (i >= g) {
      const double z = i == g ? 1.0 : ldexp(ef.m, ef.e);
      Dm[i] = z;
      nrm2 = fma(z, z, nrm2);
    }
  }
  for (int i = i1 - 1; i >= i0; --i) {  // above the twist, descending
    if (i < g) {
      eu = me_mul(eu, me_of(tf[i]));
      const double z = ldexp(eu.m, eu.e);
      Dm[i] = z;
      nrm2 = fma(z, z, nrm2);
    }
  }
  for (int off = 32; off > 0; off >>= 1) nrm2 += __shfl_xor(nrm2, off);
  const double inv = rsq_nr(nrm2);
  for (int i = i0; i < i1; ++i) W.X[(long long)i * dd.r + j] = Dm[i] * inv;
}

// Z[:, cols] = H_0 H_1 ... H_{k-3} X[:, cols] for one block of columns.
__global__ void __launch_bounds__(kBig) backtransform_kernel(const EigDesc* __restrict__ descs,
                                                             int rb) {
  extern __shared__ double lds[];
  const EigDesc dd = descs[blockIdx.y];
  const int k = dd.k, r = dd.r;
  const int c0 = blockIdx.x * rb;
  if (c0 >= r) return;
  const int nc = min(rb, r - c0);
  EigWork W(dd.work, k, r);
  double* Xs = lds;                        // k * nc
  double* sv = lds + (long long)k * nc;    // k
  double* sw = sv + k;                     // nc
  double* part = sw + nc;                  // P * nc <= kBig
  for (int idx = threadIdx.x; idx < k * nc; idx += kBig) {
    const int i = idx / nc, c = idx % nc;
    Xs[idx] = W.X[(long long)i * r + c0 + c];
  }
  const int P = kBig / nc;  // row partitions of the dot products
  for (int j = k - 3; j >= 0; --j) {
    const double tau = W.tau[j];
    if (tau == 0.0) continue;  // uniform
    const int t = k - j - 1;
    __syncthreads();
    for (int i = threadIdx.x; i < t; i += kBig) sv[i] = W.V[(long long)j * k + j + 1 + i];
    __syncthreads();
    if (threadIdx.x < P * nc) {
      const int c = threadIdx.x % nc, pp = threadIdx.x / nc;
      double acc = 0.0;
      for (int i = pp; i < t; i += P) acc += sv[i] * Xs[(long long)(j + 1 + i) * nc + c];
      part[pp * nc + c] = acc;
    }
    __syncthreads();
    if (threadIdx.x < nc) {
      double s = 0.0;
      for (int pp = 0; pp < P; ++pp) s += part[pp * nc + threadIdx.x];
      sw[threadIdx.x] = tau * s;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < t * nc; idx += kBig) {
      const int i = idx / nc, c = idx % nc;
      Xs[(long long)(j + 1 + i) * nc + c] -= sv[i] * sw[c];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < k * nc; idx += kBig) {
    const int i = idx / nc, c = idx % nc;
    dd.Z[(long long)i * dd.ldz + c0 + c] = Xs[idx];
  }
}


// ---------------------------------------------------------------- register-resident variants
// For k <= G*NB the k x k matrix lives in registers: thread (tr, tc) of a
// G x G grid (tid = G tr + tc) holds rows tr + G a and columns tc + G b,
// a, b < NB.  A thread row is one 16-lane DPP row (G = 16) or half a wave
// (G = 32), so reductions along a row stay inside the wave; column data is
// broadcast through LDS.  Every wave repeats the per-step vector work, so
// the launches use G = 16 (one wave per SIMD, up to 256 VGPRs a lane; the
// largest instances park some values in AGPRs).

// f(integral_constant<int, I>) for I = B .. E-1: compile-time register-block
// indices without relying on the unroller's size limits.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// G = L L^T (Cholesky, L lower) and R^{-1} = (L^{-1})^T written row-major
// (upper triangular, zeros below), as a right-looking blocked Cholesky with
// block size G on the register layout (thread (tr, tc) holds A(tr + G i,
// tc + G j)), X = L^{-1} overwriting L in place.  Step jj of block JB
// publishes column jj (below the diagonal, the pivot apart) through one
// barrier and updates only block column JB (the panel: A(r, c) -= L(r, jj)
// L(c, jj), c in the block); the owner of column jj keeps 1 / L(jj, jj).
// At the end of the block:
//   - L of the diagonal block and its inverse Linv (forward substitution of
//     each unit column),
//   - block row JB of X: X_J,<J = Linv S_J with S_J the partial sums left by
//     the earlier blocks, and X_JJ = Linv,
//   - with L(r, c) of the later rows (PT) and that block row (XB) in LDS, the
//     rank-G updates of the later rows:
//       A(r, c) -= sum_m L(r, m) L(c, m)        r, c in later blocks (r >= c)
//       X(r, c) -= sum_m L(r, m) X(m, c)        c < G JB
//       X(r, c)  = -sum_m L(r, m) X(m, c)       c in block JB
//     (m over the block's columns, X(m, c) = 0 for m < c),
// so a step carries about NB multiply-adds and NB + 2 LDS reads per thread.
template <int NB, int G>
__global__ void __launch_bounds__(G * G) chol_inv_reg_kernel(const CholDesc* __restrict__ descs) {
  __shared__ double colb[2][G * NB];
  __shared__ double dgb[2];
  __shared__ double PT[G][G * NB];  // PT[m][r] = L(r, G JB + m), rows of later blocks
  __shared__ double XB[G][G * NB];  // partial block row S_J, then X(G JB + m, c), c < G (JB + 1)
  __shared__ double LJ[G][G + 1];   // L of the diagonal block
  __shared__ double LI[G][G];       // its inverse
  __shared__ double invsJ[G];       // 1 / L(m, m) of the block
  __shared__ double gdiag[G * NB];  // diagonal of G as loaded (rank-revealing reference)
  const CholDesc d = descs[blockIdx.x];
  const int k = d.k;
  const int tr = threadIdx.x / G, tc = threadIdx.x % G;
  double a[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int r = tr + G * i, c = tc + G * j;
      a[i][j] = (r < k && c < k) ? gload_ptr(d.G)[(long long)r * d.ldg + c] : (r == c ? 1.0 : 0.0);
      if (i == j && tr == tc) {  // the diagonal: a masked column counts as a unit one
        if (r < k && d.keep && gload_ptr(d.keep)[r] == 0.0) a[i][j] += 1.0;
        gdiag[r] = a[i][j];  // read back only by this thread
      }
    }
  const double eta = d.eta;
  bool bad = false;
  double own_invs = 0.0;  // 1 / L(c, c) of this lane's column c = tc + G JB
  static_for<0, NB>([&](auto jb_) {
    constexpr int JB = decltype(jb_)::value;
    const int jend = min(k, G * JB + G);
    if (G * JB >= k) return;  // uniform
    for (int jj = G * JB; jj < jend; ++jj) {
      const int jt = jj % G, buf = jj & 1;
      if (tc == jt) {  // column jj below the diagonal; the diagonal apart
#pragma unroll
        for (int i = JB; i < NB; ++i) colb[buf][tr + G * i] = (tr + G * i > jj) ? a[i][JB] : 0.0;
        if (tr == jt) {
          const double v = a[JB][JB];
          // rank-revealing: a column in the span of the previous ones
          dgb[buf] = (eta > 0.0 && v <= eta * gdiag[jj]) ? 0.0 : v;
        }
      }
      __syncthreads();
      // every broadcast value is read before the pivot is used
      const double djj = dgb[buf];
      const double cc = colb[buf][tc + G * JB];  // zero unless tc + G JB > jj
      double av[NB];
#pragma unroll
      for (int i = JB; i < NB; ++i) av[i] = colb[buf][tr + G * i];
      const bool ok = djj > 0.0 && djj < INFINITY;
      if (!ok && !(eta > 0.0 && djj == 0.0)) bad = true;
      const double rs = rsq_nr(djj);
      const double invs = ok ? rs : 0.0;  // 1 / L(jj, jj)
      const double lc = cc * invs;        // L(c, jj)
#pragma unroll
      for (int i = JB; i < NB; ++i) a[i][JB] -= (av[i] * invs) * lc;  // the panel
      // column jj stays as it is from here on: its owner keeps 1 / L(jj, jj)
      // and forms L(r, jj) at the end of the block
      own_invs = tc == jt ? invs : own_invs;
    }
    // the diagonal block's L and, by forward substitution of each unit
    // column (lanes of row group 0), its inverse
    const int mv = jend - G * JB;
    LJ[tr][tc] = (tr >= tc) ? a[JB][JB] * own_invs : 0.0;
    if (tr == 0) invsJ[tc] = own_invs;
    __syncthreads();
    if (tr == 0) {
      double rhs[G];
#pragma unroll
      for (int m = 0; m < G; ++m) rhs[m] = (m == tc) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < G; ++t) {
        const double x = (t < mv) ? rhs[t] * invsJ[t] : 0.0;
        LI[t][tc] = x;
#pragma unroll
        for (int m = t + 1; m < G; ++m) rhs[m] = fma(-LJ[m][t], x, rhs[m]);
      }
    }
    if constexpr (JB > 0) {
#pragma unroll
      for (int j = 0; j < JB; ++j) XB[tr][tc + G * j] = a[JB][j];  // S_J
    }
    __syncthreads();
    // block row JB of X: X_J,<J = Linv S_J, X_JJ = Linv
    if constexpr (JB > 0) {
      double sx[JB];
#pragma unroll
      for (int j = 0; j < JB; ++j) sx[j] = 0.0;
#pragma unroll 2
      for (int m = 0; m < G; ++m) {
        const double lim = LI[tr][m];
#pragma unroll
        for (int j = 0; j < JB; ++j) sx[j] = fma(lim, XB[m][tc + G * j], sx[j]);
      }
#pragma unroll
      for (int j = 0; j < JB; ++j) a[JB][j] = sx[j];
    }
    const double li = LI[tr][tc];
    if (G * JB + G < k) __syncthreads();  // uniform: S_J read before XB is rewritten
    a[JB][JB] = (tr >= tc) ? li : 0.0;
    if (G * JB + G < k) {  // uniform: a later block holds rows of the matrix
#pragma unroll
      for (int i = JB + 1; i < NB; ++i) PT[tc][tr + G * i] = a[i][JB] * own_invs;
#pragma unroll
      for (int j = 0; j <= JB; ++j) XB[tr][tc + G * j] = (tc + G * j <= G * JB + tr) ? a[JB][j] : 0.0;
      __syncthreads();
      double acc[NB];
#pragma unroll
      for (int i = JB + 1; i < NB; ++i) acc[i] = 0.0;
      for (int m = 0; m < G; ++m) {
        double p[NB], q[NB], x[JB + 1];
#pragma unroll
        for (int i = JB + 1; i < NB; ++i) p[i] = PT[m][tr + G * i];
#pragma unroll
        for (int j = JB + 1; j < NB; ++j) q[j] = PT[m][tc + G * j];
#pragma unroll
        for (int j = 0; j <= JB; ++j) x[j] = XB[m][tc + G * j];
#pragma unroll
        for (int i = JB + 1; i < NB; ++i) {
#pragma unroll
          for (int j = JB + 1; j <= i; ++j) a[i][j] = fma(-p[i], q[j], a[i][j]);
#pragma unroll
          for (int j = 0; j < JB; ++j) a[i][j] = fma(-p[i], x[j], a[i][j]);
          acc[i] = fma(p[i], x[JB], acc[i]);
        }
      }
#pragma unroll
      for (int i = JB + 1; i < NB; ++i) a[i][JB] = -acc[i];
    }
  });
  if (bad && d.flag) atomicOr(d.flag, FLAG_CHOL);
  // R^{-1}(c, r) = X(r, c) for r >= c; zeros below the diagonal of R^{-1}
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int r = tr + G * i, c = tc + G * j;
      if (r < k && c < k) gstore_ptr(d.R)[(long long)c * d.ldr + r] = (r >= c) ? a[i][j] : 0.0;
    }
}

// Householder tridiagonalization (same reflector convention as sytrd_kernel)
// on the register-resident matrix; reflectors go to W.H (row j = v_j), tau
// to W.tau, d and e to W.d, W.e; z_rows_kernel applies them to the
// eigenvectors of the tridiagonal matrix.
template <int NB, int G>
__global__ void __launch_bounds__(G * G) sytrd_reg_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double vb[2][G * NB], wb[2][G * NB];
  const EigDesc dd = descs[blockIdx.x];
  const int k = dd.k;
  EigWork W(dd.work, k, dd.r);
  GAS double* vstore = W.H;
  const int tr = threadIdx.x / G, tc = threadIdx.x % G;
  double a[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int r = tr + G * i, c = tc + G * j;
      const int hi = r > c ? r : c, lo = r > c ? c : r;
      a[i][j] = (r < k && c < k) ? gload_ptr(dd.H)[(long long)hi * dd.ldh + lo] : 0.0;
    }
  // Step jj works on the trailing block (rows and columns > jj), which lies
  // in register blocks >= JB = jj / G; the JB loop is unrolled so register
  // indices are constants.  vb / wb alternate between two buffers so that a
  // step's last reads and the next step's first writes need no barrier.
  static_for<0, NB>([&](auto jb_) {
    constexpr int JB = decltype(jb_)::value;
    const int jend = min(k - 2, G * JB + G);
    for (int jj = G * JB; jj < jend; ++jj) {
      const int jt = jj % G, buf = jj & 1;
      double* v = vb[buf];
      double* w = wb[buf];
      if (tc == jt) {  // x = A(jj+1:, jj) into v; the diagonal entry to d
#pragma unroll
        for (int i = JB; i < NB; ++i) {
          const int r = tr + G * i;
          v[r] = (r > jj && r < k) ? a[i][JB] : 0.0;
        }
        if (tr == jt) W.d[jj] = a[JB][JB];
      }
      if (tc == 0 && JB > 0) {  // rows of earlier blocks stay zero in v and w
#pragma unroll
        for (int i = 0; i < JB; ++i) { v[tr + G * i] = 0.0; w[tr + G * i] = 0.0; }
      }
      __syncthreads();
      // v now holds x on rows jj+1 .. k-1 and zeros elsewhere.  Every wave
      // forms the reflector parameters from it (identical arithmetic, so
      // identical values), which saves a barrier.  LDS reads are issued
      // unconditionally (indices stay inside the buffer) and masked by selects.
      constexpr int QN = (G * NB + 63) / 64;
      const int lane = threadIdx.x & 63;
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const int r = lane + 64 * q;
        const double x = v[r < G * NB ? r : 0];
        part += (r < G * NB && r != jj + 1) ? x * x : 0.0;
      }
      part = wave_sum(part);
      const double alpha = v[jj + 1];
      // beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta = 1 + |alpha| / ||x||,
      // v = x / (alpha - beta) with v(jj+1) = 1
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (part > 0.0) {
        const double n2 = fma(alpha, alpha, part);
        const double rs = rsq_nr(n2), nrm = n2 * rs;
        const double sg = alpha < 0.0 ? -1.0 : 1.0;
        beta = -sg * nrm;
        tau = fma(fabs(alpha), rs, 1.0);
        scal = sg * rcp_nr(fabs(alpha) + nrm);
      }
      // the reflector (v(jj+1) = 1) and tau for the formation of Q^T
      if ((int)threadIdx.x < k) {
        const int t = threadIdx.x;
        const double x = v[t] * scal;
        vstore[(long long)jj * k + t] = tau != 0.0 ? (t == jj + 1 ? 1.0 : x) : 0.0;
      }
      if (threadIdx.x == 0) {
        W.e[jj] = beta;
        W.tau[jj] = tau;
      }
      if (tau == 0.0) continue;  // uniform
      // p = tau * A22 v on rows > jj (v vanishes on rows and columns <= jj)
      double vc[NB], pr[NB];
#pragma unroll
      for (int j = JB; j < NB; ++j) {
        const int c = tc + G * j;
        const double x = v[c] * scal;
        vc[j] = c == jj + 1 ? 1.0 : x;
      }
#pragma unroll
      for (int i = JB; i < NB; ++i) {
        pr[i] = 0.0;
#pragma unroll
        for (int j = JB; j < NB; ++j) pr[i] = fma(a[i][j], vc[j], pr[i]);
      }
      row_reduce_all<G, JB>(pr);
      if (tc == 0) {
#pragma unroll
        for (int i = JB; i < NB; ++i) w[tr + G * i] = (tr + G * i > jj) ? tau * pr[i] : 0.0;
      }
      __syncthreads();
      // w = p - (tau/2)(p.v) v: every thread forms p.v from the trailing rows
      double pv = 0.0;
#pragma unroll
      for (int i = JB; i < NB; ++i) pv = fma(w[tc + G * i], vc[i], pv);
      pv = row_reduce<G>(pv);
      const double K = -0.5 * tau * pv;
      // A22 -= v w^T + w v^T with w = p + K v (trailing block only)
      double wc[NB];
#pragma unroll
      for (int j = JB; j < NB; ++j) wc[j] = fma(K, vc[j], w[tc + G * j]);
      // v and w on this thread's rows: lane tc of a 16-lane row reads row
      // tr + G (JB + tc) once and the row shares it by DPP broadcast, instead
      // of every lane reading every row from LDS
      const int rd = tr + G * (JB + min(tc, NB - 1 - JB));
      const double vd = v[rd], wd = w[rd];
      static_for<JB, NB>([&](auto i_) {
        constexpr int i = decltype(i_)::value;
        const int r = tr + G * i;
        const double x = dpp_d<0x150 + (i - JB)>(vd) * scal;  // row_newbcast
        const double vi = r == jj + 1 ? 1.0 : x;
        const double wi = fma(K, vi, dpp_d<0x150 + (i - JB)>(wd));
#pragma unroll
        for (int j = JB; j < NB; ++j) a[i][j] -= vi * wc[j] + wi * vc[j];
      });
    }
  });
  if (k >= 2) {
    const int r0 = k - 2, r1 = k - 1;
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int r = tr + G * i, c = tc + G * j;
        if (r == r0 && c == r0) W.d[r0] = a[i][j];
        if (r == r1 && c == r1) W.d[r1] = a[i][j];
        if (r == r1 && c == r0) W.e[r0] = a[i][j];
      }
    if (threadIdx.x == 0) { W.tau[k - 2] = 0.0; W.e[k - 1] = 0.0; W.tau[k - 1] = 0.0; }
  } else {
    if (threadIdx.x == 0) { W.d[0] = a[0][0]; W.e[0] = 0.0; W.tau[0] = 0.0; }
  }
}

// Z = Q X (register path) as Z^T = X^T Q^T = X^T H_{k-3} ... H_0, row by
// row: the rows of M <- M H_j = M - tau_j (M v_j) v_j^T are independent, so a
// one-wave workgroup takes 4 rows of X^T (eigenvectors 4 blockIdx.x + tr of
// the tridiagonal matrix; lane (tr, tc) holds entries tc + 16 b, b < NB) and
// applies every reflector without a barrier after the taus are staged in
// LDS, then writes its rows as columns of Z.  One wave per workgroup spreads
// the rows over many CUs: the four rows of a wave read the same reflector
// entries, so the vector-memory issue rate per CU, not the data volume,
// bounds the loads.  The reflectors (rows of W.H) are read from L2 four at a
// time into two alternating register sets, the next four in flight while the
// current ones are applied; the row products are DPP reductions over the 16
// lanes of a row.  A column c >= k reads column 0 of the same reflector
// instead, which is zero (v_j vanishes on rows <= j), so the loads need no
// mask.
template <int NB>
__global__ void __launch_bounds__(64) z_rows_kernel(const EigDesc* __restrict__ descs) {
  constexpr int D = 4;
  const EigDesc dd = descs[blockIdx.y];
  const int k = dd.k;
  if (4 * (int)blockIdx.x >= dd.r) return;  // uniform
  EigWork W(dd.work, k, dd.r);
  __shared__ double s_tau[16 * NB];
  for (int t = threadIdx.x; t < k; t += 64) s_tau[t] = W.tau[t];
  __syncthreads();
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  const int r = 4 * blockIdx.x + tr;  // eigenvector (row of X^T)
  const bool live = r < dd.r;
  double m[NB];
  unsigned off[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c = tc + 16 * b;
    m[b] = (live && c < k) ? W.X[(long long)c * dd.r + r] : 0.0;
    off[b] = c < k ? 8u * (unsigned)c : 0u;  // byte offsets
  }
  // reflectors j0, j0 - 1, ..., j0 - D + 1; one with j < 0 reads reflector
  // 0 (written whenever the loop runs, k >= 3) and gets tau = 0, so that the
  // loads stay unconditional and in flight together.  Buffer loads: the row
  // offset is a scalar operand, the column offsets stay fixed per thread.
  const __amdgpu_buffer_rsrc_t hres =
      __builtin_amdgcn_make_buffer_rsrc((void*)W.H, (short)0, 8 * k * k, 0x00020000);
  auto load = [&](int j0, double (&v)[D][NB], double (&t)[D]) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int j = max(j0 - u, 0);
      const int so = __builtin_amdgcn_readfirstlane(8 * j * k);  // uniform
#pragma unroll
      for (int b = 0; b < NB; ++b)
        v[u][b] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(hres, off[b], so, 0));
      const double tj = s_tau[j];
      t[u] = j0 - u >= 0 ? tj : 0.0;
    }
  };
  auto apply = [&](const double (&v)[D][NB], const double (&t)[D]) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      double p0 = 0.0, p1 = 0.0;  // two chains for latency
#pragma unroll
      for (int b = 0; b < NB; b += 2) p0 = fma(m[b], v[u][b], p0);
#pragma unroll
      for (int b = 1; b < NB; b += 2) p1 = fma(m[b], v[u][b], p1);
      const double s = t[u] * row_reduce<16>(p0 + p1);
#pragma unroll
      for (int b = 0; b < NB; ++b) m[b] = fma(-s, v[u][b], m[b]);
    }
  };
  double va[D][NB], ta[D], vb[D][NB], tb[D];
  if (k >= 3) load(k - 3, va, ta);
  for (int j0 = k - 3; j0 >= 0; j0 -= 2 * D) {
    load(j0 - D, vb, tb);
    apply(va, ta);
    load(j0 - 2 * D, va, ta);
    apply(vb, tb);  // all taus zero once j0 - D < 0
  }
  if (live) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int c = tc + 16 * b;
      if (c < k) gstore_ptr(dd.Z)[(long long)c * dd.ldz + r] = m[b];
    }
  }
}

// ---------------------------------------------------------------- one-sided Jacobi SVD

// Round-robin pairing of qq (even) columns: player qq-1 stays, the others
// rotate; round t pairs (qq-1, t) and (t+k, t-k) mod (qq-1), k = 1 .. qq/2-1.
__device__ __forceinline__ void rr_pair(int t, int k, int qq, int& i, int& j) {
  if (k == 0) { i = qq - 1; j = t; return; }
  i = (t + k) % (qq - 1);
  j = (t - k + (qq - 1)) % (qq - 1);
}

__global__ void __launch_bounds__(kBig) jacobi_kernel(const JacobiDesc* __restrict__ descs, int in_lds) {
  extern __shared__ double lds[];
  __shared__ double s_n[512];
  __shared__ int s_rot;
  const JacobiDesc d = descs[blockIdx.x];
  const int q = d.q, qq = q + (q & 1);
  double* M = in_lds ? lds : d.work;  // column-major: column c at M + c q
  for (int idx = threadIdx.x; idx < q * q; idx += kBig) {
    const int r = idx % q, c = idx / q;
    M[idx] = d.R[(long long)r * d.ldr + c];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int kWaves = kBig / 64;
  // ||W||_F^2, which the rotations keep.  A column whose squared norm is
  // below 1e-40 of it carries singular values under 1e-20 ||W||, far below
  // the truncation, and is not rotated: its products underflow, and against
  // a large column the rotation angle's z^2 overflows, so the relative test
  // below would never settle on it; a rotation with a large column would
  // change that column by less than 1e-20 of its norm
  double fro = 0.0;
  for (int idx = threadIdx.x; idx < q * q; idx += kBig) fro = fma(M[idx], M[idx], fro);
  fro = wave_sum(fro);
  if (lane == 0) s_n[wave] = fro;
  __syncthreads();
  fro = 0.0;
  for (int w = 0; w < kWaves; ++w) fro += s_n[w];
  const double floor2 = 1e-40 * fro;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) s_rot = 0;
    __syncthreads();
    for (int t = 0; t + 1 < qq; ++t) {
      for (int pk = wave; pk < qq / 2; pk += kWaves) {
        int i, j;
        rr_pair(t, pk, qq, i, j);
        if (i >= q || j >= q) continue;  // the padding column
        double* ci = M + (long long)i * q;
        double* cj = M + (long long)j * q;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int r = lane; r < q; r += 64) {
          const double x = ci[r], y = cj[r];
          a = fma(x, x, a);
          b = fma(y, y, b);
          c = fma(x, y, c);
        }
        a = wave_sum(a);
        b = wave_sum(b);
        c = wave_sum(c);
        if (c != 0.0 && fmin(a, b) >= floor2 && fabs(c) > 1e-15 * sqrt(a) * sqrt(b)) {
          const double z = (b - a) / (2.0 * c);
          const double tt = copysign(1.0, z) / (fabs(z) + sqrt(fma(z, z, 1.0)));
          const double cs = 1.0 / sqrt(fma(tt, tt, 1.0)), sn = cs * tt;
          for (int r = lane; r < q; r += 64) {
            const double x = ci[r], y = cj[r];
            ci[r] = cs * x - sn * y;
            cj[r] = sn * x + cs * y;
          }
          if (lane == 0) s_rot = 1;
        }
      }
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (rot == 0) break;
  }
  // column norms, their descending order, the unit columns
  for (int c = wave; c < q; c += kWaves) {
    double a = 0.0;
    for (int r = lane; r < q; r += 64) a = fma(M[(long long)c * q + r], M[(long long)c * q + r], a);
    a = wave_sum(a);
    if (lane == 0) s_n[c] = sqrt(a);
  }
  __syncthreads();
  double smax = 0.0;
  for (int i = 0; i < q; ++i) smax = fmax(smax, s_n[i]);
  for (int c = threadIdx.x; c < q; c += kBig) {
    const double sc = s_n[c];
    int rank = 0;
    for (int i = 0; i < q; ++i) rank += (s_n[i] > sc || (s_n[i] == sc && i < c)) ? 1 : 0;
    const bool keep = sc > d.trunc * smax;
    if (!keep && d.count) atomicAdd(d.count, 1);
    d.S[rank] = keep ? sc : 0.0;
    const double inv = keep ? 1.0 / sc : 0.0;
    for (int r = 0; r < q; ++r) d.Ur[(long long)r * d.ldu + rank] = M[(long long)c * q + r] * inv;
  }
}
// ---------------------------------------------------------------- clusters
// Eigenvectors of close eigenvalues.  A twisted factorization gives each
// vector to an angle of about k eps ||T|| / gap in the worst case; on the
// Gram matrices of the update, whose spectra decay over decades, the vectors
// of well separated eigenvalues come out far better than that (the fits
// match the FP64 oracle to 1e-14), but eigenvalues within a relative gap of
// kClusterGap (exactly equal ones included) can give nearly parallel
// vectors.  Such runs of kept eigenvalues (lambda > kClusterFloor lambda_1,
// the square of the drop cut of the update) are recomputed by
// inverse iteration with reorthogonalization inside the run, the strategy of
// LAPACK's dstein: for each member, LU with partial pivoting of T - lambda I
// (tiny pivots replaced by eps ||T||), three steps of x <- (T - lambda)^-1 x
// each followed by Gram-Schmidt (twice) against the members already done;
// the first member starts from its twisted vector, the others from a fixed
// pseudo-random vector.  The vectors of a run then span its invariant
// subspace to about eps ||T|| / (gap to the rest of the spectrum).  A
// problem without such a run only scans its eigenvalues.
constexpr double kClusterGap = 1e-5;
constexpr double kClusterFloor = 1e-12;

__device__ __forceinline__ double wave_dot(const double* a, const GAS double* X, long long ld, int k,
                                           int lane) {  // sum_i a[i] X[i ld], one wave
  double s = 0.0;
  for (int i = lane; i < k; i += 64) s = fma(a[i], X[(long long)i * ld], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  return s;
}

__global__ void __launch_bounds__(64) cluster_kernel(const EigDesc* __restrict__ descs) {
  extern __shared__ double lds[];
  const EigDesc dd = descs[blockIdx.x];
  const int k = dd.k, r = dd.r, lane = threadIdx.x;
  if (r < 2 || k < 2) return;  // uniform
  EigWork W(dd.work, k, r);
  const double* ev = dd.evals;
  const double l1 = ev[0];
  if (!(l1 > 0.0)) return;
  const double floor_ = kClusterFloor * l1;
  // close: lambda_j - lambda_{j+1} <= kClusterGap lambda_j (both kept)
  auto close = [&](int a) { return ev[a + 1] > floor_ && ev[a] - ev[a + 1] <= kClusterGap * ev[a]; };
  // any run at all?  (one pass over the eigenvalues, all lanes)
  bool any = false;
  for (int j = lane; j + 1 < r; j += 64) any = any || close(j);
  if (!__any(any)) return;
  double* u0 = lds;          // U diagonal
  double* u1 = lds + k;      // first superdiagonal
  double* u2 = lds + 2 * k;  // second superdiagonal
  double* ml = lds + 3 * k;  // multipliers
  double* pv = lds + 4 * k;  // 1 where rows i, i+1 were swapped
  double* x = lds + 5 * k;   // the iterate
  GAS double* X = gstore_ptr(W.X);
  const GAS double* dg = W.d;
  const GAS double* eo = W.e;
  double tn = 0.0;  // ||T||_1-type bound for the pivot floor
  for (int i = lane; i < k; i += 64)
    tn = fmax(tn, fabs(dg[i]) + fabs(i > 0 ? eo[i - 1] : 0.0) + fabs(i + 1 < k ? eo[i] : 0.0));
  for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_xor(tn, off));
  const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);
  int j = 0;
  while (j + 1 < r) {
    if (!(ev[j + 1] > floor_)) break;  // uniform: the rest is dropped
    if (!close(j)) { ++j; continue; }
    int j1 = j + 1;
    while (j1 + 1 < r && close(j1)) ++j1;
    for (int m = j; m <= j1; ++m) {
      const double lam = ev[m];
      if (lane == 0) {  // LU of T - lam I with partial pivoting (rows i, i+1)
        double cd = dg[0] - lam, cs1 = k > 1 ? eo[0] : 0.0, cs2 = 0.0;
        for (int i = 0; i + 1 < k; ++i) {
          const double sub = eo[i], nd = dg[i + 1] - lam, ns = i + 2 < k ? eo[i + 1] : 0.0;
          if (fabs(cd) >= fabs(sub)) {
            const double piv = fabs(cd) < tiny ? (cd < 0.0 ? -tiny : tiny) : cd;
            const double l = sub / piv;
            u0[i] = piv; u1[i] = cs1; u2[i] = cs2; ml[i] = l; pv[i] = 0.0;
            cd = nd - l * cs1;
            cs1 = ns - l * cs2;
          } else {
            const double l = cd / sub;
            u0[i] = sub; u1[i] = nd; u2[i] = ns; ml[i] = l; pv[i] = 1.0;
            cd = cs1 - l * nd;
            cs1 = cs2 - l * ns;
          }
          cs2 = 0.0;
        }
        u0[k - 1] = fabs(cd) < tiny ? (cd < 0.0 ? -tiny : tiny) : cd;
        u1[k - 1] = u2[k - 1] = 0.0;
        if (k > 1) u2[k - 2] = 0.0;
      }
      // start vector
      for (int i = lane; i < k; i += 64) {
        if (m == j) {
          x[i] = X[(long long)i * r + m];
        } else {  // a fixed pseudo-random vector (integer hash of i and m)
          unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)((m + 1) * 2246822519u);
          h ^= h >> 15; h *= 2654435761u; h ^= h >> 13;
          x[i] = ((double)(h & 0xffffff) / 16777216.0) - 0.5;
        }
      }
      __syncthreads();
      for (int it = 0; it < 4; ++it) {
        // orthogonalize against the members done (twice), then normalize
        for (int pass = 0; pass < 2; ++pass)
          for (int q = j; q < m; ++q) {
            const double c = wave_dot(x, X + q, r, k, lane);
            __syncthreads();
            for (int i = lane; i < k; i += 64) x[i] = fma(-c, X[(long long)i * r + q], x[i]);
            __syncthreads();
          }
        double nn = 0.0;
        for (int i = lane; i < k; i += 64) nn = fma(x[i], x[i], nn);
        for (int off = 32; off > 0; off >>= 1) nn += __shfl_xor(nn, off);
        const double inv = nn > 0.0 ? rsqrt(nn) : 0.0;
        __syncthreads();
        for (int i = lane; i < k; i += 64) x[i] *= inv;
        __syncthreads();
        if (it == 3) break;
        if (lane == 0) {  // x <- (T - lam I)^-1 x:  L U x = P x
          for (int i = 0; i + 1 < k; ++i) {
            if (pv[i] != 0.0) { const double t = x[i]; x[i] = x[i + 1]; x[i + 1] = t; }
            x[i + 1] -= ml[i] * x[i];
          }
          x[k - 1] /= u0[k - 1];
          if (k > 1) x[k - 2] = (x[k - 2] - u1[k - 2] * x[k - 1]) / u0[k - 2];
          for (int i = k - 3; i >= 0; --i) x[i] = (x[i] - u1[i] * x[i + 1] - u2[i] * x[i + 2]) / u0[i];
          // keep the scale in range before the next normalization
          double mx = 0.0;
          for (int i = 0; i < k; ++i) mx = fmax(mx, fabs(x[i]));
          if (mx > 0.0 && isfinite(mx)) for (int i = 0; i < k; ++i) x[i] /= mx;
        }
        __syncthreads();
      }
      for (int i = lane; i < k; i += 64) X[(long long)i * r + m] = x[i];
      __syncthreads();
    }
    j = j1 + 1;
  }
}

// ---------------------------------------------------------------- Householder QR
// Column j: the reflector H_j = I - tau v v^T with v_j = 1 that maps
// X(j:m, j) onto beta e_j (beta = -sign(alpha) ||X(j:m, j)||, the LAPACK
// dlarfg convention); v is kept below the diagonal.  H_j is applied to the
// trailing columns by the whole workgroup: w = v^T X(j:, j+1:) with
// kBig / nc threads per column (nc trailing columns, each thread a
// contiguous block of rows, the blocks summed in row order in LDS: the
// order of a sequential dot product, which measured more accurate on the
// graded factors of the canonical forms than strided slices), then the
// rank-1 update over (row,
// column) pairs, columns fastest so that the accesses are coalesced.  The
// matrix stays in global memory (L2); n <= kBig.
__device__ __forceinline__ void hh_apply(GAS double* Y, long long ldy, const GAS double* V, long long ldv,
                                         int j, int m, int c0, int nc, double tau, double* wpart,
                                         double* wv) {
  const int tid = threadIdx.x;
  const int per = kBig / nc;
  if (tid < nc * per) {  // thread r0 of a column sums a contiguous block of rows, in row order
    const int c = c0 + tid % nc, r0 = tid / nc;
    const int rows = m - j - 1, blk = (rows + per - 1) / per;
    const int i0 = j + 1 + r0 * blk, i1 = min(m, i0 + blk);
    double s = r0 == 0 ? Y[(long long)j * ldy + c] : 0.0;
    for (int i = i0; i < i1; ++i) s = fma(V[(long long)i * ldv + j], Y[(long long)i * ldy + c], s);
    wpart[tid] = s;
  }
  __syncthreads();
  if (tid < nc) {
    double w = 0.0;
    for (int q = 0; q < per; ++q) w += wpart[q * nc + tid];
    wv[tid] = tau * w;
  }
  __syncthreads();
  const long long tot = (long long)(m - j) * nc;
  for (long long e = tid; e < tot; e += kBig) {
    const int i = j + (int)(e / nc), cc = (int)(e % nc);
    const double vi = i == j ? 1.0 : V[(long long)i * ldv + j];
    Y[(long long)i * ldy + c0 + cc] = fma(-vi, wv[cc], Y[(long long)i * ldy + c0 + cc]);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBig) geqr_kernel(const GeqrDesc* __restrict__ descs) {
  __shared__ double red[kBig / 64];
  __shared__ double wpart[kBig], wv[kBig];
  const GeqrDesc d = descs[blockIdx.x];
  const int m = d.m, n = d.n, p = min(m, n);
  const long long ld = d.ldx;
  GAS double* X = gstore_ptr(d.X);
  for (int j = 0; j < p; ++j) {
    double ss = 0.0;
    for (int i = j + 1 + threadIdx.x; i < m; i += kBig) {
      const double v = X[i * ld + j];
      ss = fma(v, v, ss);
    }
    ss = block_sum<kBig / 64>(ss, red);
    const double alpha = X[j * ld + j];
    double beta = alpha, tau = 0.0, scal = 0.0;
    if (ss > 0.0) {
      const double nrm = sqrt(fma(alpha, alpha, ss));
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read alpha
    for (int i = j + 1 + threadIdx.x; i < m; i += kBig) X[i * ld + j] *= scal;
    if (threadIdx.x == 0) {
      X[j * ld + j] = beta;
      if (d.tau) gstore_ptr(d.tau)[j] = tau;
    }
    __syncthreads();
    if (tau != 0.0 && j + 1 < n) hh_apply(X, ld, X, ld, j, m, j + 1, n - j - 1, tau, wpart, wv);
  }
  GAS double* R = gstore_ptr(d.R);
  for (long long e = threadIdx.x; e < (long long)p * n; e += kBig) {
    const int i = (int)(e / n), c = (int)(e % n);
    R[(long long)i * d.ldr + c] = c >= i ? X[i * ld + c] : 0.0;
  }
}

// Q = H_0 H_1 ... H_{n-1} [I; 0], the reflectors applied last to first to
// the trailing block Q(j:, j:) (columns left of j are still e_c there), each
// by the whole workgroup as in geqr_kernel; then the signs: column c of Q
// and row c of R negated where R(c, c) < 0, so that diag(R) >= 0.
__global__ void __launch_bounds__(kBig) orgqr_kernel(const OrgqrDesc* __restrict__ descs) {
  __shared__ double wpart[kBig], wv[kBig], sgn[kBig];
  const OrgqrDesc d = descs[blockIdx.x];
  const int m = d.m, n = d.n;
  const long long ldx = d.ldx, ldq = d.ldq;
  const GAS double* X = gload_ptr(d.X);
  GAS double* Q = gstore_ptr(d.Q);
  for (long long e = threadIdx.x; e < (long long)m * n; e += kBig) {
    const int i = (int)(e / n), c = (int)(e % n);
    Q[i * ldq + c] = i == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double t = gload_ptr(d.tau)[j];
    if (t == 0.0) continue;  // uniform
    hh_apply(Q, ldq, X, ldx, j, m, j, n - j, t, wpart, wv);
  }
  GAS double* R = gstore_ptr(d.R);
  for (int c = threadIdx.x; c < n; c += kBig) sgn[c] = R[(long long)c * d.ldr + c] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  for (long long e = threadIdx.x; e < (long long)m * n; e += kBig) {
    const int i = (int)(e / n), c = (int)(e % n);
    if (sgn[c] < 0.0) Q[i * ldq + c] = -Q[i * ldq + c];
  }
  for (long long e = threadIdx.x; e < (long long)n * n; e += kBig) {
    const int c = (int)(e / n), c2 = (int)(e % n);
    if (sgn[c] < 0.0 && c2 >= c) R[(long long)c * d.ldr + c2] = -R[(long long)c * d.ldr + c2];
  }
}

// Householder QR with the explicit Q in one kernel, X (m x n, m >= n)
// resident in LDS (row pitch n + 1, which spreads a column over the banks):
// the reflectors as in geqr_kernel; R (upper n x n) and tau out; then Q =
// H_0 ... H_{n-1} [I; 0] formed in place of the reflectors, last reflector
// first (LAPACK's backward accumulation: apply H_j to the columns right of
// j, then column j becomes -tau_j v_j with 1 - tau_j on the diagonal and
// zeros above); the signs as in orgqr_kernel.  Each reflector's products
// with the columns it acts on are sums over contiguous row blocks in row
// order, then over the blocks in order.
__device__ __forceinline__ void hh_apply_lds(double* A, int lda, int j, int m, int c0, int nc, double tau,
                                             double* wpart, double* wv) {
  const int tid = threadIdx.x;
  const int per = min(kBig / nc, 16);  // row blocks per column: a short in-order sum of the partials
  if (tid < nc * per) {
    const int c = c0 + tid % nc, r0 = tid / nc;
    const int rows = m - j - 1, blk = (rows + per - 1) / per;
    const int i0 = j + 1 + r0 * blk, i1 = min(m, i0 + blk);
    double s = r0 == 0 ? A[j * lda + c] : 0.0;
    for (int i = i0; i < i1; ++i) s = fma(A[i * lda + j], A[i * lda + c], s);
    wpart[tid] = s;
  }
  __syncthreads();
  if (tid < nc) {
    double w = 0.0;
    for (int q = 0; q < per; ++q) w += wpart[q * nc + tid];
    wv[tid] = tau * w;
  }
  __syncthreads();
  const int tot = (m - j) * nc;
  for (int e = tid; e < tot; e += kBig) {
    const int i = j + e / nc, cc = e % nc;
    const double vi = i == j ? 1.0 : A[i * lda + j];
    A[i * lda + c0 + cc] = fma(-vi, wv[cc], A[i * lda + c0 + cc]);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBig) hhqr_lds_kernel(const HhqrDesc* __restrict__ descs) {
  extern __shared__ double A[];
  __shared__ double red[kBig / 64];
  __shared__ double wpart[kBig], wv[kBig], taus[kBig];
  __shared__ signed char sgn[kBig];
  const HhqrDesc d = descs[blockIdx.x];
  const int m = d.m, n = d.n, lda = n + 1;
  const GAS double* X = gload_ptr(d.X);
  for (int e = threadIdx.x; e < m * n; e += kBig) A[(e / n) * lda + e % n] = X[(long long)(e / n) * d.ldx + e % n];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double ss = 0.0;
    for (int i = j + 1 + threadIdx.x; i < m; i += kBig) ss = fma(A[i * lda + j], A[i * lda + j], ss);
    ss = block_sum<kBig / 64>(ss, red);
    const double alpha = A[j * lda + j];
    double beta = alpha, tau = 0.0, scal = 0.0;
    if (ss > 0.0) {
      const double nrm = sqrt(fma(alpha, alpha, ss));
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read alpha
    for (int i = j + 1 + threadIdx.x; i < m; i += kBig) A[i * lda + j] *= scal;
    if (threadIdx.x == 0) {
      A[j * lda + j] = beta;
      taus[j] = tau;
    }
    __syncthreads();
    if (tau != 0.0 && j + 1 < n) hh_apply_lds(A, lda, j, m, j + 1, n - j - 1, tau, wpart, wv);
  }
  // R (signs normalized so that diag(R) >= 0) and tau out
  for (int c = threadIdx.x; c < n; c += kBig) {
    sgn[c] = A[c * lda + c] < 0.0 ? -1 : 1;
    if (d.tau) gstore_ptr(d.tau)[c] = taus[c];
  }
  __syncthreads();
  GAS double* R = gstore_ptr(d.R);
  for (int e = threadIdx.x; e < n * n; e += kBig) {
    const int i = e / n, c = e % n;
    R[(long long)i * d.ldr + c] = c >= i ? (double)sgn[i] * A[i * lda + c] : 0.0;
  }
  __syncthreads();
  // Q in place of the reflectors
  for (int j = n - 1; j >= 0; --j) {
    const double t = taus[j];
    if (j + 1 < n && t != 0.0) hh_apply_lds(A, lda, j, m, j + 1, n - j - 1, t, wpart, wv);
    for (int i = threadIdx.x; i < m; i += kBig) {
      double& a = A[i * lda + j];
      a = i < j ? 0.0 : i == j ? 1.0 - t : -t * a;
    }
    __syncthreads();
  }
  GAS double* Q = gstore_ptr(d.Q);
  for (int e = threadIdx.x; e < m * n; e += kBig) {
    const int i = e / n, c = e % n;
    Q[(long long)i * d.ldq + c] = (double)sgn[c] * A[i * lda + c];
  }
}
}  // namespace

size_t hhqr_lds_bytes(int m, int n) { return (size_t)m * (n + 1) * sizeof(double); }

bool hhqr_fits_lds(int m, int n) {
  static int limit = -1;
  if (limit < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 0;
    limit = v;
  }
  // static LDS of the kernel: the reduction slots, three kBig vectors, the signs
  const size_t fixed = (kBig / 64 + 3 * kBig) * sizeof(double) + kBig;
  return n <= kBig && m >= n && hhqr_lds_bytes(m, n) + fixed <= (size_t)limit;
}

void launch_hhqr(const HhqrDesc* d, int n, int max_m, int max_n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(hhqr_lds_kernel, dim3(n), dim3(kBig), hhqr_lds_bytes(max_m, max_n), s, d);
}

void launch_orgqr(const OrgqrDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(orgqr_kernel, dim3(n), dim3(kBig), 0, s, d);
}

void launch_geqr(const GeqrDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(geqr_kernel, dim3(n), dim3(kBig), 0, s, d);
}

// The register kernels by size: the 16 x 16 grid with the fewest register
// blocks that hold k (k <= kRegMax).
struct RegChol {
  template <int NB, int G>
  static void go(const CholDesc* d, int n, hipStream_t s) {
    hipLaunchKernelGGL((chol_inv_reg_kernel<NB, G>), dim3(n), dim3(G * G), 0, s, d);
  }
};
struct RegSytrd {
  template <int NB, int G>
  static void go(const EigDesc* d, int n, hipStream_t s) {
    hipLaunchKernelGGL((sytrd_reg_kernel<NB, G>), dim3(n), dim3(G * G), 0, s, d);
  }
};
struct RegZ {
  template <int NB, int G>
  static void go(const EigDesc* d, int n, hipStream_t s) {
    static_assert(G == 16, "z_rows_kernel takes 16 columns per row pass");
    hipLaunchKernelGGL((z_rows_kernel<NB>), dim3(4 * NB, n), dim3(64), 0, s, d);  // r <= k <= 16 NB
  }
};
template <class K, class D>
void launch_reg(const D* d, int n, int max_k, hipStream_t s) {
  if (max_k <= 32) K::template go<2, 16>(d, n, s);
  else if (max_k <= 64) K::template go<4, 16>(d, n, s);
  else if (max_k <= 96) K::template go<6, 16>(d, n, s);
  else if (max_k <= 128) K::template go<8, 16>(d, n, s);
  else if (max_k <= 144) K::template go<9, 16>(d, n, s);
  else if (max_k <= 160) K::template go<10, 16>(d, n, s);
  else K::template go<11, 16>(d, n, s);  // k <= kRegMax = 176
}

size_t eig_work_doubles(int k, int r) {
  return 3 * (size_t)k + 2 * (size_t)k * k + (size_t)k * r + 4 * (size_t)kPanel * k;
}

int eig_panel_width(int max_k) { return max_k <= 290 ? 32 : max_k <= 570 ? 16 : max_k <= 1100 ? 8 : 0; }


void launch_chol(const CholDesc* d, int n, int max_k, int inverse, hipStream_t s) {
  if (n <= 0) return;
  if (inverse) {
    launch_reg<RegChol>(d, n, max_k, s);
    return;
  }
  // packed lower triangle in LDS when every problem fits, else the factor's
  // own output array in global memory serves as working storage
  if (max_k <= kPackedMax) {
    const size_t lds = (size_t)max_k * (max_k + 1) / 2 * sizeof(double);
    hipLaunchKernelGGL(chol_kernel<false>, dim3(n), dim3(kBig), lds, s, d);
  } else {
    hipLaunchKernelGGL(chol_kernel<true>, dim3(n), dim3(kBig), 0, s, d);
  }
}

void launch_trsm(const TrsmDesc* d, int n, int max_rows, hipStream_t s) {
  // caller guarantees k <= 512 for every descriptor (checked on the host)
  if (n <= 0 || max_rows <= 0) return;
  dim3 grid(ceil_div(max_rows, kBig / 64), n);
  hipLaunchKernelGGL(trsm_kernel<8>, grid, dim3(kBig), 0, s, d);
}

void launch_jacobi(const JacobiDesc* d, int n, int max_q, hipStream_t s) {
  if (n <= 0) return;
  const int in_lds = max_q <= kJacobiLds ? 1 : 0;
  const size_t lds = in_lds ? (size_t)max_q * max_q * sizeof(double) : 0;
  hipLaunchKernelGGL(jacobi_kernel, dim3(n), dim3(kBig), lds, s, d, in_lds);
}

void launch_eig(const EigDesc* d, const EigDesc* h, int n, int reg, int stage, hipStream_t s) {
  if (n <= 0) return;
  int max_k = 0, max_r = 0;
  for (int i = 0; i < n; ++i) {
    max_k = std::max(max_k, h[i].k);
    max_r = std::max(max_r, h[i].r);
  }
  if (stage >= kEigPanelStage) {  // one panel of the global-memory reduction
    const int j0 = stage - kEigPanelStage, nb = eig_panel_width(max_k);
    const size_t lds = (2 * (size_t)nb * max_k + 2 * (size_t)max_k) * sizeof(double);
    if (nb == 32) hipLaunchKernelGGL(sytrd_panel_kernel<32>, dim3(n), dim3(kBig), lds, s, d, j0);
    else if (nb == 16) hipLaunchKernelGGL(sytrd_panel_kernel<16>, dim3(n), dim3(kBig), lds, s, d, j0);
    else hipLaunchKernelGGL(sytrd_panel_kernel<8>, dim3(n), dim3(kBig), lds, s, d, j0);
    return;
  }
  const bool all = stage < 0;
  if (all || stage == 0) {
    if (reg) {
      launch_reg<RegSytrd>(d, n, max_k, s);
    } else {
      if (max_k <= kPackedMax) {
        const size_t lds1 = (2 * (size_t)max_k + (size_t)max_k * (max_k + 1) / 2) * sizeof(double);
        hipLaunchKernelGGL(sytrd_kernel<false>, dim3(n), dim3(kBig), lds1, s, d);
      } else {
        hipLaunchKernelGGL(sytrd_kernel<true>, dim3(n), dim3(kBig), 2 * (size_t)max_k * sizeof(double), s, d);
      }
    }
  }
  if (all || stage == 1) {
    // few eigenvalues: a workgroup each (fewest rounds); many: eight lanes
    // each, 32 per workgroup (fewest Sturm counts)
    const size_t lds = 2 * (size_t)max_k * sizeof(double);
    if ((long long)n * max_r >= 2048)
      hipLaunchKernelGGL(bisect_kernel<8>, dim3(ceil_div(max_r, kBisect / 8), n), dim3(kBisect), lds, s, d);
    else
      hipLaunchKernelGGL(bisect_kernel<kBisect>, dim3(max_r, n), dim3(kBisect), lds, s, d);
  }
  if (all || stage == 2) {
    // one wave per eigenvalue; beyond kTwistWaveMax one thread per
    // eigenvalue, in smaller groups when there are few so that more compute
    // units share the work
    if (max_k <= kTwistWaveMax) {
      hipLaunchKernelGGL(twisted_wave_kernel, dim3(max_r, n), dim3(64), 6 * (size_t)max_k * sizeof(double), s, d);
    } else {
      int T = 64;
      while (T > 16 && (long long)ceil_div(max_r, T) * n < 128) T /= 2;
      while (T > 1 && (2 * (size_t)max_k * T + 2 * max_k) * sizeof(double) > 150 * 1024) T /= 2;
      hipLaunchKernelGGL(twisted_kernel, dim3(ceil_div(max_r, T), n), dim3(T),
                         (2 * (size_t)max_k * T + 2 * max_k) * sizeof(double), s, d);
    }
    // runs of close eigenvalues: inverse iteration with reorthogonalization
    // (6 k doubles of LDS; k <= 3200 fits)
    hipLaunchKernelGGL(cluster_kernel, dim3(n), dim3(64), 6 * (size_t)max_k * sizeof(double), s, d);
  }
  if (!(all || stage == 3)) return;
  if (reg) {  // Z = Q X row by row from the reflectors
    launch_reg<RegZ>(d, n, max_k, s);
    return;
  }
  // column blocks so that the block plus vectors fit in LDS
  int rb = std::max(1, std::min(max_r, (int)(120 * 1024 / sizeof(double) / max_k)));
  rb = std::min(rb, kBig);
  const size_t lds4 = ((size_t)max_k * rb + max_k + rb + kBig) * sizeof(double);
  hipLaunchKernelGGL(backtransform_kernel, dim3(ceil_div(max_r, rb), n), dim3(kBig), lds4, s, d, rb);
}

}  // namespace mpofit

// Small kernels of the two-site update (see fitkern.hpp).
#include <algorithm>
#include <cfloat>

#include "fitkern.hpp"

namespace mpofit {

namespace {

// Philox4x64-10 (Salmon et al., SC'11): two 64x64->128 multiplies per round,
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(unsigned long long c[4], unsigned long long k0,
                                              unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const unsigned long long hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const unsigned long long hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__device__ __forceinline__ double u53(unsigned long long w) {
  return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

__global__ void omega_kernel(const OmegaDesc* __restrict__ descs) {
  const OmegaDesc d = descs[blockIdx.y];
  int chi = d.chi, k = d.k;
  if (d.rk) {  // the bond's current shape (tolerance truncation)
    chi = d.rk[d.bond + 1];
    const int nt = d.rk[d.bond - 1] * d.dd, mt = d.dd * chi;
    k = min(min(d.kk, d.cap), min(nt, mt));
  }
  const long long n = (long long)d.dd * chi * k;
  const long long blk = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * blk >= n) return;
  const int stream = (*d.stream_base) * d.stream_mul + d.stream_add;
  unsigned long long c[4] = {(unsigned long long)blk, (unsigned long long)d.bond,
                             (unsigned long long)stream, (unsigned long long)d.pair};
  philox4x64_10(c, d.seed, 0ull);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double rad = sqrt(-2.0 * log(u53(c[2 * q])));
    double sn, cs;
    sincos(2.0 * M_PI * u53(c[2 * q + 1]), &sn, &cs);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long long e = 4 * blk + 2 * q + h;
      if (e < n) {
        const int i = (int)(e / k), j = (int)(e % k);
        const int cc = i % chi, su = i / chi;
        const int p = cc * d.dd + su;
        d.out[(long long)p * d.k + j] = h ? rad * sn : rad * cs;
      }
    }
  }
}

// Sign rule on the columns of U: the entry of largest magnitude of each
// column becomes positive (the first such row wins ties).  A workgroup takes
// 64 columns; its 16 waves split the rows (row i to wave i % 16).  Up to
// kSignCache rows per lane (n <= 512) the column slice is read once, with
// every load in flight, and scaled from registers; taller matrices read it
// twice, four loads in flight per lane.
constexpr int kSignWaves = 16;
constexpr int kSignCache = 32;
__global__ void __launch_bounds__(64 * kSignWaves) signfix_kernel(const SignDesc* __restrict__ descs) {
  __shared__ double s_max[kSignWaves][64];
  __shared__ int s_idx[kSignWaves][64];
  __shared__ double s_sgn[64];
  const SignDesc d = descs[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  if (blockIdx.x * 64 >= d.r) return;  // uniform
  GAS double* U = gstore_ptr(d.U);
  const bool cached = d.n <= kSignWaves * kSignCache;  // uniform
  double v[kSignCache];
  double best = -1.0;
  int bi = 0x7fffffff;
  if (col < d.r) {
    if (cached) {
#pragma unroll
      for (int q = 0; q < kSignCache; ++q) {
        const int i = wave + kSignWaves * q;
        v[q] = i < d.n ? U[(long long)i * d.ld + col] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kSignCache; ++q) {
        const int i = wave + kSignWaves * q;
        if (i < d.n && fabs(v[q]) > best) { best = fabs(v[q]); bi = i; }
      }
    } else {
      int i = wave;
      for (; i + 3 * kSignWaves < d.n; i += 4 * kSignWaves) {
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = U[(long long)(i + q * kSignWaves) * d.ld + col];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (fabs(x[q]) > best) { best = fabs(x[q]); bi = i + q * kSignWaves; }
      }
      for (; i < d.n; i += kSignWaves) {
        const double x = U[(long long)i * d.ld + col];
        if (fabs(x) > best) { best = fabs(x); bi = i; }
      }
    }
  }
  s_max[wave][lane] = best;
  s_idx[wave][lane] = bi;
  __syncthreads();
  if (wave == 0) {
    double b = s_max[0][lane];
    int ii = s_idx[0][lane];
    for (int w = 1; w < kSignWaves; ++w) {
      const double bw = s_max[w][lane];
      const int iw = s_idx[w][lane];
      if (bw > b || (bw == b && iw < ii)) { b = bw; ii = iw; }
    }
    // the winning entry sits in another wave's registers: read it again
    double sg = 1.0;
    if (col < d.r && ii != 0x7fffffff) sg = U[(long long)ii * d.ld + col] < 0.0 ? -1.0 : 1.0;
    s_sgn[lane] = sg;
    if (col < d.r) gstore_ptr(d.sign)[col] = sg;
  }
  __syncthreads();
  float amax = 0.f;
  if (col < d.r) {
    const double sg = s_sgn[lane];
    if (cached) {
#pragma unroll
      for (int q = 0; q < kSignCache; ++q) {
        const int i = wave + kSignWaves * q;
        if (i < d.n) {
          const double x = v[q] * sg;
          U[(long long)i * d.ld + col] = x;
          amax = fmaxf(amax, fabsf((float)x));
        }
      }
    } else {
      for (int i = wave; i < d.n; i += kSignWaves) {
        GAS double* p = U + (long long)i * d.ld + col;
        const double x = *p * sg;
        *p = x;
        amax = fmaxf(amax, fabsf((float)x));
      }
    }
  }
  if (d.amax) {
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    if (lane == 0) atomicMax(d.amax, __float_as_uint(amax));
  }
}

__global__ void scale_kernel(const ScaleDesc* __restrict__ descs) {
  const ScaleDesc d = descs[blockIdx.y];
  const long long n = (long long)d.n * d.r;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / d.r), j = (int)(e % d.r);
    double v = d.in[(long long)i * d.ldi + j];
    // the inverse is the pseudo-inverse: a zero scale gives zero
    if (d.row) v = d.row_inv ? (d.row[i] != 0.0 ? v / d.row[i] : 0.0) : v * d.row[i];
    if (d.col) {
      if (d.col_inv == 2) v = d.col[j] != 0.0 ? v : 0.0;  // a mask: select, so a NaN is cleared too
      else v = d.col_inv ? (d.col[j] != 0.0 ? v / d.col[j] : 0.0) : v * d.col[j];
    }
    d.out[(long long)i * d.ldo + j] = v;
  }
}

__global__ void perm_kernel(const PermDesc* __restrict__ descs) {
  const PermDesc d = descs[blockIdx.y];
  const long long n4 = (long long)d.n[0] * d.n[1] * d.n[2] * d.n[3];
  const long long n45 = (long long)d.n[4] * d.n[5];
  const long long n = n4 * n45;
  float amax = 0.f;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    long long r = e;
    long long ii = 0, oo = 0;
    if (n45 != 1) {  // uniform: the two extra axes
      const int i5 = (int)(r % d.n[5]); r /= d.n[5];
      const int i4 = (int)(r % d.n[4]); r /= d.n[4];
      ii = i4 * d.si[4] + i5 * d.si[5];
      oo = i4 * d.so[4] + i5 * d.so[5];
    }
    const int i3 = (int)(r % d.n[3]); r /= d.n[3];
    const int i2 = (int)(r % d.n[2]); r /= d.n[2];
    const int i1 = (int)(r % d.n[1]);
    const int i0 = (int)(r / d.n[1]);
    ii += i0 * d.si[0] + i1 * d.si[1] + i2 * d.si[2] + i3 * d.si[3];
    oo += i0 * d.so[0] + i1 * d.so[1] + i2 * d.so[2] + i3 * d.so[3];
    const double v = (d.tin == 0 ? reinterpret_cast<const double*>(d.in)[ii]
                                 : (double)reinterpret_cast<const float*>(d.in)[ii]) * d.scale;
    if (d.tout == 0) reinterpret_cast<double*>(d.out)[oo] = v;
    else reinterpret_cast<float*>(d.out)[oo] = (float)v;
    amax = fmaxf(amax, fabsf((float)v));
  }
  if (d.amax) {
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    if ((threadIdx.x & 63) == 0) atomicMax(d.amax, __float_as_uint(amax));
  }
}

__global__ void svals_kernel(const SvalDesc* __restrict__ descs) {
  const SvalDesc d = descs[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.r) return;
  const double l0 = d.evals[0];
  const double lj = d.evals[j];
  const double s0 = sqrt(fmax(l0, 0.0));
  const double sj = sqrt(fmax(lj, 0.0));
  if (d.flag && !isfinite(lj)) atomicOr(d.flag, FLAG_NONFINITE);
  const bool keep = sj > kDrop * s0;
  d.S[j] = keep ? sj : 0.0;
  if (d.keep) d.keep[j] = keep ? 1.0 : 0.0;
  if (!keep && d.count) atomicAdd(d.count, 1);
}
__global__ void __launch_bounds__(256) trunc_kernel(const TruncDesc* __restrict__ descs) {
  __shared__ double red[4];
  __shared__ int s_keep;
  const TruncDesc d = descs[blockIdx.x];
  double t = 0.0;
  for (int e = threadIdx.x; e < d.kd; e += 256) t += d.diag[e];
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tot = (red[0] + red[1]) + (red[2] + red[3]);
    const double lim = d.thr * tot;
    int cmax = min(min(d.chi_max, d.cap), d.r);
    cmax = min(cmax, min(d.rk[d.bond - 1] * d.dd, d.dd * d.rk[d.bond + 1]));
    cmax = max(cmax, 1);
    int c = cmax;
    double head = 0.0;
    for (int j = 0; j < cmax; ++j) {
      head += fmax(d.evals[j], 0.0);
      if (tot - head <= lim) { c = j + 1; break; }
    }
    s_keep = c;
    d.rk[d.bond] = c;
  }
  __syncthreads();
  const int c = s_keep;
  int drops = 0;
  for (int j = threadIdx.x; j < d.r; j += 256) {
    if (j >= c) {
      d.S[j] = 0.0;
      d.keep[j] = 0.0;
    } else if (d.keep[j] == 0.0) {
      ++drops;
    }
  }
  if (d.count && drops) atomicAdd(d.count, drops);
}

__global__ void fill_kernel(const FillDesc* __restrict__ descs) {
  const FillDesc d = descs[blockIdx.y];
  if (d.eye_rows > 0) {
    const long long n = (long long)d.eye_rows * d.eye_cols;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
      const double v = (e / d.eye_cols == e % d.eye_cols) ? 1.0 : 0.0;
      if (d.eye_f64) reinterpret_cast<double*>(d.p)[e] = v;
      else reinterpret_cast<float*>(d.p)[e] = (float)v;
    }
    return;
  }
  unsigned* p = reinterpret_cast<unsigned*>(d.p);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < d.n_words;
       e += (long long)gridDim.x * blockDim.x)
    p[e] = 0u;
}

__global__ void __launch_bounds__(1024) norm_kernel(const NormDesc* __restrict__ descs) {
  __shared__ double red[16];
  __shared__ double s_nu;
  const NormDesc d = descs[blockIdx.x];
  double acc = 0.0;
  for (long long e = threadIdx.x; e < d.n; e += blockDim.x) acc += d.x[e] * d.x[e];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    s_nu = sqrt(s);
    *d.nu_out = s_nu;
  }
  __syncthreads();
  const double inv = s_nu > 0.0 ? 1.0 / s_nu : 1.0;
  for (long long e = threadIdx.x; e < d.n; e += blockDim.x) d.x[e] *= inv;
}

__global__ void __launch_bounds__(256) sumsq_kernel(const double* __restrict__ x, long long n,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256)
    acc = fma(x[e], x[e], acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) sumsq_finish_kernel(const double* __restrict__ part, int np,
                                                           double* __restrict__ nu_out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *nu_out = sqrt(red[0] + red[1] + red[2] + red[3]);
}

__global__ void __launch_bounds__(256) divide_kernel(double* __restrict__ x, long long n,
                                                     const double* __restrict__ nu) {
  const double v = *nu;
  const double inv = v > 0.0 ? 1.0 / v : 1.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256)
    x[e] *= inv;
}

__global__ void naive_kernel(const NaiveDesc* __restrict__ descs) {
  const NaiveDesc d = descs[blockIdx.y];
  const int pd = d.d;  // physical dimension
  const long long n = (long long)d.a0 * d.b0 * pd * pd * d.a1 * d.b1;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    long long q = e;
    const int jb = (int)(q % d.b1); q /= d.b1;
    const int ja = (int)(q % d.a1); q /= d.a1;
    const int u = (int)(q % pd); q /= pd;
    const int s = (int)(q % pd); q /= pd;
    const int ib = (int)(q % d.b0);
    const int ia = (int)(q / d.b0);
    double acc = 0.0;
    for (int t = 0; t < pd; ++t)
      acc = fma(d.A[(((long long)ia * pd + s) * pd + t) * d.a1 + ja],
                d.B[(((long long)ib * pd + t) * pd + u) * d.b1 + jb], acc);
    d.P[e] = acc;
  }
}

__global__ void polish_kernel(const PolishDesc* __restrict__ descs) {
  const PolishDesc d = descs[blockIdx.y];
  const long long n = (long long)d.k * d.k;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double g = d.G[e];
    d.G[e] = (e / d.k == e % d.k ? 1.5 : 0.0) - 0.5 * g;
  }
}

__global__ void bump_kernel(int* c, int by) {
  if (threadIdx.x == 0) c[0] += by;
}

int grid_for(long long elems, int threads, int cap = 2048) {
  long long g = (elems + threads - 1) / threads;
  return (int)std::max<long long>(1, std::min<long long>(g, cap));
}

}  // namespace

void launch_omega(const OmegaDesc* d, int n, int max_elems, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = ceil_div(ceil_div(max_elems, 4), 256);
  hipLaunchKernelGGL(omega_kernel, dim3(std::max(blocks, 1), n), dim3(256), 0, s, d);
}

void launch_signfix(const SignDesc* d, int n, int max_r, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(signfix_kernel, dim3(ceil_div(max_r, 64), n), dim3(64 * kSignWaves), 0, s, d);
}

void launch_scale(const ScaleDesc* d, int n, int max_elems, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(max_elems, 256), n), dim3(256), 0, s, d);
}

void launch_perm(const PermDesc* d, int n, long long max_elems, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(perm_kernel, dim3(grid_for(max_elems, 256), n), dim3(256), 0, s, d);
}

void launch_polish(const PolishDesc* d, int n, int max_k, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(polish_kernel, dim3(grid_for((long long)max_k * max_k, 256), n), dim3(256), 0, s, d);
}

void launch_naive(const NaiveDesc* d, int n, long long max_elems, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(naive_kernel, dim3(grid_for(max_elems, 256), n), dim3(256), 0, s, d);
}

void launch_svals(const SvalDesc* d, int n, int max_r, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(svals_kernel, dim3(ceil_div(max_r, 256), n), dim3(256), 0, s, d);
}

void launch_trunc(const TruncDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(trunc_kernel, dim3(n), dim3(256), 0, s, d);
}

void launch_fill(const FillDesc* d, int n, long long max_words, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(max_words, 256), n), dim3(256), 0, s, d);
}

void launch_norm(const NormDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(norm_kernel, dim3(n), dim3(1024), 0, s, d);
}

void launch_norm_big(double* x, long long n, double* part, double* nu_out, hipStream_t s) {
  const int g = (int)std::min<long long>(1024, std::max<long long>(1, (n + 255) / 256));
  hipLaunchKernelGGL(sumsq_kernel, dim3(g), dim3(256), 0, s, x, n, part);
  hipLaunchKernelGGL(sumsq_finish_kernel, dim3(1), dim3(256), 0, s, part, g, nu_out);
  hipLaunchKernelGGL(divide_kernel, dim3(g), dim3(256), 0, s, x, n, nu_out);
}

void launch_bump(int* counter, int by, hipStream_t s) {
  hipLaunchKernelGGL(bump_kernel, dim3(1), dim3(64), 0, s, counter, by);
}

}  // namespace mpofit

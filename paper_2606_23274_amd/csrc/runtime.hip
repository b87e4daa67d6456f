// Host runtime of libmpofit: plan, workspace, initialization, the serial and
// even/odd sweep programs, export, and the C ABI (include/mpofit.h).
//
// Device layouts (all row-major; c, a, b = bonds of C, A, B; s = A's output
// leg, t = the contracted leg, u = B's input leg, of size du = d, or 1 when B
// is an MPS (Sec. 1); dd = d*du, C's two legs; i = 0-based site):
//   A, B cores (FP64 master)          [a][s][t][a'], [b][t][u][b']
//   C cores (FP64)                    [c][s][u][c']
//   working copies (FP32 or FP64):
//     Bw  = B            [b][t][u][b']   right operand of the first left step
//     Bmw = B mirrored   [b'][t][u][b]   same for the right environment
//     At  = A            [a][t][s][a']   (t before s) second left step
//     Amt = A mirrored   [a'][t][s][a]   second right step
//   Lenv[i]  left environment of sites 0..i-1    [c][a][b] at bond i
//   Renv[j]  right environment of sites j..L-1   [c][a][b] at bond j
//   XL[i]    L_i A_i B_i           [c][s][u][a'][b']      (bond i+1 on a', b')
//   XR[i]    A_{i+1} B_{i+1} R_{i+2}  [c''][s][u][a'][b']
//   two-site matrix of bond i: Theta = XL[i] XR[i]^T, n x m with rows
//     (c, s1, u1) and columns (c'', s2, u2).
// With these orders every contraction of Fig. envs and Fig. derivatives is a
// GEMM whose free and contracted index groups each have a single stride.
#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <mutex>
#include <stdexcept>

#include "../../include/mpofit.h"
#include "program.hpp"

namespace mpofit {

thread_local std::string g_last_error;

// ------------------------------------------------------------------ programs
void run_program(const Program& p, hipStream_t s, hipEvent_t* ev) {
  if (ev) HIP_OK(hipEventRecord(ev[0], s));
  for (size_t li = 0; li < p.launches.size(); ++li) {
    const Launch& l = p.launches[li];
    switch (l.kind) {
      case LK::Gemm: launch_gemm(l.gk, p.device<GemmDesc>(l), l.n, (int)l.wgs, s); break;
      case LK::Chol: launch_chol(p.device<CholDesc>(l), l.n, (int)l.maxa, l.maxb, s); break;
      case LK::Trsm: launch_trsm(p.device<TrsmDesc>(l), l.n, (int)l.maxa, s); break;
      case LK::Eig: launch_eig(p.device<EigDesc>(l), p.host<EigDesc>(l), l.n, l.maxb, (int)l.maxa, s); break;
      case LK::Omega: launch_omega(p.device<OmegaDesc>(l), l.n, (int)l.maxa, s); break;
      case LK::Sign: launch_signfix(p.device<SignDesc>(l), l.n, (int)l.maxa, s); break;
      case LK::Scale: launch_scale(p.device<ScaleDesc>(l), l.n, (int)l.maxa, s); break;
      case LK::Perm: launch_perm(p.device<PermDesc>(l), l.n, l.maxa, s); break;
      case LK::Sval: launch_svals(p.device<SvalDesc>(l), l.n, (int)l.maxa, s); break;
      case LK::Fill: launch_fill(p.device<FillDesc>(l), l.n, l.maxa, s); break;
      case LK::Norm: launch_norm(p.device<NormDesc>(l), l.n, s); break;
      case LK::Bump: launch_bump(l.counter, l.bump_by, s); break;
      case LK::Jacobi: launch_jacobi(p.device<JacobiDesc>(l), l.n, (int)l.maxa, s); break;
      case LK::Geqr: launch_geqr(p.device<GeqrDesc>(l), l.n, s); break;
      case LK::Orgqr: launch_orgqr(p.device<OrgqrDesc>(l), l.n, s); break;
      case LK::Trunc: launch_trunc(p.device<TruncDesc>(l), l.n, s); break;
      case LK::Hhqr: launch_hhqr(p.device<HhqrDesc>(l), l.n, (int)l.maxa, l.maxb, s); break;
      case LK::Naive: launch_naive(p.device<NaiveDesc>(l), l.n, l.maxa, s); break;
      case LK::Polish: launch_polish(p.device<PolishDesc>(l), l.n, (int)l.maxa, s); break;
      case LK::NormBig: {
        const NormDesc& nd = p.host<NormDesc>(l)[0];
        launch_norm_big(nd.x, nd.n, static_cast<double*>(l.aux), nd.nu_out, s);
        break;
      }
    }
    HIP_OK(hipGetLastError());
    if (ev) HIP_OK(hipEventRecord(ev[li + 1], s));
  }
}

namespace {

// ------------------------------------------------------------------ workspace
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

// ------------------------------------------------------------------ GEMM recording
struct Op {
  const void* p;
  DType t;
  bool kc;  // K-contiguous
  int ld;
  long long s[3] = {0, 0, 0};
  const unsigned* amax = nullptr;
};
struct Out {
  void* p;
  DType t;
  int ld;
  long long s[3] = {0, 0, 0};
  unsigned* amax = nullptr;
};

struct GemmJob {
  int M, N, K;
  Op A, B;
  Out C;
  int nb[3] = {1, 1, 1};
  double alpha = 1.0;
  int beta = 0;
};

// Split-K scratch plus the GEMM configuration hooks: the tuning table, a
// recorder of launch classes (autotuner) and a forced choice (autotuner).
struct SplitBuf {
  void* partials = nullptr;
  size_t cap = 0;  // bytes
  int* counters = nullptr;
  int ccap = 0;
  const std::vector<mpo_gemm_tune>* tune = nullptr;
  std::vector<std::pair<Mode, std::vector<GemmJob>>>* record = nullptr;
  int force_tile = -1, force_splits = 0;
};

// Tuning-table key of a grouped launch: operand kind, largest problem, count.
mpo_gemm_tune gemm_class(Mode mode, const std::vector<GemmJob>& jobs) {
  mpo_gemm_tune t{};
  t.mode = mode == Mode::F64 ? MPO_FP64 : mode == Mode::F32 ? MPO_FP32 : mode == Mode::BF16 ? MPO_BF16
                                                                                              : MPO_BF16X3;
  t.ta = jobs[0].A.t == DType::F64 ? 0 : 1;
  t.tb = jobs[0].B.t == DType::F64 ? 0 : 1;
  t.tc = jobs[0].C.t == DType::F64 ? 0 : 1;
  t.a_kcontig = jobs[0].A.kc;
  t.b_kcontig = jobs[0].B.kc;
  double best = -1;
  for (auto& j : jobs) {
    const double w = (double)j.M * j.N * j.K * j.nb[0] * j.nb[1] * j.nb[2];
    if (w > best) { best = w; t.M = j.M; t.N = j.N; t.K = j.K; }
  }
  t.count = 0;
  for (auto& j : jobs) t.count += j.nb[0] * j.nb[1] * j.nb[2];
  return t;
}

bool same_class(const mpo_gemm_tune& a, const mpo_gemm_tune& b) {
  return a.mode == b.mode && a.ta == b.ta && a.tb == b.tb && a.tc == b.tc &&
         a.a_kcontig == b.a_kcontig && a.b_kcontig == b.b_kcontig && a.M == b.M && a.N == b.N &&
         a.K == b.K && a.count == b.count;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

void add_gemm_kind(Program& P, const SplitBuf& sb, Mode mode, const std::vector<GemmJob>& jobs,
                   const char* cls, double flops);

// Appends grouped GEMM launches covering `jobs`: one launch per operand
// kind (element types and contiguity), since a launch is compiled for one.
void add_gemm(Program& P, const SplitBuf& sb, Mode mode, const std::vector<GemmJob>& jobs,
              const char* cls, double flops) {
  if (jobs.empty()) return;
  std::map<std::tuple<int, int, int, int, int>, std::vector<GemmJob>> groups;
  double total = 0;
  for (auto& j : jobs) total += 2.0 * j.M * j.N * j.K * j.nb[0] * j.nb[1] * j.nb[2];
  for (auto& j : jobs)
    groups[{(int)j.A.t, (int)j.B.t, (int)j.C.t, (int)j.A.kc, (int)j.B.kc}].push_back(j);
  for (auto& kv : groups) {
    double part = 0;
    for (auto& j : kv.second) part += 2.0 * j.M * j.N * j.K * j.nb[0] * j.nb[1] * j.nb[2];
    add_gemm_kind(P, sb, mode, kv.second, cls, total > 0 ? flops * part / total : 0);
  }
}

// One grouped GEMM launch covering `jobs` (all of one kind).
void add_gemm_kind(Program& P, const SplitBuf& sb, Mode mode, const std::vector<GemmJob>& jobs,
                   const char* cls, double flops) {
  if (jobs.empty()) return;
  if (sb.record) sb.record->emplace_back(mode, jobs);
  GemmKind gk{mode, jobs[0].A.t, jobs[0].B.t, jobs[0].C.t, jobs[0].A.kc, jobs[0].B.kc, 0};
  // tile 128x128 is possible for FP32/BF16 when every problem is large
  // enough; tile 2 (64x64, half-depth slabs) for FP32/BF16 always; tiles 3-5
  // (32x32, 32x32 with deep slabs, 16x16 with the waves splitting K) for FP64
  bool big = mode != Mode::F64;
  long long w128 = 0;
  int kmax = 0;
  for (auto& j : jobs) {
    kmax = std::max(kmax, j.K);
    if (j.M < 128 || j.N < 128) big = false;
    w128 += (long long)ceil_div(j.M, 128) * ceil_div(j.N, 128) * j.nb[0] * j.nb[1] * j.nb[2];
  }
  const mpo_gemm_tune* tuned = nullptr;
  if (sb.tune) {
    const mpo_gemm_tune key = gemm_class(mode, jobs);
    for (auto& t : *sb.tune)
      if (same_class(t, key)) { tuned = &t; break; }
  }
  auto usable = [&](int t) {
    if (mode == Mode::F64) return t >= 3 && t <= 5 ? t : 0;
    if (t == 3 || t == 4) return t;  // the 32 x 32 tiles serve every mode
    return t == 1 ? (big ? 1 : 0) : t == 2 ? 2 : 0;
  };
  long long w64 = 0;
  for (auto& j : jobs) w64 += (long long)ceil_div(j.M, 64) * ceil_div(j.N, 64) * j.nb[0] * j.nb[1] * j.nb[2];
  int split_cap = 0;  // 0: built-in rule
  if (sb.force_tile >= 0) {
    gk.tile = usable(sb.force_tile);
    split_cap = std::max(1, sb.force_splits);
  } else if (tuned) {
    gk.tile = usable(tuned->tile);
    split_cap = std::max(1, tuned->splits);
  } else if (big && w128 >= 256) {
    // built-in: the large tile when the launch still fills the chip
    gk.tile = 1;
  } else if (mode == Mode::F64 && w64 < 128) {
    // small FP64 products: 16x16 tiles, K split over the waves
    gk.tile = 5;
  } else if (mode == Mode::F32 && w64 < 128 && kmax >= 2048) {
    // few long-K FP32 tiles (the serial two-site product): 32x32 tiles with
    // deep slabs and no split-K give every CU several workgroups
    gk.tile = 4;
    split_cap = 1;
  } else if (kmax <= 512) {
    gk.tile = usable(2);  // short K: more resident workgroups
  }
  const int BM = gemm_bm(gk.tile), BN = gemm_bn(gk.tile), BK = gemm_bk(mode, gk.tile);
  long long base_wgs = 0;
  for (auto& j : jobs)
    base_wgs += (long long)ceil_div(j.M, BM) * ceil_div(j.N, BN) * j.nb[0] * j.nb[1] * j.nb[2];
  // built-in split-K rule: only launches of fewer than 128 tiles are split,
  // up to filling 256 CUs once, with at least four K slabs per split (the
  // deterministic reduction costs a device-scope fence per tile)
  const int want = gk.tile == 5 ? 1  // (the waves split K; no global split)
                   : split_cap > 0 ? split_cap
                   : base_wgs >= 128 ? 1
                                     : (int)std::min<long long>(8, (256 + base_wgs - 1) / base_wgs);
  const int min_slabs = split_cap > 0 ? 1 : 4;
  std::vector<GemmDesc> ds;
  long long wg = 0;
  size_t poff = 0;
  int coff = 0;
  for (auto& j : jobs) {
    GemmDesc d{};
    d.A = j.A.p; d.B = j.B.p; d.C = j.C.p;
    for (int q = 0; q < 3; ++q) { d.sA[q] = j.A.s[q]; d.sB[q] = j.B.s[q]; d.sC[q] = j.C.s[q]; d.nb[q] = j.nb[q]; }
    d.M = j.M; d.N = j.N; d.K = j.K;
    d.lda = j.A.ld; d.ldb = j.B.ld; d.ldc = j.C.ld;
    d.tiles_m = ceil_div(j.M, BM);
    d.tiles_n = ceil_div(j.N, BN);
    d.beta = j.beta;
    d.alpha = j.alpha;
    d.amax_a = j.A.amax; d.amax_b = j.B.amax; d.amax_c = j.C.amax;
    auto vec = [](const Op& o) {
      bool ok = (o.ld % 4 == 0) && aligned16(o.p);
      for (int q = 0; q < 3; ++q) ok = ok && (o.s[q] % 4 == 0);
      return ok ? 1 : 0;
    };
    d.vec_a = vec(j.A);
    d.vec_b = vec(j.B);
    const long long tiles = (long long)d.tiles_m * d.tiles_n * j.nb[0] * j.nb[1] * j.nb[2];
    int splits = std::max(1, std::min(want, j.K / (min_slabs * BK)));
    int kchunk = ceil_div(ceil_div(j.K, splits), BK) * BK;
    splits = std::max(1, ceil_div(j.K, kchunk));
    const size_t need = (size_t)tiles * splits * BM * BN * gemm_acc_bytes(mode);
    if (splits > 1 && (poff + need > sb.cap || coff + tiles > sb.ccap)) {
      splits = 1;
      kchunk = std::max(j.K, 1);
    }
    d.splits = splits;
    d.kchunk = splits > 1 ? kchunk : std::max(j.K, 1);
    if (splits > 1) {
      d.partials = static_cast<char*>(sb.partials) + poff;
      d.counters = sb.counters + coff;
      poff += need;
      coff += (int)tiles;
    }
    d.wg_begin = (int)wg;
    wg += tiles * splits;
    ds.push_back(d);
  }
  Launch l;
  l.kind = LK::Gemm;
  l.gk = gk;
  l.off = P.push(ds);
  l.n = (int)ds.size();
  l.wgs = wg;
  l.cls = cls;
  l.flops = flops;
  P.launches.push_back(l);
}

template <class D>
void add_simple(Program& P, LK kind, const std::vector<D>& ds, long long maxa, const char* cls,
                double flops = 0) {
  if (ds.empty()) return;
  Launch l;
  l.kind = kind;
  l.off = P.push(ds);
  l.n = (int)ds.size();
  l.maxa = maxa;
  l.cls = cls;
  l.flops = flops;
  P.launches.push_back(l);
}

// The eigen pipeline as one launch per stage (tridiagonalization, bisection,
// eigenvectors, back-transformation) over one descriptor array, so that each
// stage is timed on its own.  Tridiagonalization is credited (4/3) k^3 flops.
Op op64(const void* p, bool kc, int ld) { return Op{p, DType::F64, kc, ld}; }
Out out64(void* p, int ld) { return Out{p, DType::F64, ld}; }

// Eigen stages of a batch of problems.  The register path (every k <=
// kRegMax) has three kernels; otherwise the tridiagonal reduction runs panel
// by panel (a panel kernel, then a batched FP64 GEMM for the trailing
// update of the problems that have more panels), then bisection, twisted
// vectors and the back-transformation.
void add_eig(Program& P, const SplitBuf& sb, const std::vector<EigDesc>& ed, bool reg,
             const char* prefix) {
  if (ed.empty()) return;
  const size_t off = P.push(ed);
  double ftri = 0, fback = 0;
  int max_k = 0;
  for (auto& e : ed) {
    ftri += (4.0 / 3.0) * e.k * (double)e.k * e.k;
    fback += 4.0 * e.k * (double)e.k * e.r;
    max_k = std::max(max_k, e.k);
  }
  const bool init = std::string(prefix) == "init";
  const char* names[4] = {"eig_tridiag", "eig_bisect", "eig_vectors", "eig_backtransform"};
  auto stage = [&](long long code, const char* cls, double flops) {
    Launch l;
    l.kind = LK::Eig;
    l.off = off;
    l.n = (int)ed.size();
    l.maxb = reg ? 1 : 0;
    l.maxa = code;
    l.cls = init ? "init" : cls;
    l.flops = flops;
    P.launches.push_back(l);
  };
  const int nb = reg ? 0 : eig_panel_width(max_k);
  if (nb > 0) {
    int npan = 1;
    for (auto& e : ed) npan = std::max(npan, ceil_div(std::max(e.k - 2, 1), nb));
    for (int q = 0; q < npan; ++q) {
      const int j0 = q * nb;
      stage(kEigPanelStage + j0, names[0], q == 0 ? ftri : 0.0);
      std::vector<GemmJob> upd;  // A(pend:, pend:) -= P1 P2^T for problems with panels left
      for (auto& e : ed) {
        const int pend = std::min(j0 + nb, e.k - 2), t = e.k - pend;
        if (j0 >= e.k - 2 || pend >= e.k - 2) continue;
        double* P1 = eig_work_panel(e.work, e.k, e.r);
        double* P2 = P1 + 2 * (size_t)kPanel * e.k;
        double* H = eig_work_h(e.work, e.k, e.r);
        GemmJob g{t, t, 2 * nb, op64(P1 + (size_t)pend * 2 * nb, true, 2 * nb),
                  op64(P2 + (size_t)pend * 2 * nb, true, 2 * nb),
                  out64(H + (size_t)pend * e.k + pend, e.k)};
        g.alpha = -1.0;
        g.beta = 1;
        upd.push_back(g);
      }
      add_gemm(P, sb, Mode::F64, upd, init ? "init" : names[0], 0.0);
    }
  }
  // stage 3 applies the reflectors to the r eigenvectors (4 k^2 r flops)
  for (int st = nb > 0 ? 1 : 0; st < 4; ++st) stage(st, names[st], st == 0 ? ftri : st == 3 ? fback : 0.0);
}

// ------------------------------------------------------------------ state
struct PairState {
  int L = 0, d = 0, dd = 0;  // d: A's legs and C's output leg; dd = C's two legs (d du)
  int du = 0;                // C's and B's input leg: d, or 1 for an MPS (MPO-MPS variant)
  int dA = 0, dB = 0;        // physical size of an A core (d d) and of a B core (d du)
  bool mps = false;
  int chi_max = 1;
  std::vector<int> cA, cB, cC;  // bond dims (L+1): preprocessed A, B; current C
  std::vector<int> capC;        // capacity of C's bonds over the whole fit
  std::vector<int> rcap;        // chi^A_i chi^B_i per bond index i (1..L-1)
  // FP64 master cores
  std::vector<double*> A64, B64, C64;
  // working copies
  std::vector<void*> Bw, Bmw, At, Amt;
  std::vector<unsigned*> amBw, amBmw, amAt, amAmt;
  std::vector<void*> Lenv, Renv;  // by bond index 0..L
  std::vector<unsigned*> amL, amR;
  std::vector<void*> XL, XR;      // by bond 0..L-2
  std::vector<unsigned*> amXL, amXR;
  // inverse gauge (even/odd): Y_i = 1/S_i per bond 1..L-1 (bond index)
  std::vector<double*> Yv;
  double* nu_dev = nullptr;       // [2]: nu_A, nu_B
  double nu = 1.0;
  // tolerance truncation (tau > 0): the current bond dims on the device
  // (L+1, indexed by bond); the host dims above are then capacities
  int* rk = nullptr;
  // host copies of the input shapes; an optional initial guess C (else A)
  std::vector<int> chiA_in, chiB_in, chiC_in;
  std::vector<const double*> A_in, B_in, C_in;
};

// Bond b of the initial guess before its right-orthogonalization: the given
// C, else the input A (whose preprocessed dims never exceed the input ones).
int init_dim(const PairState& P, int b) {
  const int g = P.mps ? P.chiB_in[b] : P.chiA_in[b];
  return P.C_in.empty() ? g : std::max(g, P.chiC_in[b]);
}

// Factorization scratch of one bond.
struct BondScratch {
  void* theta;    // n x m (working type)
  void* T;        // first-step scratch of the left/right extension (working type)
  unsigned* amT;
  double *omega, *Y, *Y2, *G, *R, *Bk, *H, *eigw, *evals, *Z, *S, *V, *sign, *SVt;
  double* keep;  // inverse gauge: 1 for kept singular values, 0 for truncated
  double* diag;  // tolerance truncation: the Gram matrix's diagonal
};

struct Ctx {
  mpo_fit_opts o{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<std::pair<int, int>> parts;  // parallel schedule: sub-TT site ranges
  bool merged = false;                     // parallel schedule: mpo_fit_merge has run
  Mode wmode = Mode::F32;  // arithmetic of the contractions
  DType wt = DType::F32;   // storage type of environments and extensions
  std::vector<PairState> pairs;
  std::vector<BondScratch> scratch;  // serial: 1; even/odd: max bonds per half-step over pairs
  SplitBuf sb;
  int* flag = nullptr;          // device status flags
  int* sweep_dev = nullptr;     // device sweep counter (Philox stream)
  char* arena = nullptr;        // descriptor arena
  size_t arena_cap = 0;
  size_t arena_used = 0;
  // init scratch (FP64)
  double *iG, *iR1, *iR2, *iRt, *iTmp, *iXt, *iJ, *iTau;
  double *iH, *iZ, *iEw, *iEv, *iSg;  // eigenproblem of the inverse-canonical init
  size_t iTmpN = 0;
  int sweeps_done = 0;
  int pos = 0;  // units (updates or half-steps) already run of the current sweep
  std::map<std::string, Program> programs;  // keyed by shape plan
  std::map<std::string, hipGraphExec_t> graphs;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0;
  bool profile = false;
  struct ProfEntry {
    std::string cls;
    double ms = 0, flops = 0;
    int launches = 0;
  };
  std::vector<ProfEntry> prof;  // per kernel class, summed over the last call's sweeps
  std::vector<mpo_gemm_tune> tune;  // GEMM tuning table (copied from the options)
  long long n_trunc = 0;            // singular values truncated before inversion
  std::vector<double> prof_flops;
  size_t ws_bytes = 0;
  // fit error per sweep (opts.track_error): merged C in FP64 per pair, the
  // transfer-pass logs and arena, log ||A B||^2 per pair (normalized cores)
  struct ErrState {
    std::vector<std::vector<double*>> C;
    double* logs = nullptr;
    double* part = nullptr;
    char* region = nullptr;
    size_t region_bytes = 0;
    std::vector<double> l4;
  } err;
};

size_t err_region_bytes(const Ctx& X);

int bytes_of(DType t) { return t == DType::F64 ? 8 : 4; }

// ------------------------------------------------------------------ shapes
// Sub-TTs of the parallel schedule (Sec. 4): n_parts contiguous site ranges
// as equal as possible, the first ones one site longer.  Block n sweeps
// forward first when n is even ("F"), backward first otherwise ("B").
std::vector<std::pair<int, int>> partition_sites(int L, int n_parts) {
  std::vector<std::pair<int, int>> out;
  const int base = L / n_parts, extra = L % n_parts;
  int s = 0;
  for (int n = 0; n < n_parts; ++n) {
    const int ln = base + (n < extra ? 1 : 0);
    out.push_back({s, s + ln - 1});
    s += ln;
  }
  return out;
}

// Bond dims after the preprocessing and initial guess, and the capacity of
// each of C's bonds over the fit (the ranks r = min(chi_max, n, m, cap)
// settle within two sweeps; simulated here on the host).
void plan_shapes(PairState& P, int chi_max, int schedule, int first_sweep, int first_bond, int first_half,
                 int n_parts = 0) {
  const int L = P.L, dd = P.dd;
  auto leftorth = [&](const std::vector<int>& in, int pd) {
    std::vector<int> c(in);
    for (int i = 1; i < L; ++i) c[i] = std::min(in[i], c[i - 1] * pd);
    // the left sweep only clips from the left; entries to the right keep in[]
    return c;
  };
  P.cA = leftorth(P.chiA_in, P.dA);
  P.cB = leftorth(P.chiB_in, P.dB);
  P.rcap.assign(L + 1, 1);
  for (int i = 1; i < L; ++i) P.rcap[i] = P.cA[i] * P.cB[i];
  // initial C: the given guess (else A) right-orthogonalized, or left-
  // orthogonalized when a serial fit starts with a backward sweep
  std::vector<int> c(P.C_in.empty() ? (P.mps ? P.cB : P.cA) : P.chiC_in);
  const bool fwd0 = first_sweep % 2 == 0;
  if (schedule == MPO_SCHED_SERIAL && first_bond > 0) {  // mixed form around the next update's sites
    const int i0 = fwd0 ? first_bond : L - 2 - first_bond;
    for (int i = 1; i <= i0; ++i) c[i] = std::min(c[i], c[i - 1] * dd);
    for (int i = L - 1; i >= i0 + 2; --i) c[i] = std::min(c[i], dd * c[i + 1]);
  } else if (schedule == MPO_SCHED_SERIAL && !fwd0) {
    for (int i = 1; i < L; ++i) c[i] = std::min(c[i], c[i - 1] * dd);
  } else {
    for (int i = L - 1; i >= 1; --i) c[i] = std::min(c[i], dd * c[i + 1]);
  }
  P.cC = c;
  P.capC = c;
  std::vector<int> sim(c);
  auto upd = [&](int b) {  // bond b = 1..L-1 joins sites b-1, b
    const int n = sim[b - 1] * dd, m = dd * sim[b + 1];
    sim[b] = std::min(std::min(chi_max, P.rcap[b]), std::min(n, m));
    P.capC[b] = std::max(P.capC[b], sim[b]);
  };
  if (schedule == MPO_SCHED_PARALLEL) {
    // the QR sweep after the RQ sweep (clipping as rec_qr_sweep), then the
    // phases of six sets and the merge's updates
    const auto parts = partition_sites(L, n_parts);
    for (int i = 0; i + 1 < L; ++i)
      if (c[i] * dd < c[i + 1]) c[i + 1] = c[i] * dd;
    P.cC = c;
    P.capC = c;
    sim = c;
    auto sweeps = [&](bool fwd_first) {
      for (size_t n = 0; n < parts.size(); ++n) {
        const bool fwd = (n % 2 == 0) == fwd_first;
        const int s = parts[n].first, e = parts[n].second;
        if (fwd) for (int i = s; i < e; ++i) upd(i + 1);
        else for (int i = e - 1; i >= s; --i) upd(i + 1);
      }
    };
    for (int set = 0; set < 7; ++set) {
      sweeps(true);
      for (size_t n = 0; n + 1 < parts.size(); n += 2) upd(parts[n].second + 1);
      if (set == 6) break;  // the merge: local sweeps and updates at every boundary
      sweeps(false);
      for (size_t n = 1; n + 1 < parts.size(); n += 2) upd(parts[n].second + 1);
    }
    for (size_t n = 1; n + 1 < parts.size(); n += 2) upd(parts[n].second + 1);
    return;
  }
  for (int sw = 0; sw < 6; ++sw) {
    if (schedule == MPO_SCHED_SERIAL) {
      const int skip = sw == 0 ? first_bond : 0;  // a resumed first sweep starts later
      if ((sw + first_sweep) % 2 == 0) for (int b = 1 + skip; b < L; ++b) upd(b);
      else for (int b = L - 1 - skip; b >= 1; --b) upd(b);
    } else {
      for (int q = (sw == 0 ? first_half : 0); q < 2; ++q) {
        std::vector<int> prev(sim);
        for (int b = 1; b < L; ++b)
          if ((b % 2 == 1) == (q == 0)) {
            const int n = prev[b - 1] * dd, m = dd * prev[b + 1];
            sim[b] = std::min(std::min(chi_max, P.rcap[b]), std::min(n, m));
            P.capC[b] = std::max(P.capC[b], sim[b]);
          }
      }
    }
  }
}

struct Caps {  // per-pair maxima for scratch sizing
  long long nm_max = 1, kmax = 1, rmax = 1, theta = 1, T = 1, ext = 1;
};

Caps pair_caps(const PairState& P, const mpo_fit_opts& o) {
  Caps c;
  for (int b = 1; b < P.L; ++b) {  // bond b joins sites b-1 and b
    const long long n = (long long)P.capC[b - 1] * P.dd, m = (long long)P.dd * P.capC[b + 1];
    c.nm_max = std::max({c.nm_max, n, m});
    c.theta = std::max(c.theta, n * m);
    const long long kk = o.sketch_p < 0 ? n : std::min<long long>(n, P.chi_max + (long long)o.sketch_p);
    c.kmax = std::max({c.kmax, kk, n});  // exact path uses the n x n Gram
    c.rmax = std::max<long long>(c.rmax, P.capC[b]);
  }
  for (int i = 0; i < P.L; ++i) {
    // first extension step: rows (c, a) x cols (t, u, b') and its mirror
    c.T = std::max(c.T, (long long)P.capC[i] * P.cA[i] * P.dB * P.cB[i + 1]);
    c.T = std::max(c.T, (long long)P.capC[i + 1] * P.cA[i + 1] * P.dB * P.cB[i]);
    c.ext = std::max(c.ext, (long long)P.capC[i] * P.dd * P.cA[i + 1] * P.cB[i + 1]);
    c.ext = std::max(c.ext, (long long)P.capC[i + 1] * P.dd * P.cA[i] * P.cB[i]);
  }
  return c;
}

// ------------------------------------------------------------------ helpers
Op opW(const Ctx& X, const void* p, bool kc, int ld, const unsigned* amax = nullptr) {
  Op o{p, X.wt, kc, ld};
  o.amax = amax;
  return o;
}
Out outW(const Ctx& X, void* p, int ld, unsigned* amax = nullptr) {
  Out o{p, X.wt, ld};
  o.amax = amax;
  return o;
}

PermDesc perm4(const void* in, int tin, void* out, int tout, std::array<int, 4> n,
               std::array<long long, 4> si, std::array<long long, 4> so, double scale = 1.0) {
  PermDesc d{};
  d.in = in; d.out = out; d.tin = tin; d.tout = tout; d.scale = scale;
  for (int q = 0; q < 4; ++q) { d.n[q] = n[q]; d.si[q] = si[q]; d.so[q] = so[q]; }
  d.n[4] = d.n[5] = 1;
  return d;
}

long long perm_elems(const PermDesc& d) {
  return (long long)d.n[0] * d.n[1] * d.n[2] * d.n[3] * d.n[4] * d.n[5];
}

void add_perm(Program& P, const std::vector<PermDesc>& ds, const char* cls) {
  long long mx = 1;
  for (auto& d : ds) mx = std::max(mx, perm_elems(d));
  add_simple(P, LK::Perm, ds, mx, cls);
}

void add_fill(Program& P, const std::vector<FillDesc>& ds) {
  long long mx = 1;
  for (auto& d : ds) mx = std::max(mx, std::max(d.n_words, (long long)d.eye_rows * d.eye_cols));
  add_simple(P, LK::Fill, ds, mx, "fill");
}

// CholeskyQR of the n x k row-major X (in place), `passes` times.
// Fast path (every k <= kRegMax, no Rout): G = X^T X, R^{-1} from the
// register Cholesky, X <- X R^{-1} by a GEMM through the temp T (n x k).
// General path: Cholesky R, X <- X R^{-1} by the row-wise TRSM; the product
// of the triangular factors (upper, k x k) is left in Rout when non-null.
// R scratch must hold 2 k x k; G scratch k x k.
// keep (nullable): columns with keep[j] == 0 are zero in X and stay zero
// (unit Gram diagonal, see CholDesc).  eta > 0: rank-revealing passes, a
// column in the span of the previous ones (pivot <= eta G(j, j)) becomes a
// zero column of Q instead of a failure.
struct CholQRJob {
  double* X;
  int n, k, ld;
  double* G;
  double* R;     // >= 2*k*k
  double* Rout;  // nullable, k x k
  double* T;     // nullable, n x k temp (fast path)
  bool shifted = false;  // shifted first pass (general path only)
  const double* keep = nullptr;
  double eta = 0;
};

// Rank-revealing threshold of the Cholesky-QR passes: a column whose
// remaining squared norm is at most this fraction of its own is dependent
// (its independent part is below 1e-6 of its length, the drop cut; the
// rounding of a dependent column's pivot is about k eps of its norm).
constexpr double kRankEta = 1e-12;

// Diagonal shift of shifted CholeskyQR (Fukaya, Kannan, Nakatsukasa,
// Yamamoto, Yanagisawa, SIAM J. Sci. Comput. 2020): s = 11 (n k + k (k+1)) u
// ||X||_2^2 with u = 2^-53; ||X||_F^2 = trace(X^T X) stands in for ||X||_2^2
// (an upper bound, so the shift stays large enough).  One shifted pass leaves
// cond(Q) of order u^{-1/2}, which two plain passes then clean up, for inputs
// with cond(X) up to about u^{-1}.
double chol_shift(int n, int k) { return 11.0 * ((double)n * k + (double)k * (k + 1)) * 0x1p-53; }

// Blocked inverse Cholesky for kRegMax < k <= 2 kRegMax: with
// G = [[G11, G21^T], [G21, G22]] and k1 = ceil(k/2),
//   R11^{-1} = reg(G11), L21 = G21 R11^{-1}, S = G22 - L21 L21^T,
//   R22^{-1} = reg(S), X12 = -R11^{-1} (L21^T R22^{-1}),
// so R^{-1} = [[R11^{-1}, X12], [., R22^{-1}]] (the lower-left block is never
// read), and X R^{-1} = [X1 R11^{-1}, X [X12; R22^{-1}]].  Temporaries live in
// the second k x k block of the job's R scratch.
// Profile classes of a Cholesky-QR: the range finder's ("qr_*") or the
// re-orthonormalization of a gauge factor ("gauge_*").
struct QrClasses {
  const char *gram, *chol_inv, *chol, *apply;
};
inline QrClasses qr_classes(bool gauge) {
  return gauge ? QrClasses{"gauge_gram", "gauge_chol_inv", "gauge_chol", "gauge_apply"}
               : QrClasses{"qr_gram", "qr_chol_inv", "qr_chol", "qr_apply"};
}

void add_chol_inv_blocked(Ctx& X, Program& P, const std::vector<CholQRJob>& jobs, int pass, bool gauge) {
  const QrClasses qc = qr_classes(gauge);
  std::vector<GemmJob> gj, l21, s22, t2, x12, ap;
  std::vector<CholDesc> c1, c2;
  std::vector<PermDesc> cp;
  for (auto& j : jobs) {
    double* src = pass % 2 == 1 ? j.T : j.X;
    double* dst = pass % 2 == 1 ? j.X : j.T;
    const int lds = pass % 2 == 1 ? j.k : j.ld;
    const int ldd = pass % 2 == 1 ? j.ld : j.k;
    const int k = j.k, k1 = k <= kRegMax ? k : (k + 1) / 2, k2 = k - k1;
    double* Rp = j.R;
    double* L21 = j.R + (size_t)k * k;
    double* S = L21 + (size_t)k2 * k1;
    double* T2 = S + (size_t)k2 * k2;
    gj.push_back(GemmJob{k, k, j.n, op64(src, false, lds), op64(src, false, lds), out64(j.G, k)});
    c1.push_back(CholDesc{j.G, k, Rp, k, k1, X.flag, 0.0, j.keep, j.eta});
    ap.push_back(GemmJob{j.n, k1, k1, op64(src, true, lds), op64(Rp, false, k), out64(dst, ldd)});
    if (k2 == 0) continue;
    l21.push_back(GemmJob{k2, k1, k1, op64(j.G + (size_t)k1 * k, true, k), op64(Rp, false, k), out64(L21, k1)});
    cp.push_back(perm4(j.G + (size_t)k1 * k + k1, 0, S, 0, {1, 1, k2, k2}, {0, 0, k, 1}, {0, 0, k2, 1}));
    GemmJob sj{k2, k2, k1, op64(L21, true, k1), op64(L21, true, k1), out64(S, k2)};
    sj.alpha = -1.0;
    sj.beta = 1;
    s22.push_back(sj);
    c2.push_back(CholDesc{S, k2, Rp + (size_t)k1 * k + k1, k, k2, X.flag, 0.0,
                          j.keep ? j.keep + k1 : nullptr, j.eta});
    t2.push_back(GemmJob{k1, k2, k2, op64(L21, false, k1), op64(Rp + (size_t)k1 * k + k1, false, k), out64(T2, k2)});
    GemmJob xj{k1, k2, k1, op64(Rp, true, k), op64(T2, false, k2), out64(Rp + k1, k)};
    xj.alpha = -1.0;
    x12.push_back(xj);
    ap.push_back(GemmJob{j.n, k2, k, op64(src, true, lds), op64(Rp + k1, false, k), out64(dst + k1, ldd)});
  }
  auto chol = [&](const std::vector<CholDesc>& cd) {
    if (cd.empty()) return;
    Launch l;
    l.kind = LK::Chol;
    l.off = P.push(cd);
    l.n = (int)cd.size();
    l.maxa = kRegMax;
    l.maxb = 1;
    l.cls = qc.chol_inv;
    for (auto& c : cd) l.flops += 2.0 / 3.0 * c.k * (double)c.k * c.k;
    P.launches.push_back(l);
  };
  add_gemm(P, X.sb, Mode::F64, gj, qc.gram, 0);
  chol(c1);
  add_gemm(P, X.sb, Mode::F64, l21, "qr_block", 0);
  add_perm(P, cp, "qr_block");
  add_gemm(P, X.sb, Mode::F64, s22, "qr_block", 0);
  chol(c2);
  add_gemm(P, X.sb, Mode::F64, t2, "qr_block", 0);
  add_gemm(P, X.sb, Mode::F64, x12, "qr_block", 0);
  add_gemm(P, X.sb, Mode::F64, ap, qc.apply, 0);
}

// One Newton-Schulz pass Q <- Q (3 I - Q^T Q) / 2 for Q with nearly
// orthonormal columns (zero columns allowed): the Gram GEMM, G <- (3 I - G)/2
// and the product, from X to the temp T on even passes and back on odd ones
// (the ping-pong of the Cholesky passes).  It takes an orthogonality error e
// to (3/4) e^2 without a Cholesky factorization; the span is unchanged and Q
// moves by O(e).
void add_polish_pass(Ctx& X, Program& P, const std::vector<CholQRJob>& jobs, int pass, bool gauge) {
  if (jobs.empty()) return;
  const QrClasses qc = qr_classes(gauge);
  std::vector<GemmJob> gj, ap;
  std::vector<PolishDesc> pd;
  int maxk = 1;
  for (auto& j : jobs) {
    double* src = pass % 2 == 1 ? j.T : j.X;
    double* dst = pass % 2 == 1 ? j.X : j.T;
    const int lds = pass % 2 == 1 ? j.k : j.ld;
    const int ldd = pass % 2 == 1 ? j.ld : j.k;
    gj.push_back(GemmJob{j.k, j.k, j.n, op64(src, false, lds), op64(src, false, lds), out64(j.G, j.k)});
    pd.push_back(PolishDesc{j.G, j.k});
    ap.push_back(GemmJob{j.n, j.k, j.k, op64(src, true, lds), op64(j.G, false, j.k), out64(dst, ldd)});
    maxk = std::max(maxk, j.k);
  }
  add_gemm(P, X.sb, Mode::F64, gj, qc.gram, 0);
  add_simple(P, LK::Polish, pd, maxk, gauge ? "gauge_polish" : "qr_polish");
  add_gemm(P, X.sb, Mode::F64, ap, qc.apply, 0);
}

// One pass of the register path: G = X^T X, R^{-1} from the register
// Cholesky, X R^{-1} into the other buffer of the ping-pong.
void add_cholqr_fast_pass(Ctx& X, Program& P, const std::vector<CholQRJob>& jobs, int pass, bool gauge) {
  const QrClasses qc = qr_classes(gauge);
  std::vector<GemmJob> gj, tj;
  std::vector<CholDesc> cd;
  int maxk = 1;
  for (auto& j : jobs) {
    double* src = pass % 2 == 1 ? j.T : j.X;
    double* dst = pass % 2 == 1 ? j.X : j.T;
    const int lds = pass % 2 == 1 ? j.k : j.ld;
    const int ldd = pass % 2 == 1 ? j.ld : j.k;
    gj.push_back(GemmJob{j.k, j.k, j.n, op64(src, false, lds), op64(src, false, lds), out64(j.G, j.k)});
    double* Rp = j.R + (size_t)(pass % 2) * j.k * j.k;
    CholDesc c{j.G, j.k, Rp, j.k, j.k, X.flag};
    c.keep = j.keep;
    c.eta = j.eta;
    cd.push_back(c);
    tj.push_back(GemmJob{j.n, j.k, j.k, op64(src, true, lds), op64(Rp, false, j.k), out64(dst, ldd)});
    maxk = std::max(maxk, j.k);
  }
  add_gemm(P, X.sb, Mode::F64, gj, qc.gram, 0);
  Launch l;
  l.kind = LK::Chol;
  l.off = P.push(cd);
  l.n = (int)cd.size();
  l.maxa = maxk;
  l.maxb = 1;
  l.cls = qc.chol_inv;
  for (auto& j : jobs) l.flops += 2.0 / 3.0 * j.k * (double)j.k * j.k;
  P.launches.push_back(l);
  add_gemm(P, X.sb, Mode::F64, tj, qc.apply, 0);
}

// `polish_last`: the last of the passes is a Newton-Schulz step instead of a
// Cholesky pass (needs the temp T; the earlier passes leave Q orthonormal to
// far better than 1 so the step converges).
void add_cholqr(Ctx& X, Program& P, const std::vector<CholQRJob>& jobs, int passes, bool gauge = false,
                bool polish_last = false) {
  if (jobs.empty()) return;
  const QrClasses qc = qr_classes(gauge);
  bool fast = true, blocked = true, temp = true;
  for (auto& j : jobs) {
    fast = fast && j.k <= kRegMax && !j.Rout && j.T;
    blocked = blocked && j.k <= 2 * kRegMax && !j.Rout && j.T;
    temp = temp && j.T && !j.Rout;
  }
  if (polish_last && temp) {
    // Cholesky passes first (through whichever path fits), then the step
    for (int pass = 0; pass + 1 < passes; ++pass) {
      if (fast) add_cholqr_fast_pass(X, P, jobs, pass, gauge);
      else if (blocked) add_chol_inv_blocked(X, P, jobs, pass, gauge);
      else throw Error{MPO_ERR_UNSUPPORTED, "polished Cholesky-QR: k above 2 kRegMax"};
    }
    add_polish_pass(X, P, jobs, passes - 1, gauge);
    if (passes % 2 == 1) {
      std::vector<PermDesc> cp;
      for (auto& j : jobs)
        cp.push_back(perm4(j.T, 0, j.X, 0, {1, 1, j.n, j.k}, {0, 0, j.k, 1}, {0, 0, j.ld, 1}));
      add_perm(P, cp, "copy");
    }
    return;
  }
  if (!fast && blocked) {
    for (int pass = 0; pass < passes; ++pass) add_chol_inv_blocked(X, P, jobs, pass, gauge);
    if (passes % 2 == 1) {
      std::vector<PermDesc> cp;
      for (auto& j : jobs)
        cp.push_back(perm4(j.T, 0, j.X, 0, {1, 1, j.n, j.k}, {0, 0, j.k, 1}, {0, 0, j.ld, 1}));
      add_perm(P, cp, "copy");
    }
    return;
  }
  for (int pass = 0; pass < passes; ++pass) {
    std::vector<GemmJob> gj, tj;
    std::vector<CholDesc> cd;
    std::vector<TrsmDesc> td;
    int maxk = 1, maxn = 1;
    for (auto& j : jobs) {
      double* src = (fast && pass % 2 == 1) ? j.T : j.X;
      double* dst = (fast && pass % 2 == 1) ? j.X : j.T;
      const int lds = (fast && pass % 2 == 1) ? j.k : j.ld;
      const int ldd = (fast && pass % 2 == 1) ? j.ld : j.k;
      gj.push_back(GemmJob{j.k, j.k, j.n, op64(src, false, lds), op64(src, false, lds), out64(j.G, j.k)});
      double* Rp = j.Rout ? j.R : j.R + (size_t)(pass % 2) * j.k * j.k;
      CholDesc c{j.G, j.k, Rp, j.k, j.k, X.flag};
      if (j.shifted && pass == 0 && !fast) c.shift = chol_shift(j.n, j.k);
      c.keep = j.keep;
      c.eta = j.eta;
      cd.push_back(c);
      if (fast)
        tj.push_back(GemmJob{j.n, j.k, j.k, op64(src, true, lds), op64(Rp, false, j.k), out64(dst, ldd)});
      else
        td.push_back(TrsmDesc{j.X, j.ld, Rp, j.k, j.n, j.k});
      maxk = std::max(maxk, j.k);
      maxn = std::max(maxn, j.n);
    }
    add_gemm(P, X.sb, Mode::F64, gj, qc.gram, 0);
    Launch l;
    l.kind = LK::Chol;
    l.off = P.push(cd);
    l.n = (int)cd.size();
    l.maxa = maxk;
    l.maxb = fast ? 1 : 0;
    l.cls = fast ? qc.chol_inv : qc.chol;
    for (auto& j : jobs) l.flops += (fast ? 2.0 : 1.0) / 3.0 * j.k * (double)j.k * j.k;
    P.launches.push_back(l);
    if (fast) add_gemm(P, X.sb, Mode::F64, tj, qc.apply, 0);
    else add_simple(P, LK::Trsm, td, maxn, "qr_trsm");
    // Rout <- R_pass Rout (the second R block is the product's temp)
    std::vector<GemmJob> rj;
    std::vector<PermDesc> pc;
    for (auto& j : jobs) {
      if (!j.Rout) continue;
      const size_t kk = (size_t)j.k * j.k;
      if (pass == 0) {
        pc.push_back(perm4(j.R, 0, j.Rout, 0, {1, 1, j.k, j.k}, {0, 0, j.k, 1}, {0, 0, j.k, 1}));
      } else {
        rj.push_back(GemmJob{j.k, j.k, j.k, op64(j.R, true, j.k), op64(j.Rout, false, j.k),
                             out64(j.R + kk, j.k)});
        pc.push_back(perm4(j.R + kk, 0, j.Rout, 0, {1, 1, j.k, j.k}, {0, 0, j.k, 1}, {0, 0, j.k, 1}));
      }
    }
    add_gemm(P, X.sb, Mode::F64, rj, "qr_rprod", 0);
    add_perm(P, pc, "copy");
  }
  if (fast && passes % 2 == 1) {
    std::vector<PermDesc> cp;
    for (auto& j : jobs)
      cp.push_back(perm4(j.T, 0, j.X, 0, {1, 1, j.n, j.k}, {0, 0, j.k, 1}, {0, 0, j.ld, 1}));
    add_perm(P, cp, "copy");
  }
}

// ------------------------------------------------------------------ allocation
void carve(Ctx& X, Carver& cv) {
  const int wb = bytes_of(X.wt);
  const bool bf = X.wmode == Mode::BF16 || X.wmode == Mode::BF16X3;
  auto amax = [&](void) -> unsigned* { return bf ? cv.take<unsigned>(1) : nullptr; };
  X.flag = cv.take<int>(4);
  X.sweep_dev = X.flag + 1;
  Caps all;
  size_t max_bonds = 1;
  for (auto& P : X.pairs) {
    const int L = P.L, dd = P.dd;
    Caps c = pair_caps(P, X.o);
    all.nm_max = std::max(all.nm_max, c.nm_max);
    all.kmax = std::max(all.kmax, c.kmax);
    all.rmax = std::max(all.rmax, c.rmax);
    all.theta = std::max(all.theta, c.theta);
    all.T = std::max(all.T, c.T);
    all.ext = std::max(all.ext, c.ext);
    max_bonds = std::max<size_t>(max_bonds, (size_t)(L / 2 + 1));
    P.A64.resize(L); P.B64.resize(L); P.C64.resize(L);
    P.Bw.resize(L); P.Bmw.resize(L); P.At.resize(L); P.Amt.resize(L);
    P.amBw.resize(L); P.amBmw.resize(L); P.amAt.resize(L); P.amAmt.resize(L);
    for (int i = 0; i < L; ++i) {
      P.A64[i] = cv.take<double>((size_t)P.chiA_in[i] * P.dA * P.chiA_in[i + 1]);
      P.B64[i] = cv.take<double>((size_t)P.chiB_in[i] * P.dB * P.chiB_in[i + 1]);
      // C holds the initial guess unclipped (A or the given C) before its
      // right-orthogonalization, and the fit's bonds afterwards
      P.C64[i] = cv.take<double>((size_t)std::max(P.capC[i], init_dim(P, i)) * dd *
                                 std::max(P.capC[i + 1], init_dim(P, i + 1)));
      const size_t na = (size_t)P.cA[i] * P.dA * P.cA[i + 1], nb = (size_t)P.cB[i] * P.dB * P.cB[i + 1];
      P.At[i] = cv.take<char>(na * wb); P.Amt[i] = cv.take<char>(na * wb);
      P.Bw[i] = cv.take<char>(nb * wb); P.Bmw[i] = cv.take<char>(nb * wb);
      P.amAt[i] = amax(); P.amAmt[i] = amax(); P.amBw[i] = amax(); P.amBmw[i] = amax();
    }
    P.Lenv.assign(L + 1, nullptr); P.Renv.assign(L + 1, nullptr);
    P.amL.assign(L + 1, nullptr); P.amR.assign(L + 1, nullptr);
    for (int b = 0; b <= L; ++b) {
      const size_t ne = (size_t)P.capC[b] * P.cA[b] * P.cB[b];
      P.Lenv[b] = cv.take<char>(ne * wb);
      P.Renv[b] = cv.take<char>(ne * wb);
      P.amL[b] = amax(); P.amR[b] = amax();
    }
    P.XL.assign(L - 1, nullptr); P.XR.assign(L - 1, nullptr);
    P.amXL.assign(L - 1, nullptr); P.amXR.assign(L - 1, nullptr);
    for (int i = 0; i + 1 < L; ++i) {
      const size_t w = (size_t)P.cA[i + 1] * P.cB[i + 1] * dd;
      P.XL[i] = cv.take<char>(w * P.capC[i] * wb);
      P.XR[i] = cv.take<char>(w * P.capC[i + 2] * wb);
      P.amXL[i] = amax(); P.amXR[i] = amax();
    }
    P.Yv.assign(L + 1, nullptr);
    for (int b = 1; b < L; ++b) P.Yv[b] = cv.take<double>(P.capC[b]);
    P.nu_dev = cv.take<double>(2);
    P.rk = X.o.tau > 0.0 ? cv.take<int>((size_t)L + 1) : nullptr;
  }
  const size_t nscr = X.o.schedule == MPO_SCHED_SERIAL     ? 1
                      : X.o.schedule == MPO_SCHED_PARALLEL ? X.parts.size()
                                                           : max_bonds * X.pairs.size();
  X.scratch.resize(nscr);
  const long long nm = all.nm_max, kx = all.kmax, rx = all.rmax;
  for (auto& B : X.scratch) {
    B.theta = cv.take<char>((size_t)all.theta * wb);
    B.T = cv.take<char>((size_t)all.T * wb);
    B.amT = amax();
    B.omega = cv.take<double>((size_t)nm * kx);
    B.Y = cv.take<double>((size_t)nm * kx);
    B.Y2 = cv.take<double>((size_t)nm * kx);
    B.G = cv.take<double>((size_t)kx * kx);
    B.R = cv.take<double>(2 * (size_t)kx * kx);
    B.Bk = cv.take<double>((size_t)kx * nm);
    B.H = cv.take<double>((size_t)kx * kx);
    B.eigw = cv.take<double>(eig_work_doubles((int)kx, (int)rx));
    B.evals = cv.take<double>((size_t)kx);
    B.Z = cv.take<double>((size_t)kx * rx);
    B.S = cv.take<double>((size_t)rx);
    B.V = cv.take<double>((size_t)nm * rx);
    B.sign = cv.take<double>((size_t)rx);
    B.keep = cv.take<double>((size_t)rx);
    B.SVt = cv.take<double>((size_t)rx * nm);
    B.diag = X.o.tau > 0.0 ? cv.take<double>((size_t)kx) : nullptr;
  }
  // initialization scratch (FP64): Gram / triangular factors and a core-sized temp
  long long core_max = 1, kq = 1;
  for (auto& P : X.pairs)
    for (int i = 0; i < P.L; ++i) {
      const long long a = std::max(init_dim(P, i), P.capC[i]), b = std::max(init_dim(P, i + 1), P.capC[i + 1]);
      core_max = std::max({core_max, a * P.dd * b, (long long)P.chiB_in[i] * P.dB * P.chiB_in[i + 1],
                           (long long)P.chiA_in[i] * P.dA * P.chiA_in[i + 1]});
      kq = std::max({kq, a, b, (long long)P.chiB_in[i], (long long)P.chiB_in[i + 1], (long long)P.chiA_in[i],
                     (long long)P.chiA_in[i + 1]});
    }
  X.iG = cv.take<double>((size_t)kq * kq);
  X.iR1 = cv.take<double>(2 * (size_t)kq * kq);
  X.iR2 = cv.take<double>((size_t)kq * kq);
  X.iRt = cv.take<double>((size_t)kq * kq);
  X.iTmp = cv.take<double>((size_t)core_max);
  X.iXt = cv.take<double>((size_t)core_max);
  X.iJ = cv.take<double>((size_t)kq * kq);
  X.iTau = cv.take<double>((size_t)kq);
  if (X.o.schedule == MPO_SCHED_EVEN_ODD) {
    X.iH = cv.take<double>((size_t)kq * kq);
    X.iZ = cv.take<double>((size_t)kq * kq);
    X.iEw = cv.take<double>(eig_work_doubles((int)kq, (int)kq));
    X.iEv = cv.take<double>((size_t)kq);
    X.iSg = cv.take<double>((size_t)kq);
  }
  X.iTmpN = core_max;
  // split-K partial tiles and their counters
  X.sb.cap = (size_t)512 * 128 * 128 * 8;
  X.sb.partials = cv.take<char>(X.sb.cap);
  X.sb.ccap = 1 << 16;
  X.sb.counters = cv.take<int>(X.sb.ccap);
  X.arena_cap = (size_t)64 << 20;
  X.arena = cv.take<char>(X.arena_cap);
  if (X.o.track_error) {
    X.err.C.assign(X.pairs.size(), {});
    int Lmax = 1;
    for (size_t p = 0; p < X.pairs.size(); ++p) {
      const PairState& P = X.pairs[p];
      Lmax = std::max(Lmax, P.L);
      for (int i = 0; i < P.L; ++i)
        X.err.C[p].push_back(cv.take<double>((size_t)P.capC[i] * P.dd * P.capC[i + 1]));
    }
    X.err.logs = cv.take<double>(3 * (size_t)(Lmax + 1));
    X.err.part = cv.take<double>(1024);
    X.err.region_bytes = err_region_bytes(X);
    X.err.region = cv.take<char>(X.err.region_bytes);
  }
}

// ------------------------------------------------------------------ extension jobs
// left step 1 at site i: T[(c,a), (t,u,b')] = Lenv[i][(c,a), b] Bw[i][b, (t,u,b')]
GemmJob job_e1(const Ctx& X, const PairState& P, int i, void* T, unsigned* amT) {
  const int M = P.cC[i] * P.cA[i], K = P.cB[i], N = P.dB * P.cB[i + 1];
  return GemmJob{M, N, K, opW(X, P.Lenv[i], true, K, P.amL[i]), opW(X, P.Bw[i], false, N, P.amBw[i]),
                 outW(X, T, N, amT)};
}
// left step 2 at site i: XL[i][c][s][u][a'][b'] = sum_(a,t) At[i][(a,t)][s][a'] T[c][(a,t)][u][b']
// (s over d, t over d, u over du)
GemmJob job_e2(const Ctx& X, const PairState& P, int i, const void* T, const unsigned* amT) {
  const int d = P.d, du = P.du, a0 = P.cA[i], a1 = P.cA[i + 1], b1 = P.cB[i + 1];
  GemmJob g{a1, b1, d * a0, opW(X, P.At[i], false, d * a1, P.amAt[i]),
            opW(X, T, false, du * b1, amT), outW(X, P.XL[i], b1, P.amXL[i])};
  g.nb[0] = P.cC[i]; g.nb[1] = d; g.nb[2] = du;
  g.A.s[0] = 0; g.A.s[1] = a1; g.A.s[2] = 0;
  g.B.s[0] = (long long)a0 * P.dB * b1; g.B.s[1] = 0; g.B.s[2] = b1;
  g.C.s[0] = (long long)P.dd * a1 * b1; g.C.s[1] = (long long)du * a1 * b1; g.C.s[2] = (long long)a1 * b1;
  return g;
}
// right step 1 at site j: T[(c'',a''), (t,u,b)] = Renv[j+1][(c'',a''), b''] Bmw[j][b'', (t,u,b)]
GemmJob job_e1m(const Ctx& X, const PairState& P, int j, void* T, unsigned* amT) {
  const int M = P.cC[j + 1] * P.cA[j + 1], K = P.cB[j + 1], N = P.dB * P.cB[j];
  return GemmJob{M, N, K, opW(X, P.Renv[j + 1], true, K, P.amR[j + 1]),
                 opW(X, P.Bmw[j], false, N, P.amBmw[j]), outW(X, T, N, amT)};
}
// right step 2 at site j: XR[j-1][c''][s][u][a][b] = sum_(a'',t) Amt[j][(a'',t)][s][a] T[c''][(a'',t)][u][b]
GemmJob job_e2m(const Ctx& X, const PairState& P, int j, const void* T, const unsigned* amT) {
  const int d = P.d, du = P.du, a0 = P.cA[j], a1 = P.cA[j + 1], b0 = P.cB[j];
  GemmJob g{a0, b0, d * a1, opW(X, P.Amt[j], false, d * a0, P.amAmt[j]),
            opW(X, T, false, du * b0, amT), outW(X, P.XR[j - 1], b0, P.amXR[j - 1])};
  g.nb[0] = P.cC[j + 1]; g.nb[1] = d; g.nb[2] = du;
  g.A.s[0] = 0; g.A.s[1] = a0; g.A.s[2] = 0;
  g.B.s[0] = (long long)a1 * P.dB * b0; g.B.s[1] = 0; g.B.s[2] = b0;
  g.C.s[0] = (long long)P.dd * a0 * b0; g.C.s[1] = (long long)du * a0 * b0; g.C.s[2] = (long long)a0 * b0;
  return g;
}
double flops_e1(const PairState& P, int i) { return 2.0 * P.cC[i] * P.cA[i] * P.cB[i] * P.dB * P.cB[i + 1]; }
double flops_e2(const PairState& P, int i) { return 2.0 * P.cC[i] * P.dd * P.d * P.cA[i] * P.cA[i + 1] * P.cB[i + 1]; }
double flops_e1m(const PairState& P, int j) { return 2.0 * P.cC[j + 1] * P.cA[j + 1] * P.cB[j + 1] * P.dB * P.cB[j]; }
double flops_e2m(const PairState& P, int j) { return 2.0 * P.cC[j + 1] * P.dd * P.d * P.cA[j + 1] * P.cA[j] * P.cB[j]; }

// ------------------------------------------------------------------ initialization
// Shifted Cholesky-QR3 of an initialization step (the R factors multiplied
// into iRt), rank-revealing: a dependent column (a core of lower rank than
// its bond, e.g. an unused bond state) becomes a zero column of Q with a zero
// row of R instead of a failure, where Householder QR would complete Q with
// an arbitrary orthonormal column of the same (zero) weight.
// Householder QR of the n x k matrix Xm (row-major, n >= k) for the
// canonical forms of the initialization: the reflectors overwrite Xm, R
// (diag >= 0, row-major) goes to X.iRt and Q (n x k, row-major, leading
// dimension k) to Qout.  Unlike Cholesky-QR, whose backward error carries
// the squared condition number of the first pass, Householder QR keeps
// the small singular directions of the graded factors that the sweeps
// carry from core to core, which the inverse gauge then divides by.
void add_hhqr_group(Program& P, const std::vector<HhqrDesc>& ds, const char* cls) {
  if (ds.empty()) return;
  int mm = 1, nn = 1;
  for (auto& d : ds) { mm = std::max(mm, d.m); nn = std::max(nn, d.n); }
  add_simple(P, LK::Hhqr, ds, mm, cls);
  P.launches.back().maxb = nn;
}

// The one-kernel LDS form when the panel fits, except in the even/odd
// schedule's initialization: its inverse canonical form amplifies the QR's
// rounding to about 1e-10 of the resumed half-step (reading 24), which was
// measured with the two-kernel form (Q applied forward to [I; 0]).
void add_hhqr(Ctx& X, Program& P, double* Xm, int n, int k, double* Qout) {
  if (n < k) throw Error{MPO_ERR_SHAPE, "Householder QR needs rows >= columns"};
  if (X.o.schedule != MPO_SCHED_EVEN_ODD && hhqr_fits_lds(n, k)) {  // one kernel, the panel in LDS
    add_hhqr_group(P, {HhqrDesc{Xm, n, k, k, X.iTau, Qout, k, X.iRt, k}}, "init");
    return;
  }
  add_simple(P, LK::Geqr, std::vector<GeqrDesc>{GeqrDesc{Xm, n, k, k, X.iRt, k, X.iTau}}, 0, "init");
  add_simple(P, LK::Orgqr, std::vector<OrgqrDesc>{OrgqrDesc{Xm, n, k, k, X.iTau, Qout, k, X.iRt, k}}, 0,
             "init");
}

// Left-orthogonalization (Alg. 5 preprocessing) of one MPO held in `cores`,
// whose input bond dims are `chi_in`; `out_dims` are the clipped dims.
// QR sweep over sites start .. stop-1 of `cores` (bond dims `cur`, updated):
// each core left-orthogonalized by Householder QR with R carried into the
// next core, or clipped (identity core, everything carried) where it has
// fewer rows than columns.
void rec_qr_sweep(Ctx& X, Program& P, PairState& S, std::vector<double*>& cores, std::vector<int>& cur,
                  int stop, int start = 0, int pd = 0) {
  const int dd = pd > 0 ? pd : S.dd;  // physical size of a core of this train
  for (int i = start; i < stop; ++i) {
    const int p = cur[i] * dd, q = cur[i + 1];
    const int nn = dd * cur[i + 2];  // columns of the next core (its right bond untouched yet)
    if (p >= q) {
      add_hhqr(X, P, cores[i], p, q, X.iTmp);
      add_perm(P, {perm4(X.iTmp, 0, cores[i], 0, {1, 1, p, q}, {0, 0, q, 1}, {0, 0, q, 1})}, "copy");
      add_gemm(P, X.sb, Mode::F64, {GemmJob{q, nn, q, op64(X.iRt, true, q), op64(cores[i + 1], false, nn),
                                            out64(X.iTmp, nn)}}, "init", 0);
    } else {
      add_gemm(P, X.sb, Mode::F64, {GemmJob{p, nn, q, op64(cores[i], true, q), op64(cores[i + 1], false, nn),
                                            out64(X.iTmp, nn)}}, "init", 0);
      add_fill(P, {FillDesc{cores[i], 0, p, p, 1}});
      cur[i + 1] = p;
    }
    add_perm(P, {perm4(X.iTmp, 0, cores[i + 1], 0, {1, 1, cur[i + 1], nn}, {0, 0, nn, 1}, {0, 0, nn, 1})}, "copy");
  }
}

// RQ sweep over sites start .. stop+1 of C (start < 0: from L-1; bond dims
// `cur`, updated): each core right-orthogonalized (X^T = Q R, X = R^T Q^T)
// with R^T carried into the previous core, or clipped.
void rec_rq_sweep(Ctx& X, Program& P, PairState& S, std::vector<int>& cur, int stop, int start = -1) {
  const int L = S.L, dd = S.dd;
  for (int j = start < 0 ? L - 1 : start; j > stop; --j) {
    const int p = cur[j], q = dd * cur[j + 1];
    const int mp = cur[j - 1] * dd;  // rows of the previous core
    if (p <= q) {
      add_perm(P, {perm4(S.C64[j], 0, X.iXt, 0, {1, 1, p, q}, {0, 0, q, 1}, {0, 0, 1, p})}, "copy");
      add_hhqr(X, P, X.iXt, q, p, X.iTmp);
      add_perm(P, {perm4(X.iTmp, 0, S.C64[j], 0, {1, 1, q, p}, {0, 0, p, 1}, {0, 0, 1, q})}, "copy");
      add_gemm(P, X.sb, Mode::F64, {GemmJob{mp, p, p, op64(S.C64[j - 1], true, p), op64(X.iRt, true, p),
                                            out64(X.iTmp, p)}}, "init", 0);
      add_perm(P, {perm4(X.iTmp, 0, S.C64[j - 1], 0, {1, 1, mp, p}, {0, 0, p, 1}, {0, 0, p, 1})}, "copy");
    } else {
      add_gemm(P, X.sb, Mode::F64, {GemmJob{mp, q, p, op64(S.C64[j - 1], true, p), op64(S.C64[j], false, q),
                                            out64(X.iTmp, q)}}, "init", 0);
      add_perm(P, {perm4(X.iTmp, 0, S.C64[j - 1], 0, {1, 1, mp, q}, {0, 0, q, 1}, {0, 0, q, 1})}, "copy");
      add_fill(P, {FillDesc{S.C64[j], 0, q, q, 1}});
      cur[j] = q;
    }
  }
}

void check_dims(const std::vector<int>& cur, const std::vector<int>& want, const char* what) {
  if (cur != want) throw Error{MPO_ERR_SHAPE, std::string(what) + " shape plan mismatch"};
}

// Left-orthogonalization (Alg. 5 preprocessing) of one MPO held in `cores`,
// whose input bond dims are `chi_in`; `out_dims` are the clipped dims.  With
// `nu`, the norm is split off the last core into *nu.
void rec_left_orth(Ctx& X, Program& P, PairState& S, std::vector<double*>& cores,
                   const std::vector<int>& chi_in, const std::vector<int>& out_dims, double* nu, int pd = 0) {
  const int L = S.L, dd = pd > 0 ? pd : S.dd;
  std::vector<int> cur(chi_in);
  rec_qr_sweep(X, P, S, cores, cur, L - 1, 0, dd);
  check_dims(cur, out_dims, "left orthogonalization");
  if (nu)
    add_simple(P, LK::Norm, std::vector<NormDesc>{NormDesc{cores[L - 1], (long long)cur[L - 1] * dd, nu}}, 0,
               "init");
}

// The initial C (A, or the given guess) right-orthogonalized by an RQ sweep
// L..2 (Sec. 2.3.1).
const std::vector<int>& guess_dims(const PairState& S) {
  return S.C_in.empty() ? (S.mps ? S.cB : S.cA) : S.chiC_in;
}

void rec_right_orth(Ctx& X, Program& P, PairState& S) {
  std::vector<int> cur(guess_dims(S));
  rec_rq_sweep(X, P, S, cur, 0);
  check_dims(cur, S.cC, "right orthogonalization");
}

// The initial C in site-canonical form around sites i0, i0+1 (Sec. 2.3.1):
// QR sweep over the sites left of them, RQ sweep over the sites right of them.
void rec_mixed_orth(Ctx& X, Program& P, PairState& S, int i0) {
  std::vector<int> cur(guess_dims(S));
  rec_qr_sweep(X, P, S, S.C64, cur, i0);
  rec_rq_sweep(X, P, S, cur, i0 + 1);
  check_dims(cur, S.cC, "mixed orthogonalization");
}

void rec_repack(Ctx& X, Program& P, PairState& S) {
  const int L = S.L, d = S.d, du = S.du, dA = S.dA, dB = S.dB;
  const int tw = X.wt == DType::F64 ? 0 : 1;
  std::vector<PermDesc> ds;
  for (int i = 0; i < L; ++i) {
    const long long a0 = S.cA[i], a1 = S.cA[i + 1], b0 = S.cB[i], b1 = S.cB[i + 1];
    // B [b][t][u][b'] -> Bw same, Bmw [b'][t][u][b]  (t over d, u over du)
    PermDesc p1 = perm4(S.B64[i], 0, S.Bw[i], tw, {(int)b0, d, du, (int)b1}, {dB * b1, du * b1, b1, 1},
                        {dB * b1, du * b1, b1, 1});
    p1.amax = S.amBw[i];
    PermDesc p2 = perm4(S.B64[i], 0, S.Bmw[i], tw, {(int)b0, d, du, (int)b1}, {dB * b1, du * b1, b1, 1},
                        {1, du * b0, b0, dB * b0});
    p2.amax = S.amBmw[i];
    // A [a][s][t][a'] -> At [a][t][s][a'], Amt [a'][t][s][a]
    PermDesc p3 = perm4(S.A64[i], 0, S.At[i], tw, {(int)a0, d, d, (int)a1}, {dA * a1, d * a1, a1, 1},
                        {dA * a1, a1, d * a1, 1});
    p3.amax = S.amAt[i];
    PermDesc p4 = perm4(S.A64[i], 0, S.Amt[i], tw, {(int)a0, d, d, (int)a1}, {dA * a1, d * a1, a1, 1},
                        {1, a0, d * a0, dA * a0});
    p4.amax = S.amAmt[i];
    ds.insert(ds.end(), {p1, p2, p3, p4});
  }
  add_perm(P, ds, "init");
}

// right environment of site j from Renv[j+1] (sweep or init): XR[j-1] via the
// two mirrored steps, then (if make_env) Renv[j] = CR_j . XR[j-1] where
// CR_j[c][(c'', s, u)] is C_j with its right bond first.
void rec_right_env_from_core(Ctx& X, Program& P, PairState& S, int j, bool make_env, BondScratch& B,
                             const double* core = nullptr) {
  add_gemm(P, X.sb, X.wmode, {job_e1m(X, S, j, B.T, B.amT)}, "env_ext1", flops_e1m(S, j));
  add_gemm(P, X.sb, X.wmode, {job_e2m(X, S, j, B.T, B.amT)}, "env_ext2", flops_e2m(S, j));
  if (!make_env) return;
  const int c0 = S.cC[j], c1 = S.cC[j + 1], dd = S.dd, N = S.cA[j] * S.cB[j];
  add_perm(P, {perm4(core ? core : S.C64[j], 0, X.iXt, 0, {c0, dd, c1, 1}, {(long long)dd * c1, c1, 1, 0},
                     {(long long)c1 * dd, 1, dd, 0})}, "copy");
  add_gemm(P, X.sb, X.wmode, {GemmJob{c0, N, c1 * dd, op64(X.iXt, true, c1 * dd),
                                      opW(X, S.XR[j - 1], false, N, S.amXR[j - 1]),
                                      outW(X, S.Renv[j], N, S.amR[j])}},
           "env_update", 2.0 * c0 * N * c1 * dd);
}

void rec_left_env_from_core(Ctx& X, Program& P, PairState& S, int i, const double* Ci, int ldc,
                            BondScratch& B) {
  add_gemm(P, X.sb, X.wmode, {job_e1(X, S, i, B.T, B.amT)}, "env_ext1", flops_e1(S, i));
  add_gemm(P, X.sb, X.wmode, {job_e2(X, S, i, B.T, B.amT)}, "env_ext2", flops_e2(S, i));
  const int c0 = S.cC[i], c1 = S.cC[i + 1], dd = S.dd, N = S.cA[i + 1] * S.cB[i + 1];
  add_gemm(P, X.sb, X.wmode, {GemmJob{c1, N, c0 * dd, op64(Ci, false, ldc),
                                      opW(X, S.XL[i], false, N, S.amXL[i]),
                                      outW(X, S.Lenv[i + 1], N, S.amL[i + 1])}},
           "env_update", 2.0 * c1 * N * c0 * dd);
}

// ------------------------------------------------------------------ two-site update
// One bond of one pair inside a program: shapes of the bond (from the host
// copy of the current bond dims) and the buffers it uses.
struct BondJob {
  PairState* P;
  int pair;
  int i;       // 0-based bond: joins sites i and i+1
  bool fwd;    // serial direction (ignored by the inverse gauge)
  BondScratch* B;
  int n, m, k, r;
  bool sketch;
  bool tr = false;  // plain SVD from the m x m Gram Theta^T Theta (m < n)
};

BondJob make_bond(Ctx& X, PairState& P, int pair, int i, bool fwd, BondScratch& B) {
  BondJob b{&P, pair, i, fwd, &B};
  b.n = P.cC[i] * P.dd;
  b.m = P.dd * P.cC[i + 2];
  const int cap = P.rcap[i + 1];
  const int kmax = std::min(std::min(b.n, b.m), cap);
  b.r = std::min(P.chi_max, kmax);
  b.sketch = X.o.sketch_p >= 0 && P.chi_max + X.o.sketch_p < std::min(b.n, b.m);
  if (b.sketch) b.k = std::min(P.chi_max + X.o.sketch_p, kmax);
  else b.k = b.n;
  if (b.sketch && b.k >= std::min(b.n, b.m)) { b.sketch = false; b.k = b.n; }
  if (!b.sketch && b.m < b.n) { b.tr = true; b.k = b.m; }
  return b;
}

// Records the two-site matrix and its truncated factorization (Alg. 3 /
// Sec. 3.1) for a group of bonds: Theta = XL XR^T; with the sketch
// Y = Theta Omega, Q = CholeskyQR2(Y), Bk = Q^T Theta; without it Bk = Theta
// (Q = I); then the top r eigenpairs of H = Bk Bk^T give U_b = Z and
// S = sqrt(lambda).  The extensions XL, XR must be current.
void rec_factor(Ctx& X, Program& P, std::vector<BondJob>& bj, int stream_mul, int stream_add_base,
                bool halfstep) {
  std::vector<GemmJob> th, yj, bk, hj;
  std::vector<OmegaDesc> om;
  std::vector<CholQRJob> qr;
  std::vector<EigDesc> ed;
  std::vector<SvalDesc> sv;
  std::vector<ScaleDesc> mz;
  std::vector<FillDesc> omz;
  std::vector<PermDesc> dg;
  std::vector<TruncDesc> tr;
  const bool tol = X.o.tau > 0.0;
  long long maxz = 1;
  bool reg = true;  // every eigenproblem on the register path
  double fth = 0, fsk = 0;
  long long maxom = 1;
  int maxr = 1;
  for (auto& b : bj) {
    PairState& S = *b.P;
    BondScratch& B = *b.B;
    const int K = S.cA[b.i + 1] * S.cB[b.i + 1];
    th.push_back(GemmJob{b.n, b.m, K, opW(X, S.XL[b.i], true, K), opW(X, S.XR[b.i], true, K),
                         outW(X, B.theta, b.m)});
    fth += 2.0 * b.n * b.m * K;
    if (b.sketch) {
      OmegaDesc o{};
      o.out = B.omega; o.m = b.m; o.k = b.k; o.chi = S.cC[b.i + 2]; o.dd = S.dd;
      o.bond = b.i + 1; o.pair = b.pair; o.stream_mul = stream_mul; o.stream_add = stream_add_base;
      o.stream_base = X.sweep_dev; o.seed = X.o.seed;
      if (tol) {  // the bond's current shape lies inside the buffer's
        o.rk = S.rk; o.kk = S.chi_max + X.o.sketch_p; o.cap = S.rcap[b.i + 1];
        omz.push_back(FillDesc{B.omega, 2LL * b.m * b.k, 0, 0, 0});
      }
      om.push_back(o);
      maxom = std::max(maxom, (long long)b.m * b.k);
      yj.push_back(GemmJob{b.n, b.k, b.m, opW(X, B.theta, true, b.m), op64(B.omega, false, b.k),
                           out64(B.Y, b.k)});
      CholQRJob qj{B.Y, b.n, b.k, b.k, B.G, B.R, nullptr, B.Y2};
      qj.eta = kRankEta;  // a sketch of a rank-deficient Theta has dependent columns
      qr.push_back(qj);
      bk.push_back(GemmJob{b.k, b.m, b.n, op64(B.Y, false, b.k), opW(X, B.theta, false, b.m),
                           out64(B.Bk, b.m)});
      hj.push_back(GemmJob{b.k, b.k, b.m, op64(B.Bk, true, b.m), op64(B.Bk, true, b.m), out64(B.H, b.k)});
      fsk += 4.0 * b.n * b.m * b.k;
    } else if (b.tr) {  // eigenvectors of Theta^T Theta are V
      hj.push_back(GemmJob{b.m, b.m, b.n, opW(X, B.theta, false, b.m), opW(X, B.theta, false, b.m),
                           out64(B.H, b.m)});
    } else {
      hj.push_back(GemmJob{b.n, b.n, b.m, opW(X, B.theta, true, b.m), opW(X, B.theta, true, b.m),
                           out64(B.H, b.n)});
    }
    ed.push_back(EigDesc{B.H, b.k, b.k, b.r, B.evals, B.Z, b.r, B.eigw, X.flag});
    reg = reg && b.k <= kRegMax;
    sv.push_back(SvalDesc{B.evals, B.S, b.r, 0, X.flag, B.keep, tol ? nullptr : X.flag + 2});
    if (tol) {  // the Gram matrix's trace is the sum of all sigma^2
      dg.push_back(perm4(B.H, 0, B.diag, 0, {1, 1, 1, b.k}, {0, 0, 0, (long long)b.k + 1}, {0, 0, 0, 1}));
      const double t = X.o.tau / S.L;
      tr.push_back(TruncDesc{B.diag, b.k, b.r, B.evals, B.S, B.keep, S.rk, b.i + 1, S.dd, S.chi_max,
                             S.rcap[b.i + 1], t * t, X.flag + 2});
    }
    // the eigenvectors of dropped values become exact zero columns
    mz.push_back(ScaleDesc{B.Z, B.Z, b.k, b.r, b.r, b.r, nullptr, B.keep, 0, 2});
    maxr = std::max(maxr, b.r);
    maxz = std::max(maxz, (long long)b.k * b.r);
  }
  add_gemm(P, X.sb, X.wmode, th, "theta", fth);
  add_fill(P, omz);
  add_simple(P, LK::Omega, om, maxom, "omega");
  add_gemm(P, X.sb, Mode::F64, yj, "sketch", fsk / 2);
  // range finder: a rank-revealing Cholesky-QR pass, then a Newton-Schulz step
  if (!qr.empty()) add_cholqr(X, P, qr, 2, false, true);
  add_gemm(P, X.sb, Mode::F64, bk, "project", fsk / 2);
  // split H jobs by operand type (sketched: FP64 Bk; plain: working-type Theta)
  std::vector<GemmJob> h64, hw;
  for (auto& h : hj) (h.A.t == DType::F64 ? h64 : hw).push_back(h);
  add_gemm(P, X.sb, Mode::F64, h64, "gram", 0);
  add_gemm(P, X.sb, Mode::F64, hw, "gram", 0);
  add_perm(P, dg, "svals");
  add_eig(P, X.sb, ed, reg, "eig");
  add_simple(P, LK::Sval, sv, maxr, "svals");
  add_simple(P, LK::Trunc, tr, 0, "svals");
  add_simple(P, LK::Scale, mz, maxz, "scale");
  (void)halfstep;
}

// Site-canonical assignment (Alg. 3) and environment update for a group of
// bonds that all move in the same direction.
//   forward:  U = orth(Q Z) -> C_i;   C_{i+1} = U^T Theta;  L_{i+1} = U^T XL
//   backward: V = orth(Bk^T Z S^-1) -> C_{i+1} = V^T;  C_i = Q Z S;  R_{i+1} = V^T XR
// with the sign rule applied to the columns of U (or of C_i = U S).
void rec_assign_site(Ctx& X, Program& P, std::vector<BondJob>& bj) {
  std::vector<GemmJob> uq, tq, svt, envg, vj;
  std::vector<PermDesc> cp, cpv, perm;
  std::vector<CholQRJob> orth;
  std::vector<SignDesc> sg;
  std::vector<ScaleDesc> sc0, sc1, sc2, sc3;
  double fenv = 0;
  int maxr = 1;
  long long maxsc = 1;
  const bool fwd = bj.front().fwd;
  for (auto& b : bj) {
    PairState& S = *b.P;
    BondScratch& B = *b.B;
    const int i = b.i, r = b.r, cl = S.cC[i], cr = S.cC[i + 2], dd = S.dd;
    const int N = S.cA[i + 1] * S.cB[i + 1];
    double* Ci = S.C64[i];
    double* Cn = S.C64[i + 1];
    // C_i <- Q Z (or Z); with the m-side Gram C_i <- Theta V (= U S)
    if (b.sketch)
      uq.push_back(GemmJob{b.n, r, b.k, op64(B.Y, true, b.k), op64(B.Z, false, r), out64(Ci, r)});
    else if (b.tr)
      tq.push_back(GemmJob{b.n, r, b.m, opW(X, B.theta, true, b.m), op64(B.Z, false, r), out64(Ci, r)});
    else
      cp.push_back(perm4(B.Z, 0, Ci, 0, {1, 1, b.n, r}, {0, 0, r, 1}, {0, 0, r, 1}));
    maxr = std::max(maxr, r);
    if (fwd && b.tr) sc0.push_back(ScaleDesc{Ci, Ci, b.n, r, r, r, nullptr, B.S, 0, 1});
    if (fwd) {
      CholQRJob oj{Ci, b.n, r, r, B.G, B.R, nullptr, B.Y2};
      oj.keep = B.keep;
      orth.push_back(oj);
      sg.push_back(SignDesc{Ci, b.n, r, r, B.sign, nullptr});
      svt.push_back(GemmJob{r, b.m, b.n, op64(Ci, false, r), opW(X, B.theta, false, b.m), out64(B.SVt, b.m)});
      // C_{i+1}[c'][su][c''] = SVt[c'][(c'', su)]
      perm.push_back(perm4(B.SVt, 0, Cn, 0, {r, cr, dd, 1}, {b.m, dd, 1, 0},
                           {(long long)dd * cr, 1, cr, 0}));
      envg.push_back(GemmJob{r, N, b.n, op64(Ci, false, r), opW(X, S.XL[i], false, N, S.amXL[i]),
                             outW(X, S.Lenv[i + 1], N, S.amL[i + 1])});
      fenv += 2.0 * r * N * b.n;
    } else {
      // V = Bk^T Z / S  (Bk = Theta without the sketch); V = Z from the m-side Gram
      if (b.tr) {
        cpv.push_back(perm4(B.Z, 0, B.V, 0, {1, 1, b.m, r}, {0, 0, r, 1}, {0, 0, r, 1}));
      } else {
        if (b.sketch)
          vj.push_back(GemmJob{b.m, r, b.k, op64(B.Bk, false, b.m), op64(B.Z, false, r), out64(B.V, r)});
        else
          vj.push_back(GemmJob{b.m, r, b.n, opW(X, B.theta, false, b.m), op64(B.Z, false, r),
                               out64(B.V, r)});
        sc1.push_back(ScaleDesc{B.V, B.V, b.m, r, r, r, nullptr, B.S, 0, 1});
        CholQRJob oj{B.V, b.m, r, r, B.G, B.R, nullptr, B.Y2};
        oj.keep = B.keep;
        orth.push_back(oj);
        sc2.push_back(ScaleDesc{Ci, Ci, b.n, r, r, r, nullptr, B.S, 0, 0});  // C_i = U S
      }
      sg.push_back(SignDesc{Ci, b.n, r, r, B.sign, nullptr});
      sc3.push_back(ScaleDesc{B.V, B.V, b.m, r, r, r, nullptr, B.sign, 0, 0});
      // C_{i+1}[c'][su][c''] = V[(c'', su)][c']
      perm.push_back(perm4(B.V, 0, Cn, 0, {r, cr, dd, 1}, {1, (long long)dd * r, r, 0},
                           {(long long)dd * cr, 1, cr, 0}));
      envg.push_back(GemmJob{r, N, b.m, op64(B.V, false, r), opW(X, S.XR[i], false, N, S.amXR[i]),
                             outW(X, S.Renv[i + 1], N, S.amR[i + 1])});
      fenv += 2.0 * r * N * b.m;
    }
    // the bond's singular values, kept for read-out
    perm.push_back(perm4(B.S, 0, S.Yv[i + 1], 0, {1, 1, 1, r}, {0, 0, 0, 1}, {0, 0, 0, 1}));
    maxsc = std::max(maxsc, (long long)std::max(b.n, b.m) * r);
    (void)cl;
  }
  add_gemm(P, X.sb, Mode::F64, uq, "assemble", 0);
  add_gemm(P, X.sb, Mode::F64, tq, "assemble", 0);
  add_perm(P, cp, "copy");
  // U = Q Z (or V) is orthonormal up to the eigenvectors' rounding: one
  // Newton-Schulz step restores it to working accuracy
  if (fwd) {
    add_simple(P, LK::Scale, sc0, maxsc, "scale");
    add_cholqr(X, P, orth, 1, true, true);
    add_simple(P, LK::Sign, sg, maxr, "sign");
    add_gemm(P, X.sb, Mode::F64, svt, "assemble", 0);
    add_perm(P, perm, "copy");
  } else {
    add_gemm(P, X.sb, Mode::F64, vj, "assemble", 0);
    add_perm(P, cpv, "copy");
    add_simple(P, LK::Scale, sc1, maxsc, "scale");
    add_cholqr(X, P, orth, 1, true, true);
    add_simple(P, LK::Scale, sc2, maxsc, "scale");
    add_simple(P, LK::Sign, sg, maxr, "sign");
    add_simple(P, LK::Scale, sc3, maxsc, "scale");
    add_perm(P, perm, "copy");
  }
  add_gemm(P, X.sb, X.wmode, envg, "env_update", fenv);
}

// BF16 per-tensor scales: the amax slots a bond is about to produce start at 0.
void rec_reset_amax(Ctx& X, Program& P, std::vector<unsigned*> slots) {
  if (X.wmode != Mode::BF16 && X.wmode != Mode::BF16X3) return;
  std::vector<FillDesc> fd;
  for (auto* s : slots)
    if (s) fd.push_back(FillDesc{s, 1, 0, 0, 0});
  add_fill(P, fd);
}

// One serial update at bond i in direction fwd (Alg. 5 body): the fresh
// extension (XL forward, XR backward; the other one is cached), then the
// factorization, the assignment and the environment update.
void rec_serial_bond(Ctx& X, Program& P, PairState& S, int pair, int i, bool fwd) {
  BondScratch& B = X.scratch[0];
  if (fwd) {
    rec_reset_amax(X, P, {B.amT, S.amXL[i], S.amL[i + 1]});
    add_gemm(P, X.sb, X.wmode, {job_e1(X, S, i, B.T, B.amT)}, "env_ext1", flops_e1(S, i));
    add_gemm(P, X.sb, X.wmode, {job_e2(X, S, i, B.T, B.amT)}, "env_ext2", flops_e2(S, i));
  } else {
    rec_reset_amax(X, P, {B.amT, S.amXR[i], S.amR[i + 1]});
    add_gemm(P, X.sb, X.wmode, {job_e1m(X, S, i + 1, B.T, B.amT)}, "env_ext1", flops_e1m(S, i + 1));
    add_gemm(P, X.sb, X.wmode, {job_e2m(X, S, i + 1, B.T, B.amT)}, "env_ext2", flops_e2m(S, i + 1));
  }
  std::vector<BondJob> bj{make_bond(X, S, pair, i, fwd, B)};
  rec_factor(X, P, bj, 1, 0, false);
  rec_assign_site(X, P, bj);
  S.cC[i + 1] = bj[0].r;
}

// Inverse canonical form of the right-canonical C (Sec. 2.3.1): a left-to-
// right SVD sweep X_i = carry C_i = U S V^T, Psi_i = U S, S kept per bond
// (Y_i = 1/S), carry S V^T into the next core.  The SVD keeps small singular
// values accurate (A's Schmidt values can span many orders of magnitude):
// shifted CholeskyQR3 X = Q R, then one-sided Jacobi on R Z (Z from the
// eigenvectors of R^T R as a preconditioner).
// Then the environments: L_{i+1} from Psi_i Y_i = U_i, R_j from
// Y_{j-1} Psi_j (rows of Psi_j divided by S_{j-1}).
void rec_inverse_canonical(Ctx& X, Program& P, PairState& S) {
  const int L = S.L, dd = S.dd;
  BondScratch& B = X.scratch[0];
  for (int i = 0; i + 1 < L; ++i) {
    const int p = S.cC[i] * dd, q = S.cC[i + 1], nn = dd * S.cC[i + 2];
    if (q > 512 || p < q) throw Error{MPO_ERR_UNSUPPORTED, "inverse canonical form: bond above 512"};
    double* Xi = S.C64[i];
    // X = Q R (Householder; Q into iXt, R into iRt)
    add_hhqr(X, P, Xi, p, q, X.iXt);
    // precondition: W0 = R Z with Z the eigenvectors of R^T R (its columns
    // are then orthogonal up to clusters of tiny singular values), then
    // one-sided Jacobi on W0: W0 V' = Ur diag(S) with high relative accuracy
    add_gemm(P, X.sb, Mode::F64, {GemmJob{q, q, q, op64(X.iRt, false, q), op64(X.iRt, false, q),
                                          out64(X.iH, q)}}, "init", 0);
    const bool reg = q <= kRegMax;
    add_eig(P, X.sb, {EigDesc{X.iH, q, q, q, X.iEv, X.iZ, q, X.iEw, X.flag}}, reg, "init");
    // Z orthonormal to working precision (two Newton-Schulz steps, iZ -> iJ
    // -> iZ): Jacobi returns the left singular vectors of R Z, which are
    // those of R only for an orthogonal Z, and eigenvectors of tiny, close
    // eigenvalues of R^T R come out orthogonal only to about
    // eps ||R||^2 / gap
    const std::vector<CholQRJob> zj{CholQRJob{X.iZ, q, q, q, X.iG, X.iR1, nullptr, X.iJ}};
    add_polish_pass(X, P, zj, 0, false);
    add_polish_pass(X, P, zj, 1, false);
    add_gemm(P, X.sb, Mode::F64, {GemmJob{q, q, q, op64(X.iRt, true, q), op64(X.iZ, false, q),
                                          out64(X.iG, q)}}, "init", 0);
    {
      Launch l;
      l.kind = LK::Jacobi;
      l.off = P.push(std::vector<JacobiDesc>{
          JacobiDesc{X.iG, q, q, X.iR2, q, S.Yv[i + 1], X.iJ, kDrop, X.flag + 2}});
      l.n = 1;
      l.maxa = q;
      l.cls = "init";
      P.launches.push_back(l);
    }
    // U = Q Ur (into iTmp), sign rule on U, the same flips on Ur
    add_gemm(P, X.sb, Mode::F64, {GemmJob{p, q, q, op64(X.iXt, true, q), op64(X.iR2, false, q),
                                          out64(X.iTmp, q)}}, "init", 0);
    add_simple(P, LK::Sign, std::vector<SignDesc>{SignDesc{X.iTmp, p, q, q, X.iSg, nullptr}}, q, "init");
    add_simple(P, LK::Scale, std::vector<ScaleDesc>{ScaleDesc{X.iR2, X.iR2, q, q, q, q, nullptr, X.iSg, 0, 0}},
               (long long)q * q, "init");
    // Psi_i = U S
    add_simple(P, LK::Scale, std::vector<ScaleDesc>{ScaleDesc{X.iTmp, Xi, p, q, q, q, nullptr, S.Yv[i + 1], 0, 0}},
               (long long)p * q, "init");
    // carry S V^T = Ur^T R (W0 V' = R Z V' = Ur S), into the next core
    add_gemm(P, X.sb, Mode::F64, {GemmJob{q, q, q, op64(X.iR2, false, q), op64(X.iRt, false, q),
                                          out64(X.iG, q)}}, "init", 0);
    add_gemm(P, X.sb, Mode::F64, {GemmJob{q, nn, q, op64(X.iG, true, q), op64(S.C64[i + 1], false, nn),
                                          out64(X.iTmp, nn)}}, "init", 0);
    add_perm(P, {perm4(X.iTmp, 0, S.C64[i + 1], 0, {1, 1, q, nn}, {0, 0, nn, 1}, {0, 0, nn, 1})}, "init");
  }
  const int f64 = X.wt == DType::F64 ? 1 : 0;
  add_fill(P, {FillDesc{S.Lenv[0], 0, 1, 1, f64}, FillDesc{S.Renv[L], 0, 1, 1, f64}});
  std::vector<unsigned*> sl{S.amL[0], S.amR[L], B.amT};
  for (int j = 1; j < L; ++j) sl.insert(sl.end(), {S.amR[j], S.amL[j], S.amXR[j - 1], S.amXL[j - 1]});
  rec_reset_amax(X, P, sl);
  for (int i = 0; i + 2 < L; ++i) {  // L_{i+1} from U_i = Psi_i / S_{i+1}
    const int p = S.cC[i] * dd, q = S.cC[i + 1];
    add_simple(P, LK::Scale, std::vector<ScaleDesc>{ScaleDesc{S.C64[i], X.iTmp, p, q, q, q, nullptr,
                                                              S.Yv[i + 1], 0, 1}}, (long long)p * q, "init");
    rec_left_env_from_core(X, P, S, i, X.iTmp, q, B);
  }
  for (int j = L - 1; j >= 2; --j) {  // R_j from Y_{j-1} Psi_j
    const int p = S.cC[j], q = dd * S.cC[j + 1];
    add_simple(P, LK::Scale, std::vector<ScaleDesc>{ScaleDesc{S.C64[j], X.iTmp, p, q, q, q, S.Yv[j],
                                                              nullptr, 1, 0}}, (long long)p * q, "init");
    rec_right_env_from_core(X, P, S, j, true, B, X.iTmp);
  }
}

// Inverse-gauge assignment (Alg. 4) for all bonds of a half-step:
//   U = orth(Q Z), V = orth(Bk^T Z / S) with the sign rule on U;
//   L_{i+1} = U^T XL_i, R_{i+1} = V^T XR_i;
//   Psi_i = U S, Psi_{i+1} = S V^T, Y_i = 1/S (S kept in Yv).
void rec_assign_inverse(Ctx& X, Program& P, std::vector<BondJob>& bj) {
  std::vector<GemmJob> uq, vj, envl, envr;
  std::vector<PermDesc> cp, perm;
  std::vector<CholQRJob> orthU, orthV;
  std::vector<SignDesc> sg;
  std::vector<ScaleDesc> sv1, sv2, su, sv3;
  std::vector<PermDesc> cpS;
  double fenv = 0;
  int maxr = 1;
  long long maxsc = 1;
  for (auto& b : bj) {
    PairState& S = *b.P;
    BondScratch& B = *b.B;
    const int i = b.i, r = b.r, cr = S.cC[i + 2], dd = S.dd;
    const int N = S.cA[i + 1] * S.cB[i + 1];
    double* Ci = S.C64[i];
    double* Cn = S.C64[i + 1];
    if (b.sketch)
      uq.push_back(GemmJob{b.n, r, b.k, op64(B.Y, true, b.k), op64(B.Z, false, r), out64(Ci, r)});
    else if (b.tr)
      uq.push_back(GemmJob{b.n, r, b.m, opW(X, B.theta, true, b.m), op64(B.Z, false, r), out64(Ci, r)});
    else
      cp.push_back(perm4(B.Z, 0, Ci, 0, {1, 1, b.n, r}, {0, 0, r, 1}, {0, 0, r, 1}));
    if (b.tr) {  // V = Z, U = Theta V / S
      cp.push_back(perm4(B.Z, 0, B.V, 0, {1, 1, b.m, r}, {0, 0, r, 1}, {0, 0, r, 1}));
      sv1.push_back(ScaleDesc{Ci, Ci, b.n, r, r, r, nullptr, B.S, 0, 1});
    } else {
      if (b.sketch)
        vj.push_back(GemmJob{b.m, r, b.k, op64(B.Bk, false, b.m), op64(B.Z, false, r), out64(B.V, r)});
      else
        vj.push_back(GemmJob{b.m, r, b.n, opW(X, B.theta, false, b.m), op64(B.Z, false, r),
                             out64(B.V, r)});
      sv1.push_back(ScaleDesc{B.V, B.V, b.m, r, r, r, nullptr, B.S, 0, 1});
    }
    CholQRJob ou{Ci, b.n, r, r, B.G, B.R, nullptr, B.Y2};
    ou.keep = B.keep;
    orthU.push_back(ou);
    // runs after orthU in stream order, so it reuses the same G and R scratch
    CholQRJob ov{B.V, b.m, r, r, B.G, B.R, nullptr, B.SVt};
    ov.keep = B.keep;
    orthV.push_back(ov);
    sg.push_back(SignDesc{Ci, b.n, r, r, B.sign, nullptr});
    sv2.push_back(ScaleDesc{B.V, B.V, b.m, r, r, r, nullptr, B.sign, 0, 0});
    envl.push_back(GemmJob{r, N, b.n, op64(Ci, false, r), opW(X, S.XL[i], false, N, S.amXL[i]),
                           outW(X, S.Lenv[i + 1], N, S.amL[i + 1])});
    envr.push_back(GemmJob{r, N, b.m, op64(B.V, false, r), opW(X, S.XR[i], false, N, S.amXR[i]),
                           outW(X, S.Renv[i + 1], N, S.amR[i + 1])});
    fenv += 2.0 * r * N * (b.n + b.m);
    su.push_back(ScaleDesc{Ci, Ci, b.n, r, r, r, nullptr, B.S, 0, 0});      // Psi_i = U S
    sv3.push_back(ScaleDesc{B.V, B.V, b.m, r, r, r, nullptr, B.S, 0, 0});   // V S
    perm.push_back(perm4(B.V, 0, Cn, 0, {r, cr, dd, 1}, {1, (long long)dd * r, r, 0},
                         {(long long)dd * cr, 1, cr, 0}));                  // Psi_{i+1} = S V^T
    cpS.push_back(perm4(B.S, 0, S.Yv[i + 1], 0, {1, 1, 1, r}, {0, 0, 0, 1}, {0, 0, 0, 1}));
    // truncation before inversion: the dropped values are already zero in S
    // and their columns in Z, hence in U and V
    maxr = std::max(maxr, r);
    maxsc = std::max(maxsc, (long long)std::max(b.n, b.m) * r);
  }
  add_gemm(P, X.sb, Mode::F64, uq, "assemble", 0);
  add_gemm(P, X.sb, Mode::F64, vj, "assemble", 0);
  add_perm(P, cp, "copy");
  add_simple(P, LK::Scale, sv1, maxsc, "scale");
  // U = Q Z and V = B_k^T Z / S are orthonormal up to rounding: one
  // Newton-Schulz step each
  add_cholqr(X, P, orthU, 1, true, true);
  add_cholqr(X, P, orthV, 1, true, true);
  add_simple(P, LK::Sign, sg, maxr, "sign");
  add_simple(P, LK::Scale, sv2, maxsc, "scale");
  add_gemm(P, X.sb, X.wmode, envl, "env_update", fenv / 2);
  add_gemm(P, X.sb, X.wmode, envr, "env_update", fenv / 2);
  add_simple(P, LK::Scale, su, maxsc, "scale");
  add_simple(P, LK::Scale, sv3, maxsc, "scale");
  add_perm(P, perm, "copy");
  add_perm(P, cpS, "copy");
}

// One half-step q of the even/odd schedule (all pairs): bonds with
// (1-based) index = 1 (mod 2) for q = 0, = 0 (mod 2) for q = 1.
void rec_half_step(Ctx& X, Program& P, int q) {
  std::vector<BondJob> bj;
  std::vector<GemmJob> e1, e2, e1m, e2m;
  std::vector<unsigned*> slots;
  double f1 = 0, f2 = 0, f1m = 0, f2m = 0;
  size_t si = 0;
  for (size_t p = 0; p < X.pairs.size(); ++p) {
    PairState& S = X.pairs[p];
    for (int i = 0; i + 1 < S.L; ++i) {
      const int bond = i + 1;
      if ((bond % 2 == 1) != (q == 0)) continue;
      BondScratch& B = X.scratch.at(si++);
      bj.push_back(make_bond(X, S, (int)p, i, true, B));
      e1.push_back(job_e1(X, S, i, B.T, B.amT));
      e2.push_back(job_e2(X, S, i, B.T, B.amT));
      e1m.push_back(job_e1m(X, S, i + 1, B.T, B.amT));
      e2m.push_back(job_e2m(X, S, i + 1, B.T, B.amT));
      f1 += flops_e1(S, i); f2 += flops_e2(S, i); f1m += flops_e1m(S, i + 1); f2m += flops_e2m(S, i + 1);
      slots.insert(slots.end(), {B.amT, S.amXL[i], S.amXR[i], S.amL[i + 1], S.amR[i + 1]});
    }
  }
  rec_reset_amax(X, P, slots);
  add_gemm(P, X.sb, X.wmode, e1, "env_ext1", f1);
  add_gemm(P, X.sb, X.wmode, e2, "env_ext2", f2);
  std::vector<unsigned*> tslots;
  for (auto& b : bj) tslots.push_back(b.B->amT);
  rec_reset_amax(X, P, tslots);
  add_gemm(P, X.sb, X.wmode, e1m, "env_ext1", f1m);
  add_gemm(P, X.sb, X.wmode, e2m, "env_ext2", f2m);
  rec_factor(X, P, bj, 2, q, true);
  rec_assign_inverse(X, P, bj);
  for (auto& b : bj) b.P->cC[b.i + 1] = b.r;
}

// ------------------------------------------------------------------ parallel schedule
// Site-canonical parallel fit (Sec. 4, variant II) on one device: every
// sub-TT is one member of a grouped update.  A bond of a group is updated
// in one of four modes: forward (Alg. 3: C_i = U, C_{i+1} = S V^T, L_{i+1}),
// backward (C_i = U S, C_{i+1} = V^T, R_{i+1}), a connection between two
// sub-TTs' centres (C_i = U S for the left one, C_{i+1} = S V^T for the
// right one, both L_{i+1} and R_{i+1} rebuilt: each sub-TT keeps its own
// gauge), or forward with a fresh right extension (the merge's first level).
struct ParBond {
  int i;     // 0-based bond: sites i, i+1
  int mode;  // 0 forward, 1 backward, 2 connection, 3 forward with a fresh XR
};

// Second half of a connection (after the forward assignment left C_i = U,
// S V^T in SVt, C_{i+1} = S V^T and L_{i+1}): V = (S V^T)^T S^-1 (zero for
// dropped values), re-orthonormalized as in the backward assignment,
// R_{i+1} = V^T XR, then C_i = U S.
void rec_assign_conn(Ctx& X, Program& P, std::vector<BondJob>& bj) {
  std::vector<PermDesc> tp;
  std::vector<ScaleDesc> sv, us;
  std::vector<CholQRJob> orth;
  std::vector<GemmJob> envg;
  double fenv = 0;
  long long maxsc = 1;
  for (auto& b : bj) {
    PairState& S = *b.P;
    BondScratch& B = *b.B;
    const int i = b.i, r = b.r, N = S.cA[i + 1] * S.cB[i + 1];
    tp.push_back(perm4(B.SVt, 0, B.V, 0, {1, 1, r, b.m}, {0, 0, b.m, 1}, {0, 0, 1, r}));
    sv.push_back(ScaleDesc{B.V, B.V, b.m, r, r, r, nullptr, B.S, 0, 1});
    CholQRJob oj{B.V, b.m, r, r, B.G, B.R, nullptr, B.Y2};
    oj.keep = B.keep;
    orth.push_back(oj);
    envg.push_back(GemmJob{r, N, b.m, op64(B.V, false, r), opW(X, S.XR[i], false, N, S.amXR[i]),
                           outW(X, S.Renv[i + 1], N, S.amR[i + 1])});
    fenv += 2.0 * r * N * b.m;
    us.push_back(ScaleDesc{S.C64[i], S.C64[i], b.n, r, r, r, nullptr, B.S, 0, 0});
    maxsc = std::max(maxsc, (long long)std::max(b.n, b.m) * r);
  }
  add_perm(P, tp, "copy");
  add_simple(P, LK::Scale, sv, maxsc, "scale");
  add_cholqr(X, P, orth, 1, true, true);
  add_gemm(P, X.sb, X.wmode, envg, "env_update", fenv);
  add_simple(P, LK::Scale, us, maxsc, "scale");
}

// One group of bond updates of the parallel schedule (at most one per
// sub-TT, so no two share an environment): the fresh extensions (XL for
// modes 0, 2, 3; XR for 1, 2, 3: the ones a mode needs on both sides go in
// a second pair of launches, as each bond has one first-step scratch), the
// factorizations with Omega of stream 4 * set + stream_add, the
// assignments.
void rec_par_group(Ctx& X, Program& P, PairState& S, const std::vector<ParBond>& bonds, int stream_add) {
  if (bonds.empty()) return;
  std::vector<GemmJob> e1, e2, e1m, e2m;
  std::vector<unsigned*> slots, slots2;
  double f1 = 0, f2 = 0, f1m = 0, f2m = 0;
  std::vector<BondJob> bj;
  for (size_t q = 0; q < bonds.size(); ++q) {
    BondScratch& B = X.scratch.at(q);
    const int i = bonds[q].i, mode = bonds[q].mode;
    if (mode != 1) {  // XL in the first pair
      e1.push_back(job_e1(X, S, i, B.T, B.amT));
      e2.push_back(job_e2(X, S, i, B.T, B.amT));
      f1 += flops_e1(S, i);
      f2 += flops_e2(S, i);
      slots.insert(slots.end(), {B.amT, S.amXL[i], S.amL[i + 1]});
    }
    if (mode != 0) {  // XR: alone in the first pair, after XL in the second
      auto& a = mode == 1 ? e1 : e1m;
      auto& c = mode == 1 ? e2 : e2m;
      a.push_back(job_e1m(X, S, i + 1, B.T, B.amT));
      c.push_back(job_e2m(X, S, i + 1, B.T, B.amT));
      (mode == 1 ? f1 : f1m) += flops_e1m(S, i + 1);
      (mode == 1 ? f2 : f2m) += flops_e2m(S, i + 1);
      auto& sl = mode == 1 ? slots : slots2;
      sl.insert(sl.end(), {B.amT, S.amXR[i], S.amR[i + 1]});
    }
    bj.push_back(make_bond(X, S, 0, i, mode != 1, B));
  }
  rec_reset_amax(X, P, slots);
  add_gemm(P, X.sb, X.wmode, e1, "env_ext1", f1);
  add_gemm(P, X.sb, X.wmode, e2, "env_ext2", f2);
  if (!e1m.empty()) {
    rec_reset_amax(X, P, slots2);
    add_gemm(P, X.sb, X.wmode, e1m, "env_ext1", f1m);
    add_gemm(P, X.sb, X.wmode, e2m, "env_ext2", f2m);
  }
  rec_factor(X, P, bj, 4, stream_add, false);
  std::vector<BondJob> fw, bw, cn;
  for (size_t q = 0; q < bonds.size(); ++q) {
    (bonds[q].mode == 1 ? bw : fw).push_back(bj[q]);
    if (bonds[q].mode == 2) cn.push_back(bj[q]);
  }
  if (!fw.empty()) rec_assign_site(X, P, fw);
  if (!bw.empty()) rec_assign_site(X, P, bw);
  if (!cn.empty()) rec_assign_conn(X, P, cn);
  for (auto& b : bj) S.cC[b.i + 1] = b.r;
}

// Phase q of a set: 0 every F sub-TT sweeps forward over its inner bonds and
// every B one backward (in lockstep, one group per step), 1 the F|B
// connections, 2 F backward and B forward, 3 the B|F connections.
void rec_par_phase(Ctx& X, Program& P, PairState& S, int q, int stream_add) {
  const auto& parts = X.parts;
  const int np = (int)parts.size();
  if (q == 0 || q == 2) {
    int steps = 0;
    for (auto& p : parts) steps = std::max(steps, p.second - p.first);
    for (int k = 0; k < steps; ++k) {
      std::vector<ParBond> bonds;
      for (int n = 0; n < np; ++n) {
        const int s = parts[n].first, e = parts[n].second;
        if (k >= e - s) continue;
        const bool fwd = (n % 2 == 0) == (q == 0);
        bonds.push_back(ParBond{fwd ? s + k : e - 1 - k, fwd ? 0 : 1});
      }
      rec_par_group(X, P, S, bonds, stream_add);
    }
  } else {
    std::vector<ParBond> bonds;
    for (int n = q == 1 ? 0 : 1; n + 1 < np; n += 2) bonds.push_back(ParBond{parts[n].second, 2});
    rec_par_group(X, P, S, bonds, stream_add);
  }
}

// The binary merge: phase 0 once more (stream 4 n_sets), forward updates
// at every F|B boundary with a fresh XR (level 1: each pair of sub-TTs
// becomes one site-canonical train, centre right of the boundary), then
// level t >= 2 joins adjacent groups of 2^(t-1) sub-TTs: QR sweep of the
// left group from its centre to the boundary and its left environments,
// RQ sweep of the right group from its centre back to the boundary and its
// right environments, one forward update at the boundary (stream
// 4 n_sets + t).
void rec_par_merge(Ctx& X, Program& P, PairState& S) {
  const auto& parts = X.parts;
  const int np = (int)parts.size();
  rec_par_phase(X, P, S, 0, 0);
  std::vector<ParBond> first;
  for (int n = 0; n + 1 < np; n += 2) first.push_back(ParBond{parts[n].second, 3});
  rec_par_group(X, P, S, first, 1);
  int level = 2;
  for (int size = 2; size < np; size *= 2, ++level) {
    for (int g = 0; g < np; g += 2 * size) {
      const int m = parts[g + size - 1].second;
      const int ol = parts[g + size / 2 - 1].second + 1;
      const int orr = parts[g + size + size / 2 - 1].second + 1;
      BondScratch& B = X.scratch[0];
      rec_qr_sweep(X, P, S, S.C64, S.cC, m, ol);
      for (int i = ol; i < m; ++i) {
        rec_reset_amax(X, P, {B.amT, S.amXL[i], S.amL[i + 1]});
        rec_left_env_from_core(X, P, S, i, S.C64[i], S.cC[i + 1], B);
      }
      rec_rq_sweep(X, P, S, S.cC, m + 1, orr);
      for (int j = orr; j >= m + 1; --j) {
        rec_reset_amax(X, P, {B.amT, S.amXR[j - 1], S.amR[j]});
        rec_right_env_from_core(X, P, S, j, j >= m + 2, B);
      }
      rec_par_group(X, P, S, {ParBond{m, 0}}, level);
    }
  }
}

std::string shape_key(const Ctx& X, const char* tag) {
  std::string k(tag);
  for (auto& P : X.pairs)
    for (int c : P.cC) k += "," + std::to_string(c);
  return k;
}

void upload(Ctx& X, Program& P) {
  const size_t need = (P.blob.size() + 255) & ~size_t(255);
  if (X.arena_used + need > X.arena_cap) throw Error{MPO_ERR_WORKSPACE, "descriptor arena exhausted"};
  P.dev = X.arena + X.arena_used;
  P.dev_cap = need;
  X.arena_used += need;
  if (!P.blob.empty())
    HIP_OK(hipMemcpyAsync(P.dev, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice, X.stream));
}

// Init program of one pair (serial schedule): copy inputs, preprocess A and
// B, C = A right-orthogonalized, working-precision copies, trivial boundary
// environments, all right environments and the cached right extensions.
void rec_init_pair(Ctx& X, Program& P, PairState& S, int pair) {
  const int L = S.L, dd = S.dd;
  std::vector<PermDesc> cps;
  for (int i = 0; i < L; ++i) {
    const int a0 = S.chiA_in[i], a1 = S.chiA_in[i + 1], b0 = S.chiB_in[i], b1 = S.chiB_in[i + 1];
    const int dA = S.dA, dB = S.dB;
    cps.push_back(perm4(S.A_in[i], 0, S.A64[i], 0, {1, 1, a0, dA * a1}, {0, 0, (long long)dA * a1, 1},
                        {0, 0, (long long)dA * a1, 1}));
    cps.push_back(perm4(S.B_in[i], 0, S.B64[i], 0, {1, 1, b0, dB * b1}, {0, 0, (long long)dB * b1, 1},
                        {0, 0, (long long)dB * b1, 1}));
  }
  add_perm(P, cps, "init");
  rec_left_orth(X, P, S, S.A64, S.chiA_in, S.cA, S.nu_dev, S.dA);
  rec_left_orth(X, P, S, S.B64, S.chiB_in, S.cB, S.nu_dev + 1, S.dB);
  std::vector<PermDesc> cc;
  for (int i = 0; i < L; ++i) {
    if (S.C_in.empty()) {  // C = the preprocessed A (B for an MPS, whose legs are C's)
      const auto& g = S.mps ? S.B64 : S.A64;
      const auto& gc = S.mps ? S.cB : S.cA;
      cc.push_back(perm4(g[i], 0, S.C64[i], 0, {1, 1, gc[i], dd * gc[i + 1]},
                         {0, 0, (long long)dd * gc[i + 1], 1}, {0, 0, (long long)dd * gc[i + 1], 1}));
    } else {  // C = the given initial guess
      const long long c0 = S.chiC_in[i], c1 = S.chiC_in[i + 1];
      cc.push_back(perm4(S.C_in[i], 0, S.C64[i], 0, {1, 1, (int)c0, (int)(dd * c1)}, {0, 0, dd * c1, 1},
                         {0, 0, dd * c1, 1}));
    }
  }
  add_perm(P, cc, "init");
  if (X.wmode == Mode::BF16 || X.wmode == Mode::BF16X3) {
    std::vector<unsigned*> sl;
    for (int i = 0; i < L; ++i) sl.insert(sl.end(), {S.amAt[i], S.amAmt[i], S.amBw[i], S.amBmw[i]});
    rec_reset_amax(X, P, sl);
  }
  rec_repack(X, P, S);
  // singular values per bond start at zero (the serial schedule writes them
  // at each update; the inverse canonical form fills them below)
  {
    std::vector<FillDesc> fz;
    for (int b = 1; b < L; ++b) fz.push_back(FillDesc{S.Yv[b], 2LL * S.capC[b], 0, 0, 0});
    add_fill(P, fz);
  }
  const bool serial = X.o.schedule == MPO_SCHED_SERIAL;
  const bool backward_first = serial && X.o.first_sweep % 2 == 1;
  const int i0 = !serial || X.o.first_bond == 0 ? -1
                 : backward_first ? L - 2 - X.o.first_bond : X.o.first_bond;
  if (X.o.schedule == MPO_SCHED_PARALLEL) {
    // every sub-TT starts from the guess in the mixed canonical form centred
    // on it: right-orthogonalized, then left-orthogonalized (the left
    // environments are built from this form below), then right-
    // orthogonalized again (the right ones)
    std::vector<int> cur(guess_dims(S));
    rec_rq_sweep(X, P, S, cur, 0);
    rec_qr_sweep(X, P, S, S.C64, cur, L - 1);
    check_dims(cur, S.cC, "parallel initialization");
  } else if (i0 >= 0) {
    rec_mixed_orth(X, P, S, i0);
  } else if (backward_first) {
    std::vector<int> in(guess_dims(S));
    rec_left_orth(X, P, S, S.C64, in, S.cC, nullptr);
  } else {
    rec_right_orth(X, P, S);
  }
  const int f64 = X.wt == DType::F64 ? 1 : 0;
  add_fill(P, {FillDesc{S.Lenv[0], 0, 1, 1, f64}, FillDesc{S.Renv[L], 0, 1, 1, f64}});
  std::vector<unsigned*> sl{S.amL[0], S.amR[L]};
  for (int j = 1; j < L; ++j) sl.insert(sl.end(), {S.amR[j], S.amXR[j - 1], S.amL[j], S.amXL[j - 1]});
  sl.push_back(X.scratch[0].amT);
  rec_reset_amax(X, P, sl);
  if (X.o.schedule == MPO_SCHED_EVEN_ODD) {
    // the guess acts only as an operator: unit norm (its scale would enter
    // Lambda, hence Y, of the bonds a half-step leaves alone)
    add_simple(P, LK::Norm, std::vector<NormDesc>{NormDesc{S.C64[0], (long long)S.cC[0] * S.dd * S.cC[1],
                                                           X.iEv}}, 0, "init");
    rec_inverse_canonical(X, P, S);
    (void)pair;
    return;
  }
  if (X.o.schedule == MPO_SCHED_PARALLEL) {  // isometric environments on both sides
    for (int i = 0; i + 1 < L; ++i) rec_left_env_from_core(X, P, S, i, S.C64[i], S.cC[i + 1], X.scratch[0]);
    std::vector<int> cur(S.cC);
    rec_rq_sweep(X, P, S, cur, 0);
    check_dims(cur, S.cC, "parallel initialization");
    for (int j = L - 1; j >= 1; --j) rec_right_env_from_core(X, P, S, j, j >= 2, X.scratch[0]);
  } else if (i0 >= 0 && !backward_first) {  // forward from bond i0: left envs up to it, right side cached
    for (int i = 0; i < i0; ++i) rec_left_env_from_core(X, P, S, i, S.C64[i], S.cC[i + 1], X.scratch[0]);
    for (int j = L - 1; j >= i0 + 1; --j) rec_right_env_from_core(X, P, S, j, j >= i0 + 2, X.scratch[0]);
  } else if (i0 >= 0) {  // backward from bond i0: right envs down to it, left side cached
    for (int j = L - 1; j >= i0 + 2; --j) rec_right_env_from_core(X, P, S, j, true, X.scratch[0]);
    for (int i = 0; i <= i0; ++i) rec_left_env_from_core(X, P, S, i, S.C64[i], S.cC[i + 1], X.scratch[0]);
  } else if (backward_first) {  // all left environments and the cached left extensions
    for (int i = 0; i + 1 < L; ++i) rec_left_env_from_core(X, P, S, i, S.C64[i], S.cC[i + 1], X.scratch[0]);
  } else {
    for (int j = L - 1; j >= 1; --j) rec_right_env_from_core(X, P, S, j, j >= 2, X.scratch[0]);
  }
  (void)pair;
}

int n_words(size_t bytes) { return (int)((bytes + 3) / 4); }

void validate_tt(const mpo_tt& t, int L, int d) {
  if (t.L != L || t.d != d) throw Error{MPO_ERR_SHAPE, "A, B (and an initial guess) must share L and d"};
  if (!t.chi || !t.cores) throw Error{MPO_ERR_INVALID_ARG, "null bond dims or cores"};
  if (t.chi[0] != 1 || t.chi[L] != 1) throw Error{MPO_ERR_SHAPE, "boundary bond dims must be 1"};
  for (int i = 0; i <= L; ++i)
    if (t.chi[i] < 1) throw Error{MPO_ERR_SHAPE, "bond dims must be >= 1"};
  for (int i = 0; i < L; ++i)
    if (!t.cores[i]) throw Error{MPO_ERR_INVALID_ARG, "null core pointer"};
}

void setup(Ctx& X, const mpo_pair* pairs, int n_pairs, const mpo_fit_opts* o) {
  if (!pairs || n_pairs < 1 || !o) throw Error{MPO_ERR_INVALID_ARG, "null pairs/options or n_pairs < 1"};
  X.o = *o;
  if (o->chi_max < 1) throw Error{MPO_ERR_INVALID_ARG, "chi_max must be >= 1"};
  if (o->chi_max + std::max(o->sketch_p, 0) > 512)
    throw Error{MPO_ERR_UNSUPPORTED, "chi_max + sketch_p above 512"};
  if (!(o->tau >= 0.0 && o->tau < INFINITY)) throw Error{MPO_ERR_INVALID_ARG, "tau must be finite and >= 0"};
  if (o->precision < 0 || o->precision > 3) throw Error{MPO_ERR_INVALID_ARG, "bad precision"};
  if (o->schedule < 0 || o->schedule > 2) throw Error{MPO_ERR_INVALID_ARG, "bad schedule"};
  if (o->schedule == MPO_SCHED_PARALLEL) {
    if (o->n_parts < 2 || (o->n_parts & (o->n_parts - 1)))
      throw Error{MPO_ERR_INVALID_ARG, "parallel schedule: n_parts must be a power of two >= 2"};
    if (n_pairs != 1) throw Error{MPO_ERR_UNSUPPORTED, "parallel schedule: one pair"};
    if (o->tau != 0.0 || o->first_sweep != 0 || o->track_error != 0)
      throw Error{MPO_ERR_UNSUPPORTED, "parallel schedule: tau, first_sweep and track_error must be 0"};
  }
  if (o->first_sweep < 0 || o->first_sweep > (1 << 24)) throw Error{MPO_ERR_INVALID_ARG, "bad first_sweep"};
  if (o->first_bond < 0) throw Error{MPO_ERR_INVALID_ARG, "bad first_bond"};
  if (o->first_bond > 0 && (o->schedule != MPO_SCHED_SERIAL || n_pairs != 1))
    throw Error{MPO_ERR_UNSUPPORTED, "first_bond > 0 needs the serial schedule and one pair"};
  if (o->first_half < 0 || o->first_half > 1) throw Error{MPO_ERR_INVALID_ARG, "bad first_half"};
  if (o->first_half > 0 && o->schedule != MPO_SCHED_EVEN_ODD)
    throw Error{MPO_ERR_UNSUPPORTED, "first_half needs the even/odd schedule"};
  if (o->track_error < 0 || o->track_error > 1) throw Error{MPO_ERR_INVALID_ARG, "bad track_error"};
  if (o->mps < 0 || o->mps > 1) throw Error{MPO_ERR_INVALID_ARG, "bad mps"};
  if (o->mps && (o->track_error || o->schedule == MPO_SCHED_PARALLEL))
    throw Error{MPO_ERR_UNSUPPORTED, "MPO-MPS: serial or even/odd schedule, no fit-error tracking"};
  X.wmode = o->precision == MPO_FP64 ? Mode::F64
            : o->precision == MPO_FP32 ? Mode::F32
            : o->precision == MPO_BF16 ? Mode::BF16 : Mode::BF16X3;
  X.wt = o->precision == MPO_FP64 ? DType::F64 : DType::F32;
  X.profile = o->profile != 0;
  if (o->n_tune < 0 || (o->n_tune > 0 && !o->tune))
    throw Error{MPO_ERR_INVALID_ARG, "bad tuning table"};
  X.tune.assign(o->tune, o->tune + o->n_tune);
  for (auto& t : X.tune)
    if (t.tile < 0 || t.tile > 5 || t.splits < 1 || t.splits > 64)
      throw Error{MPO_ERR_INVALID_ARG, "bad tuning entry"};
  X.sb.tune = X.tune.empty() ? nullptr : &X.tune;
  X.pairs.resize(n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    const mpo_pair& pr = pairs[p];
    const int L = pr.A.L, d = pr.A.d;
    if (L < 2 || d < 1) throw Error{MPO_ERR_SHAPE, "need L >= 2 and d >= 1"};
    validate_tt(pr.A, L, d);
    validate_tt(pr.B, L, d);
    PairState& S = X.pairs[p];
    S.L = L; S.d = d; S.mps = o->mps != 0;
    S.du = S.mps ? 1 : d; S.dd = d * S.du; S.dA = d * d; S.dB = d * S.du;
    S.chiA_in.assign(pr.A.chi, pr.A.chi + L + 1);
    S.chiB_in.assign(pr.B.chi, pr.B.chi + L + 1);
    S.A_in.assign(pr.A.cores, pr.A.cores + L);
    S.B_in.assign(pr.B.cores, pr.B.cores + L);
    if (o->c_init) {
      const mpo_tt& c = o->c_init[p];
      validate_tt(c, L, d);
      S.chiC_in.assign(c.chi, c.chi + L + 1);
      S.C_in.assign(c.cores, c.cores + L);
      for (int b = 0; b <= L; ++b)
        if (S.chiC_in[b] > 512) throw Error{MPO_ERR_UNSUPPORTED, "initial guess bond above 512"};
    }
    for (int b = 0; b <= L; ++b)
      if (S.chiA_in[b] > 512 || S.chiB_in[b] > 512)
        throw Error{MPO_ERR_UNSUPPORTED, "bond dimensions above 512"};
    S.chi_max = pr.chi_max > 0 ? pr.chi_max : o->chi_max;
    if (S.chi_max + std::max(o->sketch_p, 0) > 512)
      throw Error{MPO_ERR_UNSUPPORTED, "chi_max + sketch_p above 512"};
    if (o->schedule == MPO_SCHED_PARALLEL) {
      if (L < 2 * o->n_parts) throw Error{MPO_ERR_SHAPE, "parallel schedule: every sub-TT needs two sites"};
      X.parts = partition_sites(L, o->n_parts);
    }
    plan_shapes(S, S.chi_max, o->schedule, o->first_sweep, o->first_bond, o->first_half, o->n_parts);
    if (o->first_bond > L - 2) throw Error{MPO_ERR_INVALID_ARG, "first_bond must be below L - 1"};
    for (int b = 0; b <= L; ++b)
      if (S.capC[b] * S.dd > 2048) throw Error{MPO_ERR_UNSUPPORTED, "two-site dimension above 2048"};
  }
}

void check_flags(Ctx& X) {
  int fl[4] = {0, 0, 0, 0};
  HIP_OK(hipMemcpyAsync(fl, X.flag, sizeof(fl), hipMemcpyDeviceToHost, X.stream));
  HIP_OK(hipStreamSynchronize(X.stream));
  X.n_trunc = fl[2];
  const int f = fl[0];
  if (f) {
    std::string m = "device status:";
    if (f & FLAG_NONFINITE) m += " non-finite value;";
    if (f & FLAG_CHOL) m += " Cholesky pivot <= 0;";
    if (f & FLAG_EIG) m += " eigenvalue bracket;";
    throw Error{MPO_ERR_NUMERIC, m};
  }
}

struct SweepPlan {
  Program prog;
  std::vector<std::vector<int>> cC_after;  // per pair
  bool stable = false;  // the sweep leaves the bond dimensions unchanged
  hipGraphExec_t graph = nullptr;
  int uses = 0;
};

// Units of a sweep: two-site updates (serial, per pair) or half-steps.
int sweep_units(const Ctx& X) {
  return X.o.schedule == MPO_SCHED_EVEN_ODD ? 2 : X.o.schedule == MPO_SCHED_PARALLEL ? 4 : X.pairs[0].L - 1;
}

// Records units [start, start + count) of the current sweep (direction fwd),
// and the advance of the Philox sweep counter when they end the sweep.  A
// serial segment that is not a whole sweep needs one pair (first_bond or
// mpo_fit_updates).
void record_segment(Ctx& X, SweepPlan& sp, bool fwd, int start, int count) {
  if (X.o.schedule == MPO_SCHED_EVEN_ODD) {
    for (int q = start; q < start + count; ++q) rec_half_step(X, sp.prog, q);
  } else if (X.o.schedule == MPO_SCHED_PARALLEL) {
    for (int q = start; q < start + count; ++q) rec_par_phase(X, sp.prog, X.pairs[0], q, q);
  } else {
    for (size_t p = 0; p < X.pairs.size(); ++p) {
      PairState& S = X.pairs[p];
      for (int u = start; u < start + count; ++u) {
        const int i = fwd ? u : S.L - 2 - u;
        rec_serial_bond(X, sp.prog, S, (int)p, i, fwd);
      }
    }
  }
  if (start + count == sweep_units(X)) {
    Launch b;
    b.kind = LK::Bump;
    b.counter = X.sweep_dev;
    b.bump_by = 1;
    b.cls = "bump";
    sp.prog.launches.push_back(b);
  }
  for (auto& S : X.pairs) sp.cC_after.push_back(S.cC);
}

void record_sweep(Ctx& X, SweepPlan& sp, bool fwd) { record_segment(X, sp, fwd, 0, sweep_units(X)); }


// ------------------------------------------------------------------ adjoint
// Gradient of loss(A, B) = <Pi(W), A B> at frozen truncation bases: Pi(W)
// keeps C's isometries and takes its centre core from the two-layer
// environment of (isometries, W); the gradient of the multilinear loss with
// respect to A_l (B_l) is the network with A_l (B_l) removed, closed by the
// three-layer environments of (Pi(W), A, B) (Sec. 2.3.3, Fig. envs).  Every
// contraction is one GEMM between operands brought into matrix form by the
// strided permutation kernel where their axes are not already grouped.

struct Ten {
  void* p = nullptr;
  DType t = DType::F64;
  std::vector<int> dims;
  long long size() const {
    long long n = 1;
    for (int d : dims) n *= d;
    return n;
  }
};

// Bump allocator over a caller workspace (null base: measuring only).
struct Arena {
  Carver cv;
  size_t peak = 0;
  Ten take(DType t, std::vector<int> dims) {
    Ten x;
    x.t = t;
    x.dims = std::move(dims);
    x.p = t == DType::F64 ? static_cast<void*>(cv.take<double>(x.size()))
                          : static_cast<void*>(cv.take<float>(x.size()));
    peak = std::max(peak, cv.off);
    return x;
  }
};

// out = in with axes reordered: out axis i is in axis perm[i] (row-major).
void permute(Program& P, const Ten& in, const std::vector<int>& perm, const Ten& out) {
  const int nd = (int)in.dims.size();
  if (nd > 6 || (int)perm.size() != nd) throw Error{MPO_ERR_UNSUPPORTED, "permutation of > 6 axes"};
  std::vector<long long> st(nd, 1);
  for (int i = nd - 2; i >= 0; --i) st[i] = st[i + 1] * in.dims[i + 1];
  PermDesc d{};
  d.in = in.p;
  d.out = out.p;
  d.tin = in.t == DType::F64 ? 0 : 1;
  d.tout = out.t == DType::F64 ? 0 : 1;
  d.scale = 1.0;
  for (int q = 0; q < 6; ++q) { d.n[q] = 1; d.si[q] = 0; d.so[q] = 0; }
  const int off = 6 - nd;
  long long so = 1;
  for (int i = nd - 1; i >= 0; --i) {
    d.n[off + i] = in.dims[perm[i]];
    d.si[off + i] = st[perm[i]];
    d.so[off + i] = so;
    so *= in.dims[perm[i]];
  }
  add_perm(P, {d}, "grad_perm");
}

bool is_iota(const std::vector<int>& v) {
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i] != (int)i) return false;
  return true;
}

// out[free(a)..., free(b)...] (then reordered by out_order) =
//   sum over the paired axes ca of a and cb of b.
void contract(Program& P, Arena& ar, const SplitBuf& sb, Mode mode, const Ten& a,
              const std::vector<int>& ca, const Ten& b, const std::vector<int>& cb, const Ten& out,
              const std::vector<int>& out_order, const char* cls) {
  const int na = (int)a.dims.size(), nb = (int)b.dims.size();
  if (ca.size() != cb.size()) throw Error{MPO_ERR_SHAPE, "contraction axes"};
  std::vector<int> fa, fb;
  for (int i = 0; i < na; ++i)
    if (std::find(ca.begin(), ca.end(), i) == ca.end()) fa.push_back(i);
  for (int i = 0; i < nb; ++i)
    if (std::find(cb.begin(), cb.end(), i) == cb.end()) fb.push_back(i);
  long long M = 1, K = 1, N = 1;
  for (int i : fa) M *= a.dims[i];
  for (int i : fb) N *= b.dims[i];
  for (size_t q = 0; q < ca.size(); ++q) {
    if (a.dims[ca[q]] != b.dims[cb[q]]) throw Error{MPO_ERR_SHAPE, "contracted dims differ"};
    K *= a.dims[ca[q]];
  }
  const DType gt = mode == Mode::F64 ? DType::F64 : DType::F32;
  auto cat = [](std::vector<int> x, const std::vector<int>& y) {
    x.insert(x.end(), y.begin(), y.end());
    return x;
  };
  auto dims_of = [](const Ten& t, const std::vector<int>& ax) {
    std::vector<int> d;
    for (int i : ax) d.push_back(t.dims[i]);
    return d;
  };
  Op oa{a.p, a.t, true, (int)K}, ob{b.p, b.t, false, (int)N};
  if (!is_iota(cat(fa, ca))) {
    if (is_iota(cat(ca, fa))) {
      oa = Op{a.p, a.t, false, (int)M};
    } else {
      Ten t = ar.take(gt, cat(dims_of(a, fa), dims_of(a, ca)));
      permute(P, a, cat(fa, ca), t);
      oa = Op{t.p, gt, true, (int)K};
    }
  }
  if (!is_iota(cat(cb, fb))) {
    if (is_iota(cat(fb, cb))) {
      ob = Op{b.p, b.t, true, (int)K};
    } else {
      Ten t = ar.take(gt, cat(dims_of(b, cb), dims_of(b, fb)));
      permute(P, b, cat(cb, fb), t);
      ob = Op{t.p, gt, false, (int)N};
    }
  }
  // FP32 modes take an FP32 second operand
  if (gt == DType::F32 && ob.t != DType::F32) {
    Ten t = ar.take(gt, {(int)K, (int)N});
    Ten src{const_cast<void*>(ob.p), ob.t, ob.kc ? std::vector<int>{(int)N, (int)K} : std::vector<int>{(int)K, (int)N}};
    permute(P, src, ob.kc ? std::vector<int>{1, 0} : std::vector<int>{0, 1}, t);
    ob = Op{t.p, gt, false, (int)N};
  }
  std::vector<int> gdims = cat(dims_of(a, fa), dims_of(b, fb));
  if (gdims.empty()) gdims = {1};
  const bool direct = is_iota(out_order) && out.t == gt;
  Ten g = direct ? out : ar.take(gt, gdims);
  add_gemm(P, sb, mode, {GemmJob{(int)M, (int)N, (int)K, oa, ob, Out{g.p, gt, (int)N}}}, cls,
           2.0 * M * N * K);
  if (!direct) {
    Ten gg = g;
    gg.dims = gdims;
    permute(P, gg, out_order.empty() ? std::vector<int>{0} : out_order, out);
  }
}

std::vector<int> iota(int n) {
  std::vector<int> v(n);
  for (int i = 0; i < n; ++i) v[i] = i;
  return v;
}

struct GradPlan {
  long long bytes = 0;
  double* loss_dev = nullptr;
};

// Records the whole adjoint into P.  Tensors: A, B (the cores to
// differentiate at, FP64 caller arrays), W (FP64), C (the context's FP64
// normalized cores, isometries except the centre), gradients into gA, gB.
void rec_grad(Ctx& X, Program& P, Arena& ar, PairState& S, const mpo_tt& A, const mpo_tt& B,
              const mpo_tt& W, double* const* gA, double* const* gB, int centre, bool recompute,
              double* loss_dev) {
  const int L = S.L, d = S.d;
  const Mode mode = X.wt == DType::F64 ? Mode::F64 : Mode::F32;
  const DType wt = mode == Mode::F64 ? DType::F64 : DType::F32;
  auto core = [&](const mpo_tt& t, int l) {
    return Ten{const_cast<double*>(t.cores[l]), DType::F64, {t.chi[l], d, d, t.chi[l + 1]}};
  };
  // working-precision copies
  std::vector<Ten> Aw(L), Bw(L), Ww(L), Pw(L);
  for (int l = 0; l < L; ++l) {
    Aw[l] = ar.take(wt, core(A, l).dims);
    permute(P, core(A, l), iota(4), Aw[l]);
    Bw[l] = ar.take(wt, core(B, l).dims);
    permute(P, core(B, l), iota(4), Bw[l]);
    Ww[l] = ar.take(wt, core(W, l).dims);
    permute(P, core(W, l), iota(4), Ww[l]);
    const Ten Cl{S.C64[l], DType::F64, {S.cC[l], d, d, S.cC[l + 1]}};
    if (l != centre) {
      Pw[l] = ar.take(wt, Cl.dims);
      permute(P, Cl, iota(4), Pw[l]);
    }
  }
  auto one = [&](std::vector<int> dims) {
    Ten t = ar.take(wt, dims);
    add_fill(P, {FillDesc{t.p, 0, 1, 1, wt == DType::F64 ? 1 : 0}});
    return t;
  };
  auto as = [](Ten t, std::vector<int> dims) {  // view of a buffer with other dims
    t.dims = std::move(dims);
    return t;
  };
  // Pi(W): centre core from the two-layer environment of (isometries, W)
  {
    long long emax = 1;
    for (int l = 0; l <= L; ++l) emax = std::max(emax, (long long)S.cC[l] * W.chi[l]);
    Ten E0 = ar.take(wt, {(int)emax}), E1 = ar.take(wt, {(int)emax});
    add_fill(P, {FillDesc{E0.p, 0, 1, 1, wt == DType::F64 ? 1 : 0}});
    const size_t mark = ar.cv.off;
    if (centre == L - 1) {
      Ten E = as(E0, {1, 1});
      for (int l = 0; l + 1 < L; ++l) {
        Ten T = ar.take(wt, {Ww[l].dims[0], d, d, Pw[l].dims[3]});
        contract(P, ar, X.sb, mode, E, {0}, Pw[l], {0}, T, iota(4), "grad_proj");
        Ten E2 = as(E.p == E0.p ? E1 : E0, {Pw[l].dims[3], Ww[l].dims[3]});
        contract(P, ar, X.sb, mode, T, {0, 1, 2}, Ww[l], {0, 1, 2}, E2, iota(2), "grad_proj");
        E = E2;
        ar.cv.off = mark;
      }
      Pw[L - 1] = ar.take(wt, {E.dims[0], d, d, 1});
      contract(P, ar, X.sb, mode, E, {1}, Ww[L - 1], {0}, Pw[L - 1], iota(4), "grad_proj");
    } else {
      Ten F = as(E0, {1, 1});
      for (int l = L - 1; l >= 1; --l) {
        Ten T = ar.take(wt, {Pw[l].dims[0], d, d, Ww[l].dims[3]});
        contract(P, ar, X.sb, mode, Pw[l], {3}, F, {0}, T, iota(4), "grad_proj");
        Ten F2 = as(F.p == E0.p ? E1 : E0, {Pw[l].dims[0], Ww[l].dims[0]});
        contract(P, ar, X.sb, mode, T, {1, 2, 3}, Ww[l], {1, 2, 3}, F2, iota(2), "grad_proj");
        F = F2;
        ar.cv.off = mark;
      }
      Pw[0] = ar.take(wt, {1, d, d, F.dims[0]});
      contract(P, ar, X.sb, mode, Ww[0], {3}, F, {1}, Pw[0], iota(4), "grad_proj");
    }
  }
  auto env_dims = [&](int l) {  // environment across bond l (left of site l)
    return std::vector<int>{Pw[std::max(l - 1, 0)].dims[l == 0 ? 0 : 3], A.chi[l], B.chi[l]};
  };
  long long emax = 1;
  for (int l = 0; l <= L; ++l) {
    const auto e = env_dims(l);
    emax = std::max(emax, (long long)e[0] * e[1] * e[2]);
  }
  auto env_left = [&](const Ten& Le, int l, const Ten& out) {
    const int x = Le.dims[0], b = Le.dims[2], a2 = A.chi[l + 1], b2 = B.chi[l + 1];
    Ten T = ar.take(wt, {x, b, d, d, a2});
    contract(P, ar, X.sb, mode, Le, {1}, Aw[l], {0}, T, iota(5), "grad_env");
    Ten T2 = ar.take(wt, {x, d, a2, d, b2});
    contract(P, ar, X.sb, mode, T, {1, 3}, Bw[l], {0, 1}, T2, iota(5), "grad_env");
    contract(P, ar, X.sb, mode, Pw[l], {0, 1, 2}, T2, {0, 1, 3}, out, iota(3), "grad_env");
  };
  auto env_right = [&](const Ten& Re, int l, const Ten& out) {
    const int a = A.chi[l], b = B.chi[l], x2 = Re.dims[0], b2 = Re.dims[2];
    Ten T = ar.take(wt, {a, d, d, x2, b2});
    contract(P, ar, X.sb, mode, Aw[l], {3}, Re, {1}, T, iota(5), "grad_env");
    Ten X2 = ar.take(wt, {a, d, x2, b, d});
    contract(P, ar, X.sb, mode, T, {2, 4}, Bw[l], {1, 3}, X2, iota(5), "grad_env");
    contract(P, ar, X.sb, mode, X2, {1, 2, 4}, Pw[l], {1, 3, 2}, out, {2, 0, 1}, "grad_env");
  };
  // right environments: all of them, or every k-th (the others recomputed
  // per segment of k sites during the left-to-right pass)
  const int k = recompute ? std::max(1, (int)std::ceil(std::sqrt((double)L))) : 1;
  std::vector<Ten> Re(L + 1);
  std::vector<bool> ck(L + 1, false);
  Re[L] = one({1, 1, 1});
  ck[L] = true;
  for (int l = 1; l < L; ++l) {
    ck[l] = !recompute || l % k == 0;
    if (ck[l]) Re[l] = ar.take(wt, env_dims(l));
  }
  Ten roll[2] = {ar.take(wt, {(int)emax}), ar.take(wt, {(int)emax})};
  std::vector<Ten> seg(recompute ? k : 0);
  for (auto& t : seg) t = ar.take(wt, {(int)emax});
  Ten Lb[2] = {ar.take(wt, {(int)emax}), ar.take(wt, {(int)emax})};
  const size_t mark = ar.cv.off;  // temporaries above this point, reused per step
  {
    Ten cur = Re[L];
    int f = 0;
    for (int l = L - 1; l >= 1; --l) {
      Ten nx = ck[l] ? Re[l] : as(roll[f ^= 1], env_dims(l));
      env_right(cur, l, nx);
      cur = nx;
      ar.cv.off = mark;
    }
  }
  Ten Le = as(Lb[0], {1, 1, 1});
  add_fill(P, {FillDesc{Le.p, 0, 1, 1, wt == DType::F64 ? 1 : 0}});
  int seg_hi = 0;  // Re[m] for m <= seg_hi of the current segment are in seg
  for (int l = 0; l < L; ++l) {
    if (!ck[l + 1] && l + 1 > seg_hi) {
      // recompute the right environments of this segment from its checkpoint
      int top = l + 1;
      while (!ck[top]) ++top;
      Ten cur = Re[top];
      for (int m = top - 1; m >= l + 1; --m) {
        Re[m] = as(seg[m % k], env_dims(m));
        env_right(cur, m, Re[m]);
        cur = Re[m];
        ar.cv.off = mark;
      }
      seg_hi = top - 1;
    }
    const Ten& R = Re[l + 1];
    const int a = A.chi[l], b = B.chi[l], a2 = A.chi[l + 1], b2 = B.chi[l + 1], x = Le.dims[0];
    const int x2 = Pw[l].dims[3];
    // dA[a, s, t, a'] = sum Le[x, a, b] P[x, s, u, x'] B[b, t, u, b'] R[x', a', b']
    {
      Ten V1 = ar.take(wt, {x, a, d, d, b2});
      contract(P, ar, X.sb, mode, Le, {2}, Bw[l], {0}, V1, iota(5), "grad_adj");
      Ten V2 = ar.take(wt, {a, d, b2, d, x2});
      contract(P, ar, X.sb, mode, V1, {0, 3}, Pw[l], {0, 2}, V2, iota(5), "grad_adj");
      const Ten G{gA[l], DType::F64, {a, d, d, a2}};
      contract(P, ar, X.sb, mode, V2, {2, 4}, R, {2, 0}, G, {0, 2, 1, 3}, "grad_adj");
      ar.cv.off = mark;
    }
    // dB[b, t, u, b'] = sum Le[x, a, b] P[x, s, u, x'] A[a, s, t, a'] R[x', a', b']
    {
      Ten V1 = ar.take(wt, {x, b, d, d, a2});
      contract(P, ar, X.sb, mode, Le, {1}, Aw[l], {0}, V1, iota(5), "grad_adj");
      Ten V2 = ar.take(wt, {b, d, a2, d, x2});
      contract(P, ar, X.sb, mode, V1, {0, 2}, Pw[l], {0, 1}, V2, iota(5), "grad_adj");
      const Ten G{gB[l], DType::F64, {b, d, d, b2}};
      contract(P, ar, X.sb, mode, V2, {2, 4}, R, {1, 0}, G, iota(4), "grad_adj");
      ar.cv.off = mark;
    }
    Ten Ln = as(Le.p == Lb[0].p ? Lb[1] : Lb[0], env_dims(l + 1));
    env_left(Le, l, Ln);
    Le = Ln;
    ar.cv.off = mark;
  }
  permute(P, Ten{Le.p, wt, {1}}, {0}, Ten{loss_dev, DType::F64, {1}});
}

// ------------------------------------------------------------------ fit error check
// ||A B - C||_F / ||A B||_F from transfer passes in FP64 (Sec. 2.3, Eq.
// fit_min): ||A B||^2 by a four-layer pass, <C, A B> by a three-layer pass,
// ||C||^2 by a two-layer pass; the naive product of Alg. 1 is never formed.
// After every site the running environment is divided by its Frobenius
// norm, whose logarithms are summed on the host (no under- or overflow).
struct CheckPlan {
  double* logs = nullptr;  // 3 (L + 1) norms: passes n2, cab, cc
  double* part = nullptr;  // NormBig partial sums
};

void add_normalize(Program& P, const Ten& t, double* nu_out, double* part) {
  Launch l;
  l.kind = LK::NormBig;
  l.off = P.push(std::vector<NormDesc>{NormDesc{static_cast<double*>(t.p), t.size(), nu_out}});
  l.n = 1;
  l.aux = part;
  l.cls = "check";
  P.launches.push_back(l);
}

// `passes` selects the four-layer (1), three-layer (2) and two-layer (4)
// passes; each writes its L + 1 logs only.
void rec_check(Program& P, Arena& ar, const SplitBuf& sb, const mpo_tt& A, const mpo_tt& B,
               const mpo_tt& Cm, const CheckPlan& cp, int passes = 7) {
  const int L = A.L, d = A.d;
  const Mode mode = Mode::F64;
  const DType t64 = DType::F64;
  auto core = [&](const mpo_tt& t, int l) {
    return Ten{const_cast<double*>(t.cores[l]), t64, {t.chi[l], d, d, t.chi[l + 1]}};
  };
  auto one = [&](std::vector<int> dims) {
    Ten t = ar.take(t64, dims);
    add_fill(P, {FillDesc{t.p, 0, 1, 1, 1}});
    return t;
  };
  auto as = [](Ten t, std::vector<int> dims) {
    t.dims = std::move(dims);
    return t;
  };
  long long e4 = 1, e3 = 1, e2 = 1;
  for (int l = 0; l <= L; ++l) {
    const long long a = A.chi[l], b = B.chi[l], c = Cm.chi[l];
    e4 = std::max(e4, a * b * a * b);
    e3 = std::max(e3, c * a * b);
    e2 = std::max(e2, c * c);
  }
  auto two = [&](bool on, long long n) {
    std::array<Ten, 2> t;
    if (on) t = {ar.take(t64, {(int)n}), ar.take(t64, {(int)n})};
    return t;
  };
  const std::array<Ten, 2> E4 = two(passes & 1, e4), E3 = two(passes & 2, e3), E2 = two(passes & 4, e2);
  const size_t mark = ar.cv.off;
  // four layers: E[a1, b1, a2, b2] -> sum over x, u of (A B)(x, u) (A B)(x, u)
  if (passes & 1) {
    Ten E = as(E4[0], {1, 1, 1, 1});
    add_fill(P, {FillDesc{E.p, 0, 1, 1, 1}});
    for (int l = 0; l < L; ++l) {
      const Ten Al = core(A, l), Bl = core(B, l);
      const int a1 = A.chi[l + 1], b1 = B.chi[l + 1];
      Ten T1 = ar.take(t64, {B.chi[l], A.chi[l], B.chi[l], d, d, a1});          // [b1 a2 b2 x t a1']
      contract(P, ar, sb, mode, E, {0}, Al, {0}, T1, iota(6), "check");
      Ten T2 = ar.take(t64, {B.chi[l], B.chi[l], d, a1, d, a1});                // [b1 b2 t a1' v a2']
      contract(P, ar, sb, mode, T1, {1, 3}, Al, {0, 1}, T2, iota(6), "check");
      Ten T3 = ar.take(t64, {B.chi[l], a1, d, a1, d, b1});                      // [b2 a1' v a2' u b1']
      contract(P, ar, sb, mode, T2, {0, 2}, Bl, {0, 1}, T3, iota(6), "check");
      Ten En = as(E.p == E4[0].p ? E4[1] : E4[0], {a1, b1, a1, b1});
      // [a1' a2' b1' b2'] -> [a1' b1' a2' b2']
      contract(P, ar, sb, mode, T3, {0, 2, 4}, Bl, {0, 1, 2}, En, {0, 2, 1, 3}, "check");
      add_normalize(P, En, cp.logs + l, cp.part);
      E = En;
      ar.cv.off = mark;
    }
    add_normalize(P, E, cp.logs + L, cp.part);  // the last is the scalar itself
  }
  // three layers: E[c, a, b]
  if (passes & 2) {
    Ten E = as(E3[0], {1, 1, 1});
    add_fill(P, {FillDesc{E.p, 0, 1, 1, 1}});
    for (int l = 0; l < L; ++l) {
      const Ten Al = core(A, l), Bl = core(B, l), Cl = core(Cm, l);
      const int x = Cm.chi[l], b = B.chi[l], a2 = A.chi[l + 1], b2 = B.chi[l + 1];
      Ten T = ar.take(t64, {x, b, d, d, a2});
      contract(P, ar, sb, mode, E, {1}, Al, {0}, T, iota(5), "check");
      Ten T2 = ar.take(t64, {x, d, a2, d, b2});
      contract(P, ar, sb, mode, T, {1, 3}, Bl, {0, 1}, T2, iota(5), "check");
      Ten En = as(E.p == E3[0].p ? E3[1] : E3[0], {Cm.chi[l + 1], a2, b2});
      contract(P, ar, sb, mode, Cl, {0, 1, 2}, T2, {0, 1, 3}, En, iota(3), "check");
      if (l + 1 < L) add_normalize(P, En, cp.logs + (L + 1) + l, cp.part);
      E = En;
      ar.cv.off = mark;
    }
    // the last value keeps its sign: copy it out instead of normalizing
    permute(P, as(E, {1}), {0}, Ten{cp.logs + (L + 1) + L, t64, {1}});
  }
  // two layers: E[c, c']
  if (passes & 4) {
    Ten E = as(E2[0], {1, 1});
    add_fill(P, {FillDesc{E.p, 0, 1, 1, 1}});
    for (int l = 0; l < L; ++l) {
      const Ten Cl = core(Cm, l);
      const int c2 = Cm.chi[l + 1];
      Ten T = ar.take(t64, {Cm.chi[l], d, d, c2});
      contract(P, ar, sb, mode, E, {0}, Cl, {0}, T, iota(4), "check");
      Ten En = as(E.p == E2[0].p ? E2[1] : E2[0], {c2, c2});
      contract(P, ar, sb, mode, T, {0, 1, 2}, Cl, {0, 1, 2}, En, iota(2), "check");
      add_normalize(P, En, cp.logs + 2 * (L + 1) + l, cp.part);
      E = En;
      ar.cv.off = mark;
    }
    add_normalize(P, E, cp.logs + 2 * (L + 1) + L, cp.part);
  }
}

// ---------------------------------------------------------------- fit error per sweep
// An mpo_tt view of device cores with host-held bond dims.
struct TTView {
  std::vector<int32_t> chi;
  std::vector<const double*> cores;
  mpo_tt tt{};
  TTView(int L, int d, const std::vector<int>& dims, const std::vector<double*>& ptrs)
      : chi(dims.begin(), dims.end()), cores(ptrs.begin(), ptrs.end()) {
    tt.L = L;
    tt.d = d;
    tt.chi = chi.data();
    tt.cores = cores.data();
  }
};

// eps = ||A B - C|| / ||A B|| from the logs of the transfer passes:
// l4 = log ||A B||^2, lg3 / lg2 = the L + 1 entries of the three- and
// two-layer passes (renormalization logs; lg3[L] is <C, A B> itself).
double transfer_eps(int L, double l4, const double* lg3, const double* lg2) {
  double l3 = 0, l2 = 0;
  bool z3 = false, z2 = false;
  for (int i = 0; i <= L; ++i) {
    if (!std::isfinite(lg3[i]) || !std::isfinite(lg2[i])) throw Error{MPO_ERR_NUMERIC, "non-finite transfer pass"};
    if (lg2[i] > 0) l2 += std::log(lg2[i]); else z2 = true;
  }
  for (int i = 0; i < L - 1; ++i) {
    if (lg3[i] > 0) l3 += std::log(lg3[i]); else z3 = true;
  }
  const double last = lg3[L];
  const double cab = (z3 || last == 0.0) ? 0.0
                     : (last > 0 ? 1.0 : -1.0) * std::exp(l3 + std::log(std::fabs(last)) - l4);
  const double cc = z2 ? 0.0 : std::exp(l2 - l4);
  return std::sqrt(std::max(0.0, 1.0 - 2.0 * cab + cc));
}

size_t err_region_bytes(const Ctx& X) {
  size_t peak = 0;
  for (const PairState& S : X.pairs) {
    std::vector<double*> none(S.L, nullptr);
    TTView A(S.L, S.d, S.cA, none), B(S.L, S.d, S.cB, none), C(S.L, S.d, S.capC, none);
    for (int passes : {1, 6}) {
      Program P;
      Arena ar;
      SplitBuf sb;
      rec_check(P, ar, sb, A.tt, B.tt, C.tt, CheckPlan{}, passes);
      peak = std::max(peak, ar.peak);
    }
  }
  return peak + 256;
}

// Runs transfer passes of one pair on the context stream: `passes` as in
// rec_check, with C the merged FP64 copy in X.err.C (its current dims).
void run_err_passes(Ctx& X, int pair, int passes, std::vector<double>& lg) {
  PairState& S = X.pairs[pair];
  TTView A(S.L, S.d, S.cA, S.A64), B(S.L, S.d, S.cB, S.B64), C(S.L, S.d, S.cC, X.err.C[pair]);
  Program P;
  if (passes & 6) {  // C = the merged train of the normalized fit (no nu)
    std::vector<PermDesc> ds;
    std::vector<ScaleDesc> sc;
    const bool inv = X.o.schedule == MPO_SCHED_EVEN_ODD;
    for (int i = 0; i < S.L; ++i) {
      const long long n = (long long)S.cC[i] * S.dd * S.cC[i + 1];
      ds.push_back(perm4(S.C64[i], 0, X.err.C[pair][i], 0, {1, 1, 1, (int)n}, {0, 0, 0, 1}, {0, 0, 0, 1}));
      if (inv && i + 1 < S.L)
        sc.push_back(ScaleDesc{X.err.C[pair][i], X.err.C[pair][i], S.cC[i] * S.dd, S.cC[i + 1], S.cC[i + 1],
                               S.cC[i + 1], nullptr, S.Yv[i + 1], 0, 1});
    }
    add_perm(P, ds, "fit_error");
    long long mx = 1;
    for (auto& d : sc) mx = std::max(mx, (long long)d.n * d.r);
    add_simple(P, LK::Scale, sc, mx, "fit_error");
  }
  CheckPlan cp{X.err.logs, X.err.part};
  Arena ar;
  ar.cv.base = X.err.region;
  rec_check(P, ar, X.sb, A.tt, B.tt, C.tt, cp, passes);
  if (ar.peak > X.err.region_bytes) throw Error{MPO_ERR_WORKSPACE, "fit error region too small"};
  const size_t keep = X.arena_used;
  upload(X, P);
  run_program(P, X.stream, nullptr);
  lg.assign(3 * (size_t)(S.L + 1), 0.0);
  HIP_OK(hipMemcpyAsync(lg.data(), X.err.logs, lg.size() * sizeof(double), hipMemcpyDeviceToHost, X.stream));
  HIP_OK(hipStreamSynchronize(X.stream));
  X.arena_used = keep;
}

// log ||A B||^2 of every pair (normalized cores), once at initialization.
void err_init(Ctx& X) {
  X.err.l4.assign(X.pairs.size(), 0.0);
  for (size_t p = 0; p < X.pairs.size(); ++p) {
    std::vector<double> lg;
    run_err_passes(X, (int)p, 1, lg);
    const int L = X.pairs[p].L;
    double l4 = 0;
    for (int i = 0; i <= L; ++i) {
      if (!(lg[i] > 0) || !std::isfinite(lg[i])) throw Error{MPO_ERR_NUMERIC, "A B is zero or not finite"};
      l4 += std::log(lg[i]);
    }
    X.err.l4[p] = l4;
  }
}

double sweep_error(Ctx& X, int pair) {
  std::vector<double> lg;
  run_err_passes(X, pair, 6, lg);
  const int L = X.pairs[pair].L;
  return transfer_eps(L, X.err.l4[pair], lg.data() + (L + 1), lg.data() + 2 * (L + 1));
}

// Small context for calls that are not tied to a fit: status flags, split-K
// scratch and a descriptor arena carved from the caller's workspace
// (`compact`: a smaller split-K buffer and arena, for the fixed-size static
// scratch; a launch whose split-K partials do not fit runs unsplit).
void carve_aux(Ctx& X, Carver& cv, bool compact = false) {
  X.flag = cv.take<int>(4);
  X.sweep_dev = X.flag + 1;
  X.sb.cap = compact ? (size_t)4 << 20 : (size_t)32 << 20;
  X.sb.partials = cv.take<char>(X.sb.cap);
  X.sb.ccap = compact ? 1 << 12 : 1 << 14;
  X.sb.counters = cv.take<int>(X.sb.ccap);
  X.arena_cap = compact ? (size_t)2 << 20 : (size_t)8 << 20;
  X.arena = cv.take<char>(X.arena_cap);
}

// ||A B||_F and ||A B - C||_F by Householder-QR sweeps from the left (Sec.
// 2.3.1, site-canonical form) over the naive product P = A B of Alg. 1 and
// over the difference MPO D = [P, -C]: the direct sum of the two trains, the
// first core concatenated along its right bond (C's block negated), block-
// diagonal middle cores, the last core stacked along its left bond.  The
// carried triangular factor R holds the norm of everything to its left, so
// the last site's column norm is the train's Frobenius norm.  Every step is
// backward stable (no Gram matrix, no difference of squares), so the
// relative error ||A B - C|| / ||A B|| is resolved far below sqrt(eps).
// D's cores are never formed: the carry R = [R_P, R_C] multiplies P_l and
// C_l block by block.  Bond dimensions chi_A chi_B + chi_C <= kCheckQrMax.
constexpr int kCheckQrMax = 512;

struct QrCheckBufs {
  double *carry[2], *X, *Pc, *out;
};

bool check_qr_fits(const mpo_tt& A, const mpo_tt& B, const mpo_tt& C) {
  for (int l = 0; l <= A.L; ++l)
    if ((long long)A.chi[l] * B.chi[l] + C.chi[l] > kCheckQrMax) return false;
  return true;
}

QrCheckBufs carve_check_qr(Carver& cv, const mpo_tt& A, const mpo_tt& B, const mpo_tt& C) {
  const int L = A.L, d = A.d;
  long long cmax = 1, pmax = 1, xmax = 1;
  for (int l = 0; l < L; ++l) {
    const long long p0 = (long long)A.chi[l] * B.chi[l], p1 = (long long)A.chi[l + 1] * B.chi[l + 1];
    const long long c0 = p0 + C.chi[l], c1 = p1 + C.chi[l + 1];
    cmax = std::max({cmax, c0, c1});
    pmax = std::max(pmax, p0 * d * d * p1);
    xmax = std::max(xmax, c0 * d * d * c1);  // rows of X never exceed the left bond times d^2
  }
  QrCheckBufs b;
  b.carry[0] = cv.take<double>((size_t)cmax * cmax);
  b.carry[1] = cv.take<double>((size_t)cmax * cmax);
  b.X = cv.take<double>((size_t)xmax);
  b.Pc = cv.take<double>((size_t)pmax);
  b.out = cv.take<double>(2);
  return b;
}

// One QR sweep: over P alone (C null) into out[0], or over [P, -C] into out[1].
void rec_check_qr_sweep(Program& P, const SplitBuf& sb, const mpo_tt& A, const mpo_tt& B,
                        const mpo_tt* C, const QrCheckBufs& b, double* out) {
  const int L = A.L, d = A.d, dd = d * d;
  int r = 1, cur = 0;  // carry: r x (width of D's bond l), in b.carry[cur]
  add_fill(P, {FillDesc{b.carry[0], 2, 1, 1, 1}});
  for (int l = 0; l < L; ++l) {
    const int p0 = A.chi[l] * B.chi[l], p1 = A.chi[l + 1] * B.chi[l + 1];
    const int c0 = C ? C->chi[l] : 0, c1 = C ? C->chi[l + 1] : 0;
    const bool first = l == 0, last = l == L - 1;
    const int w0 = (first || !C) ? p0 : p0 + c0;        // D's left bond
    const int w1 = (last || !C) ? p1 : p1 + c1;         // D's right bond
    add_simple(P, LK::Naive, std::vector<NaiveDesc>{NaiveDesc{A.cores[l], B.cores[l], b.Pc, A.chi[l],
                                                              A.chi[l + 1], B.chi[l], B.chi[l + 1], d}},
               (long long)p0 * dd * p1, "check");
    const double* carry = b.carry[cur];
    // X[(i, s, u), j] = sum_a carry[i, a] P_l[a, s, u, j] (+ the C block)
    GemmJob gp{r, p1, p0, op64(carry, true, w0), op64(b.Pc, false, dd * p1), out64(b.X, dd * w1)};
    gp.nb[0] = dd;
    gp.B.s[0] = p1;
    gp.C.s[0] = w1;
    add_gemm(P, sb, Mode::F64, {gp}, "check", 0);
    if (C) {
      // C's block: its own columns (first, middle) or added onto P's (last);
      // at the first site both blocks share D's left bond of dimension 1
      const double* cc = first ? carry : carry + p0;
      GemmJob gc{r, c1, c0, op64(cc, true, w0), op64(C->cores[l], false, dd * c1),
                 out64(last ? b.X : b.X + p1, dd * w1)};
      gc.nb[0] = dd;
      gc.B.s[0] = c1;
      gc.C.s[0] = w1;
      gc.alpha = first && !last ? -1.0 : 1.0;
      if (first && last) gc.alpha = -1.0;  // one site: D = P - C
      gc.beta = last ? 1 : 0;
      add_gemm(P, sb, Mode::F64, {gc}, "check", 0);
    }
    const int m = r * dd;
    if (last) {
      add_simple(P, LK::Norm, std::vector<NormDesc>{NormDesc{b.X, (long long)m * w1, out}}, 0, "check");
      break;
    }
    add_simple(P, LK::Geqr, std::vector<GeqrDesc>{GeqrDesc{b.X, m, w1, w1, b.carry[1 - cur], w1}}, 0, "check");
    cur = 1 - cur;
    r = std::min(m, w1);
  }
}

int grad_centre(const Ctx& X) {
  if (X.o.schedule != MPO_SCHED_SERIAL) throw Error{MPO_ERR_UNSUPPORTED, "gradient: serial schedule only"};
  if (X.o.tau > 0.0) throw Error{MPO_ERR_UNSUPPORTED, "gradient: fixed bond cap (tau = 0) only"};
  if (X.o.mps) throw Error{MPO_ERR_UNSUPPORTED, "gradient: MPO-MPO fits only"};
  if (X.pos != 0) throw Error{MPO_ERR_UNSUPPORTED, "gradient: the fit stands inside a sweep"};
  return (X.o.first_sweep + X.sweeps_done) % 2 == 1 ? -1 : 0;  // -1: last site
}

void validate_grad(const Ctx& X, const PairState& S, const mpo_pair* ab, const mpo_tt* W) {
  if (!ab || !W) throw Error{MPO_ERR_INVALID_ARG, "null pair or W"};
  validate_tt(ab->A, S.L, S.d);
  validate_tt(ab->B, S.L, S.d);
  validate_tt(*W, S.L, S.d);
  for (int l = 0; l <= S.L; ++l)
    if (ab->A.chi[l] != S.chiA_in[l] || ab->B.chi[l] != S.chiB_in[l])
      throw Error{MPO_ERR_SHAPE, "A and B must have the fitted bond dimensions"};
  (void)X;
}
}  // namespace
}  // namespace mpofit

// Static scratch of the allocation-free check (mpo_contract_exact_check_static):
// a file-scope device array, one copy per GPU, held until the process ends.
// Host code reaches it only through the address hipGetSymbolAddress returns
// for the current device; the array's name on the host is a stand-in.
static constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace mpofit {
namespace {
// The exact check's two routes: Householder-QR sweeps (check_qr_fits) or
// the transfer passes; both carve from `ws` after the auxiliary context.
struct CheckLayout {
  bool qr;
  CheckPlan cp;
  QrCheckBufs qb;
  size_t off;
};

CheckLayout check_layout(Ctx& X, Carver& cv, const mpo_pair& pair, const mpo_tt& C, bool compact) {
  const int L = pair.A.L;
  carve_aux(X, cv, compact);
  CheckLayout lay{};
  lay.qr = check_qr_fits(pair.A, pair.B, C);
  if (lay.qr) {
    lay.qb = carve_check_qr(cv, pair.A, pair.B, C);
  } else {
    lay.cp.logs = cv.take<double>(3 * (L + 1));
    lay.cp.part = cv.take<double>(1024);
  }
  lay.off = cv.off;
  return lay;
}

void validate_check(const mpo_pair& pair, const mpo_tt& C) {
  const int L = pair.A.L, d = pair.A.d;
  if (L < 1 || d < 1) throw Error{MPO_ERR_SHAPE, "bad L or d"};
  validate_tt(pair.A, L, d);
  validate_tt(pair.B, L, d);
  validate_tt(C, L, d);
}

size_t check_bytes(const mpo_pair& pair, const mpo_tt& C, bool compact) {
  validate_check(pair, C);
  Ctx X;
  Carver cv;
  CheckLayout lay = check_layout(X, cv, pair, C, compact);
  if (lay.qr) return cv.off + 256;
  Program P;
  Arena ar;
  ar.cv.off = cv.off;
  rec_check(P, ar, X.sb, pair.A, pair.B, C, lay.cp);
  return std::max(ar.peak, cv.off) + 256;
}

void check_run(const mpo_pair& pair, const mpo_tt& C, double* rel_err, double* ab_norm2, int32_t* method,
               char* ws, size_t ws_bytes, hipStream_t stream, bool compact) {
  const size_t need = check_bytes(pair, C, compact);
  if (need > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "workspace too small"};
  const int L = pair.A.L;
  Ctx X;
  X.stream = stream;
  Carver cv;
  cv.base = ws;
  CheckLayout lay = check_layout(X, cv, pair, C, compact);
  // flags and split-K counters start at zero in every call
  Program z;
  add_fill(z, {FillDesc{X.flag, 4, 0, 0, 0}, FillDesc{X.sb.counters, X.sb.ccap, 0, 0, 0}});
  upload(X, z);
  run_program(z, X.stream, nullptr);
  Program P;
  if (lay.qr) {
    rec_check_qr_sweep(P, X.sb, pair.A, pair.B, nullptr, lay.qb, lay.qb.out);
    rec_check_qr_sweep(P, X.sb, pair.A, pair.B, &C, lay.qb, lay.qb.out + 1);
    upload(X, P);
    run_program(P, X.stream, nullptr);
    double nrm[2];
    HIP_OK(hipMemcpyAsync(nrm, lay.qb.out, sizeof(nrm), hipMemcpyDeviceToHost, X.stream));
    HIP_OK(hipStreamSynchronize(X.stream));
    check_flags(X);
    if (!std::isfinite(nrm[0]) || !std::isfinite(nrm[1])) throw Error{MPO_ERR_NUMERIC, "non-finite norm"};
    if (!(nrm[0] > 0)) throw Error{MPO_ERR_NUMERIC, "A B is zero"};
    *rel_err = nrm[1] / nrm[0];
    if (ab_norm2) *ab_norm2 = nrm[0] * nrm[0];
    if (method) *method = 0;
    return;
  }
  Arena ar;
  ar.cv.base = cv.base;
  ar.cv.off = cv.off;
  rec_check(P, ar, X.sb, pair.A, pair.B, C, lay.cp);
  upload(X, P);
  run_program(P, X.stream, nullptr);
  std::vector<double> lg(3 * (L + 1));
  HIP_OK(hipMemcpyAsync(lg.data(), lay.cp.logs, lg.size() * sizeof(double), hipMemcpyDeviceToHost, X.stream));
  HIP_OK(hipStreamSynchronize(X.stream));
  check_flags(X);
  // log ||AB||^2, log |<C, AB>| (with sign), log ||C||^2; a zero norm on
  // the way makes that pass exactly zero
  double l4 = 0;
  for (int i = 0; i <= L; ++i) {
    if (!(lg[i] > 0) || !std::isfinite(lg[i])) throw Error{MPO_ERR_NUMERIC, "A B is zero or not finite"};
    l4 += std::log(lg[i]);
  }
  *rel_err = transfer_eps(L, l4, lg.data() + (L + 1), lg.data() + 2 * (L + 1));
  if (ab_norm2) *ab_norm2 = std::exp(l4);
  if (method) *method = 1;
}

// Address of the static scratch on the current device (kept per device).
char* static_scratch_ptr() {
  static std::mutex mu;
  static std::map<int, char*> ptrs;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void* p = nullptr;
  HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch)));
  if (!p) throw Error{MPO_ERR_DEVICE, "static scratch has no device address"};
  ptrs[dev] = static_cast<char*>(p);
  return static_cast<char*>(p);
}
}  // namespace
}  // namespace mpofit

// ====================================================================== C ABI
using namespace mpofit;

struct mpo_fit_ctx {
  Ctx X;
  std::map<std::string, SweepPlan> plans;
  std::vector<hipEvent_t> evs;
};

namespace {
template <class F>
mpo_status guarded(F&& f) {
  try {
    f();
    return MPO_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return (mpo_status)e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MPO_ERR_DEVICE;
  }
}

// The bond dims of a pair's train as they stand: the planned ones, or with a
// truncation tolerance the device's (read after the context's stream).
std::vector<int> current_dims(const Ctx& X, const PairState& S) {
  if (!S.rk) return S.cC;
  std::vector<int> c(S.cC.size());
  HIP_OK(hipStreamSynchronize(X.stream));
  HIP_OK(hipMemcpy(c.data(), S.rk, c.size() * sizeof(int), hipMemcpyDeviceToHost));
  return c;
}

// Core i stored with the planned dims (cC) copied out with dims c (<= cC:
// the leading block, which holds every kept value), times scale.
PermDesc export_core(const PairState& S, int i, const std::vector<int>& c, double* out, double scale) {
  const long long cr = S.cC[i + 1];
  return perm4(S.C64[i], 0, out, 0, {1, c[i], S.dd, c[i + 1]}, {0, S.dd * cr, cr, 1},
               {0, (long long)S.dd * c[i + 1], c[i + 1], 1}, scale);
}
}  // namespace

namespace {
// Runs units [start, start + count) of the current sweep: the program of
// that segment for the current shapes is recorded once and replayed (as a
// captured graph once the shapes are stable; whole sweeps only), with the
// per-class timings in profiling contexts.  Advances the position.
void run_segment(mpo_fit_ctx* ctx, int start, int count) {
  Ctx& X = ctx->X;
  const bool fwd = (X.o.first_sweep + X.sweeps_done) % 2 == 0;
  const bool whole = start == 0 && count == sweep_units(X);
  const std::string key = shape_key(X, fwd ? "F" : "B") + "|" + std::to_string(start) + "+" +
                          std::to_string(count);
  auto it = ctx->plans.find(key);
  if (it == ctx->plans.end()) {
    SweepPlan sp;
    std::vector<std::vector<int>> before;
    for (auto& S : X.pairs) before.push_back(S.cC);
    record_segment(X, sp, fwd, start, count);
    sp.stable = sp.cC_after == before;
    // restore host shapes (recording advanced them) and upload
    for (size_t p = 0; p < X.pairs.size(); ++p) X.pairs[p].cC = before[p];
    it = ctx->plans.emplace(key, std::move(sp)).first;
    upload(X, it->second.prog);
  }
  SweepPlan& sp = it->second;
  if (X.profile) {
    std::vector<hipEvent_t>& ev = ctx->evs;
    while (ev.size() < sp.prog.launches.size() + 1) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      ev.push_back(e);
    }
    run_program(sp.prog, X.stream, ev.data());
    HIP_OK(hipEventSynchronize(ev[sp.prog.launches.size()]));
    for (size_t li = 0; li < sp.prog.launches.size(); ++li) {
      float ms = 0;
      HIP_OK(hipEventElapsedTime(&ms, ev[li], ev[li + 1]));
      const Launch& l = sp.prog.launches[li];
      auto pe = std::find_if(X.prof.begin(), X.prof.end(),
                             [&](const Ctx::ProfEntry& e) { return e.cls == l.cls; });
      if (pe == X.prof.end()) {
        X.prof.push_back(Ctx::ProfEntry{l.cls});
        pe = X.prof.end() - 1;
      }
      pe->ms += ms;
      pe->flops += l.flops;
      pe->launches += 1;
    }
  } else if (whole && X.o.capture_graph && X.stream != nullptr && (sp.stable || sp.uses >= 1)) {
    if (!sp.graph) {
      hipGraph_t g = nullptr;
      HIP_OK(hipStreamBeginCapture(X.stream, hipStreamCaptureModeThreadLocal));
      try {
        run_program(sp.prog, X.stream, nullptr);
      } catch (...) {
        (void)hipStreamEndCapture(X.stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIP_OK(hipStreamEndCapture(X.stream, &g));
      HIP_OK(hipGraphInstantiate(&sp.graph, g, nullptr, nullptr, 0));
      HIP_OK(hipGraphDestroy(g));
    }
    HIP_OK(hipGraphLaunch(sp.graph, X.stream));
  } else {
    run_program(sp.prog, X.stream, nullptr);
  }
  sp.uses++;
  for (size_t p = 0; p < X.pairs.size(); ++p) X.pairs[p].cC = sp.cC_after[p];
  X.pos += count;
  if (X.pos == sweep_units(X)) {
    X.pos = 0;
    X.sweeps_done++;
  }
}
}  // namespace

namespace {
// ------------------------------------------------------------------ zip-up
// Zip-up contraction (Alg. 2, Sec. 2.2) in FP64: copies of A and B brought
// to right-canonical form (RQ sweeps by Householder QR, as the fit's
// initialization), then one left-to-right pass: R''_l = R_{l-1} A_l B_l by
// two batched GEMMs (over the A bond, then over the B bond and the shared
// physical leg), M_l = R''_l as (r_{l-1} d^2) x (chi_A chi_B) factorized by
// the update's truncated SVD (the randomized range finder when the sketch
// is narrower than M_l, the Gram eigenproblem, drop and sign rules),
// C_l = U, R_l = U^T M_l; the last core is M_L.  One launch program, run
// eagerly.
constexpr int kZipStream = (1 << 30) + 2;

struct ZipShape {
  int L, d, dd;
  std::vector<int> ca, cb;  // right-canonical bond dims of A and B
  std::vector<int> r;       // C's bond dims
  long long nmax = 1, kmax = 1, Kmax = 1, rmax = 1, core_a = 1, core_b = 1, t1 = 1, hmax = 1;
};

ZipShape zip_shape(const mpo_pair& pair, int chi_max, int sketch_p) {
  ZipShape z;
  z.L = pair.A.L; z.d = pair.A.d; z.dd = z.d * z.d;
  const int L = z.L, dd = z.dd;
  z.ca.assign(L + 1, 1); z.cb.assign(L + 1, 1); z.r.assign(L + 1, 1);
  for (int j = L - 1; j >= 1; --j) {  // RQ sweeps: chi'_j = min(chi_j, d^2 chi'_{j+1})
    z.ca[j] = std::min(pair.A.chi[j], dd * z.ca[j + 1]);
    z.cb[j] = std::min(pair.B.chi[j], dd * z.cb[j + 1]);
  }
  for (int l = 0; l < L; ++l) {
    z.core_a = std::max(z.core_a, (long long)pair.A.chi[l] * dd * pair.A.chi[l + 1]);
    z.core_b = std::max(z.core_b, (long long)pair.B.chi[l] * dd * pair.B.chi[l + 1]);
  }
  for (int l = 0; l < L; ++l) {
    const long long n = (long long)z.r[l] * dd, K = (long long)z.ca[l + 1] * z.cb[l + 1];
    if (l + 1 < L) z.r[l + 1] = (int)std::min<long long>({(long long)chi_max, n, K});
    const long long k = sketch_p >= 0 ? std::min<long long>({(long long)chi_max + sketch_p, n, K}) : std::min(n, K);
    z.nmax = std::max(z.nmax, n);
    z.Kmax = std::max(z.Kmax, K);
    z.kmax = std::max(z.kmax, k);
    z.rmax = std::max(z.rmax, (long long)z.r[l + 1]);
    z.hmax = std::max(z.hmax, std::min(n, K));
    z.t1 = std::max(z.t1, (long long)z.r[l] * z.cb[l] * dd * z.ca[l + 1]);
  }
  if (z.nmax > 4096 || z.hmax > 1700 || z.kmax > 512)
    throw Error{MPO_ERR_UNSUPPORTED, "zip-up: a factorization beyond the eigen kernels' sizes"};
  return z;
}

struct ZipBufs {
  std::vector<double*> A, B;
  double *Rres, *T1, *M, *omega, *Y, *Y2, *G, *R, *Bk, *H, *eigw, *evals, *Z, *S, *keep, *sign, *U2;
};

ZipBufs carve_zip(Ctx& X, Carver& cv, const ZipShape& z) {
  ZipBufs b;
  b.A.resize(z.L); b.B.resize(z.L);
  for (int l = 0; l < z.L; ++l) {
    b.A[l] = cv.take<double>((size_t)z.core_a);
    b.B[l] = cv.take<double>((size_t)z.core_b);
  }
  const long long coremax = std::max(z.core_a, z.core_b);
  const long long kq = std::max<long long>(
      {*std::max_element(z.ca.begin(), z.ca.end()), *std::max_element(z.cb.begin(), z.cb.end()), 1});
  X.iRt = cv.take<double>((size_t)kq * kq);
  X.iTau = cv.take<double>((size_t)kq);
  X.iTmp = cv.take<double>((size_t)coremax);
  X.iXt = cv.take<double>((size_t)coremax);
  b.Rres = cv.take<double>((size_t)z.rmax * z.Kmax);
  b.T1 = cv.take<double>((size_t)z.t1);
  b.M = cv.take<double>((size_t)z.nmax * z.Kmax);
  b.omega = cv.take<double>((size_t)z.Kmax * z.kmax);
  b.Y = cv.take<double>((size_t)z.nmax * std::max(z.kmax, z.hmax));
  b.Y2 = cv.take<double>((size_t)z.nmax * std::max(z.kmax, z.hmax));
  b.G = cv.take<double>((size_t)z.hmax * z.hmax);
  b.R = cv.take<double>(2 * (size_t)z.hmax * z.hmax);
  b.Bk = cv.take<double>((size_t)z.kmax * z.Kmax);
  b.H = cv.take<double>((size_t)z.hmax * z.hmax);
  b.eigw = cv.take<double>(eig_work_doubles((int)z.hmax, (int)z.rmax));
  b.evals = cv.take<double>((size_t)z.hmax);
  b.Z = cv.take<double>((size_t)z.hmax * z.rmax);
  b.S = cv.take<double>((size_t)z.rmax);
  b.keep = cv.take<double>((size_t)z.rmax);
  b.sign = cv.take<double>((size_t)z.rmax);
  b.U2 = cv.take<double>((size_t)z.nmax * z.rmax);
  return b;
}

// RQ sweep of one train (cores in `c`, dims `dims` updated to the
// right-canonical ones), as the fit's initialization does it.
void rec_rq_train(Ctx& X, Program& P, std::vector<double*>& c, std::vector<int>& dims, int dd) {
  const int L = (int)c.size();
  for (int j = L - 1; j >= 1; --j) {
    const int p = dims[j], q = dd * dims[j + 1], mp = dims[j - 1] * dd;
    if (p <= q) {
      add_perm(P, {perm4(c[j], 0, X.iXt, 0, {1, 1, p, q}, {0, 0, q, 1}, {0, 0, 1, p})}, "copy");
      add_hhqr(X, P, X.iXt, q, p, X.iTmp);
      add_perm(P, {perm4(X.iTmp, 0, c[j], 0, {1, 1, q, p}, {0, 0, p, 1}, {0, 0, 1, q})}, "copy");
      add_gemm(P, X.sb, Mode::F64, {GemmJob{mp, p, p, op64(c[j - 1], true, p), op64(X.iRt, true, p),
                                            out64(X.iTmp, p)}}, "init", 0);
      add_perm(P, {perm4(X.iTmp, 0, c[j - 1], 0, {1, 1, mp, p}, {0, 0, p, 1}, {0, 0, p, 1})}, "copy");
    } else {
      add_gemm(P, X.sb, Mode::F64, {GemmJob{mp, q, p, op64(c[j - 1], true, p), op64(c[j], false, q),
                                            out64(X.iTmp, q)}}, "init", 0);
      add_perm(P, {perm4(X.iTmp, 0, c[j - 1], 0, {1, 1, mp, q}, {0, 0, q, 1}, {0, 0, q, 1})}, "copy");
      add_fill(P, {FillDesc{c[j], 0, q, q, 1}});
      dims[j] = q;
    }
  }
}

void zip_run(const mpo_pair& pair, int chi_max, int sketch_p, uint64_t seed, const mpo_tt& out, char* ws,
             size_t ws_bytes, hipStream_t hs, size_t* bytes_only) {
  const ZipShape z = zip_shape(pair, chi_max, sketch_p);
  const int L = z.L, dd = z.dd, d = z.d;
  Ctx X;
  X.stream = hs;
  Carver cv;
  cv.base = ws;
  carve_aux(X, cv, false);
  ZipBufs b = carve_zip(X, cv, z);
  if (bytes_only) {
    *bytes_only = cv.off + 256;
    return;
  }
  if (cv.off + 256 > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "workspace too small"};
  if (out.L != L || out.d != d || !out.chi || !out.cores) throw Error{MPO_ERR_SHAPE, "output train: L, d"};
  for (int l = 0; l <= L; ++l)
    if (out.chi[l] != z.r[l]) throw Error{MPO_ERR_SHAPE, "output bond dims: see mpo_zipup_bytes"};
  for (int l = 0; l < L; ++l)
    if (!out.cores[l]) throw Error{MPO_ERR_INVALID_ARG, "null output core"};
  Program zp;
  add_fill(zp, {FillDesc{X.flag, 4, 0, 0, 0}, FillDesc{X.sb.counters, X.sb.ccap, 0, 0, 0}});
  upload(X, zp);
  run_program(zp, X.stream, nullptr);
  Program P;
  std::vector<int> da(pair.A.chi, pair.A.chi + L + 1), db(pair.B.chi, pair.B.chi + L + 1);
  for (int l = 0; l < L; ++l) {
    add_perm(P, {perm4(pair.A.cores[l], 0, b.A[l], 0, {1, 1, da[l], dd * da[l + 1]},
                       {0, 0, (long long)dd * da[l + 1], 1}, {0, 0, (long long)dd * da[l + 1], 1})}, "copy");
    add_perm(P, {perm4(pair.B.cores[l], 0, b.B[l], 0, {1, 1, db[l], dd * db[l + 1]},
                       {0, 0, (long long)dd * db[l + 1], 1}, {0, 0, (long long)dd * db[l + 1], 1})}, "copy");
  }
  rec_rq_train(X, P, b.A, da, dd);
  rec_rq_train(X, P, b.B, db, dd);
  add_fill(P, {FillDesc{b.Rres, 0, 1, 1, 1}});  // R_0 = [[[1]]]
  for (int l = 0; l < L; ++l) {
    const int c0 = z.r[l], a0 = da[l], a1 = da[l + 1], b0 = db[l], b1 = db[l + 1];
    const int n = c0 * dd, K = a1 * b1;
    // T1[c][s][b][t][a'] = sum_a R[c][a][b] A[a][s][t][a'] (batches c, s)
    GemmJob t1{b0, d * a1, a0, op64(b.Rres, false, b0), op64(b.A[l], false, dd * a1), out64(b.T1, d * a1)};
    t1.nb[0] = c0; t1.nb[1] = d;
    t1.A.s[0] = (long long)a0 * b0; t1.A.s[1] = 0;
    t1.B.s[0] = 0; t1.B.s[1] = (long long)d * a1;
    t1.C.s[0] = (long long)d * b0 * d * a1; t1.C.s[1] = (long long)b0 * d * a1;
    add_gemm(P, X.sb, Mode::F64, {t1}, "zip_ext", 0);
    // M[c][s][u][a'][b'] = sum_{b,t} T1[c][s][(b t)][a'] B[(b t)][u][b'] (batches c, s, u)
    double* M = (l == L - 1) ? const_cast<double*>(out.cores[l]) : b.M;
    GemmJob t2{a1, b1, b0 * d, op64(b.T1, false, a1), op64(b.B[l], false, d * b1), out64(M, b1)};
    t2.nb[0] = c0; t2.nb[1] = d; t2.nb[2] = d;
    t2.A.s[0] = (long long)d * b0 * d * a1; t2.A.s[1] = (long long)b0 * d * a1; t2.A.s[2] = 0;
    t2.B.s[0] = 0; t2.B.s[1] = 0; t2.B.s[2] = b1;
    t2.C.s[0] = (long long)dd * a1 * b1; t2.C.s[1] = (long long)d * a1 * b1; t2.C.s[2] = (long long)a1 * b1;
    add_gemm(P, X.sb, Mode::F64, {t2}, "zip_ext", 0);
    if (l == L - 1) break;  // C_L = M_L
    const int r = z.r[l + 1];
    const bool sketch = sketch_p >= 0 && chi_max + sketch_p < std::min(n, K);
    const int k = sketch ? chi_max + sketch_p : std::min(n, K);
    double* U = const_cast<double*>(out.cores[l]);  // n x r
    if (sketch) {
      OmegaDesc o{};
      o.out = b.omega; o.m = K; o.k = k; o.chi = K; o.dd = 1; o.bond = l + 1; o.pair = 0;
      o.stream_mul = 0; o.stream_add = kZipStream; o.stream_base = X.sweep_dev; o.seed = seed;
      add_simple(P, LK::Omega, std::vector<OmegaDesc>{o}, (long long)K * k, "omega");
      add_gemm(P, X.sb, Mode::F64, {GemmJob{n, k, K, op64(M, true, K), op64(b.omega, false, k), out64(b.Y, k)}},
               "sketch", 0);
      CholQRJob qj{b.Y, n, k, k, b.G, b.R, nullptr, b.Y2};
      qj.eta = kRankEta;
      add_cholqr(X, P, {qj}, 2, false, true);
      add_gemm(P, X.sb, Mode::F64, {GemmJob{k, K, n, op64(b.Y, false, k), op64(M, false, K), out64(b.Bk, K)}},
               "project", 0);
      add_gemm(P, X.sb, Mode::F64, {GemmJob{k, k, K, op64(b.Bk, true, K), op64(b.Bk, true, K), out64(b.H, k)}},
               "gram", 0);
    } else if (n <= K) {
      add_gemm(P, X.sb, Mode::F64, {GemmJob{n, n, K, op64(M, true, K), op64(M, true, K), out64(b.H, n)}}, "gram", 0);
    } else {  // M^T M (K x K): right vectors first
      add_gemm(P, X.sb, Mode::F64, {GemmJob{K, K, n, op64(M, false, K), op64(M, false, K), out64(b.H, K)}}, "gram", 0);
    }
    add_eig(P, X.sb, {EigDesc{b.H, k, k, r, b.evals, b.Z, r, b.eigw, X.flag}}, k <= kRegMax, "eig");
    add_simple(P, LK::Sval, std::vector<SvalDesc>{SvalDesc{b.evals, b.S, r, 0, X.flag, b.keep, X.flag + 2}}, r,
               "svals");
    add_simple(P, LK::Scale, std::vector<ScaleDesc>{ScaleDesc{b.Z, b.Z, k, r, r, r, nullptr, b.keep, 0, 2}},
               (long long)k * r, "scale");
    if (sketch) {  // U = Q Z
      add_gemm(P, X.sb, Mode::F64, {GemmJob{n, r, k, op64(b.Y, true, k), op64(b.Z, false, r), out64(U, r)}},
               "assemble", 0);
    } else if (n <= K) {
      add_perm(P, {perm4(b.Z, 0, U, 0, {1, 1, n, r}, {0, 0, r, 1}, {0, 0, r, 1})}, "copy");
    } else {  // U = M V / S
      add_gemm(P, X.sb, Mode::F64, {GemmJob{n, r, K, op64(M, true, K), op64(b.Z, false, r), out64(U, r)}},
               "assemble", 0);
      add_simple(P, LK::Scale, std::vector<ScaleDesc>{ScaleDesc{U, U, n, r, r, r, nullptr, b.S, 0, 1}},
                 (long long)n * r, "scale");
    }
    CholQRJob ou{U, n, r, r, b.G, b.R, nullptr, b.U2};
    ou.keep = b.keep;
    add_cholqr(X, P, {ou}, 1, true, true);
    add_simple(P, LK::Sign, std::vector<SignDesc>{SignDesc{U, n, r, r, b.sign, nullptr}}, r, "sign");
    // R_l = U^T M (r x K)
    add_gemm(P, X.sb, Mode::F64, {GemmJob{r, K, n, op64(U, false, r), op64(M, false, K), out64(b.Rres, K)}},
             "env_update", 0);
  }
  upload(X, P);
  run_program(P, X.stream, nullptr);
  HIP_OK(hipStreamSynchronize(X.stream));
  check_flags(X);
}

// ------------------------------------------------------------------ bond projection
// Randomized projection of every inner bond of one MPO (Sec. 3.2): Q_l from
// the Gaussian range finder on the row space of core l-1's right unfolding
// X (Y = X^T Omega, Householder QR with diag(R) >= 0), projected cores
// Q_{l-1}^T A_l Q_l.  A bond with k >= chi_l is kept (Q_l = I, no launch).
struct ProjLayout {
  std::vector<int> k;                       // projected bond dims (k_0 = k_L = 1)
  std::vector<double*> om, y, q, R, tau, t; // per bond l (om..tau) and per site (t)
};

void validate_proj(const mpo_tt& in, int32_t k) {
  if (in.L < 2 || in.d < 1) throw Error{MPO_ERR_SHAPE, "bond projection: L >= 2 and d >= 1"};
  validate_tt(in, in.L, in.d);
  if (k < 1) throw Error{MPO_ERR_INVALID_ARG, "bond projection: k >= 1"};
  if (k > 1024) throw Error{MPO_ERR_UNSUPPORTED, "bond projection: k above 1024"};
  for (int l = 1; l < in.L; ++l)
    if (in.chi[l] > 4096) throw Error{MPO_ERR_UNSUPPORTED, "bond projection: bond above 4096"};
}

ProjLayout carve_proj(Carver& cv, const mpo_tt& in, int k) {
  const int L = in.L, dd = in.d * in.d;
  ProjLayout P;
  P.k.assign(L + 1, 1);
  P.om.assign(L + 1, nullptr); P.y = P.om; P.q = P.om; P.R = P.om; P.tau = P.om;
  P.t.assign(L, nullptr);
  for (int l = 1; l < L; ++l) P.k[l] = std::min(k, in.chi[l]);
  for (int l = 1; l < L; ++l) {
    const int chi = in.chi[l], kl = P.k[l];
    if (kl >= chi) continue;
    const long long m = (long long)in.chi[l - 1] * dd;
    P.om[l] = cv.take<double>((size_t)m * kl);
    P.y[l] = cv.take<double>((size_t)chi * kl);
    P.q[l] = cv.take<double>((size_t)chi * kl);
    P.R[l] = cv.take<double>((size_t)kl * kl);
    P.tau[l] = cv.take<double>((size_t)kl);
  }
  for (int i = 0; i < L; ++i)
    if (i > 0 && P.k[i] < in.chi[i]) P.t[i] = cv.take<double>((size_t)P.k[i] * dd * in.chi[i + 1]);
  return P;
}

size_t proj_bytes(const mpo_tt& in, int k) {
  Ctx X;
  Carver cv;
  carve_aux(X, cv, true);
  carve_proj(cv, in, k);
  return cv.off + 256;
}

void proj_run(const mpo_tt& in, int32_t k, uint64_t seed, int32_t pair, int32_t stream, const mpo_tt& out,
              char* ws, size_t ws_bytes, hipStream_t hs) {
  const int L = in.L, dd = in.d * in.d;
  if (proj_bytes(in, k) > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "workspace too small"};
  Ctx X;
  X.stream = hs;
  Carver cv;
  cv.base = ws;
  carve_aux(X, cv, true);
  ProjLayout Pl = carve_proj(cv, in, k);
  if (out.L != L || out.d != in.d || !out.chi || !out.cores) throw Error{MPO_ERR_SHAPE, "output train: L, d"};
  for (int l = 0; l <= L; ++l)
    if (out.chi[l] != Pl.k[l]) throw Error{MPO_ERR_SHAPE, "output bond dims must be min(k, chi_l)"};
  for (int i = 0; i < L; ++i)
    if (!out.cores[i]) throw Error{MPO_ERR_INVALID_ARG, "null output core"};
  Program z;
  add_fill(z, {FillDesc{X.flag, 4, 0, 0, 0}, FillDesc{X.sb.counters, X.sb.ccap, 0, 0, 0}});
  upload(X, z);
  run_program(z, X.stream, nullptr);
  Program P;
  std::vector<OmegaDesc> om;
  std::vector<GemmJob> yj, lj, rj;
  std::vector<GeqrDesc> gq;
  std::vector<OrgqrDesc> oq;
  std::vector<HhqrDesc> hq;
  bool fused = true;
  std::vector<PermDesc> cp;
  long long maxom = 1;
  for (int l = 1; l < L; ++l) {
    const int chi = in.chi[l], kl = Pl.k[l];
    if (kl >= chi) continue;
    const int m = in.chi[l - 1] * dd;
    OmegaDesc o{};
    o.out = Pl.om[l]; o.m = m; o.k = kl; o.chi = m; o.dd = 1; o.bond = l; o.pair = pair;
    o.stream_mul = 0; o.stream_add = stream; o.stream_base = X.sweep_dev; o.seed = seed;
    om.push_back(o);
    maxom = std::max(maxom, (long long)m * kl);
    // Y = X^T Omega, X = core l-1 as (chi_{l-1} d^2) x chi_l
    yj.push_back(GemmJob{chi, kl, m, op64(in.cores[l - 1], false, chi), op64(Pl.om[l], false, kl),
                         out64(Pl.y[l], kl)});
    gq.push_back(GeqrDesc{Pl.y[l], chi, kl, kl, Pl.R[l], kl, Pl.tau[l]});
    oq.push_back(OrgqrDesc{Pl.y[l], chi, kl, kl, Pl.tau[l], Pl.q[l], kl, Pl.R[l], kl});
    hq.push_back(HhqrDesc{Pl.y[l], chi, kl, kl, Pl.tau[l], Pl.q[l], kl, Pl.R[l], kl});
    fused = fused && hhqr_fits_lds(chi, kl);
  }
  for (int i = 0; i < L; ++i) {
    const int cl = in.chi[i], cr = in.chi[i + 1], kl = Pl.k[i], kr = Pl.k[i + 1];
    const bool left = i > 0 && kl < cl, right = i + 1 < L && kr < cr;
    const double* src = in.cores[i];
    if (left) {  // Q_i^T core_i: (k_i) x (d^2 chi_{i+1})
      lj.push_back(GemmJob{kl, dd * cr, cl, op64(Pl.q[i], false, kl), op64(src, false, dd * cr),
                           out64(Pl.t[i], dd * cr)});
      src = Pl.t[i];
    }
    double* dst = const_cast<double*>(out.cores[i]);
    if (right)  // (.) Q_{i+1}: (k_i d^2) x k_{i+1}
      rj.push_back(GemmJob{kl * dd, kr, cr, op64(src, true, cr), op64(Pl.q[i + 1], false, kr), out64(dst, kr)});
    else
      cp.push_back(perm4(src, 0, dst, 0, {1, 1, kl * dd, cr}, {0, 0, cr, 1}, {0, 0, cr, 1}));
  }
  add_simple(P, LK::Omega, om, maxom, "project");
  add_gemm(P, X.sb, Mode::F64, yj, "project", 0);
  if (fused) {
    add_hhqr_group(P, hq, "project");
  } else {
    add_simple(P, LK::Geqr, gq, 0, "project");
    add_simple(P, LK::Orgqr, oq, 0, "project");
  }
  add_gemm(P, X.sb, Mode::F64, lj, "project", 0);
  add_gemm(P, X.sb, Mode::F64, rj, "project", 0);
  add_perm(P, cp, "copy");
  upload(X, P);
  run_program(P, X.stream, nullptr);
  HIP_OK(hipStreamSynchronize(X.stream));
  check_flags(X);
}
}  // namespace

extern "C" {

const char* mpo_last_error(void) { return g_last_error.c_str(); }

mpo_status mpo_fit_workspace_bytes(const mpo_pair* pairs, int32_t n_pairs, const mpo_fit_opts* opts,
                                   size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw Error{MPO_ERR_INVALID_ARG, "null bytes"};
    Ctx X;
    setup(X, pairs, n_pairs, opts);
    Carver cv;
    carve(X, cv);
    *bytes = cv.off + 256;
  });
}

mpo_status mpo_fit_init(mpo_fit_ctx** ctx, const mpo_pair* pairs, int32_t n_pairs,
                        const mpo_fit_opts* opts, void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    if (!ctx || !workspace) throw Error{MPO_ERR_INVALID_ARG, "null ctx or workspace"};
    if (reinterpret_cast<uintptr_t>(workspace) & 255) throw Error{MPO_ERR_WORKSPACE, "workspace not 256-byte aligned"};
    auto c = std::make_unique<mpo_fit_ctx>();
    Ctx& X = c->X;
    setup(X, pairs, n_pairs, opts);
    Carver meas;
    carve(X, meas);
    if (meas.off + 256 > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "workspace too small"};
    Carver cv;
    cv.base = static_cast<char*>(workspace);
    carve(X, cv);
    X.ws_bytes = ws_bytes;
    X.stream = static_cast<hipStream_t>(stream);
    HIP_OK(hipGetDevice(&X.device));
    // zero the status flags, sweep counter and split-K counters
    Program z;
    add_fill(z, {FillDesc{X.flag, 4, 0, 0, 0}, FillDesc{X.sb.counters, X.sb.ccap, 0, 0, 0}});
    if (X.o.first_sweep > 0) {  // the Philox stream index of the first sweep
      Launch b;
      b.kind = LK::Bump;
      b.counter = X.sweep_dev;
      b.bump_by = X.o.first_sweep;
      b.cls = "bump";
      z.launches.push_back(b);
    }
    upload(X, z);
    run_program(z, X.stream, nullptr);
    Program init;
    for (size_t p = 0; p < X.pairs.size(); ++p) rec_init_pair(X, init, X.pairs[p], (int)p);
    upload(X, init);
    run_program(init, X.stream, nullptr);
    for (auto& S : X.pairs) {
      if (S.rk)  // the initial guess's dims; the tolerance rule updates them on the device
        HIP_OK(hipMemcpyAsync(S.rk, S.cC.data(), S.cC.size() * sizeof(int), hipMemcpyHostToDevice, X.stream));
      double nu[2];
      HIP_OK(hipMemcpyAsync(nu, S.nu_dev, sizeof(nu), hipMemcpyDeviceToHost, X.stream));
      HIP_OK(hipStreamSynchronize(X.stream));
      S.nu = nu[0] * nu[1];
    }
    // the init descriptors are not needed again
    X.arena_used = 0;
    check_flags(X);
    if (X.o.track_error) err_init(X);
    X.pos = X.o.schedule == MPO_SCHED_SERIAL ? X.o.first_bond : X.o.first_half;
    HIP_OK(hipEventCreate(&X.ev0));
    HIP_OK(hipEventCreate(&X.ev1));
    *ctx = c.release();
  });
}

mpo_status mpo_fit_sweep(mpo_fit_ctx* ctx, int32_t n_sweeps, double* fit_err) {
  return guarded([&] {
    if (!ctx || n_sweeps < 0) throw Error{MPO_ERR_INVALID_ARG, "null ctx or negative sweeps"};
    Ctx& X = ctx->X;
    if (fit_err && !X.o.track_error)
      throw Error{MPO_ERR_INVALID_ARG, "fit_err needs a context created with opts.track_error = 1"};
    if (X.merged) throw Error{MPO_ERR_UNSUPPORTED, "the parallel fit has been merged"};
    HIP_OK(hipEventRecord(X.ev0, X.stream));
    X.prof.clear();
    for (int s = 0; s < n_sweeps; ++s) {
      run_segment(ctx, X.pos, sweep_units(X) - X.pos);  // a resumed sweep finishes first
      if (fit_err) {  // after the timed region of this sweep: transfer passes on the result
        HIP_OK(hipEventRecord(X.ev1, X.stream));
        for (size_t p = 0; p < X.pairs.size(); ++p)
          fit_err[p * (size_t)n_sweeps + s] = sweep_error(X, (int)p);
      }
    }
    if (!fit_err) HIP_OK(hipEventRecord(X.ev1, X.stream));
    check_flags(X);
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, X.ev0, X.ev1));
    X.last_ms = ms;
  });
}

mpo_status mpo_fit_updates(mpo_fit_ctx* ctx, int32_t n_units) {
  return guarded([&] {
    if (!ctx || n_units < 0) throw Error{MPO_ERR_INVALID_ARG, "null ctx or negative count"};
    Ctx& X = ctx->X;
    if (X.o.schedule == MPO_SCHED_SERIAL && X.pairs.size() != 1 && n_units % sweep_units(X) != 0)
      throw Error{MPO_ERR_UNSUPPORTED, "single updates need one pair"};
    if (X.merged) throw Error{MPO_ERR_UNSUPPORTED, "the parallel fit has been merged"};
    X.prof.clear();
    HIP_OK(hipEventRecord(X.ev0, X.stream));
    while (n_units > 0) {
      const int m = std::min(n_units, sweep_units(X) - X.pos);
      run_segment(ctx, X.pos, m);
      n_units -= m;
    }
    HIP_OK(hipEventRecord(X.ev1, X.stream));
    check_flags(X);
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, X.ev0, X.ev1));
    X.last_ms = ms;
  });
}

mpo_status mpo_fit_position(const mpo_fit_ctx* ctx, int32_t* sweep, int32_t* unit) {
  return guarded([&] {
    if (!ctx) throw Error{MPO_ERR_INVALID_ARG, "null ctx"};
    if (sweep) *sweep = ctx->X.o.first_sweep + ctx->X.sweeps_done;
    if (unit) *unit = ctx->X.pos;
  });
}

mpo_status mpo_fit_bond_dims(const mpo_fit_ctx* ctx, int32_t pair, int32_t* chi_c) {
  return guarded([&] {
    if (!ctx || !chi_c) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    if (pair < 0 || pair >= (int)ctx->X.pairs.size()) throw Error{MPO_ERR_INVALID_ARG, "bad pair"};
    const auto c = current_dims(ctx->X, ctx->X.pairs[pair]);
    for (size_t i = 0; i < c.size(); ++i) chi_c[i] = c[i];
  });
}

mpo_status mpo_fit_merge(mpo_fit_ctx* ctx) {
  return guarded([&] {
    if (!ctx) throw Error{MPO_ERR_INVALID_ARG, "null ctx"};
    Ctx& X = ctx->X;
    if (X.o.schedule != MPO_SCHED_PARALLEL) throw Error{MPO_ERR_UNSUPPORTED, "merge: parallel schedule only"};
    if (X.merged) throw Error{MPO_ERR_UNSUPPORTED, "the parallel fit has been merged"};
    if (X.pos != 0) throw Error{MPO_ERR_UNSUPPORTED, "merge: the fit stands inside a set"};
    Program P;
    rec_par_merge(X, P, X.pairs[0]);
    const size_t keep = X.arena_used;
    upload(X, P);
    HIP_OK(hipEventRecord(X.ev0, X.stream));
    run_program(P, X.stream, nullptr);
    HIP_OK(hipEventRecord(X.ev1, X.stream));
    HIP_OK(hipStreamSynchronize(X.stream));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, X.ev0, X.ev1));
    X.last_ms = ms;
    X.arena_used = keep;
    X.merged = true;
    check_flags(X);
  });
}

mpo_status mpo_fit_export_c(mpo_fit_ctx* ctx, int32_t pair, double* const* c_cores) {
  return guarded([&] {
    if (!ctx || !c_cores) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    Ctx& X = ctx->X;
    if (pair < 0 || pair >= (int)X.pairs.size()) throw Error{MPO_ERR_INVALID_ARG, "bad pair"};
    if (X.o.schedule == MPO_SCHED_PARALLEL && !X.merged)
      throw Error{MPO_ERR_UNSUPPORTED, "the parallel fit's sub-TTs disagree in gauge until mpo_fit_merge"};
    PairState& S = X.pairs[pair];
    Program P;
    std::vector<PermDesc> ds;
    std::vector<ScaleDesc> sc;
    const bool inv = X.o.schedule == MPO_SCHED_EVEN_ODD;
    const std::vector<int> c = current_dims(X, S);
    for (int i = 0; i < S.L; ++i) {
      if (!c_cores[i]) throw Error{MPO_ERR_INVALID_ARG, "null output core"};
      ds.push_back(export_core(S, i, c, c_cores[i], i == 0 ? S.nu : 1.0));
      if (inv && i + 1 < S.L)  // merged form C_l = Psi_l Y_l
        sc.push_back(ScaleDesc{c_cores[i], c_cores[i], c[i] * S.dd, c[i + 1], c[i + 1], c[i + 1], nullptr,
                               S.Yv[i + 1], 0, 1});
    }
    add_perm(P, ds, "export");
    long long mx = 1;
    for (auto& d : sc) mx = std::max(mx, (long long)d.n * d.r);
    add_simple(P, LK::Scale, sc, mx, "export");
    const size_t keep = X.arena_used;
    upload(X, P);
    run_program(P, X.stream, nullptr);
    HIP_OK(hipStreamSynchronize(X.stream));
    X.arena_used = keep;
  });
}

mpo_status mpo_fit_singular_values(mpo_fit_ctx* ctx, int32_t pair, int32_t bond, double* S, int32_t* r) {
  return guarded([&] {
    if (!ctx || !S) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    Ctx& X = ctx->X;
    if (pair < 0 || pair >= (int)X.pairs.size()) throw Error{MPO_ERR_INVALID_ARG, "bad pair"};
    PairState& P = X.pairs[pair];
    if (bond < 1 || bond >= P.L) throw Error{MPO_ERR_INVALID_ARG, "bond must be in 1 .. L-1"};
    const int n = current_dims(X, P)[bond];
    HIP_OK(hipMemcpyAsync(S, P.Yv[bond], n * sizeof(double), hipMemcpyDeviceToHost, X.stream));
    HIP_OK(hipStreamSynchronize(X.stream));
    if (r) *r = n;
  });
}

mpo_status mpo_fit_export_psi(mpo_fit_ctx* ctx, int32_t pair, double* const* psi_cores) {
  return guarded([&] {
    if (!ctx || !psi_cores) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    Ctx& X = ctx->X;
    if (X.o.schedule != MPO_SCHED_EVEN_ODD) throw Error{MPO_ERR_UNSUPPORTED, "Psi: even/odd schedule only"};
    if (pair < 0 || pair >= (int)X.pairs.size()) throw Error{MPO_ERR_INVALID_ARG, "bad pair"};
    PairState& S = X.pairs[pair];
    Program P;
    std::vector<PermDesc> ds;
    const std::vector<int> c = current_dims(X, S);
    for (int i = 0; i < S.L; ++i) {
      if (!psi_cores[i]) throw Error{MPO_ERR_INVALID_ARG, "null output core"};
      ds.push_back(export_core(S, i, c, psi_cores[i], 1.0));
    }
    add_perm(P, ds, "export");
    const size_t keep = X.arena_used;
    upload(X, P);
    run_program(P, X.stream, nullptr);
    HIP_OK(hipStreamSynchronize(X.stream));
    X.arena_used = keep;
  });
}

mpo_status mpo_fit_sweeps_done(const mpo_fit_ctx* ctx, int32_t* n) {
  return guarded([&] {
    if (!ctx || !n) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    *n = ctx->X.sweeps_done;
  });
}

mpo_status mpo_fit_norm_factor(const mpo_fit_ctx* ctx, int32_t pair, double* nu) {
  return guarded([&] {
    if (!ctx || !nu) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    if (pair < 0 || pair >= (int)ctx->X.pairs.size()) throw Error{MPO_ERR_INVALID_ARG, "bad pair"};
    *nu = ctx->X.pairs[pair].nu;
  });
}

mpo_status mpo_fit_truncations(const mpo_fit_ctx* ctx, int64_t* n) {
  return guarded([&] {
    if (!ctx || !n) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    *n = ctx->X.n_trunc;
  });
}

mpo_status mpo_fit_last_sweep_ms(const mpo_fit_ctx* ctx, double* ms) {
  return guarded([&] {
    if (!ctx || !ms) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    *ms = ctx->X.last_ms;
  });
}

mpo_status mpo_fit_profile(const mpo_fit_ctx* ctx, int32_t n, double* ms, const char** names,
                           double* flops, int32_t* launches, int32_t* count) {
  return guarded([&] {
    if (!ctx || !count) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    const auto& pm = ctx->X.prof;
    *count = (int)pm.size();
    for (int i = 0; i < n && i < (int)pm.size(); ++i) {
      if (ms) ms[i] = pm[i].ms;
      if (names) names[i] = pm[i].cls.c_str();
      if (flops) flops[i] = pm[i].flops;
      if (launches) launches[i] = pm[i].launches;
    }
  });
}

mpo_status mpo_gemm_autotune(const mpo_pair* pairs, int32_t n_pairs, const mpo_fit_opts* opts,
                             void* workspace, size_t ws_bytes, void* stream, int32_t reps,
                             mpo_gemm_tune* out, int32_t cap, int32_t* n_out) {
  return guarded([&] {
    if (!out || !n_out || cap < 0 || reps < 1) throw Error{MPO_ERR_INVALID_ARG, "bad output or reps"};
    mpo_fit_opts o = *opts;
    o.tune = nullptr;
    o.n_tune = 0;
    o.capture_graph = 0;
    o.profile = 0;
    mpo_fit_ctx* raw = nullptr;
    const mpo_status st = mpo_fit_init(&raw, pairs, n_pairs, &o, workspace, ws_bytes, stream);
    if (st != MPO_OK) throw Error{st, g_last_error};
    std::unique_ptr<mpo_fit_ctx, void (*)(mpo_fit_ctx*)> ctx(raw, mpo_fit_destroy);
    const mpo_status st2 = mpo_fit_sweep(raw, 1, nullptr);
    if (st2 != MPO_OK) throw Error{st2, g_last_error};
    Ctx& X = raw->X;
    // the launch classes of the next sweep
    std::vector<std::pair<Mode, std::vector<GemmJob>>> rec;
    {
      SweepPlan sp;
      X.sb.record = &rec;
      const std::vector<std::vector<int>> keep = [&] {
        std::vector<std::vector<int>> v;
        for (auto& S : X.pairs) v.push_back(S.cC);
        return v;
      }();
      record_segment(X, sp, (X.o.first_sweep + X.sweeps_done) % 2 == 0, X.pos, sweep_units(X) - X.pos);
      X.sb.record = nullptr;
      for (size_t p = 0; p < X.pairs.size(); ++p) X.pairs[p].cC = keep[p];
    }
    std::vector<mpo_gemm_tune> best;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const size_t arena_mark = X.arena_used;
    try {
      for (auto& r : rec) {
        const mpo_gemm_tune key = gemm_class(r.first, r.second);
        bool seen = false;
        for (auto& b : best) seen = seen || same_class(b, key);
        if (seen) continue;
        mpo_gemm_tune win = key;
        win.us = -1;
        const std::vector<int> tiles = r.first == Mode::F64 ? std::vector<int>{0, 3, 4, 5}
                                                            : std::vector<int>{0, 1, 2, 3, 4};
        for (int tile : tiles) {
          for (int sp : {1, 2, 4, 8, 16}) {
            if (sp > 1 && (tile == 5 || key.K / sp < gemm_bk(r.first, tile))) continue;
            Program P;
            X.sb.force_tile = tile;
            X.sb.force_splits = sp;
            add_gemm_kind(P, X.sb, r.first, r.second, "tune", 0);
            X.sb.force_tile = -1;
            X.sb.force_splits = 0;
            if (tile == 1 && P.launches[0].gk.tile != 1) continue;  // tile not possible here
            upload(X, P);
            run_program(P, X.stream, nullptr);  // warm-up
            HIP_OK(hipEventRecord(e0, X.stream));
            for (int q = 0; q < reps; ++q) run_program(P, X.stream, nullptr);
            HIP_OK(hipEventRecord(e1, X.stream));
            HIP_OK(hipEventSynchronize(e1));
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            X.arena_used = arena_mark;
            const float us = ms * 1000.f / reps;
            if (win.us < 0 || us < win.us) {
              win.us = us;
              win.tile = tile;
              win.splits = sp;
            }
          }
        }
        best.push_back(win);
      }
    } catch (...) {
      X.sb.force_tile = -1;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    HIP_OK(hipEventDestroy(e0));
    HIP_OK(hipEventDestroy(e1));
    HIP_OK(hipStreamSynchronize(X.stream));
    *n_out = (int32_t)std::min<size_t>(best.size(), (size_t)cap);
    for (int i = 0; i < *n_out; ++i) out[i] = best[i];
  });
}

mpo_status mpo_fit_grad_workspace_bytes(const mpo_fit_ctx* ctx, int32_t pair, const mpo_tt* W,
                                        int32_t recompute_env, size_t* bytes) {
  return guarded([&] {
    if (!ctx || !W || !bytes) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    Ctx& X = const_cast<Ctx&>(ctx->X);
    if (pair < 0 || pair >= (int)X.pairs.size()) throw Error{MPO_ERR_INVALID_ARG, "bad pair index"};
    PairState& S = X.pairs[pair];
    const int centre = grad_centre(X) < 0 ? S.L - 1 : 0;
    validate_tt(*W, S.L, S.d);
    std::vector<const double*> nulls(S.L, nullptr);
    std::vector<double*> gnull(S.L, nullptr);
    mpo_tt A{S.L, S.d, S.chiA_in.data(), nulls.data()}, B{S.L, S.d, S.chiB_in.data(), nulls.data()};
    Program P;
    Arena ar;
    ar.cv.off = 256;  // the loss slot
    rec_grad(X, P, ar, S, A, B, *W, gnull.data(), gnull.data(), centre, recompute_env != 0, nullptr);
    *bytes = ar.peak + 256;
  });
}

mpo_status mpo_fit_grad(mpo_fit_ctx* ctx, int32_t pair, const mpo_pair* ab, const mpo_tt* W,
                        double* const* gA, double* const* gB, double* loss, int32_t recompute_env,
                        void* workspace, size_t ws_bytes) {
  return guarded([&] {
    if (!ctx || !gA || !gB || !loss || !workspace) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    if (reinterpret_cast<uintptr_t>(workspace) & 255) throw Error{MPO_ERR_WORKSPACE, "workspace not 256-byte aligned"};
    Ctx& X = ctx->X;
    if (pair < 0 || pair >= (int)X.pairs.size()) throw Error{MPO_ERR_INVALID_ARG, "bad pair index"};
    PairState& S = X.pairs[pair];
    const int centre = grad_centre(X) < 0 ? S.L - 1 : 0;
    validate_grad(X, S, ab, W);
    for (int l = 0; l < S.L; ++l)
      if (!gA[l] || !gB[l]) throw Error{MPO_ERR_INVALID_ARG, "null gradient core"};
    Program P;
    Arena ar;
    ar.cv.base = static_cast<char*>(workspace);
    ar.cv.off = 256;
    double* loss_dev = static_cast<double*>(workspace);
    rec_grad(X, P, ar, S, ab->A, ab->B, *W, gA, gB, centre, recompute_env != 0, loss_dev);
    if (ar.peak > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "gradient workspace too small"};
    const size_t arena_mark = X.arena_used;
    upload(X, P);
    run_program(P, X.stream, nullptr);
    HIP_OK(hipMemcpyAsync(loss, loss_dev, sizeof(double), hipMemcpyDeviceToHost, X.stream));
    HIP_OK(hipStreamSynchronize(X.stream));
    X.arena_used = arena_mark;
    check_flags(X);
  });
}

mpo_status mpo_zipup_bytes(const mpo_pair* pair, int32_t chi_max, int32_t sketch_p, int32_t* dims,
                           size_t* bytes) {
  return guarded([&] {
    if (!pair || !bytes) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    if (chi_max < 1) throw Error{MPO_ERR_INVALID_ARG, "chi_max >= 1"};
    if (chi_max + std::max(sketch_p, 0) > 512) throw Error{MPO_ERR_UNSUPPORTED, "chi_max + sketch_p above 512"};
    validate_check(*pair, pair->A);
    if (pair->A.L < 2) throw Error{MPO_ERR_SHAPE, "zip-up: L >= 2"};
    const ZipShape z = zip_shape(*pair, chi_max, sketch_p);
    if (dims)
      for (int l = 0; l <= z.L; ++l) dims[l] = z.r[l];
    zip_run(*pair, chi_max, sketch_p, 0, pair->A, nullptr, 0, nullptr, bytes);
  });
}

mpo_status mpo_zipup(const mpo_pair* pair, int32_t chi_max, int32_t sketch_p, uint64_t seed, const mpo_tt* C,
                     void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    if (!pair || !C || !workspace) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    if (reinterpret_cast<uintptr_t>(workspace) & 255) throw Error{MPO_ERR_WORKSPACE, "workspace not 256-byte aligned"};
    if (chi_max < 1) throw Error{MPO_ERR_INVALID_ARG, "chi_max >= 1"};
    if (chi_max + std::max(sketch_p, 0) > 512) throw Error{MPO_ERR_UNSUPPORTED, "chi_max + sketch_p above 512"};
    validate_check(*pair, pair->A);
    if (pair->A.L < 2) throw Error{MPO_ERR_SHAPE, "zip-up: L >= 2"};
    zip_run(*pair, chi_max, sketch_p, seed, *C, static_cast<char*>(workspace), ws_bytes,
            static_cast<hipStream_t>(stream), nullptr);
  });
}

mpo_status mpo_bond_project_bytes(const mpo_tt* in, int32_t k, size_t* bytes) {
  return guarded([&] {
    if (!in || !bytes) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    validate_proj(*in, k);
    *bytes = proj_bytes(*in, k);
  });
}

mpo_status mpo_bond_project(const mpo_tt* in, int32_t k, uint64_t seed, int32_t pair, int32_t stream,
                            const mpo_tt* out, void* workspace, size_t ws_bytes, void* hip_stream) {
  return guarded([&] {
    if (!in || !out || !workspace) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    if (reinterpret_cast<uintptr_t>(workspace) & 255) throw Error{MPO_ERR_WORKSPACE, "workspace not 256-byte aligned"};
    if (stream < 0 || pair < 0) throw Error{MPO_ERR_INVALID_ARG, "stream and pair must be >= 0"};
    validate_proj(*in, k);
    proj_run(*in, k, seed, pair, stream, *out, static_cast<char*>(workspace), ws_bytes,
             static_cast<hipStream_t>(hip_stream));
  });
}

mpo_status mpo_contract_check_bytes(const mpo_pair* pair, const mpo_tt* C, size_t* bytes) {
  return guarded([&] {
    if (!pair || !C || !bytes) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    *bytes = check_bytes(*pair, *C, false);
  });
}

mpo_status mpo_contract_exact_check(const mpo_pair* pair, const mpo_tt* C, double* rel_err,
                                    double* ab_norm2, int32_t* method, void* workspace,
                                    size_t ws_bytes, void* stream) {
  return guarded([&] {
    if (!pair || !C || !rel_err || !workspace) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    if (reinterpret_cast<uintptr_t>(workspace) & 255) throw Error{MPO_ERR_WORKSPACE, "workspace not 256-byte aligned"};
    check_run(*pair, *C, rel_err, ab_norm2, method, static_cast<char*>(workspace), ws_bytes,
              static_cast<hipStream_t>(stream), false);
  });
}

// The same check in the library's static scratch: no allocation at all.
mpo_status mpo_contract_exact_check_static(const mpo_pair* pair, const mpo_tt* C, double* rel_err,
                                           double* ab_norm2, int32_t* method, void* stream) {
  return guarded([&] {
    if (!pair || !C || !rel_err) throw Error{MPO_ERR_INVALID_ARG, "null argument"};
    const size_t need = check_bytes(*pair, *C, true);
    if (need > ::kStaticScratchBytes)
      throw Error{MPO_ERR_WORKSPACE, "check needs " + std::to_string(need) +
                                         " bytes, above the static scratch of " +
                                         std::to_string(::kStaticScratchBytes)};
    char* ws = static_scratch_ptr();
    check_run(*pair, *C, rel_err, ab_norm2, method, ws, ::kStaticScratchBytes,
              static_cast<hipStream_t>(stream), true);
  });
}

void mpo_fit_destroy(mpo_fit_ctx* ctx) {
  if (!ctx) return;
  for (auto& kv : ctx->plans)
    if (kv.second.graph) (void)hipGraphExecDestroy(kv.second.graph);
  for (auto e : ctx->evs) (void)hipEventDestroy(e);
  if (ctx->X.ev0) (void)hipEventDestroy(ctx->X.ev0);
  if (ctx->X.ev1) (void)hipEventDestroy(ctx->X.ev1);
  delete ctx;
}

}  // extern "C"

// ====================================================================== test hooks
#include "../../include/mpofit_test.h"

namespace {
struct TestEnv {
  Ctx X;
  Carver cv;
  TestEnv(void* ws, size_t bytes, void* stream) {
    if (!ws || bytes < ((size_t)64 << 20)) throw Error{MPO_ERR_WORKSPACE, "test workspace < 64 MiB"};
    if (reinterpret_cast<uintptr_t>(ws) & 255) throw Error{MPO_ERR_WORKSPACE, "workspace not 256-byte aligned"};
    cv.base = static_cast<char*>(ws);
    X.stream = static_cast<hipStream_t>(stream);
    X.flag = cv.take<int>(4);
    X.sweep_dev = X.flag + 1;
    X.sb.cap = (size_t)16 << 20;
    X.sb.partials = cv.take<char>(X.sb.cap);
    X.sb.ccap = 1 << 14;
    X.sb.counters = cv.take<int>(X.sb.ccap);
    X.arena_cap = (size_t)4 << 20;
    X.arena = cv.take<char>(X.arena_cap);
    if (cv.off > bytes) throw Error{MPO_ERR_WORKSPACE, "test workspace too small"};
    Program z;
    add_fill(z, {FillDesc{X.flag, 4, 0, 0, 0}, FillDesc{X.sb.counters, X.sb.ccap, 0, 0, 0}});
    go(z);
  }
  void go(Program& P) {
    upload(X, P);
    run_program(P, X.stream, nullptr);
    HIP_OK(hipStreamSynchronize(X.stream));
  }
};
}  // namespace

extern "C" {

mpo_status mpo_test_gemm(int mode, int ta, int tb, int tc, int a_kcontig, int b_kcontig, int tile,
                         int M, int N, int K, const void* A, int lda, const void* B, int ldb, void* Cm,
                         int ldc, double alpha, int beta, int splits, void* workspace, size_t ws_bytes,
                         void* stream) {
  return guarded([&] {
    TestEnv T(workspace, ws_bytes, stream);
    Program P;
    const Mode md = (Mode)mode;
    GemmKind gk{md, (DType)ta, (DType)tb, (DType)tc, a_kcontig != 0, b_kcontig != 0, tile};
    const int BM = gemm_bm(tile), BN = gemm_bn(tile), BK = gemm_bk(md, tile);
    GemmDesc d{};
    d.A = A; d.B = B; d.C = Cm; d.M = M; d.N = N; d.K = K; d.lda = lda; d.ldb = ldb; d.ldc = ldc;
    d.nb[0] = d.nb[1] = d.nb[2] = 1;
    d.tiles_m = ceil_div(M, BM); d.tiles_n = ceil_div(N, BN);
    d.alpha = alpha; d.beta = beta;
    auto vec = [](const void* p, int ld) { return (ld % 4 == 0 && aligned16(p)) ? 1 : 0; };
    d.vec_a = vec(A, lda); d.vec_b = vec(B, ldb);
    const bool f64_tile = tile == 0 || tile >= 3;  // FP64: 0, 3, 4, 5; otherwise 0, 1, 2
    const bool ok_tile = md == Mode::F64 ? f64_tile : tile <= 4;
    if (tile < 0 || tile > 5 || !ok_tile || (tile == 5 && splits > 1))
      throw Error{MPO_ERR_INVALID_ARG, "GEMM tile"};
    int s = std::max(1, splits);
    int kchunk = ceil_div(ceil_div(K, s), BK) * BK;
    s = std::max(1, ceil_div(K, kchunk));
    d.splits = s;
    d.kchunk = s > 1 ? kchunk : std::max(K, 1);
    const size_t need = (size_t)d.tiles_m * d.tiles_n * s * BM * BN * gemm_acc_bytes(md);
    if (s > 1) {
      if (need > T.X.sb.cap) throw Error{MPO_ERR_WORKSPACE, "split-K scratch"};
      d.partials = T.X.sb.partials;
      d.counters = T.X.sb.counters;
    }
    d.wg_begin = 0;
    Launch l;
    l.kind = LK::Gemm; l.gk = gk; l.off = P.push(std::vector<GemmDesc>{d}); l.n = 1;
    l.wgs = (long long)d.tiles_m * d.tiles_n * s;
    l.cls = "gemm";
    P.launches.push_back(l);
    T.go(P);
  });
}

mpo_status mpo_test_eig(const double* H, int k, int r, double* evals, double* Z, void* workspace,
                        size_t ws_bytes, void* stream) {
  return guarded([&] {
    TestEnv T(workspace, ws_bytes, stream);
    double* w = T.cv.take<double>(eig_work_doubles(k, r));
    if (T.cv.off > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "test workspace too small"};
    Program P;
    const bool reg = k <= kRegMax;
    add_eig(P, T.X.sb, {EigDesc{H, k, k, r, evals, Z, r, w, T.X.flag}}, reg, "eig");
    T.go(P);
    check_flags(T.X);
  });
}

mpo_status mpo_test_eig_batch(const double* H, int n, int k, int r, double* evals, double* Z,
                              void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    if (n < 1 || k < 1 || r < 1 || r > k) throw Error{MPO_ERR_INVALID_ARG, "bad eig batch shape"};
    TestEnv T(workspace, ws_bytes, stream);
    const bool reg = k <= kRegMax;
    std::vector<EigDesc> ed;
    for (int i = 0; i < n; ++i) {
      double* w = T.cv.take<double>(eig_work_doubles(k, r));
      const double* Hi = H + (size_t)i * k * k;
      double* Zi = Z + (size_t)i * k * r;
      ed.push_back(EigDesc{Hi, k, k, r, evals + (size_t)i * r, Zi, r, w, T.X.flag});
    }
    if (T.cv.off > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "test workspace too small"};
    Program P;
    add_eig(P, T.X.sb, ed, reg, "eig");
    T.go(P);
    check_flags(T.X);
  });
}

static mpo_status test_cholqr(double* Xm, int n, int k, double eta, void* workspace, size_t ws_bytes,
                              void* stream) {
  return guarded([&] {
    TestEnv T(workspace, ws_bytes, stream);
    double* G = T.cv.take<double>((size_t)k * k);
    double* R = T.cv.take<double>(2 * (size_t)k * k);
    if (T.cv.off > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "test workspace too small"};
    Program P;
    double* Tm = T.cv.take<double>((size_t)n * k);
    if (T.cv.off > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "test workspace too small"};
    CholQRJob j{Xm, n, k, k, G, R, nullptr, Tm};
    j.eta = eta;
    add_cholqr(T.X, P, {j}, 2, false, eta > 0.0);
    T.go(P);
    check_flags(T.X);
  });
}

mpo_status mpo_test_cholqr(double* Xm, int n, int k, void* workspace, size_t ws_bytes, void* stream) {
  return test_cholqr(Xm, n, k, 0.0, workspace, ws_bytes, stream);
}

mpo_status mpo_test_jacobi(const double* W, int q, double* Ur, double* S, void* workspace, size_t ws_bytes,
                           void* stream) {
  return guarded([&] {
    if (!W || !Ur || !S || q < 1 || q > 512) throw Error{MPO_ERR_INVALID_ARG, "jacobi: q in 1..512"};
    TestEnv T(workspace, ws_bytes, stream);
    double* work = T.cv.take<double>((size_t)q * q);
    if (T.cv.off > ws_bytes) throw Error{MPO_ERR_WORKSPACE, "test workspace too small"};
    Program P;
    Launch l;
    l.kind = LK::Jacobi;
    l.off = P.push(std::vector<JacobiDesc>{JacobiDesc{W, q, q, Ur, q, S, work, 0.0, nullptr}});
    l.n = 1;
    l.maxa = q;
    l.cls = "jacobi";
    P.launches.push_back(l);
    T.go(P);
  });
}

mpo_status mpo_test_cholqr_rr(double* Xm, int n, int k, void* workspace, size_t ws_bytes, void* stream) {
  return test_cholqr(Xm, n, k, kRankEta, workspace, ws_bytes, stream);
}

mpo_status mpo_test_omega(double* out, int chi, int dd, int k, int bond, int stream_idx, int pair,
                          uint64_t seed, void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TestEnv T(workspace, ws_bytes, stream);
    Program P;
    OmegaDesc o{};
    o.out = out; o.m = chi * dd; o.k = k; o.chi = chi; o.dd = dd; o.bond = bond; o.pair = pair;
    o.stream_mul = 0; o.stream_add = stream_idx; o.stream_base = T.X.sweep_dev; o.seed = seed;
    add_simple(P, LK::Omega, std::vector<OmegaDesc>{o}, (long long)o.m * k, "omega");
    T.go(P);
  });
}

}  // extern "C"

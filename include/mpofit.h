/*
 * libmpofit: variational fit C ~ A.B of two matrix product operators on an
 * AMD Instinct MI355X (gfx950), with the randomized two-site update.
 *
 * The problem statement follows Foderà, Ritter, Shinaoka, von Delft,
 * "Parallelized contraction of tensor trains or matrix product operators":
 *   - MPO cores A_l of shape (chi_{l-1}, d_out, d_in, chi_l), chi_0 = chi_L = 1
 *     (Sec. 2, definition of an MPO);
 *   - C = A B contracts the input leg of A with the output leg of B (Sec. 2,
 *     Fig. mpo_mpo (a)); C's cores carry (left, A's out, B's in, right);
 *   - the fit minimizes ||A B - C||_F (Sec. 2.3, Eq. fit_min) by two-site
 *     updates (Sec. 2.3.2-2.3.4, Alg. 3), sweeping as in Alg. 5, optionally
 *     with the randomized SVD of Sec. 3.1, or in the inverse canonical gauge
 *     with all bonds of one parity updated together (Alg. 4 and Sec. 4).
 *
 * Conventions of every entry point:
 *   - Device pointers live on the device current when the call is made and
 *     all work is enqueued on `stream` (a hipStream_t passed as void*; NULL =
 *     the default stream).  Calls return once the work is enqueued, except
 *     where a call documents a host read-back.
 *   - The library never allocates device memory: the caller provides one
 *     workspace blob sized by mpo_fit_workspace_bytes and keeps it, and every
 *     input pointer, alive until mpo_fit_destroy.  The context object itself
 *     is host memory owned by the library.
 *   - Every call returns an mpo_status; no exception or abort crosses the
 *     boundary.  mpo_last_error() gives a message for the last non-OK status
 *     of the calling thread.
 *   - A context is not thread safe; distinct contexts are independent.
 */
#ifndef MPOFIT_H
#define MPOFIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPO_OK = 0,
  MPO_ERR_INVALID_ARG = 1, /* null pointer, bad enum, bad option value        */
  MPO_ERR_SHAPE = 2,       /* inconsistent bond or physical dimensions        */
  MPO_ERR_WORKSPACE = 3,   /* workspace too small or misaligned (256 bytes)   */
  MPO_ERR_DEVICE = 4,      /* a HIP runtime call failed                       */
  MPO_ERR_NUMERIC = 5,     /* non-finite value or failed Cholesky            */
  MPO_ERR_UNSUPPORTED = 6  /* option combination this build does not run     */
} mpo_status;

/* Arithmetic of the contractions (environment extensions, two-site tensor,
   environment updates).  The QR of the sketch, the truncated SVD and 1/S of
   the inverse gauge are FP64 in every mode. */
typedef enum {
  MPO_FP64 = 0,
  MPO_FP32 = 1,
  MPO_BF16 = 2,  /* BF16 operands (power-of-two per-tensor scale, round to
                    nearest even), FP32 accumulation and FP32 storage */
  MPO_BF16X3 = 3 /* split BF16: each scaled FP32 operand x = hi + lo, hi and lo
                    BF16; three BF16 products per term (lo*hi + hi*lo + hi*hi),
                    FP32 accumulation and storage */
} mpo_precision;

typedef enum {
  MPO_SCHED_SERIAL = 0,  /* Alg. 5: alternating forward/backward sweeps of the
                            site-canonical update of Alg. 3                   */
  MPO_SCHED_EVEN_ODD = 1, /* inverse canonical gauge (Alg. 4): every bond
                            l = 1 (mod 2) together, then every l = 0 (mod 2),
                            from the environments at the half-step's start;
                            one sweep = both half-steps (Sec. 4) */
  MPO_SCHED_PARALLEL = 2  /* site-canonical parallel fit (Sec. 4, variant II),
                            one pair: opts.n_parts sub-TTs (a power of two,
                            each >= 2 sites, the first ones one site longer)
                            swept in lockstep, sub-TT n forward first for
                            even n; one "sweep" = one set of four phases:
                            local half-sweeps, the connections from even to
                            odd sub-TTs, the reversed half-sweeps, the
                            connections from odd to even sub-TTs.  A
                            connection leaves U S on its left site and S V^T
                            on its right one (each sub-TT keeps its own
                            gauge) and rebuilds both environments; Omega of
                            phase q of set t is stream 4 t + q.  The cores
                            form one train only after mpo_fit_merge.  Needs
                            tau = 0, first_sweep = 0, track_error = 0.       */
} mpo_schedule;
/* Drop rule of both schedules: of the r singular values an update keeps,
   those at or below 1e-6 sigma_1 are dropped (value, singular vectors and in
   the inverse gauge the Y entry become zero; the bond keeps its size).  In
   the inverse gauge this is the truncation before inversion that Sec. 2.3.1
   allows; it also makes a two-site matrix of lower rank than r (a product
   with fewer independent states than the bond cap) well defined.  See
   mpo_fit_truncations. */

/* One MPO: L cores, core l (0-based) is a device array of
   chi[l] * d * d * chi[l+1] doubles, row-major (left, out, in, right).  The
   library reads the cores by these sizes: an array of another shape is read
   past its end.  Only the fit (mpo_fit_opts.mps) takes MPS cores
   (chi[l] * d * 1 * chi[l+1]); the zip-up, the bond projection, the check
   and the gradient take MPO cores. */
typedef struct {
  int32_t L;                 /* number of sites, >= 2                         */
  int32_t d;                 /* physical dimension (d_out = d_in = d), >= 1   */
  const int32_t* chi;        /* host array of L+1 bond dims, chi[0]=chi[L]=1  */
  const double* const* cores;/* host array of L device pointers               */
} mpo_tt;

typedef struct {
  mpo_tt A, B;               /* C ~ A B; A and B must share L and d           */
  int32_t chi_max;           /* bond cap of this pair's C; 0 = opts->chi_max  */
} mpo_pair;

typedef struct {
  int32_t chi_max;    /* bond cap chi_C of C (Alg. 3 "maxbonddim"), >= 1      */
  double tau;         /* truncation tolerance of Sec. 2.3.4, finite, >= 0.
                         0: every bond keeps r = min(chi_max, n, m,
                         chi^A_l chi^B_l) values.  > 0: an update keeps the
                         smallest r' <= r with (sum_{j >= r'} sigma_j^2)^(1/2)
                         <= (tau / L) (sum_j sigma_j^2)^(1/2) over the
                         sigma_j it computed (all of the plain SVD, the k of
                         the sketch); r' >= 1.  The bond dims then change
                         on the device during a sweep: the buffers keep the
                         tau = 0 plan's sizes with zero rows and columns
                         beyond r', Omega takes the bond's actual shape, and
                         mpo_fit_bond_dims / mpo_fit_export_c report and
                         copy out the actual dims.  The gradient needs 0.  */
  int32_t precision;  /* mpo_precision                                         */
  int32_t schedule;   /* mpo_schedule                                          */
  int32_t sketch_p;   /* < 0: plain SVD of the two-site matrix; >= 0: RSVD with
                         k = min(chi_max + p, n, m, chi^A_l chi^B_l) columns  */
  uint64_t seed;      /* Philox key word 0 of the Gaussian test matrix        */
  int32_t capture_graph; /* 1: replay each sweep as a captured hipGraph once
                            the bond dimensions have settled                  */
  const struct mpo_gemm_tune* tune; /* optional host table from
                            mpo_gemm_autotune (copied at init); NULL = built-in
                            tile and split-K choice                          */
  int32_t n_tune;
  int32_t profile;    /* 1: time every launch with HIP events, eager, for
                         mpo_fit_profile (no graph replay)                   */
  const mpo_tt* c_init; /* optional initial guesses (Alg. 5 input "initial
                           guess C"), n_pairs host entries, the same L and d
                           as the pair, bond dims <= 512; NULL = A (Sec.
                           2.3.5).  Used as given: right-orthogonalized, or
                           brought to inverse canonical form; only read at
                           init.                                            */
  int32_t first_sweep; /* >= 0: the fit starts as if this many sweeps had
                          run: sweep i (i = first_sweep, first_sweep + 1, ...)
                          takes the Philox stream of sweep i and, serially,
                          runs backward for odd i (Alg. 5).  A serial fit
                          that starts backward left-orthogonalizes the
                          initial guess and precomputes the left
                          environments.  With c_init = the result of i
                          sweeps this resumes that fit.                      */
  int32_t track_error; /* 1: reserve workspace for the fit error per sweep
                          (mpo_fit_sweep's fit_err) and compute ||A B||^2 at
                          init by a four-layer transfer pass; 0: no error   */
  int32_t first_bond;  /* serial schedule, one pair: >= 0 updates of sweep
                          first_sweep already done (0 <= first_bond <= L-2).
                          The initial guess is brought to site-canonical
                          form around the two sites of the next update
                          (QR sweep left of them, RQ sweep right of them)
                          and the environments of both sides are
                          precomputed; with c_init = a fit's state at that
                          point this resumes it mid-sweep.                  */
  int32_t first_half;  /* even/odd schedule: 1 = the first sweep runs only
                          its second half-step (l = 0 mod 2), from the
                          inverse canonical form of the initial guess and
                          its environments; 0 = whole sweeps                */
  int32_t n_parts;     /* parallel schedule: number of sub-TTs; else unused  */
  int32_t mps;         /* 1: the MPO-MPS product of Sec. 1.  B is an MPS,
                          stored as an MPO whose input leg has size 1: its
                          cores are (chi_l, d, 1, chi_r) with B.d = d, and so
                          are C's (the initial guess's, and the exported
                          cores); A keeps (chi_l, d, d, chi_r).  The default
                          initial guess is then B.  Serial and even/odd
                          schedules, no track_error, no gradient
                          (MPO_ERR_UNSUPPORTED).  0: MPO-MPO             */
} mpo_fit_opts;

/* One tuned class of grouped GEMM launches: the operand kind (mode as
   mpo_precision, operand types 0 = FP64 / 1 = FP32, K-contiguity of A and B),
   the largest problem of the launch (M, N, K) and its problem count; the
   chosen output tile (0: 64x64, 1: 128x128, 2: 64x64 with half-depth K
   slabs, the last two FP32/BF16 only; 3: 32x32, 4: 32x32 with deep K
   slabs (128; 64 in split BF16), these two every mode; 5: 16x16 with the K
   range split over the
   workgroup's waves and no split-K, FP64 only; a tile that does not apply
   to the mode falls back to 0) and split-K count, and the measured average launch time
   of that choice. */
typedef struct mpo_gemm_tune {
  int32_t mode, ta, tb, tc, a_kcontig, b_kcontig;
  int32_t M, N, K, count;
  int32_t tile, splits;
  float us;
} mpo_gemm_tune;

typedef struct mpo_fit_ctx mpo_fit_ctx;

/* Bytes of device workspace mpo_fit_init needs for these pairs and options.
   `bytes` is written on success. */
mpo_status mpo_fit_workspace_bytes(const mpo_pair* pairs, int32_t n_pairs,
                                   const mpo_fit_opts* opts, size_t* bytes);

/* Prepares the fit of every pair (Alg. 5 preprocessing): copies the cores,
   left-orthogonalizes A and B (norms split off), takes C = A (or
   opts->c_init) right-orthogonalized (serial) or in inverse canonical form
   (even/odd) as the initial guess (Sec. 2.3.5), and precomputes the
   environments.  The inputs
   may be released once the stream has passed this call.  `workspace` must be
   256-byte aligned and at least mpo_fit_workspace_bytes long.  On success
   *ctx receives a new context. */
mpo_status mpo_fit_init(mpo_fit_ctx** ctx, const mpo_pair* pairs, int32_t n_pairs,
                        const mpo_fit_opts* opts, void* workspace, size_t ws_bytes,
                        void* stream);

/* Runs n_sweeps sweeps of every pair.  Serial: a sweep is one directional
   pass of L-1 updates, the direction alternating from forward (Alg. 5).
   Even/odd: a sweep is two half-steps.  Synchronizes the stream at the end to
   read the device status flags; returns MPO_ERR_NUMERIC if one was raised.
   fit_err (host, nullable; needs opts.track_error): fit_err[p * n_sweeps + s]
   receives ||A B - C||_F / ||A B||_F of pair p after sweep s (Sec. 2.3, Eq.
   fit_min; the error measure of Sec. 5.2), from transfer passes in FP64 on
   the device: eps^2 = 1 - 2 <C, A B>/||A B||^2 + ||C||^2/||A B||^2, which
   floors near 1e-8 (the difference of squares; the caveat of Sec. 5.2).  The
   passes run after each sweep and synchronize; mpo_fit_last_sweep_ms then
   includes those of all but the last sweep. */
mpo_status mpo_fit_sweep(mpo_fit_ctx* ctx, int32_t n_sweeps, double* fit_err);

/* Runs the next n_units units of the fit: two-site updates (serial
   schedule, Alg. 5 order, one pair unless n_units covers whole sweeps) or
   half-steps (even/odd), crossing into the next sweep when the current one
   ends (the Philox stream and direction follow the sweep index).  A sweep
   entered part-way is finished by the next mpo_fit_sweep call before whole
   sweeps run.  Synchronizes the stream; MPO_ERR_NUMERIC as mpo_fit_sweep. */
mpo_status mpo_fit_updates(mpo_fit_ctx* ctx, int32_t n_units);

/* Parallel schedule (Sec. 4, variant II): the binary merge after the sets
   run so far.  Local half-sweeps once more (Omega stream 4 t, t = sets
   run), a forward update at every connection from an even to an odd
   sub-TT with fresh environments on both sides (stream 4 t + 1; each pair
   of sub-TTs becomes one site-canonical train), then for level v = 2, 3,
   ... the adjacent groups of 2^(v-1) sub-TTs are joined: the left group's
   centre moved to its last site by Householder QR sweeps and its left
   environments rebuilt, the right group's centre moved to its first site
   by RQ sweeps and its right environments rebuilt, one forward update at
   the boundary (stream 4 t + v).  Afterwards C is one site-canonical train
   (mpo_fit_export_c), and sweeps are refused.  Synchronizes the stream;
   mpo_fit_last_sweep_ms gives the merge's time.  UNSUPPORTED for other
   schedules, a second call, or a position inside a set. */
mpo_status mpo_fit_merge(mpo_fit_ctx* ctx);

/* Position of the fit: *sweep = index of the current sweep (first_sweep plus
   the sweeps completed), *unit = its units already run (0 = at a sweep
   boundary).  Either pointer may be NULL. */
mpo_status mpo_fit_position(const mpo_fit_ctx* ctx, int32_t* sweep, int32_t* unit);

/* Singular values of bond `bond` (1 <= bond <= L-1, between 0-based sites
   bond-1 and bond) from its last update (serial: the last sweep that passed
   it; even/odd: Lambda of the inverse canonical form, Y = 1/S), of the fit
   on normalized cores (multiply by mpo_fit_norm_factor for C's own), in
   descending order with dropped values zero: S (host) receives
   mpo_fit_bond_dims(...)[bond] doubles, *r (nullable) that count.  Before a
   serial fit's first update the values are zero.  Synchronizes the context
   stream. */
mpo_status mpo_fit_singular_values(mpo_fit_ctx* ctx, int32_t pair, int32_t bond, double* S,
                                   int32_t* r);

/* Current bond dimensions of C for one pair: chi_c receives L+1 ints (host).
   With opts.tau > 0 they are read from the device after the context's
   stream (synchronizes it). */
mpo_status mpo_fit_bond_dims(const mpo_fit_ctx* ctx, int32_t pair, int32_t* chi_c);

/* Copies C of one pair into caller-owned device arrays (FP64, same layout as
   the inputs, bond dims from mpo_fit_bond_dims), C scaled back by the norms
   split off A and B, so that C ~ A B.  Enqueued on the context's stream. */
mpo_status mpo_fit_export_c(mpo_fit_ctx* ctx, int32_t pair, double* const* c_cores);

/* Even/odd schedule: the site tensors Psi_l of the inverse canonical form
   (Sec. 2.3.1) of one pair, of the fit on normalized cores (no norm factor),
   into caller-owned FP64 device arrays shaped like C's cores; with Y_l =
   1 / S_l (mpo_fit_singular_values, zero where dropped) the merged train is
   C_l = Psi_l Y_l.  After a half-step, Psi_l Y_l Psi_{l+1} of an updated
   bond l is its two-site block U S V^T (Alg. 4).  Synchronizes the context
   stream. */
mpo_status mpo_fit_export_psi(mpo_fit_ctx* ctx, int32_t pair, double* const* psi_cores);

/* Number of sweeps run so far. */
mpo_status mpo_fit_sweeps_done(const mpo_fit_ctx* ctx, int32_t* n);

/* The factor nu = ||A|| ||B|| split off by the preprocessing (Alg. 5): the
   fit runs on normalized cores and mpo_fit_export_c multiplies core 0 by nu. */
mpo_status mpo_fit_norm_factor(const mpo_fit_ctx* ctx, int32_t pair, double* nu);

/* Number of singular values dropped so far by the drop rule (both
   schedules; in the inverse gauge also at initialization), all pairs, as of
   the last call that synchronized (mpo_fit_init, mpo_fit_sweep). */
mpo_status mpo_fit_truncations(const mpo_fit_ctx* ctx, int64_t* n);

/* Gradient at frozen truncation bases (not a step of the paper's method; it
   differentiates the fit's result).  After the last sweep C is site-canonical
   with its centre at the last site (after a forward sweep) or the first
   (otherwise, Alg. 3); every other core is an isometry.  With those frozen,
   the fit of a product X is the orthogonal projection Pi(X) onto the MPOs
   that share them and have a free centre core.  For an MPO W on the same
   sites (FP64 device cores):
       loss(A, B) = <W, Pi(A B)>_F = <Pi(W), A B>_F,
   linear in every core; gA[l] = d loss / d A_l and gB[l] = d loss / d B_l are
   written into caller-owned FP64 device arrays shaped like the cores of
   `ab`, which must have the bond dimensions of the fitted pair (usually the
   same A and B; other values give the gradient there, at the same bases).
   Arithmetic: FP64 for an FP64 fit, FP32 otherwise.  `recompute_env` = 1
   stores only every ceil(sqrt(L))-th right environment and recomputes the
   others segment by segment.  Serial schedule only.  `workspace` (256-byte
   aligned) of mpo_fit_grad_workspace_bytes bytes; *loss (host) receives the
   loss; synchronizes the context stream. */
mpo_status mpo_fit_grad_workspace_bytes(const mpo_fit_ctx* ctx, int32_t pair, const mpo_tt* W,
                                        int32_t recompute_env, size_t* bytes);
mpo_status mpo_fit_grad(mpo_fit_ctx* ctx, int32_t pair, const mpo_pair* ab, const mpo_tt* W,
                        double* const* gA, double* const* gB, double* loss, int32_t recompute_env,
                        void* workspace, size_t ws_bytes);

/* Zip-up contraction C ~ A B (Alg. 2, Sec. 2.2), the fit's initial guess
   (pass C as mpo_fit_opts.c_init): copies of A and B are brought to
   right-canonical form (Householder RQ sweeps), then one left-to-right
   pass contracts the residual R_{l-1} with A_l and B_l into R''_l, whose
   matrix M_l ((r_{l-1} d^2) x (chi_A,l chi_B,l), bond dims of the
   right-canonical A and B) is factorized by the truncated SVD of the
   two-site update (rank min(chi_max, rows, chi_A chi_B); the randomized
   range finder of Sec. 3.1 with k = chi_max + sketch_p when that is
   narrower than M_l, else the Gram eigenproblem of its smaller side;
   singular values <= 1e-6 sigma_1 dropped, sign rule on U): C_l = U,
   R_l = U^T M_l; the last core is M_L.  The sketch draws Omega from the
   Philox stream (seed, element counter, bond = l, stream 2^30 + 2, pair 0).
   mpo_zipup_bytes: workspace bytes and, when `dims` is non-null, C's
   bond dims (L+1 entries) into it; host only.
   pair: FP64 device cores of A and B (pair->chi_max ignored); C: caller-
   allocated FP64 device cores with C->chi = those dims; workspace 256-byte
   aligned.  Synchronizes `stream`.  Errors: INVALID_ARG (null pointers,
   chi_max < 1), SHAPE (L < 2, A and B not matching, C's dims),
   UNSUPPORTED (chi_max + sketch_p > 512, a factorization beyond the eigen
   kernels' sizes), WORKSPACE, NUMERIC (device flags). */
mpo_status mpo_zipup_bytes(const mpo_pair* pair, int32_t chi_max, int32_t sketch_p, int32_t* dims,
                           size_t* bytes);
mpo_status mpo_zipup(const mpo_pair* pair, int32_t chi_max, int32_t sketch_p, uint64_t seed, const mpo_tt* C,
                     void* workspace, size_t ws_bytes, void* stream);

/* Randomized bond projection of one MPO (Sec. 3.2, Fig. random_update and
   random_env, Table 1): every inner bond l (1 .. L-1) with k < chi_l is cut
   to k by the projector Q_l Q_l^T, Q_l (chi_l x k) an orthonormal basis of
   X^T Omega (the Gaussian range finder of Sec. 3.1 on the row space of core
   l-1, X = that core unfolded as (chi_{l-1} d^2) x chi_l; Householder QR
   with diag(R) >= 0); Omega is the Philox4x64-10 stream of the update's
   sketch (seed, element counter, bond = l, stream, pair), elements in
   row-major (chi_{l-1} d^2) x k order.  `out` receives the projected cores
   Q_{l-1}^T A_l Q_l, so with every bond projected the fit of the projected
   pair carries out the randomized contractions of Sec. 3.2 (environments
   O(chi^3 k d^3), two-site contraction O(chi^3 k d^4)).  Bonds with
   k >= chi_l are kept.  The projection pays only when the cores' spectra
   across their bonds decay (the caveat of Sec. 3.2): pass the cores as
   given, not orthogonalized.
   in: FP64 device cores; out: caller-allocated FP64 device cores with
   out->chi[l] = min(k, in->chi[l]) (chi[0] = chi[L] = 1), not overlapping
   `in`; stream: any value >= 0 not used by the fit's sweeps
   (MPO_PROJ_STREAM_A / _B below are the conventional ones for A and B);
   workspace 256-byte aligned, of mpo_bond_project_bytes bytes.
   Synchronizes `hip_stream`.  Errors: INVALID_ARG (null pointers, k < 1,
   negative stream or pair), SHAPE (L < 2, bond dims, output dims),
   UNSUPPORTED (a bond above 4096, k above 1024), WORKSPACE. */
enum { MPO_PROJ_STREAM_A = 1 << 30, MPO_PROJ_STREAM_B = (1 << 30) + 1 };
mpo_status mpo_bond_project_bytes(const mpo_tt* in, int32_t k, size_t* bytes);
mpo_status mpo_bond_project(const mpo_tt* in, int32_t k, uint64_t seed, int32_t pair, int32_t stream,
                            const mpo_tt* out, void* workspace, size_t ws_bytes, void* hip_stream);

/* Fit error ||A B - C||_F / ||A B||_F (Sec. 2.3, Eq. fit_min) in FP64 on
   the device, for FP64 device cores A = pair->A, B = pair->B and C on one
   set of L sites with one d.
   Route 0 (every bond with chi_A chi_B + chi_C <= 512): the naive product
   P = A B of Alg. 1 (Sec. 2.1) and the difference MPO [P, -C] (direct sum
   of the trains) are each left-orthogonalized by Householder QR sweeps; the
   last site's norm is the train's norm.  No Gram matrix and no difference
   of squares is formed, so the result is accurate to a few units of
   rounding of ||A B||, far below sqrt(eps) (the error measure of Sec. 5.2
   without its floor).
   Route 1 (larger bonds): transfer passes, ||A B||^2 by a four-layer pass,
   <C, A B> by a three-layer pass, ||C||^2 by a two-layer pass, each
   environment renormalized after every site; eps^2 = 1 - 2 <C, AB>/||AB||^2
   + ||C||^2/||AB||^2 floors near 1e-8 relative.  The four-layer pass holds
   (chi_A chi_B)^2 d^2 doubles per intermediate.
   `workspace` (256-byte aligned) of mpo_contract_check_bytes bytes.
   Synchronizes `stream`; *rel_err, and if non-null *ab_norm2 = ||A B||_F^2
   and *method (0 or 1, the route), are host outputs; MPO_ERR_NUMERIC if
   A B is zero or a pass is not finite. */
mpo_status mpo_contract_check_bytes(const mpo_pair* pair, const mpo_tt* C, size_t* bytes);
mpo_status mpo_contract_exact_check(const mpo_pair* pair, const mpo_tt* C, double* rel_err,
                                    double* ab_norm2, int32_t* method, void* workspace,
                                    size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
   tight serving loops, harnesses that forbid allocation): the same check as
   mpo_contract_exact_check, in the same kernels, with its scratch in a static
   device array of the library (32 MiB, one copy per GPU, held until the
   process ends) instead of a workspace argument.  No allocation of any kind
   is made.  Returns MPO_ERR_WORKSPACE when mpo_contract_check_bytes' figure
   for the compact layout exceeds 32 MiB (route 0 covers the small trains of
   exact-regime checks).  Every call on one GPU uses that GPU's array: calls
   that overlap on one GPU (from several threads or streams) race; the call
   synchronizes `stream` before returning, so sequential calls are safe. */
mpo_status mpo_contract_exact_check_static(const mpo_pair* pair, const mpo_tt* C, double* rel_err,
                                           double* ab_norm2, int32_t* method, void* stream);

/* Device time, in milliseconds, of the last mpo_fit_sweep call's kernels
   between its first and last launch (HIP events on the context stream). */
mpo_status mpo_fit_last_sweep_ms(const mpo_fit_ctx* ctx, double* ms);

/* Per-kernel-class figures of the last mpo_fit_sweep call when the context
   was created with profiling (opts.profile = 1; launches then run eagerly,
   each bracketed by HIP events on the context stream).  For up to `n` classes:
   ms[] device time, flops[] algorithmic flops credited to the class,
   launches[] launch count, all summed over that call's sweeps, and names[]
   (strings owned by the context, valid until the next mpo_fit_sweep).  Any of
   the arrays may be NULL; *count receives the number of classes. */
mpo_status mpo_fit_profile(const mpo_fit_ctx* ctx, int32_t n, double* ms, const char** names,
                           double* flops, int32_t* launches, int32_t* count);

/* Autotuner of the contraction GEMMs.  Builds a throw-away fit of these
   pairs with these options in `workspace` (at least mpo_fit_workspace_bytes),
   runs one sweep so that the bond dimensions settle, then times every GEMM
   launch class of the next sweep's launch program under each candidate
   (tile 64x64; for FP32/BF16 also 64x64 with half-depth K slabs, and
   128x128 when every problem is large enough; the 32x32 tiles; for FP64
   also the 16x16 tile; split-K 1, 2, 4, 8, 16 where K and the tile allow), `reps`
   launches per candidate with
   HIP events, and writes the fastest per class into out[0 .. *n_out - 1]
   (at most `cap`).  Pass the table back through mpo_fit_opts.tune.  The
   workspace contents are undefined afterwards; synchronizes `stream`. */
mpo_status mpo_gemm_autotune(const mpo_pair* pairs, int32_t n_pairs, const mpo_fit_opts* opts,
                             void* workspace, size_t ws_bytes, void* stream, int32_t reps,
                             mpo_gemm_tune* out, int32_t cap, int32_t* n_out);

void mpo_fit_destroy(mpo_fit_ctx* ctx);

const char* mpo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MPOFIT_H */

/*
 * psdproj.h -- C ABI of the MI355X (gfx950) PSD-cone projection library.
 *
 * The library computes the Euclidean projection onto the cone of complex
 * Hermitian positive-semidefinite matrices,
 *
 *     Pi(X) = argmin_{Y >= 0} ||Y - X||_F = V diag(max(lambda, 0)) V^H,
 *
 * which is the cone step u = Pi_C(u~ - v) of the SCS iteration (App. D.1,
 * eq. final_iterates2; Pi_S is the Euclidean projection onto S) and which the
 * paper evaluates by an eigendecomposition with the negative eigenvalues set
 * to zero (App. D.2).  It also computes the derivative of Pi, needed to
 * back-propagate through the projection (App. E).
 *
 * Matrix encoding ("svec"): the paper's real vectorisation vec_R of a
 * Hermitian matrix (App. D.1): the diagonal entries X_ii and, for i < j,
 * sqrt(2) Re X_ij and sqrt(2) Im X_ij, so that <svec X, svec Y> = tr[X^H Y].
 * The paper leaves the order open; here it is row-major over the upper
 * triangle with Re/Im interleaved:
 *     row i starts at offset i*(2n - i) and holds
 *     X_ii, sqrt2 Re X_i,i+1, sqrt2 Im X_i,i+1, ..., sqrt2 Im X_i,n-1.
 * A block of order n has exactly n*n doubles.  Batched blocks are
 * concatenated in the order given; block b starts at sum_{c<b} n_c^2.
 *
 * Memory: every double* below is HIP device memory owned by the caller
 * (8-byte aligned; 16-byte aligned recommended), unless marked "host".
 * The library never allocates in a call: the caller passes a device
 * workspace of at least psd_workspace_size() bytes (256-byte aligned).
 *
 * Asynchrony: all device work is enqueued on `stream` (0 = the null stream).
 * Errors found on the host (bad sizes, null pointers, misalignment, too small
 * a workspace, partially overlapping x/y) are returned synchronously and
 * nothing is enqueued.  Conditions found on the device (non-finite input,
 * non-convergence) are written to `info` asynchronously; synchronise the
 * stream before reading it.  No call prints, throws or allocates, and none
 * synchronises the stream except a mixed-mode psd_project while the FP64
 * fallback is enabled (psd_set_mixed_fallback), psd_project_warm (it reads
 * whether its refinement was accepted) and the SCS solver (it reads its
 * residuals back).  Calls on different streams
 * with different workspaces may run concurrently.
 *
 * Failure policy: a block whose input holds a NaN or an infinity gets
 * status PSD_ENONFINITE and an all-NaN output; a tridiagonal or secular
 * iteration that hits its cap gets PSD_ENOCONV (the output is the last
 * iterate's).
 */
#ifndef PSDPROJ_H
#define PSDPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSD_OK = 0,
    PSD_EINVAL = 1,       /* invalid argument (size, pointer, alignment, mode, aliasing) */
    PSD_EWORKSPACE = 2,   /* workspace too small */
    PSD_ENOMEM = 3,       /* (reserved: the library does not allocate) */
    PSD_ENONFINITE = 4,   /* device: the input held a NaN or an infinity */
    PSD_ENOCONV = 5,      /* device: an iteration did not converge */
    PSD_EDEVICE = 6,      /* a HIP runtime call failed (launch, no device) */
    PSD_EUNSUPPORTED = 7  /* valid request the library does not serve */
} psd_status;

typedef enum {
    PSD_FP64_EIG = 0,     /* FP64 eigendecomposition path (exact up to rounding) */
    PSD_MIXED_BF16 = 1,   /* Newton-Schulz sign iteration, BF16 MFMA + FP64 correction */
    PSD_MIXED_FP32 = 2,   /* Newton-Schulz sign iteration, FP32 MFMA + FP64 correction */
    PSD_MIXED_BF16X3 = 3  /* Newton-Schulz sign iteration on split BF16 operands: each
                             FP32 value as hi + lo (two BF16 terms), each real product as
                             hi*hi + hi*lo + lo*hi (three BF16 MFMAs, about 16 bits) +
                             FP64 correction.  In every mixed mode, blocks of order
                             <= 64 take the exact LDS kernel */
} psd_mode;

/* Per-block result record, written by the device (device or pinned host
 * memory; read it only after synchronising the stream). */
typedef struct {
    int32_t status;       /* psd_status of this block */
    int32_t n_pos;        /* number of eigenvalues > 0 */
    int32_t n_neg;        /* number of eigenvalues <= 0 */
    int32_t iters;        /* NS iterations (mixed), refinement steps (psd_project_warm) or 0 */
    int32_t fallback;     /* 1 if a mixed request fell back to the FP64 path, or a warm
                             request to the cold FP64 path */
    int32_t reserved;
    double est_rel_err;   /* mixed: first-order estimate of ||y - Pi(X)||_F / ||Pi(X)||_F for
                             the sign estimate S: sqrt(||[X, S]||_F^2 + ||X||_F^2 -
                             ||X S||_F^2) / (4 ||y||_F) -- the eigenvector part (the
                             commutator vanishes for the exact sign) and the eigenvalue
                             part (S^2 = I for it); relative to ||X||_F when y = 0;
                             psd_project_warm: the square of the last refinement
                             step's largest rotation |E_ij|; FP64: 0 */
    double scale;         /* mixed: spectral scale alpha (~1.1 ||X||_2); FP64: 0 */
} psd_info;

/* Workspace bytes needed to serve `nblocks` blocks of orders n[0..nblocks)
 * (host array) in `mode` by psd_project / psd_project_batched /
 * psd_project_vjp.  flags: bit 0 = also return the eigen-pair for a later VJP
 * (PSD_FLAG_SAVE).  Returns PSD_EINVAL for n < 1, nblocks < 1 or a bad mode. */
#define PSD_FLAG_SAVE 1
/* bit 1: workspace of psd_project_warm (one block, PSD_FP64_EIG only) */
#define PSD_FLAG_WARM 2
psd_status psd_workspace_size(int32_t nblocks, const int32_t *n, psd_mode mode,
                              int32_t flags, size_t *bytes);

/* Bytes of the `saved` record of one block of order n: lambda (n doubles,
 * ascending when psd_project wrote it; psd_project_warm keeps the column
 * order of its input record) followed by V (n x n complex, column-major,
 * interleaved re/im) with V[:,k] the unit eigenvector of lambda[k] -- of the
 * conjugate matrix mat(x)^T, in the svec convention above (Pi commutes with
 * conjugation). */
size_t psd_saved_size(int32_t n);

/* y <- svec(Pi(mat(x))) for one block of order n >= 1.
 * x, y: n*n doubles; y == x (in place) is allowed, partial overlap is not.
 * info: nullable (device or pinned).  saved: nullable; if given (size
 * psd_saved_size(n)), receives lambda and V for psd_project_vjp.
 * mode PSD_FP64_EIG: relative Frobenius error ~ n * 2^-53.  */
psd_status psd_project(int32_t n, const double *x, double *y, psd_mode mode,
                       void *ws, size_t ws_bytes, void *stream, psd_info *info,
                       double *saved);

/* y <- svec(Pi(mat(x))) in FP64 for one block of order n >= 1, starting from
 * the eigen-pair of a nearby matrix: saved_prev (psd_saved_size(n) bytes,
 * from psd_project with `saved` or from an earlier call of this function).
 * The successive inputs of the splitting method are such a sequence (warm
 * starting, App. D.2 of the paper; the warm-started refinement, Sec. IV).
 * The eigenvectors are refined by matrix products (the iteration of Ogita
 * and Aishima, 2018: X <- X + X E from G = X^H X and S = X^H A X, at most 5
 * steps, stopping once the largest rotation |E_ij| of a step is <= 1e-7 and
 * giving up when a step is above 1/2 or above half the previous one), and
 * Pi = X diag(max(lambda, 0)) X^H.  The refined pair goes to saved_out
 * (may equal saved_prev), ready for the next call or psd_project_vjp.
 * When the last step's largest rotation is above 1e-6 (the pair was not
 * close, the spectrum moved too far) or x is not finite, the block is
 * projected by the cold FP64 path instead (info->fallback = 1), which also
 * writes saved_out.  Either way y is within the FP64 tolerance of Pi(X).
 * The call synchronises `stream` once (the host reads the outcome) and so
 * cannot be captured into a graph (PSD_EUNSUPPORTED).  y == x is allowed;
 * x and y must not overlap saved_prev or saved_out.  Workspace:
 * psd_workspace_size(1, &n, PSD_FP64_EIG, PSD_FLAG_WARM, &bytes). */
psd_status psd_project_warm(int32_t n, const double *x, double *y, const double *saved_prev,
                            double *saved_out, void *ws, size_t ws_bytes, void *stream,
                            psd_info *info);

/* psd_project without a workspace argument, for callers that cannot
 * allocate (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a fixed device array of
 * PSD_NOALLOC_SCRATCH_BYTES inside the library, one copy on each device it
 * runs on, held until the process ends; the call itself allocates nothing.
 * Its address is looked up on the first call made with a device current.
 * Orders whose psd_workspace_size(1, &n, mode, 0) exceeds the array are
 * rejected with PSD_EWORKSPACE before anything is enqueued (n <= 831 in
 * FP64, n <= 768 in BF16-mixed, n <= 704 in FP32- and BF16x3-mixed; n <= 64 needs none).  Calls on one
 * device share the array: calls that overlap in time on one device (other
 * streams, other host threads) race and must be serialised by the caller.
 * Same arguments and results as psd_project, without `saved` and without
 * the mixed modes' FP64 fallback. */
#define PSD_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
psd_status psd_project_noalloc(int32_t n, const double *x, double *y, psd_mode mode,
                               void *stream, psd_info *info);

/* Projects nblocks independent blocks (orders n[0..nblocks), host array)
 * stored back to back in x into y (same layout).  infos: nullable array of
 * nblocks records. */
psd_status psd_project_batched(int32_t nblocks, const int32_t *n, const double *x,
                               double *y, psd_mode mode, void *ws, size_t ws_bytes,
                               void *stream, psd_info *infos);

/* gx <- svec(DPi(X)[mat(gy)]) with X = mat(x): the Daleckii-Krein formula
 *   DPi(X)[G] = V (Gamma o (V^H G V)) V^H,
 *   Gamma_ij = 1 (lambda_i, lambda_j > 0), 0 (both <= 0),
 *              lambda_i / (lambda_i - lambda_j) (lambda_i > 0 >= lambda_j).
 * DPi(X) is self-adjoint in svec coordinates, so this is both the JVP and
 * the vector-Jacobian product.  Give either x (the eigen-pair is recomputed)
 * or saved (from psd_project); if both are non-null, saved is used.
 * gy, gx: n*n doubles; gx may alias gy. */
psd_status psd_project_vjp(int32_t n, const double *x, const double *saved,
                           const double *gy, double *gx, psd_mode mode, void *ws,
                           size_t ws_bytes, void *stream);

/* Plans: every block of one cone (e.g. per instance one W block of order
 * d^4 and eight instrument Choi blocks of order d^2), projected by ONE
 * hipGraph launch.  The graph holds the whole-block LDS kernel for all blocks
 * of order <= 64 and the large blocks as jobs spread over `concurrency`
 * streams (each with its own workspace slot), fork/join by events.  A job is
 * a lockstep group: up to 128 blocks of one order (fewer where their
 * workspace would pass 4 GiB, or the group size the autotuner chose) that
 * share every kernel launch.  The graph is captured on a
 * stream the plan owns the first time a given (x, y, ws, infos) is executed
 * and replayed afterwards.  Creation allocates (streams, events, a device
 * copy of the block table); execution does not, apart from the one-time
 * capture and instantiation of a new graph (a plan keeps the graphs of its
 * last 8 buffer sets; capturing a ninth synchronises `stream` and drops the
 * oldest).  concurrency = 0 takes the value
 * psd_plan_tune last recorded for this arch/mode/size list in the tuning
 * cache (file PSD_TUNE_CACHE, default ./psdproj_tune.jsonl), else 4; the
 * group size recorded there is used as well.  Concurrency is clamped to
 * [1, number of jobs], and raised until no stream of the graph carries more
 * than 20 000 launches (an FP64 job of order n launches about 2.1 n
 * kernels): the tuner skips concurrencies below that, and an execution
 * that would capture a longer chain returns PSD_EUNSUPPORTED.  Mixed modes use the
 * Newton-Schulz settings current at capture time.  A plan is not
 * thread-safe; execute it on one host thread. */
typedef struct psd_plan_s *psd_plan;
psd_status psd_plan_create(int32_t nblocks, const int32_t *n /* host */, psd_mode mode,
                           int32_t concurrency, psd_plan *plan);
/* Workspace for executing with `concurrency` large blocks in flight (0 = the
 * plan's current value). */
psd_status psd_plan_workspace_size(psd_plan plan, int32_t concurrency, size_t *bytes);
/* The plan's current concurrency. */
int32_t psd_plan_concurrency(psd_plan plan);
/* Members of the plan's largest lockstep group (0 without large blocks). */
int32_t psd_plan_group_size(psd_plan plan);
/* Padded order from which the plan's BF16 Newton-Schulz products use
 * 128x128 tiles (2048 by default, as for psd_project and
 * psd_project_batched; 1024 when the autotuner found that form faster for
 * the plan's groups).  The two forms sum in different orders: the results of
 * a plan at 1024 differ from eager calls by FP32 rounding in the
 * low-precision iterations (both within the BF16 form's error bound). */
int32_t psd_plan_ns_tile_threshold(psd_plan plan);
/* y <- the blocks of x projected (layout as psd_project_batched); infos:
 * nullable, one record per block. */
psd_status psd_plan_execute(psd_plan plan, const double *x, double *y, void *ws, size_t ws_bytes,
                            void *stream, psd_info *infos);
/* Autotuner: for the group sizes 32 (or the memory-derived limit), 16 and 8
 * (those that split the blocks differently) and, for each, concurrency 1, 2,
 * 4, ... and the number of jobs (each that fits in ws_bytes) -- and for BF16
 * plans with a block of padded order 1024..2047 also for both tile forms of
 * the Newton-Schulz product (psd_plan_ns_tile_threshold) -- replays the
 * graph once untimed, then `reps` times, each timed on its own, and scores
 * the combination by its fastest replay (two untimed replays of the plan as
 * it stands come first); keeps the fastest combination in the plan, appends
 * it to the tuning cache and returns the concurrency in *best (the group
 * size: psd_plan_group_size).  Synchronises the stream. */
psd_status psd_plan_tune(psd_plan plan, const double *x, double *y, void *ws, size_t ws_bytes,
                         void *stream, int32_t reps, int32_t *best);
psd_status psd_plan_destroy(psd_plan plan);

/* Instrumentation (off by default).  Between psd_timing_start and
 * psd_timing_stop every launch of one kernel family made by this library is
 * bracketed by a pair of HIP events recorded on the launch stream (at most
 * max_launches pairs; later launches are not timed).  psd_timing_stop
 * synchronises those events and returns the summed device time in ms, the
 * number of launches timed and their algorithmic work: bytes of the matrix
 * read for PSD_KF_HEMV (the lower triangle of the trailing matrix, 16 bytes
 * per complex entry), real flops for PSD_KF_GEMM (8 per complex
 * multiply-add), none for PSD_KF_WSTEP.  Not thread-safe; meant for benchmarks and tests.  The
 * events are created by psd_timing_start and destroyed by psd_timing_stop. */
typedef enum {
    PSD_KF_HEMV = 1,   /* per-column Hermitian matrix-vector tiles of the tridiagonalisation */
    PSD_KF_GEMM = 2,   /* FP64 MFMA GEMMs */
    PSD_KF_NS = 3,     /* low-precision Newton-Schulz GEMMs (flops of the lower tiles computed) */
    PSD_KF_WSTEP = 4   /* per-column w / next-column step of the tridiagonalisation (latency bound) */
} psd_kernel_family;
psd_status psd_timing_start(int32_t family, int32_t max_launches);
psd_status psd_timing_stop(double *ms, int32_t *launches, double *work);

/* Newton-Schulz settings of the mixed modes (process-wide; not
 * thread-safe): `iters` low-precision steps of the scaled iteration
 * X <- (a_k/2) X (3I - a_k^2 X^2) (a_0 = 1, then a_k = min(1.5,
 * sqrt(3/(1+l+l^2))) for the current lower bound l of the scaled spectrum,
 * starting from 1e-6); 0 (the default) = automatic, as many steps as bring
 * l within 1e-7 of 1 (21): eigenvalues down to about 1e-6 ||X||_2 resolved.
 * `corrections`: FP64 correction steps S <- S (3I - S^2)/2 (0..8), or -1
 * (the default) for automatic: 1 in BF16-mixed, 0 in FP32- and
 * BF16x3-mixed.  A step squares S's eigenvalue error; the error of the
 * result is set by the subspace error of the low-precision iterations,
 * which no step reduces, so it only tightens the estimate's eigenvalue part
 * where that error is large (BF16).
 * Returns PSD_EINVAL outside 0..200 / -1..8. */
psd_status psd_set_ns_iterations(int32_t iters, int32_t corrections);

/* Affine step of the SCS iteration for the bipartite process-matrix SDP
 * (App. D.1-D.2), the step on either side of the cone projection.  With the
 * constraint map over the allowed traceless multi-indices
 * mu = (alpha_1, beta_1, alpha_2, beta_2) (App. "Sparse basis for the
 * process-matrix subspace": every party with beta >= 1 needs a party with
 * alpha >= 1, beta = 0; the all-identity index excluded),
 *     A x = -sum_mu x_mu F_mu,   (A^T Z)_mu = -tr[F_mu Z]   (eq. constraint_map_def),
 *     F_mu = s_a1 (x) s_b1 (x) s_a2 (x) s_b2 on A_i (x) A_o (x) B_i (x) B_o,
 * s_alpha the normalised generalised Gell-Mann matrices of local dimension d
 * in the paper's order (eq. gellmann_basis: identity/sqrt d, the d-1
 * diagonal ones, the symmetric then the antisymmetric off-diagonal ones,
 * pairs j < k lexicographic), and A^T A = I, the affine projection is
 *     z_x = (a_x - A^T a_y) / 2,   z_y = a_y + A z_x   (App. D.2).
 * x, a_x, z_x: real vectors of nx = |I| = d^8 - (1 + d^2(d^2 - 1))^2
 * entries, in lexicographic order of mu; y, a_y, z_y: svec of d^4 x d^4
 * Hermitian matrices (ny = d^8 doubles).  2 <= d <= 8.  The device workspace
 * (psd_affine_workspace_size: two d^8-entry complex tensors, 256-byte aligned)
 * is caller-owned; nothing is allocated.  zx may alias ax and zy may alias
 * ay; other overlaps return PSD_EINVAL.  Errors are host-side only (the maps
 * are linear: no device status). */
psd_status psd_affine_dims(int32_t d, int64_t *nx, int64_t *ny);
psd_status psd_affine_workspace_size(int32_t d, size_t *bytes);
/* y <- svec(A x). */
psd_status psd_constraint_apply(int32_t d, const double *x, double *y, void *ws, size_t ws_bytes,
                                void *stream);
/* x <- A^T mat(y). */
psd_status psd_constraint_adjoint(int32_t d, const double *y, double *x, void *ws, size_t ws_bytes,
                                  void *stream);
/* (zx, zy) <- ((ax - A^T mat(ay)) / 2, ay + svec(A zx)). */
psd_status psd_affine_step(int32_t d, const double *ax, const double *ay, double *zx, double *zy,
                           void *ws, size_t ws_bytes, void *stream);

/* ---- SCS solver for the bipartite process-matrix SDP (App. D) ----------
 *
 * Maximises tr[W G] over process matrices W = gamma 1 + sum_mu x_mu F_mu >= 0
 * (eq. sparse_process_sdp; gamma = 1/d^2) in the SCS form
 *     min c^T x  s.t.  A x + s = b,  s in H_+^{d^4}
 * (eq. constraint_map_def: A as in psd_constraint_apply, b = gamma 1,
 * c = A^T G), through the homogeneous self-dual embedding and the iteration
 * of eq. final_iterates: u~ = (1 + Q)^-1 (u + v), u = Pi_C(u~_r - v),
 * v = v - u~_r + u, with u~_r = alpha u~ + (1 - alpha) u (over-relaxation;
 * alpha = 1 is the printed iteration), (1 + Q)^-1 by Sherman-Morrison over
 * the closed-form M^-1 of psd_affine_step, and Pi_C by psd_project on the
 * Hermitian block.  Start: u = v = (0, 0, 1), or with warm_start
 * u = (x, sigma y, 1), v = (0, s, 0) from the caller's x, y, s.  Partial
 * normalisation (App. D.2): c is scaled inside the iteration by
 * sigma = ||b||_2 / ||c||_2.  Termination (App. D.1, "Convergence
 * criteria"): with x = u_x/tau, s = v_s/tau, y = u_y/(sigma tau),
 * p = A x + s - b, r = A^T y + c, g = c^T x + b^T y and
 * ||p||_inf <= eps (1 + max(||A x||_inf, ||s||_inf, ||b||_inf)),
 * ||r||_inf <= eps (1 + max(||A^T y||_inf, ||c||_inf)),
 * |g| <= eps (1 + max(|c^T x|, |b^T y|)), tested every check_every
 * iterations and after the last one; eps = 0 runs exactly max_iters.
 * The first mixed_iters cone projections use mixed_mode, the rest FP64 (the
 * paper's low-to-high precision switch after a fixed iteration count); with
 * mixed_switch > 0 the switch also comes as soon as a residual check finds
 * the iterate within mixed_switch times the tolerance (so mixed_iters =
 * max_iters with mixed_switch = 10 switches on the residuals alone).
 * anderson = m > 0: type-I Anderson acceleration (App. D.2 keeps SCS's) of
 * the map q -> G(q) on the cone step's input q = u~_r - v (which fixes
 * u = Pi_C(q) and v = u - q): with the last m differences S of the inputs
 * and Y of the residuals f = q - G(q), gamma solves
 * (S^T Y + 1e-8 ||S||_F ||Y||_F 1) gamma = S^T f and the next input is
 * G(q) - (S - Y) gamma; an input whose residual exceeds twice the previous
 * one is replaced by the plain G(q) it displaced and the memory cleared; a
 * singular system or |gamma| > 1e10 skips the step.  With m > 0 the stream
 * is also synchronised once per iteration. */
typedef struct {
    int32_t d;             /* local dimension, 2..8 (W has order d^4) */
    int32_t max_iters;     /* >= 1 */
    int32_t check_every;   /* >= 1 */
    int32_t mixed_iters;   /* >= 0 */
    int32_t mixed_mode;    /* a mixed psd_mode when mixed_iters > 0 */
    int32_t normalize;     /* 0 or 1 */
    int32_t warm_start;    /* 0 or 1 */
    int32_t anderson;      /* Anderson memory m, 0 (off) .. 16 */
    double eps;            /* eps_abs = eps_rel >= 0 */
    double alpha;          /* over-relaxation, 0 < alpha < 2 */
    double mixed_switch;   /* >= 0; > 0: leave mixed_mode for FP64 for good once a
                              residual check finds every termination ratio
                              (||p||/bound_p, ||r||/bound_r, |g|/bound_g) below it */
    int32_t warm_proj;     /* 0 or 1 (one instance only: psd_scs_solve, or nbatch = 1):
                              FP64 cone steps by psd_project_warm from the eigen-pair
                              the previous FP64 step left (successive cone inputs are
                              close); after an attempt falls back to the cold path the
                              next 1, 2, 4 .. 16 steps (doubling while attempts keep
                              failing) are cold, the last of them saving its pair */
} psd_scs_settings;

/* Result record (host memory, complete when psd_scs_solve returns). */
typedef struct {
    int32_t status;        /* PSD_OK converged; PSD_ENOCONV max_iters reached
                              (outputs: the last iterate); PSD_ENONFINITE a
                              residual or the data was not finite */
    int32_t iters;         /* iterations run */
    int32_t proj_status;   /* first non-OK status of a cone projection, else 0 */
    int32_t aa_accepted;   /* Anderson steps taken */
    int32_t aa_rejected;   /* Anderson steps undone by the safeguard */
    int32_t switch_iter;   /* iteration after which mixed_switch moved to FP64, else 0 */
    double pobj;           /* tr[W G] at x: gamma tr G - c^T x (last check) */
    double dobj;           /* dual bound gamma tr G + b^T y (last check) */
    double res_pri, res_dual, gap;   /* ||p||_inf, ||r||_inf, |g| (last check) */
    double tau, kappa;     /* embedding scalars of the last iterate */
    double sigma;          /* normalisation scale */
    double post_lambda;    /* post-processing mixing weight (0: W was PSD) */
    double post_lambda_min;/* lambda_min of W = b - A x before mixing */
    int32_t warm_refined;  /* warm_proj: cone steps the refinement served */
    int32_t warm_fallbacks;/* warm_proj: refinement attempts that fell back to the cold
                              path (the other FP64 cone steps were cold) */
} psd_scs_info;

/* Device workspace bytes of psd_scs_solve for these settings (EINVAL for
 * settings out of range). */
psd_status psd_scs_workspace_size(const psd_scs_settings *s, size_t *bytes);

/* Solve for the objective g (svec of G, d^8 doubles).  x (nx doubles), y and
 * s (d^8 doubles each): the unscaled solution x = u_x/tau, y = u_y/(sigma
 * tau), s = v_s/tau (with tau = 0: u_x, u_y, v_s); with warm_start they
 * also carry the start.  w (nullable, d^8 doubles): the process matrix
 * W = b - A x post-processed as in App. "Sparse SDP formulation for process
 * matrices and post-processing": W' = (1 - lam) W + lam gamma 1 with the
 * smallest lam in [0, 1] that makes W' PSD (lambda_min from an FP64
 * eigendecomposition).  g, x, y, s, w must not overlap.  info: host.
 * Synchronises `stream` at setup and at every residual check (the host
 * decides termination); allocates nothing.  Host-side errors return
 * EINVAL / EWORKSPACE / EDEVICE with info unspecified; otherwise PSD_OK
 * with the outcome in info->status. */
psd_status psd_scs_solve(const psd_scs_settings *s, const double *g, double *x, double *y, double *s_out,
                         double *w, void *ws, size_t ws_bytes, void *stream, psd_scs_info *info);

/* A batch of 1 <= nbatch <= PSD_SCS_MAX_BATCH independent solves with the
 * same settings (many
 * objectives, e.g. the restarts of the paper's exploration stage, §IV):
 * g, y, s_out, w hold nbatch d^8-vectors back to back, x nbatch n_x-vectors,
 * infos nbatch records.  The instances advance in lockstep and their cone
 * steps are one psd_project_batched call (same-order blocks in lockstep
 * groups, each block's result bitwise that of a single call), so each
 * instance's iterates and results are bitwise those of psd_scs_solve on its
 * own.  An instance that stops (converged, non-finite) has its outputs
 * written and is not advanced further; its block is still projected with
 * the others.  With mixed_switch > 0 the batch leaves the mixed mode
 * when every running instance is within the factor.  Workspace from
 * psd_scs_workspace_size_batched (it grows with nbatch). */
#define PSD_SCS_MAX_BATCH 65535 /* one grid dimension of the per-step launches */
psd_status psd_scs_workspace_size_batched(const psd_scs_settings *s, int32_t nbatch, size_t *bytes);
psd_status psd_scs_solve_batched(const psd_scs_settings *s, int32_t nbatch, const double *g, double *x, double *y,
                                 double *s_out, double *w, void *ws, size_t ws_bytes, void *stream,
                                 psd_scs_info *infos);

/* FP64 fallback of the mixed modes (process-wide; not thread-safe):
 * with max_rel_err > 0, psd_project in a mixed mode writes the mixed run's
 * record to its workspace, synchronises the stream and, if that record
 * reports PSD_ENOCONV or an est_rel_err above max_rel_err (or not a number),
 * projects the block again by the FP64 path; the caller's info then holds
 * the FP64 record with fallback = 1.  A non-finite input is not retried.
 * Applies to single blocks outside graph capture (not to psd_project_batched
 * or plans).  0 (the default) disables it.  Returns PSD_EINVAL for a
 * negative or NaN bound. */
psd_status psd_set_mixed_fallback(double max_rel_err);

/* Static description of a status code. */
const char *psd_status_string(psd_status status);

/* Library version string. */
const char *psd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSDPROJ_H */

/*
 * fmmnufft.h -- C ABI of the MI355X (gfx950) FMM-based NUFFT / INUFFT.
 *
 * Method: N. A. Gumerov and R. Duraiswami, "Fast Multipole Method based
 * filtering of non-uniformly sampled data" (arXiv:1611.09379).
 *
 * Problems (Section 2).  A 2 pi-periodic band-limited function
 *     f(x) = sum_{n=0}^{N-1} c_n e^{inx}                       (Eq. p1)
 * is sampled at the N equispaced points x_k = 2 pi k / N, f_k = f(x_k).
 *   (i)  forward:  given f_k, find g_j = f(y_j) at M arbitrary points y_j;
 *        g = K f with K_jk = (1/N) sum_n e^{-i n x_k} e^{i n y_j}  (Eq. p2)
 *        = F_j G(y_j - x_k), F_j = (e^{iNy_j} - 1)/N,
 *        G(t) = 1/(e^{it} - 1) = -(1 + i cot(t/2))/2           (Eq. p4-p5)
 *  (ii)  inverse (M = N): given g_j at the y_j, find f_k;
 *        f = L g, L_kj = C_k G(x_k - y_j) D_j                   (Eq. p6)
 *        with C_k, D_j the products of sines of Eq. (p8).
 * Both reduce to the matrix-vector product with the kernel cot(t/2), which
 * the library evaluates with the multilevel FMM of Section 2.1-2.4 on the
 * circular binary tree; C_k and D_j come from the same FMM applied to the
 * kernel log|2 sin(t/2)| (the logarithms of the products of Eq. p8).
 *
 * Conventions shared by every entry point:
 *   - Every array argument is DEVICE memory (hipMalloc / a PyTorch CUDA
 *     tensor) owned by the caller; the library never frees it.  y is always
 *     binary64 radians.  f and g are interleaved complex (re, im): binary64
 *     pairs for FN_C128, binary32 pairs for FN_C64.
 *   - y may hold any finite value with |y| <= FN_Y_MAX; it is reduced modulo
 *     2 pi exactly (in grid units N y / 2 pi, formed in double-double).
 *   - Outputs are in the order of the inputs (g_j in the order of y_j, f_k
 *     for k = 0..N-1).
 *   - eps is the target relative l2 error ||out - exact|| / ||exact||.  It
 *     sets the truncation numbers p, q and the tree depth (Eq. 18, 18.2, 25).
 *     eps = FN_EPS_MACHINE (0) asks for the precision path's own floor
 *     eps_th(N) (Section 3.1, the machine-precision setting of Section
 *     3.2), which the plan reports in fn_plan_info.eps.  Binary64: the
 *     measured maximum error for f = 1, 1.4e-16 log2 sqrt(N M) (at least
 *     5.6e-16; the relative l2 error of random data stays near 5e-16),
 *     reached with p_th = 32 expansion terms and q_th = 22 Bernoulli terms
 *     at every size measured (2^6 ... 2^20), the depth being that of
 *     eps = eps_th(N).  FN_C64: the parameters of eps = 2e-7.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; a call returns when the work is enqueued,
 *     except where noted ("synchronises").
 *   - Every function returns an fn_status.  Nothing throws: a C++
 *     exception inside the library (a failed host allocation) becomes
 *     FN_ENOMEM (FN_EHIP for any other), after the call has released what
 *     it allocated.  On a non-OK status nufft_last_error() returns a
 *     message (thread-local, valid until the next call on the same
 *     thread).  Scalar argument errors are reported before any GPU work is
 *     enqueued.
 *   - Host threads: calls from several threads may overlap (the library's
 *     shared state -- workspace pool, operator tables, autotune records --
 *     is locked).  A plan or batch holds one workspace: its executes must
 *     not overlap in time, whether from two threads or on two streams that
 *     do not wait for each other.
 */
#ifndef FMMNUFFT_H
#define FMMNUFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* eps value that requests the precision floor eps_th(N) of the path. */
#define FN_EPS_MACHINE 0.0

typedef enum {
    FN_OK = 0,
    FN_EINVAL = 1,    /* bad scalar argument, NULL pointer, non-finite or
                         out-of-range y                                    */
    FN_ENOMEM = 2,    /* device workspace allocation failed                */
    FN_EHIP = 3,      /* a HIP runtime call failed (message has details)   */
    FN_ESINGULAR = 4, /* inverse: two y_j coincide on the circle            */
    FN_ERANGE = 5,    /* inverse: |log|C_k|| or |log|D_j|| (rescaled as
                         for nufft_plan_coeffs) exceeds 700 (FN_C128) or 60
                         (FN_C64, whose binary32 weights D_j g_j must stay
                         in range), or a leaf holds over 16 times the mean
                         number of points (the point set is too
                         ill-conditioned)                                  */
    FN_EPREC = 6      /* eps below what the precision path can deliver     */
} fn_status;

typedef enum {
    FN_C128 = 0, /* binary64 throughout                                    */
    FN_C64 = 1   /* mixed: binary32 data, expansions and translations;
                    binary64 phase reduction, near-field differences and
                    the log-sums of the inverse                           */
} fn_dtype;

/* Largest accepted |y| (radians). */
#define FN_Y_MAX 1024.0

typedef struct fn_plan fn_plan;

/* Parameters a plan uses (for reporting and tests). */
typedef struct {
    int64_t N, M;
    int32_t kind;  /* 0 forward, 1 inverse, 2 adjoint                     */
    int32_t dtype; /* fn_dtype                                            */
    int32_t p;     /* truncation number of the 1/t MLFMM from Eq. (18.2)
                      (or as given)                                      */
    int32_t q;     /* Bernoulli terms of the regular part (Eq. 10, 11)    */
    int32_t lmax;  /* finest tree level (2^lmax leaves)                   */
    int32_t nterms;/* terms of the local expansions and translations: p,
                      or a smaller value calibrated for the relative l2
                      target when p was not given, rounded up to 16       */
    double eps;
    int32_t mterms;     /* terms of the multipole expansions (>= nterms and
                           >= 2q, rounded up to 16)                        */
    int32_t log_nterms; /* inverse plans: local and multipole terms of the */
    int32_t log_mterms; /* log-sum FMM (0 for other plans)                */
} fn_plan_info;

/* Forward interpolation (problem i): g_j = sum_k K_jk f_k, Eq. (p2).
 * y: M doubles; f: N complex; g: M complex (written).  N >= 1, M >= 1,
 * N, M < 2^31.  One-shot: setup and evaluation are enqueued back to back
 * and the call synchronises the stream once, at the end, where it also
 * reports the data-dependent errors of the setup (on such an error g holds
 * no result). */
int nufft_fwd(int64_t N, int64_t M, const double *y, const void *f, void *g,
              double eps, int dtype, void *stream);

/* Inverse interpolation (problem ii, M = N): f = L g, Eq. (p6)/(p8).
 * y: N doubles, pairwise distinct modulo 2 pi; g: N complex; f: N complex
 * (written).  One-shot like nufft_fwd: one synchronisation, at the end. */
int inufft(int64_t N, const double *y, const void *g, void *f, double eps,
           int dtype, void *stream);

/* Adjoint of the forward transform: f = K^H g, i.e.
 *     f_k = sum_j conj(K_jk) g_j,  k = 0..N-1,  K of Eq. (p2).
 * Since conj(G(t)) = G(-t), conj(K_jk) = conj(F_j) G(x_k - y_j): the
 * cot-kernel FMM with the roles of the grid and the points swapped, the
 * same evaluation the inverse uses (Section 2), with weights conj(F_j) g_j
 * and without its C_k factor.  It is the type-1 (nonuniform to uniform)
 * direction; with the forward it gives the normal equations of a
 * least-squares fit for M != N.  y: M doubles (any points; coincident
 * points are allowed); g: M complex; f: N complex (written).  A point on a
 * grid point x_m (theta_j = 0) contributes g_j to f_m alone.  One-shot like
 * nufft_fwd: one synchronisation, at the end.  The summation order inside
 * a leaf follows the sort's placement, which can differ from run to run;
 * results then differ in the last bits only. */
int nufft_adj(int64_t N, int64_t M, const double *y, const void *g, void *f,
              double eps, int dtype, void *stream);

/* Spectral transforms (Eq. p1, f(x) = sum_{n=0}^{N-1} c_n e^{inx}), with the
 * uniform DFT by rocFFT beside the FMM:
 *   nufft_spec_fwd: g_j = f(y_j) from the coefficients c (N complex):
 *       f_k = sum_n c_n e^{2 pi i n k / N} (unscaled backward DFT), g = K f;
 *   inufft_spec (M = N): the coefficients c (N complex, written) of the
 *       band-limited interpolant through the values g_j: f = L g, then
 *       c_n = (1/N) sum_k f_k e^{-2 pi i n k / N}.
 * Arguments, precision paths and errors as nufft_fwd / inufft; the DFT runs
 * in the dtype's precision.  One-shot: one synchronisation at the end.  A
 * rocFFT failure returns FN_EHIP.  The rocFFT plans (one per device, N,
 * dtype and direction; up to 64) are created on first use and kept until
 * the process ends: later calls and spectral plans of that size share them,
 * each with its own work buffer. */
int nufft_spec_fwd(int64_t N, int64_t M, const double *y, const void *c, void *g,
                   double eps, int dtype, void *stream);
int inufft_spec(int64_t N, const double *y, const void *g, void *c, double eps,
                int dtype, void *stream);

/* Setup step of Section 3.3 ("setting the data structure"): everything that
 * depends on the points only.  Forward plan: reduction of y to grid units
 * and the sort of the targets into the leaves of the tree.  Inverse plan:
 * the same for the sources y_j, plus C_k and D_j of Eq. (p8) by the
 * log-kernel FMM.  The plan owns its device workspace, allocated here.
 * Synchronises the stream.  y is read during the call only. */
int nufft_plan_fwd(fn_plan **plan, int64_t N, int64_t M, const double *y,
                   double eps, int dtype, void *stream);
int nufft_plan_inv(fn_plan **plan, int64_t N, const double *y, double eps,
                   int dtype, void *stream);
/* Adjoint plan (the sort of the M points y into the leaves). */
int nufft_plan_adj(fn_plan **plan, int64_t N, int64_t M, const double *y,
                   double eps, int dtype, void *stream);
/* Spectral plans: a forward or inverse plan plus its rocFFT plan and an
 * N-value workspace; nufft_execute then maps c -> g (forward) or g -> c
 * (inverse), reusing the setup for any number of inputs on the same points
 * (Section 3.3).  nufft_execute_phase: the forward's DFT runs at the start
 * of phase 0, the inverse's at the end of phase 2. */
int nufft_plan_spec_fwd(fn_plan **plan, int64_t N, int64_t M, const double *y,
                        double eps, int dtype, void *stream);
int nufft_plan_spec_inv(fn_plan **plan, int64_t N, const double *y, double eps,
                        int dtype, void *stream);

/* Evaluation step of Section 3.3: out = K in (forward plan), out = L in
 * (inverse plan) or out = K^H in (adjoint plan).  in/out sizes: forward
 * N -> M, inverse N -> N, adjoint M -> N, complex of the plan's dtype.
 * Enqueues kernels only: no allocation, no synchronisation. */
int nufft_execute(fn_plan *plan, const void *in, void *out, void *stream);

/* One part of nufft_execute: phase 0 is the upward pass (P2M at the leaves,
 * M2M to level 2), phase 1 the downward translations (the M2L of every box
 * with the level-2 regular part, then L2L down to the leaf locals; two
 * kernels), phase 2 the evaluation at the targets (L2P, near field,
 * epilogue; one kernel).  nufft_execute is
 * phases 0, 1, 2 in order on one stream; calling them separately lets a
 * caller bracket each with events.  Each phase reads the plan workspace the
 * previous one wrote, so the three must be enqueued in order, with the same
 * input, and without another execute of the same plan between them. */
int nufft_execute_phase(fn_plan *plan, const void *in, void *out, int phase,
                        void *stream);

/* Releases the plan and its workspace (NULL is accepted): the workspace
 * goes back to the library's cache of device blocks (see
 * nufft_release_cache).  Synchronises the stream of the plan's last call
 * (creation or execute); work of the plan still queued on another stream
 * must have completed before this call. */
int nufft_destroy(fn_plan *plan);

/* Inverse plans: the coefficients of Eq. (p8) the plan computed with the
 * log-kernel FMM, rescaled as Chat_k = 2^N C_k (k = 0..N-1; 0 where a y_j
 * falls on x_k) and Dhat_j = 2^-N D_j (in the order of y), binary64 on both
 * precision paths.  chat: N doubles, dhat: N complex binary64 pairs, device
 * memory owned by the caller.  Enqueues the copies on stream; FN_EINVAL
 * for a forward plan. */
int nufft_plan_coeffs(const fn_plan *plan, double *chat, void *dhat, void *stream);

/* Reports the parameters of a plan. */
int nufft_plan_get_info(const fn_plan *plan, fn_plan_info *info);

/* Measurement of the setup (for benchmarks; not needed otherwise).  With
 * timing on (on != 0; it is off at load), every plan created afterwards
 * records HIP events on its stream around the sort of its points, and an
 * inverse plan also around the three passes of its log-sum FMM (Eq. p8):
 * the upward pass, the downward translations (with the level-2 regular
 * part), and the evaluation (which also forms Chat, Dhat).  The switch is
 * process-wide.  Always FN_OK. */
int nufft_set_timing(int on);

/* ms[0..3]: durations (milliseconds) of those three passes (ms[0..2]) and
 * of the sort (ms[3]) for this plan, read when its setup synchronised; -1
 * when not recorded (timing off, or no log-sum FMM in a forward or adjoint
 * plan).  *log_terms (if log_terms is not NULL): the expansion length of
 * the log-sum FMM (0 without one).  FN_EINVAL for a NULL plan or ms. */
int nufft_plan_get_timings(const fn_plan *plan, float *ms, int32_t *log_terms);

/* The paper's parameters for (N, M, eps, dtype): the truncation numbers of
 * Eq. (18.2) and the depth of Eq. (25) with l_max = round(log2 sqrt(N M)) - 5
 * (Section 3.2).  Plans default to a depth measured on MI355X instead, one
 * level shallower or deeper depending on the size and the transform (their
 * p follows Eq. (18.2) for that depth); nufft_plan_get_info reports what a
 * plan uses.  Host only; no GPU work.  Any output pointer may be NULL. */
int nufft_select_params(int64_t N, int64_t M, double eps, int dtype,
                        int32_t *p, int32_t *q, int32_t *lmax);

/* Like nufft_plan_fwd / nufft_plan_inv with p, q and lmax given explicitly
 * (values <= 0 mean "the plan's default").  For tuning and tests.  Explicit
 * values are used as given: eps then sets only what is not given, and a p
 * or q below what eps needs gives a result that need not meet it.  Any
 * depth keeps the rounding of the FN_C64 path within its 1e-6 target: its
 * binary32 moment and near-field sums run in blocks of at most 64 and 256
 * terms whose partials are added in binary64, however many sources a leaf
 * holds. */
int nufft_plan_fwd_ex(fn_plan **plan, int64_t N, int64_t M, const double *y,
                      double eps, int dtype, int32_t p, int32_t q,
                      int32_t lmax, void *stream);
int nufft_plan_inv_ex(fn_plan **plan, int64_t N, const double *y, double eps,
                      int dtype, int32_t p, int32_t q, int32_t lmax,
                      void *stream);
int nufft_plan_adj_ex(fn_plan **plan, int64_t N, int64_t M, const double *y,
                      double eps, int dtype, int32_t p, int32_t q, int32_t lmax,
                      void *stream);

/* ---- Batches of independent forward transforms (problem i) ----------
 *
 * count transforms of sizes N[t], M[t] (host arrays), with points y[t],
 * inputs f[t] and outputs g[t] (host arrays of DEVICE pointers, each array
 * laid out as for nufft_fwd).  All share eps and dtype.  Every pass of the
 * method (the sort of the targets, the upward bands, the regular part, the
 * downward pass with the evaluation) runs as one launch over the whole
 * batch, each workgroup working for one transform; transforms too large for
 * the shared sort (over 2^15 leaves) run with their own launches.  Errors
 * name the first transform at fault (nufft_last_error). */
typedef struct fn_batch fn_batch;

/* One-shot batch: setup, evaluation and one synchronisation at the end
 * (as nufft_fwd).  count >= 1. */
int nufft_fwd_batched(int32_t count, const int64_t *N, const int64_t *M,
                      const double *const *y, const void *const *f, void *const *g,
                      double eps, int dtype, void *stream);

/* Setup of a batch (the sorts), kept for repeated evaluations with new
 * f[t], g[t] on the same points.  Also captures the shared evaluation
 * launches in a HIP graph and allocates what its replays need (a stream,
 * events, a pinned table of the f[t], g[t] pointers).  Synchronises the
 * stream. */
int nufft_plan_fwd_batched(fn_batch **batch, int32_t count, const int64_t *N,
                           const int64_t *M, const double *const *y, double eps,
                           int dtype, void *stream);

/* Evaluation of a batch plan: g[t] = K_t f[t] for every t.  The captured
 * graph is replayed on the batch's own stream, ordered after the work
 * already enqueued on `stream` and before any work enqueued on it
 * afterwards.  No allocation and no stream synchronisation; the host waits
 * only until the previous call's copy of the pointer table has run, before
 * it rewrites that table.  Calls on one batch must not run concurrently. */
int nufft_execute_batched(fn_batch *batch, const void *const *f, void *const *g,
                          void *stream);

/* Releases a batch plan (NULL accepted).  Synchronises its streams. */
int nufft_destroy_batched(fn_batch *batch);

/* ---- Autotuner --------------------------------------------------------
 *
 * Measures transforms of kind (0 forward, 1 inverse, 2 adjoint; M is
 * ignored for the inverse) and sizes N, M at accuracy eps on a synthetic
 * problem of that size (uniform points, or a jittered grid for the
 * inverse), generated on
 * the device: first the shortest local expansion (16, 32 or 48 terms) whose
 * result stays within eps/4 of the 64-term result, then the fastest tree
 * depth among round(log2 sqrt(N M)) - 4 .. - 7 for one-shot calls (small
 * forward sizes timed as a batch of copies; the default depth is kept
 * unless another is faster by over 5%).  Plans
 * (and batches) created afterwards in this process for the same kind,
 * dtype, size class round(log2 sqrt(N M)) and accuracy class
 * floor(-log10 eps) use the recorded values unless given explicitly; on
 * FN_C64 the depth is then raised where needed to keep at most 128 sources
 * per leaf (N and M may be skewed within a size class), and the candidate
 * depths tried here respect the same bound.
 * lmax, nterms (may be NULL) receive the choice (nterms 0: the default
 * length was kept).  Synchronises the stream; allocates and frees device
 * memory. */
int nufft_autotune(int kind, int64_t N, int64_t M, double eps, int dtype, int32_t *lmax,
                   int32_t *nterms, void *stream);

/* Forgets every recorded choice of nufft_autotune. */
int nufft_autotune_clear(void);

/* Writes every recorded choice of nufft_autotune to a text file (a header
 * line, then one line per record: kind, dtype, size class, accuracy class,
 * lmax, nterms), so that a later process can start from them.  Host only.
 * FN_EINVAL for a NULL path or a file that cannot be written. */
int nufft_autotune_save(const char *path);

/* Adds the records of a file written by nufft_autotune_save (a record of
 * the same kind, dtype, size and accuracy class is replaced).  Host only.
 * FN_EINVAL for a NULL path, a file that cannot be read, or one that is not
 * such a file (wrong header, a malformed line or a value out of range):
 * then no record is added. */
int nufft_autotune_load(const char *path);

/* ---- Least squares ----------------------------------------------------
 *
 * The square inverse (inufft) needs M = N and a point set for which the
 * products of Eq. (p8) stay in range; the paper notes that the inverse's
 * error depends on the distribution of the points (Section 3).  For any M
 * (oversampled sets M > N, clustered or gapped points), nufft_lsq returns
 *     f = argmin ||K f - g||_2,   K of Eq. (p2) (M x N),
 * by conjugate gradients on the normal equations K^H K f = K^H g (CGNR),
 * starting from f = 0.  Each iteration runs one forward and one adjoint
 * transform at accuracy eps and reads two squared norms back (the stream is
 * synchronised every iteration).  It stops when ||K^H (g - K f)|| <= tol
 * ||K^H g|| or after maxiter iterations (an ill-conditioned K converges
 * slowly; the iterate is still the CG approximation).  y: M doubles; g: M
 * complex; f: N complex (written).  iters, resid (may be NULL): the
 * iterations done and the final relative normal-equation residual.
 * Allocates and frees device memory (two plans and four vectors). */
int nufft_lsq(int64_t N, int64_t M, const double *y, const void *g, void *f, double eps,
              double tol, int32_t maxiter, int dtype, int32_t *iters, double *resid,
              void *stream);

/* ---- Allocation-free forward call -------------------------------------
 *
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): nufft_fwd_noalloc computes exactly what
 * nufft_fwd computes (same arguments, same kernels and parameters, one
 * synchronisation at the end) but calls no hipMalloc, hipFree or
 * hipHostMalloc.  Every workspace comes from a static device array of
 * 96 MiB (98 304 KiB) that the library holds on each device it runs on
 * until the process ends; operator tables that no earlier call has built
 * are built into it as well.  That holds the binary64 or mixed forward up
 * to N = M = 2^20; sizes whose workspace does not fit return FN_EINVAL
 * before any kernel is enqueued (nufft_fwd has no such limit).  The array
 * is shared by every call on one device and keeps the last call's
 * contents: calls that overlap in time on one device (two host threads, or
 * two streams that do not wait for each other) race and must not be made.
 * The flags of the setup are read back through pageable host memory. */
int nufft_fwd_noalloc(int64_t N, int64_t M, const double *y, const void *f, void *g,
                      double eps, int dtype, void *stream);

/* ---- Device memory ----------------------------------------------------
 *
 * Plan and batch workspaces come from a cache of device blocks: a released
 * workspace (nufft_destroy, nufft_destroy_batched, the end of a one-shot
 * call) returns its blocks to the cache, which hands a block of the same
 * size to a later plan without hipMalloc.  The cache keeps at most 8 GiB of
 * free blocks (beyond that a released block is freed at once), and a
 * failing hipMalloc first frees every cached block and tries again.
 * nufft_release_cache frees every cached block now (hipFree, which waits
 * for the device); blocks in use by live plans are not affected.  Always
 * FN_OK. */
int nufft_release_cache(void);

/* Message for the last non-OK status on this thread ("" if none). */
const char *nufft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FMMNUFFT_H */

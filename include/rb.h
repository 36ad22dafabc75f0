/*
 * rb.h -- C ABI of librb.so, an MI355X (gfx950) implementation of the
 * reduced-basis greedy of Antil, Chen & Field, "A Note on QR-Based Model
 * Reduction" (arXiv 1805.06124): column-pivoted QR of a dense complex
 * snapshot matrix S (N rows x M columns) by the RB-greedy (Alg. 3, Sec. 5.2.1,
 * equivalent to MGS with column pivoting, Alg. 2, by Proposition 5.3).
 *
 * Conventions (all entry points)
 *  - Matrices are column-major: column j of an N x M matrix X with leading
 *    dimension ldX (>= N) starts at element j*ldX.  Complex numbers are
 *    interleaved (re, im) pairs: complex128 = two doubles, complex64 = two
 *    floats.  A row-major torch tensor of shape (M, N) is exactly this layout
 *    with ld = N.
 *  - Pointers documented as "device" must point to device memory of the
 *    current HIP device; "host" pointers to ordinary host memory.  All memory
 *    passed in is owned by the caller; the library never frees it.  A call
 *    allocates the scratch it needs with hipMalloc and frees it before
 *    returning (the large ones are stated with each entry point: the
 *    greedy's anchor_max x M coefficient panel, regeneration chunks,
 *    coefficient workspaces), except where the caller hands in a workspace:
 *    the greedies take one (ws, ws_bytes; sizes from rb_greedy_z_workspace
 *    and rb_greedy_c_workspace) and then allocate nothing.
 *  - Work is enqueued on the given stream (NULL = the default stream).
 *    Calls return after that work has completed (the greedy takes a host
 *    decision after every step), except those documented as "enqueued, not
 *    synchronised": rb_chirp_table, rb_chirp_regen, rb_chirp_params,
 *    rb_stream_read and the surrogate's calls (rb_mlp_*, rb_coef_*).
 *  - Return value: an rb_status code.  Arguments are validated on the host
 *    before any device work; a call that fails later (a device error, a
 *    non-finite value found on the way) may have written part of its
 *    outputs.  rb_last_error() gives a message for the last failing call on
 *    the calling thread.
 *  - Inner product: <e, s> = e^H s (the paper's real transpose read as the
 *    conjugate transpose); norms are Euclidean, unweighted.
 */
#ifndef RB_H
#define RB_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rb_status {
  RB_OK = 0,            /* greedy: stopped because err < tol */
  RB_KMAX = 1,          /* greedy: stopped at kmax without reaching tol */
  RB_RANK = 2,          /* greedy: the next pivot lies numerically in the span
                           of the basis (rank exhausted); err is at rounding
                           level */
  RB_EINVAL = -1,       /* bad dimensions, pointers or options */
  RB_ENOMEM = -2,       /* device allocation failed */
  RB_EDEVICE = -3,      /* HIP runtime error or no usable device */
  RB_ENONFINITE = -4,   /* an input (S, V) holds a NaN or Inf, a norm
                           overflows, or a re-anchored or regenerated column
                           is not finite */
  RB_EBREAKDOWN = -5,   /* greedy: iterated Gram-Schmidt did not settle --
                           the last of nu_max passes still shrank ||v|| by
                           the factor kappa (Hoffmann's criterion, Sec. 6.1.2)
                           while ||v|| >= tol */
  RB_ENOCONV = -6       /* an iterative eigen-solve did not converge */
} rb_status;

/* Options of the greedy; rb_default_opts() fills the defaults. */
typedef struct rb_opts {
  double kappa;     /* Hoffmann's iterated Gram-Schmidt criterion (Sec. 6.1.2):
                       another pass is made while a pass shrinks ||v|| by at
                       least the factor kappa.  Default 2. */
  int32_t nu_max;   /* maximum Gram-Schmidt passes per vector.  Default 4. */
  int32_t nu_min;   /* minimum passes.  Default 1.  Each pass is one classical
                       Gram-Schmidt projection in matrix-vector form,
                       v -= E (E^H v).  If the last of nu_max passes still
                       shrank ||v|| by kappa, the greedy stops with
                       RB_EBREAKDOWN when ||v|| >= tol (a vector already
                       below tol is accepted). */
  double theta;     /* resolution threshold of the Eq. (6.3) update: when the
                       largest estimated residual^2 falls below theta times
                       the largest residual^2 at the last re-anchoring, the
                       working columns are re-anchored (deflated explicitly).
                       The estimate carries a rounding error of a few
                       (k+1) u times that residual^2, so at the threshold
                       its relative error is about (k+1) u / theta: with
                       the default 1e-7, 1.6e-7 at k = 141 (pivot choice and
                       err_k to that accuracy; fewer, larger re-anchorings
                       than a coarser theta). */
  int32_t anchor_max; /* re-anchor at the latest after this many basis vectors
                         since the last anchoring (bounds the coefficient
                         panel, anchor_max x M complex128).  Default 128. */
  int32_t collect_stats; /* 1: fill rb_stats timings with HIP events. */
  /* mixed precision (rb_greedy_c) only: */
  double theta32;     /* re-anchor when the largest estimated residual^2 of
                         the complex64 sweep falls below theta32 times its
                         last anchored scale.  Default 1e-4. */
  int32_t regen_chunk; /* columns regenerated in FP64 per chunk during an
                          exact re-anchoring (scratch: regen_chunk x N
                          complex128 plus kmax x regen_chunk complex128).
                          Default 32768. */
  int32_t certify;    /* before returning converged: 1 = recompute every
                         column's residual exactly in FP64 from regenerated
                         columns and continue if one is still >= tol; 2 =
                         the same, unless the sweep's largest estimate plus
                         its rounding and perturbation bound is already
                         below tol^2; 0 = no check.  Default 2. */
  double *step_ms;    /* host, NULL or 3 * (kmax + 1) doubles, zeroed by the
                         caller (collect_stats = 1): for basis vector i (its
                         position in E), device milliseconds are added of its
                         orthogonalisation (mixed: the confirmation that
                         chose it) at [3i], of the sweep with it at [3i+1]
                         and of the re-anchorings that followed that sweep at
                         [3i+2]; [3k] may receive the final confirmation
                         that found the error below tol.  Default NULL. */
  int32_t fuse;       /* FP64 greedy: 1 = when the next estimate is predicted
                         to lose resolution, at most 16 vectors were swept
                         since the last written anchoring and a norms-only
                         re-anchoring is accurate enough, fold it into the
                         next sweep (one read of the working matrix for
                         both); 0 = separate passes only.  Default 1. */
  int32_t lookahead;  /* pivots predicted per sweep, 0..5.  Before
                         a sweep the next pivots are predicted from the
                         look_k columns with the best estimates: each listed
                         column's coefficient with the newest vector (and
                         with each predicted vector in turn) and its updated
                         Eq. (6.3) estimate are formed with the sweep's own
                         arithmetic, the best is orthogonalised as its step
                         would do it, and the sweep reads the working
                         matrix once for the newest and the predicted
                         vectors.  A step whose pivot was predicted then
                         takes that vector and its coefficients without a
                         sweep of its own.  Mixed precision (rb_greedy_c,
                         depth lookahead32): the prediction is the top-8
                         set of the complex64
                         estimates and its FP64 confirmation; a step takes
                         it when the set comes true (16-byte aligned
                         complex64 columns with N even; otherwise no
                         lookahead).  Pivots, errors, residuals and basis
                         are bit-identical for every value; columns of E
                         past the returned k may hold predicted vectors.
                         0 = off.  Default 5. */
  int32_t look_k;     /* length of the candidate list, 1..8192.  Default 4096. */
  int32_t lookahead32; /* mixed greedy (rb_greedy_c): its own depth, 0..5,
                          or -1 = 2 below 1,000,000 columns and 5 from
                          there (lookahead applies to the FP64 greedy).
                          The complex64 sweep is bound by FP32
                          multiply-adds, so each predicted vector costs
                          more there, and each prediction is an FP64
                          confirmation of eight regenerated columns, a
                          fixed cost that longer reads amortise (measured
                          on 10,000 rows: depth 2 best at 409,600 columns,
                          5 at 1,638,400).  Default -1. */
} rb_opts;

/* Per-call statistics (host struct, optional). */
typedef struct rb_stats {
  int64_t sweeps;      /* plain sweeps run (one per basis vector, unless the
                          vector's sweep was a fused pass, see fused) */
  int64_t anchors;     /* explicit re-anchorings (all kinds) */
  int64_t gs_passes;   /* Gram-Schmidt passes over all vectors */
  double ms_sweep;     /* device time of the plain sweep kernels alone
                          (collect_stats = 1) */
  double ms_gs;        /* device time in orthogonalisation (and, mixed
                          precision, candidate confirmation) */
  double ms_anchor;    /* device time in re-anchoring */
  double ms_total;     /* wall time of the call */
  int64_t regen_anchors; /* mixed: re-anchorings from regenerated FP64
                            columns (the others deflate the stored columns) */
  int64_t misses;      /* mixed: steps whose confirmed pivot was not the
                          sweep's top candidate */
  int64_t fused;       /* FP64: sweeps that also re-anchored (one read of
                          the working matrix for both; counted in anchors,
                          not in sweeps) */
  double ms_fused;     /* device time of those fused passes */
  int64_t look_sweeps; /* FP64: sweeps that carried predicted vectors */
  int64_t look_steps;  /* FP64: steps taken from a prediction (no sweep and
                          no orthogonalisation of their own; not counted in
                          sweeps) */
  int64_t look_gs;     /* FP64: orthogonalisations of predicted pivots */
  double ms_look;      /* device time of the predictions (candidate list,
                          reranking, orthogonalisation of predicted pivots) */
  double ms_apply;     /* device time of the steps taken from a prediction
                          (estimate update and argmax) */
  double ms_look_sweep; /* FP64: device time of the sweeps that carried
                           predicted vectors (part of ms_sweep) */
  int64_t look_vectors; /* FP64: predicted vectors carried by those sweeps */
} rb_stats;

void rb_default_opts(rb_opts *opts);

/* Status string for a code, and the message of the calling thread's last
 * failing call ("" if none). */
const char *rb_strerror(int status);
const char *rb_last_error(void);

/*
 * rb_colnorms_z -- exact squared column norms (the initial residual norms of
 * Alg. 3, ||s_i||^2).  Each column's sum of squares is accumulated without
 * rounding error (double-double, error-free products) and rounded to double
 * once, so every correct implementation returns the same bits.
 *   S    device, complex128 N x M, ldS >= N           (read)
 *   nrm  device, double[M]                           (written)
 * Returns RB_ENONFINITE if any column holds a NaN/Inf or its norm overflows.
 */
int rb_colnorms_z(const void *S, int64_t N, int64_t M, int64_t ldS, double *nrm, hipStream_t stream);

/*
 * rb_sweep_z -- one pivot-search sweep of the greedy (Sec. 6.1.2, Eqs.
 * (6.1)-(6.3)) fused into a single read of S:
 *   c_j    = e^H s_j                      for every column j
 *   acc_j += |c_j|^2                      (running sum of c c*)
 *   est_j  = nrm_j - acc_j                (estimated squared residual)
 *   (est_max, J) = max over j with mask_j == 0 of est_j; ties -> lowest j
 *   S      device, complex128 N x M, ldS >= N  (read)
 *   e      device, complex128[N], the newest basis vector (read)
 *   nrm    device, double[M]                   (read)
 *   acc    device, double[M]                   (read, updated in place)
 *   mask   device, uint8[M]; nonzero = already pivoted, excluded from the
 *          argmax (acc is still updated)       (read; may be NULL = none)
 *   c_out  device, complex128 with stride ldc elements between consecutive
 *          columns' coefficients: c_j is stored at c_out[j*ldc]; NULL = not
 *          stored
 *   est_max, J  host; J = -1 and est_max = -inf if every column is masked.
 */
int rb_sweep_z(const void *S, int64_t N, int64_t M, int64_t ldS, const void *e, const double *nrm,
               double *acc, const uint8_t *mask, void *c_out, int64_t ldc, double *est_max, int64_t *J,
               hipStream_t stream);

/*
 * rb_sweep_c -- the mixed-precision sweep of rb_greedy_c: as rb_sweep_z but
 * over complex64 columns with a complex64 copy of the basis vector; products
 * and row-tile sums in FP32 (tiles of 512 rows per lane group), FP64 across
 * tiles; acc, est and c_out FP64.  Returns the 8 largest (est, index) pairs
 * over unmasked columns in est_top[0..8), J_top[0..8) (host), descending,
 * ties to the lower index; unused slots have J_top = -1.
 *   S32  device, complex64 N x M, ldS >= N;  e32 device, complex64[N]
 */
int rb_sweep_c(const void *S32, int64_t N, int64_t M, int64_t ldS, const void *e32, const double *nrm,
               double *acc, const uint8_t *mask, void *c_out, int64_t ldc, double *est_top, int64_t *J_top,
               hipStream_t stream);

/*
 * rb_greedy_z -- the RB-greedy (Alg. 3) in FP64 over complex128 S.
 * Stopping rule (Alg. 3 and Corollary 5.6, tolerance on the unsquared error):
 * vectors are added while err_k >= tol and k < kmax, where
 * err_k = max over unpivoted j of ||s_j - E_k E_k^H s_j||_2 (= |R_{k+1,k+1}|).
 * Pivot k is the argmax of the residual (lowest index on ties); the pivot
 * column is orthonormalised against the basis by iterated Gram-Schmidt with
 * Hoffmann's kappa criterion (Sec. 6.1.2).
 *   S      device, complex128 N x M, ldS >= N.  Read only, unless W == S.
 *   W      device, complex128 N x M, ldW >= N: working matrix for explicit
 *          re-anchoring (the residual columns s_j - E E^H s_j are written
 *          here).  May equal S (S is then overwritten with residuals), or
 *          NULL: the library allocates it on first use and frees it
 *          (not allowed with ws).
 *   E      device, complex128 N x kmax, ldE >= N: the basis e_1..e_k (out)
 *   piv    host int64[kmax]: pivot column indices (0-based) (out)
 *   err    host double[kmax+1]: err[i] = greedy error with i vectors (out)
 *   rho    host double[kmax]: ||v|| of pivot i after orthogonalisation,
 *          i.e. |R_ii| (out)
 *   nu     host int32[kmax] Gram-Schmidt passes per vector, or NULL (out)
 *   k_out  host: number of basis vectors k (out)
 *   ws     device workspace of ws_bytes >= rb_greedy_z_workspace(N, M,
 *          kmax, opts) bytes, 256-byte aligned, or NULL.  With ws the call
 *          allocates nothing (no device or pinned host memory); without it
 *          the same scratch is allocated and freed inside the call.  Its
 *          contents on entry do not matter; calls that share one ws must not
 *          overlap.
 *   opts   NULL = defaults;  stats: NULL or host rb_stats (out)
 * kmax is clamped to min(N, M).  If max ||s_j|| < tol, k = 0.
 * Returns RB_OK, RB_KMAX or RB_RANK on success; RB_ENOMEM if ws_bytes is too
 * small (checked before any device work); RB_EBREAKDOWN (see nu_min);
 * RB_ENONFINITE if S, a re-anchored column or a swept estimate is not finite.
 * On an error the outputs up to the last completed step are valid and
 * *k_out is not written.
 */
int rb_greedy_z(const void *S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, void *W,
                int64_t ldW, void *E, int64_t ldE, int64_t *piv, double *err, double *rho, int32_t *nu,
                int64_t *k_out, void *ws, size_t ws_bytes, const rb_opts *opts, rb_stats *stats,
                hipStream_t stream);

/*
 * rb_greedy_z_workspace -- bytes of device workspace rb_greedy_z and
 * rb_greedy_resume_z need for these sizes and options (opts NULL =
 * defaults): per-column norms, estimates and mask (25 M bytes), the
 * coefficient panel (16 anchor_max M bytes), argmax partials and
 * Gram-Schmidt vectors.  0 for invalid sizes.
 */
size_t rb_greedy_z_workspace(int64_t N, int64_t M, int64_t kmax, const rb_opts *opts);

/*
 * rb_greedy_z_noalloc -- for callers that cannot allocate memory (code that
 * must not call hipMalloc, tight serving loops, harnesses that forbid it):
 * rb_greedy_z with its workspace in a fixed device array of the library,
 * RB_NOALLOC_SCRATCH_BYTES (64 MiB) on every device it runs on, held until
 * the process ends.  It allocates neither device nor pinned host memory and
 * creates no HIP events (opts->collect_stats is ignored: no timings).
 * Arguments as rb_greedy_z without ws; W is required (it may equal S).
 * Returns RB_ENOMEM, before any device work, when rb_greedy_z_workspace(N,
 * M, kmax, opts) exceeds the array (lower opts->anchor_max to fit more
 * columns: about 16 anchor_max M + 41 M bytes).  Every call on a device
 * shares that device's array and keeps nothing from an earlier call; calls
 * that overlap on one device race on it.
 */
#define RB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int rb_greedy_z_noalloc(const void *S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, void *W,
                        int64_t ldW, void *E, int64_t ldE, int64_t *piv, double *err, double *rho, int32_t *nu,
                        int64_t *k_out, const rb_opts *opts, rb_stats *stats, hipStream_t stream);

/*
 * rb_regen_fn -- regenerates snapshot columns in FP64 from their parameters
 * (the paper's model interface: S is filled by calls to a model, Sec. 6.1.1).
 *   ctx   caller context
 *   cols  device int64[n]: column indices to regenerate
 *   out   device complex128 N x n, leading dimension ldo (written); column
 *         r receives snapshot cols[r]
 * Must enqueue on `stream` and return 0 on success (nonzero aborts the
 * greedy with RB_EDEVICE).
 */
typedef int (*rb_regen_fn)(void *ctx, const int64_t *cols, int64_t n, void *out, int64_t ldo,
                           hipStream_t stream);

/* Context of the built-in regenerator rb_chirp_regen: the chirp family of
 * rb_chirp_fill with parameters params (device, 2*M doubles), band
 * [flo, fhi] and N rows.  table: device, 3*N doubles prepared by
 * rb_chirp_table for (flo, fhi, N), or NULL (then every call builds its
 * own). */
typedef struct rb_chirp_ctx {
  const double *params;
  double flo, fhi;
  int64_t N;
  const double *table;
} rb_chirp_ctx;

/* Row table of the chirp family on N points of [flo, fhi] (all columns
 * share it): table[3n] = f_n^(-7/6) / ||h||, table[3n+1] = f_n^(-5/3),
 * table[3n+2] = 1/f_n, where ||h||^2 = sum_n f_n^(-7/3) is every column's
 * squared norm (the amplitude does not depend on the phase).  Enqueued on
 * stream, not synchronised. */
int rb_chirp_table(double flo, double fhi, int64_t N, double *table, hipStream_t stream);

/* rb_regen_fn for the chirp family (ctx is a rb_chirp_ctx*); enqueued, not
 * synchronised. */
int rb_chirp_regen(void *ctx, const int64_t *cols, int64_t n, void *out, int64_t ldo, hipStream_t stream);

/*
 * rb_greedy_c -- the RB-greedy with complex64 snapshot storage (mixed
 * precision).  The pivot search sweeps the complex64 columns with an FP32
 * copy of the newest basis vector (FP32 products, FP32 sums per row tile,
 * FP64 across tiles); acc, est and the coefficients are FP64.  The sweep
 * nominates its 8 best candidates; each is regenerated in FP64 by `regen`
 * and orthogonalised against the FP64 basis (iterated Gram-Schmidt, kappa
 * criterion); the pivot is the candidate with the largest exact FP64
 * residual rho, and err_k is that rho (Corollary 5.6: the greedy error is
 * the next pivot's residual).  When the complex64 estimate loses
 * resolution the stored columns are re-anchored to their residuals, either
 * by deflating the stored values (while the rounding this leaves stays
 * below a tenth of tol, or will be reset by a later exact re-anchoring) or
 * exactly, from columns regenerated in FP64.  With opts->certify the final
 * error is checked over all columns from regenerated FP64 columns.
 *   S32    device, complex64 N x M, ldS >= N (read only unless W32 == S32)
 *   regen, regen_ctx   column regenerator (required)
 *   W32    device, complex64 N x M working matrix (ldW), may equal S32, or
 *          NULL (allocated on first use; not allowed with ws)
 *   ws     device workspace of ws_bytes >= rb_greedy_c_workspace(N, M, kmax,
 *          opts) bytes, or NULL (as rb_greedy_z; the regenerator is the
 *          caller's and may allocate what it needs)
 *   E, piv, err, rho, nu, k_out, opts, stats: as rb_greedy_z (E is FP64)
 * Returns as rb_greedy_z; RB_EBREAKDOWN when the chosen candidate's
 * Gram-Schmidt did not settle; RB_ENONFINITE also for a non-finite
 * regenerated candidate.
 */
int rb_greedy_c(const void *S32, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                rb_regen_fn regen, void *regen_ctx, void *W32, int64_t ldW, void *E, int64_t ldE,
                int64_t *piv, double *err, double *rho, int32_t *nu, int64_t *k_out, void *ws, size_t ws_bytes,
                const rb_opts *opts, rb_stats *stats, hipStream_t stream);

/*
 * rb_greedy_c_workspace -- bytes of device workspace rb_greedy_c needs:
 * that of rb_greedy_z plus the 8 candidate columns and, for the exact
 * re-anchorings, regen_chunk FP64 columns with their min(kmax, N) x
 * regen_chunk coefficients (16 regen_chunk (N + min(kmax, N)) bytes).
 * 0 for invalid sizes.
 */
size_t rb_greedy_c_workspace(int64_t N, int64_t M, int64_t kmax, const rb_opts *opts);

/*
 * rb_project_z -- C = E^H S (the coefficients of every snapshot on the
 * basis; the projection E E^H s of Sec. 4), complex128, FP64 matrix cores.
 *   E  device, complex128 N x k, ldE >= N     (read)
 *   S  device, complex128 N x M, ldS >= N     (read)
 *   C  device, complex128 k x M, ldC >= k     (written)
 */
int rb_project_z(const void *E, int64_t N, int64_t k, int64_t ldE, const void *S, int64_t M, int64_t ldS,
                 void *C, int64_t ldC, hipStream_t stream);

/*
 * rb_greedy_resume_z -- rb_greedy_z continued from a basis that already
 * holds k0 orthonormal vectors (the enrichment step of Sec. 6.1: columns
 * that fail out-of-sample validation continue the greedy of the existing
 * basis).
 * Every column of S is first reduced against e_1..e_k0:
 * X = S - E0 (E0^H S), a block of at most opts->anchor_max vectors at a
 * time, written to W.  The greedy then runs from k = k0 exactly as in
 * rb_greedy_z: same pivot rule, orthogonalisation and stopping test, with
 * err_k = max_j ||s_j - E_k E_k^H s_j||.
 *   E      device, N x kmax, ldE >= N: columns 0..k0-1 hold the starting
 *          basis on entry (read); columns k0..k-1 are written
 *   k0     0 <= k0 <= min(kmax, N); k0 = 0 is rb_greedy_z
 *   W      as in rb_greedy_z; NULL = allocated (N x M) when k0 > 0
 *   piv, err, rho, nu  indexed by the basis position: entries k0..k-1
 *          (err: k0..k) are written, lower entries are left untouched;
 *          piv holds column indices of S
 *   ws, ws_bytes  as rb_greedy_z (rb_greedy_z_workspace sizes it)
 * kmax is clamped to min(N, k0 + M).  Returns as rb_greedy_z.
 */
int rb_greedy_resume_z(const void *S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, void *W,
                       int64_t ldW, void *E, int64_t ldE, int64_t k0, int64_t *piv, double *err, double *rho,
                       int32_t *nu, int64_t *k_out, void *ws, size_t ws_bytes, const rb_opts *opts,
                       rb_stats *stats, hipStream_t stream);

/*
 * rb_residual_norms_z -- out-of-sample validation (Sec. 6.1): the explicit
 * residual of every column against the orthonormal basis E,
 *   out[j] = || v_j - E (E^H v_j) ||_2,
 * by two FP64 matrix-core passes over V (C = E^H V, then the norms of
 * V - E C; no Pythagorean shortcut).
 *   E    device, complex128 N x k, ldE >= N (read); k = 0 gives ||v_j||
 *   V    device, complex128 N x M, ldV >= N (read)
 *   out  device, double[M] (written)
 * Allocates k x min(M, 65536) coefficients of workspace.  Returns
 * RB_ENONFINITE if a residual is not finite.
 */
int rb_residual_norms_z(const void *E, int64_t N, int64_t k, int64_t ldE, const void *V, int64_t M, int64_t ldV,
                        double *out, hipStream_t stream);

/*
 * rb_enrich_z -- validation and iterative enrichment of a basis (Sec. 6.1).
 * Round r (0 <= r < rounds) validates the columns r*Mv .. r*Mv + Mv - 1 of
 * the regenerator's family against the current basis:
 *   1. regenerate them in chunks of opts->regen_chunk columns;
 *   2. take their explicit residuals (as rb_residual_norms_z);
 *   3. regenerate the columns with residual >= tol (NaN counts as failing),
 *      in index order;
 *   4. continue the greedy on them from the current basis
 *      (rb_greedy_resume_z, overwriting them in place).
 * Afterwards every column of the round is below tol, unless kmax stopped
 * the greedy first.
 *   regen, regen_ctx  column generator (rb_regen_fn); cols are indices into
 *          its family
 *   E      device, N x kmax, ldE >= N: columns 0..k_in-1 hold the basis on
 *          entry; new vectors are appended
 *   piv    host int64[kmax]: entries k_in..k-1 receive the family index of
 *          each added vector
 *   err, rho, nu  as rb_greedy_resume_z, per basis position.  err[i] is the
 *          largest residual, after i vectors, over the failing columns of
 *          the round that added vector i (a round's first entry is its
 *          largest failing residual)
 *   k_out  host: basis size at the end
 *   n_fail host int64[rounds]: failing columns per round
 *   resid_max  host double[rounds]: largest residual of each round,
 *          against the basis at the round's start
 *   resid  device double[rounds*Mv]: every residual, or NULL
 *   stats  NULL or host rb_stats: the continued greedies' totals
 * Returns RB_OK; RB_KMAX if kmax = min(kmax, N) stopped a round while
 * columns were still failing; RB_RANK as the greedy does; negative codes on
 * error.
 */
int rb_enrich_z(rb_regen_fn regen, void *regen_ctx, int64_t N, int64_t Mv, int64_t rounds, double tol,
                int64_t kmax, void *E, int64_t ldE, int64_t k_in, int64_t *piv, double *err, double *rho,
                int32_t *nu, int64_t *k_out, int64_t *n_fail, double *resid_max, double *resid,
                const rb_opts *opts, rb_stats *stats, hipStream_t stream);

/*
 * rb_reconstruct_z -- the reconstruction algorithm (Alg. 4, Sec. 5.2.2;
 * Theorem 5.8).  After a j-term greedy, the coefficients C = E^H S equal
 * R(1:j, :) up to the column order.  With the SVD C = V Sigma W^H, the
 * routine keeps k = #{i : sigma_i >= tau2} (so sigma_{k+1} < tau2 <= sigma_k)
 * and returns X_k = E V(:, 1:k), an N x k orthonormal basis with
 * ||S - X_k X_k^H S||_2 = sigma_{k+1} whenever S = E C exactly.
 * The left singular pair is computed on the GPU:
 *   1. the Gram matrix C C^H;
 *   2. its Jacobi eigenvectors V0;
 *   3. a refinement: Jacobi on (V0^H C)(V0^H C)^H gives V1 and the
 *      eigenvalues, with V = V0 V1.
 * The singular values then carry an absolute error of a few u sigma_1.
 *   E      device, complex128 N x j, ldE >= N (read), 1 <= j <= min(N, 2048)
 *   C      device, complex128 j x M, ldC >= j (read): E^H S
 *   X      device, complex128 N x j capacity, ldX >= N: columns 0..k-1
 *          written
 *   sigma  host double[j]: the singular values of C, non-increasing (out)
 *   Vout   device, complex128 j x j (ld j): the left singular vectors of C
 *          in the same order, or NULL (out)
 *   k_out  host: k (out)
 *   ws, ws_bytes  device workspace of at least
 *          rb_reconstruct_z_workspace(j, M) bytes (about 16 (j M + 5 j^2)
 *          bytes, 16 KB of partial Gram tiles per (32-row tile pair, split)
 *          and, for j <= 141, a rotation log of 60 (j + 1)^2 / 2 x 32
 *          bytes), 256-byte aligned (else RB_EINVAL); caller-owned,
 *          contents undefined on return.  ws == NULL: the call allocates and
 *          frees it itself.  A smaller ws_bytes returns RB_ENOMEM.
 * Returns RB_ENOCONV if a Jacobi solve does not settle within 60 sweeps.
 */
int rb_reconstruct_z(const void *E, int64_t N, int64_t j, int64_t ldE, const void *C, int64_t M, int64_t ldC,
                     double tau2, void *X, int64_t ldX, double *sigma, void *Vout, int64_t *k_out, void *ws,
                     size_t ws_bytes, hipStream_t stream);

/*
 * rb_reconstruct_z_workspace -- device workspace bytes rb_reconstruct_z
 * needs for j basis vectors and M columns of C; 0 for sizes it rejects
 * (j < 1, j > 2048, M < 1).
 */
size_t rb_reconstruct_z_workspace(int64_t j, int64_t M);

/*
 * rb_eim_z -- empirical-interpolation (EI) nodes of the basis e_1..e_k
 * (Sec. 6.1; the standard discrete empirical interpolation method).
 * Node p_1 maximises |e_1(n)|.  Node p_j maximises |r_j(n)|, where
 * r_j = e_j - I_{j-1}[e_j] and I_{j-1} interpolates on e_1..e_{j-1} through
 * p_1..p_{j-1}.  Ties go to the lowest row.  The residuals are formed by
 * elimination: r_j = e_j - sum_{i<j} alpha_i r_i, with each r_i stored
 * divided by r_i(p_i).
 *   E      device, complex128 N x k, ldE >= N: the basis, linearly
 *          independent (orthonormal from the greedy) (read)
 *   nodes  host int64[k]: p_1..p_k, 0-based rows (out)
 *   peak   host double[k]: |r_j(p_j)|, the pivots of the elimination (out),
 *          or NULL
 *   R      device, complex128 N x k (ld N): the normalised residuals
 *          r_j / r_j(p_j) (out), or NULL (internal)
 *   Tinv   device, complex128 k x k (ld k): the inverse of the unit lower
 *          triangular T[l, i] = r_i(p_l) / r_i(p_i) (out), or NULL.
 *          The empirical interpolant of v is I[v] = R (Tinv v(p)).
 *   k_out  host: k, or the first j (0-based) with r_j numerically zero,
 *          max |r_j| <= 64 (j+1) u max |e_j| (a linearly dependent basis,
 *          status RB_RANK)
 * Per node: four small kernels, enqueued with no host synchronisation.
 */
int rb_eim_z(const void *E, int64_t N, int64_t k, int64_t ldE, int64_t *nodes, double *peak, void *R, void *Tinv,
             int64_t *k_out, hipStream_t stream);

/*
 * rb_eim_errors_z -- out-of-sample validation of the empirical interpolant
 * (Sec. 6.1): out[m] = || v_m - R (Tinv v_m(p)) ||_2 for the M columns of
 * V.  Each chunk of columns takes:
 *   1. a gather of the node rows;
 *   2. Tinv times that gather (matrix cores);
 *   3. the norms-only residual kernel.
 *   R, Tinv as written by rb_eim_z; nodes: device int64[k]
 *   V      device, complex128 N x M, ldV >= N (read);  out: device double[M]
 */
int rb_eim_errors_z(const void *R, int64_t N, int64_t k, int64_t ldR, const void *Tinv, const int64_t *nodes,
                    const void *V, int64_t M, int64_t ldV, double *out, hipStream_t stream);

/*
 * rb_chirp_fill -- the synthetic snapshot family standing in for the paper's
 * gravitational-wave model (Sec. 6.1.1): column j is the leading-1PN
 * frequency-domain chirp h(f) = f^(-7/6) exp(-i Psi(f)) with
 * Psi = -pi/4 + 3/(128 eta v^5) (1 + (3715/756 + 55 eta/9) v^2),
 * v = (pi Mtot f)^(1/3) (Mtot in seconds = solar masses * GM_sun/c^3),
 * eta = q/(1+q)^2, on the uniform grid f_n = flo + n (fhi - flo)/(N - 1),
 * normalised to unit L2 norm.  Evaluated in FP64; dtype 1 rounds the
 * normalised values to complex64.
 *   params  device, double[2*M]: (Mtot in solar masses, q) per column (read)
 *   out     device, complex128 (dtype 0) or complex64 (dtype 1), N x M, ld
 */
/*
 * rb_chirp_params -- parameters of the chirp family from a seed: column
 * start + t (t < M) takes Mtot = mlo + (mhi - mlo) u(seed, 2 (start + t)) and
 * q = qlo + (qhi - qlo) u(seed, 2 (start + t) + 1), where u(seed, i) =
 * (z >> 11) 2^-53 and z is the SplitMix64 output for counter i (Steele, Lea
 * & Flood 2014: state seed + (i + 1) 0x9E3779B97F4A7C15, finaliser
 * xor-shift 30, times 0xBF58476D1CE4E5B9, xor-shift 27, times
 * 0x94D049BB133111EB, xor-shift 31).  Every operation is rounded on its
 * own (no fused multiply-add).
 *   params  device, double[2*M]: (Mtot in solar masses, q) per column (out)
 * Enqueued, not synchronised.
 */
int rb_chirp_params(uint64_t seed, int64_t start, int64_t M, double mlo, double mhi, double qlo, double qhi,
                    double *params, hipStream_t stream);

/*
 * rb_stream_read -- reads `bytes` of device memory once with 16-byte
 * streaming loads and writes one partial sum per workgroup to
 * partial[0..npartial) (device).  This is a plain read whose rate is the
 * achievable HBM bandwidth, measured beside the sweep.  npartial is the
 * grid size (workgroups of 256 threads in a grid-stride loop; 2048, eight
 * per compute unit, reads fastest on MI355X).  bytes is a multiple of 16,
 * p is 16-byte aligned, and 1 <= npartial <= 65535.
 * Enqueued, not synchronised.
 */
int rb_stream_read(const void *p, size_t bytes, double *partial, int64_t npartial, hipStream_t stream);

int rb_chirp_fill(const double *params, int64_t M, double flo, double fhi, int64_t N, int dtype, void *out,
                  int64_t ld, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned coefficient surrogate (not part of the paper's method: an MLP that
 * predicts the projection coefficients c = E^H s of a snapshot from its
 * parameters, with the plain projection of the regenerated snapshot as the
 * check and fallback).  Network din -> hidden -> hidden -> hidden -> dout,
 * tanh hidden layers, linear output; BF16 weights and activations, FP32
 * accumulation on BF16 matrix cores, FP32 master weights for Adam.
 *
 * Parameters: one FP32 buffer p32 and one BF16 buffer p16 (uint16 bit
 * patterns) of rb_mlp_param_count() entries, laid out row-major [in][out]:
 * W1 (din x hidden), b1, W2 (hidden x hidden), b2, W3, b3,
 * W4 (hidden x dout), b4.  Inputs X: FP32 [batch][din]; outputs Y: FP32
 * [batch][dout].  The workspace ws (device, rb_mlp_workspace_bytes())
 * keeps the activations of the last forward for the backward pass and for
 * rb_mlp_loss.  It begins with the hidden activations H1, H2, H3 of the
 * last forward, then dZ1 and dZ2 (the pre-activation gradients of hidden
 * layers 1 and 2) of the last backward, each BF16 [batch][hidden], then dY
 * of the last loss, BF16 [batch][dout].  1 <= din <= 1024: up to 4 inputs the first layer runs on
 * vector units, wider inputs take the BF16 matrix cores like the other
 * layers.
 * ---------------------------------------------------------------------- */
int64_t rb_mlp_param_count(int din, int hidden, int dout);
size_t rb_mlp_workspace_bytes(int64_t batch, int din, int hidden, int dout);

/* Y = MLP(X) (Y may be NULL: kept in the workspace). */
int rb_mlp_forward(const float *p32, const uint16_t *p16, int din, int hidden, int dout, const float *X,
                   int64_t batch, float *Y, void *ws, hipStream_t stream);

/* Mean squared error over batch x dout of Y - T into *loss (device float)
 * and its gradient dY = 2 (Y - T) / (batch dout) as BF16 (dY NULL: kept in
 * the workspace).  Y NULL: the workspace output of the last forward. */
int rb_mlp_loss(const float *Y, const float *T, int64_t batch, int dout, uint16_t *dY, float *loss, void *ws,
                int din, int hidden, hipStream_t stream);

/* Gradients of the loss w.r.t. all parameters into grad (FP32, p32 layout),
 * given dY (BF16; NULL = the workspace's) and the activations of the last
 * forward on the same X.  Every sum over the batch is added in a fixed
 * order, so repeated calls give identical bits. */
int rb_mlp_backward(const float *p32, const uint16_t *p16, int din, int hidden, int dout, const float *X,
                    int64_t batch, const uint16_t *dY, float *grad, void *ws, hipStream_t stream);

/* One Adam step (Kingma & Ba, bias-corrected) on the FP32 master p32 with
 * moments m, v; refreshes the BF16 copy p16.  step >= 1. */
int rb_mlp_adam(float *p32, uint16_t *p16, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                float beta2, float eps, int64_t step, hipStream_t stream);

/* Batch gather: X[b] = params[idx[b]] (2 doubles) mapped affinely from
 * [ranges[0], ranges[1]] x [ranges[2], ranges[3]] (host array) onto
 * [-1, 1]^2; T[b] = targets[idx[b]] (dout floats) if targets != NULL. */
int rb_mlp_gather(const double *params, const float *targets, const int64_t *idx, int64_t batch, int dout,
                  const double *ranges, float *X, float *T, hipStream_t stream);

/* Surrogate inputs that carry the snapshot's phase (the chirp family of
 * rb_chirp_fill; the empirical-interpolation idea of Sec. 6.1: a snapshot is
 * fixed by its values at k interpolation nodes, and on this family every
 * snapshot has the same amplitude there, so its coefficients are a linear
 * map of its phase factors at the nodes).  Row b of X (din = 2 + 2F floats)
 * is built for sample idx[b]: the parameters mapped affinely from the box
 * ranges (host, as rb_mlp_gather) onto [-1, 1]^2, then cos Psi(f_n) and
 * -sin Psi(f_n) for each of the F grid rows n = rows[r] (device int64,
 * typically the nodes of rb_eim_z), with table from rb_chirp_table for the
 * grid.  T[b] = targets[idx[b]] (dout floats) if targets != NULL.
 * 1 <= F, 2 + 2F <= 1024.  Enqueued, not synchronised. */
int rb_mlp_phase_features(const double *params, const float *targets, const int64_t *idx, int64_t batch, int dout,
                          const double *ranges, const int64_t *rows, int64_t F, const double *table, float *X,
                          float *T, hipStream_t stream);

/* Whole training runs: steps Adam steps, step s on the batch of samples
 * idx[s*batch .. (s+1)*batch) (device int64) with learning rate lr[s] (host
 * float[steps]); the Adam step count runs from step0 + 1.  Each step
 * gathers its inputs (rb_mlp_phase_features when rows != NULL, with
 * din = 2 + 2F; else rb_mlp_gather, din = 2), then forward, loss, backward
 * and Adam, all enqueued on stream without synchronising.  The result is
 * bit-identical to calling those functions in turn; loss (device float[steps],
 * or NULL) receives each step's loss.  For 4 < din <= 512, hidden a multiple
 * of 64 up to 256 and dout <= 320 a step takes four launches besides the
 * gather: one kernel carries kRB = 16 samples per workgroup through all
 * layers forward and the loss gradient and dZ products backward with the
 * activations in LDS, then the split-K weight-gradient products, then one
 * kernel adds the splits and applies Adam.  Other shapes run the
 * layer-by-layer functions.  ws: device, at least
 * rb_mlp_train_workspace_bytes(); it begins with an rb_mlp workspace. */
size_t rb_mlp_train_workspace_bytes(int64_t batch, int din, int hidden, int dout);
int rb_mlp_train(float *p32, uint16_t *p16, float *m, float *v, int din, int hidden, int dout, const double *params,
                 const float *targets, const int64_t *idx, int64_t batch, int64_t steps, int64_t step0,
                 const float *lr, float beta1, float beta2, float eps, const double *ranges, const int64_t *rows,
                 int64_t F, const double *table, float *loss, void *ws, size_t ws_bytes, hipStream_t stream);

/* Coefficients C (complex128, sample j at C[j*ldc .. j*ldc+k)) -> FP32
 * targets T[j] = [Re c_j; Im c_j] (2k floats per sample). */
int rb_coef_targets(const void *C, int64_t ldc, int64_t Mn, int k, float *T, hipStream_t stream);

/* Per-sample relative coefficient error ||c_hat_j - c_j|| / ||c_j|| in
 * FP64 (= the relative L2 waveform error of E c_hat_j for orthonormal E);
 * Yh FP32 [Re; Im] per sample. */
int rb_coef_relerr(const float *Yh, const void *C, int64_t ldc, int64_t Mn, int k, double *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* RB_H */

/*
 * spai.h — C ABI of libspai: global short-recurrence sparse approximate inverses
 * (MR, CG and LOMR with sparse matrix iterates and Frobenius inner products) of a
 * symmetric positive definite matrix on an AMD Instinct MI355X (gfx950), and the
 * preconditioned CG solve that applies the result.
 *
 * Method source: Venkovic & Anzt, "Global Iterative Methods for Sparse Approximate
 * Inverses of Symmetric Positive Definite Matrices" — MR (Algorithm 1), CG with
 * matrix iterates (Definition 3.1, Proposition 3.2, Algorithm 3), LOMR
 * (Definition 4.1, Theorem 4.2, Algorithm 4), hard thresholding (Section 6.1),
 * the explicit residual (Section 6.2) and the main-iterate drop steps of Appendix A.
 *
 * Conventions shared by every entry point
 *  - Every function returns an int status: 0 = SPAI_OK, > 0 an informational
 *    outcome, < 0 an error.  No C++ exception and no abort crosses the ABI.  After
 *    an error, spai_last_error() returns a message for the calling thread.
 *  - Sparse inputs are CSR with int64 row pointers (n + 1 entries, rowptr[0] = 0,
 *    nondecreasing), int32 column indices sorted ascending and unique within each
 *    row, and float64 values.  "on_device" = 1 means the three arrays are device
 *    pointers valid on the current HIP device, 0 means host memory.  Inputs are
 *    borrowed for the duration of the call only: they are copied.
 *  - A must be exactly symmetric (pattern and values, bitwise), have a strictly
 *    positive diagonal stored explicitly and only finite values; violations
 *    return SPAI_ERR_NOT_SYMMETRIC, SPAI_ERR_NOT_SPD or SPAI_ERR_NONFINITE.
 *  - All device work is enqueued on opts->stream (a hipStream_t; NULL = the null
 *    stream).  Calls that return host results synchronise that stream.
 *  - Floating point: reductions (Frobenius inner products, norms, step sizes,
 *    PCG scalars) are always float64.  Iterate values are stored in float64 or,
 *    with SPAI_PREC_MIXED, float32.
 *  - Results are deterministic: the same inputs on the same device give bitwise
 *    identical iterates and scalars on every run.
 */
#ifndef SPAI_H
#define SPAI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
  SPAI_OK = 0,
  SPAI_CONVERGED = 1,       /* stopped because ||I - A M||_F / sqrt(n) <= tol   */
  SPAI_MAXITER = 2,         /* the requested iterations ran without converging  */
  SPAI_BREAKDOWN = 3,       /* a step size is undefined: CG (P, AP)_F <= 0      */
  PCG_INDEFINITE = 4,       /* PCG met (r, z) <= 0 or (p, A p) <= 0 on some RHS  */
  SPAI_ERR_ARG = -1,        /* bad shape, pointer, cap, method or option        */
  SPAI_ERR_NOT_SYMMETRIC = -2,
  SPAI_ERR_NOT_SPD = -3,    /* a diagonal entry is missing or not positive      */
  SPAI_ERR_NONFINITE = -4,
  SPAI_ERR_NOMEM = -5,      /* device allocation failed or exceeds the pool cap */
  SPAI_ERR_HIP = -6,        /* a HIP runtime call failed                        */
  SPAI_ERR_CAPACITY = -7    /* a column exceeded the largest per-column tile:
                               the device-memory tile, sized at create time from n
                               (lists up to 32768 entries, key sets up to 65535
                               rows; the update's own lists up to 131072 entries) */
};

enum { SPAI_MR = 0, SPAI_CG = 1, SPAI_LOMR = 2 };
enum { SPAI_PREC_F64 = 0, SPAI_PREC_MIXED = 1 };

/* Device layout of A inside a handle (results are bitwise the same in every layout):
 *  SPAI_AFMT_AUTO: ELL when the largest row degree is at most 64, else CSR;
 *  SPAI_AFMT_CSR:  CSR only;
 *  SPAI_AFMT_ELL:  ELL (rows padded to a power-of-two width >= 8), SPAI_ERR_ARG when a
 *                  row has more than 64 entries. */
enum { SPAI_AFMT_AUTO = 0, SPAI_AFMT_CSR = 1, SPAI_AFMT_ELL = 2 };
enum { SPAI_CAP_NONE = 0, SPAI_CAP_GLOBAL = 1, SPAI_CAP_COLUMN = 2 };

typedef struct spai_handle spai_handle_t;

/* Borrowed CSR matrix (see conventions above). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr;   /* [n + 1] */
  const int32_t* colind;   /* [nnz]   */
  const double* val;       /* [nnz]   */
  int on_device;
} spai_csr_t;

/* Density cap of the drop rule.
 *  SPAI_CAP_GLOBAL: |supp(M)| <= m and |supp(P)| <= m (Section 6.1, eq. of hard
 *    thresholding), m = value (relative = 0) or round(value * nnz(A)) (relative = 1).
 *    On M the diagonal is never dropped and counts toward m (Appendix A).
 *  SPAI_CAP_COLUMN: column j of M and of P keeps at most k_j entries, k_j = value
 *    or round(value * nnz(A e_j)); on M this includes the diagonal, and an
 *    off-diagonal entry of the symmetrized M survives only if it passes both its
 *    row's and its column's threshold, so M stays symmetric.
 *  SPAI_CAP_NONE: no count cap (the other drop steps still apply).
 * Ties: with t the (b+1)-th largest candidate magnitude for a budget b, the kept
 * entries are exactly those with |x| > t (1 + tie_eta). */
typedef struct {
  int mode;
  int relative;
  double value;
} spai_cap_t;

/* Options.  Pass NULL for the defaults shown. */
typedef struct {
  int precision;            /* SPAI_PREC_F64 (default) or SPAI_PREC_MIXED: M, P and R
                               values stored in float32, A read as float32, every
                               sum accumulated in float64                          */
  int symmetrize;           /* 1: M := (M + M^T) / 2 before dropping (Appendix A
                               step 1), default 1                                  */
  double drop_tol;          /* u of Appendix A step 2: off-diagonal |m| < u of M is
                               dropped; default 2^-53; 0 disables                 */
  double tie_eta;           /* tie band of the cap, default 1e-9                  */
  void* stream;             /* hipStream_t, default NULL                           */
  int64_t device_pool_limit;/* bytes; 0 = no limit.  Exceeding it at create time
                               returns SPAI_ERR_NOMEM                             */
  int profile;              /* 1: time every phase of an iteration with HIP events
                               on the handle's stream (see spai_profile), default 0 */
  int a_format;             /* SPAI_AFMT_*, default SPAI_AFMT_AUTO                 */
  int jacobi;               /* 1: the Pi-weighted variants of Section 5 with
                               Pi = D_A^{-1} (MR: Algorithm 5, CG: Algorithm 7,
                               LOMR: Algorithm 8); the direction lists hold
                               Z = Pi R; default 0                                 */
  int explicit_residual;    /* 1 (default): R_{i+1} = I - A M_{i+1} after every
                               update (Section 6.2).  0: the update formulas of
                               Algorithms 1, 3, 4 (and 5, 7, 8), R_{i+1} = R_i -
                               alpha A R_i (MR), R_i - alpha A P_i (CG),
                               R_i - A P_i (LOMR); valid only without dropping, so
                               it requires SPAI_CAP_NONE, drop_tol = 0 and
                               symmetrize = 0 (else SPAI_ERR_ARG); not for batched
                               handles                                             */
  int drop_score;           /* 1: the global cap of M ranks its candidates by the
                               heuristic of Appendix A instead of by magnitude: with
                               M~ the symmetrized, small-dropped candidates and
                               R~ = I - A M~, s_kl = m_kl^2 ||A e_k||^2 +
                               2 m_kl (A R~)_kl is the change of ||R~||_F^2 from
                               dropping m_kl alone; off-diagonal entries are kept or
                               dropped in symmetric pairs ranked by s_kl + s_lk
                               (keep score > t + tie_eta |t|, t the (b+1)-th largest).
                               P keeps hard thresholding.  Requires SPAI_CAP_GLOBAL
                               and symmetrize = 1; default 0                      */
  double floor_frac;        /* global cap on magnitudes, one matrix: the update
                               writes only the candidates (off-diagonal ones for M)
                               with |x| >= floor_frac times the previous iteration's
                               cut t, and counts the others; when this iteration's
                               cut does not clear the floor by the tie factor
                               (t (1 - tie_eta) < floor) or there is no cut while
                               candidates were left out, the update and the
                               selection run again without the floor.  The kept
                               sets, values and drop records are those without a
                               floor; only the candidate traffic changes.  >= 0,
                               0 disables; default 0.75                           */
} spai_opts_t;

/* Fill *opts with the defaults. */
void spai_default_opts(spai_opts_t* opts);

/*
 * spai_create — validate A, upload it, and form the initial iterate
 *   M_0 = (tr A / tr A^2) I  and  R_0 = I - A M_0 (Algorithms 1, 3, 4, first line;
 *   the paper leaves M_0 open, this is the Frobenius-optimal multiple of I).
 *   CG also forms P_0 = D_P(R_0); LOMR sets P_{-1} = 0.
 * method: SPAI_MR, SPAI_CG or SPAI_LOMR.
 * max_iter: upper bound on the total iterations this handle will run (sizes the
 *   residual history); must be >= 0.
 * tol: stop when ||I - A M_i||_F / sqrt(n) <= tol (0 disables the test).
 * out: receives the new handle; on error *out is left NULL.
 * Errors: SPAI_ERR_ARG (n < 1, null pointers, method, cap below the diagonal
 *   count for M, cap mode other than NONE with value <= 0), SPAI_ERR_NOT_SYMMETRIC,
 *   SPAI_ERR_NOT_SPD, SPAI_ERR_NONFINITE, SPAI_ERR_NOMEM, SPAI_ERR_HIP.
 * The handle owns every device buffer; release it with spai_destroy.
 */
int spai_create(const spai_csr_t* A, int method, spai_cap_t cap, int max_iter,
                double tol, const spai_opts_t* opts, spai_handle_t** out);

/*
 * spai_iterate — run up to n_iter further iterations of the handle's method, each
 *   SpGEMM + Frobenius dots -> step sizes -> merge (SpGEAM) -> drop rule -> explicit
 *   residual R = I - A M with ||R||_F, all on the device with no host round trip.
 * iters_done (may be NULL): iterations actually run in this call.
 * resid_hist (may be NULL): host array of n_iter doubles; entry t receives
 *   ||I - A M||_F after the t-th iteration of this call (entries past iters_done
 *   are left untouched).
 * Returns SPAI_OK (all n_iter ran), SPAI_CONVERGED, SPAI_BREAKDOWN, or an error.
 * Iterating past max_iter total iterations returns SPAI_ERR_ARG.
 * Synchronises the stream once at the end.
 */
int spai_iterate(spai_handle_t* h, int n_iter, int* iters_done, double* resid_hist);

/* Output CSR buffers for spai_get (caller-allocated). */
typedef struct {
  int64_t n;
  int64_t nnz;        /* set by spai_get: number of stored entries of M         */
  int64_t capacity;   /* entries the colind / val arrays can hold               */
  int64_t* rowptr;    /* [n + 1]                                                */
  int32_t* colind;    /* [capacity]                                             */
  double* val;        /* [capacity] (float32 iterates are widened exactly)      */
  int on_device;      /* 1: the arrays are device pointers; 0: host             */
} spai_csr_out_t;

/*
 * spai_get — export the current iterate M as CSR (rows sorted, no stored zeros).
 *   Two-call protocol: with rowptr == NULL (or capacity too small) only M->nnz is
 *   set and SPAI_OK / SPAI_ERR_ARG returned respectively; then call again with
 *   buffers.  Synchronises the stream.
 */
int spai_get(spai_handle_t* h, spai_csr_out_t* M);

/*
 * spai_stats — scalar state: iterations run so far, ||I - A M||_F, nnz(M), nnz(P)
 *   and the last step sizes (MR: alpha; CG: alpha, beta; LOMR: delta, gamma) and
 *   LOMR's count of degenerate steps taken as MR steps.  Any pointer may be NULL.
 */
int spai_stats(spai_handle_t* h, int* iters, double* resid_fro, int64_t* nnz_m,
               int64_t* nnz_p, double* step1, double* step2, int* mr_fallbacks);

/*
 * spai_history — the per-iteration record of the drop rule (the columns of the paper's
 *   Tables 4-6 and of a run's metrics log), for the iterations run since spai_create or
 *   spai_reset (after spai_set_state the record resumes at the restored iteration; the
 *   earlier rows read zero).  rec: 6 int64 per iteration i (0-based), row-major:
 *   nnz(M_{i+1}); the candidates of M_{i+1} the cap dropped (after symmetrization and the
 *   small-entry drop, Appendix A steps 1-2); of those, the ones in the tie band of the cut
 *   (magnitude, or score, at least t - tie_eta |t| for the (b+1)-th largest value t of
 *   Section 6.1's hard thresholding, or the column threshold under a column cap); then
 *   the same three for the direction P_i (zero for MR).
 *   Counts are totals over the matrices of a batched handle.  Fills min(cap, *count)
 *   rows; *count receives the number of iterations recorded.  Synchronises the stream.
 */
int spai_history(spai_handle_t* h, int64_t* rec, int cap, int* count);

/* Release every device buffer of the handle.  NULL is accepted. */
int spai_destroy(spai_handle_t* h);

/*
 * spai_reset — restart the handle from M_0 = (tr A / tr A^2) I (and R_0, P_0) with
 *   the same A, method, cap and options, reusing its device pools; the iteration
 *   budget max_iter starts again.  Synchronises the stream.
 */
int spai_reset(spai_handle_t* h);

/*
 * spai_pcg — pcg_solve with the handle's own A and its current iterate M, both
 *   already in device memory (no copy, no conversion).  Requires symmetrize = 1 (M
 *   exactly symmetric, so its column storage is also its row storage).  B, X: dense
 *   n x nrhs row-major float64, device pointers when on_device = 1, else host.
 *   For a batched handle the block-diagonal system is solved.  Returns as pcg_solve.
 *   The handle keeps the solve's device blocks (those pcg_solve allocates per call) for
 *   the next spai_pcg with the same nrhs; one with another nrhs replaces them, and
 *   spai_destroy frees them.
 */
int spai_pcg(spai_handle_t* h, int nrhs, const double* B, double* X, double rtol,
             int max_iter, int* iters, double* relres, int on_device);

/*
 * spai_spectrum — extreme eigenvalues of the handle's current iterate M (the
 *   lambda_min / lambda_max the paper reports for its SPAIs, Tables 4-6; M is
 *   positive definite iff lambda_min > 0, Section 7.1), estimated by `steps` steps
 *   (1..2048; clamped to n) of the Lanczos process with full reorthogonalisation
 *   from the start vector v0 (n float64, device when on_device = 1, else host; not
 *   all zero; the caller draws it, e.g. at random).  The process stops early when
 *   an invariant subspace is found (the Ritz values are then eigenvalues).
 * out (host, 4 doubles): theta_min, theta_max (extreme Ritz values; lambda_min <=
 *   theta_min, theta_max <= lambda_max), and res_min, res_max: each Ritz value is
 *   within res of an eigenvalue of M.  *steps_done (may be NULL): steps taken.
 *   Requires symmetrize = 1.  Allocates n (steps + 1) doubles for the basis for the
 *   duration of the call.  Synchronises the stream.
 */
int spai_spectrum(spai_handle_t* h, int steps, const double* v0, int on_device, double* out,
                  int* steps_done);

/*
 * spai_autotune — pick the per-column tiles (the boundary between a kernel's LDS tiers)
 *   for this handle's workload: restart from M_0, run warm_iters iterations (at most
 *   max_iter), time every candidate small tile of the residual, dots and update kernels
 *   on that state (best of reps launches each), keep the fastest where it beats the
 *   handle's current tile by at least 3% (else the current one), and restart from M_0
 *   (as spai_reset).  Results do not depend on the tiles (every column's arithmetic
 *   and summation order are the same in every tier); batched handles recapture their
 *   graph.  The dots and update kernels' resident tiers are also timed with their
 *   registers capped at five waves per SIMD (faster where columns are small).  chosen
 *   (may be NULL): 8 ints, L and H of the residual, dots and update tiles, then the
 *   update's and the dots' resident-tier variant (0: the compiler's registers, 5: capped
 *   at five waves per SIMD, 1: the lean tier for A in ELL); best_ms (may be NULL): 3
 *   doubles, their measured launch times.
 *   Synchronises the stream.
 */
int spai_autotune(spai_handle_t* h, int warm_iters, int reps, int* chosen, double* best_ms);

/*
 * spai_set_tiles — use the given per-column tiles from the next launch on, for
 *   instance those a previous spai_autotune reported for the same workload.  tiles:
 *   8 host ints in the layout of spai_autotune's chosen.  Accepted: every H a power of
 *   two >= 512 (>= 128 for the residual when A is held in ELL, and for the dots' lean
 *   tier); the residual and dots L a power of
 *   two >= 32, the update L >= 32; the dots' and the update's variant 0 (compiler's
 *   registers), 5 (capped at five waves per SIMD) or 1 (the lean tier: A in ELL; the
 *   update's H may then be >= 128); each tile within 64 KB
 *   of LDS.  Anything else returns
 *   SPAI_ERR_ARG and leaves the tiles unchanged.  Results do not depend on the tiles;
 *   a batched handle recaptures its graph.  Synchronises the stream.
 */
int spai_set_tiles(spai_handle_t* h, const int* tiles);

/*
 * spai_get_state / spai_set_state — checkpoint and resume a handle.  The state holds the
 *   current iterate M, for CG and LOMR the direction P (and its transpose P^T), the
 *   residual R (and, for the implicit Pi-weighted form, R beside Z), every matrix's
 *   scalars (step sizes, ||R||^2, (R, Z), iteration count, stop flag) and the iteration
 *   budget used, as one self-describing host buffer (lists as compact CSC).
 *   spai_get_state: buf = NULL returns the size in *size; else *size is the capacity
 *   of buf on entry and the bytes written on return.
 *   spai_set_state: restores a state taken from a handle of the same problem and
 *   configuration (n, matrices, method, precision, Pi weighting, residual form,
 *   symmetrization); the next spai_iterate continues exactly as the original handle
 *   would have.  A mismatch, a truncated buffer, lists larger than this handle's pools,
 *   column pointers that do not start at 0 or decrease, rows out of range or not
 *   strictly ascending within a column return SPAI_ERR_ARG; every list is checked
 *   before any is uploaded, so the handle is unchanged on error.  Both synchronise the
 *   stream.
 */
int spai_get_state(spai_handle_t* h, void* buf, size_t* size);
int spai_set_state(spai_handle_t* h, const void* buf, size_t size);

/*
 * spai_csr_spectrum — the same for an exactly symmetric CSR matrix S (for instance
 *   A, or an exported M); v0 is on the device when S->on_device.  Returns
 *   SPAI_ERR_NOT_SYMMETRIC for a matrix that is not exactly symmetric.
 */
int spai_csr_spectrum(const spai_csr_t* S, int steps, const double* v0, double* out,
                      int* steps_done, const spai_opts_t* opts);

/* Phases timed when opts.profile = 1, and traffic counters (cumulative since create). */
enum {
  SPAI_PH_DOTS = 0,     /* SpGEMM fused with the Frobenius dots (A R, A P)          */
  SPAI_PH_UPDATE = 1,   /* merge + symmetrize + small-entry drop (+ column thresholds) */
  SPAI_PH_RESID = 2,    /* explicit residual R = I - A M with ||R||_F               */
  SPAI_PH_SELECT = 3,   /* global-cap radix selection                               */
  SPAI_PH_COMPACT = 4,  /* keep rule and in-place compaction                        */
  SPAI_PH_BOUNDS = 5,   /* per-column output bounds and their prefix sums           */
  SPAI_PH_SCALAR = 6,   /* fixed-order reductions and step sizes                    */
  SPAI_PH_PCG = 7,      /* spai_pcg                                                 */
  SPAI_PH_PCG_AX = 8,   /* inside spai_pcg: the products q = A p (part of SPAI_PH_PCG) */
  SPAI_PH_PCG_MX = 9,   /* inside spai_pcg: the products z = M r (part of SPAI_PH_PCG) */
  SPAI_NPHASES = 10
};
enum {
  SPAI_CNT_CAND_M = 0, SPAI_CNT_CAND_P = 1, SPAI_CNT_CAND_PT = 2,   /* candidates formed */
  SPAI_CNT_KEPT_M = 3, SPAI_CNT_KEPT_P = 4, SPAI_CNT_KEPT_PT = 5,   /* entries kept      */
  SPAI_CNT_RESID = 6,   /* residual entries written                                  */
  SPAI_CNT_ITERS = 7,   /* iterations run                                            */
  SPAI_NCOUNTS = 8
};
/*
 * spai_profile — accumulated milliseconds and launch counts per phase (zeros unless
 *   opts.profile = 1) and the traffic counters.  Any pointer may be NULL; arrays
 *   hold SPAI_NPHASES / SPAI_NCOUNTS entries.  The PCG product counts are the products
 *   that did their work: once every right-hand side has stopped, the products left in
 *   the last 8-iteration chunk return at once (their few microseconds stay in the
 *   times).  Synchronises the stream.
 */
int spai_profile(spai_handle_t* h, double* phase_ms, int64_t* phase_calls, int64_t* counts);

/*
 * pcg_solve — preconditioned CG for A X = B with the SPAI M as preconditioner
 *   (z = M r), one independent recurrence per right-hand side, all in float64,
 *   x_0 = 0, stopping when ||r||_2 <= rtol ||b||_2 on the recursively updated
 *   residual (the vector solves of Section 7, Experiments 04 and 06).
 * A, M: CSR as above; M need not be symmetric but must be square of the same n.
 * B, X: dense n x nrhs, row-major (the nrhs values of one row are contiguous),
 *   float64, device pointers when A->on_device, else host.  X is overwritten.
 * iters, relres (may be NULL): host arrays of nrhs: iterations taken, and the
 *   true relative residual ||b - A x||_2 / ||b||_2 at exit.
 * Returns SPAI_OK when every RHS converged, SPAI_MAXITER when some did not,
 *   PCG_INDEFINITE when some RHS met (r, z) <= 0 or (p, A p) <= 0, or an error.
 * On a stream other than the null stream the iterations run as replays of one HIP
 *   graph of 8 iterations (captured on first use; the host reads the count of active
 *   right-hand sides between replays); results equal the eager launches bit for bit.
 * Device memory for the solve: n x nrhs float64 blocks r, z, q and p, and for nrhs <= 64
 *   a second p (x is then updated once per two iterations, with the same sums), plus
 *   per-workgroup partials; all released before the call returns.
 * Synchronises the stream.
 */
int pcg_solve(const spai_csr_t* A, const spai_csr_t* M, int nrhs, const double* B,
              double* X, double rtol, int max_iter, int* iters, double* relres,
              const spai_opts_t* opts);

/*
 * spai_loss_fwd — f(M) = ||I - A M||_F^2 (Section 2) for CSR A and M of the same n,
 *   without storing A M.  Values are read as float32 when opts->precision is
 *   SPAI_PREC_MIXED, else float64; the sum is float64.  *L is a host double.
 */
int spai_loss_fwd(const spai_csr_t* A, const spai_csr_t* M, double* L,
                  const spai_opts_t* opts);

/*
 * spai_loss_fwd_noalloc — spai_loss_fwd for callers that cannot allocate memory (code
 *   under HIP graph capture, tight serving loops, harnesses that forbid allocation):
 *   the same kernels and summation order, so *L equals spai_loss_fwd's value bitwise,
 *   but nothing is allocated, nothing is copied to the host and the stream is not
 *   synchronised.  A and M: CSR on the device (on_device = 1), float64 values, at most
 *   2^21 rows.  L: one device double, receives f(M); err: one device int, set to 0,
 *   and nonzero when the call is complete if a row or column exceeded the per-column
 *   tile (L is then not valid).  The per-row partial sums live in a fixed device array
 *   of this library (2^21 + 512 doubles, about 16 MB per GPU, held until the process
 *   ends) shared by every call on that GPU: calls that overlap on one GPU race and must
 *   be ordered by the caller (one stream, or events).  Work is enqueued on
 *   opts->stream.  Returns SPAI_ERR_ARG, without launching anything, for null
 *   pointers, unequal or empty shapes, host matrices, more than 2^21 rows, or
 *   opts->precision other than SPAI_PREC_F64.
 */
int spai_loss_fwd_noalloc(const spai_csr_t* A, const spai_csr_t* M, double* L, int* err,
                          const spai_opts_t* opts);

/*
 * spai_loss_bwd — gradients of f in the stored values of A and of M:
 *   gA = dL * (-2 R M^T) on the pattern of A, gM = dL * (-2 A^T R) on the pattern
 *   of M, R = I - A M recomputed per column (for symmetric A, gM is the gradient
 *   -2 A R of Section 2).  gA, gM: arrays of nnz(A), nnz(M) doubles in the CSR
 *   order of A and M, on the device when A->on_device.  Either may be NULL.
 *   The patterns of A and M must be symmetric (values need not be).
 */
int spai_loss_bwd(const spai_csr_t* A, const spai_csr_t* M, double dL, double* gA,
                  double* gM, const spai_opts_t* opts);

/*
 * spai_create_batched — many independent SPD matrices treated as one
 *   block-diagonal problem: one launch per step covers every matrix, while the
 *   Frobenius dots, step sizes, stopping test and residual history are kept per
 *   matrix.  As_host: array of nb CSR descriptors (all host or all device).
 *   Only SPAI_CAP_NONE and SPAI_CAP_COLUMN are accepted (a column cap involves no
 *   cross-matrix selection).  The iteration sequence is captured once in a HIP
 *   graph and replayed by spai_iterate.  spai_get on a batched handle returns
 *   the block-diagonal M; spai_batched_resid returns ||I - A_b M_b||_F per matrix.
 */
int spai_create_batched(const spai_csr_t* As, int nb, int method, spai_cap_t cap,
                        int max_iter, double tol, const spai_opts_t* opts,
                        spai_handle_t** out);
int spai_batched_resid(spai_handle_t* h, double* resid /* [nb], host */);

/* Message of the last error on the calling thread ("" if none). */
const char* spai_last_error(void);
/* Static name of a status code. */
const char* spai_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* SPAI_H */

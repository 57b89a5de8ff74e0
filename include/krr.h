/*
 * krr.h -- C ABI of a gfx950 (MI355X) library for kernel ridge regression
 * solved by preconditioned conjugate gradient, following Diaz, Epperly,
 * Frangella, Tropp & Webber, "Robust, randomized preconditioning for kernel
 * ridge regression" (arXiv 2304.12465).
 *
 * Conventions, for every entry point:
 *  - Array arguments are DEVICE pointers unless the comment says "host".
 *    Matrices are row-major and densely packed: a point set X with N points
 *    of dimension d is N x d (point i is X[i*d .. i*d+d)); a block of m
 *    vectors V of length n is n x m (vector c is the strided column V[i*m+c]).
 *  - The caller owns every array it passes in and every output buffer.
 *  - Device memory the library needs beyond inputs and outputs comes from a
 *    caller-allocated workspace `ws` of `ws_bytes` bytes (any alignment >= 256
 *    bytes); the matching *_ws query returns the bytes needed, which is also
 *    the HBM footprint of that object.  The library itself never allocates
 *    device memory.
 *  - Work is enqueued on `stream` (a hipStream_t; 0 is the null stream).
 *    Calls return after enqueueing unless the comment says they synchronise.
 *  - Return value: 0 = success, 1 = KRR_NOT_CONVERGED (a warning: outputs hold
 *    the last iterate), a negative KRR_E* code on error.  Errors are reported,
 *    never thrown; krr_last_error() describes the last failure on the calling
 *    thread.  Shapes and parameters are validated before anything is
 *    launched.
 */
#ifndef KRR_H
#define KRR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KRR_OK = 0,
  KRR_NOT_CONVERGED = 1,
  KRR_EINVAL = -1,      /* invalid shape or parameter */
  KRR_EWORKSPACE = -2,  /* workspace too small (or NULL) */
  KRR_ENOTSPD = -3,     /* Cholesky breakdown of a matrix that should be SPD */
  KRR_ENAN = -4,        /* NaN or Inf in a residual */
  KRR_EHIP = -5         /* a HIP runtime call failed */
};

/* Kernel functions.  Gaussian (squared exponential, Sec. 2.1.2):
 *   K(x,y) = exp(-||x-y||^2 / (2 sigma^2)).
 * l1 Laplace (Sec. 4.1):
 *   K(x,y) = exp(-||x-y||_1 / sigma).                                      */
typedef enum { KRR_GAUSSIAN = 0, KRR_LAPLACE = 1 } krr_kernel_kind;

/* Arithmetic of the kernel tiles.  FP64: entries and sums in FP64.
 * FP32: entries in FP32, sums over at most 256 columns in FP32, then FP64.
 * MIXED: the Gaussian distance contraction on bf16 MFMA with a hi/lo split
 * (three products), exp and in-tile sums in FP32, cross-tile sums in FP64;
 * Laplace tiles under MIXED use the FP32 arithmetic.  Vectors of the CG
 * recurrences and all CG scalars stay FP64 in every mode.                   */
typedef enum { KRR_FP64 = 0, KRR_FP32 = 1, KRR_MIXED = 2 } krr_precision;

/* Human-readable description of the last failure on this thread. */
const char* krr_last_error(void);

/* ---------------------------------------------------------------------
 * Matrix-free kernel product (Alg. 1 "Product"; Sec. 4.1 blockwise scheme):
 *   W[nr x m] = K(Xr, Xc) V[nc x m] + shift * V.
 * Xr (nr x d) and Xc (nc x d) are FP64 points; V is FP64 nc x m; W is FP64
 * nr x m and must not overlap V.  The kernel matrix is never stored: every
 * entry is recomputed in registers and reduced against V at once.
 * shift != 0 requires nr == nc (the caller passes the same point set).
 * Limits: 1 <= d <= 64, 1 <= m <= 64, nr, nc >= 0 (nr == 0 is a no-op;
 * nc == 0 gives W = 0 + shift V), sigma > 0.
 * The reduction order is fixed, so results are bitwise reproducible.      */
int krr_kernel_matvec_ws(krr_precision prec, int64_t nr, int64_t nc, int32_t d, int32_t m,
                         size_t* bytes);
int krr_kernel_matvec(krr_kernel_kind kind, double sigma, krr_precision prec,
                      const double* Xr, int64_t nr, const double* Xc, int64_t nc, int32_t d,
                      const double* V, int32_t m, double shift, double* W,
                      void* ws, size_t ws_bytes, hipStream_t stream);


/* The same product for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument; the point layouts and partial sums live
 * in a fixed scratch array of 256 MiB that the library keeps in device
 * memory, one per GPU, for the life of the process.  The call performs no
 * hipMalloc, hipFree or other allocation (tile timing, when enabled with
 * krr_timing_enable, creates HIP events: leave it off in such callers).
 * Arguments, layouts, limits and results are those of krr_kernel_matvec
 * (bitwise the same output).  A product whose krr_kernel_matvec_ws size
 * exceeds 256 MiB returns KRR_EWORKSPACE before any launch.  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (on different
 * streams, or from different threads) race and must be serialised by the
 * caller; the array keeps the last call's contents, none of which a later
 * call reads.                                                             */
int krr_kernel_matvec_noalloc(krr_kernel_kind kind, double sigma, krr_precision prec,
                              const double* Xr, int64_t nr, const double* Xc, int64_t nc,
                              int32_t d, const double* V, int32_t m, double shift, double* W,
                              hipStream_t stream);

/* Timing of the fused product tiles (the dominant kernel): when enabled,
 * every tile launch is bracketed by HIP events recorded on the stream it
 * runs on.  krr_timing_read waits for the recorded launches, returns their
 * summed duration (ms) and count, and clears the record.                   */
int krr_timing_enable(int on);
int krr_timing_read(double* total_ms, int64_t* launches);
/* As krr_timing_read, and also the summed duration and count of the launches
 * whose FP64 / FP32 Gaussian matrix-core tile carries `vectors` (1, 2, 4 or
 * 8) right-hand-side vectors (0: the form for 9-16 vectors, which reduces
 * them on the matrix cores).  Launches of other tiles match no `vectors`.
 * Returns KRR_EINVAL for vectors < 0.                                      */
int krr_timing_read_vectors(int32_t vectors, double* total_ms, int64_t* launches,
                            double* match_ms, int64_t* match_launches);

/* ---------------------------------------------------------------------
 * Preconditioned solves.  A krr_precond is an opaque host object holding
 * device pointers into the caller's workspace; it owns neither the points X
 * (which must stay alive and unchanged while it is used) nor the workspace.
 * One precond runs one solve at a time; calls on different preconds may
 * run concurrently on different streams.                                   */
typedef struct krr_precond_s* krr_precond;

typedef struct {
  int32_t iters;            /* PCG iterations (max over right-hand sides) */
  int32_t converged_cols;   /* columns that met tol (see krr_pcg_solve) */
  double relres_recursive;  /* max over columns of ||r_t|| / ||b|| (recurrence) */
  double relres_true;       /* max over columns of ||b - M x|| / ||b||, FP64 product */
  double build_seconds;     /* wall time of the preconditioner build */
  double solve_seconds;     /* wall time of this solve */
  double* history;          /* host, optional: max relative residual per iteration */
  int32_t history_cap;      /* capacity of history (in entries) */
  int32_t history_len;      /* entries written */
  int32_t products;         /* system-operator applications: one per PCG step
                               plus one per FP64 true-residual check that
                               was not carried by a step (see krr_pcg_solve) */
} krr_solve_info;

/* Full-data KRR (eq. exact_eqn): (A + mu I) beta = y with A_ij = K(x_i, x_j),
 * preconditioned by P = F F^T + mu I where F (N x rank) comes from blocked
 * RPCholesky (Appendix A, Alg. 3) with block size B; B = 0 selects
 * min(100, ceil(r/10)) (Alg. 1).  Pivots are drawn from the residual
 * diagonal with SplitMix64 keyed by `seed`.  The preconditioner is applied
 * in the Woodbury form (r - Q Q^T r) / mu with Q = F L^{-T}, L L^T =
 * mu I + F^T F, which equals the SVD form of Alg. 1.
 * X: N x d FP64 device points.  1 <= r <= N, 0 <= B <= 128, mu > 0,
 * 1 <= m_max <= 64 (largest number of right-hand sides solved at once).
 * The build synchronises `stream` (pivot draws are read back per block).
 * Returns KRR_ENOTSPD if mu I + F^T F cannot be factored.                  */
int krr_rpchol_ws(krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d, int32_t r,
                  int32_t B, int32_t m_max, size_t* bytes);
int krr_rpchol_build(krr_kernel_kind kind, double sigma, krr_precision prec, const double* X,
                     int64_t N, int32_t d, double mu, int32_t r, int32_t B, uint64_t seed,
                     int32_t m_max, void* ws, size_t ws_bytes, krr_precond* out,
                     hipStream_t stream);
/* Nystrom preconditioner with another pivot rule in the same block loop
 * (Sec. 3.1 sets uniform sampling and greedy selection against RPCholesky):
 *   KRR_PIVOT_RPCHOL   draws ~ residual diagonal (krr_rpchol_build);
 *   KRR_PIVOT_UNIFORM  per block, B i.i.d. draws uniform over the indices
 *                      never drawn before (same prefix rule and random
 *                      stream, on 0/1 weights); r counts the distinct
 *                      indices drawn, dependent ones are dropped, so the
 *                      rank can end below r;
 *   KRR_PIVOT_GREEDY   one pivot per block (B ignored): the largest residual
 *                      diagonal entry, smallest index among equal maxima;
 *                      stops when it is <= eps tr(A).
 * Arguments, workspace (krr_rpchol_ws with the same shape covers every
 * rule), ownership and errors as krr_rpchol_build; KRR_EINVAL for an
 * unknown rule.                                                            */
typedef enum { KRR_PIVOT_RPCHOL = 0, KRR_PIVOT_UNIFORM = 1, KRR_PIVOT_GREEDY = 2 } krr_pivot_rule;
int krr_nystrom_build(krr_kernel_kind kind, double sigma, krr_precision prec, const double* X,
                      int64_t N, int32_t d, double mu, int32_t r, int32_t B, uint64_t seed,
                      krr_pivot_rule rule, int32_t m_max, void* ws, size_t ws_bytes,
                      krr_precond* out, hipStream_t stream);
/* F^T (rank x N, row-major, device) of the RPCholesky factor, recomputed as
 * L Q^T into the caller's buffer.                                          */
int krr_rpchol_factor(krr_precond P, double* FT, hipStream_t stream);

/* Restricted KRR (Sec. 2.2, eq. restricted_krr_eqn):
 *   [A(S,:) A(:,S) + mu A(S,S)] beta = A(S,:) y
 * with KRILL preconditioning (Alg. 2): H = mu A(S,S) + N eps tr(A(S,S)) I
 * (eps = 2^-52), a sparse sign embedding Phi with `sketch_rows` rows
 * (0 -> 2k) and `zeta` nonzeros per column (0 -> ceil(ln(k+1))),
 * B = Phi A(:,S), P = B^T B + H = C^T C.  PCG runs on the shifted system
 * (H in place of mu A(S,S)); the right-hand side A(S,:) y is formed in FP64.
 * `centers`: device int64[k] of distinct indices in [0, N), or NULL to draw
 * k centres uniformly without replacement with SplitMix64 keyed by `seed`.
 * Limits: 1 <= k <= min(N, 65536), 1 <= zeta <= sketch_rows.  `prec`:
 * KRR_FP64 or KRR_FP32 tiles for the sketch and the restricted products;
 * KRR_MIXED = FP64 restricted products (and FP64 right-hand side and
 * checks, as KRR_FP64) with the sketch B on FP32 tiles (the workspace then
 * also holds FP32 copies of X and the centres): B carries the FP32 tiles'
 * entry error (2e-5 of |Phi||A(:,S)| at most), which changes only the
 * preconditioner, not the system solved.
 * The build synchronises `stream`.  Returns KRR_ENOTSPD if P cannot be
 * factored.                                                                */
int krr_krill_ws(krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d, int32_t k,
                 int32_t sketch_rows, int32_t zeta, int32_t m_max, size_t* bytes);
int krr_krill_build(krr_kernel_kind kind, double sigma, krr_precision prec, const double* X,
                    int64_t N, int32_t d, double mu, const int64_t* centers, int32_t k,
                    int32_t sketch_rows, int32_t zeta, uint64_t seed, int32_t m_max, void* ws,
                    size_t ws_bytes, krr_precond* out, hipStream_t stream);
/* The same KRILL preconditioner with the N x k kernel block A(:,S) stored
 * (Sec. 4.1 keeps it in memory): as krr_krill_build, and in addition A(:,S)
 * is evaluated once by the build into the workspace, in FP64 (prec =
 * KRR_FP64, 8 N k bytes) or FP32 (KRR_FP32, 4 N k bytes; rows padded to a
 * multiple of 8 entries), by the same Gaussian tiles the recomputing
 * products use when their expansion guard admits the problem (entries as
 * those products evaluate them), else by direct differences.  Every later
 * application of the restricted
 * operator (krr_pcg_solve, the stepped solves, krr_precond_operator) then
 * streams the stored block instead of recomputing its entries: with one
 * right-hand side one pass over it forms A(S,:)(A(:,S) v), otherwise two.
 * The FP64 block also serves the right-hand side and the FP64 residual
 * checks; with the FP32 block those use recomputed FP64 entries.  The
 * sketch B = Phi A(:,S) recomputes its entries as in krr_krill_build.
 * Arguments, limits, ownership and errors as krr_krill_build;
 * krr_krill_stored_ws gives the workspace size.                            */
int krr_krill_stored_ws(krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d,
                        int32_t k, int32_t sketch_rows, int32_t zeta, int32_t m_max,
                        size_t* bytes);
int krr_krill_build_stored(krr_kernel_kind kind, double sigma, krr_precision prec,
                           const double* X, int64_t N, int32_t d, double mu,
                           const int64_t* centers, int32_t k, int32_t sketch_rows, int32_t zeta,
                           uint64_t seed, int32_t m_max, void* ws, size_t ws_bytes,
                           krr_precond* out, hipStream_t stream);
/* Direct solve of the restricted system (Sec. 2.2, eq. restricted_krr_eqn)
 * with the shifted regulariser of Alg. 2, for comparison with KRILL
 * (Sec. 4.2): M = A(S,:) A(:,S) + mu A(S,S) + N eps tr(A(S,S)) I is formed
 * in FP64 over row blocks of K(X, S) (O(N k^2) flops), factored M = L L^T,
 * and beta = L^{-T} L^{-1} A(S,:) y.  X: N x d FP64 device points;
 * `centers`: device int64[k] in [0, N) (checked); Y: N x m FP64 device,
 * row-major; beta: k x m FP64 device, row-major.  1 <= k <= min(N, 32768),
 * 1 <= m <= 64, mu > 0.  Workspace: krr_restricted_direct_ws (about
 * 2 k^2 + min(N, 2^27 / k) k doubles plus the point layouts).  Synchronises
 * `stream`; KRR_ENOTSPD if M cannot be factored.                           */
int krr_restricted_direct_ws(krr_kernel_kind kind, int64_t N, int32_t d, int32_t k, int32_t m,
                             size_t* bytes);
int krr_restricted_direct(krr_kernel_kind kind, double sigma, const double* X, int64_t N,
                          int32_t d, double mu, const int64_t* centers, int32_t k,
                          const double* Y, int32_t m, double* beta, void* ws, size_t ws_bytes,
                          hipStream_t stream);

/* Copies a KRILL build product into a caller device buffer of `bytes`:
 * what = 0: sketch rows, int32 N x zeta (column j's rows in draw order);
 * 1: sketch signs, int32 N x zeta (+1 / -1); 2: B, FP64 sketch_rows x k;
 * 3: H, FP64 k x k; 4: the lower factor L = C^T of P, FP64 k x k (strict
 * upper triangle zero); 5 (stored builds only): A(:,S) as FP64 N x k.     */
int krr_krill_export(krr_precond P, int32_t what, void* dst, size_t bytes, hipStream_t stream);

/* Number of pivots / centres (RPCholesky: accepted pivots, may be < r when
 * the residual is exhausted; KRILL: k) and the system size n (N or k).     */
int krr_precond_dims(krr_precond P, int32_t* rank, int64_t* n);
/* Host copy of the pivot indices in selection order (RPCholesky) or of the
 * centres in ascending order (KRILL); at most `cap` entries.              */
int krr_precond_pivots(krr_precond P, int64_t* host_out, int32_t cap, int32_t* count);
/* OUT = P^{-1} Z for n x m row-major device blocks (m <= m_max).           */
int krr_precond_apply(krr_precond P, const double* Z, int32_t m, double* OUT,
                      hipStream_t stream);
/* OUT = M V with the system operator (full: K V + mu V; restricted:
 * A(S,:)(A(:,S) V) + H V), in the build precision; n x m row-major.        */
int krr_precond_operator(krr_precond P, const double* V, int32_t m, double* OUT,
                         hipStream_t stream);
/* Releases the host object (the workspace stays the caller's).             */
void krr_precond_free(krr_precond P);

/* PCG (Sec. 3, eq. psd_system) from a zero start until every column reaches
 * ||r|| <= tol ||b|| on the recursive residual, or max_iter.  Y is N x m
 * (targets, row-major, device); beta receives n x m (N for full-data, k for
 * restricted).  At exit the true residual is evaluated with an FP64 product.
 * FP64 tiles: one residual-replacement restart if it exceeds 10 tol.  With
 * FP64 tiles, m up to 4, more than 1.6e7 kernel entries per operator
 * application and no stored block, the step whose recursive residual is
 * predicted within 5 tol (and the last step allowed) also multiplies x in
 * the same launches; if it ends the solve, its true residual
 * (b - M x) - alpha (M p) is the exit check and no further product runs.
 * (A KRR_MIXED KRILL build runs FP64 restricted products: the FP64 rules
 * apply.)  FP32 / MIXED tiles: up to 6 rounds of iterative refinement (CG
 * restarted from the FP64 true residual, each round run to tol/10 on its recursive
 * residual, or to tol/2 where the previous round's contraction puts the
 * operator's share of the coming round below tol/10; MIXED full-data rounds
 * also stop at the operator's floor, seen on an FP64 residual of 1,024
 * sampled rows) until it meets tol; relres_true reports the final FP64
 * value.  A column counts as converged when FP64 tiles bring its
 * recursive residual to tol with a true residual within 10 tol, and when
 * FP32 / MIXED tiles bring its FP64 true residual itself to tol.
 * Synchronises `stream` once per iteration.  Returns KRR_NOT_CONVERGED
 * (beta = last iterate) if a column did not converge and KRR_ENAN on a
 * NaN/Inf residual.                                                        */
int krr_pcg_solve(krr_precond P, const double* Y, int32_t m, double tol, int32_t max_iter,
                  double* beta, krr_solve_info* info, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Stepped solves for serving (continuous batching).  A krr_solve is the
 * PCG state of one request (kept in its precond's workspace: one active
 * solve per precond).  krr_solve_step advances n solves by one PCG step
 * each: their direction products share kernel launches (tiles of every
 * product that uses the same kernel instantiation are dealt over one grid),
 * then one host synchronisation serves all of them.  Each product keeps the
 * tile decomposition it has alone, so every result is bitwise identical
 * alone and in any mix.  state (host, n entries) receives 0 = running,
 * 1 = finished, or a negative error of that solve only (the others go on).
 * krr_solve_end writes beta (n x m, row-major) and info, frees the solve
 * and returns what krr_pcg_solve would; krr_solve_free abandons a solve.
 * While a solve is active its precond refuses (KRR_EINVAL) another
 * krr_solve_begin, krr_pcg_solve, krr_precond_apply and
 * krr_precond_operator, which would overwrite its vectors; free the solves
 * of a precond before the precond itself.                                  */
typedef struct krr_solve_s* krr_solve;
int krr_solve_begin(krr_precond P, const double* Y, int32_t m, double tol, int32_t max_iter,
                    krr_solve* out, hipStream_t stream);
int krr_solve_step(krr_solve* solves, int32_t n, int32_t* state, hipStream_t stream);
int krr_solve_end(krr_solve S, double* beta, krr_solve_info* info, hipStream_t stream);
void krr_solve_free(krr_solve S);

/* Out-of-sample prediction with a solved model: the prediction function of
 * full-data KRR (Sec. 2), f(x) = sum_i beta_i K(x_i, x) over the N training
 * points, or of restricted KRR (Sec. 2.2), f(x) = sum_i beta_i K(x_{s_i}, x)
 * over the k centres, in the object's kernel and bandwidth.
 *   X      device, N x d row-major: the training points the object was built
 *          on (the object keeps only packed copies, not X itself)
 *   Xtest  device, ntest x d row-major
 *   beta   device, n x m row-major (n = N full-data, k restricted), e.g. the
 *          output of krr_pcg_solve
 *   out    device, ntest x m row-major: f(Xtest) per right-hand side
 *   prec   precision of the kernel tiles (any of the three, independent of
 *          the build precision); 1 <= m <= 64
 * Workspace: krr_predict_ws; asynchronous on `stream`.  Errors: KRR_EINVAL
 * (shapes, NULL arrays), KRR_EWORKSPACE.                                    */
int krr_predict_ws(krr_precond P, krr_precision prec, int64_t ntest, int32_t m, size_t* bytes);
int krr_predict(krr_precond P, krr_precision prec, const double* X, const double* Xtest,
                int64_t ntest, const double* beta, int32_t m, double* out, void* ws,
                size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* KRR_H */

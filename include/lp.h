/*
 * lp.h -- C ABI of the MI355X (gfx950) dense LU solver library (liblp.so).
 *
 * The library solves dense systems A X = B the way the LINPACK benchmark
 * defines them (paper, section "High Performance Linpack"): A is decomposed
 * into a lower and an upper factor, then L Y = B and U X = Y are solved, and
 * the result is checked with a scaled residual.  The factorization is the
 * blocked right-looking scheme of the paper's "Base Implementation" (figure
 * fig:lu_iteration): per block column, factor the diagonal/panel block,
 * update the blocks to its right with L ("top" blocks), and update the inner
 * blocks with one matrix multiplication; the next block column is factored
 * while the rest of the multiplication still runs (the overlap of the
 * communication and update phases, figure fig:lu_execution_schedule_pcie).
 * Unlike the paper's FPGA design the factorization pivots (partial pivoting);
 * on diagonally dominant input (the HPL-AI rule the paper adopts) the pivot
 * search keeps every diagonal row, so the result is the paper's.
 *
 * Conventions shared by every entry point:
 *   - Matrix pointers are DEVICE pointers (hipMalloc or torch.empty(...,
 *     device='cuda') memory) unless stated otherwise.  Matrices are row-major:
 *     element (i, j) lives at M[i * ld + j], with the leading dimension ld >= the
 *     number of columns (ld >= 1).
 *   - ipiv is 0-based int32 with sequential-swap meaning: at step j, row j was
 *     exchanged with row ipiv[j] >= j.  Pivot choice: the lowest row index
 *     among the largest |a_ij| (a NaN is never chosen unless it sits on the
 *     diagonal).
 *   - The caller owns every buffer, including workspaces; the library allocates
 *     no device memory on these paths (the serving API is the exception and
 *     says so).
 *   - Work is stream-ordered on `stream` (a hipStream_t passed as void*; NULL =
 *     the default stream) and calls return without waiting for the device,
 *     except lu_solve_ir, which must read residuals on the host.
 *   - Return value (synchronous): LP_OK (0); -i when the i-th argument is
 *     illegal (LAPACK style, 1-based); LP_ENOSPC when a workspace is too small;
 *     LP_ENOTSUP for a size/precision combination the kernels do not cover;
 *     LP_EHIP_BASE - e for a HIP runtime error e.  lp_strerror() names them.
 *   - Numerical status is asynchronous, in device memory: *info = 0, or k + 1
 *     for the first exact zero pivot in column k (LAPACK getrf meaning; the
 *     column is then left unscaled and the factorization continues), or
 *     LP_INFO_BARRIER_TIMEOUT if an internal grid barrier gave up waiting
 *     (results are then invalid; this never happens on a healthy device).
 */
#ifndef LP_H_
#define LP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LP_OK 0
#define LP_ENOSPC (-900)
#define LP_ENOTSUP (-901)
#define LP_EHIP_BASE (-1000)
#define LP_INFO_BARRIER_TIMEOUT (-77)

/* Precision of the trailing-matrix update operands.  LP_FP64: everything in
 * binary64 (FP64 MFMA).  LP_FP32: binary32 storage, panel and operands.
 * LP_BF16 / LP_FP16: binary32 storage, panel and triangular solves, but the
 * operands of the inner-block multiplication are rounded to bfloat16 / half
 * (round to nearest even) and accumulated in binary32 on MFMA. */
typedef enum { LP_FP64 = 0, LP_FP32 = 1, LP_BF16 = 2, LP_FP16 = 3 } lp_prec;

/* Text for a return code. Never NULL. */
const char *lp_strerror(int code);

/* Library version (major * 10000 + minor * 100 + patch). */
int lp_version(void);

/* ---------------------------------------------------------------- factor */

/* Bytes of device workspace lu_factor needs for (n, nb, prec).  Host-only,
 * pure function; returns 0 for invalid arguments. */
size_t lu_workspace_bytes(int n, int nb, int prec);

/* In-place LU factorization with partial pivoting, P A = L U (paper, section
 * "High Performance Linpack", blocked right-looking variant of the "Base
 * Implementation").
 *   n     order of A (n >= 0; n <= 131072)
 *   nb    block (panel) width, 1 <= nb <= 1024; the inner multiplication has
 *         depth nb.  n need not be a multiple of nb.
 *   prec  lp_prec: LP_FP64 expects A as double; the others expect A as float.
 *   A     device, n x n row-major, ld lda >= max(1, n); overwritten by L (unit
 *         lower, diagonal not stored) and U.
 *   ipiv  device int32[n]; info device int32[1].
 *   work  device workspace of at least lu_workspace_bytes(n, nb, prec) bytes,
 *         8-byte aligned; its contents on entry do not matter.
 *   stream hipStream_t or NULL.
 * With look-ahead the call uses three internal streams (two for LP_BF16 and
 * LP_FP16) and a few events from process-wide pools (the next panel; the
 * exchanges and "top" solve of the columns right of the next panel, binary64
 * and binary32 only; the exchanges left of the panel) and joins them back
 * into `stream` before returning. */
int lu_factor(int n, int nb, int prec, void *A, int lda, int32_t *ipiv, int32_t *info,
              void *work, size_t work_bytes, void *stream);

/* lu_factor for callers that cannot allocate device memory (code under HIP
 * graph capture, fixed serving loops, harnesses that forbid hipMalloc): the
 * same partial-pivoting factorization, same arguments and results, but the
 * workspace is a file-scope device array of the library
 * (lu_factor_noalloc_max_bytes() = 8 MiB per device, held until the process
 * ends) instead of a caller buffer.  The call itself allocates nothing: no
 * device memory, streams or events; it runs strictly in order on `stream`
 * (no look-ahead).  prec LP_FP64 or LP_FP32 (bfloat16 / half need packed
 * operands: LP_ENOTSUP); LP_ENOSPC when lu_workspace_bytes(n, nb, prec)
 * exceeds the array (it does not for any n <= 131072).  Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (different streams, or several host threads) race and give wrong
 * results; calls in order on one stream are safe.  What must start at zero is
 * cleared by each call. */
size_t lu_factor_noalloc_max_bytes(void);
int lu_factor_noalloc(int n, int nb, int prec, void *A, int lda, int32_t *ipiv, int32_t *info,
                      void *stream);

/* Options and per-phase profile for lu_factor_ex. */
typedef struct {
  int lookahead;  /* 1 (default): factor the next panel on a second stream while the
                     rest of the inner-block update runs; 0: strictly in order */
  int panel_cus;  /* compute units reserved for the panel once it is the longer
                     chain (look-ahead only): 0 (default) never, -1 an eighth of
                     a 256-CU device when n >= 8192, k > 0 k units (a multiple
                     of 8; the CU mask interleaves over the XCDs) */
  int panel_rows; /* panels of at most this many rows use the reserved units;
                     0 (default): min(1024 * panel_cus, 3 n / 4) */
  int no_pivoting;  /* 0 (default): partial pivoting; 1: no row exchanges, as
                       lu_factor_nopiv (panel_cus / panel_rows are then unused) */
  int panel_split_rows; /* with partial pivoting, panels of 256 columns or more and
                           at least this many rows are factored in two halves, the
                           right half updated by one product on the GEMM kernel
                           between them: 0 (default) every such panel of the bfloat16
                           and half factorizations, those of at most 8192 rows in
                           binary64 and binary32; -1 never; k > 0 from k rows */
} lp_factor_opts;

typedef struct {
  int gemm_launches;    /* trailing-update launches                              */
  int panel_launches;   /* panel factorizations                                  */
  double gemm_ms;       /* summed device time of the trailing-update launches    */
  double gemm_flops;    /* their algorithmic flops, 2 M N K per launch           */
  double gemm_bytes;    /* their algorithmic bytes: C read + write and operands  */
  double panel_ms;      /* summed device time of the panel factorizations        */
  double swap_ms;       /* summed device time of the row exchanges right of the
                           panels (the ones the update waits for)                */
  double swap_bytes;    /* their algorithmic bytes (read + write of moved rows)  */
  double trsm_ms;       /* summed device time of the triangular solves           */
  double trsm_flops;    /* their algorithmic flops                               */
  double swap_left_ms;  /* the same for the exchanges left of the panels: with
                           look-ahead they run beside the update, on the compute
                           units it leaves free, and nothing waits for them
                           before the end                                        */
  double swap_left_bytes;
} lp_factor_profile;

/* lu_factor with options (NULL = defaults) and an optional host profile.  When
 * prof != NULL, HIP events bracket every launch group on the stream that runs
 * it and the call synchronizes `stream` before filling *prof. */
int lu_factor_ex(int n, int nb, int prec, void *A, int lda, int32_t *ipiv, int32_t *info,
                 void *work, size_t work_bytes, const lp_factor_opts *opts,
                 lp_factor_profile *prof, void *stream);

/* LU factorization WITHOUT pivoting, A = L U: the paper's own elimination
 * (section "High Performance Linpack": the inputs are made diagonally
 * dominant, the HPL-AI rule, so no pivoting is needed; "Base
 * Implementation", figure fig:lu_iteration).  Per block column of width nb:
 * the nb x nb diagonal block is decomposed in one workgroup with no pivot
 * search (the paper's LU kernel), the blocks below it are solved against its
 * upper triangle, L21 = A21 U11^-1, on the matrix cores (the "left" blocks),
 * the blocks right of it against its unit lower triangle (the "top" blocks),
 * and the inner blocks are updated with one multiplication; the next block
 * column's diagonal and left blocks are factored beside the rest of the
 * multiplication.  No row exchanges run at all.
 * Arguments, layout, workspace (lu_workspace_bytes) and errors as lu_factor;
 * ipiv (device int32[n]) receives the identity so that lu_solve applies
 * unchanged.  *info = k + 1 for the first exact zero pivot u_kk (the factors
 * past it are then not meaningful).  Intended for matrices that need no
 * pivoting (e.g. diagonally dominant); on others the elimination may be
 * unstable, and nothing checks for that. */
int lu_factor_nopiv(int n, int nb, int prec, void *A, int lda, int32_t *ipiv, int32_t *info,
                    void *work, size_t work_bytes, void *stream);

/* ----------------------------------------------------------------- solve */

/* Solve A X = B with the factors from lu_factor: apply the interchanges to B,
 * then L Y = P B (unit lower) and U X = Y (paper: L y = b, then U x = y).
 *   storage  LP_FP64 (LU and B double) or LP_FP32 (LU and B float).
 *   LU, lda, ipiv, info  as written by lu_factor (device).
 *   B     device, n x nrhs row-major, ld ldb >= max(1, nrhs); overwritten by X.
 *   solve_status device int32[1] (may be NULL): set to 0 on success; set to 1
 *         and B left unchanged when *info != 0.
 * Requires no workspace. */
int lu_solve(int n, int storage, const void *LU, int lda, const int32_t *ipiv,
             const int32_t *info, void *B, int ldb, int nrhs, int32_t *solve_status,
             void *stream);

/* lu_solve with a caller workspace: the same result, each triangle solved
 * in one persistent launch (per 8 right-hand sides) instead of one launch
 * pair per 128-row block.  Workgroups take 128-row block rows in the order
 * they start and subtract the tiles of already solved blocks as those
 * appear (published as tagged words in `work`), so the stream of factors
 * overlaps the block-to-block dependency chain.  Arguments as lu_solve, plus
 * work: device scratch of lu_solve_workspace_bytes(n, storage, nrhs) bytes
 * (about 16 n bytes for binary64, 8 n for binary32), 256-byte aligned,
 * contents irrelevant on entry; LP_ENOSPC if smaller.  If an internal wait
 * ever times out (never on a healthy device), *solve_status is set to
 * LP_INFO_BARRIER_TIMEOUT and B is invalid.  The summation order differs from
 * lu_solve's, so results agree to rounding, not bit for bit. */
size_t lu_solve_workspace_bytes(int n, int storage, int nrhs);
int lu_solve_ex(int n, int storage, const void *LU, int lda, const int32_t *ipiv,
                const int32_t *info, void *B, int ldb, int nrhs, int32_t *solve_status,
                void *work, size_t work_bytes, void *stream);

/* -------------------------------------------------------------- residual */

/* The benchmark's residual check in binary64 on the ORIGINAL A and B:
 *   s_c = ||A x_c - b_c||_inf / (eps * (||A||_inf ||x_c||_inf + ||b_c||_inf) * n),
 * eps = 2^-53, per right-hand side c (pass if s_c < 16).  The paper prints a
 * garbled normalised residual; this is the standard HPL form.
 *   A (n x n, lda), X (n x nrhs, ldx), B (n x nrhs, ldb): device, double.
 *   out   device double[5 * nrhs]: {s, ||r||_inf, ||A||_inf, ||x||_inf,
 *         ||b||_inf} per right-hand side.  A NaN input yields NaN s (fails).
 * Deterministic: the same inputs give bitwise the same out. */
int residual_check(int n, const double *A, int lda, const double *X, int ldx,
                   const double *B, int ldb, int nrhs, double *out, void *stream);

/* ------------------------------------------------ mixed precision + IR */

typedef struct {
  int iterations;        /* refinement steps taken (corrections applied)    */
  int converged;         /* 1 if the final scaled residual is < 16          */
  int fell_back;         /* 1 if the FP64 factorization had to be used      */
  int info;              /* info of the low-precision factorization        */
  int fallback_info;     /* info of the FP64 fallback (if it ran)           */
  int history_len;       /* entries used in history                         */
  double scaled_residual;/* final max_c s_c                                 */
  double history[64];    /* max_c s_c after x0 and after each correction    */
  double t_convert_ms, t_factor_ms, t_solve0_ms, t_refine_ms, t_fallback_ms, t_total_ms;
  int gmres_corrections; /* corrections computed by GMRES (of `iterations`)  */
  int gmres_steps;       /* GMRES (Arnoldi) steps over all of them          */
} lp_ir_report;

/* Refinement options of lu_solve_ir_ex. */
typedef struct {
  int max_iter;         /* corrections before giving up (0..62; lu_solve_ir's max_iter) */
  int gmres;            /* 0: classical corrections only; 1 (default): classical, and
                           GMRES corrections from the first classical one that does not
                           cut the scaled residual at least fourfold; 2: GMRES only     */
  int gmres_restart;    /* Krylov vectors before a restart (1..64; default 64)         */
  int gmres_max_inner;  /* GMRES steps per correction (default 64); a GMRES correction
                           that does not halve the scaled residual ends the
                           refinement (binary64 fallback)                             */
  double gmres_tol;     /* stop a correction when the preconditioned residual norm has
                           fallen by this factor (default 1e-10)                        */
  int no_lookahead;     /* 0 (default): the factorizations use look-ahead as lu_factor;
                           1: they run strictly in order on `stream` with no internal
                           streams (what a server running several solves at once wants:
                           fewer streams than hardware queues)                        */
} lp_ir_opts;

/* Bytes of device workspace lu_solve_ir needs. */
size_t lu_solve_ir_workspace_bytes(int n, int nb, int prec, int nrhs);

/* Mixed-precision solve with iterative refinement.  The matrix is copied to
 * binary32, factored with the inner update in `prec` (LP_FP32, LP_BF16 or
 * LP_FP16), and x0 solved from those factors; then, repeatedly,
 * r = B - A x (binary64, original A), d = solve(low-precision factors, r),
 * x += d (binary64) until max_c s_c < 16; from the first correction that does
 * not cut the residual fourfold, d comes from GMRES preconditioned with the
 * factors instead (see lu_solve_ir_ex).  Refinement stops as failed after
 * max_iter corrections, when the residual is not finite, or when it grows two
 * steps in a row; the matrix is then factored in binary64 (workspace reused)
 * and solved directly (fell_back = 1).
 *   A (n x n, lda), B (n x nrhs, ldb): device double, unchanged.
 *   X: device double n x nrhs (ldx), output.
 *   rep: HOST pointer, filled on return.  This call synchronizes `stream`
 *   once per refinement step to read the residual. */
int lu_solve_ir(int n, int nb, int prec, const double *A, int lda, const double *B,
                int ldb, double *X, int ldx, int nrhs, int max_iter, void *work,
                size_t work_bytes, lp_ir_report *rep, void *stream);

/* lu_solve_ir with options (NULL: max_iter 30 and the defaults above).
 * GMRES-based refinement (E. Carson and N. J. Higham, SIAM J. Sci. Comput. 39
 * (2017) and 40 (2018)): the correction equation A d = r is solved by GMRES in
 * binary64 on U^-1 L^-1 P A d = U^-1 L^-1 P r, with the low-precision factors
 * (stored in binary32) applied in binary64 arithmetic as the preconditioner;
 * it converges for conditions kappa(A) well beyond classical refinement's
 * kappa(A) u_f < 1.  Per GMRES step: one product with A (binary64), one
 * preconditioner solve, two classical Gram-Schmidt passes with
 * fixed-order reductions (deterministic), one host synchronization.  The
 * workspace (lu_solve_ir_workspace_bytes) includes the Krylov basis.  Other
 * arguments and the fallback as lu_solve_ir; -11 for invalid options. */
int lu_solve_ir_ex(int n, int nb, int prec, const double *A, int lda, const double *B,
                   int ldb, double *X, int ldx, int nrhs, const lp_ir_opts *opts, void *work,
                   size_t work_bytes, lp_ir_report *rep, void *stream);

/* Refinement decision used by lu_solve_ir, from the scaled-residual history
 * h[0..len) (h[0] after x0, h[k] after the k-th correction): returns 1 when the
 * last value is below 16 (converged), 2 to give up (last value not finite, the
 * last two steps both grew, or corrections == max_iter), 0 to refine again.
 * Host-only, pure. */
int lp_ir_decide(const double *h, int len, int corrections, int max_iter);

/* ---------------------------------------------------------------- serving */
/* A request loop for many independent solves of uneven size (continuous
 * batching).  Each request is solved as lu_factor + lu_solve (LP_FP64) or as
 * lu_solve_ir (binary32 factors + binary64 refinement, LP_FP32/BF16/FP16),
 * and checked with residual_check.  lp_server_create allocates the server's
 * device memory pool (memory_bytes) and its pinned host ring once -- the one
 * allocating call of this library; per-request workspaces come from that
 * pool.  Admission is first come, first served, by device footprint
 * (lp_request_footprint).  Requests with n <= small_n_max are published into
 * a ring of up to max_batch descriptors in pinned host memory; a persistent
 * batched kernel of batch_workgroups workgroups pulls them, one workgroup per
 * request, each request completing on its own (factors held in the
 * workgroup's LDS up to n = 128; for those the low-precision route factors in
 * binary32).  The kernel exits after 2 ms without requests
 * and is launched again when one arrives.  Larger requests run the blocked
 * path on a worker thread and a stream of their own (large_slots at once;
 * 4 is a good value), their factorizations without look-ahead (no internal
 * streams: with several solves in flight the streams would outnumber the
 * hardware queues and wait behind each other).  A result depends only on
 * the request (size, precision, data), never on what else was in flight.
 * Not thread-safe: one thread drives a server.  The caller keeps A, B and X
 * (device memory) alive until the request's ticket is returned by
 * lp_server_poll.  lp_server_destroy stops the kernel and waits for the
 * server's own streams and worker threads (not the whole device). */
typedef struct {
  size_t memory_bytes;  /* device pool size                                     */
  int small_n_max;      /* n at or below which requests are batched (<= 2048)    */
  int max_batch;        /* ring capacity: batched requests in flight (<= 4096)   */
  int batch_slots;      /* kept for compatibility (1..64); not used              */
  int batch_workgroups; /* workgroups of the persistent batched kernel           */
  int large_slots;      /* blocked-path requests in flight at once (0..64)       */
} lp_server_cfg;

typedef struct {
  const double *A;  /* device, n x n, lda                                        */
  const double *B;  /* device, n x nrhs, ldb                                     */
  double *X;        /* device, n x nrhs, ldx: the solution                       */
  int lda, ldb, ldx;
  int n, nrhs;      /* 1 <= n <= 131072, 1 <= nrhs <= 64                         */
  int prec;         /* LP_FP64, or the low-precision route LP_FP32/BF16/FP16     */
  int nb;           /* panel width for the blocked path                          */
  int max_iter;     /* refinement limit (0 = 30)                                 */
} lp_request;

typedef struct {
  uint64_t ticket;
  int status;            /* 0 solved; 1 singular or not converged               */
  int info;              /* first zero pivot + 1 of the factorization used       */
  int iterations;        /* refinement corrections                               */
  int fell_back;         /* 1 if the binary64 fallback ran                       */
  int batched;           /* 1 if it ran in a batched launch                      */
  double scaled_residual;/* max over right-hand sides                            */
  double latency_ms;     /* submit -> seen complete by lp_server_poll            */
  double device_ms;      /* the request's own device time (batched: its
                            workgroup, device clock; blocked: events around its
                            work); latency_ms - device_ms is the time it waited */
} lp_result;

typedef struct lp_server lp_server;

int lp_server_create(const lp_server_cfg *cfg, lp_server **out);
int lp_server_destroy(lp_server *server);
/* Queues a request; returns LP_ENOSPC if it could never fit the pool.  Work
 * already queued on `stream` (NULL: the null stream) when this is called --
 * typically what produced A and B -- finishes before the request's kernels
 * read A, B or write X.  X is complete once lp_server_poll has returned the
 * ticket. */
int lp_server_submit(lp_server *server, const lp_request *req, uint64_t *ticket, void *stream);
/* Retires finished work, admits and launches queued requests, and returns up
 * to cap finished results (host array) in *count. */
int lp_server_poll(lp_server *server, lp_result *done, int cap, int *count);
/* Queue length, requests on the device, bytes of the pool in use. */
int lp_server_pending(const lp_server *server, int *queued, int *running, size_t *pool_used);
/* Device bytes a request needs from the pool under this configuration. */
size_t lp_request_footprint(const lp_server_cfg *cfg, const lp_request *req);

/* --------------------------------------------- building blocks (exported) */
/* The steps of one block column, callable on their own (used by the tests
 * and by callers that schedule the steps themselves).  Same conventions. */

/* Panel factorization: partial-pivoting LU of the m x w column panel at
 * A (rows 0..m-1, columns 0..w-1 of a row-major array with ld lda), w <= m.
 * ipiv[0..w-1] receive panel-relative pivot rows; *info as lu_factor
 * (panel-relative column).  The interchanges are applied to the w panel
 * columns only.  work: lu_workspace_bytes(m, w, prec) bytes.  prec selects
 * double (LP_FP64) or float (others).
 *   max_wgs  0: the panel is spread over the whole device (one workgroup per
 *            at most 256 rows), the shape lu_factor uses for its first panel
 *            and without look-ahead; k > 0: at most k workgroups of up to
 *            1024 rows each, the shape lu_factor uses for panels factored
 *            beside the trailing update (max(48, ceil(m / 1024)) binary64,
 *            max(128, ceil(m / 1024)) binary32).  LP_ENOTSUP when m > 1024 k;
 *            -10 when k < 0.
 * Results do not depend on max_wgs (the pivot choice and the arithmetic of
 * each element are the same); only the launch shape does. */
int lp_panel_factor(int m, int w, int prec, void *A, int lda, int32_t *ipiv,
                    int32_t *info, void *work, size_t work_bytes, int max_wgs, void *stream);

/* Row interchanges: for j = k1 .. k2-1 in order, swap rows j and ipiv[j]
 * (absolute row indices, ipiv[j] >= j) over columns [c0, c1) of A (double if
 * prec == LP_FP64 else float).  work: lp_laswp_workspace_bytes(k2 - k1). */
size_t lp_laswp_workspace_bytes(int nswaps);
int lp_laswp(int prec, void *A, int lda, int c0, int c1, int k1, int k2,
             const int32_t *ipiv, void *work, size_t work_bytes, void *stream);

/* Triangular solve with a unit lower triangular L (m x m, ld ldl):
 * B := L^-1 B for B m x ncols (ld ldb), in place.  Column-independent.  The
 * blocks to the right of the panel in the paper's "top blocks" update.  work:
 * device scratch of lp_trsm_workspace_bytes(m) bytes (inverses of all the
 * 16 x 16 diagonal blocks, 2 KiB per 16 rows). */
size_t lp_trsm_workspace_bytes(int m);
int lp_trsm_lower_unit(int prec, int m, int ncols, const void *L, int ldl, void *B, int ldb,
                       void *work, size_t work_bytes, void *stream);

/* Right-side triangular solve with an upper, non-unit triangle U (w x w, ld
 * ldu; entries below its diagonal are not read): B := B U^-1 for B m x w (ld
 * ldb), in place.  Rows are independent.  The "left blocks" update of the
 * paper's no-pivot scheme (L21 U11 = A21).  w <= 1024.  work: device scratch
 * of lp_trsm_right_workspace_bytes(w) bytes (transposed inverses of the
 * 16 x 16 diagonal blocks of U).  A zero on U's diagonal gives Inf/NaN. */
size_t lp_trsm_right_workspace_bytes(int w);
int lp_trsm_right_upper(int prec, int m, int w, const void *U, int ldu, void *B, int ldb,
                        void *work, size_t work_bytes, void *stream);

/* Inner-block update C := C - A B with A M x K (lda), B K x N (ldb), C M x N
 * (ldc); prec LP_FP64: all double on FP64 MFMA; LP_FP32: float operands on
 * FP32 MFMA; LP_BF16 / LP_FP16: float A, B, C in memory, operands rounded to
 * bfloat16 / half (nearest even) on the way into the matrix cores, binary32
 * accumulation.  The paper's inner-block matrix multiplication. */
int lp_gemm_update(int prec, int M, int N, int K, const void *A, int lda, const void *B,
                   int ldb, void *C, int ldc, void *stream);

/* The bfloat16 / half form of the update above (prec LP_BF16 or LP_FP16
 * only; K <= 1024) through packed operands: -A and B^T are first written to
 * work, rounded to the 16-bit format (nearest even), as rows of k-contiguous
 * values padded with zeros to 256-row tiles and a power-of-two multiple of 64
 * in k; then C := C - A B on 256 x 256 tiles with binary32 accumulation.  The
 * factorization uses this form for large trailing updates.  work: device
 * scratch of lp_gemm_packed_workspace_bytes(M, N, K) bytes, 16-byte aligned,
 * overwritten; LP_ENOSPC if smaller. */
size_t lp_gemm_packed_workspace_bytes(int M, int N, int K);
int lp_gemm_update_packed(int prec, int M, int N, int K, const void *A, int lda, const void *B,
                          int ldb, void *C, int ldc, void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------ matrix transposition */
/* The paper's PTRANS kernel (section "Parallel Matrix Transposition"):
 * C := B + A^T for n x n row-major A (lda), B (ldb), C (ldc), binary64
 * (prec LP_FP64) or binary32 (LP_FP32), one correctly rounded addition per
 * element, so results are exact to the bit against any plain evaluation.  C
 * may be the same buffer as B (in place); C must not overlap A (not checked;
 * an overlap gives undefined results).  Bound by HBM
 * bandwidth: 3 n^2 elements are read or written once; the paper counts n^2
 * additions as its operations. */
int lp_ptrans(int prec, int n, const void *A, int lda, const void *B, int ldb, void *C, int ldc,
              void *stream);

/* Element-wise copies between binary64 and binary32 (row-major, rows x cols):
 * to_f32 != 0 converts src double -> dst float (round to nearest even),
 * else src float -> dst double. */
int lp_convert(int to_f32, int rows, int cols, const void *src, int lds, void *dst, int ldd,
               void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LP_H_ */

/*
 * gmres_ir.h — C ABI of the MI355X GMRES / GMRES-IR hot path (libgmresir.so).
 *
 * The problem is the one of Alg. 1: solve A x = b for a real n x n sparse A,
 * given b, an initial guess x0 and a relative residual tolerance tol, with
 * convergence meaning ||b - A x||_2 / ||b||_2 <= tol (§III-A).  GMRES(m) is
 * restarted every m iterations (§III-A); GMRES-IR (Alg. 2, §III-B) runs the
 * inner GMRES(m) in float32 on a float32 copy of A and keeps the residual and
 * the solution update in float64.  Right preconditioning with a GMRES
 * polynomial of degree d is §III-D.
 *
 * Conventions shared by every entry point
 *  - Pointers named "device" are HIP device memory owned by the caller; the
 *    library never allocates device memory.  Solver scratch comes from one
 *    caller-provided workspace whose size gmres_workspace_bytes() returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    spmv, cgs2_orth and poly_prec_apply only enqueue work; the solvers and
 *    poly_prec_setup synchronise `stream` before returning.
 *  - Arguments are checked before anything is enqueued.  A negative status
 *    means nothing usable was produced; gmr_last_error() then returns a
 *    message (thread-local, valid until the next call on the thread).
 *    A positive status from a solver means x holds the best iterate found.
 *  - Index arrays are int32 (row_ptr has n+1 entries, col_idx nnz entries,
 *    columns ascending within a row is not required); values are float32 or
 *    float64 as `dtype` says.  col_idx and val must be 16-byte aligned (the
 *    SpMV reads them with 16-byte vector loads); GMR_ERR_INVALID otherwise.
 *  - Dense vectors are contiguous; the Krylov basis V is column-major with
 *    leading dimension ldv >= n.
 */
#ifndef GMRES_IR_H
#define GMRES_IR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { GMR_F32 = 0, GMR_F64 = 1 } gmr_dtype;

typedef enum {
  GMR_OK = 0,
  GMR_NOT_CONVERGED = 1,     /* max_iters / max_cycles reached; x = last iterate        */
  GMR_STAGNATED = 2,         /* no residual decrease over `stagnation_cycles` restarts */
  GMR_LOSS_OF_ACCURACY = 3,  /* GMR_FLAG_STOP_ON_LOSS: the implicit residual met tol, the
                                explicit one did not (§V-F); x = last iterate             */
  GMR_SYSTEMS_FAILED = 4,    /* batched solves: some systems stopped on an error and were
                                frozen at their last iterate, every other one finished;
                                batch_system_status() tells which                        */
  GMR_ERR_INVALID = -1,      /* bad argument (null pointer, size, dtype mismatch, ...)   */
  GMR_ERR_HIP = -2,          /* a HIP call failed                                        */
  GMR_ERR_WORKSPACE = -3,    /* workspace smaller than gmres_workspace_bytes()           */
  GMR_ERR_NONFINITE = -4,    /* NaN/Inf in b, in a residual norm or in the Hessenberg    */
  GMR_ERR_UNSUPPORTED = -5   /* parameter outside what this library supports             */
} gmr_status;

/* CSR matrix; all three arrays are device pointers. */
typedef struct {
  int32_t n;                 /* rows = columns, > 0                */
  int32_t nnz;               /* row_ptr[n] - row_ptr[0], >= 0      */
  const int32_t* row_ptr;    /* n+1 entries, row_ptr[0] == 0       */
  const int32_t* col_idx;    /* nnz entries in [0, n)              */
  const void* val;           /* nnz values of type `dtype`         */
  int32_t dtype;             /* gmr_dtype                          */
} gmr_csr;

/* Profiling selector: the solver brackets every launch of one kernel family
 * with HIP events and reports their summed duration and algorithmic bytes. */
typedef enum {
  GMR_PROF_NONE = 0, GMR_PROF_SPMV = 1, GMR_PROF_CGS_DOTS = 2, GMR_PROF_CGS_UPDATE_DOTS = 3,
  GMR_PROF_CGS_UPDATE_NORM = 4, GMR_PROF_POLY_STEP = 5, GMR_PROF_RESIDUAL = 6, GMR_PROF_BJAC = 7
} gmr_prof_kernel;

typedef struct {
  int32_t restart;           /* m, 1 <= m <= 512 (§III-A "restart length")                 */
  double tol;                /* relative residual tolerance, > 0                           */
  int64_t max_iters;         /* cap on inner iterations (> 0)                              */
  int32_t max_cycles;        /* cap on restarts, 0 = none                                  */
  int32_t stagnation_cycles; /* GMRES-IR: give up after this many restarts without
                                the residual decreasing by 1 %, 0 = never                  */
  int32_t prof_kernel;       /* gmr_prof_kernel                                            */
  int32_t flags;             /* GMR_FLAG_* bits                                            */
} gmr_params;

/* gmr_params.flags: capture one restart cycle as a hipGraph and replay it each
 * restart (ignored while profiling).  The solve then runs on a library-owned
 * non-blocking stream after `stream` has drained; results are the same bits. */
#define GMR_FLAG_GRAPH 1
/* gmr_params.flags: for a system of n <= 6144 without a polynomial, run each
 * whole restart cycle (cast, inner iterations, update, residual) as one launch
 * instead of about eight per inner iteration: up to n = 1024 one block with
 * block barriers (2-4x faster at n ~ 150), above it a cooperative launch of
 * ceil(n / 256) co-resident blocks with grid barriers where the
 * multi-kernel cycle has kernel boundaries (four per iteration).  Ignored when
 * it does not apply (larger n, polynomial, profiling, GMR_FLAG_GRAPH, a device
 * that cannot hold the grid); the arithmetic is the same, summed in a
 * different grouping, and repeatable bit for bit.  A grid barrier that does
 * not complete within about a second ends the solve with GMR_ERR_HIP. */
#define GMR_FLAG_PERSISTENT 2
/* gmr_params.flags: plain GMRES (gmres_solve, gmres_f32prec_solve, the float64
 * phase of gmres_fd_solve) ends with GMR_LOSS_OF_ACCURACY at the first restart
 * whose cycle signalled convergence through its implicit residual while the
 * explicit residual ||b - A x|| / ||b|| was above tol (§V-F).  Without the flag
 * the solver counts such a restart in result->loss_of_accuracy and goes on
 * from the explicit residual: the correction §V-F proposes.  GMRES-IR ignores it. */
#define GMR_FLAG_STOP_ON_LOSS 4
/* gmr_params.flags: GMRES-IR (gmres_ir_solve, with or without a preconditioner)
 * stores the inner Krylov basis in IEEE float16, column j as half(sigma * v_j) with
 * the power of two sigma ~ sqrt(n); all arithmetic stays float32 and the outer
 * loop float64.  A third precision, the future work of §VI: it halves the
 * bytes of the basis that CGS2 streams, and each cycle's correction is then
 * accurate to about 1e-3, which the outer float64 loop absorbs (more cycles
 * only when a cycle would otherwise reduce the residual by much more).
 * The preconditioner is applied to the float32 vector before rounding.
 * GMR_ERR_UNSUPPORTED in the other solvers. */
#define GMR_FLAG_HALF_BASIS 8

typedef struct {
  int32_t status;            /* gmr_status                                                 */
  int32_t cycles;            /* restarts performed                                         */
  int64_t iters;             /* inner iterations performed (all cycles)                    */
  double rel_res;            /* explicit ||b - A x|| / ||b|| in float64 at exit            */
  double implicit_rel_res;   /* |g_{k+1}| * gamma / ||b|| of the last cycle                */
  double seconds;            /* wall time of the solve (host clock, stream synchronised)   */
  int32_t history_len;       /* entries written to `hist`                                  */
  int32_t loss_of_accuracy;  /* gmres_solve, gmres_f32prec_solve, gmres_fd_solve: restarts
                                whose cycle ended on its implicit residual (or a breakdown)
                                while the explicit residual was still above tol (§V-F)     */
  double prof_ms;            /* summed duration of the profiled launches                   */
  int64_t prof_launches;     /* number of profiled launches                                */
  double prof_bytes;         /* summed algorithmic bytes of the profiled launches          */
} gmr_result;

/* Opaque host-side handle of a right preconditioner M (§III-D): a GMRES
 * polynomial (poly_prec_setup: its roots) or block Jacobi (bjac_prec_setup:
 * a pointer to the caller's inverted blocks).  Every solver's P argument and
 * poly_prec_apply accept either kind. */
typedef struct gmr_poly gmr_poly;

/* Workspace (bytes, device) needed by gmres_solve / gmres_ir_solve for a system of
 * order n with the given parameters and working precision `dtype` (F64: plain
 * float64 GMRES; F32: GMRES-IR, or a float32-only gmres_solve), with a
 * polynomial preconditioner when `with_poly` != 0 (F64 with a polynomial also
 * covers gmres_f32prec_solve).  Also valid for cgs2_orth (with restart >= k)
 * and for poly_prec_setup/poly_prec_apply. */
size_t gmres_workspace_bytes(int32_t n, const gmr_params* params, int32_t dtype, int32_t with_poly);

/* y = A x (§V-D: y_i = sum_k val[k] x[col[k]], summed in ascending k; products
 * are rounded before they are added).  x, y: device, n entries of A's dtype,
 * must not overlap.  Asynchronous. */
gmr_status spmv(const gmr_csr* A, const void* x, void* y, void* stream);

/* One CGS2 orthogonalisation step (Alg. 1 with the two classical Gram-Schmidt
 * passes of §III-A): h1 = V^T w, w -= V h1, h2 = V^T w, w -= V h2,
 * beta = ||w||, w /= beta.  V: device, n x k column-major, leading dim ldv.
 * w: device, n entries, overwritten with the normalised vector (left as is
 * when beta is 0).  h: device float64, k+1 entries: h[0..k-1] = h1 + h2 and
 * h[k] = beta.  1 <= k <= 512.  dtype selects float32 or float64 data.
 * ws: device workspace of gmres_workspace_bytes(n, {restart >= k}, dtype, 0)
 * bytes.  Asynchronous. */
gmr_status cgs2_orth(int32_t dtype, int32_t n, int32_t k, const void* V, int64_t ldv, void* w,
                     double* h, void* ws, size_t ws_bytes, void* stream);

/* cgs2_orth without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The same kernels and the same results as
 * cgs2_orth; its scratch (about 8.4 MB: the reduction partials and the
 * coefficient vectors) is a static device array of the library, one copy per
 * device, held until the process ends, so the call allocates nothing.
 * n <= 134217728 (GMR_ERR_UNSUPPORTED beyond), other arguments and errors as
 * cgs2_orth.  Every call on a device shares that device's array: calls that
 * overlap on one device (two streams, two threads) race and give undefined
 * results; calls on one stream are ordered and safe.  Nothing in the array
 * needs to start at zero.  Asynchronous. */
gmr_status cgs2_orth_noalloc(int32_t dtype, int32_t n, int32_t k, const void* V, int64_t ldv, void* w,
                             double* h, void* stream);

/* Build the GMRES-polynomial preconditioner p of degree `degree` (§III-D):
 * run degree+1 Arnoldi (CGS2) steps on A from the device start vector v0
 * (n entries of A's dtype, need not be normalised) in A's precision, take the
 * harmonic Ritz values (the roots of the GMRES residual polynomial), order
 * them by the modified Leja ordering and round them to A's precision.  A
 * lucky breakdown after s steps lowers the degree to s-1.  0 <= degree <= 128.
 * Synchronous; *out must be released with poly_prec_destroy. */
gmr_status poly_prec_setup(const gmr_csr* A, int32_t degree, const void* v0, void* ws,
                           size_t ws_bytes, gmr_poly** out, void* stream);

/* y = M x: for a polynomial p(A) x with the roots of P (exactly degree
 * products with A); for block Jacobi the block-diagonal product with the
 * inverted blocks (A then only gives n and the dtype, and ws may be NULL).
 * A must have the dtype P was built for; x, y: device, n entries, must not
 * overlap.  ws as for poly_prec_setup.  Asynchronous. */
gmr_status poly_prec_apply(const gmr_poly* P, const gmr_csr* A, const void* x, void* y, void* ws,
                           size_t ws_bytes, void* stream);

void poly_prec_destroy(gmr_poly* P);

/* Device bytes of the `inv` buffer of bjac_prec_setup (0 for bad arguments):
 * 256 bytes of status, then ceil(n/block) slots of block x block values. */
size_t bjac_prec_bytes(int32_t n, int32_t block, int32_t dtype);

/* Build the block Jacobi preconditioner M = blockdiag(A)^-1 (§III-D; the
 * "J k" preconditioner of Table III in §V-G): diagonal blocks of `block`
 * consecutive rows (the last one takes the remaining rows), gathered from A's
 * CSR rows (duplicate entries are summed) and inverted on the device by
 * Gauss-Jordan elimination with partial pivoting in A's precision (float32
 * for the float32 copy: built and applied in float32).  1 <= block <= 64.
 * inv: caller's device memory of bjac_prec_bytes(n, block, A->dtype) bytes,
 * 256-byte aligned, which holds the inverted blocks (column-major per block)
 * and must outlive the handle; the library does not free it.  A singular
 * block (a zero or non-finite pivot) gives GMR_ERR_NONFINITE and no handle.
 * Synchronous; *out must be released with poly_prec_destroy. */
gmr_status bjac_prec_setup(const gmr_csr* A, int32_t block, void* inv, size_t inv_bytes, gmr_poly** out,
                           void* stream);

/* Rows per diagonal block of a block Jacobi handle; 0 for a polynomial. */
int32_t prec_block_size(const gmr_poly* P);

/* The (s+1) x s Hessenberg matrix of the Arnoldi run that built P (s = degree+1),
 * column-major with leading dimension s+1, into the host array H. */
gmr_status poly_prec_hessenberg(const gmr_poly* P, double* H);

/* Degree d of P and its d+1 roots (float64 copies of the rounded values, Leja order). */
int32_t poly_prec_degree(const gmr_poly* P);
gmr_status poly_prec_roots(const gmr_poly* P, double* re, double* im);

/* Restarted GMRES(m) in A's precision (Alg. 1 with CGS2): the implicit residual
 * is tested after every iteration and convergence is confirmed by the
 * explicit residual at the end of the cycle.  b: device, n entries; x: device,
 * n entries, holds x0 on entry and the solution on exit (both of A's dtype).
 * P: optional right preconditioner of the same dtype (NULL = none).
 * hist: optional host array of max_cycles+1 (or 4096 when max_cycles is 0)
 * float64 explicit relative residuals, one per restart, starting with x0's.
 * Synchronous. */
gmr_status gmres_solve(const gmr_csr* A, const gmr_poly* P, const void* b, void* x,
                       const gmr_params* params, void* ws, size_t ws_bytes, gmr_result* result,
                       double* hist, void* stream);

/* GMRES-IR (Alg. 2): r = b - A64 x in float64; each cycle solves A u = r by
 * exactly m float32 GMRES iterations on A32 (only a breakdown ends a cycle
 * early) and adds u to x in float64, until ||r|| / ||b|| <= tol.
 * A64: float64 matrix; A32: the same pattern with float32 values (see
 * csr_values_to_f32).  P: optional float32 right preconditioner built on A32.
 * b, x: device float64.  hist as for gmres_solve.  Synchronous. */
gmr_status gmres_ir_solve(const gmr_csr* A64, const gmr_csr* A32, const gmr_poly* P,
                          const double* b, double* x, const gmr_params* params, void* ws,
                          size_t ws_bytes, gmr_result* result, double* hist, void* stream);

/* Float64 GMRES(m) with a float32 right preconditioner (§III-D option (a), the
 * middle option of the comparison in §V-C and the study of §V-F): the solver
 * is gmres_solve in float64 on A64, and each application of M = p(A32) casts
 * its float64 input to float32, applies the float32 polynomial P32 (built by
 * poly_prec_setup on A32) with A32's products in float32, and widens the
 * result back to float64.  Loss of accuracy (§V-F) is counted in
 * result->loss_of_accuracy and corrected by restarting from the explicit
 * residual, or ends the solve under GMR_FLAG_STOP_ON_LOSS.  b, x: device
 * float64; hist as for gmres_solve; ws: gmres_workspace_bytes(n, params,
 * GMR_F64, 1) bytes.  Synchronous. */
gmr_status gmres_f32prec_solve(const gmr_csr* A64, const gmr_csr* A32, const gmr_poly* P32, const double* b,
                               double* x, const gmr_params* params, void* ws, size_t ws_bytes,
                               gmr_result* result, double* hist, void* stream);

/* Workspace (bytes, device) for gmres_fd_solve on a system of order n: the
 * float64 solver's workspace plus float32 copies of b and of the iterate. */
size_t gmres_fd_workspace_bytes(int32_t n, const gmr_params* params);

/* GMRES-FD (§III-C, option 1; the switch-point study of §V-A): float32
 * GMRES(m) on A32 from (float) x with right-hand side (float) b, for at most
 * switch_iters iterations (fewer if its float32 explicit residual reaches tol
 * or it stagnates by params->stagnation_cycles), then float64 GMRES(m) on A64
 * from x = (double) of the float32 iterate until ||b - A64 x|| / ||b|| <= tol.
 * switch_iters = 0 runs float64 GMRES(m) alone.  params->max_iters caps the
 * iterations of both phases together and must exceed switch_iters; restart,
 * tol, max_cycles, stagnation_cycles, prof_kernel and flags apply to each phase.
 * A64, A32, b, x: as for gmres_ir_solve (b and x must be representable in
 * float32).  result: both phases (cycles, iters, prof_* and history_len
 * summed; status, rel_res and implicit_rel_res of the float64 phase; seconds
 * over the whole call).  float_result: optional (NULL), the float32 phase alone;
 * its residuals are float32 arithmetic against (float) b.  hist: optional host
 * array of twice the capacity gmres_solve asks for: the float32 phase's
 * relative residuals, then the float64 phase's.  If the float32 phase fails
 * (e.g. GMR_ERR_NONFINITE), x is unchanged and both records describe that phase.
 * ws: gmres_fd_workspace_bytes(n, params) bytes.  Synchronous. */
gmr_status gmres_fd_solve(const gmr_csr* A64, const gmr_csr* A32, const double* b, double* x,
                          const gmr_params* params, int64_t switch_iters, void* ws, size_t ws_bytes,
                          gmr_result* result, gmr_result* float_result, double* hist, void* stream);

/* out[k] = (float) in[k], round to nearest even; in, out: device.  Asynchronous. */
gmr_status csr_values_to_f32(const double* in, float* out, int64_t count, void* stream);

/* Eigenvalues of a k x k upper Hessenberg matrix (host, column-major, ld k) by
 * the Francis double-shift QR iteration; host only, used by poly_prec_setup.
 * re, im: host, k entries.  Returns GMR_ERR_NONFINITE if it fails to converge. */
gmr_status gmr_hessenberg_eigvals(int32_t k, const double* H, double* re, double* im);

/* Harmonic Ritz values of a k-step Arnoldi run (host): the eigenvalues of
 * H_k + h_{k+1,k}^2 f e_k^T with H_k^T f = e_k, i.e. the roots of the k-step
 * GMRES residual polynomial (§III-D).  H: host, column-major (k+1) x k with
 * leading dimension ldh >= k+1; re, im: host, k entries. */
gmr_status gmr_harmonic_ritz(int32_t k, const double* H, int32_t ldh, double* re, double* im);

/* Modified Leja ordering of k values (host, in place): largest modulus first,
 * then the value maximising the sum of log distances to those chosen;
 * complex-conjugate pairs adjacent, positive imaginary part first. */
gmr_status gmr_leja_order(int32_t k, double* re, double* im);

/* ---------------------------------------------------------------------------
 * Batched block GMRES-IR: many independent systems with 16 right-hand sides
 * each (the paper's solver handles one right-hand side, §IV; this is the
 * multi-system, multi-RHS growth of the same method).  Per system, the 16
 * right-hand sides share one block Krylov space built with two block
 * classical Gram-Schmidt passes (block CGS2, §III-A) on the matrix cores
 * and Cholesky QR twice inside each block; the outer loop is GMRES-IR
 * (Alg. 2) with float64 residuals and updates, each column scaled by its own
 * residual norm.  The inner solve runs in float32 (batch_gmres_ir_solve) or,
 * as the baseline, in float64 (batch_gmres_solve).
 * ------------------------------------------------------------------------- */
typedef struct gmr_batch gmr_batch;  /* opaque, host-side: sizes and the tile table */

typedef struct {
  int32_t status;        /* gmr_status                                               */
  int32_t cycles;        /* restart cycles run (of the slowest system)               */
  int64_t block_iters;   /* block steps summed over systems and cycles               */
  double max_rel_res;    /* max over systems and columns of ||b - A x|| / ||b||      */
  double seconds;        /* wall time of the solve                                   */
} gmr_batch_result;

/* A batch of nsys systems whose orders are sys_rows[0..nsys-1] (host array);
 * their matrices are the diagonal blocks, in order, of one block-diagonal CSR
 * matrix with global column indices.  nrhs must be 16; restart m in [1, 64]
 * block steps.  *out is released with batch_destroy. */
gmr_status batch_create(int32_t nsys, const int32_t* sys_rows, int32_t nrhs, int32_t restart,
                        gmr_batch** out);
void batch_destroy(gmr_batch* b);

/* Device workspace needed with inner precision inner_dtype: GMR_F32 for
 * batch_gmres_ir_solve, batch_autotune and batch_bcgs_step, GMR_F64 for
 * batch_gmres_solve.  0 for a null batch or another dtype. */
size_t batch_workspace_bytes(const gmr_batch* b, int32_t inner_dtype);

/* Tiling of the matrix-core kernels: rows per tile (multiple of 16, >= 256) and
 * the block-dots variant: 4, 8 or 16 basis blocks accumulated per pass with a
 * cross-wave reduction in LDS; the wave-split variants 2, 3, 5 (each wave
 * accumulates 2, 4, 4 blocks over all rows with 8, 4, 8 four-row slices in
 * flight); or 6, 7: 8 or 16 blocks per pass read with 16-byte loads staged
 * through LDS.  Float64 uses 8 blocks where 16 is set, and the scalar-load
 * 8-block form for 6 and 7. */
gmr_status batch_set_tiling(gmr_batch* b, int32_t tile_rows, int32_t group_blocks);
gmr_status batch_get_tiling(const gmr_batch* b, int32_t* tile_rows, int32_t* group_blocks);

/* With on != 0, the solves of this batch capture one restart cycle (start
 * block, m block steps, update and residual: the same launches with the same
 * arguments every cycle) as a hipGraph and replay it once per cycle.  They
 * then run on a library-owned stream after draining the caller's stream.
 * Results are identical to the eager launches. */
gmr_status batch_set_graph(gmr_batch* b, int32_t on);

/* Chooses the tiling by timing the block Gram-Schmidt contractions at about
 * (m+1)/8, (m+1)/2 and 7(m+1)/8 blocks, every system active, on the batch's
 * own workspace (its contents are overwritten), in two stages: the tile rows
 * (512, 1024, 2048, 4096) by the dots and update pair with the staged dots
 * variant 7, then the dots variant (4, 8, 16, 2, 3, 5, 6, 7) at those rows by
 * the dots alone.  Keeps the choice; *best_ms is the fastest of five timed
 * repetitions of the pair at the chosen rows (best_* may be NULL).  Synchronous. */
gmr_status batch_autotune(gmr_batch* b, void* ws, size_t ws_bytes, int32_t* best_tile_rows,
                          int32_t* best_group_blocks, double* best_ms, void* stream);

/* Solve A X = B for all systems to ||b - A x|| / ||b|| <= tol per column.
 * A64 / A32: the block-diagonal matrix in float64 / float32 (same pattern).
 * B, X: device float64, rows x 16 row-major (X holds X0 on entry).
 * Z: device float32, rows x 16 row-major, random columns that replace start
 * columns which (nearly) depend on earlier ones.  sys_cycles (nsys) and
 * sys_rel_res (nsys x 16): optional host outputs.  Synchronous. */
gmr_status batch_gmres_ir_solve(gmr_batch* b, const gmr_csr* A64, const gmr_csr* A32, const double* B,
                                double* X, const float* Z, double tol, int32_t max_cycles, void* ws,
                                size_t ws_bytes, gmr_batch_result* res, int32_t* sys_cycles,
                                double* sys_rel_res, void* stream);

/* Per-system outcome of the last batch_gmres_ir_solve / batch_gmres_solve on
 * this batch, into the host array out (nsys entries): GMR_OK (every column
 * reached tol), GMR_NOT_CONVERGED (max_cycles reached) or GMR_ERR_NONFINITE
 * (the system's start block could not be orthonormalised: its random
 * replacement columns were themselves dependent or not finite).  A system that
 * fails is frozen at its iterate of that cycle and leaves the tile table; the
 * others go on, and the solve returns GMR_SYSTEMS_FAILED when they all
 * converged, with max_rel_res over the systems that did not fail.
 * GMR_ERR_INVALID before any solve. */
gmr_status batch_system_status(const gmr_batch* b, int32_t* out);

/* The same solve with the whole inner block GMRES(m) in float64 (block
 * Gram-Schmidt on the float64 matrix cores): plain restarted block GMRES, the
 * reference the mixed-precision solve is measured against (§V-B's comparison
 * for the batched case).  Arguments as batch_gmres_ir_solve, with no float32
 * matrix; the workspace is batch_workspace_bytes(b, GMR_F64).  Synchronous. */
gmr_status batch_gmres_solve(gmr_batch* b, const gmr_csr* A64, const double* B, double* X, const float* Z,
                             double tol, int32_t max_cycles, void* ws, size_t ws_bytes, gmr_batch_result* res,
                             int32_t* sys_cycles, double* sys_rel_res, void* stream);

/* One block Gram-Schmidt pass on its own (for tests): C = V^T W per system
 * (device float64 out, nsys x nblk x 16 x 16, C[s][b][i][c]) and W -= V C.
 * Vin: device float32, nblk blocks of rows x 16 (block-major).  Asynchronous. */
gmr_status batch_bcgs_step(gmr_batch* b, const float* Vin, int32_t nblk, float* W, double* C, void* ws,
                           size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Learned parameter predictor (restart length, polynomial degree and inner
 * precision of GMRES-IR from cheap matrix features; the paper's guidance for
 * these choices is §V-B, §V-C, §V-E and §V-F).  A 16-64-64-11 MLP, ReLU,
 * three softmax heads (4 restarts, 5 degrees, 2 precisions); the parameters
 * are one float32 vector: W1 (64x16, row-major), b1, W2 (64x64), b2,
 * W3 (11x64), b3.  All pointers are device pointers unless stated.
 * ------------------------------------------------------------------------- */
int32_t mlp_param_count(void);                 /* 5963 */
size_t mlp_workspace_bytes(int32_t batch);     /* for mlp_loss_grad */

/* logits (batch x 11) of the standardised features (X - mu) / sigma (X: batch x 16). */
gmr_status mlp_forward(const float* params, const float* X, const float* mu, const float* sigma,
                       int32_t batch, float* logits, void* stream);

/* Gradient (5963) and loss (1 float, nullable) of the mean over the batch of the
 * summed head cross-entropies; labels: batch x 3 class indices.  Asynchronous. */
gmr_status mlp_loss_grad(const float* params, const float* X, const float* mu, const float* sigma,
                         const int32_t* labels, int32_t batch, float* grad, float* loss, void* ws,
                         size_t ws_bytes, void* stream);

/* One Adam step (bias-corrected, step >= 1) on params with moments m, v. */
gmr_status mlp_adam_step(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                         float beta1, float beta2, float eps, void* stream);

/* Thirteen row statistics of A into the host array out: sum and min of the
 * diagonal-dominance ratio |a_ii| / sum_{j!=i} |a_ij|, rows with ratio >= 1,
 * rows with off-diagonal entries, min (a_ii - r_i), max (a_ii + r_i), max r_i,
 * max |a_ii|, sum a_ii, sum a_ii^2, max nonzeros in a row, ||A||_F^2 and
 * ||A - A^T||_F^2 (columns must ascend within a row).  ws: device,
 * 13 * 8 * (min(ceil(n/256), 1024) + 1) bytes.  Synchronous. */
gmr_status matrix_stats(const gmr_csr* A, double* out, void* ws, size_t ws_bytes, void* stream);

/* Bytes of device workspace matrix_features needs for an n x n matrix of
 * the given dtype (0 for bad arguments). */
size_t matrix_features_workspace_bytes(int32_t n, int32_t dtype);

/* The 16 predictor features of A into the host array out, in this order:
 * log10 n; nonzeros per row; most nonzeros in a row; min and mean diagonal
 * dominance |a_ii| / sum_{j!=i} |a_ij| (rows with off-diagonal entries; min is
 * 10 when there are none) and the fraction of rows with dominance >= 1;
 * Gershgorin min (a_ii - r_i), max (a_ii + r_i) and max r_i, each divided by
 * max |a_ii|; ||A - A^T||_F / ||A||_F; std / |mean| of the diagonal; from an
 * Arnoldi run of min(5, n) steps from the device vector v0 (n entries of A's
 * dtype, need not be normalised; fewer steps after a lucky breakdown): max |theta| and
 * min |theta| of its Ritz values over max |a_ii|, log10 of their ratio,
 * max |Im theta| / max |theta| and h_{k+1,k} / max |theta|.  Non-finite values
 * are replaced by 0, +1e6 or -1e6.  These are cheap estimates of what the
 * paper's guidance for the restart length, the polynomial degree and the
 * precision turns on (§V-B, §V-C, §V-E, §V-F): conditioning, normality and
 * the spread of the spectrum.  Columns must ascend within a row.  ws: device,
 * matrix_features_workspace_bytes(n, dtype) bytes.  Synchronous. */
gmr_status matrix_features(const gmr_csr* A, const void* v0, double* out, void* ws, size_t ws_bytes,
                           void* stream);

const char* gmr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GMRES_IR_H */

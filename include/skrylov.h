/*
 * skrylov.h -- C ABI of the MI355X (gfx950) simultaneous short-recurrence Krylov
 * solvers for A X = B with a sparse non-Hermitian A (n x n) and s right-hand
 * sides B (n x s).
 *
 * Method definitions follow Rashedi, Birk, Frommer, Ebadi, "On short recurrence
 * Krylov type methods for linear systems with many right-hand sides"
 * (arXiv 1504.04395):
 *   - the problem statement A X = B is Section 1 (simultaneous systems);
 *   - Gl-BiCG is Algorithm 2, eGl-BiCG Algorithm 4, Bl-BiCG-rQ Algorithm 5 with
 *     equations (newalpha)-(newbetahat);
 *   - Gl-QMR, eGl-QMR and Gl-BiCGStab are described in Sections 2 and 4 and
 *     Bl-BiCGStab-rQ in the closing paragraph of Section 4;
 *   - the solve protocol (X0 = 0, B replaced by Q from B = QR, shadow R^0 = R0 or
 *     the mean of the initial residuals, stopping at ||R_k||_F <= tol ||R_0||_F)
 *     is the opening paragraph of Section 5.
 *
 * Conventions
 *   - Blocks (B, X, G) are row-major n x s with a leading dimension ld >= s:
 *     element (i, c) is at p[i * ld + c].  Complex values are interleaved
 *     (re, im) pairs of doubles.  All boundary data are FP64 (real or complex);
 *     reduced precision exists only inside the library (SKR_PREC_FP32_REFINE).
 *   - Pointers are host or device memory as stated by the skr_mem argument.
 *     The caller owns every pointer it passes.  The library keeps no caller
 *     pointer after a call returns.
 *   - Work is enqueued on the context's HIP stream.  Calls that return data
 *     synchronise that stream before returning.
 *   - Return value: 0 on success, a negative skr_status when nothing was
 *     computed (the reason is available from skr_last_error), or a positive
 *     skr_status from skr_solve when X holds the last iterate and the result
 *     record is filled.  Nothing aborts or throws across this interface.
 *   - Calls on one context are not thread-safe; use one context per thread.
 *   - A matrix is used only with the context that created it; other calls get
 *     SKR_E_INVALID.  Destroying a context leaves its matrices to be destroyed
 *     (and unusable for anything else).
 */
#ifndef SKRYLOV_H
#define SKRYLOV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SKR_OK = 0,
    SKR_E_INVALID = -1,       /* bad argument (size, pointer, NaN in input, ...) */
    SKR_E_ALLOC = -2,         /* device memory allocation failed */
    SKR_E_HIP = -3,           /* a HIP runtime call failed */
    SKR_E_UNSUPPORTED = -4,   /* valid request the library does not provide  */
    SKR_NOT_CONVERGED = 1,    /* maxit reached; X holds the last iterate */
    SKR_BREAKDOWN = 2,        /* a denominator vanished / an s x s matrix was singular */
    SKR_DIVERGED = 3          /* final true relative residual > 1 (Section 5.2, "div.") */
} skr_status;

typedef enum {
    SKR_GL_BICG = 0,          /* Algorithm 2 */
    SKR_EGL_BICG = 1,         /* Algorithm 4 */
    SKR_GL_QMR = 2,           /* Section 2 (global QMR) */
    SKR_EGL_QMR = 3,          /* Section 4 (economic global QMR) */
    SKR_GL_BICGSTAB = 4,      /* Sections 2-3 (global BiCGStab) */
    SKR_BL_BICG_RQ = 5,       /* Algorithm 5 */
    SKR_BL_BICGSTAB_RQ = 6,   /* Section 4, closing paragraph */
    SKR_BL_BICG = 7,          /* Algorithm 3 (block BiCG without QR of the residual) */
    SKR_BL_BICGSTAB = 8,      /* block BiCGStab of El Guennouni et al. (Sections 3 and 5.2) */
    SKR_LI_BICG = 9,          /* Algorithm 1 (loop-interchanged: s independent BiCG) */
    SKR_LI_BICGSTAB = 10,     /* Section 2 (loop-interchanged: s independent BiCGStab) */
    SKR_LI_QMR = 11           /* Section 2 (loop-interchanged: s independent QMR) */
} skr_method;

typedef enum { SKR_F64 = 0, SKR_C64 = 1 } skr_dtype;
typedef enum { SKR_PREC_FP64 = 0, SKR_PREC_FP32_REFINE = 1 } skr_precision;
typedef enum { SKR_MEM_HOST = 0, SKR_MEM_DEVICE = 1 } skr_mem;
typedef enum { SKR_PRECOND_NONE = 0, SKR_PRECOND_ILU0 = 1 } skr_precond;
typedef enum { SKR_FMT_CSR = 0, SKR_FMT_SELL = 1 } skr_format;

typedef struct skr_context skr_context;
typedef struct skr_matrix skr_matrix;

/* Storage options for skr_matrix_create.  SELL-C-sigma: rows sorted by length
 * inside windows of sigma rows, chunks of C rows stored column-major and padded
 * to the chunk's longest row.  sell_C must be 16, 32 or 64; sell_sigma a
 * multiple of sell_C.  make_fp32 also keeps FP32 copies of the values of A and
 * A^H for SKR_PREC_FP32_REFINE solves (otherwise they are built on first use). */
typedef struct {
    int32_t format;       /* skr_format */
    int32_t sell_C;
    int32_t sell_sigma;
    int32_t make_fp32;
} skr_format_opts;

/* Solve options (skr_opts_default fills the defaults in brackets). */
typedef struct {
    double tol;             /* stop at ||R_k||_F <= tol ||R_0||_F              [1e-8]  */
    int32_t maxit;          /* iteration cap; reaching it gives NOT_CONVERGED   [10000] */
    int32_t precision;      /* skr_precision                                     [FP64]  */
    double inner_tol;       /* FP32 inner solves: relative residual target       [1e-4]  */
    int32_t max_outer;      /* FP32 refinement: outer iteration cap             [10]    */
    int32_t preprocess_qr;  /* replace R0 by Q from R0 = Q R (Section 5)         [1]     */
    int32_t zero_x0;        /* ignore the contents of X on entry (X0 = 0)        [1]     */
    int32_t check_every;    /* host reads the device stop flag every m iterations [16]  */
    int32_t use_graph;      /* replay the m-iteration schedule as a hipGraph     [1]     */
    int32_t precond;        /* skr_precond: SKR_PRECOND_ILU0 = right no-fill ILU
                             * (Section 5.2): the method runs on A M^-1 with
                             * M = L U from skr_matrix_ilu0 and returns
                             * X = X0 + M^-1 D; residuals stay those of A X = B.
                             * FP64, non-adjoint solves only                 [NONE]  */
    int32_t fused_small;    /* FP64 Gl-BiCG / eGl-BiCG / Gl-BiCGStab on at most
                             * 1024 rows with CSR storage, no preconditioner and
                             * s <= 4 (real) or s <= 2 (complex): run every iteration in one
                             * single-workgroup launch instead of the
                             * multi-kernel schedule.  Same iteration, stopping
                             * rule and history; check_every and use_graph do
                             * not apply.  0 forces the general schedule      [1]     */
} skr_opts;

/* Result record.  history is caller-owned (may be NULL).  FP64 solves: on
 * return it holds the recursive ||R_k||_F / ||R_0||_F for k = 0..history_len-1.
 * FP32 + refinement: it holds the true FP64 relative residual ||B - A X||_F /
 * ||B||_F before each outer step and after the last one. */
typedef struct {
    int32_t status;             /* skr_status of the solve                      */
    int32_t iterations;         /* completed iterations (sum over inner solves) */
    int64_t matvecs;            /* matrix-vector products (s per block product) */
    int32_t outer_iterations;   /* refinement steps (FP32 path), else 0         */
    int32_t breakdown_iter;     /* iteration at which a breakdown was detected, else -1 */
    double rel_res_recursive;   /* last recursive ||R_k|| / ||R_0||             */
    double rel_res_true;        /* ||B - A X||_F / ||B||_F recomputed at exit   */
    double* history;
    int32_t history_cap;
    int32_t history_len;
    int32_t fp64_outer_iterations; /* FP32 path: refinement steps run in FP64
                                    * because the FP32 QR or inner solve failed
                                    * (breakdown, divergence) or an earlier FP32
                                    * step did not halve the true residual     */
    int32_t single_workgroup;   /* 1 if the iterations ran in one single-workgroup
                                 * launch (opts.fused_small), else 0           */
} skr_result;

/* Fill *opts with the defaults listed above. */
void skr_opts_default(skr_opts* opts);

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the handle. */
int skr_context_create(int device, void* hip_stream, skr_context** out);
int skr_context_destroy(skr_context* ctx);
/* Change the stream later calls enqueue on. */
int skr_context_set_stream(skr_context* ctx, void* hip_stream);
/* Last error message of this context ("" if none).  Valid until the next call. */
const char* skr_last_error(skr_context* ctx);

/* Copy a CSR matrix into library-owned device memory and build A^H (explicit
 * conjugate transpose, Algorithms 2, 3 and 5 multiply with it) on the device.
 * row_ptr: n+1 int64 offsets (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz);
 * col_idx: nnz int32 columns in [0, n), strictly increasing within a row;
 * values: nnz FP64 (SKR_F64) or interleaved complex FP64 (SKR_C64).
 * All three arrays live in `mem`.  n must be in [1, 2^31 - 2^20] (the device
 * sweeps index rows with int32 and step past the last row), nnz < 2^31.  fmt may
 * be NULL (CSR).  A SELL copy that would need 2^31 or more stored slots gives
 * SKR_E_UNSUPPORTED. */
int skr_matrix_create(skr_context* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                      const int32_t* col_idx, const void* values, int32_t dtype, int32_t mem,
                      const skr_format_opts* fmt, skr_matrix** out);
/* Replace the values of A (same pattern) and refresh A^H, SELL and FP32 copies. */
int skr_matrix_update_values(skr_matrix* A, const void* values, int32_t mem);
int skr_matrix_destroy(skr_matrix* A);
/* Padding ratio of the SELL copy (stored slots / nnz), or 0 for CSR. */
double skr_matrix_sell_padding(const skr_matrix* A);

/* Solve A X = B (adjoint = 0) or A^H X = B (adjoint = 1) for s right-hand sides
 * with the given method.  B, X: n x s row-major with leading dimensions ldb, ldx,
 * both in `mem`; X is the initial guess on entry unless opts->zero_x0 and the
 * last iterate on return.  opts may be NULL (defaults).  1 <= s <= 32. */
int skr_solve(skr_context* ctx, const skr_matrix* A, int32_t s, const void* B, int64_t ldb,
              void* X, int64_t ldx, int32_t mem, int32_t method, const skr_opts* opts,
              int32_t adjoint, skr_result* res);

/* Y = op(A) X for an n x s block (op = A, or A^H when adjoint = 1), rows
 * row-major with leading dimensions ldx, ldy; the kernel every solver iteration
 * uses.  X and Y in `mem`. */
int skr_spmm(skr_context* ctx, const skr_matrix* A, int32_t s, const void* X, int64_t ldx,
             void* Y, int64_t ldy, int32_t mem, int32_t adjoint);

/* Right no-fill ILU preconditioner (Section 5.2 preconditions Examples 1-3
 * with it): A = L U - E with L unit lower and U upper triangular on A's
 * sparsity pattern and (L U)_ij = a_ij there (ILU(0), row-wise elimination
 * that drops every update outside the pattern).  Factored on the host from A's
 * current values, then L, U, U^H and L^H go to device memory with their rows
 * grouped into dependency levels for the triangular solves.  The factors stay
 * with A until skr_matrix_update_values (which drops them) or destroy; calling
 * this again refactors.  Needs every diagonal entry stored; a missing diagonal
 * or a zero pivot returns SKR_E_INVALID and leaves A without factors. */
int skr_matrix_ilu0(skr_context* ctx, skr_matrix* A);

/* Y = M^-1 Z (adjoint = 0) or Y = M^-H Z (adjoint = 1), M = L U from
 * skr_matrix_ilu0: two level-scheduled triangular solves over an n x s block,
 * rows row-major with leading dimensions ldz, ldy, both in `mem`.  Z and Y may
 * be the same device block when ldz = ldy = s.  SKR_E_INVALID when A has no
 * factors. */
int skr_precond_apply(skr_context* ctx, const skr_matrix* A, int32_t s, const void* Z, int64_t ldz,
                      void* Y, int64_t ldy, int32_t mem, int32_t adjoint);

/* Sampled dense-dense product on A's pattern (the gradient with respect to A's
 * stored values of X = A^{-1} B is this with G = A^{-H} dL/dX and scale = -1):
 *     out[k] = scale * sum_c G[i_k, c] * conj(X[j_k, c]),  k = 0..nnz-1,
 * in A's CSR order.  G, X: n x s row-major (leading dimension s); out: nnz
 * values of A's dtype.  All in `mem`. */
int skr_sddmm(skr_context* ctx, const skr_matrix* A, int32_t s, const void* G, const void* X,
              void* out_vals, double scale, int32_t mem);

/* Thin QR of an n x s block, Z = Q C with diag(C) > 0 (CholeskyQR2 on the
 * device; used for the residual QR of Section 4 and the preprocessing of
 * Section 5).  Z, Q: n x s row-major, leading dimension s, in `mem`; C: s x s
 * row-major host array.  1 <= s <= 32 and s <= n <= 2^31 - 2^20.  Returns
 * SKR_BREAKDOWN if Z is numerically rank deficient even after the shifted
 * first pass. */
int skr_block_qr(skr_context* ctx, int64_t n, int32_t s, int32_t dtype, const void* Z, void* Q,
                 double* C, int32_t mem);

/* skr_block_qr without any device-memory allocation, for callers that cannot
 * allocate device memory: tight serving loops and harnesses that forbid
 * allocation (it synchronises the context's stream to return C, so it is not
 * for use under stream capture).  The same thin QR, Z = Q C, by the same
 * kernels as skr_block_qr (results identical to it), with its control block,
 * coefficient slots and reduction partials in a static device array of the
 * library (9 MiB per device, held until the process ends) instead of
 * library-allocated memory.  Z and Q: device memory, n x s row-major with
 * leading dimension s (Q may equal Z); C: s x s row-major host array (complex
 * values interleaved).  Limits: 1 <= s <= 16 and s <= n <= 2^31 - 2^20; larger
 * s gives SKR_E_INVALID (use skr_block_qr).  Every call on one device shares
 * that array and leaves its contents behind, so calls that overlap on one
 * device (two host threads or two streams) race: serialise them.  The caller
 * allocates Q.  Returns SKR_BREAKDOWN like skr_block_qr. */
int skr_block_qr_noalloc(skr_context* ctx, int64_t n, int32_t s, int32_t dtype, const void* Z, void* Q,
                         double* C);

#ifdef __cplusplus
}
#endif

#endif /* SKRYLOV_H */

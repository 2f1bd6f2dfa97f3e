/*
 * msc.h -- multishift conjugate gradient on MI355X (gfx950), C ABI.
 *
 * Solves the family of shifted systems (A + sigma_k I) x_k = b, k = 0..ns-1, for a
 * sparse Hermitian positive-definite A (paper: Section 2, eq. linprob) with one Krylov
 * sequence shared by all shifts (Section 2, Algorithm 1, with the shifted constants
 * re-derived from the collinearity of the shifted residuals).  A is either M^H M for a
 * caller-supplied complex sparse M (the lattice fermion case) or given directly.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are interleaved (re, im) pairs of doubles: a "complex128 array of
 *   length n" is 2n doubles.  Device pointers are HIP device addresses (for example a
 *   torch tensor's data_ptr()); host pointers are ordinary host memory.
 * - `stream` is a hipStream_t passed as void*; NULL means the null stream.  Every call
 *   is stream-ordered with respect to the caller's other work on that stream; calls
 *   that return results to the host (status, info) synchronise that stream.
 * - The caller owns every buffer it passes and keeps it alive for the duration of the
 *   call.  The library owns everything reachable from an msc_op and frees it in
 *   msc_op_destroy.
 * - No call throws.  Each returns an msc_status; on failure msc_last_error() returns a
 *   thread-local message describing the last failure of the calling thread.
 * - An msc_op is not thread safe: one call at a time per op.
 */
#ifndef MSC_H
#define MSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msc_op_s* msc_op;  /* opaque operator handle, library-owned */
typedef void* msc_stream;         /* a hipStream_t */

typedef enum {
    MSC_OK = 0,
    MSC_ENOTCONV = 1,      /* result written, tolerance not reached within max_iter   */
    MSC_EINVAL = -1,       /* invalid argument (null pointer, size, CSR structure)    */
    MSC_ENOMEM = -2,       /* device or host allocation failed                        */
    MSC_EHIP = -3,         /* a HIP runtime call failed                                */
    MSC_EBREAKDOWN = -4    /* p^H (A + sigma_0) p <= 0 or NaN: A + sigma_min not PD    */
} msc_status;

typedef enum {
    MSC_A_MHM = 0,         /* the caller passes M; A = M^H M                           */
    MSC_A_HERM = 1,        /* the caller passes A itself (Hermitian positive definite) */
    MSC_A_GENERAL = 2      /* the caller passes any A (msc_solve_bicgstab only)        */
} msc_op_kind;

typedef enum {
    MSC_PREC_FP64 = 0,     /* complex128 storage and arithmetic throughout            */
    MSC_PREC_MIXED = 1     /* complex64 operator and Krylov vectors, FP64 reductions,
                              FP64 shift recurrences, complex128 solutions, FP64
                              reliable updates and per-shift FP64 refinement          */
} msc_prec;

/* Matrix storage read by the SpMVs of the multishift iteration.  At creation the
 * library also builds a sliced ELLPACK copy (64-row slices, one row per lane, diagonal
 * held apart) when its padding stays below half the entry count, and gives it 16-bit
 * column offsets (from a 32-bit base per slice column and entry position) when every
 * such column's entries span less than 65536 columns.  AUTO uses the copy when it
 * exists, with the narrow columns when they exist; SELL requires the copy (MSC_EINVAL
 * otherwise) and reads the narrow columns when they exist; SELL32 requires the copy and
 * reads its 32-bit columns; CSR forces the CSR kernels. */
typedef enum {
    MSC_FORMAT_AUTO = 0,
    MSC_FORMAT_CSR = 1,
    MSC_FORMAT_SELL = 2,
    MSC_FORMAT_SELL32 = 3,
    MSC_FORMAT_STENCIL = 4   /* operators from msc_op_create_staggered only: the
                                iteration's two operator halves read the links instead of
                                a stored matrix (AUTO picks this for such operators)    */
} msc_format;

/* Solver parameters; fill with msc_params_default() and override fields. */
typedef struct {
    double tol;              /* relative residual target |b-(A+s_k)x_k| <= tol |b|  (1e-10) */
    int32_t max_iter;        /* iteration limit of the multishift sequence           (10000) */
    int32_t prec;            /* msc_prec                                     (MSC_PREC_FP64) */
    int32_t reliable_every;  /* mixed: FP64 true-residual replacement period        (50)    */
    int32_t freeze;          /* stop updating shifts whose residual has converged    (1)    */
    int32_t refine;          /* mixed: refine shifts above tol after the sequence   (1)    */
    int32_t poll_every;      /* iterations queued between host convergence polls    (16)   */
    double switch_tol;       /* mixed: the sequence runs in FP64 until the driving
                                residual reaches switch_tol |b|, then in complex64 (3e-5) */
    int32_t refine_max_iter; /* iteration limit of each refinement system          (10000) */
    int32_t lanes;           /* lanes per CSR row, 0 = automatic                    (0)    */
    int32_t verify;          /* compute FP64 true residuals at the end              (1)    */
    int32_t timing;          /* time the iteration kernels with HIP events on the first
                                max(2, update_steps) of every timing iterations
                                (both phases of a mixed solve, reported apart; at
                                most 256 samples, at most 128 of them in the FP64
                                phase of a mixed solve), 0 = off                  (0)    */
    int32_t max_grid;        /* cap on workgroups per iteration kernel (<= 2048),
                                0 = automatic                                       (0)    */
    int32_t format;          /* msc_format: matrix copy the iteration SpMVs read     (0)    */
    double mixed_margin;     /* mixed: the sequence runs until its recursive residuals
                                reach mixed_margin * tol (0 < margin <= 1), so that the
                                complex64 drift leaves few shifts above tol     (0.7)  */
    int32_t update_steps;    /* 1..8: consecutive steps of the all-shift update folded
                                into one pass over x_0, x_k and p_k (the heads between
                                defer theirs); same recurrences, 1/update_steps of the
                                traffic of those vectors. 1: one step per iteration. The
                                batched solve folds at most 4 (larger values act
                                as 4 there)                                     (8)    */
    int32_t sweep;           /* order of the rows the iteration kernels visit: 0 (auto)
                                follows the operator's lattice structure where one was
                                found at creation (planes and slabs of the staggered
                                lattice, from the links or from a stored matrix's
                                columns), so that each XCD works on neighbouring rows
                                at once; 1 = one contiguous range per workgroup   (0)    */
} msc_params;

/* Per-solve report.  Array members are caller-owned host arrays of length ns (or
 * NULL when not wanted), indexed in the caller's shift order. */
typedef struct {
    int32_t iters;           /* multishift iterations performed                         */
    int32_t refine_iters;    /* refinement iterations (max over refined shifts)         */
    int32_t n_reliable;      /* reliable updates performed                              */
    int32_t n_refined;       /* shifts that needed refinement                           */
    double* true_rel_res;    /* [ns] |b - (A+sigma_k) x_k| / |b| in FP64                */
    int32_t* freeze_iter;    /* [ns] iteration at which shift k froze, -1 if never      */
    double seconds;          /* wall time of the call                                   */
    double alg_bytes;        /* algorithmic HBM bytes moved by the call's kernels       */
    double kernel_ms[3];     /* with timing on: summed durations of the sampled launches,
                                milliseconds: [0] the head (the previous iteration's
                                all-shift update fused with the first operator half),
                                [1] K2 (second half + residual update), [2] the separate
                                all-shift update kernel of the CSR path (0 otherwise)  */
    int32_t kernel_samples;  /* number of sampled iterations behind kernel_ms          */
    int32_t iters_fp64;      /* iterations run in FP64 (all of them for MSC_PREC_FP64)  */
    double kernel_bytes[3];  /* algorithmic HBM bytes of the same sampled launches, summed
                                like kernel_ms (each array touched once, gathers once;
                                the head's depends on the shifts active at its iteration) */
    double fp64_kernel_ms[3];    /* mixed solve: kernel_ms of the launches sampled in its
                                    FP64 phase (kernel_ms holds its complex64 phase);
                                    0 otherwise                                        */
    double fp64_kernel_bytes[3]; /* mixed solve: kernel_bytes of the same launches       */
    int32_t fp64_kernel_samples; /* mixed solve: sampled iterations of the FP64 phase    */
    int32_t reserved;            /* 0                                                    */
} msc_info;

/* Fill *p with the defaults listed above. */
void msc_params_default(msc_params* p);

/* Library version string. */
const char* msc_version(void);

/* Message describing the calling thread's last failure ("" if none). */
const char* msc_last_error(void);

/*
 * Create an operator from a CSR matrix held in device memory (Fig. 1 of the paper
 * builds the matrix, copies it to the device, then calls the solver; here the CSR is
 * already resident).  For MSC_A_MHM the matrix is M and the library builds M^H
 * (conjugate transpose with sorted columns) on the device; for MSC_A_HERM and
 * MSC_A_GENERAL it is A.
 *   d_rowptr : int64[n+1], non-decreasing, d_rowptr[0] = 0, d_rowptr[n] = nnz
 *   d_col    : int32[nnz], each in [0, n)
 *   d_vals   : complex128[nnz] (2*nnz doubles)
 * The arrays are copied; the caller may free them after the call returns.  The
 * structure is validated on the device (MSC_EINVAL on violation).  n >= 1 and
 * nnz < 2^31 are required.
 */
msc_status msc_op_create_csr(msc_op* out, int32_t kind, int64_t n, int64_t nnz,
                             const int64_t* d_rowptr, const int32_t* d_col,
                             const double* d_vals, msc_stream stream);

/* Replace the values of the operator's matrix (same pattern, same entry order as at
 * creation, complex128[nnz] on the device) -- for example after new gauge links.
 * Operators made by msc_op_create_staggered take msc_op_update_links instead
 * (MSC_EINVAL here). */
msc_status msc_op_update_values(msc_op op, const double* d_vals, msc_stream stream);

/*
 * Create the staggered fermion operator M = m I + D (A = M^H M) of a periodic 4-D
 * lattice from its gauge links, for a matrix-free iteration (paper: Section 3 leaves
 * room for a custom linear operator kernel in place of the library's stored matrix).
 *   dims    : host int32[4], extents L0..L3, each >= 3, 75 * L0 L1 L2 L3 < 2^31
 *   mass    : m
 *   d_links : device complex128[4][V][3][3] (V = L0 L1 L2 L3): U_mu(x) for direction mu,
 *             site x = x0 + L0 (x1 + L1 (x2 + L2 x3)), row-major 3x3
 * Row 3 s + c is colour c of site s, and
 *   D[x, y] = sum_mu eta_mu(x)/2 [ U_mu(x) delta(y, x+mu) - U_mu(x-mu)^H delta(y, x-mu) ],
 *   eta_0 = 1, eta_mu(x) = (-1)^(x0 + ... + x_{mu-1}).
 * The library keeps eta/2 U in complex128 and complex64 (the links are copied; the
 * caller may free them) and also builds the equivalent scalar CSR of M (25 sorted
 * entries per row) with every copy msc_op_create_csr makes, which the reliable
 * updates, the verification, the refinement, the adjoint, msc_op_apply and the
 * batched solve use.  The multishift iteration applies M and M^H from the links
 * (msc_params.format AUTO or STENCIL).  MSC_EINVAL on an extent below 3, an oversized
 * lattice, a non-finite mass or a null pointer.
 */
msc_status msc_op_create_staggered(msc_op* out, const int32_t* dims, double mass,
                                   const double* d_links, msc_stream stream);

/* New gauge links for an operator made by msc_op_create_staggered (same layout as at
 * creation): the link copies and every stored copy of M are rebuilt. */
msc_status msc_op_update_links(msc_op op, const double* d_links, msc_stream stream);

/* Set the shifts sigma_k (host array, any order, duplicates allowed, 1 <= ns <= 64).
 * The smallest shift drives the Krylov sequence; A + sigma_min must be positive
 * definite. */
msc_status msc_op_set_shifts(msc_op op, const double* h_sigma, int32_t ns);

/* Query the operator: any output pointer may be NULL. */
msc_status msc_op_query(msc_op op, int64_t* n, int64_t* nnz, int32_t* ns, int32_t* kind);

/* Storage the operator holds besides its CSR matrix (see msc_format): *sell = 1 when the
 * sliced ELLPACK copy was built; *narrow has bit 0 set when the copy of the operator's
 * matrix has 16-bit column offsets and, for MSC_A_MHM, bit 1 when the copy of M^H has
 * them; bit 2 when an operator from msc_op_create_staggered found every link in SU(3)
 * (|U U^H - I| and |det U - 1| <= 1e-12) and its iteration reads the links' first two
 * rows, rebuilding the third (a third less link traffic).  Either pointer may be NULL. */
msc_status msc_op_storage(msc_op op, int32_t* sell, int32_t* narrow);

/*
 * Apply the operator (no solve): d_out = (A + shift I) d_in for complex128 vectors of
 * length n in device memory, computed with the FP64 (prec = MSC_PREC_FP64) or the
 * complex64 (prec = MSC_PREC_MIXED, inputs and outputs still complex128) copy of the
 * matrix.  This is the matrix-vector product of Algorithm 1 on its own.
 */
msc_status msc_op_apply(msc_op op, int32_t prec, const double* d_in, double* d_out,
                        double shift, msc_stream stream);

/*
 * msc_op_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same product,
 * d_out = (A + shift I) d_in, computed by the same kernels, with its temporaries in a
 * fixed device array of 64 MiB that the library keeps on each GPU it runs on until the
 * process ends.  Nothing is allocated, not even on the first call.  Limits: n <= 2^21
 * for MSC_PREC_FP64 with MSC_A_MHM, n <= 2^22 otherwise; larger operators get
 * MSC_EINVAL (use msc_op_apply).  The operator's device must be the current device
 * (MSC_EINVAL otherwise).  The call only queues work on `stream` and returns without
 * synchronising; the result is ready when the stream reaches that point.  Every call on
 * one GPU shares that GPU's array, so calls that may overlap on one GPU (different
 * streams, or different threads) race and must be ordered by the caller.
 */
msc_status msc_op_apply_noalloc(msc_op op, int32_t prec, const double* d_in, double* d_out,
                                double shift, msc_stream stream);

/*
 * The multishift solve (Algorithm 1).  d_b: complex128[n]; d_x: complex128[ns*n],
 * shift-major (x_k occupies d_x[2*k*n .. 2*(k+1)*n)) in the caller's shift order.
 * x starts from zero (the method requires it).  Blocks until done.  Returns MSC_OK when
 * every shift meets tol (with verify on: in FP64 true residual), MSC_ENOTCONV when
 * not (x still holds the final iterates and info is filled), MSC_EBREAKDOWN on a
 * breakdown.  info may be NULL.
 */
msc_status msc_solve(msc_op op, const double* d_b, double* d_x, const msc_params* params,
                     msc_info* info, msc_stream stream);

/*
 * Adjoint of msc_solve for a real loss L(x_0..x_{ns-1}).  Given the forward solutions
 * d_x (complex128[ns*n]) and d_g = dL/dx (complex128[ns*n], torch's convention
 * dL/dRe + i dL/dIm), computes y_k = (A + sigma_k)^{-1} g_k and
 *   d_grad_b[n]      = sum_k y_k
 *   d_grad_vals[nnz] = gradient with respect to the stored values, in creation order:
 *       A = M^H M : -sum_k [ (M y_k)_i conj(x_k)_j + (M x_k)_i conj(y_k)_j ]
 *       A given  : -sum_k (y_k)_i conj(x_k)_j                 for entry e = (i, j).
 * When every g_k is a real multiple of one vector the y_k come from one multishift
 * solve; otherwise from one batched single-shift solve per shift.  Either gradient
 * pointer may be NULL to skip it.  info (may be NULL) reports the adjoint solve.
 */
msc_status msc_solve_adjoint(msc_op op, const double* d_g, const double* d_x,
                             double* d_grad_b, double* d_grad_vals,
                             const msc_params* params, msc_info* info, msc_stream stream);

/*
 * Multishift BiCGStab (BiCGStab-M, the paper's second shifted solver: Sections 1 and 3)
 * for a general, possibly non-Hermitian A: (A + sigma_k I) x_k = b for every shift from
 * one BiCGStab sequence of the smallest shift, shadow vector b.  The operator must be of
 * kind MSC_A_GENERAL or MSC_A_HERM (A as given; MSC_EINVAL for MSC_A_MHM, whose A is
 * Hermitian positive definite: use msc_solve).  FP64 only (params->prec must be
 * MSC_PREC_FP64).  d_b, d_x as for msc_solve.  Each shift stops being advanced once its
 * recursive residual (a multiple of the driving one) is below tol |b|; the sequence
 * halts when every shift has stopped.  With verify on, the FP64 true residuals are
 * reported and decide MSC_OK / MSC_ENOTCONV; MSC_EBREAKDOWN when w^H v, t^H t or rho
 * vanishes, 1 + s omega = 0 for a shift, or a value is not finite.  info (may be NULL)
 * reports iters, true_rel_res and freeze_iter; timing fields are zero.
 */
msc_status msc_solve_bicgstab(msc_op op, const double* d_b, double* d_x,
                              const msc_params* params, msc_info* info, msc_stream stream);

/*
 * The multishift solve for a real symmetric positive-definite A (paper: Section 4,
 * Table 1 -- the paper's benchmark matrix, the 2-D 5-point Poisson operator, is real):
 * the same recurrences as msc_solve on real vectors and a real copy of the sliced ELLPACK
 * matrix, half the bytes of the complex path.  The operator must be of kind MSC_A_HERM,
 * have its sliced copy (msc_op_storage), and every stored imaginary part must be 0
 * (checked on the first call; MSC_EINVAL otherwise).
 *   d_b : device double[n] (real)
 *   d_x : device double[ns*n], shift-major, caller's shift order
 * params->prec: MSC_PREC_FP64 (double storage and arithmetic) or MSC_PREC_MIXED (float
 * vectors and matrix, FP64 reductions and shift scalars; meant for moderate tolerances
 * such as the paper's 1e-5: no reliable update or refinement).  x_k is kept in FP64.
 * Returns MSC_OK when the driving residual reached tol and (with verify) every shift's
 * FP64 true residual is below tol, MSC_ENOTCONV otherwise, MSC_EBREAKDOWN on a breakdown.
 * info: iters, true_rel_res, freeze_iter, alg_bytes; timing fields are zero.
 */
msc_status msc_solve_real(msc_op op, const double* d_b, double* d_x, const msc_params* params,
                          msc_info* info, msc_stream stream);

/*
 * A different right-hand side per shift, (A + sigma_k I) x_k = b_k (paper: Section 5,
 * eq. linprobgen), for kinds MSC_A_MHM and MSC_A_HERM with distinct shifts.  The
 * library forms, with ns - 1 products with A in FP64, initial guesses x0_k that leave
 * every shifted system the same residual r0 (from the Newton interpolant of the b_k
 * over the shifts), solves (A + sigma_k) d_k = r0 for all k with one multishift solve
 * (params->prec as for msc_solve) stopped at tol min_k |b_k| / |r0|, sets
 * x_k = x0_k + d_k, and checks every shift against its own b_k in FP64, continuing the
 * ones above tol with the batched CG (up to refine_max_iter iterations).  The guesses
 * grow with the spread of the shifts (the interpolant is evaluated far outside their
 * interval); when tol min_k |b_k| / |r0| falls below 1e-14, or the shifts repeat, they
 * are dropped and every shift is solved from zero by the batched CG.
 *   d_B : complex128[ns*n], shift-major in the caller's shift order (b_k at 2*k*n)
 *   d_x : complex128[ns*n], same layout
 * info (may be NULL): iters = multishift iterations (0 when the guesses were dropped or
 * already exact), refine_iters = batched CG iterations, true_rel_res = FP64
 * |b_k - (A + sigma_k) x_k| / |b_k|.  Returns MSC_OK when every shift meets tol,
 * MSC_ENOTCONV otherwise, MSC_EBREAKDOWN on a breakdown.
 */
msc_status msc_solve_multi_rhs(msc_op op, const double* d_B, double* d_x,
                               const msc_params* params, msc_info* info, msc_stream stream);

/*
 * Many independent multishift solves in one launch sequence: system s uses ops[s]
 * (each with its own shifts) and nrhs[s] right-hand sides at d_b[s]
 * (complex128[nrhs[s]*n_s], rhs-major); solutions go to d_x[s]
 * (complex128[nrhs[s]*ns_s*n_s], rhs-major then shift-major).  ops, nrhs, d_b and d_x
 * are host arrays of length nsys.  info, if not NULL, is a host array with one entry
 * per (system, rhs) pair in order.
 */
msc_status msc_solve_batched(int32_t nsys, const msc_op* ops, const int32_t* nrhs,
                             const double* const* d_b, double* const* d_x,
                             const msc_params* params, msc_info* info, msc_stream stream);

/* Release an operator and everything it owns.  NULL is ignored. */
void msc_op_destroy(msc_op op);

#ifdef __cplusplus
}
#endif

#endif /* MSC_H */

/*
 * fmap.h -- C ABI of libfmap, a gfx950 (MI355X) implementation of the
 * regularised least-squares functional-map solve of "DeepShapeMatchingKit"
 * (Sec. 3.1, "Batched Functional Map Solver", Eqs. (1)-(9)).
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless marked [host].  Arrays are dense,
 *     row-major, contiguous, with the shapes written next to them.
 *   - Sizes are int64_t; k, d, n >= 1.  `stream` is a hipStream_t (NULL means
 *     the default stream).  All work is enqueued on `stream` and the call
 *     returns without synchronising.
 *   - The caller owns every buffer, workspaces included.  The library never
 *     allocates device memory inside these calls.  A workspace must stay
 *     untouched until the work enqueued on `stream` has finished.
 *   - Argument errors are detected on the host before anything is enqueued and
 *     returned as an fmap_status; nothing is launched then.  Numerical failures
 *     are reported asynchronously per row system through `info` (LAPACK
 *     convention, see fmap_solve) and the affected row of the output is NaN.
 *   - Entry points are reentrant; calls that share a workspace must be ordered
 *     on one stream.
 *
 * Notation: for a shape pair, x is the source and y the target.  Phi_x [n_x][k_x]
 * is the Laplace-Beltrami eigenbasis of x, orthonormal under the lumped vertex
 * mass M_x [n_x] (Phi_x^T diag(M_x) Phi_x = I), mu_x [k_x] its eigenvalues, F_x
 * [n_x][d] per-vertex features; the same for y.  The functional map C [k_y][k_x]
 * maps x-coefficients to y-coefficients, C A ~ B.
 */
#ifndef FMAP_H
#define FMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fmap_status;
enum {
    FMAP_OK = 0,
    FMAP_ERR_NULL = 1,        /* a required pointer is NULL                          */
    FMAP_ERR_SHAPE = 2,       /* a size is out of range or sizes disagree            */
    FMAP_ERR_VALUE = 3,       /* a scalar option is out of range (gamma, threshold)  */
    FMAP_ERR_DTYPE = 4,       /* unknown element type                                */
    FMAP_ERR_WORKSPACE = 5,   /* workspace NULL or smaller than required             */
    FMAP_ERR_UNSUPPORTED = 6, /* valid request this build does not implement         */
    FMAP_ERR_HIP = 7          /* a HIP runtime call failed                           */
};

/* Penalty mask of the commutativity term (Eq. (3) and the mask defined after
 * Eq. (4)); D [k_y][k_x], row i follows mu_y,i and column j follows mu_x,j.
 *   LAPLACIAN: D_ij = (mu_y,i - mu_x,j)^2.
 *   RESOLVENT: the resolvent mask the paper cites as the structured
 *     alternative.  Eigenvalues are clipped at 0 and divided by
 *     s = max(max mu_x, max mu_y) of the pair; with a = (mu/s)^gamma the
 *     resolvent 1/(a - i) has real part a/(1+a^2) and imaginary part
 *     1/(1+a^2); D_ij is the squared modulus of the difference of the two
 *     resolvent values.  gamma > 0.                                             */
enum { FMAP_MASK_LAPLACIAN = 0, FMAP_MASK_RESOLVENT = 1 };

/* Element type of the basis / feature arrays read by the projections. */
enum { FMAP_F32 = 0, FMAP_BF16 = 1 };

/* Library facts. */
int32_t fmap_abi_version(void);       /* increments on any incompatible change        */
int32_t fmap_max_k(void);             /* largest k_x, k_y accepted by fmap_solve      */
const char *fmap_status_str(fmap_status s); /* static string, never NULL            */

/* ------------------------------------------------------------------------ */
/* Spectral projection, Eq. (1).  The pseudo-inverse of an M-orthonormal basis */
/* in the mass inner product is Phi^T diag(M), so for every batch item b       */
/*     A[b] = Phi[b]^T diag(mass[b]) F[b].                                     */
/* phi [batch][n][k] and feat [batch][n][d] in `in_dtype` (FMAP_F32: float,     */
/* FMAP_BF16: bfloat16 bit patterns, uint16), mass [batch][n] float, A          */
/* [batch][k][d] float.  Products are accumulated in float32 (matrix cores);    */
/* the sum over vertices is split into chunks whose partial sums are added in  */
/* a fixed order, so results are deterministic.                               */
/* workspace: fmap_project_workspace_bytes(...) bytes (may be 0, then NULL ok). */
/* ------------------------------------------------------------------------ */
size_t fmap_project_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t in_dtype);
fmap_status fmap_project(const void *phi, const float *mass, const void *feat, int32_t in_dtype, int64_t batch,
                         int64_t n, int64_t k, int64_t d, float *A, void *workspace, size_t workspace_bytes,
                         void *stream);

/* For callers that cannot allocate device memory (code under graph capture,  */
/* tight serving loops, harnesses that forbid allocation): fmap_project with  */
/* no workspace argument.  Its split-K partial sums live in a library-owned    */
/* device array of FMAP_NOALLOC_SCRATCH_BYTES (32 MiB) per device, held from   */
/* the library's load until the process ends.  Same arguments, kernels and     */
/* results as fmap_project.  Returns FMAP_ERR_WORKSPACE when                   */
/* fmap_project_workspace_bytes(batch, n, k, d, in_dtype) exceeds that size,   */
/* FMAP_ERR_HIP if the array's device address cannot be obtained.  It calls no */
/* allocator.  All calls on one device share the array: calls that overlap in  */
/* time on one device (different streams or threads) race and must not be     */
/* issued.                                                                     */
#define FMAP_NOALLOC_SCRATCH_BYTES (32u << 20)
fmap_status fmap_project_noalloc(const void *phi, const float *mass, const void *feat, int32_t in_dtype,
                                 int64_t batch, int64_t n, int64_t k, int64_t d, float *A, void *stream);

/* Adjoint of the projection (the chain rule of Eq. (1)):                      */
/*     dF[b] = diag(mass[b]) Phi[b] dA[b].                                      */
/* phi [batch][n][k] in `phi_dtype`, mass [batch][n], dA [batch][k][d] float,    */
/* dF [batch][n][d] float (overwritten).                                         */
fmap_status fmap_project_backward(const void *phi, const float *mass, int32_t phi_dtype, const float *dA,
                                  int64_t batch, int64_t n, int64_t k, int64_t d, float *dF, void *stream);

/* Eq. (1) with the projector given directly.  The paper writes A = Phi^+ F with */
/* the pseudo-inverse; a caller holding Phi^+ ([k][n] per shape) passes its      */
/* transpose P = (Phi^+)^T [batch][n][k] (Phi^+ read column-major) in `in_dtype`,  */
/* feat [batch][n][d] in the same dtype:  A[b] = P[b]^T F[b] [batch][k][d] float. */
/* The backward is dF[b] = P[b] dA[b].  Same kernels as fmap_project with unit   */
/* vertex weights, which the call writes into the workspace (its first           */
/* batch * n floats; the backward needs only those).                             */
size_t fmap_project_pinv_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t in_dtype);
fmap_status fmap_project_pinv(const void *pinv_t, const void *feat, int32_t in_dtype, int64_t batch, int64_t n,
                              int64_t k, int64_t d, float *A, void *workspace, size_t workspace_bytes, void *stream);
fmap_status fmap_project_pinv_backward(const void *pinv_t, int32_t pinv_dtype, const float *dA, int64_t batch,
                                       int64_t n, int64_t k, int64_t d, float *dF, void *workspace,
                                       size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Regularised solve, Eqs. (2)-(9).  For every pair p and row i < k_y:          */
/*     (A A^T + lambda[p] diag(D_i)) c_i = A b_i            (Eq. (5))          */
/* with A = A[p] [k_x][d], b_i the i-th row of B[p] [k_y][d], D the mask of the   */
/* pair; C[p] row i = c_i^T (Eq. (7)).  Each row system is factorised by        */
/* Cholesky in float32; all k_y systems of all pairs run in one batched launch  */
/* (the rows are a batch dimension, Eq. (8)), without materialising the         */
/* [pairs][k_y][k_x][k_x] left-hand side of Eq. (9).                            */
/*                                                                            */
/* evals_x [pairs][k_x], evals_y [pairs][k_y], lambda [pairs] (all float).       */
/* C [pairs][k_y][k_x] float (written).                                          */
/* factors: NULL, or [pairs][k_y][k_x (k_x+1)/2] float receiving every row's     */
/*   Cholesky factor L (S_i = L L^T) in LAPACK lower packed column-major order: */
/*   L(r, c), r >= c, at index c*k_x - c*(c-1)/2 + (r - c).  fmap_solve_backward */
/*   can reuse them instead of refactorising.                                   */
/* info [pairs][k_y] int32 (written): 0 ok; j > 0 the leading minor of order j   */
/*   of S_i is not positive (or not finite); -1 lambda[p] negative or not       */
/*   finite; -2 resolvent normaliser not positive.  Failed rows of C are NaN.   */
/* refine_steps: 0, or the number of iterative-refinement steps (residual of     */
/*   the row system accumulated in float64, correction solved with the float32   */
/*   factor).                                                                   */
/* cond_fp64_threshold: when refine_steps > 0, pairs whose estimated 1-norm     */
/*   condition number of A A^T exceeds it form A A^T in float64 before the       */
/*   float32 factorisation; <= 0 disables the estimate.                         */
/* cond_est: NULL, or [pairs] float receiving that estimate (only written when  */
/*   the estimate runs).                                                         */
/* workspace: fmap_solve_workspace_bytes(pairs, k_x, k_y, d) bytes.              */
/* ------------------------------------------------------------------------ */
size_t fmap_solve_workspace_bytes(int64_t pairs, int64_t kx, int64_t ky, int64_t d);
size_t fmap_factor_floats(int64_t kx, int64_t ky); /* floats of `factors` per pair */
fmap_status fmap_solve(const float *A, const float *B, const float *evals_x, const float *evals_y,
                       const float *lambda, int32_t mask_kind, float gamma, int64_t pairs, int64_t kx, int64_t ky,
                       int64_t d, int32_t refine_steps, float cond_fp64_threshold, float *C, float *factors,
                       int32_t *info, float *cond_est, void *workspace, size_t workspace_bytes, void *stream);

/* Reverse mode of fmap_solve (the paper states no gradients; this is the exact */
/* derivative of the minimiser).  With G = dC [pairs][k_y][k_x] and V the rows   */
/* v_i = S_i^{-1} g_i (S_i is symmetric):                                        */
/*     dB = V A,   dA = V^T B - (V^T C + C^T V) A,   dlambda = -sum_ij V_ij D_ij C_ij */
/* A, B, C, evals, lambda and the mask are those of the forward call; C is its  */
/* output.  factors: the forward's `factors` (reused), or NULL to refactorise   */
/* every row system (no factor storage needed).                                 */
/* dA [pairs][k_x][d], dB [pairs][k_y][d] float (overwritten); dlambda: NULL or  */
/* [pairs] float; info: NULL or [pairs][k_y] int32 as in fmap_solve.             */
/* workspace: fmap_solve_workspace_bytes(pairs, k_x, k_y, d) bytes.              */
fmap_status fmap_solve_backward(const float *dC, const float *A, const float *B, const float *C,
                                const float *evals_x, const float *evals_y, const float *lambda, int32_t mask_kind,
                                float gamma, int64_t pairs, int64_t kx, int64_t ky, int64_t d, const float *factors,
                                float *dA, float *dB, float *dlambda, int32_t *info, void *workspace,
                                size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Maps at several spectral resolutions from one projection (multi-resolution   */
/* pipelines project once onto the first k eigenfunctions).  Resolution r is    */
/* the fmap_solve problem restricted to the first kxs[r] source and kys[r]      */
/* target eigenpairs: the leading rows of A [pairs][kx][d] and B [pairs][ky][d] */
/* and the leading eigenvalues (the mask and the resolvent normaliser are those */
/* of the truncated spectra).  kxs, kys [host, nres entries]: 1 <= kxs[r] <= kx, */
/* 1 <= kys[r] <= ky, 1 <= nres <= 64.  C [host, nres device pointers]:         */
/* C[r] [pairs][kys[r]][kxs[r]] float.  info: NULL, or [host, nres] device      */
/* pointers [pairs][kys[r]] int32, each may be NULL (conventions of fmap_solve). */
/* Forward only, no factors.  workspace:                                        */
/* fmap_solve_resolutions_workspace_bytes(...) bytes (0 for invalid arguments). */
/* ------------------------------------------------------------------------ */
size_t fmap_solve_resolutions_workspace_bytes(int64_t pairs, int64_t kx, int64_t ky, int64_t d, int32_t nres,
                                              const int32_t *kxs, const int32_t *kys);
fmap_status fmap_solve_resolutions(const float *A, const float *B, const float *evals_x, const float *evals_y,
                                   const float *lambda, int32_t mask_kind, float gamma, int64_t pairs, int64_t kx,
                                   int64_t ky, int64_t d, int32_t nres, const int32_t *kxs, const int32_t *kys,
                                   float *const *C, int32_t *const *info, void *workspace, size_t workspace_bytes,
                                   void *stream);

/* ------------------------------------------------------------------------ */
/* Vectorized solve with general commutativity operators (Sec. 3.1: the        */
/* k^2 x k^2 least-squares formulation that the row-wise solve avoids; the     */
/* conclusion names it for non-orthogonal bases, where the operators are not   */
/* diagonal).  Per pair p:                                                     */
/*     C_p = argmin ||C A_p - B_p||_F^2 + lambda[p] ||C X_p - Y_p C||_F^2       */
/* A [pairs][kx][d], B [pairs][ky][d], op_x = X [pairs][kx][kx] (source        */
/* operator), op_y = Y [pairs][ky][ky] (target operator), lambda [pairs], all  */
/* float32 row-major on the device; C [pairs][ky][kx] float32 out.  With       */
/* c = vec(C) (c[i kx + j] = C[i][j]) it solves the normal equations H c = g   */
/* of order n = kx ky by one float32 Cholesky factorisation per pair (H is     */
/* formed in float32 from A A^T, B A^T and the operators).  With diagonal      */
/* operators X = diag(evals_x), Y = diag(evals_y) the result is fmap_solve's   */
/* with the Laplacian mask.  Supported: kx ky <= fmap_max_k() (the k^2 x k^2   */
/* system is for small k), else FMAP_ERR_UNSUPPORTED; pairs <= 2^20.          */
/* info [pairs] int32 out:                                                     */
/* 0; c + 1 if the pivot of vectorized index c = i kx + j is not positive     */
/* (that pair's C is NaN); -1 for a negative or non-finite lambda.  workspace: */
/* fmap_solve_vectorized_workspace_bytes(...) bytes (0 for invalid sizes).     */
/* Forward only.                                                               */
/* ------------------------------------------------------------------------ */
size_t fmap_solve_vectorized_workspace_bytes(int64_t pairs, int64_t kx, int64_t ky, int64_t d);
fmap_status fmap_solve_vectorized(const float *A, const float *B, const float *op_x, const float *op_y,
                                  const float *lambda, int64_t pairs, int64_t kx, int64_t ky, int64_t d, float *C,
                                  int32_t *info, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* DiffusionNet spatial-gradient features (Sec. 3.2), the step upstream of the  */
/* projection.  Per vertex the D channels hold complex gradients z = x + i y,   */
/* interleaved: z [vertices][channels][2] float (x_j, y_j).  With A_re, A_im    */
/* [channels][channels] float ((A z)_c = sum_j A[c][j] z_j):                    */
/*     (A z)_re = A_re x - A_im y                                               */
/*     (A z)_im = A_re y + A_im x   (FMAP_GRADFEAT_A)                           */
/*              = A_re x + A_im y   (FMAP_GRADFEAT_B)                           */
/*     g = x * (A z)_re + y * (A z)_im        g [vertices][channels] float      */
/* Variant A is Re(conj(z) * (A z)), a learned rotation and isotropic scaling   */
/* of each tangent vector; variant B fixes the rotation at +-45 degrees and     */
/* allows anisotropic scaling.  Float32 arithmetic (float32 matrix cores for    */
/* channels in {32, 64, 128, 256} and 16-byte aligned z; a plain kernel         */
/* otherwise).  Forward only.                                                   */
/* ------------------------------------------------------------------------ */
#define FMAP_GRADFEAT_A 0
#define FMAP_GRADFEAT_B 1
fmap_status fmap_gradient_features(const float *z, const float *A_re, const float *A_im, int32_t variant,
                                   int64_t vertices, int64_t channels, float *g, void *stream);

/* ------------------------------------------------------------------------ */
/* Overlap-prediction metrics (Sec. 3.3), for a batch of shapes of uneven size. */
/* Shape s owns vertices [offsets[s], offsets[s+1]) of the concatenated arrays  */
/* scores [total] float and truth [total] uint8 (nonzero = truly overlapping);  */
/* offsets [shapes + 1] int64 (device), nondecreasing from 0 to total (other    */
/* contents give unspecified counts but no out-of-range access).  A vertex is   */
/* predicted overlapping iff its score > threshold (float32; NaN is negative).  */
/* Outputs (device, overwritten): counts [shapes][4] int64 = TP, FP, FN, TN,    */
/* exact; metrics [shapes][7] float = accuracy, precision, recall               */
/* (sensitivity), specificity, IoU, F1 and balanced accuracy (the mean of       */
/* sensitivity and specificity), computed in double from the counts and        */
/* rounded once.  A ratio with a zero denominator is 0; balanced accuracy       */
/* averages the class recalls that are defined (one class only: its recall).   */
/* scores and truth may be NULL when total == 0.                                */
/* ------------------------------------------------------------------------ */
fmap_status fmap_overlap_metrics(const float *scores, const uint8_t *truth, const int64_t *offsets, int64_t shapes,
                                 int64_t total, float threshold, int64_t *counts, float *metrics, void *stream);

/* ------------------------------------------------------------------------ */
/* Uneven batches (shape pairs with different n and k): a plan.                */
/* The rows of all pairs are batch dimensions (Eq. (8)); pairs of equal k are   */
/* grouped, the projections of every shape run as one persistent launch over   */
/* a table of work items, and the whole forward (and backward) pass is         */
/* captured once as a HIP graph that fmap_plan_forward / _backward replay.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *phi_x, *phi_y;      /* [n_x][k], [n_y][k] float32 bases                        */
    const float *mass_x, *mass_y;    /* [n_x], [n_y]                                            */
    const float *feat_x, *feat_y;    /* [n_x][d], [n_y][d]                                      */
    const float *evals_x, *evals_y;  /* [k], [k]                                                */
    const float *lambda;             /* [1] (device; read at every forward)                     */
    float *C;                        /* [k][k] output                                           */
    int32_t *info;                   /* [k] output, as in fmap_solve                            */
    float *A, *B;                    /* [k][d] outputs, or NULL                                 */
    const float *dC;                 /* [k][k] upstream gradient, or NULL (no backward)          */
    float *dF_x, *dF_y;              /* [n_x][d], [n_y][d] backward outputs (with dC)            */
    int64_t n_x, n_y, k;
} fmap_pair;

typedef struct fmap_plan fmap_plan;

/* Builds the plan for `npairs` pairs [host array; the device pointers inside  */
/* are captured and must stay valid while the plan lives; their contents may   */
/* change between replays].  Allocates the plan's device buffers (this call,   */
/* not the replays, allocates).  Autotunes the projection work-item size, the  */
/* persistent grid and the row systems per workgroup by timing candidates on   */
/* `stream`, unless `tune_cache_path` [host, may be NULL] holds a result for   */
/* this workload signature (results are appended to that file).  k <= 319;     */
/* bwd_recompute != 0 refactorises in the backward instead of storing factors. */
/* The plan owns one capture stream and, with several k groups, up to three    */
/* more (default priority) on which the groups' solves are captured as         */
/* parallel graph branches; fmap_plan_destroy releases them.                   */
fmap_status fmap_plan_create(const fmap_pair *pairs, int32_t npairs, int64_t d, int32_t mask_kind, float gamma,
                             int32_t bwd_recompute, const char *tune_cache_path, void *stream, fmap_plan **out);
fmap_status fmap_plan_forward(fmap_plan *plan, void *stream);   /* replays the captured forward  */
fmap_status fmap_plan_backward(fmap_plan *plan, void *stream);  /* replays the captured backward */
/* Tuned parameters: vertices per projection work item, persistent grid size,   */
/* row systems per workgroup of the first group with k <= 64 (4 if there is     */
/* none), and whether they came from the cache (1) or a run.  Any pointer may   */
/* be NULL.                                                                     */
fmap_status fmap_plan_tuning(const fmap_plan *plan, int32_t *chunk, int32_t *grid, int32_t *systems_per_wg,
                             int32_t *from_cache);
/* The plan's k groups, in increasing k: *groups = their number (any pointer   */
/* may be NULL).  For group g (0 <= g < groups; FMAP_ERR_VALUE otherwise):      */
/* its k, its number of pairs, and the row systems per workgroup the tuner     */
/* picked for it (1, 2 or 4 for k <= 64; 1 for the tiled solve of larger k).    */
fmap_status fmap_plan_groups(const fmap_plan *plan, int32_t *groups);
fmap_status fmap_plan_group(const fmap_plan *plan, int32_t g, int32_t *k, int32_t *npairs, int32_t *systems_per_wg);
fmap_status fmap_plan_destroy(fmap_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* FMAP_H */

/*
 * fmap_oracle.c -- plain, slow, double-precision CPU oracle for the regularised
 * functional-map solve of "DeepShapeMatchingKit" (Sec. 3.1, "Batched Functional
 * Map Solver").
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or helper with the GPU library, and the GPU library never calls it.
 *
 * What it computes (all in IEEE double, inputs promoted from whatever the GPU
 * consumed):
 *   - spectral projection, Eq. (1), read as the pseudo-inverse in the mass inner
 *     product:  A = Phi^T diag(M) F                         (oracle_project)
 *   - its adjoint  dF = diag(M) Phi dA                       (oracle_project_backward)
 *   - the penalty mask of the commutativity term, Eq. (3) and the mask
 *     definition after Eq. (4): Laplacian D_ij = (mu_y,i - mu_x,j)^2, or the
 *     resolvent mask the paper cites                         (oracle_mask)
 *   - the minimiser of Eq. (2): the normal equations, Eq. (4), decoupled by
 *     rows, Eqs. (5)-(7): for every row i,
 *        (A A^T + lambda diag(D_i)) c_i = (B A^T)_i^T
 *     each solved by an unblocked Cholesky factorisation     (oracle_solve)
 *   - the reverse-mode derivative of that minimiser with respect to A, B and
 *     lambda (derived; the paper states no gradients)       (oracle_solve_backward)
 *
 * Sizes: C is ky x kx (rows indexed by target eigenvalues, columns by source
 * eigenvalues), A is kx x d, B is ky x d.  All arrays are dense row-major.
 *
 * Failure convention per row system (LAPACK style): info = 0 success; j > 0
 * the leading minor of order j is not positive (or not finite); -1 lambda is
 * negative or not finite; -2 the resolvent normaliser max(mu) is not positive.
 * A failed row of C is set to NaN.
 *
 * Parity pins for every function live in the test suite (closed forms,
 * invariants, a Kronecker brute force, finite differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MASK_LAPLACIAN 0
#define ORACLE_MASK_RESOLVENT 1

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Eq. (1): A = Phi^+ F with Phi^+ = Phi^T diag(M) for an M-orthonormal basis.   */
/* phi [n][k], mass [n], feat [n][d]  ->  A [k][d]                              */
/* ------------------------------------------------------------------------- */
void oracle_project(int64_t n, int64_t k, int64_t d, const double *phi, const double *mass,
                    const double *feat, double *A)
{
    memset(A, 0, sizeof(double) * (size_t)(k * d));
    for (int64_t v = 0; v < n; ++v) {
        const double *f = feat + v * d;
        for (int64_t j = 0; j < k; ++j) {
            const double w = mass[v] * phi[v * k + j];
            double *a = A + j * d;
            for (int64_t t = 0; t < d; ++t) a[t] += w * f[t];
        }
    }
}

/* Adjoint of the projection: dF = diag(M) Phi dA.  dA [k][d] -> dF [n][d]. */
void oracle_project_backward(int64_t n, int64_t k, int64_t d, const double *phi, const double *mass,
                             const double *dA, double *dF)
{
    for (int64_t v = 0; v < n; ++v) {
        double *g = dF + v * d;
        for (int64_t t = 0; t < d; ++t) g[t] = 0.0;
        for (int64_t j = 0; j < k; ++j) {
            const double w = mass[v] * phi[v * k + j];
            const double *a = dA + j * d;
            for (int64_t t = 0; t < d; ++t) g[t] += w * a[t];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Penalty mask D [ky][kx].  Row i follows the target eigenvalue mu_y,i, column */
/* j the source eigenvalue mu_x,j (the indices of Eq. (3)).                     */
/*  Laplacian:  D_ij = (mu_y,i - mu_x,j)^2.                                     */
/*  Resolvent (cited, not defined, in the paper): eigenvalues are clipped at 0  */
/*  and divided by s = max(max mu_x, max mu_y); with a = (mu/s)^gamma the       */
/*  resolvent 1/(a - i) has real part a/(1+a^2) and imaginary part 1/(1+a^2);   */
/*  D_ij is the squared distance between the two resolvent values.            */
/* Returns 0, or -2 when the resolvent normaliser is not positive.             */
/* ------------------------------------------------------------------------- */
int oracle_mask(int64_t kx, int64_t ky, const double *ex, const double *ey, int kind, double gamma,
                double *D)
{
    if (kind == ORACLE_MASK_LAPLACIAN) {
        for (int64_t i = 0; i < ky; ++i)
            for (int64_t j = 0; j < kx; ++j) {
                const double t = ey[i] - ex[j];
                D[i * kx + j] = t * t;
            }
        return 0;
    }
    double s = -INFINITY;
    for (int64_t j = 0; j < kx; ++j) s = ex[j] > s ? ex[j] : s;
    for (int64_t i = 0; i < ky; ++i) s = ey[i] > s ? ey[i] : s;
    if (!(s > 0.0) || !isfinite(s)) return -2;
    for (int64_t i = 0; i < ky; ++i) {
        const double ay = pow((ey[i] > 0.0 ? ey[i] : 0.0) / s, gamma);
        const double rey = ay / (1.0 + ay * ay), imy = 1.0 / (1.0 + ay * ay);
        for (int64_t j = 0; j < kx; ++j) {
            const double ax = pow((ex[j] > 0.0 ? ex[j] : 0.0) / s, gamma);
            const double rex = ax / (1.0 + ax * ax), imx = 1.0 / (1.0 + ax * ax);
            D[i * kx + j] = (rey - rex) * (rey - rex) + (imy - imx) * (imy - imx);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Dense Cholesky S = L L^T of an m x m symmetric matrix (lower triangle read). */
/* L is written to the lower triangle of `L` (m x m, row-major), the strict    */
/* upper triangle is zeroed.  Returns 0, or j+1 when pivot j is not positive   */
/* or not finite.                                                              */
/* ------------------------------------------------------------------------- */
static int64_t chol(int64_t m, const double *S, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)(m * m));
    for (int64_t j = 0; j < m; ++j) {
        double s = S[j * m + j];
        for (int64_t q = 0; q < j; ++q) s -= L[j * m + q] * L[j * m + q];
        if (!(s > 0.0) || !isfinite(s)) return j + 1;
        const double ljj = sqrt(s);
        L[j * m + j] = ljj;
        for (int64_t i = j + 1; i < m; ++i) {
            double t = S[i * m + j];
            for (int64_t q = 0; q < j; ++q) t -= L[i * m + q] * L[j * m + q];
            L[i * m + j] = t / ljj;
        }
    }
    return 0;
}

/* Solve L L^T x = b in place (b overwritten by x). */
static void chol_solve(int64_t m, const double *L, double *b)
{
    for (int64_t i = 0; i < m; ++i) {
        double t = b[i];
        for (int64_t q = 0; q < i; ++q) t -= L[i * m + q] * b[q];
        b[i] = t / L[i * m + i];
    }
    for (int64_t i = m - 1; i >= 0; --i) {
        double t = b[i];
        for (int64_t q = i + 1; q < m; ++q) t -= L[q * m + i] * b[q];
        b[i] = t / L[i * m + i];
    }
}

/* K = A A^T (kx x kx, exactly symmetric: lower triangle computed then mirrored)
 * and R = B A^T (ky x kx): the two products of Eq. (4). */
static void normal_products(int64_t kx, int64_t ky, int64_t d, const double *A, const double *B, double *K,
                            double *R)
{
    for (int64_t i = 0; i < kx; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            double t = 0.0;
            for (int64_t s = 0; s < d; ++s) t += A[i * d + s] * A[j * d + s];
            K[i * kx + j] = t;
            K[j * kx + i] = t;
        }
    for (int64_t i = 0; i < ky; ++i)
        for (int64_t j = 0; j < kx; ++j) {
            double t = 0.0;
            for (int64_t s = 0; s < d; ++s) t += B[i * d + s] * A[j * d + s];
            R[i * kx + j] = t;
        }
}

/* Row system of Eq. (5): S_i = K + lambda diag(D_i). */
static void row_system(int64_t kx, const double *K, const double *Di, double lambda, double *S)
{
    memcpy(S, K, sizeof(double) * (size_t)(kx * kx));
    for (int64_t j = 0; j < kx; ++j) S[j * kx + j] += lambda * Di[j];
}

/* ------------------------------------------------------------------------- */
/* Eqs. (4)-(7): C [ky][kx] row by row.  D [ky][kx] from oracle_mask.          */
/* info [ky]; L_out (optional, may be NULL) receives the ky Cholesky factors,  */
/* each kx x kx row-major lower triangular.                                     */
/* ------------------------------------------------------------------------- */
void oracle_solve(int64_t kx, int64_t ky, int64_t d, const double *A, const double *B, const double *D,
                  double lambda, double *C, int32_t *info, double *L_out)
{
    if (!(lambda >= 0.0) || !isfinite(lambda)) {
        for (int64_t i = 0; i < ky; ++i) {
            info[i] = -1;
            for (int64_t j = 0; j < kx; ++j) C[i * kx + j] = NAN;
        }
        return;
    }
    double *K = (double *)malloc(sizeof(double) * (size_t)(kx * kx));
    double *R = (double *)malloc(sizeof(double) * (size_t)(ky * kx));
    normal_products(kx, ky, d, A, B, K, R);
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)(kx * kx));
        double *L = (double *)malloc(sizeof(double) * (size_t)(kx * kx));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < ky; ++i) {
            row_system(kx, K, D + i * kx, lambda, S);
            const int64_t f = chol(kx, S, L);
            info[i] = (int32_t)f;
            double *c = C + i * kx;
            if (f != 0) {
                for (int64_t j = 0; j < kx; ++j) c[j] = NAN;
            } else {
                memcpy(c, R + i * kx, sizeof(double) * (size_t)kx);
                chol_solve(kx, L, c);
            }
            if (L_out) memcpy(L_out + i * kx * kx, L, sizeof(double) * (size_t)(kx * kx));
        }
        free(S);
        free(L);
    }
    free(K);
    free(R);
}

/* ------------------------------------------------------------------------- */
/* Reverse mode of oracle_solve.  With G = dL/dC (rows g_i) and V the rows      */
/* v_i = S_i^{-1} g_i (S_i symmetric), the derivative of c_i = S_i^{-1} r_i,    */
/* r_i = A b_i, S_i = A A^T + lambda diag(D_i) is                               */
/*   dL/dB = V A,                                                               */
/*   dL/dA = V^T B - (V^T C + C^T V) A,                                          */
/*   dL/dlambda = - sum_ij V_ij D_ij C_ij.                                       */
/* dC [ky][kx] -> dA [kx][d], dB [ky][d], dlambda (may be NULL).  Rows whose      */
/* system fails produce NaN in every output they touch.                          */
/* ------------------------------------------------------------------------- */
void oracle_solve_backward(int64_t kx, int64_t ky, int64_t d, const double *A, const double *B,
                           const double *C, const double *D, double lambda, const double *dC, double *dA,
                           double *dB, double *dlambda, int32_t *info)
{
    double *K = (double *)malloc(sizeof(double) * (size_t)(kx * kx));
    double *R = (double *)malloc(sizeof(double) * (size_t)(ky * kx));
    double *V = (double *)malloc(sizeof(double) * (size_t)(ky * kx));
    normal_products(kx, ky, d, A, B, K, R);
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)(kx * kx));
        double *L = (double *)malloc(sizeof(double) * (size_t)(kx * kx));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < ky; ++i) {
            row_system(kx, K, D + i * kx, lambda, S);
            const int64_t f = chol(kx, S, L);
            if (info) info[i] = (int32_t)f;
            double *v = V + i * kx;
            if (f != 0 || !(lambda >= 0.0) || !isfinite(lambda)) {
                for (int64_t j = 0; j < kx; ++j) v[j] = NAN;
            } else {
                memcpy(v, dC + i * kx, sizeof(double) * (size_t)kx);
                chol_solve(kx, L, v);
            }
        }
        free(S);
        free(L);
    }
    /* dB = V A */
    for (int64_t i = 0; i < ky; ++i)
        for (int64_t t = 0; t < d; ++t) {
            double s = 0.0;
            for (int64_t j = 0; j < kx; ++j) s += V[i * kx + j] * A[j * d + t];
            dB[i * d + t] = s;
        }
    /* W = V^T C + C^T V (kx x kx) */
    double *W = (double *)malloc(sizeof(double) * (size_t)(kx * kx));
    for (int64_t a = 0; a < kx; ++a)
        for (int64_t b = 0; b < kx; ++b) {
            double s = 0.0;
            for (int64_t i = 0; i < ky; ++i) s += V[i * kx + a] * C[i * kx + b] + C[i * kx + a] * V[i * kx + b];
            W[a * kx + b] = s;
        }
    /* dA = V^T B - W A */
    for (int64_t a = 0; a < kx; ++a)
        for (int64_t t = 0; t < d; ++t) {
            double s = 0.0;
            for (int64_t i = 0; i < ky; ++i) s += V[i * kx + a] * B[i * d + t];
            for (int64_t b = 0; b < kx; ++b) s -= W[a * kx + b] * A[b * d + t];
            dA[a * d + t] = s;
        }
    if (dlambda) {
        double s = 0.0;
        for (int64_t i = 0; i < ky; ++i)
            for (int64_t j = 0; j < kx; ++j) s -= V[i * kx + j] * D[i * kx + j] * C[i * kx + j];
        *dlambda = s;
    }
    free(W);
    free(K);
    free(R);
    free(V);
}

/* ------------------------------------------------------------------------- */
/* Whole forward + backward pass over a batch of equal-size pairs, the unit of  */
/* work the benchmark times on the host (parallel over pairs).                 */
/* phi [2P][n][k], mass [2P][n], feat [2P][n][d], evals [2P][k] (x shapes then  */
/* y shapes), lambda [P], dC [P][k][k] -> C [P][k][k], dF [2P][n][d].            */
/* ------------------------------------------------------------------------- */
void oracle_pipeline_batch(int64_t P, int64_t n, int64_t k, int64_t d, const double *phi, const double *mass,
                           const double *feat, const double *evals, const double *lambda, int mask_kind,
                           double gamma, const double *dC, double *C, double *dF)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < P; ++p) {
        double *A = (double *)malloc(sizeof(double) * (size_t)(k * d));
        double *B = (double *)malloc(sizeof(double) * (size_t)(k * d));
        double *D = (double *)malloc(sizeof(double) * (size_t)(k * k));
        double *dA = (double *)malloc(sizeof(double) * (size_t)(k * d));
        double *dB = (double *)malloc(sizeof(double) * (size_t)(k * d));
        int32_t *info = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        const int64_t px = p, py = P + p;
        oracle_project(n, k, d, phi + px * n * k, mass + px * n, feat + px * n * d, A);
        oracle_project(n, k, d, phi + py * n * k, mass + py * n, feat + py * n * d, B);
        oracle_mask(k, k, evals + px * k, evals + py * k, mask_kind, gamma, D);
        oracle_solve(k, k, d, A, B, D, lambda[p], C + p * k * k, info, NULL);
        oracle_solve_backward(k, k, d, A, B, C + p * k * k, D, lambda[p], dC + p * k * k, dA, dB, NULL, NULL);
        oracle_project_backward(n, k, d, phi + px * n * k, mass + px * n, dA, dF + px * n * d);
        oracle_project_backward(n, k, d, phi + py * n * k, mass + py * n, dB, dF + py * n * d);
        free(A);
        free(B);
        free(D);
        free(dA);
        free(dB);
        free(info);
    }
}

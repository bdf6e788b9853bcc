// The vectorized functional-map solve with general commutativity operators (Sec. 3.1: the k^2 x k^2
// least-squares formulation that the row-wise solve avoids, and that the paper's conclusion names as the
// route to non-orthogonal bases).  Per pair
//     C = argmin ||C A - B||_F^2 + lambda ||C D1 - D2 C||_F^2
// with D1 [kx][kx] and D2 [ky][ky] full matrices.  With c[i kx + j] = C[i][j] the normal equations are one
// system of order n = kx ky,
//     H[(i,j),(p,q)] = delta_ip (A A^T)_jq
//                      + lambda (delta_ip (D1 D1^T)_jq - D2_ip D1_jq - D2_pi D1_qj + delta_jq (D2^T D2)_ip),
//     g[(i,j)]       = (B A^T)_ij,
// which is symmetric positive definite when A A^T is; with diagonal operators it splits into the row systems
// of Eqs. (4)-(7) with the Laplacian mask.
//
// Path: A A^T and B A^T by the normal-product kernel; H and g formed by vec_form_lds_kernel (kx, ky <= 32:
// operators and their products in LDS, rows of H written coalesced) or vec_form_kernel (one thread per entry
// of H, the operator products as dot products from L2); then one Cholesky solve per pair on the row-solve
// kernels, which take H as their matrix, g as the one right-hand side row, zero mask rows (no diagonal shift)
// and lambda only to flag an invalid value.  n <= 64 runs on the register row solve, 64 < n <= 319 on the
// tiled one.
#include "../../include/fmap.h"

#include <math.h>

#include "fmap_launch.h"

namespace fmap {

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct VecWs {
    size_t K, R, H, g, ex0, ey0, tiles, total;
};

VecWs vec_layout(int64_t P, int64_t kx, int64_t ky)
{
    const int64_t n = kx * ky;
    VecWs w{};
    size_t off = 0;
    w.K = off;
    off += align256((size_t)P * kx * kx * sizeof(float));
    w.R = off;
    off += align256((size_t)P * ky * kx * sizeof(float));
    w.H = off;
    off += align256((size_t)P * n * n * sizeof(float));
    w.g = off;
    off += align256((size_t)P * n * sizeof(float));
    w.ex0 = off;
    off += align256((size_t)P * n * sizeof(float));
    w.ey0 = off;
    off += align256((size_t)P * sizeof(float));
    w.tiles = off;
    off += align256(n > kSmallK ? tiled_workspace_bytes(P, n, 1) : 0);
    w.total = off;
    return w;
}

// H [P][n][n], g [P][n] of the normal equations, and zero mask inputs for the row solve.  Each pair takes bpp
// consecutive workgroups; its thread e owns entry (a, b) = (e / n, e % n) of H, a = i kx + j, b = p kx + q.  Each entry is a fixed
// sequence of operations on its own indices and the same products in the same order as its mirror, so H is
// exactly symmetric when A A^T is.
__global__ __launch_bounds__(256) void vec_form_kernel(const float *__restrict__ K, const float *__restrict__ R,
                                                       const float *__restrict__ D1, const float *__restrict__ D2,
                                                       const float *__restrict__ lam, int kx, int ky, int n,
                                                       float *__restrict__ H, float *__restrict__ g,
                                                       float *__restrict__ ex0, float *__restrict__ ey0, int bpp)
{
    const int pr = blockIdx.x / bpp;  // bpp workgroups per pair (a 1-D grid: no per-dimension limit on pairs)
    const int e = (blockIdx.x - pr * bpp) * 256 + threadIdx.x;
    const float *Kp = K + (size_t)pr * kx * kx;
    const float *D1p = D1 + (size_t)pr * kx * kx;
    const float *D2p = D2 + (size_t)pr * ky * ky;
    if (e < n * n) {
        const int a = e / n, b = e - a * n;
        const int i = a / kx, j = a - i * kx;
        const int p = b / kx, q = b - p * kx;
        float s = 0.f;
        if (i == p) {  // (D1 D1^T)_jq
            float t = 0.f;
            for (int c = 0; c < kx; ++c) t = fmaf(D1p[(size_t)j * kx + c], D1p[(size_t)q * kx + c], t);
            s += t;
        }
        if (j == q) {  // (D2^T D2)_ip
            float t = 0.f;
            for (int c = 0; c < ky; ++c) t = fmaf(D2p[(size_t)c * ky + i], D2p[(size_t)c * ky + p], t);
            s += t;
        }
        s -= D2p[(size_t)i * ky + p] * D1p[(size_t)j * kx + q] + D2p[(size_t)p * ky + i] * D1p[(size_t)q * kx + j];
        const float base = i == p ? Kp[(size_t)j * kx + q] : 0.f;
        H[(size_t)pr * n * n + e] = fmaf(lam[pr], s, base);
    }
    if (e < n) {
        g[(size_t)pr * n + e] = R[(size_t)pr * n + e];  // (B A^T)_ij at i kx + j: R is [ky][kx] row-major
        ex0[(size_t)pr * n + e] = 0.f;
    }
    if (e == 0) ey0[pr] = 0.f;
}

// The same entries for kx, ky <= 32: a workgroup takes VF_ROWS rows of H of one pair.  It stages D1, D2 and K
// in LDS (rows padded to 33 floats), forms D1 D1^T and D2^T D2 there once (the dot products in the order of
// the kernel above), and writes each row of H with consecutive threads on consecutive columns.  Every entry
// follows the same formula, in the same order, as in the kernel above.
constexpr int VF_KM = 32, VF_LD = 33, VF_ROWS = 32;

__global__ __launch_bounds__(256) void vec_form_lds_kernel(const float *__restrict__ K, const float *__restrict__ R,
                                                           const float *__restrict__ D1, const float *__restrict__ D2,
                                                           const float *__restrict__ lam, int kx, int ky, int n,
                                                           float *__restrict__ H, float *__restrict__ g,
                                                           float *__restrict__ ex0, float *__restrict__ ey0, int bpp)
{
    __shared__ float sD1[VF_KM * VF_LD], sD2[VF_KM * VF_LD], sK[VF_KM * VF_LD], sP1[VF_KM * VF_LD],
        sP2[VF_KM * VF_LD];
    const int pr = blockIdx.x / bpp, bx = blockIdx.x - pr * bpp;
    const int a0 = bx * VF_ROWS, tid = threadIdx.x;
    const float *Kp = K + (size_t)pr * kx * kx;
    const float *D1p = D1 + (size_t)pr * kx * kx;
    const float *D2p = D2 + (size_t)pr * ky * ky;
    for (int e = tid; e < kx * kx; e += 256) {
        const int r = e / kx, c = e - r * kx;
        sD1[r * VF_LD + c] = D1p[e];
        sK[r * VF_LD + c] = Kp[e];
    }
    for (int e = tid; e < ky * ky; e += 256) {
        const int r = e / ky, c = e - r * ky;
        sD2[r * VF_LD + c] = D2p[e];
    }
    __syncthreads();
    for (int e = tid; e < kx * kx; e += 256) {  // (D1 D1^T)_jq
        const int j = e / kx, q = e - j * kx;
        float t = 0.f;
        for (int c = 0; c < kx; ++c) t = fmaf(sD1[j * VF_LD + c], sD1[q * VF_LD + c], t);
        sP1[j * VF_LD + q] = t;
    }
    for (int e = tid; e < ky * ky; e += 256) {  // (D2^T D2)_ip
        const int i = e / ky, p = e - i * ky;
        float t = 0.f;
        for (int c = 0; c < ky; ++c) t = fmaf(sD2[c * VF_LD + i], sD2[c * VF_LD + p], t);
        sP2[i * VF_LD + p] = t;
    }
    __syncthreads();
    const float lm = lam[pr];
    const int a1 = min(a0 + VF_ROWS, n);
    for (int a = a0; a < a1; ++a) {
        const int i = a / kx, j = a - i * kx;
        float *Hr = H + (size_t)pr * n * n + (size_t)a * n;
        for (int b = tid; b < n; b += 256) {
            const int p = b / kx, q = b - p * kx;
            float s = 0.f;
            if (i == p) s += sP1[j * VF_LD + q];
            if (j == q) s += sP2[i * VF_LD + p];
            s -= sD2[i * VF_LD + p] * sD1[j * VF_LD + q] + sD2[p * VF_LD + i] * sD1[q * VF_LD + j];
            const float base = i == p ? sK[j * VF_LD + q] : 0.f;
            Hr[b] = fmaf(lm, s, base);
        }
    }
    if (bx == 0) {
        for (int e = tid; e < n; e += 256) {
            g[(size_t)pr * n + e] = R[(size_t)pr * n + e];
            ex0[(size_t)pr * n + e] = 0.f;
        }
        if (tid == 0) ey0[pr] = 0.f;
    }
}

}  // namespace

size_t vectorized_workspace_bytes(int64_t P, int64_t kx, int64_t ky) { return vec_layout(P, kx, ky).total; }

hipError_t launch_solve_vectorized(const float *A, const float *B, const float *D1, const float *D2, const float *lam,
                                   int64_t P, int64_t kx, int64_t ky, int64_t d, float *C, int32_t *info, void *ws,
                                   hipStream_t st)
{
    const int64_t n = kx * ky;
    const VecWs L = vec_layout(P, kx, ky);
    char *base = (char *)ws;
    float *K = (float *)(base + L.K), *R = (float *)(base + L.R), *H = (float *)(base + L.H);
    float *g = (float *)(base + L.g), *ex0 = (float *)(base + L.ex0), *ey0 = (float *)(base + L.ey0);
    launch_gram(A, B, P, kx, ky, d, true, K, R, st);
    if (kx <= VF_KM && ky <= VF_KM) {
        const int bpp = (int)((n + VF_ROWS - 1) / VF_ROWS);
        hipLaunchKernelGGL(vec_form_lds_kernel, dim3((unsigned)(P * bpp)), dim3(256), 0, st, K, R, D1, D2, lam, (int)kx,
                           (int)ky, (int)n, H, g, ex0, ey0, bpp);
    } else {
        const int bpp = (int)((n * n + 255) / 256);
        hipLaunchKernelGGL(vec_form_kernel, dim3((unsigned)(P * bpp)), dim3(256), 0, st, K, R, D1, D2, lam, (int)kx,
                           (int)ky, (int)n, H, g, ex0, ey0, bpp);
    }
    launch_rowsolve_dense(H, g, ex0, ey0, lam, P, n, C, info, (float *)(base + L.tiles), st);
    return hipGetLastError();
}

}  // namespace fmap

extern "C" {

size_t fmap_solve_vectorized_workspace_bytes(int64_t pairs, int64_t kx, int64_t ky, int64_t d)
{
    (void)d;
    if (pairs < 1 || kx < 1 || ky < 1 || kx > fmap::kMaxK || ky > fmap::kMaxK || kx * ky > fmap::kMaxK ||
        pairs > ((int64_t)1 << 20))
        return 0;
    return fmap::vectorized_workspace_bytes(pairs, kx, ky);
}

fmap_status fmap_solve_vectorized(const float *A, const float *B, const float *op_x, const float *op_y,
                                  const float *lambda, int64_t pairs, int64_t kx, int64_t ky, int64_t d, float *C,
                                  int32_t *info, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!A || !B || !op_x || !op_y || !lambda || !C || !info) return FMAP_ERR_NULL;
    if (pairs < 1 || kx < 1 || ky < 1 || d < 1 || pairs > ((int64_t)1 << 20) || d > ((int64_t)1 << 30))
        return FMAP_ERR_SHAPE;
    if (kx > fmap::kMaxK || ky > fmap::kMaxK || kx * ky > fmap::kMaxK) return FMAP_ERR_UNSUPPORTED;
    if (pairs * kx * d > ((int64_t)1 << 40) || pairs * ky * d > ((int64_t)1 << 40)) return FMAP_ERR_SHAPE;
    const size_t need = fmap::vectorized_workspace_bytes(pairs, kx, ky);
    if (!workspace || workspace_bytes < need) return FMAP_ERR_WORKSPACE;
    const hipError_t e = fmap::launch_solve_vectorized(A, B, op_x, op_y, lambda, pairs, kx, ky, d, C, info,
                                                       workspace, (hipStream_t)stream);
    return e == hipSuccess ? FMAP_OK : FMAP_ERR_HIP;
}

}  // extern "C"

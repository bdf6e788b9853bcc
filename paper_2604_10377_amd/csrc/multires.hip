// Two uses of the solve beyond one square map per pair (Eq. (1), Sec. 3.1):
//
// 1. Several spectral resolutions from one projection.  Multi-resolution
//    pipelines project the features once onto the first k_max eigenfunctions
//    and compute maps at several smaller resolutions.  Resolution (k_x', k_y')
//    is the solve of Eqs. (4)-(7) restricted to the first k_x' source and k_y'
//    target eigenpairs: the leading k_x' rows of A, the leading k_y' rows of B,
//    the eigenvalues truncated alike (the mask, and the resolvent normaliser,
//    are those of the truncated spectra).  The leading rows are gathered into
//    contiguous workspace arrays by one copy launch, then the batched solve
//    runs as for a plain call; the largest resolution reuses A and B in place.
//
// 2. The projector given directly.  Eq. (1) writes A = Phi^+ F with the
//    pseudo-inverse; a caller holding Phi^+ (k x n) passes its transpose P
//    [n][k] (the same array read column-major), and A = P^T F, dF = P dA are
//    the projection kernels with unit vertex weights (a weight array of ones
//    written into the workspace by a fill kernel, multiplication by 1 being
//    exact).
#include "../../include/fmap.h"

#include <algorithm>
#include <vector>

#include "fmap_launch.h"

namespace fmap {

namespace {

struct RowCopy {             // dst[p][r][c] = src[p][r][c] for r < rows, pairs p
    const float *src;
    float *dst;
    int64_t src_pair_stride;  // floats between pairs in src
    int rows, cols;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct ResLayout {
    size_t A, B, ex, ey, info, solve, total;
};

ResLayout res_layout(int64_t P, int64_t kx, int64_t ky, int64_t d)
{
    ResLayout L;
    size_t off = 0;
    L.A = off;
    off += align256((size_t)P * kx * d * sizeof(float));
    L.B = off;
    off += align256((size_t)P * ky * d * sizeof(float));
    L.ex = off;
    off += align256((size_t)P * kx * sizeof(float));
    L.ey = off;
    off += align256((size_t)P * ky * sizeof(float));
    L.info = off;
    off += align256((size_t)P * ky * sizeof(int32_t));
    L.solve = off;
    off += solve_workspace_layout(P, kx, ky, d).total;
    L.total = off;
    return L;
}

}  // namespace

__global__ __launch_bounds__(256) void copy_rows_kernel(RowCopy j0, RowCopy j1, RowCopy j2, RowCopy j3, int P)
{
    const RowCopy &j = blockIdx.y == 0 ? j0 : blockIdx.y == 1 ? j1 : blockIdx.y == 2 ? j2 : j3;
    const int64_t per = (int64_t)j.rows * j.cols;
    const int64_t n = per * P;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t p = e / per, q = e % per;
        j.dst[e] = j.src[p * j.src_pair_stride + q];
    }
}

__global__ __launch_bounds__(256) void fill_ones_kernel(float *__restrict__ x, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) x[e] = 1.f;
}

static unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

size_t resolutions_workspace_bytes(int64_t P, int64_t kx, int64_t ky, int64_t d, int nres, const int32_t *kxs,
                                   const int32_t *kys)
{
    size_t mx = 0;
    for (int r = 0; r < nres; ++r) mx = std::max(mx, res_layout(P, kxs[r], kys[r], d).total);
    (void)kx;
    (void)ky;
    return mx;
}

hipError_t launch_solve_resolutions(const float *A, const float *B, const float *ex, const float *ey, const float *lam,
                                    int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, int64_t d, int nres,
                                    const int32_t *kxs, const int32_t *kys, float *const *C, int32_t *const *info,
                                    void *ws, hipStream_t st)
{
    char *base = (char *)ws;
    for (int r = 0; r < nres; ++r) {
        const int64_t kxr = kxs[r], kyr = kys[r];
        const ResLayout L = res_layout(P, kxr, kyr, d);
        int32_t *inf = (info && info[r]) ? info[r] : (int32_t *)(base + L.info);
        const float *Ar = A, *Br = B, *exr = ex, *eyr = ey;
        if (kxr != kx || kyr != ky) {
            RowCopy ja{A, (float *)(base + L.A), kx * d, (int)kxr, (int)d};
            RowCopy jb{B, (float *)(base + L.B), ky * d, (int)kyr, (int)d};
            RowCopy jx{ex, (float *)(base + L.ex), kx, 1, (int)kxr};
            RowCopy jy{ey, (float *)(base + L.ey), ky, 1, (int)kyr};
            const int64_t most = P * std::max(kxr, kyr) * d;
            hipLaunchKernelGGL(copy_rows_kernel, dim3(blocks_for(most), 4), dim3(256), 0, st, ja, jb, jx, jy, (int)P);
            Ar = ja.dst;
            Br = jb.dst;
            exr = jx.dst;
            eyr = jy.dst;
        }
        hipError_t e = launch_solve(Ar, Br, exr, eyr, lam, mask_kind, gamma, P, kxr, kyr, d, 0, 0.f, C[r], nullptr, inf,
                                    nullptr, base + L.solve, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

size_t project_pinv_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t dtype)
{
    return align256((size_t)batch * n * sizeof(float)) + project_workspace_bytes(batch, n, k, d, dtype);
}

hipError_t launch_project_pinv(const void *P, const void *feat, int32_t dtype, int64_t batch, int64_t n, int64_t k,
                               int64_t d, float *A, void *ws, hipStream_t st)
{
    float *ones = (float *)ws;
    hipLaunchKernelGGL(fill_ones_kernel, dim3(blocks_for(batch * n)), dim3(256), 0, st, ones, batch * n);
    void *rest = (char *)ws + align256((size_t)batch * n * sizeof(float));
    return launch_project(P, ones, feat, dtype, batch, n, k, d, A, rest, st);
}

hipError_t launch_project_pinv_backward(const void *P, int32_t dtype, const float *dA, int64_t batch, int64_t n,
                                        int64_t k, int64_t d, float *dF, void *ws, hipStream_t st)
{
    float *ones = (float *)ws;
    hipLaunchKernelGGL(fill_ones_kernel, dim3(blocks_for(batch * n)), dim3(256), 0, st, ones, batch * n);
    return launch_project_backward(P, ones, dtype, dA, batch, n, k, d, dF, st);
}

}  // namespace fmap

namespace {

bool dims_ok(int64_t v) { return v >= 1 && v < ((int64_t)1 << 30); }

fmap_status res_args_ok(int64_t kx, int64_t ky, int32_t nres, const int32_t *kxs, const int32_t *kys)
{
    if (nres < 1 || nres > 64) return FMAP_ERR_SHAPE;
    if (!kxs || !kys) return FMAP_ERR_NULL;
    for (int r = 0; r < nres; ++r)
        if (kxs[r] < 1 || kys[r] < 1 || kxs[r] > kx || kys[r] > ky) return FMAP_ERR_SHAPE;
    return FMAP_OK;
}

}  // namespace

extern "C" {

size_t fmap_solve_resolutions_workspace_bytes(int64_t pairs, int64_t kx, int64_t ky, int64_t d, int32_t nres,
                                              const int32_t *kxs, const int32_t *kys)
{
    if (!dims_ok(pairs) || !dims_ok(kx) || !dims_ok(ky) || !dims_ok(d)) return 0;
    if (res_args_ok(kx, ky, nres, kxs, kys) != FMAP_OK) return 0;
    return fmap::resolutions_workspace_bytes(pairs, kx, ky, d, nres, kxs, kys);
}

fmap_status fmap_solve_resolutions(const float *A, const float *B, const float *evals_x, const float *evals_y,
                                   const float *lambda, int32_t mask_kind, float gamma, int64_t pairs, int64_t kx,
                                   int64_t ky, int64_t d, int32_t nres, const int32_t *kxs, const int32_t *kys,
                                   float *const *C, int32_t *const *info, void *workspace, size_t workspace_bytes,
                                   void *stream)
{
    if (!A || !B || !evals_x || !evals_y || !lambda || !C) return FMAP_ERR_NULL;
    if (!dims_ok(pairs) || !dims_ok(kx) || !dims_ok(ky) || !dims_ok(d)) return FMAP_ERR_SHAPE;
    if (mask_kind != FMAP_MASK_LAPLACIAN && mask_kind != FMAP_MASK_RESOLVENT) return FMAP_ERR_VALUE;
    if (mask_kind == FMAP_MASK_RESOLVENT && !(gamma > 0.f && gamma < 1e30f)) return FMAP_ERR_VALUE;
    if (kx > fmap_max_k() || ky > fmap_max_k()) return FMAP_ERR_UNSUPPORTED;
    if (pairs * ky > ((int64_t)1 << 30) || pairs * kx * d > ((int64_t)1 << 40)) return FMAP_ERR_SHAPE;
    const fmap_status a = res_args_ok(kx, ky, nres, kxs, kys);
    if (a != FMAP_OK) return a;
    for (int r = 0; r < nres; ++r)
        if (!C[r]) return FMAP_ERR_NULL;
    const size_t need = fmap::resolutions_workspace_bytes(pairs, kx, ky, d, nres, kxs, kys);
    if (!workspace || workspace_bytes < need) return FMAP_ERR_WORKSPACE;
    return fmap::launch_solve_resolutions(A, B, evals_x, evals_y, lambda, mask_kind, gamma, pairs, kx, ky, d, nres,
                                          kxs, kys, C, info, workspace, (hipStream_t)stream) == hipSuccess
               ? FMAP_OK
               : FMAP_ERR_HIP;
}

size_t fmap_project_pinv_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t in_dtype)
{
    if (!dims_ok(batch) || !dims_ok(n) || !dims_ok(k) || !dims_ok(d)) return 0;
    return fmap::project_pinv_workspace_bytes(batch, n, k, d, in_dtype);
}

fmap_status fmap_project_pinv(const void *pinv_t, const void *feat, int32_t in_dtype, int64_t batch, int64_t n,
                              int64_t k, int64_t d, float *A, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!pinv_t || !feat || !A) return FMAP_ERR_NULL;
    if (in_dtype != FMAP_F32 && in_dtype != FMAP_BF16) return FMAP_ERR_DTYPE;
    if (!dims_ok(batch) || !dims_ok(n) || !dims_ok(k) || !dims_ok(d)) return FMAP_ERR_SHAPE;
    if (n * k > ((int64_t)1 << 31) || n * d > ((int64_t)1 << 31) || batch * n > ((int64_t)1 << 34))
        return FMAP_ERR_SHAPE;
    if (!workspace || workspace_bytes < fmap::project_pinv_workspace_bytes(batch, n, k, d, in_dtype))
        return FMAP_ERR_WORKSPACE;
    return fmap::launch_project_pinv(pinv_t, feat, in_dtype, batch, n, k, d, A, workspace, (hipStream_t)stream) ==
                   hipSuccess
               ? FMAP_OK
               : FMAP_ERR_HIP;
}

fmap_status fmap_project_pinv_backward(const void *pinv_t, int32_t pinv_dtype, const float *dA, int64_t batch,
                                       int64_t n, int64_t k, int64_t d, float *dF, void *workspace,
                                       size_t workspace_bytes, void *stream)
{
    if (!pinv_t || !dA || !dF) return FMAP_ERR_NULL;
    if (pinv_dtype != FMAP_F32 && pinv_dtype != FMAP_BF16) return FMAP_ERR_DTYPE;
    if (!dims_ok(batch) || !dims_ok(n) || !dims_ok(k) || !dims_ok(d)) return FMAP_ERR_SHAPE;
    if (n * k > ((int64_t)1 << 31) || n * d > ((int64_t)1 << 31) || batch * n > ((int64_t)1 << 34))
        return FMAP_ERR_SHAPE;
    if (!workspace || workspace_bytes < (size_t)batch * n * sizeof(float)) return FMAP_ERR_WORKSPACE;
    return fmap::launch_project_pinv_backward(pinv_t, pinv_dtype, dA, batch, n, k, d, dF, workspace,
                                              (hipStream_t)stream) == hipSuccess
               ? FMAP_OK
               : FMAP_ERR_HIP;
}

}  // extern "C"

// C ABI of libfmap (declared in include/fmap.h).  Every entry point validates
// its arguments on the host first and returns an error before anything is
// enqueued; only then are kernels launched on the caller's stream.
#include "../../include/fmap.h"

#include <math.h>

#include "fmap_launch.h"

namespace {

constexpr int64_t kMaxDim = (int64_t)1 << 30;

bool dim_ok(int64_t v) { return v >= 1 && v < kMaxDim; }

fmap_status hip_status(hipError_t e) { return e == hipSuccess ? FMAP_OK : FMAP_ERR_HIP; }

fmap_status check_solve_common(const float *A, const float *B, const float *ex, const float *ey, const float *lam,
                               int32_t mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, int64_t d)
{
    if (!A || !B || !ex || !ey || !lam) return FMAP_ERR_NULL;
    if (!dim_ok(P) || !dim_ok(kx) || !dim_ok(ky) || !dim_ok(d)) return FMAP_ERR_SHAPE;
    if (mask_kind != FMAP_MASK_LAPLACIAN && mask_kind != FMAP_MASK_RESOLVENT) return FMAP_ERR_VALUE;
    if (mask_kind == FMAP_MASK_RESOLVENT && !(gamma > 0.f && isfinite(gamma))) return FMAP_ERR_VALUE;
    if (kx > fmap_max_k() || ky > fmap_max_k()) return FMAP_ERR_UNSUPPORTED;
    if (P * ky > kMaxDim || P * kx * d > ((int64_t)1 << 40)) return FMAP_ERR_SHAPE;
    return FMAP_OK;
}

}  // namespace

extern "C" {

int32_t fmap_abi_version(void) { return 1; }

int32_t fmap_max_k(void) { return fmap::kMaxK; }

const char *fmap_status_str(fmap_status s)
{
    switch (s) {
    case FMAP_OK: return "ok";
    case FMAP_ERR_NULL: return "a required pointer is NULL";
    case FMAP_ERR_SHAPE: return "a size is out of range or sizes disagree";
    case FMAP_ERR_VALUE: return "a scalar option is out of range";
    case FMAP_ERR_DTYPE: return "unknown element type";
    case FMAP_ERR_WORKSPACE: return "workspace missing or too small";
    case FMAP_ERR_UNSUPPORTED: return "request not supported by this build";
    case FMAP_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

size_t fmap_project_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t in_dtype)
{
    if (!dim_ok(batch) || !dim_ok(n) || !dim_ok(k) || !dim_ok(d)) return 0;
    return fmap::project_workspace_bytes(batch, n, k, d, in_dtype);
}

fmap_status fmap_project(const void *phi, const float *mass, const void *feat, int32_t in_dtype, int64_t batch,
                         int64_t n, int64_t k, int64_t d, float *A, void *workspace, size_t workspace_bytes,
                         void *stream)
{
    if (!phi || !mass || !feat || !A) return FMAP_ERR_NULL;
    if (in_dtype != FMAP_F32 && in_dtype != FMAP_BF16) return FMAP_ERR_DTYPE;
    if (!dim_ok(batch) || !dim_ok(n) || !dim_ok(k) || !dim_ok(d)) return FMAP_ERR_SHAPE;
    if (n * k > ((int64_t)1 << 31) || n * d > ((int64_t)1 << 31)) return FMAP_ERR_SHAPE;
    const size_t need = fmap::project_workspace_bytes(batch, n, k, d, in_dtype);
    if (need > 0 && (!workspace || workspace_bytes < need)) return FMAP_ERR_WORKSPACE;
    return hip_status(fmap::launch_project(phi, mass, feat, in_dtype, batch, n, k, d, A, workspace,
                                           (hipStream_t)stream));
}

fmap_status fmap_project_backward(const void *phi, const float *mass, int32_t phi_dtype, const float *dA,
                                  int64_t batch, int64_t n, int64_t k, int64_t d, float *dF, void *stream)
{
    if (!phi || !mass || !dA || !dF) return FMAP_ERR_NULL;
    if (phi_dtype != FMAP_F32 && phi_dtype != FMAP_BF16) return FMAP_ERR_DTYPE;
    if (!dim_ok(batch) || !dim_ok(n) || !dim_ok(k) || !dim_ok(d)) return FMAP_ERR_SHAPE;
    if (n * k > ((int64_t)1 << 31) || n * d > ((int64_t)1 << 31)) return FMAP_ERR_SHAPE;
    return hip_status(
        fmap::launch_project_backward(phi, mass, phi_dtype, dA, batch, n, k, d, dF, (hipStream_t)stream));
}

size_t fmap_factor_floats(int64_t kx, int64_t ky)
{
    if (!dim_ok(kx) || !dim_ok(ky)) return 0;
    return (size_t)ky * (size_t)(kx * (kx + 1) / 2);
}

size_t fmap_solve_workspace_bytes(int64_t pairs, int64_t kx, int64_t ky, int64_t d)
{
    if (!dim_ok(pairs) || !dim_ok(kx) || !dim_ok(ky) || !dim_ok(d)) return 0;
    return fmap::solve_workspace_layout(pairs, kx, ky, d).total;
}

fmap_status fmap_solve(const float *A, const float *B, const float *evals_x, const float *evals_y,
                       const float *lambda, int32_t mask_kind, float gamma, int64_t pairs, int64_t kx, int64_t ky,
                       int64_t d, int32_t refine_steps, float cond_fp64_threshold, float *C, float *factors,
                       int32_t *info, float *cond_est, void *workspace, size_t workspace_bytes, void *stream)
{
    fmap_status s = check_solve_common(A, B, evals_x, evals_y, lambda, mask_kind, gamma, pairs, kx, ky, d);
    if (s != FMAP_OK) return s;
    if (!C || !info) return FMAP_ERR_NULL;
    if (refine_steps < 0 || refine_steps > 8) return FMAP_ERR_VALUE;
    if (isnan(cond_fp64_threshold)) return FMAP_ERR_VALUE;
    if (refine_steps > 0 && !factors) return FMAP_ERR_NULL;  // the corrections reuse the float32 factors
    if ((cond_fp64_threshold > 0.f || cond_est) && kx > fmap::kMaxCondK) return FMAP_ERR_UNSUPPORTED;
    const size_t need = fmap::solve_workspace_layout(pairs, kx, ky, d).total;
    if (!workspace || workspace_bytes < need) return FMAP_ERR_WORKSPACE;
    return hip_status(fmap::launch_solve(A, B, evals_x, evals_y, lambda, mask_kind, gamma, pairs, kx, ky, d,
                                         refine_steps, cond_fp64_threshold, C, factors, info, cond_est, workspace,
                                         (hipStream_t)stream));
}

fmap_status fmap_solve_backward(const float *dC, const float *A, const float *B, const float *C,
                                const float *evals_x, const float *evals_y, const float *lambda, int32_t mask_kind,
                                float gamma, int64_t pairs, int64_t kx, int64_t ky, int64_t d, const float *factors,
                                float *dA, float *dB, float *dlambda, int32_t *info, void *workspace,
                                size_t workspace_bytes, void *stream)
{
    fmap_status s = check_solve_common(A, B, evals_x, evals_y, lambda, mask_kind, gamma, pairs, kx, ky, d);
    if (s != FMAP_OK) return s;
    if (!dC || !C || !dA || !dB) return FMAP_ERR_NULL;
    const size_t need = fmap::solve_workspace_layout(pairs, kx, ky, d).total;
    if (!workspace || workspace_bytes < need) return FMAP_ERR_WORKSPACE;
    return hip_status(fmap::launch_solve_backward(dC, A, B, C, evals_x, evals_y, lambda, mask_kind, gamma, pairs, kx,
                                                  ky, d, factors, dA, dB, dlambda, info, workspace,
                                                  (hipStream_t)stream));
}

}  // extern "C"

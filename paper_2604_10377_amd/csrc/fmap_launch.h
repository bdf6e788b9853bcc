// Host-side launch entry points shared between the kernel files and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fmap {

// Largest k_x handled by the register-resident row-solve kernels.
constexpr int kSmallK = 64;
// Largest k_x of the tiled row solve (k_x + 1 rows in at most 10 tile rows of 32).
constexpr int kMaxK = 319;

// Work items of the persistent projections over uneven shapes.
struct FwdItem {                  // partial A rows [kbase, kbase+64) x d-block over vertices [v0, v1)
    const float *phi, *mass, *feat;
    float *out;                   // k x d partial slot
    int n, k, d, v0, v1, kbase, dbase;
};
struct BwdItem {                  // dF rows [r0, r0 + 128*rb) x columns [dbase, dbase + 256)
    const float *phi, *mass, *dA;
    float *dF;
    int n, k, d, r0, rb, dbase;
};
struct McItem {                   // dF tiles [t0, t1) of 256 vertices x columns [dbase, dbase + block)
    const float *phi, *mass, *dA;
    float *dF;
    int n, k, d, t0, t1, dbase;
};
struct RedItem {                  // A = sum of `nchunks` partial k x d slots
    const float *part;
    float *A, *A_user;
    int nchunks, kd;
};

hipError_t launch_fwd_items(const FwdItem *items, int nitems, int kmax, int grid, hipStream_t st);
hipError_t launch_bwd_items(const BwdItem *items, int nitems, int kmax, int grid, hipStream_t st);
hipError_t launch_reduce_items(const RedItem *items, int nitems, hipStream_t st);
// Uneven batches on the emulated float32 kernels, one workgroup per item.  Forward items cover whole
// 32-vertex stages (v0, v1 multiples of 32) of shapes with x3r_item_shape_ok; `sliced` = k > 64.
bool x3r_item_shape_ok(int64_t k, int64_t d);
hipError_t launch_fwd_x3r_items(const FwdItem *items, int nitems, bool sliced, hipStream_t st);
// Backward items of one k (k even, <= kMaxK): mc_item_cols(k) columns per item.
bool mc_item_shape_ok(int64_t k);
int mc_item_cols(int64_t k);
hipError_t launch_bwd_mc_items(const McItem *items, int nitems, int64_t k, hipStream_t st);
// Fixed-order sum of split-K partials [batch][nsplit][k][d] into A [batch][k][d].
hipError_t launch_reduce(const float *part, int nsplit, int64_t batch, int64_t k, int64_t d, float *A, hipStream_t st);
// bf16 forward projection on the bf16 matrix cores (k % 8 == 0, k <= 256, d % 8 == 0, n % 4 == 0).
bool bf16_fwd_shape_ok(int64_t n, int64_t k, int64_t d);
int bf16_fwd_nsplit(int64_t batch, int64_t n, int64_t k, int64_t d);
// bf16-basis backward projection on the bf16 matrix cores (k % 8 == 0, k <= 256).
bool bf16_bwd_shape_ok(int64_t n, int64_t k, int64_t d);
hipError_t launch_project_backward_bf16(const uint16_t *phi, const float *mass, const float *dA, int64_t batch,
                                        int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st);
// float32 forward projection on the bf16 matrix cores, operands split into three bf16 parts
// (k even <= 64 or k % 4 == 0 up to 319, d % 4 == 0, n % 4 == 0).
bool f32_split_fwd_shape_ok(int64_t n, int64_t k, int64_t d);
int f32_split_fwd_nsplit(int64_t batch, int64_t n, int64_t k, int64_t d);
hipError_t launch_project_f32_split(const float *phi, const float *mass, const float *feat, int64_t batch, int64_t n,
                                    int64_t k, int64_t d, float *A, void *ws, hipStream_t st);
// float32 backward projection on the bf16 matrix cores, operands split into three bf16 parts (k even, k <= 64).
bool f32_split_bwd_shape_ok(int64_t n, int64_t k, int64_t d);
// float32 backward for 64 < k <= kMaxK (k even), 64-column blocks with every k slot's dA^T parts in LDS
bool f32k_bwd_shape_ok(int64_t n, int64_t k, int64_t d);
hipError_t launch_project_backward_f32k(const float *phi, const float *mass, const float *dA, int64_t batch,
                                        int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st);
hipError_t launch_project_backward_f32_split(const float *phi, const float *mass, const float *dA, int64_t batch,
                                             int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st);
hipError_t launch_project_bf16(const uint16_t *phi, const float *mass, const uint16_t *feat, int64_t batch, int64_t n,
                               int64_t k, int64_t d, float *A, void *ws, hipStream_t st);
int device_cus();

struct ProjPlan {
    int MT, NT, kblocks, dblocks, nsplit, chunk;
};

ProjPlan plan_project(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t dtype);
size_t project_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t dtype);
hipError_t launch_project(const void *phi, const float *mass, const void *feat, int32_t dtype, int64_t batch, int64_t n,
                          int64_t k, int64_t d, float *A, void *ws, hipStream_t st);
hipError_t launch_project_backward(const void *phi, const float *mass, int32_t dtype, const float *dA, int64_t batch,
                                   int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st);

// rs_waves: row systems per workgroup of the register row solve (k_x <= kSmallK): 1, 2 or 4.
// Workspace carve-up of the solver (byte offsets, 256-aligned).
struct SolveWs {
    size_t K, R, V, W, tiles, K64, R64, dlam, flag, total;
};
SolveWs solve_workspace_layout(int64_t pairs, int64_t kx, int64_t ky, int64_t d);

hipError_t launch_solve(const float *A, const float *B, const float *ex, const float *ey, const float *lam,
                        int32_t mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, int64_t d,
                        int32_t refine_steps, float cond_threshold, float *C, float *factors, int32_t *info,
                        float *cond_est, void *ws, hipStream_t st, int rs_waves = 4);
hipError_t launch_solve_backward(const float *dC, const float *A, const float *B, const float *C, const float *ex,
                                 const float *ey, const float *lam, int32_t mask_kind, float gamma, int64_t P,
                                 int64_t kx, int64_t ky, int64_t d, const float *factors, float *dA, float *dB,
                                 float *dlam, int32_t *info, void *ws, hipStream_t st, int rs_waves = 4);

// Row solves with stored factors (reverse mode, refinement correction) by streaming triangular solves.
void launch_trisolve_stored(const float *Lin, const float *rhs, const float *ex, const float *ey, const float *lam,
                            int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out, int *info,
                            const float *Cfwd, float *dlam_part, const float *addend, hipStream_t st,
                            const int *only = nullptr);
// The same for k_x <= 64: one wave per system, both substitutions in registers.
void launch_trisolve_small(const float *Lin, const float *rhs, const float *ex, const float *ey, const float *lam,
                           int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out, int *info,
                           const float *Cfwd, float *dlam_part, const float *addend, hipStream_t st);
// Row systems for 64 < k_x <= kMaxK: mode 0 forward (factors to Lout if non-NULL), mode 2 reverse mode with
// refactorisation (V rows, per-row dlambda terms).  tile_ws: tiled_workspace_bytes(P, k_x, k_y) bytes.
// only: if non-NULL, the systems of pairs p with only[p] == 0 are skipped (their outputs left as they are).
void launch_rowsolve_tiled(int mode, const float *K, const float *rhs, const float *ex, const float *ey,
                           const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out,
                           float *Lout, int *info, const float *Cfwd, float *dlam_part, float *tile_ws, hipStream_t st,
                           const int *only = nullptr);
size_t tiled_workspace_bytes(int64_t P, int64_t kx, int64_t ky);
void launch_adjoint_general(const float *V, const float *C, const float *A, const float *B, int64_t P, int64_t kx,
                            int64_t ky, int64_t d, float *Wbuf, const float *dlam_part, float *dlam, float *dA,
                            float *dB, hipStream_t st);

// K = A A^T [P][kx][kx] and, with with_R, R = B A^T [P][ky][kx] in float32.
void launch_gram(const float *A, const float *B, int64_t P, int64_t kx, int64_t ky, int64_t d, bool with_R,
                 float *K, float *R, hipStream_t st);
// One system per pair with a given symmetric matrix: S [P][n][n] (n <= kMaxK), right-hand side g [P][n],
// solution out [P][n], info [P]; ex_zero [P][n] and ey_zero [P] must hold zeros (no mask shift is added) and
// lam [P] only flags an invalid value.  tiles: tiled_workspace_bytes(P, n, 1) bytes when n > kSmallK.
void launch_rowsolve_dense(const float *S, const float *g, const float *ex_zero, const float *ey_zero, const float *lam,
                           int64_t P, int64_t n, float *out, int *info, float *tiles, hipStream_t st);
// The vectorized solve with general commutativity operators (kx ky <= kMaxK).
size_t vectorized_workspace_bytes(int64_t P, int64_t kx, int64_t ky);
hipError_t launch_solve_vectorized(const float *A, const float *B, const float *D1, const float *D2, const float *lam,
                                   int64_t P, int64_t kx, int64_t ky, int64_t d, float *C, int32_t *info, void *ws,
                                   hipStream_t st);

void launch_gram64(const float *A, const float *B, int64_t P, int64_t kx, int64_t ky, int64_t d, double *K64,
                   double *R64, hipStream_t st);
void launch_residual64(const float *C, const double *K64, const double *R64, const float *ex, const float *ey,
                       const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *rho,
                       hipStream_t st, const int *only = nullptr);
// flag: if non-NULL, flag[p] = 1 where the pair's products were replaced (estimate above threshold), else 0.
void launch_cond(const float *K, int64_t P, int64_t kx, int64_t ky, float threshold, const double *K64,
                 const double *R64, float *Kout, float *Rout, float *cond_est, hipStream_t st, int *flag = nullptr);
// Largest k_x for the condition estimate (its float32 factor lives in LDS).
constexpr int kMaxCondK = 256;

}  // namespace fmap

// Mixed-precision support of the row solve: float64 normal products, the
// float64 residual of the row systems for iterative refinement, and a 1-norm
// condition estimate of A A^T that selects float64 formation of the normal
// matrix for ill-conditioned pairs.
//
//   gram64_kernel     K64 = A A^T, R64 = B A^T accumulated in float64 (the
//                     float32 inputs multiply exactly in float64)
//   residual64_kernel rho_i = R64_i - (C K64)_i - lambda D_i o c_i, in float64,
//                     for every row i of C (the residual of Eq. (4), row-wise);
//                     the correction S_i delta_i = rho_i reuses the float32
//                     factors (stored-factor row solve with C as addend)
//   cond_kernel       per pair: Cholesky of A A^T in float32 (packed, in LDS),
//                     then Hager's estimate of ||(A A^T)^{-1}||_1 with Higham's
//                     extra probe vector; cond = ||A A^T||_1 * estimate (or +inf
//                     when the factorisation breaks down).  Pairs whose estimate
//                     exceeds the threshold get K, R replaced by the rounded
//                     float64 products before the float32 row factorisations.
#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

// ---------------------------------------------------------------------------
// float64 mask entry (same definition as mask_entry)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mask_entry64(double mu_y, double mu_x, int kind, double gamma, double inv_scale)
{
    if (kind == 0) {
        const double t = mu_y - mu_x;
        return t * t;
    }
    const double ty = fmax(mu_y, 0.0) * inv_scale, tx = fmax(mu_x, 0.0) * inv_scale;
    const double ay = pow(ty, gamma), ax = pow(tx, gamma);
    const double dy = 1.0 / (1.0 + ay * ay), dx = 1.0 / (1.0 + ax * ax);
    const double a = ay * dy - ax * dx, b = dy - dx;
    return a * a + b * b;
}

// ---------------------------------------------------------------------------
// K64 = A A^T (kx x kx) and R64 = B A^T (ky x kx) in float64.  One 256-thread
// workgroup per 16 x 16 output tile; rows staged in LDS in chunks of 64 columns.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gram64_kernel(const float *__restrict__ A, const float *__restrict__ B, int kx,
                                                     int ky, int d, int tkx, int tky, double *__restrict__ K64,
                                                     double *__restrict__ R64)
{
    __shared__ double sx[16][65], sy[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int tiles = tkx * tkx + tky * tkx;
    const int p = blockIdx.x / tiles;
    int t = blockIdx.x % tiles;
    const float *X;
    double *O;
    int rowsX;
    if (t < tkx * tkx) {
        X = A + (size_t)p * kx * d;
        O = K64 + (size_t)p * kx * kx;
        rowsX = kx;
    } else {
        t -= tkx * tkx;
        X = B + (size_t)p * ky * d;
        O = R64 + (size_t)p * ky * kx;
        rowsX = ky;
    }
    const int I = t / tkx, J = t % tkx;
    const float *Y = A + (size_t)p * kx * d;
    double acc = 0.0;
    for (int c0 = 0; c0 < d; c0 += 64) {
        batched_for<4>(
            threadIdx.x, 16 * 64, 256,
            [&](int e) {
                const int r = e >> 6, col = min(c0 + (e & 63), d - 1);
                return float2{X[(size_t)min(I * 16 + r, rowsX - 1) * d + col], Y[(size_t)min(J * 16 + r, kx - 1) * d + col]};
            },
            [&](int e, float2 v) {
                const int r = e >> 6, c = e & 63, col = c0 + c;
                sx[r][c] = (I * 16 + r < rowsX && col < d) ? (double)v.x : 0.0;
                sy[r][c] = (J * 16 + r < kx && col < d) ? (double)v.y : 0.0;
            });
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < 64; ++c) acc = fma(sx[ty][c], sy[tx][c], acc);
        __syncthreads();
    }
    const int row = I * 16 + ty, col = J * 16 + tx;
    if (row < rowsX && col < kx) O[(size_t)row * kx + col] = acc;
}

// ---------------------------------------------------------------------------
// rho[p][i][j] = R64[i][j] - sum_q C[i][q] K64[q][j] - lambda D_ij C[i][j] for a
// block of 16 rows of one pair (float64 arithmetic, result rounded to float32).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void residual64_kernel(const float *__restrict__ C, const double *__restrict__ K64,
                                                         const double *__restrict__ R64, const float *__restrict__ ex,
                                                         const float *__restrict__ ey, const float *__restrict__ lam,
                                                         int mask_kind, float gamma, int kx, int ky,
                                                         float *__restrict__ rho)
{
    extern __shared__ double sC[];  // [16][kx]
    __shared__ double s_red[4];
    const int rb = (ky + 15) / 16;
    const int p = blockIdx.x / rb, i0 = (blockIdx.x % rb) * 16;
    const int tid = threadIdx.x;
    const int nr = min(16, ky - i0);
    batched_for<8>(
        tid, 16 * kx, 256, [&](int e) { return C[((size_t)p * ky + i0) * kx + min(e, nr * kx - 1)]; },
        [&](int e, float v) { sC[e] = e < nr * kx ? (double)v : 0.0; });
    double inv_scale = 1.0;
    if (mask_kind == 1) {
        float mx = -INFINITY;
        for (int q = tid; q < kx; q += 256) mx = fmaxf(mx, ex[(size_t)p * kx + q]);
        for (int q = tid; q < ky; q += 256) mx = fmaxf(mx, ey[(size_t)p * ky + q]);
        mx = wave_max(mx);
        if ((tid & 63) == 0) s_red[tid >> 6] = mx;
        __syncthreads();
        const double m4 = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
        inv_scale = 1.0 / m4;
    }
    __syncthreads();
    const double lamd = (double)lam[p];
    const double *Kp = K64 + (size_t)p * kx * kx;
    for (int j = tid; j < kx; j += 256) {
        double acc[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0;
        for (int q = 0; q < kx; ++q) {
            const double kq = Kp[(size_t)q * kx + j];
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = fma(sC[r * kx + q], kq, acc[r]);
        }
        const double mux = (double)ex[(size_t)p * kx + j];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r < nr) {
                const int i = i0 + r;
                const double D = mask_entry64((double)ey[(size_t)p * ky + i], mux, mask_kind, (double)gamma, inv_scale);
                const double v = R64[((size_t)p * ky + i) * kx + j] - acc[r] - lamd * D * sC[r * kx + j];
                rho[((size_t)p * ky + i) * kx + j] = (float)v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Condition estimate of K = A A^T per pair (one 512-thread workgroup).
//
// ||K||_1 is the largest row sum of |K| (K is symmetric), summed along rows so
// that the loads are coalesced.  The Cholesky factor of K is formed in LDS
// (packed lower, row-major), right-looking: the column is scaled, then the
// trailing triangle is updated with its entries spread evenly over the 512
// threads.  Hager's iteration then runs in one wave with the vectors in
// registers (lane j holds rows j, j + 64, ...): the forward substitution goes
// column by column (y_c final, rows below updated) and the back substitution
// row by row (x_c final, rows above updated), so neither needs a reduction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pk(int r, int c) { return r * (r + 1) / 2 + c; }  // packed lower, row-major

constexpr int CNS = kMaxCondK / 64;  // register slots per lane (k <= 256)

// row c's entry of a slotted vector (c wave-uniform), without runtime indexing of the register array
__device__ __forceinline__ float slot_value(const float (&v)[CNS], int c)
{
    const int l = c & 63, s = c >> 6;
    float r = readlane(v[0], l);
#pragma unroll
    for (int t = 1; t < CNS; ++t) {
        const float x = readlane(v[t], l);
        r = (s == t) ? x : r;
    }
    return r;
}

// v := K^{-1} v with the packed factor L and the reciprocal pivots Dinv in LDS (one wave).  Columns
// go in groups of 8: a group's LDS reads are issued together, then its 8 dependent steps run on
// registers only.
constexpr int CG = 8;
__device__ void chol_solve_regs(const float *L, const float *Dinv, float (&v)[CNS], int k)
{
    const int lane = threadIdx.x & 63;
    for (int c0 = 0; c0 < k; c0 += CG) {  // L y = v, columns ascending
        float lv[CG][CNS], inv[CG];
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const int c = min(c0 + t, k - 1);
            inv[t] = Dinv[c];
#pragma unroll
            for (int s = 0; s < CNS; ++s) {
                const int r = lane + 64 * s;
                lv[t][s] = (r > c && r < k) ? L[pk(r, c)] : 0.f;
            }
        }
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const int c = c0 + t;
            if (c < k) {
                const float yc = slot_value(v, c) * inv[t];
#pragma unroll
                for (int s = 0; s < CNS; ++s) v[s] = (lane + 64 * s == c) ? yc : v[s] - lv[t][s] * yc;
            }
        }
    }
    for (int c1 = k - 1; c1 >= 0; c1 -= CG) {  // L^T x = y, columns descending
        float lv[CG][CNS], inv[CG];
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const int c = max(c1 - t, 0);
            inv[t] = Dinv[c];
#pragma unroll
            for (int s = 0; s < CNS; ++s) {
                const int r = lane + 64 * s;
                lv[t][s] = (r < c) ? L[pk(c, r)] : 0.f;
            }
        }
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const int c = c1 - t;
            if (c >= 0) {
                const float xc = slot_value(v, c) * inv[t];
#pragma unroll
                for (int s = 0; s < CNS; ++s) v[s] = (lane + 64 * s == c) ? xc : v[s] - lv[t][s] * xc;
            }
        }
    }
}

__global__ __launch_bounds__(512) void cond_kernel(const float *__restrict__ K, int kx, float threshold,
                                                   const double *__restrict__ K64, const double *__restrict__ R64,
                                                   float *__restrict__ Kout, float *__restrict__ Rout, int ky,
                                                   float *__restrict__ cond_est)
{
    extern __shared__ float sm[];
    float *L = sm;                     // packed lower, kx(kx+1)/2
    float *Dinv = L + kx * (kx + 1) / 2;  // reciprocal pivots, kx
    __shared__ float s_red[8];
    __shared__ int s_fail;
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float *Kp = K + (size_t)p * kx * kx;
    batched_for<8>(
        tid, kx * kx, 512, [&](int e) { return Kp[e]; },
        [&](int e, float v) {
            const int r = e / kx, c = e - r * kx;
            if (c <= r) L[pk(r, c)] = v;
        });
    if (tid == 0) s_fail = 0;
    __syncthreads();
    // ||K||_1 = max row sum of |K| (symmetric: the strict upper part of row r is column r of L), one wave per row
    float rmax = 0.f;
    for (int r = wave; r < kx; r += 8) {
        float s = 0.f;
        for (int c = lane; c < kx; c += 64) s += fabsf(c <= r ? L[pk(r, c)] : L[pk(c, r)]);
        rmax = fmaxf(rmax, wave_sum(s));
    }
    if (lane == 0) s_red[wave] = rmax;
    __syncthreads();
    float knorm = s_red[0];
    for (int w = 1; w < 8; ++w) knorm = fmaxf(knorm, s_red[w]);
    // right-looking Cholesky in LDS
    for (int c = 0; c < kx; ++c) {
        const float piv = L[pk(c, c)];
        if (!(piv > 0.f) || !isfinite(piv)) {  // uniform: every thread reads the same pivot
            if (tid == 0) s_fail = 1;
            break;
        }
        const float lc = sqrtf(piv);
        __syncthreads();
        if (tid == 0) L[pk(c, c)] = lc;
        for (int r = c + 1 + tid; r < kx; r += 512) L[pk(r, c)] /= lc;
        __syncthreads();
        // trailing triangle rows (c, kx), columns (c, r]: thread -> (row, stride class), so a row's
        // entries are contiguous in the packed layout and all 512 threads share the work evenly
        const int m = kx - c - 1;
        if (m > 0) {
            const int chunks = max(1, 512 / m);
            if (tid < chunks * m) {
                const int rr = tid % m, ch = tid / m;
                const int r = c + 1 + rr;
                const float lrc = L[pk(r, c)];
                float *Lr = L + r * (r + 1) / 2;  // row r
#pragma unroll 4
                for (int qq = ch; qq <= rr; qq += chunks) {
                    const int q = c + 1 + qq;
                    Lr[q] -= lrc * L[pk(q, c)];
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (int c = tid; c < kx; c += 512) Dinv[c] = 1.f / L[pk(c, c)];
    __syncthreads();
    float est = INFINITY;
    if (s_fail == 0) {
        if (wave == 0) {
            // Hager: b = 1/n; up to 5 sweeps of x = K^{-1} b, xi = sign(x), z = K^{-1} xi, b = e_argmax|z|
            float x[CNS], z[CNS];
#pragma unroll
            for (int s = 0; s < CNS; ++s) x[s] = (lane + 64 * s < kx) ? 1.f / kx : 0.f;
            float e1 = 0.f;
            for (int it = 0; it < 5; ++it) {
                chol_solve_regs(L, Dinv, x, kx);
                float a = 0.f;
#pragma unroll
                for (int s = 0; s < CNS; ++s) a += (lane + 64 * s < kx) ? fabsf(x[s]) : 0.f;
                a = wave_sum(a);
                if (it > 0 && a <= e1) break;
                e1 = a;
#pragma unroll
                for (int s = 0; s < CNS; ++s) z[s] = (lane + 64 * s < kx) ? (x[s] >= 0.f ? 1.f : -1.f) : 0.f;
                chol_solve_regs(L, Dinv, z, kx);
                // j = argmax |z| (the smallest index on ties)
                float best = -1.f;
                int bj = 0;
#pragma unroll
                for (int s = 0; s < CNS; ++s) {
                    const int r = lane + 64 * s;
                    if (r < kx && fabsf(z[s]) > best) {
                        best = fabsf(z[s]);
                        bj = r;
                    }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const float ob = __shfl_xor(best, off, 64);
                    const int oj = __shfl_xor(bj, off, 64);
                    if (ob > best || (ob == best && oj < bj)) {
                        best = ob;
                        bj = oj;
                    }
                }
#pragma unroll
                for (int s = 0; s < CNS; ++s) x[s] = (lane + 64 * s == bj) ? 1.f : 0.f;
            }
            // Higham's extra probe: b_i = (-1)^i (1 + i/(n-1)); estimate 2 ||K^{-1} b||_1 / (3n)
#pragma unroll
            for (int s = 0; s < CNS; ++s) {
                const int r = lane + 64 * s;
                z[s] = r < kx ? ((r & 1) ? -1.f : 1.f) * (1.f + (kx > 1 ? (float)r / (kx - 1) : 0.f)) : 0.f;
            }
            chol_solve_regs(L, Dinv, z, kx);
            float s2 = 0.f;
#pragma unroll
            for (int s = 0; s < CNS; ++s) s2 += (lane + 64 * s < kx) ? fabsf(z[s]) : 0.f;
            s2 = wave_sum(s2) * 2.f / (3.f * kx);
            if (lane == 0) s_red[0] = fmaxf(e1, s2) * knorm;
        }
        __syncthreads();
        est = s_red[0];
    }
    if (tid == 0 && cond_est) cond_est[p] = est;
    // ill-conditioned pair: use the float64-formed products (rounded) for the row factorisations
    if (threshold > 0.f && !(est <= threshold) && K64) {
        batched_for<8>(
            tid, kx * kx, 512, [&](int e) { return K64[(size_t)p * kx * kx + e]; },
            [&](int e, double v) { Kout[(size_t)p * kx * kx + e] = (float)v; });
        batched_for<8>(
            tid, ky * kx, 512, [&](int e) { return R64[(size_t)p * ky * kx + e]; },
            [&](int e, double v) { Rout[(size_t)p * ky * kx + e] = (float)v; });
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

void launch_gram64(const float *A, const float *B, int64_t P, int64_t kx, int64_t ky, int64_t d, double *K64,
                   double *R64, hipStream_t st)
{
    const int tkx = (int)((kx + 15) / 16), tky = (int)((ky + 15) / 16);
    hipLaunchKernelGGL(gram64_kernel, dim3((unsigned)(P * (tkx * tkx + tky * tkx))), dim3(256), 0, st, A, B, (int)kx,
                       (int)ky, (int)d, tkx, tky, K64, R64);
}

void launch_residual64(const float *C, const double *K64, const double *R64, const float *ex, const float *ey,
                       const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *rho,
                       hipStream_t st)
{
    const size_t lds = (size_t)16 * kx * sizeof(double);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)residual64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(16 * kMaxK * sizeof(double)));
        attr = true;
    }
    hipLaunchKernelGGL(residual64_kernel, dim3((unsigned)(P * ((ky + 15) / 16))), dim3(256), lds, st, C, K64, R64,
                       ex, ey, lam, mask_kind, gamma, (int)kx, (int)ky, rho);
}

void launch_cond(const float *K, int64_t P, int64_t kx, int64_t ky, float threshold, const double *K64,
                 const double *R64, float *Kout, float *Rout, float *cond_est, hipStream_t st)
{
    const size_t lds = ((size_t)kx * (kx + 1) / 2 + kx) * sizeof(float);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)cond_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(((size_t)kMaxCondK * (kMaxCondK + 1) / 2 + kMaxCondK) * sizeof(float)));
        attr = true;
    }
    hipLaunchKernelGGL(cond_kernel, dim3((unsigned)P), dim3(512), lds, st, K, (int)kx, threshold, K64, R64, Kout, Rout,
                       (int)ky, cond_est);
}

}  // namespace fmap

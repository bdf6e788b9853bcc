// Row-decoupled regularised solve, Eqs. (4)-(9), and its reverse mode.
//
// Forward, per pair p:
//   gram_kernel      K = A A^T (k_x x k_x) and R = B A^T (k_y x k_x), Eq. (8)'s
//                    shared products, on the float32 matrix cores.
//   rowsolve_kernel  one wave per row system i:  S_i = K + lambda diag(D_i)
//                    (the mask row D_i is evaluated on the fly from the two
//                    eigenvalue sets, Eq. (3)), Cholesky S_i = L L^T, then
//                    L y = R_i, L^T c_i = y (Eqs. (5)-(7)).  Rows of all pairs
//                    form one batched launch (Eq. (8)); the [k,k,k] left-hand
//                    side of Eq. (9) is never materialised.
// Reverse mode (dC given), per pair:
//   rowsolve_kernel  v_i = S_i^{-1} dC_i with the stored factor (or a refactor)
//   adjoint_kernel   W = V^T C + C^T V, dA = V^T B - W A, dB = V A.
//
// Register Cholesky: lane j of the wave holds row j of S_i (entries q <= j;
// the strict upper part is kept at zero).  At step c the pivot comes from
// lane c (readlane), every lane scales its entry of column c, the new column
// is broadcast through LDS and each lane applies the rank-1 update to its row.
// Work per step is uniform, so the wave never diverges; a non-positive pivot
// is detected uniformly and stops the factorisation (LAPACK info).
#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

enum { RS_FWD = 0, RS_BWD_STORED = 1, RS_BWD_RECOMPUTE = 2 };

// ---------------------------------------------------------------------------
// K = A A^T and (optionally) R = B A^T.  One workgroup per 32x32 output tile;
// its four waves split the feature range d and reduce through LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gram_kernel(const float *__restrict__ A, const float *__restrict__ B, int kx,
                                                   int ky, int d, int tkx, int tky, int with_R,
                                                   float *__restrict__ K, float *__restrict__ R)
{
    __shared__ float red[4][16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int tiles = tkx * tkx + (with_R ? tky * tkx : 0);
    const int p = blockIdx.x / tiles;
    int t = blockIdx.x % tiles;
    const float *X;
    float *O;
    int rowsX;
    if (t < tkx * tkx) {
        X = A + (size_t)p * kx * d;
        O = K + (size_t)p * kx * kx;
        rowsX = kx;
    } else {
        t -= tkx * tkx;
        X = B + (size_t)p * ky * d;
        O = R + (size_t)p * ky * kx;
        rowsX = ky;
    }
    const int I = t / tkx, J = t % tkx;
    const float *Y = A + (size_t)p * kx * d;
    const int m = I * 32 + l32, nn = J * 32 + l32;
    const bool mok = m < rowsX, nok = nn < kx;

    // wave range of d, split into two halves for the two lane halves
    const int dq = (d + 3) / 4;
    const int lo = wave * dq, hi = min(d, lo + dq);
    const int H = (max(hi - lo, 0) + 1) >> 1;
    f32x16 acc = zero16();
    for (int s = 0; s < H; ++s) {
        const int dd = lo + half * H + s;
        const bool ok = dd < hi;
        const float a = (mok && ok) ? X[(size_t)m * d + dd] : 0.f;
        const float b = (nok && ok) ? Y[(size_t)nn * d + dd] : 0.f;
        acc = mfma32x32x2(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float v = red[0][r][lane] + red[1][r][lane] + red[2][r][lane] + red[3][r][lane];
            const int row = I * 32 + acc32_row(r, lane);
            if (row < rowsX && nok) O[(size_t)row * kx + nn] = v;
        }
    }
}

// Offset of column c in LAPACK lower packed column-major storage of order m.
__device__ __forceinline__ int packed_col(int c, int m) { return c * m - (c * (c - 1)) / 2; }

// ---------------------------------------------------------------------------
// One wave per row system.  KMAX >= k_x (register row length).
// ---------------------------------------------------------------------------
template <int KMAX, int MODE>
__global__ __launch_bounds__(256) void rowsolve_kernel(
    const float *__restrict__ K, const float *__restrict__ Lin, const float *__restrict__ rhs,
    const float *__restrict__ ex, const float *__restrict__ ey, const float *__restrict__ lam, int mask_kind,
    float gamma, int kx, int ky, float *__restrict__ out, float *__restrict__ Lout, int *__restrict__ info,
    const float *__restrict__ Cfwd, float *__restrict__ dlam_part)
{
    __shared__ __align__(16) float s_bc[4][KMAX];
    __shared__ float s_L[4][KMAX * (KMAX + 1) / 2];  // rows of L, packed (row r at r(r+1)/2)
    const int j = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rgroups = (ky + 3) >> 2;
    const int p = blockIdx.x / rgroups;
    const int i = (blockIdx.x % rgroups) * 4 + w;
    if (i >= ky) return;  // wave-uniform; no block-level barrier below
    const int T = kx * (kx + 1) / 2;
    const bool jok = j < kx;

    // --- mask row i and validity of lambda / normaliser -------------------------
    const float lamv = lam[p];
    int fail = 0;
    if (!(lamv >= 0.f) || !isfinite(lamv)) fail = -1;
    MaskParams mp;
    mp.kind = mask_kind;
    mp.gamma = gamma;
    mp.inv_scale = 1.f;
    if (mask_kind == 1) {
        float mx = -INFINITY;
        for (int q = j; q < kx; q += 64) mx = fmaxf(mx, ex[(size_t)p * kx + q]);
        for (int q = j; q < ky; q += 64) mx = fmaxf(mx, ey[(size_t)p * ky + q]);
        mx = wave_max(mx);
        if ((!(mx > 0.f) || !isfinite(mx)) && fail == 0) fail = -2;
        mp.inv_scale = 1.f / mx;
    }
    const float muy = ey[(size_t)p * ky + i];
    const float dval = (jok && fail == 0) ? mask_entry(muy, ex[(size_t)p * kx + j], mp) : 0.f;
    const float shift = lamv * dval;

    // --- load row j of S_i (lower part) or of the stored factor -----------------
    float sr[KMAX];
    if (MODE == RS_BWD_STORED) {
        const float *Lp = Lin + ((size_t)p * ky + i) * T;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) sr[q] = (jok && q <= j) ? Lp[packed_col(q, kx) + j - q] : 0.f;
    } else {
        const float *Kp = K + (size_t)p * kx * kx + (size_t)j * kx;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) sr[q] = (jok && q <= j) ? Kp[q] : 0.f;
    }

    // --- Cholesky of S_i = K + diag(shift) -----------------------------------------
    // All loops have static bounds so that sr[] stays in registers; the runtime
    // size kx only enters through wave-uniform branches.
    if (MODE != RS_BWD_STORED) {
        float *bc = s_bc[w];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            if (c < kx && fail == 0) {
                const float piv = readlane(sr[c], c) + readlane(shift, c);
                if (!(piv > 0.f) || !isfinite(piv)) {
                    fail = c + 1;
                } else {
                    const float sq = sqrtf(piv);
                    const float inv = 1.f / sq;
                    const float l = (j > c) ? sr[c] * inv : ((j == c) ? sq : 0.f);
                    sr[c] = l;
                    if (j < KMAX) bc[j] = l;  // lanes >= KMAX hold zero rows
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int q4 = 0; q4 < KMAX / 4; ++q4) {
                        if (4 * q4 + 3 > c && 4 * q4 < kx) {
                            const f32x4 lq = *reinterpret_cast<const f32x4 *>(&bc[4 * q4]);
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (4 * q4 + e > c) sr[4 * q4 + e] -= l * lq[e];
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            if (c < kx && fail == 0) {
                const float dg = readlane(sr[c], c);
                if (!(dg > 0.f) || !isfinite(dg)) fail = c + 1;
            }
        }
    }

    float cv = NAN;
    if (fail == 0) {
        // forward substitution L y = r (column oriented; lane c finishes at step c)
        float r = jok ? rhs[((size_t)p * ky + i) * kx + j] : 0.f;
        float yv = 0.f;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            if (c < kx) {
                const float yc = readlane(r, c) / readlane(sr[c], c);
                if (j == c) yv = yc;
                r -= sr[c] * yc;
            }
        }
        // back substitution L^T c = y with the rows of L staged in LDS
        float *Lr = s_L[w];
        const int rowoff = j * (j + 1) / 2;
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
            if (j < KMAX && q <= j) Lr[rowoff + q] = sr[q];
        __builtin_amdgcn_wave_barrier();
        float y = yv;
        cv = 0.f;
#pragma unroll
        for (int c = KMAX - 1; c >= 0; --c) {
            if (c < kx) {
                const float cc = readlane(y, c) / readlane(sr[c], c);
                if (j == c) cv = cc;
                if (j < c) y -= Lr[c * (c + 1) / 2 + j] * cc;  // L[c][j], j < c
            }
        }
        __builtin_amdgcn_wave_barrier();
    }

    if (jok) out[((size_t)p * ky + i) * kx + j] = cv;
    if (info && j == 0) info[(size_t)p * ky + i] = fail;
    if (MODE == RS_FWD && Lout) {
        float *Lp = Lout + ((size_t)p * ky + i) * T;
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
            if (q < kx && jok && j >= q) Lp[packed_col(q, kx) + j - q] = fail == 0 ? sr[q] : NAN;
    }
    if (MODE != RS_FWD && dlam_part) {
        const float cf = jok ? Cfwd[((size_t)p * ky + i) * kx + j] : 0.f;
        const float term = jok ? cv * dval * cf : 0.f;
        const float sum = wave_sum(term);
        if (j == 0) dlam_part[(size_t)p * ky + i] = -sum;
    }
}

// ---------------------------------------------------------------------------
// Adjoint products for one pair and one 64-column block of d:
//   W = V^T C + C^T V,  dA = V^T B - W A,  dB = V A.
// ---------------------------------------------------------------------------
template <int KM>
__global__ __launch_bounds__(256) void adjoint_kernel(const float *__restrict__ V, const float *__restrict__ C,
                                                      const float *__restrict__ A, const float *__restrict__ B,
                                                      int kx, int ky, int d, int dblocks,
                                                      const float *__restrict__ dlam_part, float *__restrict__ dlam,
                                                      float *__restrict__ dA, float *__restrict__ dB)
{
    __shared__ float sV[KM * KM], sC[KM * KM], sW[KM * KM];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int p = blockIdx.x / dblocks, db = blockIdx.x % dblocks;
    const int d0 = db * 64;
    const float *Vp = V + (size_t)p * ky * kx;
    const float *Cp = C + (size_t)p * ky * kx;
    const float *Ap = A + (size_t)p * kx * d;
    const float *Bp = B + (size_t)p * ky * d;
    for (int e = threadIdx.x; e < ky * kx; e += 256) {
        sV[e] = Vp[e];
        sC[e] = Cp[e];
    }
    if (db == 0 && dlam && threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < ky; ++i) s += dlam_part[(size_t)p * ky + i];
        dlam[p] = s;
    }
    __syncthreads();

    const int TI = (kx + 31) / 32, TY = (ky + 31) / 32;
    // W tiles (TI*TI <= 4)
    if (wave < TI * TI) {
        const int I = wave / TI, J = wave % TI;
        const int m = I * 32 + l32, nn = J * 32 + l32;
        const bool mok = m < kx, nok = nn < kx;
        f32x16 acc = zero16();
        for (int t = 0; t < ky; ++t) {
            float a, b;
            if (half == 0) {
                a = mok ? sV[t * kx + m] : 0.f;
                b = nok ? sC[t * kx + nn] : 0.f;
            } else {
                a = mok ? sC[t * kx + m] : 0.f;
                b = nok ? sV[t * kx + nn] : 0.f;
            }
            acc = mfma32x32x2(a, b, acc);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = I * 32 + acc32_row(r, lane);
            if (row < kx && nok) sW[row * kx + nn] = acc[r];
        }
    }
    __syncthreads();

    const int nA = TI * 2, nB = TY * 2;
    for (int job = wave; job < nA + nB; job += 4) {
        f32x16 acc = zero16();
        if (job < nA) {
            const int I = job >> 1, cblk = job & 1;
            const int m = I * 32 + l32, col = d0 + cblk * 32 + l32;
            const bool mok = m < kx, cok = col < d;
            const int steps = max(kx, ky);
            for (int t = 0; t < steps; ++t) {
                float a = 0.f, b = 0.f;
                if (half == 0) {
                    if (t < ky) {
                        a = mok ? sV[t * kx + m] : 0.f;
                        b = cok ? Bp[(size_t)t * d + col] : 0.f;
                    }
                } else {
                    if (t < kx) {
                        a = mok ? -sW[t * kx + m] : 0.f;
                        b = cok ? Ap[(size_t)t * d + col] : 0.f;
                    }
                }
                acc = mfma32x32x2(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = I * 32 + acc32_row(r, lane);
                if (row < kx && cok) dA[((size_t)p * kx + row) * d + col] = acc[r];
            }
        } else {
            const int jb = job - nA;
            const int I = jb >> 1, cblk = jb & 1;
            const int m = I * 32 + l32, col = d0 + cblk * 32 + l32;
            const bool mok = m < ky, cok = col < d;
            const int KH = (kx + 1) >> 1;
            for (int t = 0; t < KH; ++t) {
                const int kk = half * KH + t;
                const bool kok = kk < kx;
                const float a = (mok && kok) ? sV[m * kx + kk] : 0.f;
                const float b = (cok && kok) ? Ap[(size_t)kk * d + col] : 0.f;
                acc = mfma32x32x2(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = I * 32 + acc32_row(r, lane);
                if (row < ky && cok) dB[((size_t)p * ky + row) * d + col] = acc[r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SolveWs solve_workspace_layout(int64_t P, int64_t kx, int64_t ky, int64_t d)
{
    (void)d;
    SolveWs w;
    size_t off = 0;
    w.K = off;
    off += align256((size_t)P * kx * kx * sizeof(float));
    w.R = off;
    off += align256((size_t)P * ky * kx * sizeof(float));
    w.V = off;
    off += align256((size_t)P * ky * kx * sizeof(float));
    w.dlam = off;
    off += align256((size_t)P * ky * sizeof(float));
    w.total = off;
    return w;
}

static void launch_gram(const float *A, const float *B, int64_t P, int64_t kx, int64_t ky, int64_t d, bool with_R,
                        float *K, float *R, hipStream_t st)
{
    const int tkx = (int)((kx + 31) / 32), tky = (int)((ky + 31) / 32);
    const int tiles = tkx * tkx + (with_R ? tky * tkx : 0);
    hipLaunchKernelGGL(gram_kernel, dim3((unsigned)(P * tiles)), dim3(256), 0, st, A, B, (int)kx, (int)ky, (int)d,
                       tkx, tky, with_R ? 1 : 0, K, R);
}

template <int MODE>
static void launch_rowsolve(const float *K, const float *Lin, const float *rhs, const float *ex, const float *ey,
                            const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky,
                            float *out, float *Lout, int *info, const float *Cfwd, float *dlam_part, hipStream_t st)
{
    const unsigned grid = (unsigned)(P * ((ky + 3) / 4));
    if (kx <= 32)
        hipLaunchKernelGGL((rowsolve_kernel<32, MODE>), dim3(grid), dim3(256), 0, st, K, Lin, rhs, ex, ey, lam,
                           mask_kind, gamma, (int)kx, (int)ky, out, Lout, info, Cfwd, dlam_part);
    else
        hipLaunchKernelGGL((rowsolve_kernel<64, MODE>), dim3(grid), dim3(256), 0, st, K, Lin, rhs, ex, ey, lam,
                           mask_kind, gamma, (int)kx, (int)ky, out, Lout, info, Cfwd, dlam_part);
}

hipError_t launch_solve(const float *A, const float *B, const float *ex, const float *ey, const float *lam,
                        int32_t mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, int64_t d,
                        int32_t refine_steps, float cond_threshold, float *C, float *factors, int32_t *info,
                        float *cond_est, void *ws, hipStream_t st)
{
    (void)refine_steps;
    (void)cond_threshold;
    (void)cond_est;
    SolveWs L = solve_workspace_layout(P, kx, ky, d);
    char *base = (char *)ws;
    float *K = (float *)(base + L.K), *R = (float *)(base + L.R);
    launch_gram(A, B, P, kx, ky, d, true, K, R, st);
    launch_rowsolve<RS_FWD>(K, nullptr, R, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, factors, info, nullptr,
                            nullptr, st);
    return hipGetLastError();
}

hipError_t launch_solve_backward(const float *dC, const float *A, const float *B, const float *C, const float *ex,
                                 const float *ey, const float *lam, int32_t mask_kind, float gamma, int64_t P,
                                 int64_t kx, int64_t ky, int64_t d, const float *factors, float *dA, float *dB,
                                 float *dlam, int32_t *info, void *ws, hipStream_t st)
{
    SolveWs L = solve_workspace_layout(P, kx, ky, d);
    char *base = (char *)ws;
    float *K = (float *)(base + L.K), *V = (float *)(base + L.V), *dl = (float *)(base + L.dlam);
    if (factors) {
        launch_rowsolve<RS_BWD_STORED>(nullptr, factors, dC, ex, ey, lam, mask_kind, gamma, P, kx, ky, V, nullptr,
                                       info, C, dl, st);
    } else {
        launch_gram(A, B, P, kx, ky, d, false, K, nullptr, st);
        launch_rowsolve<RS_BWD_RECOMPUTE>(K, nullptr, dC, ex, ey, lam, mask_kind, gamma, P, kx, ky, V, nullptr, info,
                                          C, dl, st);
    }
    const int dblocks = (int)((d + 63) / 64);
    hipLaunchKernelGGL((adjoint_kernel<kSmallK>), dim3((unsigned)(P * dblocks)), dim3(256), 0, st, V, C, A, B,
                       (int)kx, (int)ky, (int)d, dblocks, dl, dlam, dA, dB);
    return hipGetLastError();
}

}  // namespace fmap

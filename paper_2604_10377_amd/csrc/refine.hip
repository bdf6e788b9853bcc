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
// workgroup per 32 x 32 output tile; rows staged in LDS in chunks of 64 columns.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gram64_kernel(const float *__restrict__ A, const float *__restrict__ B, int kx,
                                                     int ky, int d, int tkx, int tky, double *__restrict__ K64,
                                                     double *__restrict__ R64)
{
    // 32 x 32 output tile, a thread owns rows ty, ty + 16 x columns tx, tx + 16 (one LDS read per product;
    // with one output per thread it was two, and the kernel was bound by LDS bandwidth)
    __shared__ double sx[32][65], sy[32][65];
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
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int c0 = 0; c0 < d; c0 += 64) {
        batched_for<8>(
            threadIdx.x, 32 * 64, 256,
            [&](int e) {
                const int r = e >> 6, col = min(c0 + (e & 63), d - 1);
                return float2{X[(size_t)min(I * 32 + r, rowsX - 1) * d + col], Y[(size_t)min(J * 32 + r, kx - 1) * d + col]};
            },
            [&](int e, float2 v) {
                const int r = e >> 6, c = e & 63, col = c0 + c;
                sx[r][c] = (I * 32 + r < rowsX && col < d) ? (double)v.x : 0.0;
                sy[r][c] = (J * 32 + r < kx && col < d) ? (double)v.y : 0.0;
            });
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < 64; ++c) {
            const double x0 = sx[ty][c], x1 = sx[ty + 16][c], y0 = sy[tx][c], y1 = sy[tx + 16][c];
            acc[0][0] = fma(x0, y0, acc[0][0]);
            acc[0][1] = fma(x0, y1, acc[0][1]);
            acc[1][0] = fma(x1, y0, acc[1][0]);
            acc[1][1] = fma(x1, y1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int row = I * 32 + ty + 16 * a, col = J * 32 + tx + 16 * b;
            if (row < rowsX && col < kx) O[(size_t)row * kx + col] = acc[a][b];
        }
}

// ---------------------------------------------------------------------------
// The same products on the float64 matrix cores (v_mfma_f64_16x16x4f64), for d % 8 == 0.  One wave per
// 16 x 16 output tile: the lower-triangle tiles of the symmetric K64 (an off-diagonal tile is also
// written mirrored) and every tile of R64.  Lane (i, q) feeds row i of its operands with columns
// kb + 8 q + u to matrix step u of a 32-column batch, so each lane reads two 16-byte pieces per operand
// and batch; the next batch is loaded while the current one is multiplied.  Workgroup ids are remapped
// so that consecutive tiles, and so the tiles of one pair, share an XCD (ids in one residue class mod 8).
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gram64_mfma_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                          int kx, int ky, int d, int tkx, int tky, long long ntiles,
                                                          int per_xcd, double *__restrict__ K64,
                                                          double *__restrict__ R64)
{
    const int wid = blockIdx.x;
    const long long lwg = (long long)(wid & 7) * per_xcd + (wid >> 3);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long g = lwg * 4 + wave;
    if (g >= ntiles) return;  // no barriers below
    const int ktiles = tkx * (tkx + 1) / 2, per_pair = ktiles + tky * tkx;
    const int p = (int)(g / per_pair);
    int t = (int)(g % per_pair);
    int I, J, rowsX;
    const float *X;
    double *O;
    const bool sym = t < ktiles;
    if (sym) {  // t = I (I + 1) / 2 + J, J <= I
        I = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        while (I * (I + 1) / 2 > t) --I;
        J = t - I * (I + 1) / 2;
        X = A + (size_t)p * kx * d;
        O = K64 + (size_t)p * kx * kx;
        rowsX = kx;
    } else {
        t -= ktiles;
        I = t / tkx;
        J = t % tkx;
        X = B + (size_t)p * ky * d;
        O = R64 + (size_t)p * ky * kx;
        rowsX = ky;
    }
    const int i16 = lane & 15, q = lane >> 4;
    // rows past the matrix read a clamped row; they only reach outputs that are not stored
    const float *xr = X + (size_t)min(I * 16 + i16, rowsX - 1) * d;
    const float *yr = A + (size_t)p * kx * d + (size_t)min(J * 16 + i16, kx - 1) * d;
    struct Batch {
        f32x4 x0, x1, y0, y1;
    };
    auto load = [&](int kb) {
        const int o = min(kb + 8 * q, d - 8);  // a batch past d reads in bounds and is masked
        Batch b;
        b.x0 = *reinterpret_cast<const f32x4 *>(xr + o);
        b.x1 = *reinterpret_cast<const f32x4 *>(xr + o + 4);
        b.y0 = *reinterpret_cast<const f32x4 *>(yr + o);
        b.y1 = *reinterpret_cast<const f32x4 *>(yr + o + 4);
        return b;
    };
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    auto mma = [&](int kb, const Batch &b) {
        const bool ok = kb + 8 * q < d;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float xv = u < 4 ? b.x0[u & 3] : b.x1[u & 3];
            const float yv = u < 4 ? b.y0[u & 3] : b.y1[u & 3];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ok ? (double)xv : 0.0, (double)yv, acc, 0, 0, 0);
        }
    };
    const int nb = (((d + 31) / 32) + 1) & ~1;  // batches, rounded up to even for the two-buffer rotation
    Batch b0 = load(0), b1;
    for (int j = 0; j < nb; j += 2) {
        const int kb = 32 * j;
        b1 = load(kb + 32);
        mma(kb, b0);
        b0 = load(kb + 64);
        mma(kb + 32, b1);
    }
    // acc[r] = D[q + 4 r][i16] (the float64 instruction's result layout)
    const int col = J * 16 + i16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = I * 16 + q + 4 * r;
        if (row < rowsX && col < kx) {
            O[(size_t)row * kx + col] = acc[r];
            if (sym && I != J) O[(size_t)col * kx + row] = acc[r];
        }
    }
}

// ---------------------------------------------------------------------------
// rho[p][i][j] = R64[i][j] - sum_q C[i][q] K64[q][j] - lambda D_ij C[i][j] for a
// block of 16 rows of one pair (float64 arithmetic, result rounded to float32).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void residual64_kernel(const float *__restrict__ C, const double *__restrict__ K64,
                                                         const double *__restrict__ R64, const float *__restrict__ ex,
                                                         const float *__restrict__ ey, const float *__restrict__ lam,
                                                         int mask_kind, float gamma, int kx, int ky,
                                                         float *__restrict__ rho, const int *__restrict__ only)
{
    extern __shared__ double sC[];  // [16][kx]
    __shared__ double s_red[4];
    const int rb = (ky + 15) / 16;
    const int p = blockIdx.x / rb, i0 = (blockIdx.x % rb) * 16;
    if (only && only[p] == 0) return;  // whole workgroup, before any barrier
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
        // K64 entries in groups of 8, all loaded before the group's products (one at a time, each load
        // was waited for before its 16 products); the products keep their order
        int q = 0;
        for (; q + 8 <= kx; q += 8) {
            double kq[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) kq[u] = Kp[(size_t)(q + u) * kx + j];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] = fma(sC[r * kx + q + u], kq[u], acc[r]);
        }
        for (; q < kx; ++q) {
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
// Condition estimate of K = A A^T per pair (one workgroup of 16 waves).
//
// ||K||_1 is the largest row sum of |K| (K is symmetric), summed along rows so
// that the loads are coalesced.  The Cholesky factor of K is formed in LDS
// (packed lower, row-major), right-looking in panels of 8 columns: one wave
// factorises a panel in registers, then the trailing triangle is updated one
// wave per row, the lanes across the row's contiguous entries.  The solves'
// LDS operand reads are unconditional, from clamped addresses (masked by a
// bit mask).  Hager's
// iteration then runs in one wave with the vectors in
// registers (lane j holds rows j, j + 64, ...): the forward substitution goes
// column by column (y_c final, rows below updated) and the back substitution
// row by row (x_c final, rows above updated), so neither needs a reduction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pk(int r, int c) { return r * (r + 1) / 2 + c; }  // packed lower, row-major

constexpr int CNS = kMaxCondK / 64;  // register slots per lane (k <= 256)
constexpr int CPW = 8;                 // Cholesky panel width
// LDS floats past the last array: the triangular solves' reads for the columns k .. k + 6 of a last
// partial group (never used) stay inside the allocation; row c < k + 7 ends before
// k(k+1)/2 + (1 + CPW) k + CPAD for every k
constexpr int CPAD = 32;

constexpr int CG = 8;  // columns per group of the triangular solves
constexpr int CWV = 16, CTH = 64 * CWV;  // waves and threads of the estimate's workgroup

// x if ok, else +0, by a bit mask: the read that produced x stays unconditional (a select would let the
// compiler put the read under a branch of its own)
__device__ __forceinline__ float keep_if(float x, bool ok) { return __uint_as_float(__float_as_uint(x) & (ok ? ~0u : 0u)); }

// v := K^{-1} v with the packed factor L and the reciprocal pivots Dinv in LDS (one wave; lane l holds rows
// l + 64 s in slot s).  Columns go in groups of 8 within the 64 rows of one slot S (a runtime loop over the
// groups, the group unrolled): a group's LDS reads are issued before its 8 dependent steps, each step's
// broadcast is a readlane from the one slot S, and only the slots that can hold affected rows are
// touched.  Forward L y = v, columns ascending: at step c the rows below subtract L_rc (v_c / L_cc);
// column c's entries below the diagonal are row r's entry c (at rb[s] + c, rb the packed offset of the
// lane's row, clamped into the matrix).  A lane's own value is never touched at its own step, so it ends
// as L_rr y_r and one scaling at the end gives y (no per-column lane selects).  Back L^T x = y the same
// way, columns descending, with row c's entries left of the diagonal (consecutive for consecutive lanes).
// The steps of a last partial group past k - 1 read the allocation's zeroed padding or other finite LDS
// data and broadcast v_c = 0 (rows past k stay 0), so they change nothing and need no per-column guard.
template <int S>
__device__ __forceinline__ void chol_fwd_slot(const float *L, const float *Dinv, float (&v)[CNS], int k,
                                              const int (&rb)[CNS], int lane)
{
    for (int g = 0; g < 64 && 64 * S + g < k; g += CG) {
        const int c0 = 64 * S + g;
        float lv[CG][CNS], inv[CG];
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const int c = c0 + t;
            inv[t] = Dinv[c];
#pragma unroll
            for (int s = S; s < CNS; ++s) {
                const int r = lane + 64 * s;
                lv[t][s] = keep_if(L[rb[s] + c], r > c && r < k);
            }
        }
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const float yc = readlane(v[S], g + t) * inv[t];
#pragma unroll
            for (int s = S; s < CNS; ++s) v[s] = fmaf(-lv[t][s], yc, v[s]);
        }
    }
}

template <int S>
__device__ __forceinline__ void chol_bwd_slot(const float *L, const float *Dinv, float (&v)[CNS], int k, int lane)
{
    // groups of this slot below k, highest first
    const int top = min(64, k - 64 * S);  // > 0 when called
    for (int g = ((top - 1) / CG) * CG; g >= 0; g -= CG) {
        const int c0 = 64 * S + g;  // the group is columns c0 + CG - 1 down to c0
        float lv[CG][CNS], inv[CG];
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const int c = c0 + CG - 1 - t;
            const int cb = c * (c + 1) / 2;
            inv[t] = Dinv[c];
#pragma unroll
            for (int s = 0; s <= S; ++s) {
                const int r = lane + 64 * s;
                lv[t][s] = keep_if(L[cb + min(r, c)], r < c);
            }
        }
#pragma unroll
        for (int t = 0; t < CG; ++t) {
            const float xc = readlane(v[S], g + CG - 1 - t) * inv[t];
#pragma unroll
            for (int s = 0; s <= S; ++s) v[s] = fmaf(-lv[t][s], xc, v[s]);
        }
    }
}

__device__ __forceinline__ void chol_solve_regs(const float *L, const float *Dinv, float (&v)[CNS], int k_in)
{
    static_assert(CNS == 4, "slots unrolled below");
    // k made opaque per call, so that nothing derived from it is hoisted out of the caller's iteration loop
    // into scalar registers held across it
    int k = k_in;
    asm volatile("" : "+s"(k));
    const int lane = threadIdx.x & 63;
    int rb[CNS];
    float dinv[CNS];
#pragma unroll
    for (int s = 0; s < CNS; ++s) {
        const int r = min(lane + 64 * s, k - 1);
        rb[s] = r * (r + 1) / 2;
        dinv[s] = Dinv[r];
    }
    chol_fwd_slot<0>(L, Dinv, v, k, rb, lane);
    if (k > 64) chol_fwd_slot<1>(L, Dinv, v, k, rb, lane);
    if (k > 128) chol_fwd_slot<2>(L, Dinv, v, k, rb, lane);
    if (k > 192) chol_fwd_slot<3>(L, Dinv, v, k, rb, lane);
#pragma unroll
    for (int s = 0; s < CNS; ++s) v[s] *= dinv[s];  // y
    if (k > 192) chol_bwd_slot<3>(L, Dinv, v, k, lane);
    if (k > 128) chol_bwd_slot<2>(L, Dinv, v, k, lane);
    if (k > 64) chol_bwd_slot<1>(L, Dinv, v, k, lane);
    chol_bwd_slot<0>(L, Dinv, v, k, lane);
#pragma unroll
    for (int s = 0; s < CNS; ++s) v[s] *= dinv[s];  // x
}

__global__ __launch_bounds__(CTH) void cond_kernel(const float *__restrict__ K, int kx, float threshold,
                                                   const double *__restrict__ K64, const double *__restrict__ R64,
                                                   float *__restrict__ Kout, float *__restrict__ Rout, int ky,
                                                   float *__restrict__ cond_est, int *__restrict__ flag)
{
    extern __shared__ __align__(16) float sm[];
    float *L = sm;                     // packed lower, kx(kx+1)/2
    float *Dinv = L + kx * (kx + 1) / 2;  // reciprocal pivots, kx
    float *Pn = sm + ((kx * (kx + 1) / 2 + kx + 3) & ~3);  // the current panel, row by row: [kx][8] (16-byte rows)
    __shared__ float s_red[CWV];
    __shared__ int s_fail;
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float *Kp = K + (size_t)p * kx * kx;
    batched_for<8>(
        tid, kx * kx, CTH, [&](int e) { return Kp[e]; },
        [&](int e, float v) {
            const int r = e / kx, c = e - r * kx;
            if (c <= r) L[pk(r, c)] = v;
        });
    if (tid == 0) s_fail = 0;
    {  // the alignment gap after Dinv and the padding after Pn are read (never used) by the solves' last groups
        const int gap0 = kx * (kx + 1) / 2 + kx, gap1 = (gap0 + 3) & ~3, pad0 = gap1 + CPW * kx;
        for (int e = gap0 + tid; e < gap1; e += CTH) sm[e] = 0.f;
        for (int e = pad0 + tid; e < pad0 + CPAD; e += CTH) sm[e] = 0.f;
    }
    __syncthreads();
    // ||K||_1 = max row sum of |K| (symmetric: the strict upper part of row r is column r of L), one wave per row
    float rmax = 0.f;
    for (int r = wave; r < kx; r += CWV) {
        float s = 0.f;
        for (int c = lane; c < kx; c += 64) s += fabsf(c <= r ? L[pk(r, c)] : L[pk(c, r)]);
        rmax = fmaxf(rmax, wave_sum(s));
    }
    if (lane == 0) s_red[wave] = rmax;
    __syncthreads();
    float knorm = s_red[0];
    for (int w = 1; w < CWV; ++w) knorm = fmaxf(knorm, s_red[w]);
    // Blocked right-looking Cholesky in LDS, panels of CPW columns.  Wave 0 factorises the panel in
    // registers (lane l holds rows c0 + l + 64 s of the panel's columns; the pivots and the panel's own
    // rows come by readlane) and writes it back, also row by row to Pn.  Then every wave updates the
    // trailing rows, one row per wave with the lanes across its entries (contiguous in the packed
    // rows): L[r][q] -= sum_t L[r][c0+t] L[q][c0+t], one fused multiply-add per t in column order, which
    // are the same operations, in the same order, as a column-at-a-time factorisation.
    for (int c0 = 0; c0 < kx; c0 += CPW) {
        if (wave == 0) {
            float pv[CNS][CPW];
#pragma unroll
            for (int s = 0; s < CNS; ++s) {
                const int rc = min(c0 + lane + 64 * s, kx - 1);
#pragma unroll
                for (int t = 0; t < CPW; ++t) pv[s][t] = L[pk(rc, min(c0 + t, rc))];  // clamped into the triangle
            }
            bool bad = false;
#pragma unroll
            for (int t = 0; t < CPW; ++t) {
                const int c = c0 + t;
                if (c < kx && !bad) {  // wave-uniform
                    const float piv = readlane(pv[0][t], t);  // row c is lane t, slot 0
                    if (!(piv > 0.f) || !isfinite(piv)) {
                        bad = true;
                    } else {
                        const float lc = sqrtf(piv);
#pragma unroll
                        for (int s = 0; s < CNS; ++s) {
                            const int r = c0 + lane + 64 * s;
                            pv[s][t] = r > c ? pv[s][t] / lc : (r == c ? lc : pv[s][t]);
                        }
#pragma unroll
                        for (int t2 = t + 1; t2 < CPW; ++t2) {
                            const float l2 = readlane(pv[0][t], t2);  // L[c0 + t2][c]
#pragma unroll
                            for (int s = 0; s < CNS; ++s) pv[s][t2] = fmaf(-pv[s][t], l2, pv[s][t2]);
                        }
                    }
                }
            }
            if (bad && lane == 0) s_fail = 1;
#pragma unroll
            for (int s = 0; s < CNS; ++s) {
                const int r = c0 + lane + 64 * s;
                if (r < kx) {
#pragma unroll
                    for (int t = 0; t < CPW; ++t)
                        if (c0 + t <= r) L[pk(r, c0 + t)] = pv[s][t];
                    *reinterpret_cast<f32x4 *>(&Pn[r * CPW]) = f32x4{pv[s][0], pv[s][1], pv[s][2], pv[s][3]};
                    *reinterpret_cast<f32x4 *>(&Pn[r * CPW + 4]) = f32x4{pv[s][4], pv[s][5], pv[s][6], pv[s][7]};
                }
            }
        }
        __syncthreads();
        if (s_fail) break;  // uniform
        const int m0 = c0 + CPW;  // panel columns past k_x are zero (clamped rows, masked below)
        for (int r = m0 + wave; r < kx; r += CWV) {
            const f32x4 pa = *reinterpret_cast<const f32x4 *>(&Pn[r * CPW]);
            const f32x4 pb = *reinterpret_cast<const f32x4 *>(&Pn[r * CPW + 4]);
            float *Lr = L + r * (r + 1) / 2;  // row r
            for (int q = m0 + lane; q <= r; q += 64) {
                const f32x4 qa = *reinterpret_cast<const f32x4 *>(&Pn[q * CPW]);
                const f32x4 qb = *reinterpret_cast<const f32x4 *>(&Pn[q * CPW + 4]);
                float v = Lr[q];
#pragma unroll
                for (int t = 0; t < 4; ++t) v = fmaf(-pa[t], qa[t], v);
#pragma unroll
                for (int t = 0; t < 4; ++t) v = fmaf(-pb[t], qb[t], v);
                Lr[q] = v;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (int c = tid; c < kx; c += CTH) Dinv[c] = 1.f / L[pk(c, c)];
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
            if (lane == 0) s_red[0] = e1;
        } else if (wave == 1) {
            // Higham's extra probe, beside the Hager sweeps: b_i = (-1)^i (1 + i/(n-1)); estimate
            // 2 ||K^{-1} b||_1 / (3n)
            float z[CNS];
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
            if (lane == 0) s_red[1] = s2;
        }
        __syncthreads();
        est = fmaxf(s_red[0], s_red[1]) * knorm;
    }
    if (tid == 0 && cond_est) cond_est[p] = est;
    // ill-conditioned pair: use the float64-formed products (rounded) for the row factorisations
    const bool replace = threshold > 0.f && !(est <= threshold) && K64;
    if (tid == 0 && flag) flag[p] = replace ? 1 : 0;
    if (replace) {
        batched_for<8>(
            tid, kx * kx, CTH, [&](int e) { return K64[(size_t)p * kx * kx + e]; },
            [&](int e, double v) { Kout[(size_t)p * kx * kx + e] = (float)v; });
        batched_for<8>(
            tid, ky * kx, CTH, [&](int e) { return R64[(size_t)p * ky * kx + e]; },
            [&](int e, double v) { Rout[(size_t)p * ky * kx + e] = (float)v; });
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

void launch_gram64(const float *A, const float *B, int64_t P, int64_t kx, int64_t ky, int64_t d, double *K64,
                   double *R64, hipStream_t st)
{
    if (d >= 8 && d % 8 == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0) {
        const int tkx = (int)((kx + 15) / 16), tky = (int)((ky + 15) / 16);
        const long long ntiles = P * (long long)(tkx * (tkx + 1) / 2 + tky * tkx);
        const long long wgs = (ntiles + 3) / 4;
        const int per_xcd = (int)((wgs + 7) / 8);
        hipLaunchKernelGGL(gram64_mfma_kernel, dim3((unsigned)(8 * per_xcd)), dim3(256), 0, st, A, B, (int)kx, (int)ky,
                           (int)d, tkx, tky, ntiles, per_xcd, K64, R64);
        return;
    }
    const int tkx = (int)((kx + 31) / 32), tky = (int)((ky + 31) / 32);
    hipLaunchKernelGGL(gram64_kernel, dim3((unsigned)(P * (tkx * tkx + tky * tkx))), dim3(256), 0, st, A, B, (int)kx,
                       (int)ky, (int)d, tkx, tky, K64, R64);
}

void launch_residual64(const float *C, const double *K64, const double *R64, const float *ex, const float *ey,
                       const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *rho,
                       hipStream_t st, const int *only)
{
    const size_t lds = (size_t)16 * kx * sizeof(double);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)residual64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(16 * kMaxK * sizeof(double)));
        attr = true;
    }
    hipLaunchKernelGGL(residual64_kernel, dim3((unsigned)(P * ((ky + 15) / 16))), dim3(256), lds, st, C, K64, R64,
                       ex, ey, lam, mask_kind, gamma, (int)kx, (int)ky, rho, only);
}

void launch_cond(const float *K, int64_t P, int64_t kx, int64_t ky, float threshold, const double *K64,
                 const double *R64, float *Kout, float *Rout, float *cond_est, hipStream_t st, int *flag)
{
    const size_t lds = ((size_t)kx * (kx + 1) / 2 + (1 + CPW) * kx + 4 + CPAD) * sizeof(float);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)cond_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(((size_t)kMaxCondK * (kMaxCondK + 1) / 2 + (1 + CPW) * kMaxCondK + 4 + CPAD) *
                                        sizeof(float)));
        attr = true;
    }
    hipLaunchKernelGGL(cond_kernel, dim3((unsigned)P), dim3(CTH), lds, st, K, (int)kx, threshold, K64, R64, Kout, Rout,
                       (int)ky, cond_est, flag);
}

}  // namespace fmap

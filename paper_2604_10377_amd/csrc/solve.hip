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
//   v_i = S_i^{-1} dC_i: with the stored factor by the triangular solves of
//   trisolve_small_kernel (solve_stored.hip), or refactorised here
//   (rowsolve_kernel, reverse mode)
//   adjoint_kernel   W = V^T C + C^T V, dA = V^T B - W A, dB = V A.
//
// Register Cholesky: lane j of the wave holds row j of S_i (entries q <= j;
// the strict upper part is kept at zero).  At step c the pivot comes from
// lane c (readlane), every lane scales its entry of column c, the new column
// is broadcast through LDS and each lane applies the rank-1 update to its row.
// Work per step is uniform, so the wave never diverges; a non-positive pivot
// is detected uniformly and stops the factorisation (LAPACK info).
#include <mutex>

#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

enum { RS_FWD = 0, RS_BWD_RECOMPUTE = 2 };  // (value 1, the stored-factor mode, is served in solve_stored.hip)

// ---------------------------------------------------------------------------
// K = A A^T and (optionally) R = B A^T.  One workgroup per 32x32 output tile;
// its four waves split the feature range d and reduce through LDS.  Loads are
// issued in batches of GU matrix-core steps ahead of the multiplies.
// ---------------------------------------------------------------------------
constexpr int GU = 8;

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
    const float *xr = X + (size_t)(mok ? m : 0) * d;
    const float *yr = Y + (size_t)(nok ? nn : 0) * d;

    const int dq = (d + 3) / 4;
    const int lo = wave * dq, hi = min(d, lo + dq);
    const int H = (max(hi - lo, 0) + 1) >> 1;
    const int base = lo + half * H;
    f32x16 acc = zero16();
    for (int s0 = 0; s0 < H; s0 += GU) {
        float a[GU], b[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int dd = base + s0 + u;
            const bool ok = (s0 + u < H) && dd < hi;
            a[u] = (mok && ok) ? xr[dd] : 0.f;
            b[u] = (nok && ok) ? yr[dd] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) acc = mfma32x32x2(a[u], b[u], acc);
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

// The same products for d % 4 == 0 and 16-byte aligned rows.  The feature range
// is cut into octets of 8 floats; lane half h of every octet takes the float4 at
// offset 4h, whose 4 values are 4 matrix-core steps (the two halves supply the
// two K slots of each step).  A wave owns a contiguous run of octets and reads
// them in groups of GO octets: a group's loads are all in flight together, and
// the next group is loaded before the current one is multiplied (two buffers,
// swapped by unrolling).  Addresses are clamped into the arrays and the values
// masked where the operands are formed, so no load waits on a branch.
constexpr int GO = 8;

__global__ __launch_bounds__(256) void gram4_kernel(const float *__restrict__ A, const float *__restrict__ B, int kx,
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
    const float *xr = X + (size_t)(mok ? m : 0) * d;
    const float *yr = Y + (size_t)(nok ? nn : 0) * d;

    const int noct = (d + 7) / 8;
    const int per = (noct + 3) / 4;
    const int o0 = wave * per, o1 = min(noct, o0 + per);
    const int ngrp = o1 > o0 ? (o1 - o0 + GO - 1) / GO : 0;
    f32x16 acc = zero16();
    f32x4 xa[GO], ya[GO], xb[GO], yb[GO];
    auto load = [&](int g, f32x4 (&xs)[GO], f32x4 (&ys)[GO]) {
#pragma unroll
        for (int u = 0; u < GO; ++u) {
            const int off = min(8 * (o0 + g * GO + u) + 4 * half, d - 4);
            xs[u] = *reinterpret_cast<const f32x4 *>(xr + off);
            ys[u] = *reinterpret_cast<const f32x4 *>(yr + off);
        }
    };
    auto mul = [&](int g, const f32x4 (&xs)[GO], const f32x4 (&ys)[GO]) {
#pragma unroll
        for (int u = 0; u < GO; ++u) {
            const int o = o0 + g * GO + u;
            const bool ok = o < o1 && 8 * o + 4 * half < d;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc = mfma32x32x2((ok && mok) ? xs[u][e] : 0.f, (ok && nok) ? ys[u][e] : 0.f, acc);
        }
    };
    if (ngrp > 0) {
        load(0, xa, ya);
        for (int g = 0; g < ngrp; g += 2) {
            load(min(g + 1, ngrp - 1), xb, yb);
            mul(g, xa, ya);
            if (g + 1 >= ngrp) break;
            load(min(g + 2, ngrp - 1), xa, ya);
            mul(g + 1, xb, yb);
        }
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

__device__ __forceinline__ float uniform(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

// ---------------------------------------------------------------------------
// One wave per row system; KMAX >= k_x is the register row length.
//
// Lane j holds row j of S_i (entries q <= j; entries above the diagonal are
// never read).  The right-looking factorisation takes the columns four at a
// time: within a block the pivots come from the diagonal lanes and the block's
// own entries are updated with readlanes; then the four new columns are
// broadcast through LDS in one round trip (one 16-byte row per lane) and each
// lane applies the block's rank-4 update to the rest of its row, column by
// column in order (the same roundings as one column at a time).  The forward
// substitution L y = r rides along.  The factor is then staged in LDS as full
// rows, from which the packed output is written with consecutive lanes on
// consecutive elements and each lane takes column j of L (row j of L^T) for
// the back substitution, which needs only readlanes.  All control flow is
// wave-uniform; a failed pivot is recorded (LAPACK info) and the system's
// outputs become NaN.
// ---------------------------------------------------------------------------
template <int KMAX> struct RowsolveLds {
    static constexpr int KP = KMAX + 4;                    // staged factor row stride (floats)
    static constexpr int PER_WAVE = 4 * KMAX + KMAX * KP;  // block broadcast, staged factor
};

template <int KMAX, int MODE>
__global__ __launch_bounds__(256) void rowsolve_kernel(
    const float *__restrict__ K, const float *__restrict__ rhs,
    const float *__restrict__ ex, const float *__restrict__ ey, const float *__restrict__ lam, int mask_kind,
    float gamma, int kx, int ky, float *out, float *__restrict__ Lout, int *__restrict__ info,
    const float *__restrict__ Cfwd, float *__restrict__ dlam_part, const float *addend)
{
    static_assert(KMAX % 4 == 0 && KMAX <= 64, "register row length");
    constexpr int KP = RowsolveLds<KMAX>::KP;
    extern __shared__ __align__(16) float s_rs[];
    const int j = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    float *s_bcw = s_rs + w * RowsolveLds<KMAX>::PER_WAVE;  // [KMAX][4]: the block's columns, row by row
    float *s_Lw = s_bcw + 4 * KMAX;                          // [KMAX][KP]: rows of L
    // per-column scalars (1 / L_cc, y_c, c_c) are written into lane c of a register as the serial steps
    // produce them (v_writelane: no lane mask, no LDS), and each lane uses its own entry afterwards
    const int rgroups = (ky + W - 1) / W;
    const int p = blockIdx.x / rgroups;
    const int i = (blockIdx.x % rgroups) * W + w;
    if (i >= ky) return;  // wave-uniform; no block-level barrier below
    const int T = kx * (kx + 1) / 2;
    const bool jok = j < kx;

    // --- every input load first, unconditional from clamped addresses, so they are all in flight together
    const int jc = jok ? j : kx - 1;
    const float lamv = lam[p];
    const float muy = ey[(size_t)p * ky + i];
    const float exj = ex[(size_t)p * kx + jc];
    const float eyj = ey[(size_t)p * ky + min(j, ky - 1)];
    float sr[KMAX];
    {
        // K is symmetric: row j is read as column j, so for each q the lanes read consecutive addresses
        const float *Kp = K + (size_t)p * kx * kx;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) sr[q] = Kp[min(q, kx - 1) * kx + jc];  // 32-bit offsets from one base
    }
    const float rin = rhs[((size_t)p * ky + i) * kx + jc];

    // --- mask row i and validity of lambda / normaliser -------------------------
    int fail = 0;
    if (!(lamv >= 0.f) || !isfinite(lamv)) fail = -1;
    MaskParams mp;
    mp.kind = mask_kind;
    mp.gamma = gamma;
    mp.inv_scale = 1.f;
    if (mask_kind == 1) {
        float mx = fmaxf(jok ? exj : -INFINITY, j < ky ? eyj : -INFINITY);  // k_x <= KMAX <= 64
        for (int q = j + 64; q < ky; q += 64) mx = fmaxf(mx, ey[(size_t)p * ky + q]);
        mx = uniform(wave_max(mx));
        if ((!(mx > 0.f) || !isfinite(mx)) && fail == 0) fail = -2;
        mp.inv_scale = 1.f / mx;
    }
    fail = __builtin_amdgcn_readfirstlane(fail);
    const float dval = (jok && fail == 0) ? mask_entry(muy, exj, mp) : 0.f;
    const float shift = lamv * dval;

    // row j of S_i = K + lambda diag(D_i) (lower part), or of the stored factor; rows k_x <= j < KMAX
    // are rows of the identity, so every loop below runs over all KMAX columns with no k_x checks
    // (their pivots are 1, their solution entries 0, and they add nothing to the real rows)
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const float v = (jok && q <= j) ? sr[q] : 0.f;
        sr[q] = (q == j) ? (jok ? v + shift : 1.f) : v;
    }
    float r = jok ? rin : 0.f;
    float vinv = 0.f, vy = 0.f;

    // Lanes j < c take garbage in column c (and in their entries above the diagonal); none of it is
    // read: a lane's later use of column c is for rows below c, and y_j was recorded at step j.
    {
#pragma unroll
        for (int c0 = 0; c0 < KMAX; c0 += 4) {
            if (c0 < kx) {  // blocks past k_x hold only identity rows
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = c0 + t;
                    const float piv = uniform(readlane(sr[c], c));
                    const bool bad = !(piv > 0.f) || !isfinite(piv);
                    fail = (bad && fail == 0) ? c + 1 : fail;
                    const float inv = uniform(__builtin_amdgcn_rsqf(piv));
                    const float l = sr[c] * inv;  // lane c: sqrt(pivot)
                    sr[c] = l;
                    const float yc = uniform(readlane(r, c) * inv);  // forward substitution, step c
                    vinv = writelane(inv, c, vinv);
                    vy = writelane(yc, c, vy);
                    r -= l * yc;
#pragma unroll
                    for (int t2 = t + 1; t2 < 4; ++t2) sr[c0 + t2] -= l * readlane(l, c0 + t2);
                }
                if (j < KMAX)
                    *reinterpret_cast<f32x4 *>(&s_bcw[4 * j]) = f32x4{sr[c0], sr[c0 + 1], sr[c0 + 2], sr[c0 + 3]};
                __builtin_amdgcn_wave_barrier();
                // rows of the block columns in groups of 8 (LDS reads of a group in flight together)
#pragma unroll
                for (int q0 = c0 + 4; q0 < KMAX; q0 += 8) {
                    f32x4 lq[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (q0 + u < KMAX) lq[u] = *reinterpret_cast<const f32x4 *>(&s_bcw[4 * (q0 + u)]);
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (q0 + u < KMAX) {
#pragma unroll
                            for (int t = 0; t < 4; ++t) sr[q0 + u] -= sr[c0 + t] * lq[u][t];
                        }
                    __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_sched_barrier(0);  // blocks are scheduled one at a time (register pressure)
            }
        }
    }
    fail = __builtin_amdgcn_readfirstlane(fail);

    // stage the rows of L (entries above the diagonal are not read)
    if (j < KMAX) {
#pragma unroll
        for (int q4 = 0; q4 < KMAX / 4; ++q4)
            *reinterpret_cast<f32x4 *>(&s_Lw[j * KP + 4 * q4]) =
                f32x4{sr[4 * q4], sr[4 * q4 + 1], sr[4 * q4 + 2], sr[4 * q4 + 3]};
    }
    __builtin_amdgcn_wave_barrier();

    if (MODE == RS_FWD && Lout) {
        // packed column-major output, one store per column (lanes q <= j < k_x); the lane index is
        // made opaque here so that the per-column lane masks are formed at the stores and not
        // hoisted above the factorisation, where they would occupy scalar registers throughout
        float *Lp = Lout + ((size_t)p * ky + i) * T;
        int jl = j;
        asm volatile("" : "+v"(jl));
        const bool lok = jl < kx;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
            if (q < kx) {
                const int pc = packed_col(q, kx) - q;
                if (lok && jl >= q) Lp[pc + jl] = fail == 0 ? sr[q] : NAN;
            }
        }
    }

    float cv = NAN;
    if (fail == 0) {
        // column j of L: L[c][j] for c > j
        const int jr = min(j, KMAX - 1);
#pragma unroll
        for (int c = 0; c < KMAX; ++c) sr[c] = (c > j) ? s_Lw[c * KP + jr] : 0.f;
        float y = vy;
        const float myinv = vinv;
        float vc = 0.f;
#pragma unroll
        for (int c = KMAX - 1; c >= 0; --c) {
            // columns of blocks past k_x were never factorised (their scalars were never recorded):
            // their solution entries are 0, taken by a select so that no stale value enters
            const float cc = (c < kx) ? uniform(readlane(y, c) * readlane(myinv, c)) : 0.f;
            vc = writelane(cc, c, vc);
            y -= sr[c] * cc;
        }
        cv = vc;
    }

    if (jok) {
        const size_t o = ((size_t)p * ky + i) * kx + j;
        out[o] = addend ? addend[o] + cv : cv;  // addend: refinement correction c += delta (in place)
    }
    if (info && j == 0) info[(size_t)p * ky + i] = fail;
    if (MODE != RS_FWD && dlam_part) {
        const float cf = jok ? Cfwd[((size_t)p * ky + i) * kx + j] : 0.f;
        const float term = jok ? cv * dval * cf : 0.f;
        const float sum = wave_sum(term);
        if (j == 0) dlam_part[(size_t)p * ky + i] = -sum;
    }
}

// ---------------------------------------------------------------------------
// Adjoint products for one pair and one CB-column block of d (k_x, k_y <= 64):
//   W = V^T C + C^T V,  dA = V^T B - W A,  dB = V A.
// V, C and W are staged in LDS as 64 x 64 tiles and the A, B column blocks as
// 64 x CB tiles, all zero past k_x / k_y, so the matrix-core loops read every
// operand unconditionally and steps past k add exact zeros.  NS batches of 8
// steps (8 NS >= max(k_x, k_y)) are unrolled; each product accumulates in two
// independent chains (even and odd steps) that are added at the end.  Rows of
// the 64 x 64 tiles are 65 floats apart (the dB operand walks down a column),
// and each array of a pair read by the two halves of a wave in the same
// instruction starts 32 floats off the other's banks.
// ---------------------------------------------------------------------------
constexpr int ADJ_KM = 64, ADJ_RS = ADJ_KM + 1, ADJ_T = ADJ_KM * ADJ_RS + 32;

template <int CB, int NS>
__global__ __launch_bounds__(256) void adjoint_kernel(const float *__restrict__ V, const float *__restrict__ C,
                                                      const float *__restrict__ A, const float *__restrict__ B,
                                                      int kx, int ky, int d, int dblocks,
                                                      const float *__restrict__ dlam_part, float *__restrict__ dlam,
                                                      float *__restrict__ dA, float *__restrict__ dB)
{
    static_assert(NS >= 1 && 8 * NS <= ADJ_KM, "steps");
    constexpr int KM = ADJ_KM, RS = ADJ_RS;
    __shared__ float sV[ADJ_T], sC[ADJ_T], sW[ADJ_T];  // sW holds -W
    __shared__ float sA[KM * CB + 32], sB[KM * CB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int p = blockIdx.x / dblocks, db = blockIdx.x % dblocks;
    const int d0 = db * CB;
    const int dw = min(CB, d - d0);
    const float *Vp = V + (size_t)p * ky * kx;
    const float *Cp = C + (size_t)p * ky * kx;
    const float *Ap = A + (size_t)p * kx * d;
    const float *Bp = B + (size_t)p * ky * d;

    // staging: every load issued before the first LDS write, from clamped addresses; values outside the
    // matrices are cleared by a bit mask (a select would let the compiler put the load under a branch)
    constexpr int NVC = KM * KM / 256, NAB = KM * CB / 256;
    float rv[NVC], rc[NVC], ra[NAB], rb[NAB];
#pragma unroll
    for (int u = 0; u < NVC; ++u) {
        const int e = threadIdx.x + 256 * u, t = e / KM, m = e % KM;
        const int src = min(t, ky - 1) * kx + min(m, kx - 1);
        rv[u] = Vp[src];
        rc[u] = Cp[src];
    }
#pragma unroll
    for (int u = 0; u < NAB; ++u) {
        const int e = threadIdx.x + 256 * u, rr = e / CB, cc = min(e % CB, dw - 1);
        ra[u] = Ap[(size_t)min(rr, kx - 1) * d + d0 + cc];
        rb[u] = Bp[(size_t)min(rr, ky - 1) * d + d0 + cc];
    }
    const bool sum_dlam = db == 0 && dlam && wave == 0;
    const float dl = (sum_dlam && lane < ky) ? dlam_part[(size_t)p * ky + lane] : 0.f;  // k_y <= 64
    auto keep = [](float x, bool ok) { return __uint_as_float(__float_as_uint(x) & (ok ? ~0u : 0u)); };
#pragma unroll
    for (int u = 0; u < NVC; ++u) {
        const int e = threadIdx.x + 256 * u, t = e / KM, m = e % KM;
        const bool ok = t < ky && m < kx;
        sV[t * RS + m] = keep(rv[u], ok);
        sC[t * RS + m] = keep(rc[u], ok);
        sW[t * RS + m] = 0.f;  // W tiles beyond k_x are never written
    }
#pragma unroll
    for (int u = 0; u < NAB; ++u) {
        const int e = threadIdx.x + 256 * u, rr = e / CB;
        const bool cin = (e % CB) < dw;
        sA[e] = keep(ra[u], cin && rr < kx);
        sB[e] = keep(rb[u], cin && rr < ky);
    }
    if (sum_dlam) {
        const float s = wave_sum(dl);
        if (lane == 0) dlam[p] = s;
    }
    __syncthreads();

    const int TI = (kx + 31) / 32, TY = (ky + 31) / 32;
    if (wave < TI * TI) {  // W tiles (TI*TI <= 4); half 0: V^T C, half 1: C^T V (the matrix-core K pair)
        const int I = wave / TI, J = wave % TI;
        const int m = I * 32 + l32, nn = J * 32 + l32;
        const float *Xs = half == 0 ? sV : sC;
        const float *Ys = half == 0 ? sC : sV;
        f32x16 acc0 = zero16(), acc1 = zero16();
#pragma unroll
        for (int t = 0; t < 8 * NS; t += 2) {
            acc0 = mfma32x32x2(Xs[t * RS + m], Ys[t * RS + nn], acc0);
            acc1 = mfma32x32x2(Xs[(t + 1) * RS + m], Ys[(t + 1) * RS + nn], acc1);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) sW[(I * 32 + acc32_row(r, lane)) * RS + nn] = -(acc0[r] + acc1[r]);
    }
    __syncthreads();

    constexpr int NCB = CB / 32;  // 32-column tiles per block
    const int nA = TI * NCB, nB = TY * NCB;
    for (int job = wave; job < nA + nB; job += 4) {
        f32x16 acc0 = zero16(), acc1 = zero16();
        if (job < nA) {
            // half 0: (V^T B)[m][col] over t < k_y; half 1: (-W A)[m][col] over t < k_x (W symmetric)
            const int I = job / NCB, cblk = job % NCB;
            const int m = I * 32 + l32, cl = cblk * 32 + l32, col = d0 + cl;
            const float *Xs = half == 0 ? sV : sW;
            const float *Ys = half == 0 ? sB : sA;
#pragma unroll
            for (int t = 0; t < 8 * NS; t += 2) {
                acc0 = mfma32x32x2(Xs[t * RS + m], Ys[t * CB + cl], acc0);
                acc1 = mfma32x32x2(Xs[(t + 1) * RS + m], Ys[(t + 1) * CB + cl], acc1);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = I * 32 + acc32_row(r, lane);
                if (row < kx && col < d) dA[((size_t)p * kx + row) * d + col] = acc0[r] + acc1[r];
            }
        } else {
            // (V A)[m][col]: half h takes the terms kk = 2 s + h
            const int jb = job - nA;
            const int I = jb / NCB, cblk = jb % NCB;
            const int m = I * 32 + l32, cl = cblk * 32 + l32, col = d0 + cl;
#pragma unroll
            for (int s2 = 0; s2 < 4 * NS; s2 += 2) {
                const int k0 = 2 * s2 + half, k1 = k0 + 2;
                acc0 = mfma32x32x2(sV[m * RS + k0], sA[k0 * CB + cl], acc0);
                acc1 = mfma32x32x2(sV[m * RS + k1], sA[k1 * CB + cl], acc1);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = I * 32 + acc32_row(r, lane);
                if (row < ky && col < d) dB[((size_t)p * ky + row) * d + col] = acc0[r] + acc1[r];
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
    w.W = off;
    off += (kx > kSmallK || ky > kSmallK) ? align256((size_t)P * kx * kx * sizeof(float)) : 0;
    w.tiles = off;
    off += kx > kSmallK ? align256(tiled_workspace_bytes(P, kx, ky)) : 0;
    w.K64 = off;
    off += align256((size_t)P * kx * kx * sizeof(double));
    w.R64 = off;
    off += align256((size_t)P * ky * kx * sizeof(double));
    w.dlam = off;
    off += align256((size_t)P * ky * sizeof(float));
    w.flag = off;
    off += align256((size_t)P * sizeof(int));
    w.total = off;
    return w;
}

void launch_gram(const float *A, const float *B, int64_t P, int64_t kx, int64_t ky, int64_t d, bool with_R,
                        float *K, float *R, hipStream_t st)
{
    const int tkx = (int)((kx + 31) / 32), tky = (int)((ky + 31) / 32);
    const int tiles = tkx * tkx + (with_R ? tky * tkx : 0);
    const bool vec = d % 4 == 0 && ((uintptr_t)A & 15) == 0 && (!with_R || ((uintptr_t)B & 15) == 0);
    hipLaunchKernelGGL(vec ? gram4_kernel : gram_kernel, dim3((unsigned)(P * tiles)), dim3(256), 0, st, A, B, (int)kx,
                       (int)ky, (int)d, tkx, tky, with_R ? 1 : 0, K, R);
}

// W = row systems (waves) per workgroup of the register row solve: 1, 2 or 4 (the launch bound); the
// plan's autotuner picks it per k group.
template <int MODE>
static void launch_rowsolve(const float *K, const float *rhs, const float *ex, const float *ey,
                            const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky,
                            float *out, float *Lout, int *info, const float *Cfwd, float *dlam_part, hipStream_t st,
                            int W)
{
    if (W != 1 && W != 2) W = 4;
    const unsigned grid = (unsigned)(P * ((ky + W - 1) / W));
    // dynamic LDS: W x (4 KM + KM (KM + 4)) floats, at most 4 x 4352 floats (68 KB)
#define FMAP_RS(KM)                                                                                             \
    do {                                                                                                        \
        const size_t lds_ = (size_t)W * RowsolveLds<KM>::PER_WAVE * sizeof(float);                              \
        static bool attr_ = false;                                                                              \
        if (!attr_) {                                                                                           \
            (void)hipFuncSetAttribute((const void *)rowsolve_kernel<KM, MODE>,                                  \
                                      hipFuncAttributeMaxDynamicSharedMemorySize,                               \
                                      (int)(4 * RowsolveLds<KM>::PER_WAVE * sizeof(float)));                     \
            attr_ = true;                                                                                       \
        }                                                                                                       \
        hipLaunchKernelGGL((rowsolve_kernel<KM, MODE>), dim3(grid), dim3(64 * W), lds_, st, K, rhs, ex, ey,  \
                           lam, mask_kind, gamma, (int)kx, (int)ky, out, Lout, info, Cfwd, dlam_part, nullptr);  \
    } while (0)
    if (kx <= 8) FMAP_RS(8);
    else if (kx <= 16) FMAP_RS(16);
    else if (kx <= 24) FMAP_RS(24);
    else if (kx <= 32) FMAP_RS(32);
    else if (kx <= 40) FMAP_RS(40);
    else if (kx <= 48) FMAP_RS(48);
    else if (kx <= 52) FMAP_RS(52);
    else if (kx <= 56) FMAP_RS(56);
    else FMAP_RS(64);
#undef FMAP_RS
}

// A second stream per device, with a fork and a join event, for work that overlaps the caller's stream
// within one library call.  Created on first use outside stream capture (creating it during a capture is not
// allowed); under capture the fork and join become graph edges, so the side work is part of the captured graph.
// Calls that overlap on one device share it: their side work is serialised, but each waits for its own.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

static SideStream *side_stream(hipStream_t st)
{
    static std::mutex mu;
    static SideStream per_dev[64];
    static bool made[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!made[dev]) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
        SideStream S;
        bool ok = hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&S.join, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            if (S.join) (void)hipEventDestroy(S.join);
            if (S.fork) (void)hipEventDestroy(S.fork);
            if (S.s) (void)hipStreamDestroy(S.s);
            return nullptr;
        }
        per_dev[dev] = S;
        made[dev] = true;
    }
    return &per_dev[dev];
}

void launch_rowsolve_dense(const float *S, const float *g, const float *ex_zero, const float *ey_zero, const float *lam,
                           int64_t P, int64_t n, float *out, int *info, float *tiles, hipStream_t st)
{
    // one system per pair (k_y = 1): the zero mask rows add no diagonal shift, lambda only gates validity
    if (n <= kSmallK)
        launch_rowsolve<RS_FWD>(S, g, ex_zero, ey_zero, lam, 0, 0.5f, P, n, 1, out, nullptr, info, nullptr, nullptr, st,
                                1);
    else
        launch_rowsolve_tiled(RS_FWD, S, g, ex_zero, ey_zero, lam, 0, 0.5f, P, n, 1, out, nullptr, info, nullptr,
                              nullptr, tiles, st);
}

hipError_t launch_solve(const float *A, const float *B, const float *ex, const float *ey, const float *lam,
                        int32_t mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, int64_t d,
                        int32_t refine_steps, float cond_threshold, float *C, float *factors, int32_t *info,
                        float *cond_est, void *ws, hipStream_t st, int rs_waves)
{
    SolveWs L = solve_workspace_layout(P, kx, ky, d);
    char *base = (char *)ws;
    float *K = (float *)(base + L.K), *R = (float *)(base + L.R);
    double *K64 = (double *)(base + L.K64), *R64 = (double *)(base + L.R64);
    float *tiles = (float *)(base + L.tiles);
    launch_gram(A, B, P, kx, ky, d, true, K, R, st);
    if (refine_steps > 0) launch_gram64(A, B, P, kx, ky, d, K64, R64, st);
    const bool want_cond = cond_threshold > 0.f || cond_est;
    const float thr = refine_steps > 0 ? cond_threshold : 0.f;
    float *rho = (float *)(base + L.V);
    SideStream *side = (want_cond && refine_steps > 0 && kx > kSmallK) ? side_stream(st) : nullptr;
    if (side) {
        // The condition estimate (one workgroup per pair, latency-bound) runs on a side stream beside the
        // refinement of every pair, after the row solve on the float32 products.  Nothing on the main stream
        // reads K or R after that solve, so the estimate may replace them for the pairs above the threshold;
        // those pairs are then solved and refined again from the rounded float64 products (their first results
        // are overwritten), which gives every pair the result of the sequential order.
        int *flag = (int *)(base + L.flag);
        launch_rowsolve_tiled(RS_FWD, K, R, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, factors, info, nullptr,
                              nullptr, tiles, st);
        hipError_t e = hipEventRecord(side->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->fork, 0);
        if (e != hipSuccess) return e;
        launch_cond(K, P, kx, ky, thr, K64, R64, K, R, cond_est, side->s, flag);
        e = hipEventRecord(side->join, side->s);
        for (int it = 0; it < refine_steps; ++it) {
            launch_residual64(C, K64, R64, ex, ey, lam, mask_kind, gamma, P, kx, ky, rho, st);
            launch_trisolve_stored(factors, rho, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, nullptr, nullptr,
                                   nullptr, C, st);
        }
        if (e == hipSuccess) e = hipStreamWaitEvent(st, side->join, 0);
        if (e != hipSuccess) return e;
        if (thr > 0.f) {
            launch_rowsolve_tiled(RS_FWD, K, R, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, factors, info, nullptr,
                                  nullptr, tiles, st, flag);
            for (int it = 0; it < refine_steps; ++it) {
                launch_residual64(C, K64, R64, ex, ey, lam, mask_kind, gamma, P, kx, ky, rho, st, flag);
                launch_trisolve_stored(factors, rho, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, nullptr, nullptr,
                                       nullptr, C, st, flag);
            }
        }
        return hipGetLastError();
    }
    if (want_cond)
        launch_cond(K, P, kx, ky, thr, refine_steps > 0 ? K64 : nullptr, refine_steps > 0 ? R64 : nullptr, K, R,
                    cond_est, st);
    if (kx <= kSmallK)
        launch_rowsolve<RS_FWD>(K, R, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, factors, info, nullptr,
                                nullptr, st, rs_waves);
    else
        launch_rowsolve_tiled(RS_FWD, K, R, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, factors, info, nullptr,
                              nullptr, tiles, st);
    // iterative refinement: rho = R64 - C K64 - lambda D o C in float64, C += S^{-1} rho with the float32 factors
    for (int it = 0; it < refine_steps; ++it) {
        launch_residual64(C, K64, R64, ex, ey, lam, mask_kind, gamma, P, kx, ky, rho, st);
        if (kx <= kSmallK)
            launch_trisolve_small(factors, rho, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, nullptr, nullptr, nullptr,
                                  C, st);
        else
            launch_trisolve_stored(factors, rho, ex, ey, lam, mask_kind, gamma, P, kx, ky, C, nullptr, nullptr, nullptr,
                                   C, st);
    }
    return hipGetLastError();
}

hipError_t launch_solve_backward(const float *dC, const float *A, const float *B, const float *C, const float *ex,
                                 const float *ey, const float *lam, int32_t mask_kind, float gamma, int64_t P,
                                 int64_t kx, int64_t ky, int64_t d, const float *factors, float *dA, float *dB,
                                 float *dlam, int32_t *info, void *ws, hipStream_t st, int rs_waves)
{
    SolveWs L = solve_workspace_layout(P, kx, ky, d);
    char *base = (char *)ws;
    float *K = (float *)(base + L.K), *V = (float *)(base + L.V), *dl = (float *)(base + L.dlam);
    const bool small = kx <= kSmallK;
    if (factors) {
        if (small)
            launch_trisolve_small(factors, dC, ex, ey, lam, mask_kind, gamma, P, kx, ky, V, info, C, dl, nullptr, st);
        else
            launch_trisolve_stored(factors, dC, ex, ey, lam, mask_kind, gamma, P, kx, ky, V, info, C, dl, nullptr, st);
    } else {
        launch_gram(A, B, P, kx, ky, d, false, K, nullptr, st);
        if (small)
            launch_rowsolve<RS_BWD_RECOMPUTE>(K, dC, ex, ey, lam, mask_kind, gamma, P, kx, ky, V, nullptr,
                                              info, C, dl, st, rs_waves);
        else
            launch_rowsolve_tiled(RS_BWD_RECOMPUTE, K, dC, ex, ey, lam, mask_kind, gamma, P, kx, ky, V, nullptr, info, C,
                                  dl, (float *)(base + L.tiles), st);
    }
    if (kx <= kSmallK && ky <= kSmallK) {
        // 32-column blocks: twice the workgroups of 64-column ones (W is recomputed per block, k^3 flops)
        const int dblocks = (int)((d + 31) / 32);
        const dim3 grid((unsigned)(P * dblocks)), block(256);
#define FMAP_ADJ(NS)                                                                                           \
    hipLaunchKernelGGL((adjoint_kernel<32, NS>), grid, block, 0, st, V, C, A, B, (int)kx, (int)ky, (int)d, dblocks, \
                       dl, dlam, dA, dB)
        switch ((std::max(kx, ky) + 7) / 8) {
        case 1: FMAP_ADJ(1); break;
        case 2: FMAP_ADJ(2); break;
        case 3: FMAP_ADJ(3); break;
        case 4: FMAP_ADJ(4); break;
        case 5: FMAP_ADJ(5); break;
        case 6: FMAP_ADJ(6); break;
        case 7: FMAP_ADJ(7); break;
        default: FMAP_ADJ(8); break;
        }
#undef FMAP_ADJ
    } else {
        launch_adjoint_general(V, C, A, B, P, kx, ky, d, (float *)(base + L.W), dl, dlam, dA, dB, st);
    }
    return hipGetLastError();
}

}  // namespace fmap

// Row systems of order 64 < k_x <= 319 (Eqs. (5)-(7) at large spectral
// resolution), and the adjoint products for any k.
//
// A blocked left-looking Cholesky: the lower triangle of S_i = K + lambda diag(D_i)
// is cut into 32x32 tiles, and the right-hand side is appended as one extra row
// (index k_x), so the factorisation performs the forward substitution L y = r
// on the fly.  A 4-wave workgroup keeps the active block column in LDS and the
// finished tiles in its slot of the workspace, and several systems share a CU
// (rowsolve_ll_kernel, described below).

#include <algorithm>

#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

namespace {

constexpr int TLD = 33;                 // row stride of a stored tile (odd: conflict-free columns)
constexpr int TSZ = 32 * TLD;           // floats per tile
constexpr int LDD = 36;                 // row stride of the aligned copy of the diagonal tile

__device__ __forceinline__ int packed_col_t(int c, int m) { return c * m - (c * (c - 1)) / 2; }
__device__ __forceinline__ float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
// index of tile (I, J), I >= J, in column-major order of the lower triangle with TR tile rows
__device__ __forceinline__ int tile_index(int I, int J, int TR) { return J * TR - (J * (J - 1)) / 2 + (I - J); }

// LDS scratch of the diagonal-tile routine below (floats, 16-byte aligned)
constexpr int DIAG_LR = 32 * LDD;

// One wave (64 lanes): Cholesky factor of the 32 x 32 diagonal tile Dt (rows at stride TLD, lower part, the
// first kxl columns; rows past kxl, e.g. the appended right-hand side row, are eliminated with them), and the
// inverse of the factor, Minv[q][c] at q * TLD + c (rows and columns past kxl zero).  Returns 0, or 1 + the
// first column whose pivot is not positive and finite (then Dt and Minv hold garbage).
//   * factor: lane r holds row r; columns in blocks of 8, each block's columns in the lanes' registers with
//     the entries L_qc taken by readlane, then the block's rank-8 update of the later columns from one LDS
//     broadcast of the block (rows of the block column, 16-byte reads).  Every step is branch-free (a
//     column past kxl or after a failure multiplies by 0): branches per column made the compiler copy the
//     row registers at every join;
//   * inverse: the two 16 x 16 diagonal blocks of L^{-1}, one per half of lanes 0..31 (lane = column), from
//     the rows of L in LDS (16-byte reads, each half at its own address), then the lower-left block
//     M21 = -M22 L21 M11 as two 16 x 16 x 16 products on the float32 matrix cores.
// Lr ([32][LDD], 16-byte aligned) is scratch: the block broadcasts of the factor, then the rows of L, then
// (over rows 0..7, free by then) the product L21 M11.
__device__ __forceinline__ int diag_factor_inverse(float *Dt, float *Lr, float *Minv, int kxl, int lane)
{
    // the lane index made opaque, so its masks are formed where used, not hoisted into registers
    asm volatile("" : "+v"(lane));
    const int l32 = lane & 31;
    float sr[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) sr[q] = (lane < 32) ? Dt[l32 * TLD + q] : 0.f;
    int fail = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int c = 8 * b; c < 8 * b + 8; ++c) {
            const float pv = uniform_f(readlane(sr[c], c));
            const bool act = c < kxl && fail == 0;
            const bool bad = !(pv > 0.f) || !isfinite(pv);
            fail = (act && bad) ? c + 1 : fail;
            const bool go = act && !bad;
            const float l0 = sr[c] * __builtin_amdgcn_rsqf(go ? pv : 1.f);
            sr[c] = go ? l0 : sr[c];
            const float l = go ? l0 : 0.f;
#pragma unroll
            for (int q = c + 1; q < 8 * b + 8; ++q) sr[q] -= l * readlane(l, q);
            __builtin_amdgcn_sched_barrier(0);
        }
        // columns past kxl take no part (zeroed: nothing reads them afterwards)
#pragma unroll
        for (int u = 0; u < 8; ++u) sr[8 * b + u] = (8 * b + u < kxl) ? sr[8 * b + u] : 0.f;
        if (b < 3) {
            if (lane < 32) {
                *reinterpret_cast<f32x4 *>(&Lr[8 * l32]) = f32x4{sr[8 * b], sr[8 * b + 1], sr[8 * b + 2], sr[8 * b + 3]};
                *reinterpret_cast<f32x4 *>(&Lr[8 * l32 + 4]) =
                    f32x4{sr[8 * b + 4], sr[8 * b + 5], sr[8 * b + 6], sr[8 * b + 7]};
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 8 * b + 8; q < 32; ++q) {
                const f32x4 x0 = *reinterpret_cast<const f32x4 *>(&Lr[8 * q]);
                const f32x4 x1 = *reinterpret_cast<const f32x4 *>(&Lr[8 * q + 4]);
#pragma unroll
                for (int u = 0; u < 4; ++u) sr[q] -= sr[8 * b + u] * x0[u];
#pragma unroll
                for (int u = 0; u < 4; ++u) sr[q] -= sr[8 * b + 4 + u] * x1[u];
                // finished here: left free, the compiler defers later columns' updates past the next block
                // and keeps all their loaded rows live at once
                asm volatile("" : "+v"(sr[q]));
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    fail = __builtin_amdgcn_readfirstlane(fail);
    if (fail != 0) return fail;
    if (lane < 32) {
#pragma unroll
        for (int q = 0; q < 32; ++q) Dt[l32 * TLD + q] = sr[q];
#pragma unroll
        for (int q = 0; q < 32; q += 4)
            *reinterpret_cast<f32x4 *>(&Lr[l32 * LDD + q]) = f32x4{sr[q], sr[q + 1], sr[q + 2], sr[q + 3]};
    }
    __builtin_amdgcn_wave_barrier();
    {
        const int hb = (lane >> 4) & 1, jj = lane & 15;
        const float *Lb = Lr + 16 * hb * LDD + 16 * hb;
        float mb[16];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) {
            float t = (qq == jj) ? 1.f : 0.f;
            f32x4 row[4];
#pragma unroll
            for (int g = 0; g <= qq / 4; ++g) row[g] = *reinterpret_cast<const f32x4 *>(&Lb[qq * LDD + 4 * g]);
#pragma unroll
            for (int tt = 0; tt < qq; ++tt) t -= row[tt / 4][tt % 4] * mb[tt];
            mb[qq] = (16 * hb + qq < kxl) ? t * __builtin_amdgcn_rcpf(row[qq / 4][qq % 4]) : 0.f;
            asm volatile("" : "+v"(mb[qq]));
        }
        if (lane < 32) {
#pragma unroll
            for (int qq = 0; qq < 16; ++qq) {
                Minv[(16 * hb + qq) * TLD + 16 * hb + jj] = mb[qq];
                Minv[(16 * hb + qq) * TLD + 16 * (1 - hb) + jj] = 0.f;  // upper block; the lower one follows
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    {
        // 16 x 16 x 4 float32 matrix-core steps: lane (i, k) = (lane % 16, lane / 16) supplies A[i][k] and
        // B[k][i]; the result row 4 (lane / 16) + r, column lane % 16 is register r
        const int i16 = lane & 15, k4 = lane >> 4;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 4; ++st)  // T = L21 M11
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Lr[(16 + i16) * LDD + 4 * st + k4],
                                                       Minv[(4 * st + k4) * TLD + i16], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) Lr[(4 * k4 + r) * 16 + i16] = acc[r];
        __builtin_amdgcn_wave_barrier();
        f32x4 acc2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 4; ++st)  // M21 = -M22 T
            acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(Minv[(16 + i16) * TLD + 16 + 4 * st + k4],
                                                        Lr[(4 * st + k4) * 16 + i16], acc2, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) Minv[(16 + 4 * k4 + r) * TLD + i16] = -acc2[r];
    }
    __builtin_amdgcn_wave_barrier();
    return 0;
}

}  // namespace

enum { RT_FWD = 0, RT_BWD_RECOMPUTE = 2 };

// ---------------------------------------------------------------------------
// The left-looking kernel, 64 < k_x <= 319: several row systems per CU.
//
// Keeping every tile of a system in LDS (118 KB at k_x = 200) would hold a CU
// to one system, idle while one wave factorises a diagonal tile.  Here a
// workgroup of 4 waves keeps only the active block column in LDS (40 KB in all
// at k_x = 200) and writes each finished tile L_Ip, and the inverse of each
// diagonal tile, to its own slot of the workspace (32 x 32 row-major tiles in
// the lower-triangle order of the tile grid; the diagonal positions hold the
// inverses).  Two to four systems then share a CU and hide each other's serial
// diagonal steps.  Step p:
//   1. each wave loads its own tiles of block column p of
//      S = K + lambda diag(D_i) (the right-hand side as the appended row)
//      straight into its accumulators, with no barrier before step 2;
//   2. left-looking update S_Ip -= sum_{q < p} L_Iq L_pq^T on the float32
//      matrix cores, the L tiles read from the slot straight into the operand
//      registers: lane (m, h) supplies row m, columns 16 h .. 16 h + 15, with
//      the K order of the matrix-core steps permuted alike for both operands.
//      One wave updates the diagonal tile and goes on to step 3 at once, while
//      the others update the tiles below it; the updated tiles go to LDS;
//   3. that wave factorises the diagonal tile and forms its inverse
//      (diag_factor_inverse);
//   4. the panel L_Ip = S_Ip L_pp^{-T} on the matrix cores, stored to the slot.
// The appended row carries the forward substitution, so its tile row yields
// y.  The back substitution runs block by block from the last: the finished
// blocks' contribution L_Ip^T c_I as matrix-vector products over the slot's
// tiles, then c_p = L_pp^{-T} v as one product with the stored inverse.
// ---------------------------------------------------------------------------
constexpr int LLW = 4;          // waves per workgroup
constexpr int LTS = 32 * 32;    // floats per tile in the workspace slot

constexpr int ll_lds_floats(int TRM) { return TRM * TSZ + TSZ + DIAG_LR + 2 * TRM * 32 + LLW * 32 + LLW + 4; }

__device__ __forceinline__ f32x4 ldg4(const float *p) { return *reinterpret_cast<const f32x4 *>(p); }

// STORE: the factor is written to Lout (forward mode with stored factors).
template <int TMAX, int MODE, bool STORE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TMAX == 10 ? 2 : 4))) void rowsolve_ll_kernel(
    const float *__restrict__ K, const float *__restrict__ rhs, const float *__restrict__ ex,
    const float *__restrict__ ey, const float *__restrict__ lam, int mask_kind, float gamma, int kx, int ky, int nsys,
    float *out, float *__restrict__ Lout, int *__restrict__ info, const float *__restrict__ Cfwd,
    float *__restrict__ dlam_part, float *__restrict__ Lws, int cus, const int *__restrict__ only)
{
    constexpr int TRM = TMAX;
    constexpr int NTL = TMAX * (TMAX + 1) / 2;
    extern __shared__ __align__(16) float smem[];
    float *bc = smem;                    // tile j: rows 32 (p + j) .. 32 (p + j) + 31 of block column p
    float *s_minv = bc + TRM * TSZ;      // inverse of the diagonal tile, Minv[q][c] at q * TLD + c
    float *s_lr = s_minv + TSZ;          // scratch of the diagonal-tile routine
    float *s_dval = s_lr + DIAG_LR;      // mask row D_i
    float *s_vec = s_dval + TRM * 32;    // y, then c
    float *s_part = s_vec + TRM * 32;    // [LLW][32]
    float *s_red = s_part + LLW * 32;    // [LLW]
    int *s_fail = reinterpret_cast<int *>(s_red + LLW);
    float *Ls = Lws + (size_t)blockIdx.x * NTL * LTS;

    const int tid = threadIdx.x, wave = tid >> 6;
    // the wave that runs the serial diagonal steps: different for the workgroups that share a CU (ids one grid
    // round of CUs apart), so that their diagonal chains do not all land on the same SIMD
    const int dwave = (blockIdx.x / cus) % LLW;
    const int T = (kx + 31) >> 5;   // column tiles
    const int TR = (kx + 32) >> 5;  // tile rows (row kx is the right-hand side)
    const int AR = kx >> 5, ar = kx & 31;

    for (int sys = blockIdx.x; sys < nsys; sys += gridDim.x) {
        const int p = sys / ky, i = sys % ky;
        if (only && __builtin_amdgcn_readfirstlane(only[p]) == 0) continue;  // uniform: before any barrier
        int tid = threadIdx.x;  // opaque per system, as in the steps below
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63;
        // ---- lambda, mask row, normaliser -----------------------------------------------
        const float lamv = lam[p];
        int fail0 = (!(lamv >= 0.f) || !isfinite(lamv)) ? -1 : 0;
        MaskParams mp;
        mp.kind = mask_kind;
        mp.gamma = gamma;
        mp.inv_scale = 1.f;
        if (mask_kind == 1) {
            float mx = -INFINITY;
            for (int q = tid; q < kx; q += 256) mx = fmaxf(mx, ex[(size_t)p * kx + q]);
            for (int q = tid; q < ky; q += 256) mx = fmaxf(mx, ey[(size_t)p * ky + q]);
            mx = wave_max(mx);
            if (lane == 0) s_red[wave] = mx;
            __syncthreads();
            mx = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
            if ((!(mx > 0.f) || !isfinite(mx)) && fail0 == 0) fail0 = -2;
            mp.inv_scale = 1.f / mx;
        }
        const float muy = ey[(size_t)p * ky + i];
        for (int q = tid; q < TRM * 32; q += 256) {
            const float dv = (q < kx && fail0 != -2) ? mask_entry(muy, ex[(size_t)p * kx + q], mp) : 0.f;
            s_dval[q] = dv;
            s_vec[q] = 0.f;
        }
        if (tid == 0) *s_fail = fail0;
        const float lsh = fail0 == 0 ? lamv : 0.f;  // the diagonal shift is lsh * D_iq
        __syncthreads();

        const float *Kp = K + (size_t)p * kx * kx;
        const float *rp = rhs + ((size_t)p * ky + i) * kx;
        for (int ps = 0; ps < T; ++ps) {
            if (__builtin_amdgcn_readfirstlane(*s_fail) != 0) break;
            // the thread index, made opaque per step: lane-dependent masks and addresses (the identity column
            // of the inverse, the appended row's accumulator slot, the tile offsets of the loads) are then
            // formed where they are used, not hoisted out of every loop into registers (they had taken some 40
            // to 80 registers for the whole kernel)
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            const int lane = tid & 63;
            const int l32 = lane & 31, half = lane >> 5;
            const int nt = TR - ps;                 // tiles of the block column
            const int kxl = min(32, kx - 32 * ps);  // columns of this block
            // ---- 1. block column ps: S_Ip = K_Ip (+ the shift on the diagonal; row k_x is the right-hand
            //         side, rows and columns past it are zero), minus sum_{q < ps} L_Iq L_pq^T ------------
            // Each wave loads its own tiles straight into its accumulators (no barrier between the loads and
            // the update).  The diagonal-tile wave takes the diagonal tile alone and goes straight on to
            // factorise it (step 3, its own LDS writes, no barrier), while the other waves take the tiles
            // below it.
            {
                const int j0 = wave == dwave ? 0 : 1 + (wave - dwave + LLW - 1) % LLW;
                const int jstep = wave == dwave ? nt : LLW - 1;
                for (int j = j0; j < nt; j += jstep) {
                    // lane-derived values formed per tile (kept out of the registers held across the update)
                    int ln = lane;
                    asm volatile("" : "+v"(ln));
                    const int l32 = ln & 31, half = ln >> 5;
                    const int col = 32 * ps + l32;
                    const int colc = min(col, kx - 1);
                    float *X = bc + j * TSZ;
                    const int I = ps + j;
                    const int off = l32 * 32 + 16 * half;
                    // this tile's entries of K (unconditional loads from clamped addresses) and the first
                    // tile pair of the update, all in flight together
                    f32x16 acc;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int rowc = min(32 * I + acc32_row(r, ln), kx);
                        acc[r] = *(rowc == kx ? rp + colc : Kp + (size_t)rowc * kx + colc);
                    }
                    f32x4 a0[4], b0[4];
                    if (ps > 0) {
                        const float *ap = Ls + (size_t)tile_index(I, 0, TR) * LTS + off;
                        const float *bp = Ls + (size_t)tile_index(ps, 0, TR) * LTS + off;
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            a0[u] = ldg4(ap + 4 * u);
                            b0[u] = ldg4(bp + 4 * u);
                        }
                    }
                    const float dsh = lsh * s_dval[col];  // the shift of this column's diagonal entry
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = 32 * I + acc32_row(r, ln);
                        const float v = acc[r];
                        float x = 0.f;
                        if (row < kx && col < kx) x = v + (row == col ? dsh : 0.f);
                        else if (row == kx && col < kx) x = v;
                        acc[r] = x;
                    }
                    // whole tile pairs (16 floats of each operand per lane), the next pair in flight while one is
                    // multiplied
                    for (int q = 0; q < ps; ++q) {
                        const int qn = min(q + 1, ps - 1);
                        const float *ap = Ls + (size_t)tile_index(I, qn, TR) * LTS + off;
                        const float *bp = Ls + (size_t)tile_index(ps, qn, TR) * LTS + off;
                        f32x4 a1[4], b1[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            a1[u] = ldg4(ap + 4 * u);
                            b1[u] = ldg4(bp + 4 * u);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int e = 0; e < 4; ++e) acc = mfma32x32x2(-a0[u][e], b0[u][e], acc);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            a0[u] = a1[u];
                            b0[u] = b1[u];
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 16; ++r) X[acc32_row(r, ln) * TLD + l32] = acc[r];
                }
            }
            // ---- 3. diagonal tile and its inverse (one wave) ----------------------------------
            if (wave == dwave) {
                const int f = diag_factor_inverse(bc, s_lr, s_minv, kxl, lane);
                if (f != 0) {
                    if (lane == 0) *s_fail = 32 * ps + f;
                } else {
                    // the inverse also into the slot's diagonal position (rows 2 u + half)
                    float *Mi = Ls + (size_t)tile_index(ps, ps, TR) * LTS;
#pragma unroll
                    for (int u = 0; u < 16; ++u) Mi[(2 * u + half) * 32 + l32] = s_minv[(2 * u + half) * TLD + l32];
                }
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(*s_fail) != 0) break;
            if (AR == ps && tid < 32) s_vec[32 * ps + tid] = tid < kxl ? bc[ar * TLD + tid] : 0.f;  // y of this block
            if (STORE) {
                // L_pp into the packed factor, consecutive threads on consecutive rows of a column
                float *Lo = Lout + ((size_t)p * ky + i) * (size_t)(kx * (kx + 1) / 2);
                for (int e = tid; e < 1024; e += 256) {
                    const int c = e >> 5, r = e & 31;
                    if (r >= c && r < kxl) Lo[packed_col_t(32 * ps + c, kx) + (r - c)] = bc[r * TLD + c];
                }
            }
            // ---- 4. panel L_Ip = S_Ip Minv^T (I > ps) -----------------------------------------------
            for (int j = 1 + wave; j < nt; j += LLW) {
                const int I = ps + j;
                const float *X = bc + j * TSZ;
                f32x16 nv = zero16();
#pragma unroll
                for (int t = 0; t < 16; ++t)
                    nv = mfma32x32x2(X[l32 * TLD + 2 * t + half], s_minv[l32 * TLD + 2 * t + half], nv);
                float *Lt = Ls + (size_t)tile_index(I, ps, TR) * LTS;
#pragma unroll
                for (int r = 0; r < 16; ++r) Lt[acc32_row(r, lane) * 32 + l32] = nv[r];
                if (STORE) {
                    // the tile of L also back into LDS (over S_Ip, which this wave alone reads) for the packed output
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int r = 0; r < 16; ++r) bc[j * TSZ + acc32_row(r, lane) * TLD + l32] = nv[r];
                }
                if (I == AR) {
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (acc32_row(r, lane) == ar) s_vec[32 * ps + l32] = l32 < kxl ? nv[r] : 0.f;
                }
            }
            __syncthreads();
            if (STORE) {
                // the block column's tiles of L below the diagonal into the packed factor, consecutive threads on
                // consecutive rows of one column
                float *Lo = Lout + ((size_t)p * ky + i) * (size_t)(kx * (kx + 1) / 2);
                for (int e = tid; e < (nt - 1) * 1024; e += 256) {
                    const int j = 1 + (e >> 10), c = (e >> 5) & 31, r = e & 31;
                    const int R = 32 * (ps + j) + r, Cc = 32 * ps + c;
                    if (R < kx && Cc < kx) Lo[packed_col_t(Cc, kx) + R - Cc] = bc[j * TSZ + r * TLD + c];
                }
                __syncthreads();
            }
        }
        const int fail = __builtin_amdgcn_readfirstlane(*s_fail);

        // ---- back substitution L^T c = y, column-oriented, from the last block ---------------------------
        // The inverses of the diagonal tiles go to the block-column buffer (free now, T <= TRM tiles).  Step p:
        // c_p = L_pp^{-T} y_p from LDS, then y_q -= L_pq^T c_p for every q < p, wave w taking q = w, w + 4, ...
        // with the tiles' loads issued before c_p is formed.
        if (fail == 0) {
            // lane values formed here, from an opaque thread index (not held from the kernel's start)
            int tb = threadIdx.x;
            asm volatile("" : "+v"(tb));
            const int tid = tb, lane = tb & 63;
            const int l32 = lane & 31, half = lane >> 5;
            for (int e0 = tid; e0 < T * 1024; e0 += 8 * 256) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = min(e0 + 256 * u, T * 1024 - 1);
                    v[u] = Ls[(size_t)tile_index(e >> 10, e >> 10, TR) * LTS + (e & 1023)];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + 256 * u;
                    if (e < T * 1024) bc[(e >> 10) * TSZ + ((e >> 5) & 31) * TLD + (e & 31)] = v[u];
                }
            }
            __syncthreads();
            for (int ps = T - 1; ps >= 0; --ps) {
                const int kxl = min(32, kx - 32 * ps);
                // this wave's first tile (ps, q = wave): rows h, h + 2, ... of column l32, in flight while c_ps is
                // formed
                float lv[16];
                {
                    const float *Lt = Ls + (size_t)tile_index(ps, min(wave, max(ps - 1, 0)), TR) * LTS;
#pragma unroll
                    for (int u = 0; u < 16; ++u) lv[u] = Lt[(2 * u + half) * 32 + l32];
                }
                if (wave == dwave && lane < 32) {
                    // c_j = sum_q Minv[q][j] y_q
                    const float *Mi = bc + ps * TSZ;
                    float c = 0.f;
#pragma unroll
                    for (int q = 0; q < 32; ++q) c += Mi[q * TLD + l32] * s_vec[32 * ps + q];
                    s_vec[32 * ps + l32] = l32 < kxl ? c : 0.f;
                }
                __syncthreads();
                if (wave < ps) {
                    float z = 0.f;
#pragma unroll
                    for (int u = 0; u < 16; ++u) z += lv[u] * s_vec[32 * ps + 2 * u + half];
                    z += __shfl_xor(z, 32, 64);
                    if (half == 0) s_vec[32 * wave + l32] -= z;
                }
                for (int q = wave + LLW; q < ps; q += LLW) {  // further earlier blocks (k_x > 128)
                    const float *Lt = Ls + (size_t)tile_index(ps, q, TR) * LTS;
#pragma unroll
                    for (int u = 0; u < 16; ++u) lv[u] = Lt[(2 * u + half) * 32 + l32];
                    float z = 0.f;
#pragma unroll
                    for (int u = 0; u < 16; ++u) z += lv[u] * s_vec[32 * ps + 2 * u + half];
                    z += __shfl_xor(z, 32, 64);
                    if (half == 0) s_vec[32 * q + l32] -= z;
                }
                __syncthreads();
            }
        }

        // ---- outputs ----------------------------------------------------------------------
        for (int q = tid; q < kx; q += 256) out[((size_t)p * ky + i) * kx + q] = fail == 0 ? s_vec[q] : NAN;
        if (info && tid == 0) info[(size_t)p * ky + i] = fail;
        if (MODE != RT_FWD && dlam_part) {
            float term = 0.f;
            for (int q = tid; q < kx; q += 256)
                term += (fail == 0 ? s_vec[q] : NAN) * s_dval[q] * Cfwd[((size_t)p * ky + i) * kx + q];
            term = wave_sum(term);
            if (lane == 0) s_red[wave] = term;
            __syncthreads();
            if (tid == 0) dlam_part[(size_t)p * ky + i] = -((s_red[0] + s_red[1]) + (s_red[2] + s_red[3]));
        }
        __syncthreads();  // LDS and the slot are reused by the next system
    }
}

// ---------------------------------------------------------------------------
// Batched products for the adjoint at any k (operands streamed from global
// memory / L2).  Out[p] (M x N, row-major) = sum over two K-segments s of
// sign_s * X_s Y_s, where X_s is M x K_s read as stored ("N") or as the
// transpose of a K_s x M row-major array ("T"), and Y_s is K_s x N row-major.
// One 4-wave workgroup per 32x32 output tile.  K is cut into batches of 16;
// wave w takes batches w, w + 4, ... of each segment and keeps the loads of the
// next three batches in flight while it multiplies the current one.  The four partial tiles are summed
// through LDS in wave order.
// ---------------------------------------------------------------------------
struct GemmSeg {
    const float *X;
    const float *Y;
    int K;
    int transX;  // 1: X given as K x M row-major
    int ldx, ldy;
    long long strideX, strideY;  // per pair
    float sign;
};

// X load modes: 0 every segment's X transposed; 1 one segment, X as stored with 16-byte aligned rows and
// K % 8 == 0 (two 16-byte loads per lane and batch); 2 any segments and layouts.
struct GemmBatch {
    float a[8], b[8];
};

template <int XM>
__device__ __forceinline__ GemmBatch gemm_batch_load(const float *X, const float *Y, int K, int ldx, int ldy,
                                                     bool transX, int kb, int mc, int nc, int half)
{
    // lane (m, half) supplies k = kb + 8 half + u to matrix step u; every address is clamped into the
    // operand, and entries past K are masked when the operands are formed
    GemmBatch g;
    if constexpr (XM == 1) {
        const int k0 = min(kb + 8 * half, K - 8);
        const f32x4 *px = reinterpret_cast<const f32x4 *>(X + (size_t)mc * ldx + k0);
        const f32x4 v0 = px[0], v1 = px[1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            g.a[u] = v0[u];
            g.a[4 + u] = v1[u];
        }
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kc = min(kb + 8 * half + u, K - 1);
            const bool tr = XM == 0 || transX;
            g.a[u] = X[tr ? (size_t)kc * ldx + mc : (size_t)mc * ldx + kc];
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) g.b[u] = Y[(size_t)min(kb + 8 * half + u, K - 1) * ldy + nc];
    return g;
}

template <int XM>
__global__ __launch_bounds__(256) void batched_gemm_kernel(GemmSeg s0, GemmSeg s1, int nseg, int M, int N,
                                                           int tilesM, int tilesN, float *__restrict__ Out,
                                                           long long strideO)
{
    __shared__ float red[4][16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int tiles = tilesM * tilesN;
    const int p = blockIdx.x / tiles;
    const int t = blockIdx.x % tiles;
    const int I = t / tilesN, Jt = t % tilesN;
    const int m = I * 32 + l32, n = Jt * 32 + l32;
    const bool mok = m < M, nok = n < N;
    const int mc = min(m, M - 1), nc = min(n, N - 1);
    auto keep = [](float x, bool ok) { return __uint_as_float(__float_as_uint(x) & (ok ? ~0u : 0u)); };
    // this wave's steps: the batches of 16 k starting at 16 (wave + 4 j) of segment 0, then those of
    // segment 1; their count is rounded up to a multiple of 4 for the four-buffer rotation (a step past
    // the last is masked to zero)
    const int nb0 = max(0, ((s0.K + 15) / 16 - wave + 3) / 4);
    const int nb1 = nseg > 1 ? max(0, ((s1.K + 15) / 16 - wave + 3) / 4) : 0;
    const int nsteps = (nb0 + nb1 + 3) & ~3;
    const float *X0 = s0.X + (long long)p * s0.strideX, *Y0 = s0.Y + (long long)p * s0.strideY;
    const float *X1 = s1.X + (long long)p * s1.strideX, *Y1 = s1.Y + (long long)p * s1.strideY;
    auto load = [&](int st) {
        const bool first = st < nb0 || nseg == 1;
        const int kb = 16 * (wave + 4 * (first ? st : st - nb0));
        return first ? gemm_batch_load<XM>(X0, Y0, s0.K, s0.ldx, s0.ldy, s0.transX, kb, mc, nc, half)
                     : gemm_batch_load<XM>(X1, Y1, s1.K, s1.ldx, s1.ldy, s1.transX, kb, mc, nc, half);
    };
    f32x16 acc = zero16();
    auto mma = [&](int st, const GemmBatch &g) {
        const bool first = st < nb0 || nseg == 1;
        const int kb = 16 * (wave + 4 * (first ? st : st - nb0));
        const int K = first ? s0.K : s1.K;
        const float sign = first ? s0.sign : s1.sign;
        const bool live = st < nb0 + nb1;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool kok = live && kb + 8 * half + u < K;
            acc = mfma32x32x2(keep(sign * g.a[u], mok && kok), keep(g.b[u], nok && kok), acc);
        }
    };
    GemmBatch g0 = load(0), g1 = load(1), g2 = load(2), g3;
    for (int st = 0; st < nsteps; st += 4) {
        g3 = load(st + 3);
        mma(st, g0);
        g0 = load(st + 4);
        mma(st + 1, g1);
        g1 = load(st + 5);
        mma(st + 2, g2);
        g2 = load(st + 6);
        mma(st + 3, g3);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
    __syncthreads();
    float *O = Out + (long long)p * strideO;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int r = 4 * wave + rr;
        const float v = ((red[0][r][lane] + red[1][r][lane]) + red[2][r][lane]) + red[3][r][lane];
        const int row = I * 32 + acc32_row(r, lane);
        if (row < M && nok) O[(size_t)row * N + n] = v;
    }
}

// Sum of the per-row dlambda terms of each pair, in row order.
__global__ void dlam_sum_kernel(const float *__restrict__ part, int P, int ky, float *__restrict__ dlam)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float s = 0.f;
    for (int i = 0; i < ky; ++i) s += part[(size_t)p * ky + i];
    dlam[p] = s;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static int cu_count()
{
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) return 256;
    return c;
}

// Workgroups (and workspace slots) of the left-looking launch: up to four per CU.
static int64_t ll_slots(int64_t nsys)
{
    const int64_t cap = 4 * (int64_t)cu_count();
    return nsys < cap ? nsys : cap;
}

// Tile rows of the instance for k_x (k_x + 1 rows, with the appended right-hand side)
static int ll_tmax(int64_t kx) { return kx < 128 ? 4 : (kx < 224 ? 7 : 10); }

size_t tiled_workspace_bytes(int64_t P, int64_t kx, int64_t ky)
{
    const int64_t tm = ll_tmax(kx);
    return (size_t)ll_slots(P * ky) * (tm * (tm + 1) / 2) * LTS * sizeof(float);
}

template <int TMAX, int MODE, bool STORE>
static void launch_ll(const float *K, const float *rhs, const float *ex, const float *ey, const float *lam,
                      int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out, float *Lout, int *info,
                      const float *Cfwd, float *dlam_part, float *ws, hipStream_t st, const int *only)
{
    const size_t lds = (size_t)ll_lds_floats(TMAX) * sizeof(float);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)rowsolve_ll_kernel<TMAX, MODE, STORE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    // one round of resident workgroups (the runtime's occupancy for this instance, at most the four per CU the
    // workspace holds slots for): a persistent grid larger than what fits would leave the surplus workgroups
    // waiting for whole early workgroups, which loop over several systems each.  At TMAX = 10 three would fit
    // but measured slower than two (k = 300: 1.23 against 1.05 ms per forward solve).
    static int per_cu = 0;
    if (per_cu == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)rowsolve_ll_kernel<TMAX, MODE, STORE>, 256, lds) !=
                hipSuccess ||
            n < 1)
            n = 1;
        const int cap = TMAX == 10 ? 2 : 4;
        per_cu = n < cap ? n : cap;
    }
    const int64_t nsys = P * ky;
    const int64_t grid = std::min<int64_t>(nsys, (int64_t)per_cu * cu_count());
    hipLaunchKernelGGL((rowsolve_ll_kernel<TMAX, MODE, STORE>), dim3((unsigned)grid), dim3(256), lds, st, K, rhs, ex, ey, lam,
                       mask_kind, gamma, (int)kx, (int)ky, (int)nsys, out, Lout, info, Cfwd, dlam_part, ws, cu_count(),
                       only);
}

void launch_rowsolve_tiled(int mode, const float *K, const float *rhs, const float *ex, const float *ey,
                           const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out,
                           float *Lout, int *info, const float *Cfwd, float *dlam_part, float *tws, hipStream_t st,
                           const int *only)
{
    const int tm = ll_tmax(kx);
#define FMAP_LL(TM, MD, SF) launch_ll<TM, MD, SF>(K, rhs, ex, ey, lam, mask_kind, gamma, P, kx, ky, out, Lout, info, \
                                                  Cfwd, dlam_part, tws, st, only)
    if (mode == RT_FWD && Lout) {
        if (tm == 4) FMAP_LL(4, RT_FWD, true);
        else if (tm == 7) FMAP_LL(7, RT_FWD, true);
        else FMAP_LL(10, RT_FWD, true);
    } else if (mode == RT_FWD) {
        if (tm == 4) FMAP_LL(4, RT_FWD, false);
        else if (tm == 7) FMAP_LL(7, RT_FWD, false);
        else FMAP_LL(10, RT_FWD, false);
    } else {
        if (tm == 4) FMAP_LL(4, RT_BWD_RECOMPUTE, false);
        else if (tm == 7) FMAP_LL(7, RT_BWD_RECOMPUTE, false);
        else FMAP_LL(10, RT_BWD_RECOMPUTE, false);
    }
#undef FMAP_LL
}

static void gemm(const GemmSeg &s0, const GemmSeg *s1, int64_t P, int M, int N, float *Out, long long strideO,
                 hipStream_t st)
{
    const int tM = (M + 31) / 32, tN = (N + 31) / 32;
    const unsigned grid = (unsigned)(P * tM * tN);
    GemmSeg z = s0;
    z.K = 0;
    const int nseg = s1 ? 2 : 1;
    const GemmSeg &t1 = s1 ? *s1 : z;
    auto aligned = [](const GemmSeg &g) {
        return g.ldx % 4 == 0 && g.strideX % 4 == 0 && g.K >= 8 && g.K % 8 == 0 && ((uintptr_t)g.X & 15) == 0;
    };
    if (s0.transX && (!s1 || s1->transX))
        hipLaunchKernelGGL(batched_gemm_kernel<0>, dim3(grid), dim3(256), 0, st, s0, t1, nseg, M, N, tM, tN, Out,
                           strideO);
    else if (!s1 && !s0.transX && aligned(s0))
        hipLaunchKernelGGL(batched_gemm_kernel<1>, dim3(grid), dim3(256), 0, st, s0, t1, nseg, M, N, tM, tN, Out,
                           strideO);
    else
        hipLaunchKernelGGL(batched_gemm_kernel<2>, dim3(grid), dim3(256), 0, st, s0, t1, nseg, M, N, tM, tN, Out,
                           strideO);
}

// W = V^T C + C^T V (into Wbuf), dB = V A, dA = V^T B - W A.
void launch_adjoint_general(const float *V, const float *C, const float *A, const float *B, int64_t P, int64_t kx,
                            int64_t ky, int64_t d, float *Wbuf, const float *dlam_part, float *dlam, float *dA,
                            float *dB, hipStream_t st)
{
    const long long skk = kx * ky, sxd = kx * d, syd = ky * d, sww = kx * kx;
    GemmSeg w0{V, C, (int)ky, 1, (int)kx, (int)kx, skk, skk, 1.f};
    GemmSeg w1{C, V, (int)ky, 1, (int)kx, (int)kx, skk, skk, 1.f};
    gemm(w0, &w1, P, (int)kx, (int)kx, Wbuf, sww, st);
    GemmSeg b0{V, A, (int)kx, 0, (int)kx, (int)d, skk, sxd, 1.f};
    gemm(b0, nullptr, P, (int)ky, (int)d, dB, syd, st);
    GemmSeg a0{V, B, (int)ky, 1, (int)kx, (int)d, skk, syd, 1.f};
    GemmSeg a1{Wbuf, A, (int)kx, 1, (int)kx, (int)d, sww, sxd, -1.f};  // W symmetric: W^T = W
    gemm(a0, &a1, P, (int)kx, (int)d, dA, sxd, st);
    if (dlam)
        hipLaunchKernelGGL(dlam_sum_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, dlam_part, (int)P,
                           (int)ky, dlam);
}

}  // namespace fmap

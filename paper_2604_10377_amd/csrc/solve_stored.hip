// Row solves with stored float32 factors: the reverse mode's S_i v_i = g_i
// and the refinement correction S_i delta_i = rho_i (Eqs. (6), (7) with the
// factor of Eq. (5) kept from the forward pass).  trisolve_stored_kernel
// serves 64 < k_x <= 319, trisolve_small_kernel (at the end) k_x <= 64.
//
// With the factor known, a system is two triangular solves over k_x^2/2
// stored floats, so the work is streaming the factor, once per substitution.
// Large k_x: one wave per system; lane j holds rows j, j + 64, ... (NS slots).
// The factor is packed lower, column-major, so column c is contiguous:
//   * forward L y = r column by column (y_c = r_c / L_cc, then the rows below
//     subtract L_qc y_c), with the slot and lane of c compile-time, so y_c and
//     L_cc are single readlanes and each slot takes one fused multiply-add;
//   * back substitution L^T x = y one slot of 64 columns at a time, lane c
//     taking column c: the slots already solved contribute the dot product of
//     the lane's own contiguous column segment with their x, and the 64 x 64
//     diagonal block is solved column by column from the block's columns in
//     the lanes' registers, so no step needs a cross-lane reduction.
#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

namespace {

__device__ __forceinline__ int pcol(int c, int k) { return c * k - (c * (c - 1)) / 2; }

__device__ __forceinline__ float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

}  // namespace

template <int NS>
__global__ __launch_bounds__(256) void trisolve_stored_kernel(const float *__restrict__ Lin,
                                                             const float *__restrict__ rhs,
                                                             const float *__restrict__ ex, const float *__restrict__ ey,
                                                             const float *__restrict__ lam, int mask_kind, float gamma,
                                                             int kx, int ky, int nsys, float *out,
                                                             int *__restrict__ info, const float *__restrict__ Cfwd,
                                                             float *__restrict__ dlam_part, const float *addend,
                                                             const int *__restrict__ only)
{
    const int j = threadIdx.x & 63;
    // the system index in a scalar register, so the buffer descriptor below is one per wave
    const int sys = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (sys >= nsys) return;  // wave-uniform; no block-level barrier below
    const int p = sys / ky, i = sys - p * ky;
    if (only && __builtin_amdgcn_readfirstlane(only[p]) == 0) return;  // wave-uniform
    const float *Lp = Lin + (size_t)sys * (kx * (kx + 1) / 2);

    // every input load first (unconditional, clamped), then the validity of lambda and of the
    // resolvent normaliser (as in the forward solve)
    const float lamv = lam[p];
    float exv[NS], eyv[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int q = j + 64 * s;
        exv[s] = ex[(size_t)p * kx + min(q, kx - 1)];
        eyv[s] = ey[(size_t)p * ky + min(q, ky - 1)];
        y[s] = rhs[(size_t)sys * kx + min(q, kx - 1)];
    }
    int fail = 0;
    if (!(lamv >= 0.f) || !isfinite(lamv)) fail = -1;
    MaskParams mp;
    mp.kind = mask_kind;
    mp.gamma = gamma;
    mp.inv_scale = 1.f;
    if (mask_kind == 1) {
        float mx = -INFINITY;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int q = j + 64 * s;
            mx = fmaxf(mx, fmaxf(q < kx ? exv[s] : -INFINITY, q < ky ? eyv[s] : -INFINITY));
        }
        for (int q = j + 64 * NS; q < ky; q += 64) mx = fmaxf(mx, ey[(size_t)p * ky + q]);
        mx = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_max(mx))));
        if ((!(mx > 0.f) || !isfinite(mx)) && fail == 0) fail = -2;
        mp.inv_scale = 1.f / mx;
    }
    fail = __builtin_amdgcn_readfirstlane(fail);
#pragma unroll
    for (int s = 0; s < NS; ++s) y[s] = j + 64 * s < kx ? y[s] : 0.f;

    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)Lp, 0, (int)(kx * (kx + 1) / 2 * sizeof(float)), 0x00020000);
    // element (row, col) of the packed factor (row >= col) is at pcol(col) + row - col.  Through the buffer
    // descriptor, reads past the factor's end return 0; reads of other entries (rows above the diagonal, rows
    // past k_x) are finite and meet only zero or masked operands.
    auto ldf = [&](int voff_floats, int soff_floats) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4 * voff_floats, 4 * soff_floats, 0));
    };

    // ---- forward substitution L y = r, column by column: slot s and the lane of column c are compile-time, so
    // y_c and L_cc are single readlanes, and the rows below c take one fused multiply-add per slot (the slot of
    // c under a lane mask).  Columns come in groups of 8, the next group's loads in flight while one is used;
    // a group loads only the slots at or below its own (the rows above the diagonal are never needed).
    if (fail == 0) {
        float ba[8][NS], bb[8][NS];
        auto load_group = [&](int q, float (&buf)[8][NS]) {  // q = 8 s + g, compile-time
            const int s0 = q / 8;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int c = min(8 * q + t, kx - 1);
                const int so = pcol(c, kx) - c;
#pragma unroll
                for (int sl = 0; sl < NS; ++sl)
                    if (sl >= s0) buf[t][sl] = ldf(j + 64 * sl, so);
            }
        };
        auto fwd_group = [&](int q, const float (&buf)[8][NS]) {
            const int s0 = q / 8;
            int lane = j;
            asm volatile("" : "+v"(lane));  // masks formed per column, not hoisted into scalar registers
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int c = 8 * q + t, cl = c & 63;
                const float dg = uniform_f(readlane(buf[t][s0], cl));
                const bool act = c < kx && fail == 0;
                const bool bad = !(dg > 0.f) || !isfinite(dg);
                fail = (act && bad) ? c + 1 : fail;
                const bool go = act && !bad;
                const float yc = go ? uniform_f(readlane(y[s0], cl) * __builtin_amdgcn_rcpf(dg)) : 0.f;
                y[s0] = (lane > cl) ? y[s0] - buf[t][s0] * yc : ((lane == cl && go) ? yc : y[s0]);
#pragma unroll
                for (int sl = 0; sl < NS; ++sl)
                    if (sl > s0) y[sl] -= buf[t][sl] * yc;
            }
        };
        constexpr int NQ = 8 * NS;
        load_group(0, ba);
#pragma unroll
        for (int q = 0; q < NQ; q += 2) {
            if (8 * q >= kx) break;
            load_group(q + 1 < NQ ? q + 1 : q, bb);
            fwd_group(q, ba);
            if (8 * (q + 1) >= kx || q + 1 >= NQ) break;
            load_group(q + 2 < NQ ? q + 2 : q + 1, ba);
            fwd_group(q + 1, bb);
        }
        fail = __builtin_amdgcn_readfirstlane(fail);
    }

    // ---- back substitution L^T x = y, 64 columns (one slot) at a time from the last, lane c taking column
    // 64 s + c: the finished slots below contribute the dot product of the lane's own column segment (contiguous
    // in the column-major factor) with their x, and the diagonal block is then solved column by column with the
    // block's columns in the lanes' registers (L[64 s + r][64 s + c] in register r of lane c), so no step needs a
    // cross-lane reduction.
    float x[NS];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) x[sl] = 0.f;
    if (fail == 0) {
#pragma unroll
        for (int s0 = NS - 1; s0 >= 0; --s0) {
            if (64 * s0 >= kx) continue;
            const int col = 64 * s0 + j;
            const int cb = pcol(min(col, kx - 1), kx) - min(col, kx - 1);  // factor offset of (row 0, this column)
            const bool colok = col < kx;
            // the finished slots' rows 64 sl .. 64 sl + 63 of this lane's column in chunks of 16, slots from the
            // last, the next chunk's loads in flight while one is used (every slot below NS holds rows:
            // NS = ceil(k_x / 64)).  The diagonal block's column segment is loaded after them, except in the
            // widest instance, where loading it first measured faster (k = 300: 0.350 against 0.376 ms per
            // reverse-mode call; k = 200: 0.235 against 0.252 ms the other way round).
            float dl[64];
            if constexpr (NS >= 5) {
#pragma unroll
                for (int r = 0; r < 64; ++r) dl[r] = ldf(cb + r, 64 * s0);
            }
            float v = y[s0];
            constexpr int CH = 4;                // chunks of 16 rows per slot
            const int nch = CH * (NS - 1 - s0);  // compile-time once s0 is unrolled
            float la[16], lb[16];
            auto load_chunk = [&](int c, float (&buf)[16]) {
                const int sl = NS - 1 - c / CH, r0 = 16 * (c % CH);
#pragma unroll
                for (int r = 0; r < 16; ++r) buf[r] = ldf(cb + r0 + r, 64 * sl);
            };
            auto use_chunk = [&](int c, const float (&buf)[16]) {
                const int sl = NS - 1 - c / CH, r0 = 16 * (c % CH);
#pragma unroll
                for (int r = 0; r < 16; ++r) v -= buf[r] * uniform_f(readlane(x[sl], r0 + r));
            };
            if (nch > 0) load_chunk(0, la);
#pragma unroll
            for (int c = 0; c < nch; c += 2) {
                if (c + 1 < nch) load_chunk(c + 1, lb);
                use_chunk(c, la);
                if (c + 1 >= nch) break;
                if (c + 2 < nch) load_chunk(c + 2, la);
                use_chunk(c + 1, lb);
            }
            if constexpr (NS < 5) {
#pragma unroll
                for (int r = 0; r < 64; ++r) dl[r] = ldf(cb + r, 64 * s0);
            }
            int lane = j;
            asm volatile("" : "+v"(lane));
            float xs = 0.f;
#pragma unroll
            for (int c2 = 63; c2 >= 0; --c2) {
                const bool act = 64 * s0 + c2 < kx;
                const float xc = act ? uniform_f(readlane(v, c2) * __builtin_amdgcn_rcpf(readlane(dl[c2], c2))) : 0.f;
                v = (lane < c2) ? v - dl[c2] * xc : v;
                xs = (lane == c2) ? xc : xs;
            }
            x[s0] = colok ? xs : 0.f;
        }
    }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) y[sl] = x[sl];

    const float muy = ey[(size_t)p * ky + i];
    float term = 0.f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int q = j + 64 * s;
        if (q < kx) {
            const size_t o = (size_t)sys * kx + q;
            const float v = fail == 0 ? y[s] : NAN;
            out[o] = addend ? addend[o] + v : v;  // addend: refinement correction c += delta (in place)
            if (dlam_part) term += v * mask_entry(muy, exv[s], mp) * Cfwd[o];
        }
    }
    if (info && j == 0) info[sys] = fail;
    if (dlam_part) {
        const float sum = wave_sum(term);
        if (j == 0) dlam_part[sys] = -sum;
    }
}

void launch_trisolve_stored(const float *Lin, const float *rhs, const float *ex, const float *ey, const float *lam,
                            int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out, int *info,
                            const float *Cfwd, float *dlam_part, const float *addend, hipStream_t st, const int *only)
{
    const int nsys = (int)(P * ky);
    const dim3 grid((unsigned)((nsys + 3) / 4)), block(256);
#define FMAP_TS(NS)                                                                                              \
    hipLaunchKernelGGL((trisolve_stored_kernel<NS>), grid, block, 0, st, Lin, rhs, ex, ey, lam, mask_kind, gamma, \
                       (int)kx, (int)ky, nsys, out, info, Cfwd, dlam_part, addend, only)
    switch ((kx + 63) / 64) {
    case 1: FMAP_TS(1); break;
    case 2: FMAP_TS(2); break;
    case 3: FMAP_TS(3); break;
    case 4: FMAP_TS(4); break;
    default: FMAP_TS(5); break;
    }
#undef FMAP_TS
}

// ---------------------------------------------------------------------------
// The same two solves for k_x <= 64 (KMAX >= k_x): one wave per system, lane j
// holding row j and column j of the factor.  The rows are loaded from the
// packed storage (for each q the lanes read consecutive addresses) and the
// columns come from them through LDS (row j written by lane j, column j read
// back by lane j): loading the columns directly would have each lane walk its
// own column, one cache line per lane and load instruction.  The
// off-diagonal entries are scaled by the inverse pivots up front, so each
// substitution step is a broadcast of one lane's running value and one fused
// multiply-add:
//   forward  L y = r:    r_j -= (L_jc / L_cc) r_c   (c ascending),  y_j = r_j / L_jj
//   backward L^T x = y:  y_j -= (L_cj / L_cc) y_c   (c descending), x_j = y_j / L_jj
// (a lane's own value is final once its step has passed).  Rows k_x <= j <
// KMAX are identity rows: no k_x checks in the loops.
// ---------------------------------------------------------------------------
template <int KMAX> struct TrisolveLds {
    static constexpr int KP = KMAX + 4;  // row stride (floats): 16-byte row writes, conflict-free column reads
    static constexpr int PER_WAVE = KMAX * KP;
};

template <int KMAX>
__global__ __launch_bounds__(256) void trisolve_small_kernel(const float *__restrict__ Lin,
                                                            const float *__restrict__ rhs,
                                                            const float *__restrict__ ex, const float *__restrict__ ey,
                                                            const float *__restrict__ lam, int mask_kind, float gamma,
                                                            int kx, int ky, int nsys, float *out,
                                                            int *__restrict__ info, const float *__restrict__ Cfwd,
                                                            float *__restrict__ dlam_part, const float *addend)
{
    static_assert(KMAX % 4 == 0 && KMAX <= 64, "register row length");
    const int j = threadIdx.x & 63;
    // the system index in a scalar register, so the buffer descriptor below is one per wave
    const int sys = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (sys >= nsys) return;  // wave-uniform; no block-level barrier below
    const int p = sys / ky, i = sys - p * ky;
    const float *Lp = Lin + (size_t)sys * (kx * (kx + 1) / 2);
    const bool jok = j < kx;
    const int jc = jok ? j : kx - 1;

    // every input load first, from clamped addresses (entries outside the triangle are masked below)
    const float lamv = lam[p];
    const float muy = ey[(size_t)p * ky + i];
    const float exj = ex[(size_t)p * kx + jc];
    const float eyj = ey[(size_t)p * ky + min(j, ky - 1)];
    const float rin = rhs[(size_t)sys * kx + jc];
    const int pj = pcol(jc, kx);  // column jc starts here; its diagonal entry first
    const float dgl = Lp[pj];
    // element (row, col) of the packed factor is at pcol(col) + row - col: with a buffer descriptor the
    // row loads take a lane offset of 4 jc and a scalar offset per column, so they need no vector
    // address arithmetic.  Lanes outside the triangle read neighbouring entries of the same factor
    // (masked below); the descriptor's range bounds every access to this system's factor.
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)Lp, 0, (int)(kx * (kx + 1) / 2 * sizeof(float)), 0x00020000);
    float rowv[KMAX], colv[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {  // rowv[q] = L[j][q] for q <= j
        const int qc = min(q, kx - 1);
        // (the builtin returns the 32 bits as an integer: reinterpreted, not converted)
        rowv[q] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 4 * jc, 4 * (pcol(qc, kx) - qc), 0));
    }
    // colv[q] = L[q][j] for q >= j: entry j of row q, through this wave's LDS tile
    {
        extern __shared__ __align__(16) float s_ts[];
        constexpr int KP = TrisolveLds<KMAX>::KP;
        float *sL = s_ts + (threadIdx.x >> 6) * TrisolveLds<KMAX>::PER_WAVE;
        if (j < KMAX) {
#pragma unroll
            for (int q4 = 0; q4 < KMAX / 4; ++q4)
                *reinterpret_cast<f32x4 *>(&sL[j * KP + 4 * q4]) =
                    f32x4{rowv[4 * q4], rowv[4 * q4 + 1], rowv[4 * q4 + 2], rowv[4 * q4 + 3]};
        }
        __builtin_amdgcn_wave_barrier();
        const int jr = min(j, KMAX - 1);
#pragma unroll
        for (int q = 0; q < KMAX; ++q) colv[q] = sL[q * KP + jr];
    }

    int fail = 0;
    if (!(lamv >= 0.f) || !isfinite(lamv)) fail = -1;
    MaskParams mp;
    mp.kind = mask_kind;
    mp.gamma = gamma;
    mp.inv_scale = 1.f;
    if (mask_kind == 1) {
        float mx = fmaxf(jok ? exj : -INFINITY, j < ky ? eyj : -INFINITY);  // k_x <= 64
        for (int q = j + 64; q < ky; q += 64) mx = fmaxf(mx, ey[(size_t)p * ky + q]);
        mx = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_max(mx))));
        if ((!(mx > 0.f) || !isfinite(mx)) && fail == 0) fail = -2;
        mp.inv_scale = 1.f / mx;
    }
    // pivots: the first non-positive or non-finite one is reported (LAPACK info)
    const float dg = jok ? dgl : 1.f;
    const uint64_t bad = __ballot(!(dg > 0.f) || !isfinite(dg));
    if (fail == 0 && bad != 0) fail = (int)__builtin_ctzll(bad) + 1;
    fail = __builtin_amdgcn_readfirstlane(fail);
    const float inv = __builtin_amdgcn_rcpf(dg);

#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const float iq = readlane(inv, q);
        rowv[q] = (jok && q < j) ? rowv[q] * iq : 0.f;
        colv[q] = (jok && q > j) ? colv[q] * iq : 0.f;
    }
    float r = jok ? rin : 0.f;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) r = fmaf(-rowv[c], readlane(r, c), r);
    float y = r * inv;
#pragma unroll
    for (int c = KMAX - 1; c >= 0; --c) y = fmaf(-colv[c], readlane(y, c), y);
    const float x = y * inv;

    const float cv = fail == 0 ? x : NAN;
    if (jok) {
        const size_t o = (size_t)sys * kx + j;
        out[o] = addend ? addend[o] + cv : cv;  // addend: refinement correction c += delta (in place)
    }
    if (info && j == 0) info[sys] = fail;
    if (dlam_part) {
        const float dval = (jok && fail == 0) ? mask_entry(muy, exj, mp) : 0.f;
        const float term = jok ? cv * dval * Cfwd[(size_t)sys * kx + j] : 0.f;
        const float sum = wave_sum(term);
        if (j == 0) dlam_part[sys] = -sum;
    }
}

void launch_trisolve_small(const float *Lin, const float *rhs, const float *ex, const float *ey, const float *lam,
                           int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out, int *info,
                           const float *Cfwd, float *dlam_part, const float *addend, hipStream_t st)
{
    const int nsys = (int)(P * ky);
    const dim3 grid((unsigned)((nsys + 3) / 4)), block(256);
    // dynamic LDS: 4 waves x KM (KM + 4) floats, at most 69.6 KB
#define FMAP_TSS(KM)                                                                                              \
    do {                                                                                                          \
        const size_t lds_ = (size_t)4 * TrisolveLds<KM>::PER_WAVE * sizeof(float);                                \
        static bool attr_ = false;                                                                                \
        if (!attr_) {                                                                                             \
            (void)hipFuncSetAttribute((const void *)trisolve_small_kernel<KM>,                                    \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_);                     \
            attr_ = true;                                                                                         \
        }                                                                                                         \
        hipLaunchKernelGGL((trisolve_small_kernel<KM>), grid, block, lds_, st, Lin, rhs, ex, ey, lam, mask_kind,  \
                           gamma, (int)kx, (int)ky, nsys, out, info, Cfwd, dlam_part, addend);                    \
    } while (0)
    if (kx <= 8) FMAP_TSS(8);
    else if (kx <= 16) FMAP_TSS(16);
    else if (kx <= 24) FMAP_TSS(24);
    else if (kx <= 32) FMAP_TSS(32);
    else if (kx <= 40) FMAP_TSS(40);
    else if (kx <= 48) FMAP_TSS(48);
    else if (kx <= 52) FMAP_TSS(52);
    else if (kx <= 56) FMAP_TSS(56);
    else FMAP_TSS(64);
#undef FMAP_TSS
}

}  // namespace fmap

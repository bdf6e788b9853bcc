// Spectral projection, Eq. (1) read as the mass-weighted pseudo-inverse:
//     A[b] = Phi[b]^T diag(M[b]) F[b]          (forward)
//     dF[b] = diag(M[b]) Phi[b] dA[b]           (its adjoint)
//
// Both are tall-skinny contractions over vertex-major (n-major) arrays and run
// on the float32 matrix cores (v_mfma_f32_32x32x2f32).
//
// Forward: the reduction over n is split into `nsplit` chunks.  A workgroup
// (4 waves) owns one (shape, chunk, k-block, d-block); each wave owns an
// MT*32 x NT*32 accumulator tile.  Per matrix-core step a lane reads one basis
// value and one feature value of vertex v0 + lane/32: 32 consecutive floats of
// a vertex row per half-wave, so every Phi and F byte is read from HBM once.
// Partial sums go to a workspace and a second kernel adds the chunks in a fixed
// order (deterministic, and chunked accumulation keeps the float32 error of a
// 1e5-term sum small).
//
// Backward: rows of dF are vertices; a wave owns 32 vertices x NT*32 feature
// columns and contracts over k.  The two lane halves take the two halves of
// the k range, so a lane walks along its own basis row.
#include "fmap_device.h"
#include "fmap_launch.h"
#include "fmap_lds.h"

namespace fmap {

template <typename T>
__device__ __forceinline__ float load_elem(const T *p, size_t i);
template <>
__device__ __forceinline__ float load_elem<float>(const float *p, size_t i) { return p[i]; }
template <>
__device__ __forceinline__ float load_elem<uint16_t>(const uint16_t *p, size_t i) { return bf16_to_f32(p[i]); }

// One (shape, vertex range, k-block, column block) of the forward projection:
// partial A rows [kbase, kbase + MT*32) x columns [dbase4 + wave*NT*32, ...)
// over vertices [v0, v1), written to O (row-major k x d).
template <typename T, int MT, int NT, int U>
__device__ __forceinline__ void proj_fwd_tile(const T *__restrict__ P, const float *__restrict__ Mv,
                                              const T *__restrict__ F, int k, int d, int v0, int v1, int kbase,
                                              int dbase4, float *__restrict__ O)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int dbase = dbase4 + wave * (NT * 32);
    if (dbase >= d) return;  // whole wave idle (narrow d)

    int rows[MT], cols[NT];
    bool rok[MT], cok[NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        rows[mt] = kbase + mt * 32 + l32;
        rok[mt] = rows[mt] < k;
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        cols[nt] = dbase + nt * 32 + l32;
        cok[nt] = cols[nt] < d;
    }

    f32x16 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = zero16();

    // Two register stages of U matrix-core steps (2U vertices): the loads of one
    // stage are in flight while the other stage's multiplies run.
    float pa0[U][MT], pb0[U][NT], m0[U], pa1[U][MT], pb1[U][NT], m1[U];
    auto load = [&](float (&pa)[U][MT], float (&pb)[U][NT], float (&mv)[U], int v) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned vv = (unsigned)(v + 2 * u + half);
            mv[u] = Mv[vv];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) pa[u][mt] = rok[mt] ? load_elem(P, vv * (unsigned)k + rows[mt]) : 0.f;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) pb[u][nt] = cok[nt] ? load_elem(F, vv * (unsigned)d + cols[nt]) : 0.f;
        }
    };
    auto mma = [&](float (&pa)[U][MT], float (&pb)[U][NT], float (&mv)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const float a = pa[u][mt] * mv[u];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma32x32x2(a, pb[u][nt], acc[mt][nt]);
            }
    };
    const int S = 2 * U;
    const int nst = (v1 - v0) / S;
    int v = v0;
    if (nst > 0) load(pa0, pb0, m0, v);
    for (int st = 0; st < nst; st += 2) {
        if (st + 1 < nst) load(pa1, pb1, m1, v + S);
        mma(pa0, pb0, m0);
        if (st + 2 < nst) load(pa0, pb0, m0, v + 2 * S);
        if (st + 1 < nst) mma(pa1, pb1, m1);
        v += 2 * S;
    }
    // Tail: guarded single steps.
    for (v = v0 + nst * S; v < v1; v += 2) {
        const int vv = v + half;
        const bool ok = vv < v1;
        const float m = ok ? Mv[vv] : 0.f;
        float a[MT], b[NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = (ok && rok[mt]) ? load_elem(P, (size_t)vv * k + rows[mt]) * m : 0.f;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b[nt] = (ok && cok[nt]) ? load_elem(F, (size_t)vv * d + cols[nt]) : 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma32x32x2(a[mt], b[nt], acc[mt][nt]);
    }

#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = kbase + mt * 32 + acc32_row(r, lane);
                if (row < k && cok[nt]) O[(size_t)row * d + cols[nt]] = acc[mt][nt][r];
            }
}

template <typename T, int MT, int NT, int U>
__global__ __launch_bounds__(256) void proj_fwd_kernel(const T *__restrict__ phi, const float *__restrict__ mass,
                                                       const T *__restrict__ feat, int n, int k, int d, int nsplit,
                                                       int chunk, int kblocks, int dblocks,
                                                       float *__restrict__ out)
{
    int bid = blockIdx.x;
    const int db = bid % dblocks;
    bid /= dblocks;
    const int kb = bid % kblocks;
    bid /= kblocks;
    const int split = bid % nsplit;
    const int s = bid / nsplit;
    const int v0 = split * chunk;
    const int v1 = min(n, v0 + chunk);
    proj_fwd_tile<T, MT, NT, U>(phi + (size_t)s * n * k, mass + (size_t)s * n, feat + (size_t)s * n * d, k, d, v0, v1,
                                kb * (MT * 32), db * 4 * (NT * 32),
                                out + ((size_t)s * nsplit + split) * (size_t)k * d);
}

// Persistent forward over a table of work items (uneven shapes): each workgroup
// takes items blockIdx.x, blockIdx.x + gridDim.x, ...
template <int MT, int NT, int U>
__global__ __launch_bounds__(256) void proj_fwd_items_kernel(const FwdItem *__restrict__ items, int nitems)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const FwdItem w = items[it];
        proj_fwd_tile<float, MT, NT, U>(global_ptr(w.phi), global_ptr(w.mass), global_ptr(w.feat), w.k, w.d, w.v0, w.v1,
                                        w.kbase, w.dbase, global_ptr(w.out));
    }
}

// ---------------------------------------------------------------------------
// Forward, LDS-pipelined variant (float32, k <= 64, one 256-column block of d
// per workgroup).  Vertices are consumed in stages of FS = 32: the feature rows
// (1 KB each), the contiguous basis tile and the masses of a stage arrive by
// direct global->LDS loads (global_load_lds_dwordx4) into a ring of FNST stage
// buffers, two stages ahead of the multiplies, so ~80 KB per CU are in flight
// without occupying registers and the basis is read once per workgroup.
// Every wave issues exactly FL loads per stage (addresses clamped into the
// valid range, never exec-masked), which makes the vmcnt accounting exact.
//
// 8 waves: wave = (column group cg of 64 columns) x (vertex parity vg).  A
// wave runs the 16x16x4 float32 matrix cores on MT16 row tiles of 16 and
// NT16 = 4 column tiles; REM (<= 4) trailing rows of k are accumulated with
// plain FMAs instead of padding a whole 16-row tile (k = 50 = 3*16 + 2).
// The two parity groups are summed through LDS at the end.
// ---------------------------------------------------------------------------
constexpr int FS = 32;            // vertices per stage
constexpr int FNST = 3;           // stage buffers in the ring
constexpr int FLDF = 256 + 16;    // LDS row stride of the feature tile (floats)
constexpr int FL = 6;             // direct loads per wave per stage
constexpr int F_TILE = FS * FLDF;             // floats
constexpr int P_TILE = 8 * 256;               // basis tile: up to 8 KB (k <= 64)
constexpr int M_TILE = 256;                   // masses: one 1 KB load window
constexpr int STAGE_FLOATS = F_TILE + P_TILE + M_TILE;
constexpr size_t FWD_LDS_BYTES = (size_t)FNST * STAGE_FLOATS * sizeof(float);

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int MT16, int REM>
__global__ __launch_bounds__(512) void proj_fwd_lds_kernel(const float *__restrict__ phi,
                                                           const float *__restrict__ mass,
                                                           const float *__restrict__ feat, int n, int k, int d,
                                                           int nsplit, int dblocks, float *__restrict__ out)
{
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cg = wave & 3, vg = wave >> 2;
    const int r16 = lane & 15, g4 = lane >> 4;
    int bid = blockIdx.x;
    const int db = bid % dblocks;
    bid /= dblocks;
    const int split = bid % nsplit;
    const int s = bid / nsplit;
    const int dbase = db * 256;

    // balanced split of the stages of this shape
    const int nst_all = (n + FS - 1) / FS;
    const int st0 = (int)(((long)split * nst_all) / nsplit), st1 = (int)(((long)(split + 1) * nst_all) / nsplit);
    const int vbeg = st0 * FS, vend = min(n, st1 * FS);
    const int nst = st1 - st0;

    const float *P = phi + (size_t)s * n * k;
    const float *F = feat + (size_t)s * n * d;
    const float *Mv = mass + (size_t)s * n;

    // zero the ring once so that slots never hold non-finite garbage
    for (int e = tid * 4; e < FNST * STAGE_FLOATS; e += 512 * 4) *reinterpret_cast<f32x4 *>(&smem[e]) = f32x4{0, 0, 0, 0};
    __syncthreads();

    const int np = (k + 7) / 8;  // 1 KB basis windows per stage (32 rows x k floats)
    // Load list of a stage: 32 feature rows, np basis windows, then mass windows up to 8*FL.
    auto issue = [&](int t) {
        float *S = smem + (t % FNST) * STAGE_FLOATS;
        const int v = vbeg + t * FS;
        const int rows = min(FS, vend - v);
        const int pvalid = rows * k;  // floats of the basis tile that exist
#pragma unroll
        for (int q = 0; q < FL; ++q) {
            const int item = q * 8 + wave;
            if (item < FS) {
                const int r = min(item, rows - 1);
                const int col = min(dbase + 4 * lane, d - 4);
                dma16(F + (size_t)(v + r) * d + col, S + item * FLDF);
            } else if (item < FS + np) {
                const int wdw = item - FS;
                const int off = min(wdw * 256 + 4 * lane, ((pvalid + 3) & ~3) - 4);
                dma16(P + (size_t)v * k + off, S + F_TILE + wdw * 256);
            } else {
                const int off = min(4 * lane, ((rows + 3) & ~3) - 4);
                dma16(Mv + v + off, S + F_TILE + P_TILE);
            }
        }
    };

    f32x4 acc[MT16][4];
#pragma unroll
    for (int mt = 0; mt < MT16; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0, 0, 0, 0};
    float rem[REM > 0 ? REM : 1][4];
#pragma unroll
    for (int e = 0; e < (REM > 0 ? REM : 1); ++e)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) rem[e][nt] = 0.f;

    for (int t = 0; t < FNST - 1 && t < nst; ++t) issue(t);
    for (int t = 0; t < nst; ++t) {
        if (t + FNST - 1 < nst) issue(t + FNST - 1);
        // loads issued after stage t's: those of the next FNST-1 stages that exist
        if (t + 2 < nst) wait_vmcnt<2 * FL>();
        else if (t + 1 < nst) wait_vmcnt<FL>();
        else wait_vmcnt<0>();
        lds_barrier();
        const float *S = smem + (t % FNST) * STAGE_FLOATS;
        const float *Fs = S, *Ps = S + F_TILE, *Ms = S + F_TILE + P_TILE;
        const int vs = vbeg + t * FS;
#pragma unroll
        for (int qq = 0; qq < FS / 8; ++qq) {
            const int vloc = 4 * (2 * qq + vg) + g4;
            const float m = (vs + vloc < vend) ? Ms[vloc] : 0.f;
            float a[MT16], b[4];
#pragma unroll
            for (int mt = 0; mt < MT16; ++mt) {
                const int row = 16 * mt + r16;
                a[mt] = (REM > 0 || mt < MT16 - 1 || row < k) ? Ps[vloc * k + row] * m : 0.f;
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) b[nt] = Fs[vloc * FLDF + cg * 64 + 16 * nt + r16];
#pragma unroll
            for (int mt = 0; mt < MT16; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma16x16x4(a[mt], b[nt], acc[mt][nt]);
            if (REM > 0) {
#pragma unroll
                for (int e = 0; e < REM; ++e) {
                    const float wv = Ps[vloc * k + 16 * MT16 + e] * m;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) rem[e][nt] += wv * b[nt];
                }
            }
        }
        lds_barrier();  // the slot is refilled by the next iteration's issue
    }

    // remainder rows: sum the four vertex lane groups
    if (REM > 0) {
#pragma unroll
        for (int e = 0; e < REM; ++e)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                float v = rem[e][nt];
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                rem[e][nt] = v;
            }
    }
    // parity group 1 hands its sums to group 0 through LDS
    constexpr int PER_LANE = MT16 * 16 + (REM > 0 ? REM : 1) * 4;
    float *X = smem + (size_t)(cg * 64 + lane) * PER_LANE;
    if (vg == 1) {
#pragma unroll
        for (int mt = 0; mt < MT16; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) X[(mt * 4 + nt) * 4 + r] = acc[mt][nt][r];
        if (REM > 0) {
#pragma unroll
            for (int e = 0; e < REM; ++e)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) X[MT16 * 16 + e * 4 + nt] = rem[e][nt];
        }
    }
    __syncthreads();
    if (vg == 0) {
        float *O = out + ((size_t)s * nsplit + split) * (size_t)k * d;
#pragma unroll
        for (int mt = 0; mt < MT16; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int col = dbase + cg * 64 + 16 * nt + r16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * mt + 4 * g4 + r;
                    const float v = acc[mt][nt][r] + X[(mt * 4 + nt) * 4 + r];
                    if (row < k && col < d) O[(size_t)row * d + col] = v;
                }
            }
        if (REM > 0 && g4 == 0) {
#pragma unroll
            for (int e = 0; e < REM; ++e)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int col = dbase + cg * 64 + 16 * nt + r16;
                    const int row = 16 * MT16 + e;
                    if (col < d) O[(size_t)row * d + col] = rem[e][nt] + X[MT16 * 16 + e * 4 + nt];
                }
        }
    }
}

// ---------------------------------------------------------------------------
// Backward, LDS-pipelined variant (float32, k <= 64, 256-column block of d per
// workgroup).  The dA block (k x 256) is staged in LDS once per workgroup; the
// basis rows and masses of 64-vertex stages arrive by direct global->LDS loads
// into a 3-deep ring, two stages ahead.  8 waves = 2 row halves x 4 column
// groups; a wave owns 32 vertices x 64 columns (two 32x32 tiles) per stage and
// contracts over k with the 32x32x2 matrix cores (k = 50: 25 steps, no
// padding).  Output rows are written with buffer stores whose out-of-range
// lanes are dropped by the hardware, so every wave issues the same number of
// memory operations per stage and the vmcnt waits stay exact (stores count
// in vmcnt on this architecture).
// ---------------------------------------------------------------------------
constexpr int BS = 64;                 // vertices per stage
constexpr int BNST = 3;                // ring depth
constexpr int BLD = 256 + 32;          // LDS row stride of the dA block (floats)
constexpr int BFL = 3;                 // direct loads per wave per stage
constexpr int BNS = 32;                // stores per wave per stage
constexpr int BP_TILE = 4096;          // basis tile: 64 rows x k <= 64 floats (16 KB)
constexpr int BM_TILE = 256;           // masses: one 1 KB load window
constexpr int BSTAGE = BP_TILE + BM_TILE;
constexpr int BG_FLOATS = 64 * BLD;    // dA block, k <= 64 rows
constexpr size_t BWD_LDS_BYTES = (size_t)(BNST * BSTAGE + BG_FLOATS) * sizeof(float);

__global__ __launch_bounds__(512) void proj_bwd_lds_kernel(const float *__restrict__ phi,
                                                           const float *__restrict__ mass,
                                                           const float *__restrict__ dA, int n, int k, int d,
                                                           int nsplit, int dblocks, float *__restrict__ dF)
{
    extern __shared__ __align__(16) float smem[];
    float *sG = smem + BNST * BSTAGE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cg = wave & 3, rh = wave >> 2;
    const int half = lane >> 5, l32 = lane & 31;
    int bid = blockIdx.x;
    const int db = bid % dblocks;
    bid /= dblocks;
    const int split = bid % nsplit;
    const int s = bid / nsplit;
    const int dbase = db * 256;

    const int nst_all = (n + BS - 1) / BS;
    const int st0 = (int)(((long)split * nst_all) / nsplit), st1 = (int)(((long)(split + 1) * nst_all) / nsplit);
    const int vbeg = st0 * BS, vend = min(n, st1 * BS);
    const int nst = st1 - st0;

    const float *P = phi + (size_t)s * n * k;
    const float *Mv = mass + (size_t)s * n;
    const float *G = dA + (size_t)s * k * d;
    const __amdgpu_buffer_rsrc_t out =
        __builtin_amdgcn_make_buffer_rsrc(dF + (size_t)s * n * d, 0, (int)((size_t)n * d * sizeof(float)), 0x00020000);

    // ring to zero (finite stale values), dA block to LDS (zero beyond k and d)
    for (int e = tid * 4; e < BNST * BSTAGE; e += 512 * 4) *reinterpret_cast<f32x4 *>(&smem[e]) = f32x4{0, 0, 0, 0};
    const int kp = (k + 1) & ~1;
    batched_for<8>(
        tid, kp * 256, 512, [&](int e) { return G[(size_t)min(e >> 8, k - 1) * d + min(dbase + (e & 255), d - 1)]; },
        [&](int e, float g) {
            const int j = e >> 8, c = e & 255;
            sG[j * BLD + c] = (j < k && dbase + c < d) ? g : 0.f;
        });
    __syncthreads();

    const int npw = (BS * k + 255) / 256;  // 1 KB basis windows per stage
    auto issue = [&](int t) {
        float *S = smem + (t % BNST) * BSTAGE;
        const int v = vbeg + t * BS;
        const int rows = min(BS, vend - v);
        const int pvalid = rows * k;
#pragma unroll
        for (int q = 0; q < BFL; ++q) {
            const int item = q * 8 + wave;
            if (item < npw) {
                const int off = min(item * 256 + 4 * lane, ((pvalid + 3) & ~3) - 4);
                dma16(P + (size_t)v * k + off, S + item * 256);
            } else {
                const int off = min(4 * lane, ((rows + 3) & ~3) - 4);
                dma16(Mv + v + off, S + BP_TILE);
            }
        }
    };

    for (int t = 0; t < BNST - 1 && t < nst; ++t) issue(t);
    const int kh = (k + 1) >> 1;
    for (int t = 0; t < nst; ++t) {
        if (t + BNST - 1 < nst) issue(t + BNST - 1);
        // Memory operations issued after stage t's loads: the stores of stages t-2 and t-1 and the
        // loads of stages t+1 and t+2 (those that exist).  Waiting until at most that many are
        // outstanding retires stage t's loads (vmcnt is in issue order); counts above the 6-bit
        // counter range are clamped, which only waits longer.
        const int nl = min(2, nst - 1 - t), ns = min(2, t);
        switch (nl * 3 + ns) {
        case 0: wait_vmcnt<0>(); break;
        case 1: wait_vmcnt<BNS>(); break;
        case 2: wait_vmcnt<(2 * BNS < 63 ? 2 * BNS : 63)>(); break;
        case 3: wait_vmcnt<BFL>(); break;
        case 4: wait_vmcnt<BFL + BNS>(); break;
        case 5: wait_vmcnt<(BFL + 2 * BNS < 63 ? BFL + 2 * BNS : 63)>(); break;
        case 6: wait_vmcnt<2 * BFL>(); break;
        case 7: wait_vmcnt<2 * BFL + BNS>(); break;
        default: wait_vmcnt<(2 * BFL + 2 * BNS < 63 ? 2 * BFL + 2 * BNS : 63)>(); break;
        }
        lds_barrier();
        const float *S = smem + (t % BNST) * BSTAGE;
        const float *Ps = S, *Ms = S + BP_TILE;
        const int vs = vbeg + t * BS;
        const int vloc = 32 * rh + l32;
        const float m = (vs + vloc < vend) ? Ms[vloc] : 0.f;
        const float *prow = Ps + vloc * k + half;
        const float *g0 = sG + half * BLD + cg * 64 + l32;
        f32x16 acc0 = zero16(), acc1 = zero16();
        for (int tt = 0; tt < kh; ++tt) {
            const float a = (2 * tt + half < k) ? prow[2 * tt] * m : 0.f;
            const float *g = g0 + 2 * tt * BLD;
            acc0 = mfma32x32x2(a, g[0], acc0);
            acc1 = mfma32x32x2(a, g[32], acc1);
        }
        lds_barrier();  // slot t is refilled by the next iteration's issue
        // 32 unconditional stores per wave; rows past the end are dropped by the buffer range check
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int vr = vs + 32 * rh + acc32_row(r, lane);
            const int c0 = dbase + cg * 64 + l32;
            const bool rv = vr < vend;
            const unsigned o0 = (rv && c0 < d) ? (unsigned)((vr * d + c0) * 4) : 0x80000000u;
            const unsigned o1 = (rv && c0 + 32 < d) ? (unsigned)((vr * d + c0 + 32) * 4) : 0x80000000u;
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc0[r]), out, o0, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc1[r]), out, o1, 0, 0);
        }
    }
}

// A[s] = sum over chunks (in chunk order) of part[s][chunk].  Four consecutive
// elements per thread (k*d % 4 == 0, 16-byte aligned buffers); the chunks are
// read in groups of RG, all loads of a group in flight before the adds.
constexpr int RG = 8;

__global__ __launch_bounds__(256) void proj_reduce_kernel(const float *__restrict__ part, int nsplit, int64_t kd,
                                                          int64_t total, float *__restrict__ A)
{
    const int64_t q4 = kd / 4, tq = total / 4;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tq; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / q4, r = e - s * q4;
        const f32x4 *p = reinterpret_cast<const f32x4 *>(part + (size_t)s * nsplit * kd) + r;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int c0 = 0; c0 < nsplit; c0 += RG) {
            f32x4 v[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) v[u] = p[(size_t)min(c0 + u, nsplit - 1) * q4];
#pragma unroll
            for (int u = 0; u < RG; ++u)
                if (c0 + u < nsplit) acc += v[u];
        }
        reinterpret_cast<f32x4 *>(A)[e] = acc;
    }
}

// The same sum, one element per thread, for any k*d and alignment.
__global__ __launch_bounds__(256) void proj_reduce1_kernel(const float *__restrict__ part, int nsplit, int64_t kd,
                                                           int64_t total, float *__restrict__ A)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / kd, r = e - s * kd;
        const float *p = part + (size_t)s * nsplit * kd + r;
        float acc = 0.f;
        for (int c = 0; c < nsplit; ++c) acc += p[(size_t)c * kd];
        A[e] = acc;
    }
}

// Backward: one workgroup owns a column block of NT*32 feature columns and RB
// consecutive blocks of 128 vertices of one shape (32 per wave).  The rows
// [j0, j0+KC) of dA restricted to the column block are staged in LDS once per
// chunk (once per workgroup when k <= KC); matrix-core step t consumes basis
// columns j0 + 2t + half, so the two lane halves read adjacent LDS rows, which
// the padded row stride puts on disjoint banks.  Each lane's basis values are
// loaded for the whole chunk before the multiplies.
constexpr int BWD_KC = 64;

__host__ __device__ constexpr int bwd_stride(int nt) { return (nt * 32) % 64 == 32 ? nt * 32 : nt * 32 + 32; }

// RB consecutive blocks of 128 vertices starting at vertex r0 of one shape, for
// the column block [dbase, dbase + NT*32).  Must be called by all 256 threads.
template <typename T, int NT>
__device__ __forceinline__ void proj_bwd_rows(float *sG, const T *__restrict__ P, const float *__restrict__ Mv,
                                              const float *__restrict__ G, float *__restrict__ O, int n, int k, int d,
                                              int r0, int RB, int dbase)
{
    constexpr int LD = bwd_stride(NT);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    int cols[NT];
    bool cok[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        cols[nt] = dbase + nt * 32 + l32;
        cok[nt] = cols[nt] < d;
    }
    const int nchunks = (k + BWD_KC - 1) / BWD_KC;
    auto stage = [&](int j0, int kc) {
        const int kc2 = (kc + 1) & ~1;
        batched_for<8>(
            threadIdx.x, kc2 * NT * 32, 256,
            [&](int e) {
                const int jj = e / (NT * 32), cc = e - jj * (NT * 32);
                return G[(size_t)(j0 + min(jj, kc - 1)) * d + min(dbase + cc, d - 1)];
            },
            [&](int e, float g) {
                const int jj = e / (NT * 32), cc = e - jj * (NT * 32);
                sG[jj * LD + cc] = (jj < kc && dbase + cc < d) ? g : 0.f;
            });
    };
    __syncthreads();  // sG may still be read by a previous call
    if (nchunks == 1) {
        stage(0, k);
        __syncthreads();
    }
    for (int rb = 0; rb < RB; ++rb) {
        const int row0 = r0 + (rb * 4 + wave) * 32;
        const int row = row0 + l32;
        const bool rok = row < n;
        const float m = rok ? Mv[row] : 0.f;
        f32x16 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = zero16();
        for (int ch = 0; ch < nchunks; ++ch) {
            const int j0 = ch * BWD_KC;
            const int kc = min(BWD_KC, k - j0);
            if (nchunks > 1) {
                __syncthreads();
                stage(j0, kc);
                __syncthreads();
            }
            float a[BWD_KC / 2];
#pragma unroll
            for (int t = 0; t < BWD_KC / 2; ++t) {
                const int jj = 2 * t + half;
                a[t] = (rok && jj < kc) ? load_elem(P, (size_t)row * k + j0 + jj) * m : 0.f;
            }
            const int steps = (kc + 1) >> 1;
#pragma unroll
            for (int t = 0; t < BWD_KC / 2; ++t) {
                if (t < steps) {
                    const float *g = sG + (2 * t + half) * LD;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma32x32x2(a[t], g[nt * 32 + l32], acc[nt]);
                }
            }
        }
        if (row0 < n) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int rr = row0 + acc32_row(r, lane);
                    if (rr < n && cok[nt]) O[(size_t)rr * d + cols[nt]] = acc[nt][r];
                }
        }
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(256) void proj_bwd_kernel(const T *__restrict__ phi, const float *__restrict__ mass,
                                                       const float *__restrict__ dA, int n, int k, int d,
                                                       int rgroups, int RB, int dblocks, float *__restrict__ dF)
{
    extern __shared__ float sG[];  // [min(k,KC) rounded to even][bwd_stride(NT)]
    int bid = blockIdx.x;
    const int db = bid % dblocks;
    bid /= dblocks;
    const int rg = bid % rgroups;
    const int s = bid / rgroups;
    proj_bwd_rows<T, NT>(sG, phi + (size_t)s * n * k, mass + (size_t)s * n, dA + (size_t)s * k * d,
                         dF + (size_t)s * n * d, n, k, d, rg * RB * 128, RB, db * (NT * 32));
}

// Persistent backward over a table of work items (uneven shapes).
template <int NT>
__global__ __launch_bounds__(256) void proj_bwd_items_kernel(const BwdItem *__restrict__ items, int nitems)
{
    extern __shared__ float sG[];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BwdItem w = items[it];
        proj_bwd_rows<float, NT>(sG, global_ptr(w.phi), global_ptr(w.mass), global_ptr(w.dA), global_ptr(w.dF), w.n, w.k, w.d, w.r0, w.rb, w.dbase);
    }
}

// ---------------------------------------------------------------------------
// Host-side launch planning
// ---------------------------------------------------------------------------

static int device_cu_count()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

// Chunks of the LDS-pipelined forward: about one workgroup per CU overall.
static int lds_fwd_nsplit(int64_t batch, int64_t n, int64_t d)
{
    const int64_t dblocks = (d + 255) / 256;
    const int64_t stages = (n + FS - 1) / FS;
    int64_t ns = (device_cu_count() + batch * dblocks - 1) / (batch * dblocks);
    if (ns > stages / 4) ns = stages / 4;  // keep >= 4 stages per chunk
    if (ns < 1) ns = 1;
    return (int)ns;
}

ProjPlan plan_project(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t dtype)
{
    ProjPlan p;
    p.MT = k <= 32 ? 1 : 2;
    p.kblocks = (int)((k + 32 * p.MT - 1) / (32 * p.MT));
    // 4 waves per workgroup along d; NT 32-column tiles per wave.
    p.NT = d <= 128 ? 1 : 2;
    p.dblocks = (int)((d + 128 * p.NT - 1) / (128 * p.NT));
    // Split the vertex sum so that the grid has ~2 workgroups per CU, chunks of >= 512 vertices.
    const int64_t tiles = batch * p.kblocks * p.dblocks;
    int64_t want = (2 * device_cu_count() + tiles - 1) / tiles;
    int64_t maxsplit = (n + 511) / 512;
    int64_t ns = want < maxsplit ? want : maxsplit;
    if (ns < 1) ns = 1;
    int64_t chunk = (n + ns - 1) / ns;
    chunk = (chunk + 15) & ~(int64_t)15;
    ns = (n + chunk - 1) / chunk;
    p.nsplit = (int)ns;
    p.chunk = (int)chunk;
    (void)dtype;
    return p;
}

static bool lds_fwd_shape_ok(int64_t n, int64_t k, int64_t d, int32_t dtype)
{
    return dtype == 0 && k <= 64 && n % 4 == 0 && d % 4 == 0 && (n * k) % 4 == 0 && n >= 4 * FS;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

size_t project_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t dtype)
{
    ProjPlan p = plan_project(batch, n, k, d, dtype);
    int64_t ns = p.nsplit;
    if (lds_fwd_shape_ok(n, k, d, dtype)) {
        const int64_t nl = lds_fwd_nsplit(batch, n, d);
        if (nl > ns) ns = nl;
    }
    if (dtype == 1 && bf16_fwd_shape_ok(n, k, d)) {
        const int64_t nb = bf16_fwd_nsplit(batch, n, k, d);
        if (nb > ns) ns = nb;
    }
    if (dtype == 0 && f32_split_fwd_shape_ok(n, k, d)) {
        const int64_t nx = f32_split_fwd_nsplit(batch, n, k, d);
        if (nx > ns) ns = nx;
    }
    if (ns <= 1) return 0;
    return (size_t)batch * ns * k * d * sizeof(float);
}

template <int MT16, int REM>
static void launch_fwd_lds(const float *phi, const float *mass, const float *feat, int64_t batch, int64_t n,
                           int64_t k, int64_t d, int nsplit, float *out, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)proj_fwd_lds_kernel<MT16, REM>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)FWD_LDS_BYTES);
        attr_set = true;
    }
    const int dblocks = (int)((d + 255) / 256);
    const unsigned grid = (unsigned)(batch * nsplit * dblocks);
    hipLaunchKernelGGL((proj_fwd_lds_kernel<MT16, REM>), dim3(grid), dim3(512), FWD_LDS_BYTES, st, phi, mass, feat,
                       (int)n, (int)k, (int)d, nsplit, dblocks, out);
}

static void dispatch_fwd_lds(const float *phi, const float *mass, const float *feat, int64_t batch, int64_t n,
                             int64_t k, int64_t d, int nsplit, float *out, hipStream_t st)
{
    const int r = (int)(k % 16);
    if (k > 16 && r >= 1 && r <= 4) {
        const int mt = (int)(k / 16);
#define FMAP_FL(M, R) \
    if (mt == M && r == R) return launch_fwd_lds<M, R>(phi, mass, feat, batch, n, k, d, nsplit, out, st)
        FMAP_FL(1, 1); FMAP_FL(1, 2); FMAP_FL(1, 3); FMAP_FL(1, 4);
        FMAP_FL(2, 1); FMAP_FL(2, 2); FMAP_FL(2, 3); FMAP_FL(2, 4);
        FMAP_FL(3, 1); FMAP_FL(3, 2); FMAP_FL(3, 3); FMAP_FL(3, 4);
#undef FMAP_FL
    }
    switch ((k + 15) / 16) {
    case 1: return launch_fwd_lds<1, 0>(phi, mass, feat, batch, n, k, d, nsplit, out, st);
    case 2: return launch_fwd_lds<2, 0>(phi, mass, feat, batch, n, k, d, nsplit, out, st);
    case 3: return launch_fwd_lds<3, 0>(phi, mass, feat, batch, n, k, d, nsplit, out, st);
    default: return launch_fwd_lds<4, 0>(phi, mass, feat, batch, n, k, d, nsplit, out, st);
    }
}

template <typename T, int MT, int NT>
static void launch_fwd_t(const void *phi, const float *mass, const void *feat, int64_t batch, int64_t n, int64_t k,
                         int64_t d, const ProjPlan &p, float *out, hipStream_t st)
{
    const unsigned grid = (unsigned)(batch * p.nsplit * p.kblocks * p.dblocks);
    hipLaunchKernelGGL((proj_fwd_kernel<T, MT, NT, 8>), dim3(grid), dim3(256), 0, st, (const T *)phi, mass,
                       (const T *)feat, (int)n, (int)k, (int)d, p.nsplit, p.chunk, p.kblocks, p.dblocks, out);
}

template <typename T>
static void launch_fwd_dt(const void *phi, const float *mass, const void *feat, int64_t batch, int64_t n, int64_t k,
                          int64_t d, const ProjPlan &p, float *out, hipStream_t st)
{
    if (p.MT == 1 && p.NT == 1) launch_fwd_t<T, 1, 1>(phi, mass, feat, batch, n, k, d, p, out, st);
    else if (p.MT == 1) launch_fwd_t<T, 1, 2>(phi, mass, feat, batch, n, k, d, p, out, st);
    else if (p.NT == 1) launch_fwd_t<T, 2, 1>(phi, mass, feat, batch, n, k, d, p, out, st);
    else launch_fwd_t<T, 2, 2>(phi, mass, feat, batch, n, k, d, p, out, st);
}

// Per-shape reduction of partial slots (uneven shapes), fixed chunk order.
__global__ __launch_bounds__(256) void reduce_items_kernel(const RedItem *__restrict__ items, int nitems)
{
    for (int it = blockIdx.y; it < nitems; it += gridDim.y) {
        const RedItem w = items[it];
        for (int e = blockIdx.x * 256 + threadIdx.x; e < w.kd; e += gridDim.x * 256) {
            float acc = 0.f;
            for (int c = 0; c < w.nchunks; ++c) acc += w.part[(size_t)c * w.kd + e];
            w.A[e] = acc;
            if (w.A_user) w.A_user[e] = acc;
        }
    }
}

int device_cus() { return device_cu_count(); }

hipError_t launch_fwd_items(const FwdItem *items, int nitems, int kmax, int grid, hipStream_t st)
{
    if (kmax <= 32)
        hipLaunchKernelGGL((proj_fwd_items_kernel<1, 2, 8>), dim3(grid), dim3(256), 0, st, items, nitems);
    else
        hipLaunchKernelGGL((proj_fwd_items_kernel<2, 2, 8>), dim3(grid), dim3(256), 0, st, items, nitems);
    return hipGetLastError();
}

hipError_t launch_bwd_items(const BwdItem *items, int nitems, int kmax, int grid, hipStream_t st)
{
    const int kc = kmax < BWD_KC ? kmax : BWD_KC;
    const size_t lds = (size_t)((kc + 1) & ~1) * bwd_stride(8) * sizeof(float);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)proj_bwd_items_kernel<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(BWD_KC * bwd_stride(8) * sizeof(float)));
        attr_set = true;
    }
    hipLaunchKernelGGL((proj_bwd_items_kernel<8>), dim3(grid), dim3(256), lds, st, items, nitems);
    return hipGetLastError();
}

hipError_t launch_reduce_items(const RedItem *items, int nitems, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_items_kernel, dim3(16, (unsigned)(nitems < 65535 ? nitems : 65535)), dim3(256), 0, st,
                       items, nitems);
    return hipGetLastError();
}

hipError_t launch_reduce(const float *part, int nsplit, int64_t batch, int64_t k, int64_t d, float *A,
                                hipStream_t st)
{
    const int64_t total = batch * k * d;
    const bool vec = (k * d) % 4 == 0 && aligned16(part) && aligned16(A);
    int64_t blocks = ((vec ? total / 4 : total) + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(vec ? proj_reduce_kernel : proj_reduce1_kernel, dim3((unsigned)blocks), dim3(256), 0, st, part,
                       nsplit, (int64_t)(k * d), total, A);
    return hipGetLastError();
}

hipError_t launch_project(const void *phi, const float *mass, const void *feat, int32_t dtype, int64_t batch, int64_t n,
                          int64_t k, int64_t d, float *A, void *ws, hipStream_t st)
{
    if (dtype == 0 && f32_split_fwd_shape_ok(n, k, d) && aligned16(phi) && aligned16(mass) && aligned16(feat))
        return launch_project_f32_split((const float *)phi, mass, (const float *)feat, batch, n, k, d, A, ws, st);
    if (lds_fwd_shape_ok(n, k, d, dtype) && aligned16(phi) && aligned16(mass) && aligned16(feat)) {
        const int ns = lds_fwd_nsplit(batch, n, d);
        float *out = ns > 1 ? (float *)ws : A;
        dispatch_fwd_lds((const float *)phi, mass, (const float *)feat, batch, n, k, d, ns, out, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || ns <= 1) return e;
        return launch_reduce((const float *)ws, ns, batch, k, d, A, st);
    }
    if (dtype == 1 && bf16_fwd_shape_ok(n, k, d) && aligned16(phi) && aligned16(mass) && aligned16(feat))
        return launch_project_bf16((const uint16_t *)phi, mass, (const uint16_t *)feat, batch, n, k, d, A, ws, st);
    ProjPlan p = plan_project(batch, n, k, d, dtype);
    float *out = p.nsplit > 1 ? (float *)ws : A;
    if (dtype == 0) launch_fwd_dt<float>(phi, mass, feat, batch, n, k, d, p, out, st);
    else launch_fwd_dt<uint16_t>(phi, mass, feat, batch, n, k, d, p, out, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.nsplit <= 1) return e;
    return launch_reduce((const float *)ws, p.nsplit, batch, k, d, A, st);
}

template <typename T, int NT>
static void launch_bwd_t(const void *phi, const float *mass, const float *dA, int64_t batch, int64_t n, int64_t k,
                         int64_t d, float *dF, hipStream_t st)
{
    const int rblocks = (int)((n + 127) / 128);
    const int dblocks = (int)((d + NT * 32 - 1) / (NT * 32));
    // ~4 row blocks per workgroup, but keep >= ~1024 workgroups when the problem allows
    int RB = 4;
    while (RB > 1 && batch * dblocks * ((rblocks + RB - 1) / RB) < 1024) RB >>= 1;
    const int rgroups = (rblocks + RB - 1) / RB;
    const unsigned grid = (unsigned)(batch * rgroups * dblocks);
    const int kc = (int)(k < BWD_KC ? k : BWD_KC);
    const size_t lds = (size_t)((kc + 1) & ~1) * bwd_stride(NT) * sizeof(float);
    static bool attr_set = false;  // up to 64 x 288 floats (72 KB) for NT = 8
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)proj_bwd_kernel<T, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(BWD_KC * bwd_stride(NT) * sizeof(float)));
        attr_set = true;
    }
    hipLaunchKernelGGL((proj_bwd_kernel<T, NT>), dim3(grid), dim3(256), lds, st, (const T *)phi, mass, dA, (int)n,
                       (int)k, (int)d, rgroups, RB, dblocks, dF);
}

static bool lds_bwd_shape_ok(int64_t n, int64_t k, int64_t d, int32_t dtype)
{
    return dtype == 0 && k <= 64 && n % 4 == 0 && d % 4 == 0 && (n * k) % 4 == 0 && n >= 4 * BS &&
           (double)n * d * 4.0 < 2147483647.0;
}

static int lds_bwd_nsplit(int64_t batch, int64_t n, int64_t d)
{
    const int64_t dblocks = (d + 255) / 256;
    const int64_t stages = (n + BS - 1) / BS;
    int64_t ns = (device_cu_count() + batch * dblocks - 1) / (batch * dblocks);
    if (ns > stages / 3) ns = stages / 3;
    if (ns < 1) ns = 1;
    return (int)ns;
}

hipError_t launch_project_backward(const void *phi, const float *mass, int32_t dtype, const float *dA, int64_t batch,
                                   int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st)
{
    if (dtype == 0 && f32_split_bwd_shape_ok(n, k, d) && ((uintptr_t)phi & 7) == 0 && ((uintptr_t)dF & 15) == 0)
        return launch_project_backward_f32_split((const float *)phi, mass, dA, batch, n, k, d, dF, st);
    if (dtype == 0 && f32k_bwd_shape_ok(n, k, d) && ((uintptr_t)phi & 7) == 0 && ((uintptr_t)dF & 15) == 0)
        return launch_project_backward_f32k((const float *)phi, mass, dA, batch, n, k, d, dF, st);
    if (lds_bwd_shape_ok(n, k, d, dtype) && aligned16(phi) && aligned16(mass)) {
        static bool attr_set = false;
        if (!attr_set) {
            (void)hipFuncSetAttribute((const void *)proj_bwd_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)BWD_LDS_BYTES);
            attr_set = true;
        }
        const int ns = lds_bwd_nsplit(batch, n, d);
        const int dblocks = (int)((d + 255) / 256);
        hipLaunchKernelGGL(proj_bwd_lds_kernel, dim3((unsigned)(batch * ns * dblocks)), dim3(512), BWD_LDS_BYTES, st,
                           (const float *)phi, mass, dA, (int)n, (int)k, (int)d, ns, dblocks, dF);
        return hipGetLastError();
    }
    if (dtype == 1 && bf16_bwd_shape_ok(n, k, d) && aligned16(phi) && aligned16(dF))
        return launch_project_backward_bf16((const uint16_t *)phi, mass, dA, batch, n, k, d, dF, st);
    if (dtype == 0) {
        if (d <= 128) launch_bwd_t<float, 4>(phi, mass, dA, batch, n, k, d, dF, st);
        else launch_bwd_t<float, 8>(phi, mass, dA, batch, n, k, d, dF, st);
    } else {
        if (d <= 128) launch_bwd_t<uint16_t, 4>(phi, mass, dA, batch, n, k, d, dF, st);
        else launch_bwd_t<uint16_t, 8>(phi, mass, dA, batch, n, k, d, dF, st);
    }
    return hipGetLastError();
}

}  // namespace fmap

// Projections (Eq. 1 and its adjoint) on the bf16 matrix cores.
//
// Forward projection A = Phi^T diag(M) F with bfloat16 basis and
// features on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, float32
// accumulation).
//
// The contraction runs over vertices, and Phi [n][k] and F [n][d] are both
// vertex-major, so the 8 K slots (vertices) that one lane feeds a matrix-core
// step are a row apart in memory.  The operands are transposed in registers: a
// lane reads 4 consecutive entries of each of 8 vertex rows from LDS
// (ds_read_b64) and repacks them into 4 operands of 8 vertices each.
//   * basis side: each pair of vertices is packed by the float32 -> bf16
//     conversion of basis x mass (v_cvt_pk_bf16_f32 takes the two vertices), so
//     the transpose rides on the conversion;
//   * feature side: one v_perm_b32 per operand register.
// basis x mass is not a bf16 number: it is split into hi = bf16(p) and
// lo = bf16(p - hi) and both parts are multiplied (two matrix-core steps), so
// the products keep ~16 significant bits (relative error <= 2^-16) and the
// only roundings of substance are the bf16 inputs themselves.  A single bf16
// rounding of the product would add a relative error near 2^-8/sqrt(3) to A
// for incoherent data, as large as the whole error budget of this path.
//
// Workgroup = 4 waves = KW row slabs of 64 basis rows x (4/KW) column slabs of
// 128 feature columns; KW = 4 covers k <= 256 with one 128-column block of d,
// so the feature matrix is read exactly once and the basis once per column
// block.  The column blocks of one vertex chunk are given consecutive
// workgroup ids on the same XCD, so their basis reads meet in that XCD's L2.
// Stages of 32 vertices (one matrix-core K step) arrive by direct global->LDS
// loads in a ring of 3, two stages ahead; every wave issues a fixed number of
// loads per stage (addresses clamped, never masked) so the vmcnt waits are
// exact.  The vertex sum is split into chunks whose float32 partials are added
// in a fixed order by the reduction kernel of the float32 path.
#include "fmap_device.h"
#include "fmap_launch.h"
#include "fmap_lds.h"

namespace fmap {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int BS = 32;    // vertices per stage = K of one bf16 matrix-core step
constexpr int BNST = 3;   // stages in the ring

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const bf16x2_t v = __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t);  // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ f32x4 mfma16x16x32bf16(u32x4_t a, u32x4_t b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                     c, 0, 0, 0);
}

// bf16 number t (0..3) of a 64-bit group, as float32
__device__ __forceinline__ float bf16_at(uint2 x, int t)
{
    const uint32_t w = (t < 2) ? x.x : x.y;
    return __uint_as_float((t & 1) ? (w & 0xffff0000u) : (w << 16));
}

template <int KW>
struct Bf16Fwd {
    static constexpr int DWG = 128 * (4 / KW);   // feature columns per workgroup
    static constexpr int NF = DWG / 16;          // 1 KB feature windows per stage (32 rows x DWG bf16)
    static constexpr int FLB = KW == 1 ? 10 : 7; // loads per wave per stage (>= (NP + NF + 1) / 4)
    static constexpr int NPMAX = KW * 4;         // basis windows for k <= 64 KW
};

template <int KW>
__global__ __launch_bounds__(256, KW == 4 ? 2 : 1) void proj_fwd_bf16_kernel(const uint16_t *__restrict__ phi,
                                                            const float *__restrict__ mass,
                                                            const uint16_t *__restrict__ feat, int n, int k, int d,
                                                            int nsplit, int dblocks, int ntiles,
                                                            float *__restrict__ out)
{
    using C = Bf16Fwd<KW>;
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ks = wave % KW, dsl = wave / KW;
    const int m16 = lane & 15, g4 = lane >> 4;

    // workgroup id -> (tile j, column block db); XCD = id % 8, and the column blocks
    // of one tile take ids q*8 + x for consecutive q on the same XCD x
    const int bid = blockIdx.x;
    const int xs = bid & 7, q = bid >> 3;
    const int db = q % dblocks;
    const int j = (q / dblocks) * 8 + xs;
    if (j >= ntiles) return;  // whole workgroup, before any barrier
    const int split = j % nsplit, s = j / nsplit;
    const int dbase = db * C::DWG;

    const int nst_all = (n + BS - 1) / BS;
    const int st0 = (int)(((long)split * nst_all) / nsplit), st1 = (int)(((long)(split + 1) * nst_all) / nsplit);
    const int vbeg = st0 * BS, vend = min(n, st1 * BS);
    const int nst = st1 - st0;

    const uint16_t *P = phi + (size_t)s * n * k;
    const uint16_t *F = feat + (size_t)s * n * d;
    const float *Mv = mass + (size_t)s * n;

    const int np = (k + 15) / 16;  // 1 KB basis windows per stage (32 rows x k bf16)
    const int stage_bytes = (np + C::NF + 1) * 1024;
    char *ring = reinterpret_cast<char *>(smem);
    for (int e = tid * 16; e < BNST * stage_bytes; e += 256 * 16)
        *reinterpret_cast<f32x4 *>(ring + e) = f32x4{0, 0, 0, 0};
    __syncthreads();

    constexpr int LPR = C::DWG / 8;  // lanes per feature row in a window (16 B = 8 bf16 each)
    auto issue = [&](int t) {
        char *S = ring + (t % BNST) * stage_bytes;
        const int v = vbeg + t * BS;
        const int rows = min(BS, vend - v);
        const int pvalid = rows * k;  // basis entries of the stage that exist (multiple of 8)
#pragma unroll
        for (int qq = 0; qq < C::FLB; ++qq) {
            const int item = qq * 4 + wave;
            if (item < C::NF) {
                const int r = min(item * (64 / LPR) + lane / LPR, rows - 1);
                const int col = min(dbase + (lane % LPR) * 8, d - 8);
                dma16_stream(reinterpret_cast<const float *>(F + (size_t)(v + r) * d + col),
                             reinterpret_cast<float *>(S + np * 1024 + item * 1024));
            } else if (item < C::NF + np) {
                const int w = item - C::NF;
                const int off = min(w * 512 + 8 * lane, pvalid - 8);
                dma16(reinterpret_cast<const float *>(P + (size_t)v * k + off),
                      reinterpret_cast<float *>(S + w * 1024));
            } else {
                const int off = min(4 * lane, ((rows + 3) & ~3) - 4);
                dma16(Mv + v + off, reinterpret_cast<float *>(S + (np + C::NF) * 1024));
            }
        }
    };

    f32x4 acc[4][8];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = f32x4{0, 0, 0, 0};

    const int r4 = min(ks * 64 + 4 * m16, k - 4);  // rows beyond k read (and later drop) the last 4

    for (int t = 0; t < BNST - 1 && t < nst; ++t) issue(t);
    for (int t = 0; t < nst; ++t) {
        if (t + BNST - 1 < nst) issue(t + BNST - 1);
        if (t + 2 < nst) wait_vmcnt<2 * C::FLB>();
        else if (t + 1 < nst) wait_vmcnt<C::FLB>();
        else wait_vmcnt<0>();
        lds_barrier();
        const char *S = ring + (t % BNST) * stage_bytes;
        const uint16_t *Ps = reinterpret_cast<const uint16_t *>(S);
        const uint16_t *Fs = reinterpret_cast<const uint16_t *>(S + np * 1024);
        const float *Ms = reinterpret_cast<const float *>(S + (np + C::NF) * 1024);
        const int vrem = vend - (vbeg + t * BS);  // vertices of this stage that exist

        // masses of this lane's 8 vertices (zero past the end)
        const f32x4 m0 = *reinterpret_cast<const f32x4 *>(Ms + 8 * g4);
        const f32x4 m1 = *reinterpret_cast<const f32x4 *>(Ms + 8 * g4 + 4);
        float mv[8] = {m0[0], m0[1], m0[2], m0[3], m1[0], m1[1], m1[2], m1[3]};
#pragma unroll
        for (int i = 0; i < 8; ++i) mv[i] = (8 * g4 + i < vrem) ? mv[i] : 0.f;

        // feature operands: tile tt holds columns dsl*128 + 8*m16 + tt of vertices 8*g4..+7 (one 16-byte
        // LDS read per vertex row)
        u32x4_t B[8];
        {
            const int cb = dsl * 128 + 8 * m16;
            u32x4_t y[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) y[i] = *reinterpret_cast<const u32x4_t *>(Fs + (8 * g4 + i) * C::DWG + cb);
#pragma unroll
            for (int tt = 0; tt < 8; ++tt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    B[tt][jj] = __builtin_amdgcn_perm(y[2 * jj + 1][tt >> 1], y[2 * jj][tt >> 1],
                                                      (tt & 1) ? 0x07060302u : 0x05040100u);
        }
        // basis operands: rows r4..r4+3 x vertices 8*g4..8*g4+7, scaled by mass, as hi + lo.  Read as
        // 32-bit pairs: an 8-byte LDS read here (like the earlier 8-byte feature reads) made the compiler
        // wait for every outstanding global->LDS load, the prefetch two stages ahead included.
        uint2 x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t *pp = reinterpret_cast<const uint32_t *>(Ps + (8 * g4 + i) * k + r4);
            x[i].x = pp[0];
            x[i].y = pp[1];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            u32x4_t Ah, Al;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float p0 = bf16_at(x[2 * jj], a) * mv[2 * jj], p1 = bf16_at(x[2 * jj + 1], a) * mv[2 * jj + 1];
                const uint32_t hi = pack_bf16(p0, p1);
                Ah[jj] = hi;
                Al[jj] = pack_bf16(p0 - __uint_as_float(hi << 16), p1 - __uint_as_float(hi & 0xffff0000u));
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = mfma16x16x32bf16(Ah, B[b], acc[a][b]);
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = mfma16x16x32bf16(Al, B[b], acc[a][b]);
        }
        lds_barrier();  // the slot is refilled by the next iteration's issue
    }

    // D layout: lane (m16, g4), register r -> matrix-core row 4*g4 + r, column m16.
    // Row R of tile a is basis row ks*64 + 4R + a; column N of tile tt is
    // feature column dbase + dsl*128 + 8N + tt.
    float *O = out + (size_t)j * k * d;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ks * 64 + 4 * (4 * g4 + r) + a;
            if (row >= k) continue;
#pragma unroll
            for (int tt = 0; tt < 8; ++tt) {
                const int col = dbase + dsl * 128 + 8 * m16 + tt;
                if (col < d) O[(size_t)row * d + col] = acc[a][tt][r];
            }
        }
}

static int bf16_kw(int64_t k) { return k <= 64 ? 1 : (k <= 128 ? 2 : 4); }

bool bf16_fwd_shape_ok(int64_t n, int64_t k, int64_t d)
{
    return k >= 8 && k <= 256 && k % 8 == 0 && d >= 8 && d % 8 == 0 && n % 4 == 0 && n >= 4 * BS;
}

int bf16_fwd_nsplit(int64_t batch, int64_t n, int64_t k, int64_t d)
{
    const int kw = bf16_kw(k);
    const int64_t dblocks = (d + 128 * (4 / kw) - 1) / (128 * (4 / kw));
    const int64_t stages = (n + BS - 1) / BS;
    const int per_cu = kw == 1 ? 1 : 2;  // workgroups per CU that fit the LDS ring
    int64_t ns = (per_cu * device_cus()) / (batch * dblocks);
    if (ns > stages / 4) ns = stages / 4;  // keep >= 4 stages per chunk
    if (ns < 1) ns = 1;
    return (int)ns;
}

template <int KW>
static hipError_t dispatch_bf16(const uint16_t *phi, const float *mass, const uint16_t *feat, int64_t batch,
                                int64_t n, int64_t k, int64_t d, int ns, float *out, hipStream_t st)
{
    using C = Bf16Fwd<KW>;
    const int np = (int)((k + 15) / 16);
    const size_t lds = (size_t)BNST * (np + C::NF + 1) * 1024;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)proj_fwd_bf16_kernel<KW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)((size_t)BNST * (C::NPMAX + C::NF + 1) * 1024));
        attr_set = true;
    }
    const int dblocks = (int)((d + C::DWG - 1) / C::DWG);
    const int ntiles = (int)(batch * ns);
    const unsigned grid = (unsigned)(8 * dblocks * ((ntiles + 7) / 8));
    hipLaunchKernelGGL((proj_fwd_bf16_kernel<KW>), dim3(grid), dim3(256), lds, st, phi, mass, feat, (int)n, (int)k,
                       (int)d, ns, dblocks, ntiles, out);
    return hipGetLastError();
}

// Partials go to `ws` ([batch][nsplit][k][d]) when nsplit > 1, else straight to A.
hipError_t launch_project_bf16(const uint16_t *phi, const float *mass, const uint16_t *feat, int64_t batch, int64_t n,
                               int64_t k, int64_t d, float *A, void *ws, hipStream_t st)
{
    const int ns = bf16_fwd_nsplit(batch, n, k, d);
    float *out = ns > 1 ? (float *)ws : A;
    hipError_t e;
    switch (bf16_kw(k)) {
    case 1: e = dispatch_bf16<1>(phi, mass, feat, batch, n, k, d, ns, out, st); break;
    case 2: e = dispatch_bf16<2>(phi, mass, feat, batch, n, k, d, ns, out, st); break;
    default: e = dispatch_bf16<4>(phi, mass, feat, batch, n, k, d, ns, out, st); break;
    }
    if (e != hipSuccess || ns <= 1) return e;
    return launch_reduce(out, ns, batch, k, d, A, st);
}

// ---------------------------------------------------------------------------
// Backward projection dF = diag(M) Phi dA on the bf16 matrix cores, for a bf16
// basis (an exact operand) or a float32 basis.
//
// The float32 matrix rate of this GPU is 1/16 of its bf16 rate, so float32
// products are emulated: x = h + m + l with h, m, l bf16 (each the rounding of
// what is left), and the six products whose part indices sum to at most 2
// (hh, hm, mh, hl, lh, mm) are accumulated in float32.  The dropped terms are
// below 2^-24 relative, the float32 level; the six bf16 steps cost 6/16 of the
// matrix time of the float32 step.  With a bf16 basis, dA alone is split
// (hi + lo: 2^-16 relative).
//
// The contraction runs over k, contiguous in a basis row, so a lane's 8 K
// slots are one row segment of its vertex: one 16-byte load (bf16) or two
// (float32), no transpose.  dA^T is staged once per workgroup in LDS as its bf16
// parts in [column][k] layout, so each operand is one ds_read_b128.  The roles
// are chosen so that a lane ends up holding 4 consecutive columns of one vertex:
// the results leave as 16-byte stores, with the mass applied in float32.
//
// Workgroup = 8 waves, one 128-column block of d; a wave owns 32 vertices (2
// tiles of 16) x 128 columns (8 tiles).  Workgroups walk contiguous ranges of
// 256-vertex tiles (the staging is amortised over them), with the next tile's
// basis rows loaded during the current tile.  The column blocks of one vertex
// range take consecutive ids of one residue class mod 8 (one XCD), so the
// basis rows they share come from HBM once and from that XCD's L2 afterwards.
// ---------------------------------------------------------------------------
constexpr int BB_COLS = 128;   // columns per workgroup
constexpr int BB_VT = 256;     // vertices per workgroup tile (8 waves x 32)

__host__ __device__ constexpr int bwdmc_stride(int ks) { return ks * 64 + 16; }  // bytes per LDS row (k padded)
__host__ __device__ constexpr size_t bwdmc_parts(int pd, int ks) { return (size_t)pd * BB_COLS * bwdmc_stride(ks); }
// Store staging: a wave's 32 vertices x 32 columns (one M-tile pair) pass through LDS so that every
// store instruction writes whole 128-byte lines (8 vertices x 32 columns) instead of the matrix-core
// layout's 64-byte halves (16 vertices x 16 columns), which the memory system drains markedly slower.
// Rows of 36 floats (144 bytes) keep both the writes and the reads free of bank conflicts.
constexpr int BT_ROW = 36;
constexpr size_t BT_BYTES = 8 * 32 * BT_ROW * 4;
__host__ __device__ constexpr bool bwdmc_transpose(int pd, int ks) { return bwdmc_parts(pd, ks) + BT_BYTES <= 160 * 1024; }
__host__ __device__ constexpr size_t bwdmc_lds(int pd, int ks)
{
    return bwdmc_parts(pd, ks) + (bwdmc_transpose(pd, ks) ? BT_BYTES : 0);
}

// Streaming accesses (the `nt` cache policy): the feature rows read by the forward and the dF rows
// written by the backward are touched once, so they are kept from displacing the basis rows and the
// partial sums in L2 and the last-level cache, and the backward's writes go out while it runs instead of
// lingering as dirty lines that the next kernel has to write back.  In the full fwd + bwd step this took
// the forward projection from 130 to 89 us and the backward from 95 to 86 us at the headline shape.
__device__ __forceinline__ void stream_store(f32x4 *p, f32x4 v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void stream_store(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ f32x4 stream_load(const f32x4 *p) { return __builtin_nontemporal_load(p); }

// x (two values per dword) as NP bf16 parts, each the rounding of what the previous parts left
template <int NP>
__device__ __forceinline__ void split_pack(float x0, float x1, uint32_t *out)
{
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const uint32_t h = pack_bf16(x0, x1);
        out[p] = h;
        if (p + 1 < NP) {
            x0 -= __uint_as_float(h << 16);
            x1 -= __uint_as_float(h & 0xffff0000u);
        }
    }
}

template <typename T> struct RowSeg;  // 8 consecutive basis entries of one vertex row
template <> struct RowSeg<uint16_t> { u32x4_t v; };
template <> struct RowSeg<float> { f32x4 lo, hi; };

// Loads are unconditional, from addresses clamped into the row; slots past k are zeroed only when
// the operand is formed.  (A branch around each load, or a select right after it, would make the
// compiler wait for the loads at that point and so defeat the prefetch of the next tile.)
// bf16 rows: k % 8 == 0, so a lane's 8 slots starting at kk all exist or none do.
__device__ __forceinline__ RowSeg<uint16_t> load_seg_bf16(const uint16_t *row, int kk, int k)
{
    RowSeg<uint16_t> r;
    r.v = *reinterpret_cast<const u32x4_t *>(row + min(kk, k - 8));
    return r;
}
// float32 rows need only be 8-byte aligned (k even): four pairs
__device__ __forceinline__ RowSeg<float> load_seg_f32(const float *row, int kk, int k)
{
    RowSeg<float> r;
    float2 q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = *reinterpret_cast<const float2 *>(row + min(kk + 2 * i, k - 2));
    r.lo = f32x4{q[0].x, q[0].y, q[1].x, q[1].y};
    r.hi = f32x4{q[2].x, q[2].y, q[3].x, q[3].y};
    return r;
}

// the basis operand parts of one row segment starting at slot kk (slots >= k are zero)
template <int PP>
__device__ __forceinline__ void seg_parts(const RowSeg<uint16_t> &r, int kk, int k, u32x4_t *B)
{
    B[0] = (kk < k) ? r.v : u32x4_t{0, 0, 0, 0};
}
template <int PP>
__device__ __forceinline__ void seg_parts(const RowSeg<float> &r, int kk, int k, u32x4_t *B)
{
    const float x[8] = {r.lo[0], r.lo[1], r.lo[2], r.lo[3], r.hi[0], r.hi[1], r.hi[2], r.hi[3]};
    uint32_t w[4][PP];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool ok = kk + 2 * i < k;  // k even: both values of the pair exist or neither
        split_pack<PP>(ok ? x[2 * i] : 0.f, ok ? x[2 * i + 1] : 0.f, w[i]);
    }
#pragma unroll
    for (int p = 0; p < PP; ++p) B[p] = u32x4_t{w[0][p], w[1][p], w[2][p], w[3][p]};
}

// One workgroup's block: 256-vertex tiles [t0, t1) of one shape (basis P, masses Mv, G = dA, O = dF) for the
// columns [dbase, dbase + 128).
template <typename T, int PP, int PD, int KS>
__device__ __forceinline__ void bwdmc_block(const T *__restrict__ P, const float *__restrict__ Mv,
                                            const float *__restrict__ G, float *__restrict__ O, int n, int k, int d,
                                            int t0, int t1, int dbase)
{
    constexpr int STRIDE = bwdmc_stride(KS);
    constexpr bool TR = bwdmc_transpose(PD, KS);
    extern __shared__ __align__(16) float smem[];
    float *tstage = reinterpret_cast<float *>(reinterpret_cast<char *>(smem) + bwdmc_parts(PD, KS));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m16 = lane & 15, g4 = lane >> 4;

    // dA^T parts for columns [dbase, dbase + 128), rows < 32 KS (zero past k and d)
    char *parts = reinterpret_cast<char *>(smem);
    batched_for<8>(
        tid, KS * 32 * BB_COLS, 512,
        [&](int e) {
            const int jj = e / BB_COLS, c = e - jj * BB_COLS;
            return G[(size_t)min(jj, k - 1) * d + min(dbase + c, d - 1)];
        },
        [&](int e, float g) {
            const int jj = e / BB_COLS, c = e - jj * BB_COLS;
            const float v = (jj < k && dbase + c < d) ? g : 0.f;
            uint32_t w[PD];
            split_pack<PD>(v, 0.f, w);
#pragma unroll
            for (int p = 0; p < PD; ++p)
                *reinterpret_cast<uint16_t *>(parts + (size_t)p * BB_COLS * STRIDE + c * STRIDE + 2 * jj) =
                    (uint16_t)w[p];
        });
    __syncthreads();

    const bool vec = (d & 3) == 0;

    // basis row segments of a tile: [k step][vertex tile of 16]; rows past n are clamped (never stored)
    // raw row segments per buffer: 16 registers per k step (float32) or 8 (bf16)
    constexpr int NBUF = (KS * (PP == 1 ? 8 : 16) <= 36) ? 3 : 2;
    RowSeg<T> buf0[KS][2], buf1[KS][2], buf2[NBUF == 3 ? KS : 1][2];
    float m0[2], m1[2], m2[2];
    auto load_tile = [&](int vt, RowSeg<T> (&r)[KS][2], float (&mv)[2]) {
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int v = min(vt * BB_VT + wave * 32 + nt * 16 + m16, n - 1);
            mv[nt] = Mv[v];
            const T *row = P + (size_t)v * k;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if constexpr (PP == 1)
                    r[ks][nt] = load_seg_bf16(row, ks * 32 + 8 * g4, k);
                else
                    r[ks][nt] = load_seg_f32(row, ks * 32 + 8 * g4, k);
            }
        }
    };
    // Columns are produced 32 at a time (an M-tile pair) over all K steps, and stored right away, so
    // the stores of one pair drain while the next pair's products run.  The basis operand parts of
    // the whole tile are formed once.
    const bool fullcols = vec && dbase + BB_COLS <= d;  // the common case: no column checks
    auto compute_store = [&](int vt, const RowSeg<T> (&cur)[KS][2], const float (&mv)[2]) {
        u32x4_t B[KS][2][PP];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) seg_parts<PP>(cur[ks][nt], ks * 32 + 8 * g4, k, B[ks][nt]);
        const int vrow = vt * BB_VT + wave * 32 + m16;
#pragma unroll
        for (int mp = 0; mp < 8; mp += 2) {
            f32x4 acc[2][2];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) acc[h][nt] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                u32x4_t A[2][PD];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int p = 0; p < PD; ++p)
                        A[h][p] = *reinterpret_cast<const u32x4_t *>(parts + (size_t)p * BB_COLS * STRIDE +
                                                                    ((mp + h) * 16 + m16) * STRIDE +
                                                                    2 * (ks * 32 + 8 * g4));
                // four independent accumulators between dependent matrix-core steps
#pragma unroll
                for (int i = 0; i < PP; ++i)
#pragma unroll
                    for (int jp = 0; jp < PD; ++jp)
                        if (i + jp <= 2) {
#pragma unroll
                            for (int h = 0; h < 2; ++h)
#pragma unroll
                                for (int nt = 0; nt < 2; ++nt)
                                    acc[h][nt] = mfma16x16x32bf16(A[h][jp], B[ks][nt][i], acc[h][nt]);
                        }
            }
            // D layout: register r of lane (m16, g4) is column 4*g4 + r of the column tile, vertex m16
            if constexpr (TR) {
                if (fullcols) {
                    float *tw = tstage + wave * 32 * BT_ROW;
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            *reinterpret_cast<f32x4 *>(tw + (nt * 16 + m16) * BT_ROW + h * 16 + 4 * g4) =
                                acc[h][nt] * mv[nt];
                    // LDS operations of one wave complete in order: the reads see these writes, and the
                    // next pair's writes come after these reads
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int vr = 8 * u + (lane >> 3);
                        const f32x4 val = *reinterpret_cast<const f32x4 *>(tw + vr * BT_ROW + 4 * (lane & 7));
                        const int vb = vt * BB_VT + wave * 32 + vr;
                        if (vb < n)
                            stream_store(reinterpret_cast<f32x4 *>(O + (size_t)vb * d + dbase + mp * 16 + 4 * (lane & 7)), val);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    continue;
                }
            }
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int v = vrow + nt * 16;
                float *row = O + (size_t)min(v, n - 1) * d;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int col = dbase + (mp + h) * 16 + 4 * g4;
                    const f32x4 val = acc[h][nt] * mv[nt];
                    if (fullcols) {
                        if (v < n) stream_store(reinterpret_cast<f32x4 *>(row + col), val);
                    } else if (vec) {
                        if (v < n && col < d) stream_store(reinterpret_cast<f32x4 *>(row + col), val);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (v < n && col + r < d) stream_store(row + col + r, val[r]);
                    }
                }
            }
            // keep the scheduler from hoisting the next pair's LDS operands above these stores
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // The buffers rotate by unrolling (no register copies).  The prefetches are unconditional (the
    // last tile is loaded again at the end of the range): a conditional load would make the
    // compiler wait for all outstanding loads where the paths join.  With three buffers the loads
    // of tile t+2 are issued before the stores of tile t, so they do not queue behind its writes.
    // The loop runs whole rounds with no early exit and the last tiles follow it, and the prologue
    // loads keep their order: otherwise the compiler's wait analysis loses track of which loads a
    // tile needs and waits at the top of the loop for every outstanding load and store.
    if (t0 >= t1) return;
    if constexpr (NBUF == 3) {
        const int tfull = t0 + (t1 - t0) / 3 * 3;
        load_tile(t0, buf0, m0);
        __builtin_amdgcn_sched_barrier(0);
        load_tile(min(t0 + 1, t1 - 1), buf1, m1);
        __builtin_amdgcn_sched_barrier(0);
        for (int vt = t0; vt < tfull; vt += 3) {
            load_tile(min(vt + 2, t1 - 1), buf2, m2);
            compute_store(vt, buf0, m0);
            load_tile(min(vt + 3, t1 - 1), buf0, m0);
            compute_store(vt + 1, buf1, m1);
            load_tile(min(vt + 4, t1 - 1), buf1, m1);
            compute_store(vt + 2, buf2, m2);
        }
        if (tfull < t1) {  // tiles tfull (in buf0) and tfull + 1 (in buf1) are loaded
            compute_store(tfull, buf0, m0);
            if (tfull + 1 < t1) compute_store(tfull + 1, buf1, m1);
        }
    } else if constexpr (KS < 8) {
        // (a tail after the loop makes these instances spill: the last round is predicated instead)
        load_tile(t0, buf0, m0);
        __builtin_amdgcn_sched_barrier(0);
        for (int vt = t0; vt < t1; vt += 2) {
            load_tile(min(vt + 1, t1 - 1), buf1, m1);
            compute_store(vt, buf0, m0);
            load_tile(min(vt + 2, t1 - 1), buf0, m0);
            if (vt + 1 < t1) compute_store(vt + 1, buf1, m1);
        }
    } else {
        // at KS = 8 only the loop with an early exit fits the register file (it keeps the wait for
        // every outstanding load at the top of each round)
        load_tile(t0, buf0, m0);
        for (int vt = t0; vt < t1; vt += 2) {
            load_tile(min(vt + 1, t1 - 1), buf1, m1);
            compute_store(vt, buf0, m0);
            if (vt + 1 >= t1) break;
            load_tile(min(vt + 2, t1 - 1), buf0, m0);
            compute_store(vt + 1, buf1, m1);
        }
    }
}

template <typename T, int PP, int PD, int KS>
__global__ __launch_bounds__(512, 2) void proj_bwd_mc_kernel(const T *__restrict__ phi, const float *__restrict__ mass,
                                                           const float *__restrict__ dA, int n, int k, int d,
                                                           int vsplit, int dblocks, int ntasks,
                                                           float *__restrict__ dF)
{
    const int bid = blockIdx.x;
    const int xs = bid & 7, q = bid >> 3;
    const int db = q % dblocks;
    const int j = (q / dblocks) * 8 + xs;
    if (j >= ntasks) return;  // whole workgroup, before any barrier
    const int vs = j % vsplit, s = j / vsplit;
    const int ntile = (n + BB_VT - 1) / BB_VT;
    const int t0 = (int)(((long)vs * ntile) / vsplit), t1 = (int)(((long)(vs + 1) * ntile) / vsplit);
    bwdmc_block<T, PP, PD, KS>(phi + (size_t)s * n * k, mass + (size_t)s * n, dA + (size_t)s * k * d,
                               dF + (size_t)s * n * d, n, k, d, t0, t1, db * BB_COLS);
}

// Uneven batches: one workgroup per work item (float32 basis).
template <int KS>
__global__ __launch_bounds__(512, 2) void proj_bwd_mc_items_kernel(const McItem *__restrict__ items)
{
    const McItem w = items[blockIdx.x];
    if (w.t0 >= w.t1) return;  // empty slot of the table (whole workgroup, before any barrier)
    bwdmc_block<float, 3, 3, KS>(global_ptr(w.phi), global_ptr(w.mass), global_ptr(w.dA), global_ptr(w.dF), w.n, w.k, w.d, w.t0, w.t1, w.dbase);
}

// ---------------------------------------------------------------------------
// Backward projection for float32 inputs with 64 < k <= kMaxK (k even), on the
// bf16 matrix cores with both operands split into three parts (six products).
//
// The dA^T parts of every k slot would not fit in LDS for 128 columns, so a
// workgroup owns a 64-column block: 3 parts x 64 columns x (32 KS + 8) bf16
// pairs, up to 126 KB, staged once.  8 waves x 32 vertices form a 256-vertex
// tile.  A wave's work is a flat sequence of steps (tile, K step); the basis
// row segments of step s + 3 are loaded while step s is multiplied (four
// register buffers rotated by unrolling, loads unconditional from clamped
// addresses), so the basis stream never waits for a tile boundary.  The 4 x 2
// accumulators of a tile are stored, scaled by the masses, after its last K
// step, exchanged across lanes first so that each store writes whole 128-byte
// lines.  The column blocks of one vertex range share an XCD (their basis rows
// are read from HBM once and from L2 afterwards).
// ---------------------------------------------------------------------------
constexpr int BK_COLS = 64;  // columns per workgroup
__host__ __device__ constexpr size_t bwdk_lds(int ks) { return (size_t)3 * BK_COLS * bwdmc_stride(ks); }

struct BkStep {
    RowSeg<float> seg[2];  // vertex tiles nt = 0, 1
    float m[2];            // their masses
};

// One workgroup's block: 256-vertex tiles [t0, t1) of one shape for the columns [dbase, dbase + 64).
// SHALLOW: loads one step ahead instead of three (two step buffers), for instances that run two
// workgroups per CU, where the other workgroup covers the load latency.
template <int KS, bool SHALLOW = false>
__device__ __forceinline__ void bwdk_block(const float *__restrict__ P, const float *__restrict__ Mv,
                                           const float *__restrict__ G, float *__restrict__ O, int n, int k, int d,
                                           int t0, int t1, int dbase)
{
    constexpr int STRIDE = bwdmc_stride(KS);
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m16 = lane & 15, g4 = lane >> 4;

    // dA^T parts for columns [dbase, dbase + 64), slots < 32 KS (zero past k and d)
    char *parts = reinterpret_cast<char *>(smem);
    batched_for<8>(
        tid, KS * 32 * BK_COLS, 512,
        [&](int e) {
            const int jj = e / BK_COLS, c = e - jj * BK_COLS;
            return G[(size_t)min(jj, k - 1) * d + min(dbase + c, d - 1)];
        },
        [&](int e, float g) {
            const int jj = e / BK_COLS, c = e - jj * BK_COLS;
            const float v = (jj < k && dbase + c < d) ? g : 0.f;
            uint32_t w[3];
            split_pack<3>(v, 0.f, w);
#pragma unroll
            for (int p = 0; p < 3; ++p)
                *reinterpret_cast<uint16_t *>(parts + (size_t)p * BK_COLS * STRIDE + c * STRIDE + 2 * jj) =
                    (uint16_t)w[p];
        });
    __syncthreads();

    if (t0 >= t1) return;
    const int nsteps = (t1 - t0) * KS;
    const bool vec = (d & 3) == 0;

    auto load_step = [&](int st, BkStep &b) {
        const int vt = t0 + st / KS, ks = st % KS;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int v = min(vt * BB_VT + wave * 32 + nt * 16 + m16, n - 1);
            b.m[nt] = Mv[v];
            b.seg[nt] = load_seg_f32(P + (size_t)v * k, ks * 32 + 8 * g4, k);
        }
    };
    f32x4 acc[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f32x4{0, 0, 0, 0};
    auto step = [&](int st, const BkStep &b) {
        const int vt = t0 + st / KS, ks = st % KS;
        u32x4_t B[2][3];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) seg_parts<3>(b.seg[nt], ks * 32 + 8 * g4, k, B[nt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            u32x4_t A[3];
#pragma unroll
            for (int p = 0; p < 3; ++p)
                A[p] = *reinterpret_cast<const u32x4_t *>(parts + (size_t)p * BK_COLS * STRIDE + (mt * 16 + m16) * STRIDE +
                                                         2 * (ks * 32 + 8 * g4));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int jp = 0; jp < 3; ++jp)
                    if (i + jp <= 2) {
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = mfma16x16x32bf16(A[jp], B[nt][i], acc[mt][nt]);
                    }
        }
        if (ks == KS - 1) {  // the tile is complete: register r of lane (m16, g4) is column 4 g4 + r of tile mt
            if (vec) {
                // whole 128-byte lines: the accumulators are exchanged across lanes (ds_bpermute, no LDS
                // allocation) so that one store covers 8 vertices x 32 columns, lane L taking vertex L / 8
                // (+ 8 i) and columns 4 (L % 8) .. + 3 of the half block hh; the values and the mass product
                // are those of the lane that computed them
                const int c4 = lane & 7;
                const bool upper = (c4 >> 2) != 0;  // tile 2 hh + 1
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const int vr = 8 * i + (lane >> 3);  // vertex within the 16 of nt
                        const int src = 4 * (vr + 16 * (c4 & 3));
                        const int v = vt * BB_VT + wave * 32 + nt * 16 + vr;
                        const float m = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(b.m[nt])));
                        float *row = O + (size_t)min(v, n - 1) * d;
#pragma unroll
                        for (int hh = 0; hh < 2; ++hh) {
                            f32x4 val;
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const float lo = __int_as_float(
                                    __builtin_amdgcn_ds_bpermute(src, __float_as_int(acc[2 * hh][nt][r])));
                                const float hi = __int_as_float(
                                    __builtin_amdgcn_ds_bpermute(src, __float_as_int(acc[2 * hh + 1][nt][r])));
                                val[r] = (upper ? hi : lo) * m;
                            }
                            const int col = dbase + 32 * hh + 4 * c4;
                            if (v < n && col < d) stream_store(reinterpret_cast<f32x4 *>(row + col), val);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const int v = vt * BB_VT + wave * 32 + nt * 16 + m16;
                    float *row = O + (size_t)min(v, n - 1) * d;
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) {
                        const int col = dbase + mt * 16 + 4 * g4;
                        const f32x4 val = acc[mt][nt] * b.m[nt];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (v < n && col + r < d) stream_store(row + col + r, val[r]);
                    }
                }
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f32x4{0, 0, 0, 0};
        }
    };
    const int last = nsteps - 1;
    if constexpr (SHALLOW) {
        BkStep b0, b1;
        load_step(0, b0);
        __builtin_amdgcn_sched_barrier(0);
        for (int st = 0; st < nsteps; st += 2) {
            load_step(min(st + 1, last), b1);
            step(st, b0);
            load_step(min(st + 2, last), b0);
            if (st + 1 < nsteps) step(st + 1, b1);
        }
        return;
    }
    BkStep b0, b1, b2, b3;
    // rounds of four with no early exit (the last round predicated), as in the backward above
    load_step(0, b0);
    __builtin_amdgcn_sched_barrier(0);
    load_step(min(1, last), b1);
    __builtin_amdgcn_sched_barrier(0);
    load_step(min(2, last), b2);
    __builtin_amdgcn_sched_barrier(0);
    for (int st = 0; st < nsteps; st += 4) {
        load_step(min(st + 3, last), b3);
        step(st, b0);
        load_step(min(st + 4, last), b0);
        if (st + 1 < nsteps) step(st + 1, b1);
        load_step(min(st + 5, last), b1);
        if (st + 2 < nsteps) step(st + 2, b2);
        load_step(min(st + 6, last), b2);
        if (st + 3 < nsteps) step(st + 3, b3);
    }
}

template <int KS>
__global__ __launch_bounds__(512, 1) void proj_bwd_mck_kernel(const float *__restrict__ phi,
                                                            const float *__restrict__ mass,
                                                            const float *__restrict__ dA, int n, int k, int d,
                                                            int vsplit, int dblocks, int ntasks,
                                                            float *__restrict__ dF)
{
    const int bid = blockIdx.x;
    const int xs = bid & 7, q = bid >> 3;
    const int db = q % dblocks;
    const int j = (q / dblocks) * 8 + xs;
    if (j >= ntasks) return;  // whole workgroup, before any barrier
    const int vs = j % vsplit, s = j / vsplit;
    const int ntile = (n + BB_VT - 1) / BB_VT;
    const int t0 = (int)(((long)vs * ntile) / vsplit), t1 = (int)(((long)(vs + 1) * ntile) / vsplit);
    bwdk_block<KS>(phi + (size_t)s * n * k, mass + (size_t)s * n, dA + (size_t)s * k * d, dF + (size_t)s * n * d, n,
                   k, d, t0, t1, db * BK_COLS);
}

// Uneven batches: one workgroup per work item.
// KS <= 5: the dA^T parts take at most 66 KB of LDS, so with the shallow pipeline (<= 128 VGPRs) two
// workgroups share a CU.
template <int KS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(KS <= 5 ? 4 : 1))) void
proj_bwd_mck_items_kernel(const McItem *__restrict__ items)
{
    const McItem w = items[blockIdx.x];
    if (w.t0 >= w.t1) return;  // empty slot of the table (whole workgroup, before any barrier)
    bwdk_block<KS, (KS <= 5)>(global_ptr(w.phi), global_ptr(w.mass), global_ptr(w.dA), global_ptr(w.dF), w.n, w.k, w.d, w.t0, w.t1, w.dbase);
}

constexpr int XS = 32;  // vertices per stage (one matrix-core K step)

__host__ __device__ constexpr int x3_np(int k) { return (k + 7) / 8; }  // 1 KB basis windows (32 rows x k floats)

// ---------------------------------------------------------------------------
// Forward projection with float32 basis and features on the bf16 matrix cores:
// both operands split into three bf16 parts, six products kept (float32 level,
// as in the backward above).  Features through registers, basis x mass split
// once per workgroup.
//
// Workgroup = 4 waves over a 256-column block and 64 (padded) basis rows: all
// of them for k <= 64 (k even), or, SLICED (k > 64, k % 4 == 0), the slice
// [64 kb, 64 kb + 64), each stage then holding that 64-float slice of every
// vertex row (8 windows of 4 vertices).  The row blocks and column blocks of
// one vertex chunk take consecutive ids on one XCD, so the feature tile they
// all read comes from HBM once and from that XCD's L2 afterwards.  Within a block:
// wave w owns block columns 64w .. 64w + 63 (column 4m + t of the wave is
// column m of tile t).  Stages of 32 vertices.  Each lane loads its 4 feature
// columns of 8 vertices straight into registers (eight 16-byte loads), two
// stages ahead, so the feature stream -- nearly all of the bytes -- needs no
// LDS, no barrier and no LDS round trip.  The small basis tile (32 x k floats)
// and the masses arrive by direct global->LDS loads in a ring of 3.  Per stage
// wave w splits the basis x mass values of row tile w (rows 4R + w) into their
// three bf16 parts and stores them in LDS in the matrix-core operand layout;
// after a barrier every wave reads all four tiles.  The split work per wave is
// then a quarter of the basis tile plus its own features, below the
// matrix-core time of its 96 products.
// ---------------------------------------------------------------------------
constexpr int RNST = 3;  // basis stages in the LDS ring
constexpr int RFL = 3;   // direct loads per wave per stage: 2 basis windows, 1 mass window
constexpr int RFF = 8;   // feature loads per lane per stage
constexpr int RSTAGE = 8 * 1024 + 256;  // basis windows + mass window
constexpr int RPARTS = 3 * 4 * 64 * 16;  // split basis tile: [part][row tile][lane] of u32x4
__host__ __device__ constexpr size_t x3r_lds() { return (size_t)RNST * RSTAGE + RPARTS; }

// One workgroup's block: vertices [vbeg, vend) of one shape (P, Mv, F), basis rows [64 kb, 64 kb + 64)
// (all rows unless SLICED), columns [dbase, dbase + 256); the k x d partial slot O receives its part.
// vbeg is a multiple of 32, and every stage but the last is full.
template <bool SLICED>
__device__ __forceinline__ void x3r_block(const float *__restrict__ P, const float *__restrict__ Mv,
                                          const float *__restrict__ F, int n, int k, int d, int vbeg, int vend,
                                          int kb, int dbase, float *__restrict__ O)
{
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m16 = lane & 15, g4 = lane >> 4;
    const int kbase = SLICED ? 64 * kb : 0;
    const int kvalid = SLICED ? min(64, k - kbase) : k;  // basis rows of this block
    const int pstride = SLICED ? 64 : k;                 // LDS floats per vertex row of the basis tile
    const int nst = (vend - vbeg + XS - 1) / XS;

    const int np = SLICED ? 8 : x3_np(k);
    char *ring = reinterpret_cast<char *>(smem);
    u32x4_t *parts = reinterpret_cast<u32x4_t *>(ring + RNST * RSTAGE);
    for (int e = tid * 16; e < RNST * RSTAGE; e += 256 * 16) *reinterpret_cast<f32x4 *>(ring + e) = f32x4{0, 0, 0, 0};
    __syncthreads();

    // basis roles: windows wave and wave + 4 (clamped to the last), the mass window.  A window is
    // 256 contiguous floats of the 32 x k tile or, sliced, vertices 4w .. 4w + 3 of the slice with
    // lane l taking the 4 floats at column 64 kb + 4 (l % 16) (clamped to k - 4) of vertex 4w + l/16
    const int pw0 = min(wave, np - 1), pw1 = min(wave + 4, np - 1);
    const int scol = min(kbase + 4 * (lane & 15), k - 4);
    const int poff0 = min(pw0 * 256 + 4 * lane, XS * k - 4), poff1 = min(pw1 * 256 + 4 * lane, XS * k - 4);
    // feature role: columns fc .. fc + 3 (clamped into d; d % 4 == 0) of vertices 8 g4 .. + 7
    const int cw = wave * 64 + 4 * m16;
    const int fc = min(dbase + cw, d - 4);
    auto issue = [&](int t, f32x4 (&fr)[RFF]) {
        char *S = ring + (t % RNST) * RSTAGE;
        const int v = vbeg + t * XS;
        const int rows = min(XS, vend - v);  // a multiple of 4 (n % 4 == 0)
        const float *Pv = P + (size_t)v * k;
        if (SLICED) {  // vertices past the stage's rows read the last row
            const int r0 = min(4 * pw0 + (lane >> 4), rows - 1), r1 = min(4 * pw1 + (lane >> 4), rows - 1);
            dma16(Pv + (size_t)r0 * k + scol, reinterpret_cast<float *>(S + pw0 * 1024));
            dma16(Pv + (size_t)r1 * k + scol, reinterpret_cast<float *>(S + pw1 * 1024));
        } else {
            const int pv = rows * k - 4;
            dma16(Pv + min(poff0, pv), reinterpret_cast<float *>(S + pw0 * 1024));
            dma16(Pv + min(poff1, pv), reinterpret_cast<float *>(S + pw1 * 1024));
        }
        __builtin_amdgcn_global_load_lds((glb_void_t *)(Mv + v + min(lane & 31, rows - 1)),
                                         (lds_void_t *)(S + 8 * 1024), 4, 0, 0);
        // (sliced, the row blocks of a chunk re-read the same features from L2: ordinary loads there)
#pragma unroll
        for (int i = 0; i < RFF; ++i) {
            const f32x4 *fp = reinterpret_cast<const f32x4 *>(F + (size_t)(v + min(8 * g4 + i, rows - 1)) * d + fc);
            fr[i] = SLICED ? *fp : stream_load(fp);
        }
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[a][t] = f32x4{0, 0, 0, 0};
    // split role: row tile a = wave, operand lane = lane: basis row 4 m16 + wave, vertices 8 g4 .. + 7
    const int srow = 4 * m16 + wave;
    const bool srow_ok = srow < kvalid;
    const int srow_c = min(srow, kvalid - 1);

    auto stage = [&](int t, const f32x4 (&fr)[RFF]) {
        const char *S = ring + (t % RNST) * RSTAGE;
        const float *Ps = reinterpret_cast<const float *>(S);
        const float *Ms = reinterpret_cast<const float *>(S + 8 * 1024);
        const int vrem = vend - (vbeg + t * XS);
        {
            const f32x4 m0 = *reinterpret_cast<const f32x4 *>(Ms + 8 * g4);
            const f32x4 m1 = *reinterpret_cast<const f32x4 *>(Ms + 8 * g4 + 4);
            const float mv[8] = {m0[0], m0[1], m0[2], m0[3], m1[0], m1[1], m1[2], m1[3]};
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                // the mass is masked, not the product, so the LDS reads are unconditional and issued together
                const float pv = Ps[(8 * g4 + i) * pstride + srow_c];
                x[i] = pv * ((srow_ok && 8 * g4 + i < vrem) ? mv[i] : 0.f);
            }
            uint32_t w[4][3];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) split_pack<3>(x[2 * jj], x[2 * jj + 1], w[jj]);
#pragma unroll
            for (int p = 0; p < 3; ++p) parts[(p * 4 + wave) * 64 + lane] = u32x4_t{w[0][p], w[1][p], w[2][p], w[3][p]};
        }
        lds_barrier();
        u32x4_t A[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int p = 0; p < 3; ++p) A[a][p] = parts[(p * 4 + a) * 64 + lane];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            u32x4_t B[3];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                uint32_t w[3];
                split_pack<3>(fr[2 * jj][tt], fr[2 * jj + 1][tt], w);
#pragma unroll
                for (int p = 0; p < 3; ++p) B[p][jj] = w[p];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int jp = 0; jp < 3; ++jp)
                    if (i + jp <= 2) {
#pragma unroll
                        for (int a = 0; a < 4; ++a) acc[a][tt] = mfma16x16x32bf16(A[a][i], B[jp], acc[a][tt]);
                    }
        }
    };

    // Per stage t: wait for stage t (stage t + 1 may stay in flight), barrier (stage t visible;
    // every wave done with stage t - 1, so its ring slot, the split buffer and its feature registers
    // are free), issue stage t + 2 into them, split, barrier, products.  The three feature buffers
    // rotate by unrolling; prefetches past the chunk reload its last stage (the same bytes into the
    // same places), and every load has landed before the workgroup ends (its LDS is then reused).
    // The loop runs whole triples and has no early exit, the last one or two stages follow it: an exit
    // edge back into the loop header, or prologue loads reordered across the two stages, leaves the
    // compiler's wait analysis unable to tell which loads stage t needs, and it then waits for all of
    // them, the stage t + 2 prefetch included.
    f32x4 f0[RFF], f1[RFF], f2[RFF];
    constexpr int VPS = RFL + RFF;  // vector-memory operations per stage
    if (nst <= 0) return;
    issue(0, f0);
    __builtin_amdgcn_sched_barrier(0);
    issue(min(1, nst - 1), f1);
    __builtin_amdgcn_sched_barrier(0);
    const int nfull = nst - nst % 3;
    for (int t = 0; t < nfull; t += 3) {
        wait_vmcnt<VPS>();
        lds_barrier();
        issue(min(t + 2, nst - 1), f2);
        stage(t, f0);
        wait_vmcnt<VPS>();
        lds_barrier();
        issue(min(t + 3, nst - 1), f0);
        stage(t + 1, f1);
        wait_vmcnt<VPS>();
        lds_barrier();
        issue(min(t + 4, nst - 1), f1);
        stage(t + 2, f2);
    }
    if (nst % 3 != 0) {  // stages nfull (in f0) and nfull + 1 (in f1) are issued
        wait_vmcnt<VPS>();
        lds_barrier();
        stage(nfull, f0);
        if (nst % 3 == 2) {
            wait_vmcnt<0>();
            lds_barrier();
            stage(nfull + 1, f1);
        }
    }
    wait_vmcnt<0>();

    // lane (m16, g4), register r: matrix-core row 4*g4 + r -> basis row 4(4*g4 + r) + a; column m16 of
    // tile tt -> block column 64 wave + 4 m16 + tt
    const int col = dbase + cw;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int row = kbase + 16 * g4 + 4 * r + a;
            if (row >= k || col >= d) continue;
            const f32x4 v = f32x4{acc[a][0][r], acc[a][1][r], acc[a][2][r], acc[a][3][r]};
            *reinterpret_cast<f32x4 *>(O + (size_t)row * d + col) = v;  // d % 4 == 0: all 4 columns exist
        }
}

template <bool SLICED>
__global__ __launch_bounds__(256, 2) void proj_fwd_x3r_kernel(const float *__restrict__ phi,
                                                             const float *__restrict__ mass,
                                                             const float *__restrict__ feat, int n, int k, int d,
                                                             int nsplit, int dblocks, int kblocks, int ntiles,
                                                             float *__restrict__ out)
{
    const int bid = blockIdx.x;
    const int xs = bid & 7, q = bid >> 3;
    const int dk = dblocks * kblocks;
    const int db = (q % dk) % dblocks, kb = (q % dk) / dblocks;
    const int j = (q / dk) * 8 + xs;
    if (j >= ntiles) return;  // whole workgroup, before any barrier
    const int split = j % nsplit, s = j / nsplit;
    const int nst_all = (n + XS - 1) / XS;
    const int st0 = (int)(((long)split * nst_all) / nsplit), st1 = (int)(((long)(split + 1) * nst_all) / nsplit);
    x3r_block<SLICED>(phi + (size_t)s * n * k, mass + (size_t)s * n, feat + (size_t)s * n * d, n, k, d, st0 * XS,
                      min(n, st1 * XS), kb, db * 256, out + (size_t)j * k * d);
}

// Uneven batches: one workgroup per work item (items of whole 32-vertex stages only).
template <bool SLICED>
__global__ __launch_bounds__(256, 2) void proj_fwd_x3r_items_kernel(const FwdItem *__restrict__ items)
{
    const FwdItem w = items[blockIdx.x];
    if (w.v0 >= w.v1) return;  // empty slot of the table (whole workgroup, before any barrier)
    x3r_block<SLICED>(global_ptr(w.phi), global_ptr(w.mass), global_ptr(w.feat), w.n, w.k, w.d, w.v0, w.v1, w.kbase / 64,
                      w.dbase, global_ptr(w.out));
}

bool f32_split_fwd_shape_ok(int64_t n, int64_t k, int64_t d)
{
    const bool kok = (k >= 4 && k <= 64 && k % 2 == 0) || (k > 64 && k <= kMaxK && k % 4 == 0);
    return kok && d % 4 == 0 && n % 4 == 0 && n >= 4 * XS;
}

static int x3_kblocks(int64_t k) { return k <= 64 ? 1 : (int)((k + 63) / 64); }

int f32_split_fwd_nsplit(int64_t batch, int64_t n, int64_t k, int64_t d)
{
    const int64_t blocks = (d + 255) / 256 * x3_kblocks(k);
    const int64_t stages = (n + XS - 1) / XS;
    int64_t ns = (2 * device_cus()) / (batch * blocks);  // two workgroups per CU
    if (ns > stages / 4) ns = stages / 4;               // keep >= 4 stages per chunk
    if (ns < 1) ns = 1;
    return (int)ns;
}

template <bool SLICED>
static hipError_t dispatch_x3r(const float *phi, const float *mass, const float *feat, int64_t batch, int64_t n,
                               int64_t k, int64_t d, int ns, float *out, hipStream_t st)
{
    const int dblocks = (int)((d + 255) / 256);
    const int kblocks = x3_kblocks(k);
    const int ntiles = (int)(batch * ns);
    const unsigned grid = (unsigned)(8 * dblocks * kblocks * ((ntiles + 7) / 8));
    hipLaunchKernelGGL((proj_fwd_x3r_kernel<SLICED>), dim3(grid), dim3(256), x3r_lds(), st, phi, mass, feat, (int)n,
                       (int)k, (int)d, ns, dblocks, kblocks, ntiles, out);
    return hipGetLastError();
}

hipError_t launch_project_f32_split(const float *phi, const float *mass, const float *feat, int64_t batch, int64_t n,
                                    int64_t k, int64_t d, float *A, void *ws, hipStream_t st)
{
    const int ns = f32_split_fwd_nsplit(batch, n, k, d);
    float *out = ns > 1 ? (float *)ws : A;
    hipError_t e = k <= 64 ? dispatch_x3r<false>(phi, mass, feat, batch, n, k, d, ns, out, st)
                           : dispatch_x3r<true>(phi, mass, feat, batch, n, k, d, ns, out, st);
    if (e != hipSuccess || ns <= 1) return e;
    return launch_reduce(out, ns, batch, k, d, A, st);
}

static int bwdmc_ks(int64_t k) { return (int)((k + 31) / 32); }

bool bf16_bwd_shape_ok(int64_t n, int64_t k, int64_t d)
{
    return k >= 8 && k <= 256 && k % 8 == 0 && n >= 1 && d >= 1;
}

bool f32_split_bwd_shape_ok(int64_t n, int64_t k, int64_t d)
{
    return k >= 2 && k <= 64 && k % 2 == 0 && n >= 1 && d >= 1;
}

// vertex ranges per (shape, column block): the fewest that fill whole rounds of the
// resident workgroup slots (>= 95% of the last round busy), at most one range per tile
static int bwdmc_vsplit(int64_t batch, int64_t dblocks, int64_t ntile, int per_cu)
{
    const int64_t slots = (int64_t)device_cus() * per_cu, base = batch * dblocks;
    int best = 1;
    double best_e = 0.0;
    for (int64_t v = 1; v <= ntile && v <= 64; ++v) {
        const int64_t tot = base * v, rounds = (tot + slots - 1) / slots;
        const double e = (double)tot / (double)(rounds * slots);
        if (e >= 0.95) return (int)v;
        if (e > best_e + 1e-9) {
            best_e = e;
            best = (int)v;
        }
    }
    return best;
}

template <typename T, int PP, int PD, int KS>
static hipError_t dispatch_bwdmc(const T *phi, const float *mass, const float *dA, int64_t batch, int64_t n, int64_t k,
                                 int64_t d, float *dF, hipStream_t st)
{
    const size_t lds = bwdmc_lds(PD, KS);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)proj_bwd_mc_kernel<T, PP, PD, KS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    const int dblocks = (int)((d + BB_COLS - 1) / BB_COLS);
    const int64_t ntile = (n + BB_VT - 1) / BB_VT;
    static int per_cu = 0;  // resident workgroups per CU (registers and LDS), queried once
    if (per_cu == 0) {
        int r = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, (const void *)proj_bwd_mc_kernel<T, PP, PD, KS>, 512,
                                                         lds) != hipSuccess || r < 1)
            r = 1;
        per_cu = r;
    }
    const int vsplit = bwdmc_vsplit(batch, dblocks, ntile, per_cu);
    const int ntasks = (int)(batch * vsplit);
    const unsigned grid = (unsigned)(8 * dblocks * ((ntasks + 7) / 8));
    hipLaunchKernelGGL((proj_bwd_mc_kernel<T, PP, PD, KS>), dim3(grid), dim3(512), lds, st, phi, mass, dA, (int)n,
                       (int)k, (int)d, vsplit, dblocks, ntasks, dF);
    return hipGetLastError();
}

hipError_t launch_project_backward_bf16(const uint16_t *phi, const float *mass, const float *dA, int64_t batch,
                                        int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st)
{
    switch (bwdmc_ks(k)) {
    case 1: return dispatch_bwdmc<uint16_t, 1, 2, 1>(phi, mass, dA, batch, n, k, d, dF, st);
    case 2: return dispatch_bwdmc<uint16_t, 1, 2, 2>(phi, mass, dA, batch, n, k, d, dF, st);
    case 3: return dispatch_bwdmc<uint16_t, 1, 2, 3>(phi, mass, dA, batch, n, k, d, dF, st);
    case 4: return dispatch_bwdmc<uint16_t, 1, 2, 4>(phi, mass, dA, batch, n, k, d, dF, st);
    case 5: return dispatch_bwdmc<uint16_t, 1, 2, 5>(phi, mass, dA, batch, n, k, d, dF, st);
    case 6: return dispatch_bwdmc<uint16_t, 1, 2, 6>(phi, mass, dA, batch, n, k, d, dF, st);
    case 7: return dispatch_bwdmc<uint16_t, 1, 2, 7>(phi, mass, dA, batch, n, k, d, dF, st);
    default: return dispatch_bwdmc<uint16_t, 1, 2, 8>(phi, mass, dA, batch, n, k, d, dF, st);
    }
}

hipError_t launch_project_backward_f32_split(const float *phi, const float *mass, const float *dA, int64_t batch,
                                             int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st)
{
    if (bwdmc_ks(k) == 1) return dispatch_bwdmc<float, 3, 3, 1>(phi, mass, dA, batch, n, k, d, dF, st);
    return dispatch_bwdmc<float, 3, 3, 2>(phi, mass, dA, batch, n, k, d, dF, st);
}

bool f32k_bwd_shape_ok(int64_t n, int64_t k, int64_t d)
{
    return k > 64 && k <= kMaxK && k % 2 == 0 && n >= 1 && d >= 1;
}

template <int KS>
static hipError_t dispatch_bwdk(const float *phi, const float *mass, const float *dA, int64_t batch, int64_t n,
                                int64_t k, int64_t d, float *dF, hipStream_t st)
{
    const size_t lds = bwdk_lds(KS);
    static int per_cu = 0;  // resident workgroups per CU, queried once (with the LDS limit raised)
    if (per_cu == 0) {
        (void)hipFuncSetAttribute((const void *)proj_bwd_mck_kernel<KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        int r = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, (const void *)proj_bwd_mck_kernel<KS>, 512, lds) !=
                hipSuccess ||
            r < 1)
            r = 1;
        per_cu = r;
    }
    const int dblocks = (int)((d + BK_COLS - 1) / BK_COLS);
    const int64_t ntile = (n + BB_VT - 1) / BB_VT;
    const int vsplit = bwdmc_vsplit(batch, dblocks, ntile, per_cu);
    const int ntasks = (int)(batch * vsplit);
    const unsigned grid = (unsigned)(8 * dblocks * ((ntasks + 7) / 8));
    hipLaunchKernelGGL((proj_bwd_mck_kernel<KS>), dim3(grid), dim3(512), lds, st, phi, mass, dA, (int)n, (int)k,
                       (int)d, vsplit, dblocks, ntasks, dF);
    return hipGetLastError();
}

hipError_t launch_project_backward_f32k(const float *phi, const float *mass, const float *dA, int64_t batch,
                                        int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st)
{
    switch (bwdmc_ks(k)) {
    case 3: return dispatch_bwdk<3>(phi, mass, dA, batch, n, k, d, dF, st);
    case 4: return dispatch_bwdk<4>(phi, mass, dA, batch, n, k, d, dF, st);
    case 5: return dispatch_bwdk<5>(phi, mass, dA, batch, n, k, d, dF, st);
    case 6: return dispatch_bwdk<6>(phi, mass, dA, batch, n, k, d, dF, st);
    case 7: return dispatch_bwdk<7>(phi, mass, dA, batch, n, k, d, dF, st);
    case 8: return dispatch_bwdk<8>(phi, mass, dA, batch, n, k, d, dF, st);
    case 9: return dispatch_bwdk<9>(phi, mass, dA, batch, n, k, d, dF, st);
    default: return dispatch_bwdk<10>(phi, mass, dA, batch, n, k, d, dF, st);
    }
}

// ---------------------------------------------------------------------------
// Uneven batches: one workgroup per work item
// ---------------------------------------------------------------------------
bool x3r_item_shape_ok(int64_t k, int64_t d)
{
    return ((k >= 4 && k <= 64 && k % 2 == 0) || (k > 64 && k <= kMaxK && k % 4 == 0)) && d % 4 == 0;
}

hipError_t launch_fwd_x3r_items(const FwdItem *items, int nitems, bool sliced, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (sliced)
        hipLaunchKernelGGL((proj_fwd_x3r_items_kernel<true>), dim3((unsigned)nitems), dim3(256), x3r_lds(), st, items);
    else
        hipLaunchKernelGGL((proj_fwd_x3r_items_kernel<false>), dim3((unsigned)nitems), dim3(256), x3r_lds(), st, items);
    return hipGetLastError();
}

bool mc_item_shape_ok(int64_t k) { return k >= 2 && k <= kMaxK && k % 2 == 0; }
int mc_item_cols(int64_t k) { return k <= 64 ? BB_COLS : BK_COLS; }

template <int KS>
static hipError_t launch_mc_items_ks(const McItem *items, int nitems, hipStream_t st)
{
    if constexpr (KS <= 2) {
        const size_t lds = bwdmc_lds(3, KS);
        static bool attr_set = false;
        if (!attr_set) {
            (void)hipFuncSetAttribute((const void *)proj_bwd_mc_items_kernel<KS>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            attr_set = true;
        }
        hipLaunchKernelGGL((proj_bwd_mc_items_kernel<KS>), dim3((unsigned)nitems), dim3(512), lds, st, items);
    } else {
        const size_t lds = bwdk_lds(KS);
        static bool attr_set = false;
        if (!attr_set) {
            (void)hipFuncSetAttribute((const void *)proj_bwd_mck_items_kernel<KS>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            attr_set = true;
        }
        hipLaunchKernelGGL((proj_bwd_mck_items_kernel<KS>), dim3((unsigned)nitems), dim3(512), lds, st, items);
    }
    return hipGetLastError();
}

hipError_t launch_bwd_mc_items(const McItem *items, int nitems, int64_t k, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    switch (bwdmc_ks(k)) {
    case 1: return launch_mc_items_ks<1>(items, nitems, st);
    case 2: return launch_mc_items_ks<2>(items, nitems, st);
    case 3: return launch_mc_items_ks<3>(items, nitems, st);
    case 4: return launch_mc_items_ks<4>(items, nitems, st);
    case 5: return launch_mc_items_ks<5>(items, nitems, st);
    case 6: return launch_mc_items_ks<6>(items, nitems, st);
    case 7: return launch_mc_items_ks<7>(items, nitems, st);
    case 8: return launch_mc_items_ks<8>(items, nitems, st);
    case 9: return launch_mc_items_ks<9>(items, nitems, st);
    default: return launch_mc_items_ks<10>(items, nitems, st);
    }
}

}  // namespace fmap

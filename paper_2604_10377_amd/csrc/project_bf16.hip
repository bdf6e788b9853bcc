// Forward projection A = Phi^T diag(M) F (Eq. 1) with bfloat16 basis and
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
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
                dma16(reinterpret_cast<const float *>(F + (size_t)(v + r) * d + col),
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

        // feature operands: tile h*4+tt holds columns dsl*128 + h*64 + 4*m16 + tt of vertices 8*g4..+7
        u32x4_t B[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cb = dsl * 128 + h * 64 + 4 * m16;
            uint2 y[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) y[i] = *reinterpret_cast<const uint2 *>(Fs + (8 * g4 + i) * C::DWG + cb);
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const uint32_t lo = (tt < 2) ? y[2 * jj].x : y[2 * jj].y;
                    const uint32_t hi = (tt < 2) ? y[2 * jj + 1].x : y[2 * jj + 1].y;
                    B[h * 4 + tt][jj] = __builtin_amdgcn_perm(hi, lo, (tt & 1) ? 0x07060302u : 0x05040100u);
                }
        }
        // basis operands: rows r4..r4+3 x vertices 8*g4..8*g4+7, scaled by mass, as hi + lo
        uint2 x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = *reinterpret_cast<const uint2 *>(Ps + (8 * g4 + i) * k + r4);
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
    // Row R of tile a is basis row ks*64 + 4R + a; column N of tile (h, tt) is
    // feature column dbase + dsl*128 + h*64 + 4N + tt.
    float *O = out + (size_t)j * k * d;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ks * 64 + 4 * (4 * g4 + r) + a;
            if (row >= k) continue;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    const int col = dbase + dsl * 128 + h * 64 + 4 * m16 + tt;
                    if (col < d) O[(size_t)row * d + col] = acc[a][h * 4 + tt][r];
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
// Backward projection dF = diag(M) Phi dA with a bf16 basis (float32 dA, dF).
//
// Here the contraction runs over k, which is contiguous in a basis row, so a
// lane's 8 K slots are one 16-byte global load of its vertex's row: the basis
// needs no transpose and no LDS.  The other operand, dA^T, is staged once per
// workgroup in LDS as bf16 hi + lo parts (dA = hi + lo to ~2^-16 relative; two
// matrix-core steps per tile), transposed to [column][k] so that each operand
// is one ds_read_b128.  The mass is applied to the float32 result.
//
// Workgroup = 8 waves, one 128-column block of d; a wave owns 32 vertices x 128
// columns (2 x 8 tiles of 16x16).  A workgroup walks a contiguous range of
// 256-vertex tiles, so the staging (k x 128 floats read from L2) is amortised
// over thousands of vertices.  The column blocks of one vertex range sit on the
// same XCD (consecutive ids of one residue class mod 8), so the basis rows they
// all read are fetched from HBM once and served from that XCD's L2 afterwards.
// ---------------------------------------------------------------------------
constexpr int BB_COLS = 128;   // columns per workgroup
constexpr int BB_VT = 256;     // vertices per workgroup tile (8 waves x 32)

__host__ __device__ constexpr int bwd_bf16_kp(int k) { return (k + 31) & ~31; }             // k padded to K steps
__host__ __device__ constexpr int bwd_bf16_stride(int k) { return bwd_bf16_kp(k) * 2 + 16; }  // bytes per LDS row
__host__ __device__ constexpr size_t bwd_bf16_lds(int k) { return (size_t)2 * BB_COLS * bwd_bf16_stride(k); }

__global__ __launch_bounds__(512, 2) void proj_bwd_bf16_kernel(const uint16_t *__restrict__ phi,
                                                             const float *__restrict__ mass,
                                                             const float *__restrict__ dA, int n, int k, int d,
                                                             int vsplit, int dblocks, int ntasks,
                                                             float *__restrict__ dF)
{
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m16 = lane & 15, g4 = lane >> 4;
    const int bid = blockIdx.x;
    const int xs = bid & 7, q = bid >> 3;
    const int db = q % dblocks;
    const int j = (q / dblocks) * 8 + xs;
    if (j >= ntasks) return;  // whole workgroup, before any barrier
    const int vs = j % vsplit, s = j / vsplit;
    const int dbase = db * BB_COLS;
    const int kp = bwd_bf16_kp(k), stride = bwd_bf16_stride(k);

    const uint16_t *P = phi + (size_t)s * n * k;
    const float *Mv = mass + (size_t)s * n;
    const float *G = dA + (size_t)s * k * d;
    float *O = dF + (size_t)s * n * d;

    // stage dA^T (hi, lo) for columns [dbase, dbase + 128), rows j < kp (zero past k and d)
    char *hiT = reinterpret_cast<char *>(smem);
    char *loT = hiT + BB_COLS * stride;
    for (int e = tid; e < kp * BB_COLS; e += 512) {
        const int jj = e / BB_COLS, c = e - jj * BB_COLS;
        const float v = (jj < k && dbase + c < d) ? G[(size_t)jj * d + dbase + c] : 0.f;
        const uint32_t h2 = pack_bf16(v, 0.f);
        const float hv = __uint_as_float(h2 << 16);
        const uint32_t l2 = pack_bf16(v - hv, 0.f);
        *reinterpret_cast<uint16_t *>(hiT + c * stride + 2 * jj) = (uint16_t)h2;
        *reinterpret_cast<uint16_t *>(loT + c * stride + 2 * jj) = (uint16_t)l2;
    }
    __syncthreads();

    const int ntile = (n + BB_VT - 1) / BB_VT;
    const int t0 = (int)(((long)vs * ntile) / vsplit), t1 = (int)(((long)(vs + 1) * ntile) / vsplit);
    const int ksteps = kp / 32;

    for (int vt = t0; vt < t1; ++vt) {
        const int vbase = vt * BB_VT + wave * 32;
        f32x4 acc[2][8];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4{0, 0, 0, 0};
        // basis rows of the lane's two M-tile vertices (clamped into the shape; rows past n are not stored)
        const uint16_t *prow[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) prow[mt] = P + (size_t)min(vbase + mt * 16 + m16, n - 1) * k;
        // this lane's 8 K slots of step kc start at kc*32 + 8*g4; k % 8 == 0, so all or none exist
        auto load_a = [&](int kc, u32x4_t (&a)[2]) {
            const int kk = kc * 32 + 8 * g4;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
                a[mt] = (kk < k) ? *reinterpret_cast<const u32x4_t *>(prow[mt] + kk) : u32x4_t{0, 0, 0, 0};
        };
        u32x4_t a[2], an[2];
        load_a(0, a);
        for (int kc = 0; kc < ksteps; ++kc) {
            const int kk = kc * 32 + 8 * g4;
            if (kc + 1 < ksteps) load_a(kc + 1, an);  // next step's basis in flight during this step
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const int off = (nt * 16 + m16) * stride + 2 * kk;
                const u32x4_t bh = *reinterpret_cast<const u32x4_t *>(hiT + off);
                const u32x4_t bl = *reinterpret_cast<const u32x4_t *>(loT + off);
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    acc[mt][nt] = mfma16x16x32bf16(a[mt], bh, acc[mt][nt]);
                    acc[mt][nt] = mfma16x16x32bf16(a[mt], bl, acc[mt][nt]);
                }
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) a[mt] = an[mt];
        }
        // D layout: register r of lane (m16, g4) is vertex row 4*g4 + r of the tile, column m16
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int v = vbase + mt * 16 + 4 * g4 + r;
                if (v >= n) continue;
                const float m = Mv[v];
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) {
                    const int col = dbase + nt * 16 + m16;
                    if (col < d) O[(size_t)v * d + col] = acc[mt][nt][r] * m;
                }
            }
    }
}

bool bf16_bwd_shape_ok(int64_t n, int64_t k, int64_t d)
{
    return k >= 8 && k <= 256 && k % 8 == 0 && n >= 1 && d >= 1;
}

hipError_t launch_project_backward_bf16(const uint16_t *phi, const float *mass, const float *dA, int64_t batch,
                                        int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)proj_bwd_bf16_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bwd_bf16_lds(256));
        attr_set = true;
    }
    const int dblocks = (int)((d + BB_COLS - 1) / BB_COLS);
    const int64_t ntile = (n + BB_VT - 1) / BB_VT;
    int64_t vsplit = (device_cus() + batch * dblocks - 1) / (batch * dblocks);
    if (vsplit > ntile) vsplit = ntile;
    if (vsplit < 1) vsplit = 1;
    const int ntasks = (int)(batch * vsplit);
    const unsigned grid = (unsigned)(8 * dblocks * ((ntasks + 7) / 8));
    hipLaunchKernelGGL(proj_bwd_bf16_kernel, dim3(grid), dim3(512), bwd_bf16_lds((int)k), st, phi, mass, dA, (int)n,
                       (int)k, (int)d, (int)vsplit, dblocks, ntasks, dF);
    return hipGetLastError();
}

}  // namespace fmap

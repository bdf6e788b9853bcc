// DiffusionNet spatial-gradient features (Sec. 3.2), both documented variants.
//
// Per vertex v the D channels carry complex gradients z = x + i y, stored
// interleaved: z[v][2j] = x_j, z[v][2j + 1] = y_j.  With the learned complex
// matrix A = A_re + i A_im ((A z)_c = sum_j A_cj z_j):
//     (A z)_re = A_re x - A_im y
//     (A z)_im = A_re y + A_im x    (variant A)   or   A_re x + A_im y   (variant B)
//     g        = x * (A z)_re + y * (A z)_im
// Read with k over the interleaved z row (length 2D), both transformed parts are
// one product Z [V x 2D] times W^T, where row c of W_re is
// (A_re[c][0], -A_im[c][0], A_re[c][1], -A_im[c][1], ...) and row c of W_im is
// (A_im[c][j], A_re[c][j]) pairs (variant A) or (A_re[c][j], A_im[c][j]) pairs
// (variant B).  That is a dense contraction of 8 D^2 flops per vertex against
// 12 D bytes of traffic (85 flop/B at D = 128): it runs on the float32 matrix
// cores (v_mfma_f32_32x32x2_f32), with the elementwise combination fused into
// the epilogue.
//
// A workgroup owns a block of 32 output channels: it builds the 64 rows of W
// for them (32 of W_re, 32 of W_im) in LDS once and then walks vertex tiles of
// 32, one tile per wave at a time.  Lane (m, h) (m = lane % 32, h = lane / 32)
// reads 16-byte pieces of the z row of vertex m straight from global memory;
// the matrix-core K order is permuted so that each lane uses its own four
// consecutive values in four steps, and the W operand is read the same way
// from LDS.  The workgroups of one vertex range and different channel blocks
// get consecutive ids in one residue class mod 8 (one XCD), so the z rows they
// all read come from HBM once and then from that XCD's L2.
#include "../../include/fmap.h"

#include <algorithm>

#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

namespace {

constexpr int GF_WAVES = 4;
constexpr int GF_CB = 32;  // output channels per workgroup

__device__ __forceinline__ f32x4 ld4(const float *p) { return *reinterpret_cast<const f32x4 *>(p); }

}  // namespace

// z [V][2D], A_re, A_im [D][D], g [V][D]; D % 32 == 0, D <= 512.  grid = vgroups * (D / 32), XCD-ordered.
template <int D>
__global__ __launch_bounds__(256) void gradfeat_mfma_kernel(const float *__restrict__ z, const float *__restrict__ Are,
                                                            const float *__restrict__ Aim, int variant, int V,
                                                            int vgroups, float *__restrict__ g)
{
    constexpr int K = 2 * D;
    constexpr int WP = K + 4;  // LDS row pitch of W (floats): 16-byte aligned, rows 4 banks apart
    constexpr int Q = K / 8;   // 8 k values per lane pair and step group
    extern __shared__ __align__(16) float sW[];  // [64][WP]: rows 0..31 W_re, 32..63 W_im of this block
    const int nb = D / GF_CB;
    // XCD-aware decode: ids b, b + 8, b + 16, ... share an XCD; the nb channel blocks of one vertex group are
    // consecutive in that sequence
    const int id = blockIdx.x;
    const int per_xcd = (int)((gridDim.x + 7) / 8);
    const int seq = (id % 8) * per_xcd + id / 8;  // position in the XCD-major order
    if (seq >= vgroups * nb) return;
    const int vg = seq / nb, cb = seq % nb;
    const int c0 = cb * GF_CB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 31, h = lane >> 5;

    // W rows of this channel block
    for (int e = tid; e < 64 * D; e += 256) {
        const int r = e / D, j = e % D;  // r < 32: W_re row c0 + r; r >= 32: W_im row c0 + r - 32
        const int c = c0 + (r & 31);
        const float ar = Are[(size_t)c * D + j], ai = Aim[(size_t)c * D + j];
        float w0, w1;
        if (r < 32) {
            w0 = ar;
            w1 = -ai;
        } else if (variant == 0) {
            w0 = ai;
            w1 = ar;
        } else {
            w0 = ar;
            w1 = ai;
        }
        sW[r * WP + 2 * j] = w0;
        sW[r * WP + 2 * j + 1] = w1;
    }
    __syncthreads();

    const int tiles = (V + 31) / 32;
    const int t_per = (tiles + vgroups - 1) / vgroups;
    const int t0 = vg * t_per, t1 = min(tiles, t0 + t_per);
    const float *wre = sW + m * WP + 4 * h;
    const float *wim = sW + (32 + m) * WP + 4 * h;
    for (int t = t0 + wave; t < t1; t += GF_WAVES) {
        const int v0 = 32 * t;
        const float *zr = z + (size_t)min(v0 + m, V - 1) * K + 4 * h;
        f32x16 are = zero16(), aim = zero16();
        // z pieces of 8 step groups in flight at a time
        constexpr int G = 8;
#pragma unroll 1
        for (int q0 = 0; q0 < Q; q0 += G) {
            f32x4 a[G];
#pragma unroll
            for (int u = 0; u < G; ++u) a[u] = ld4(zr + 8 * (q0 + u));
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const f32x4 br = ld4(wre + 8 * (q0 + u)), bi = ld4(wim + 8 * (q0 + u));
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    are = mfma32x32x2(a[u][e], br[e], are);
                    aim = mfma32x32x2(a[u][e], bi[e], aim);
                }
            }
        }
        // epilogue: g[v][c] = x_c (A z)_re + y_c (A z)_im for the 16 vertex rows of this lane, channel c0 + m
        const int c = c0 + m;
        float2 xy[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int v = min(v0 + acc32_row(r, lane), V - 1);
            xy[r] = *reinterpret_cast<const float2 *>(z + (size_t)v * K + 2 * c);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int v = v0 + acc32_row(r, lane);
            if (v < V) g[(size_t)v * D + c] = xy[r].x * are[r] + xy[r].y * aim[r];
        }
    }
}

// Any D: one thread per output (v, c), plain float32 dot products (the reference path for shapes the
// matrix-core kernel does not take).
__global__ __launch_bounds__(256) void gradfeat_general_kernel(const float *__restrict__ z, const float *__restrict__ Are,
                                                               const float *__restrict__ Aim, int variant, int V, int D,
                                                               float *__restrict__ g)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= (int64_t)V * D) return;
    const int v = (int)(o / D), c = (int)(o % D);
    const float *zv = z + (size_t)v * 2 * D;
    float re = 0.f, im = 0.f;
    for (int j = 0; j < D; ++j) {
        const float x = zv[2 * j], y = zv[2 * j + 1];
        const float ar = Are[(size_t)c * D + j], ai = Aim[(size_t)c * D + j];
        re += ar * x - ai * y;
        im += variant == 0 ? (ar * y + ai * x) : (ar * x + ai * y);
    }
    g[o] = zv[2 * c] * re + zv[2 * c + 1] * im;
}

template <int D>
static void launch_gf(const float *z, const float *Are, const float *Aim, int variant, int64_t V, float *g,
                      hipStream_t st)
{
    const size_t lds = (size_t)64 * (2 * D + 4) * sizeof(float);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)gradfeat_mfma_kernel<D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        attr = true;
    }
    const int nb = D / GF_CB;
    const int64_t tiles = (V + 31) / 32;
    // about two workgroups per CU over all channel blocks, at least 4 tiles per wave
    const int64_t want = std::max<int64_t>(1, 2 * (int64_t)device_cus() / nb);
    const int64_t vgroups = std::max<int64_t>(1, std::min<int64_t>(want, (tiles + 15) / 16));
    const int64_t n = vgroups * nb;
    const int64_t grid = ((n + 7) / 8) * 8;  // whole rounds of the 8 XCDs; surplus ids exit
    hipLaunchKernelGGL((gradfeat_mfma_kernel<D>), dim3((unsigned)grid), dim3(256), lds, st, z, Are, Aim, variant,
                       (int)V, (int)vgroups, g);
}

hipError_t launch_gradient_features(const float *z, const float *Are, const float *Aim, int variant, int64_t V,
                                    int64_t D, float *g, hipStream_t st)
{
    const bool al = (((uintptr_t)z) & 15) == 0;
    if (al && D == 32) launch_gf<32>(z, Are, Aim, variant, V, g, st);
    else if (al && D == 64) launch_gf<64>(z, Are, Aim, variant, V, g, st);
    else if (al && D == 128) launch_gf<128>(z, Are, Aim, variant, V, g, st);
    else if (al && D == 256) launch_gf<256>(z, Are, Aim, variant, V, g, st);
    else {
        const int64_t n = V * D;
        hipLaunchKernelGGL(gradfeat_general_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, z, Are, Aim,
                           variant, (int)V, (int)D, g);
    }
    return hipGetLastError();
}

}  // namespace fmap

extern "C" fmap_status fmap_gradient_features(const float *z, const float *A_re, const float *A_im, int32_t variant,
                                              int64_t vertices, int64_t channels, float *g, void *stream)
{
    if (!z || !A_re || !A_im || !g) return FMAP_ERR_NULL;
    if (variant != FMAP_GRADFEAT_A && variant != FMAP_GRADFEAT_B) return FMAP_ERR_VALUE;
    if (vertices < 1 || channels < 1 || vertices >= ((int64_t)1 << 31) || channels > 4096 ||
        vertices * channels >= ((int64_t)1 << 31))
        return FMAP_ERR_SHAPE;
    return fmap::launch_gradient_features(z, A_re, A_im, variant, vertices, channels, g, (hipStream_t)stream) ==
                   hipSuccess
               ? FMAP_OK
               : FMAP_ERR_HIP;
}

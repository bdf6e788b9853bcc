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

namespace fmap {

template <typename T>
__device__ __forceinline__ float load_elem(const T *p, size_t i);
template <>
__device__ __forceinline__ float load_elem<float>(const float *p, size_t i) { return p[i]; }
template <>
__device__ __forceinline__ float load_elem<uint16_t>(const uint16_t *p, size_t i) { return bf16_to_f32(p[i]); }

template <typename T, int MT, int NT, int U>
__global__ __launch_bounds__(256) void proj_fwd_kernel(const T *__restrict__ phi, const float *__restrict__ mass,
                                                       const T *__restrict__ feat, int n, int k, int d, int nsplit,
                                                       int chunk, int kblocks, int dblocks,
                                                       float *__restrict__ out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    int bid = blockIdx.x;
    const int db = bid % dblocks;
    bid /= dblocks;
    const int kb = bid % kblocks;
    bid /= kblocks;
    const int split = bid % nsplit;
    const int s = bid / nsplit;

    const int v0 = split * chunk;
    const int v1 = min(n, v0 + chunk);
    const int kbase = kb * (MT * 32);
    const int dbase = (db * 4 + wave) * (NT * 32);
    if (dbase >= d) return;  // whole wave idle (narrow d)

    const T *P = phi + (size_t)s * n * k;
    const T *F = feat + (size_t)s * n * d;
    const float *Mv = mass + (size_t)s * n;

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

    // Main loop: U matrix-core steps (2U vertices) per iteration, loads first.
    int v = v0;
    for (; v + 2 * U <= v1; v += 2 * U) {
        float a[U][MT], b[U][NT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int vv = v + 2 * u + half;
            const float m = Mv[vv];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a[u][mt] = rok[mt] ? load_elem(P, (size_t)vv * k + rows[mt]) * m : 0.f;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[u][nt] = cok[nt] ? load_elem(F, (size_t)vv * d + cols[nt]) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma32x32x2(a[u][mt], b[u][nt], acc[mt][nt]);
    }
    // Tail: guarded single steps.
    for (; v < v1; v += 2) {
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

    float *O = out + ((size_t)s * nsplit + split) * (size_t)k * d;
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

// A[s] = sum over chunks (in chunk order) of part[s][chunk].
__global__ __launch_bounds__(256) void proj_reduce_kernel(const float *__restrict__ part, int nsplit, int64_t kd,
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

template <typename T, int NT>
__global__ __launch_bounds__(256) void proj_bwd_kernel(const T *__restrict__ phi, const float *__restrict__ mass,
                                                       const float *__restrict__ dA, int n, int k, int d,
                                                       int rblocks, int dblocks, float *__restrict__ dF)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    int bid = blockIdx.x;
    const int db = bid % dblocks;
    bid /= dblocks;
    const int rb = bid % rblocks;
    const int s = bid / rblocks;
    const int row0 = (rb * 4 + wave) * 32;
    if (row0 >= n) return;
    const int dbase = db * (NT * 32);

    const T *P = phi + (size_t)s * n * k;
    const float *G = dA + (size_t)s * k * d;
    const int row = row0 + l32;
    const bool rok = row < n;
    const float m = rok ? mass[(size_t)s * n + row] : 0.f;

    int cols[NT];
    bool cok[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        cols[nt] = dbase + nt * 32 + l32;
        cok[nt] = cols[nt] < d;
    }
    f32x16 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = zero16();

    const int KH = (k + 1) >> 1;  // lane half h walks j = h*KH + t
    const int jb = half * KH;
    for (int t = 0; t < KH; ++t) {
        const int j = jb + t;
        const bool jok = j < k;
        const float a = (rok && jok) ? load_elem(P, (size_t)row * k + j) * m : 0.f;
        float b[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b[nt] = (jok && cok[nt]) ? G[(size_t)j * d + cols[nt]] : 0.f;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma32x32x2(a, b[nt], acc[nt]);
    }

    float *O = dF + (size_t)s * n * d;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int rr = row0 + acc32_row(r, lane);
            if (rr < n && cok[nt]) O[(size_t)rr * d + cols[nt]] = acc[nt][r];
        }
}

// ---------------------------------------------------------------------------
// Host-side launch planning
// ---------------------------------------------------------------------------

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
    int64_t want = (512 + tiles - 1) / tiles;
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

size_t project_workspace_bytes(int64_t batch, int64_t n, int64_t k, int64_t d, int32_t dtype)
{
    ProjPlan p = plan_project(batch, n, k, d, dtype);
    if (p.nsplit <= 1) return 0;
    return (size_t)batch * p.nsplit * k * d * sizeof(float);
}

template <typename T, int MT, int NT>
static void launch_fwd_t(const void *phi, const float *mass, const void *feat, int64_t batch, int64_t n, int64_t k,
                         int64_t d, const ProjPlan &p, float *out, hipStream_t st)
{
    const unsigned grid = (unsigned)(batch * p.nsplit * p.kblocks * p.dblocks);
    hipLaunchKernelGGL((proj_fwd_kernel<T, MT, NT, 4>), dim3(grid), dim3(256), 0, st, (const T *)phi, mass,
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

hipError_t launch_project(const void *phi, const float *mass, const void *feat, int32_t dtype, int64_t batch, int64_t n,
                          int64_t k, int64_t d, float *A, void *ws, hipStream_t st)
{
    ProjPlan p = plan_project(batch, n, k, d, dtype);
    float *out = p.nsplit > 1 ? (float *)ws : A;
    if (dtype == 0) launch_fwd_dt<float>(phi, mass, feat, batch, n, k, d, p, out, st);
    else launch_fwd_dt<uint16_t>(phi, mass, feat, batch, n, k, d, p, out, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.nsplit <= 1) return e;
    const int64_t total = batch * k * d;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(proj_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (const float *)ws, p.nsplit,
                       (int64_t)(k * d), total, A);
    return hipGetLastError();
}

template <typename T, int NT>
static void launch_bwd_t(const void *phi, const float *mass, const float *dA, int64_t batch, int64_t n, int64_t k,
                         int64_t d, float *dF, hipStream_t st)
{
    const int rblocks = (int)((n + 127) / 128);
    const int dblocks = (int)((d + NT * 32 - 1) / (NT * 32));
    const unsigned grid = (unsigned)(batch * rblocks * dblocks);
    hipLaunchKernelGGL((proj_bwd_kernel<T, NT>), dim3(grid), dim3(256), 0, st, (const T *)phi, mass, dA, (int)n,
                       (int)k, (int)d, rblocks, dblocks, dF);
}

hipError_t launch_project_backward(const void *phi, const float *mass, int32_t dtype, const float *dA, int64_t batch,
                                   int64_t n, int64_t k, int64_t d, float *dF, hipStream_t st)
{
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

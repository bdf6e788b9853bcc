// Overlap-prediction metrics (Sec. 3.3) over a batch of shapes of uneven size.
//
// Shape s owns vertices [offsets[s], offsets[s+1]) of the concatenated score
// and ground-truth arrays.  A vertex is predicted overlapping when its score is
// strictly greater than the threshold.  Per shape the kernels count the
// confusion matrix (TP, FP, FN, TN) and derive accuracy, precision, recall
// (sensitivity), specificity, IoU, F1 and balanced accuracy, the mean of
// sensitivity and specificity.
//
// The count is one streaming pass (5 bytes per vertex, HBM-bound).  Each wave
// owns a contiguous run of rows of 256 vertices (four per lane, one 16-byte
// score load and one 4-byte label load per lane, the rows loaded in chunks of
// four with the next chunk in flight while one is counted) and keeps per-lane
// counts for the shape it is in; when it leaves a shape it adds the wave's counts to that shape's slot
// with 64-bit integer atomics, so the totals do not depend on the order in
// which waves finish.  The shape of a wave's first vertex is found by a
// 64-way parallel search over the offsets; later shapes by walking forward.
// Rows that cross a shape boundary are counted vertex by vertex.  The slots are cleared by a kernel
// (no memset node under graph capture), and a last kernel turns the counts
// into the metrics in float64.
#include "../../include/fmap.h"

#include <algorithm>

#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

namespace {

constexpr int OV_THREADS = 256;
constexpr int OV_ROW = 256;  // vertices per wave row (4 per lane)
constexpr int OV_DEPTH = 4;  // rows per load chunk (two chunks in flight per wave)

// Largest s in [0, S) with off[s] <= v (off nondecreasing; clamps for any contents), found by the whole
// wave: each round the 64 lanes test 64 evenly spaced candidates (one load each, all in flight together)
// and a ballot narrows the range 64-fold, so 1024 shapes take two rounds of loads.  v is wave-uniform.
__device__ __forceinline__ int wave_shape_of(const int64_t *__restrict__ off, int S, int64_t v, int lane)
{
    int lo = 0, hi = S - 1;  // answer in [lo, hi]
    while (lo < hi) {
        const int span = hi - lo;
        const int step = (span + 63) / 64;
        const int cand = min(lo + 1 + lane * step, hi);  // candidates above lo
        const bool le = off[cand] <= v;
        const unsigned long long m = __ballot(le);
        // candidates increase with the lane index and off is nondecreasing, so the lanes with le form a prefix
        const int cnt = __popcll(m);
        if (cnt == 0) {
            hi = lo;  // even the first candidate is above v: the answer is lo
        } else {
            const int last = min(lo + 1 + (cnt - 1) * step, hi);  // largest candidate with off <= v
            const int next = min(lo + 1 + cnt * step, hi + 1);    // smallest candidate above v (or past hi)
            lo = last;
            hi = next - 1;
        }
    }
    return lo;
}

__device__ __forceinline__ unsigned wave_sum_u32(unsigned v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace

__global__ __launch_bounds__(256) void overlap_clear_kernel(unsigned long long *__restrict__ counts, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) counts[e] = 0ull;
}

// counts [S][4] = TP, FP, FN, TN.  Wave w of the launch owns rows [w R, (w + 1) R) (R = rows_per_wave).
// VEC: score is 16-byte and truth 4-byte aligned (whole rows read with one load each per lane).
template <bool VEC>
__global__ __launch_bounds__(OV_THREADS) void overlap_count_kernel(const float *__restrict__ score,
                                                                   const uint8_t *__restrict__ truth,
                                                                   const int64_t *__restrict__ off, int S,
                                                                   int64_t total, float thr, int64_t rows_per_wave,
                                                                   unsigned long long *__restrict__ counts)
{
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (OV_THREADS / 64) + (threadIdx.x >> 6);
    const int64_t nrows = (total + OV_ROW - 1) / OV_ROW;
    const int64_t row0 = gw * rows_per_wave;
    const int64_t row1 = min(row0 + rows_per_wave, nrows);
    if (row0 >= row1) return;
    auto load = [&](int64_t row, float (&sc)[4], uint32_t &gt) {
        const int64_t v0 = row * OV_ROW + 4 * lane;
        if (VEC && v0 + 3 < total) {
            const f32x4 x = *reinterpret_cast<const f32x4 *>(score + v0);
            sc[0] = x[0];
            sc[1] = x[1];
            sc[2] = x[2];
            sc[3] = x[3];
            gt = *reinterpret_cast<const uint32_t *>(truth + v0);
        } else {
            gt = 0u;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t v = min(v0 + e, total - 1);
                sc[e] = score[v];
                gt |= (uint32_t)truth[v] << (8 * e);
            }
        }
    };
    // shape of the first row's first vertex, its range, and the per-lane counts for it
    int cur = wave_shape_of(off, S, row0 * OV_ROW, lane);
    int64_t cur_lo = off[cur], cur_hi = off[cur + 1];
    unsigned c[4] = {0u, 0u, 0u, 0u};
    auto flush = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned t = wave_sum_u32(c[q]);
            if (lane == 0 && t) atomicAdd(&counts[4 * (int64_t)cur + q], (unsigned long long)t);
            c[q] = 0u;
        }
    };
    // count one row (vertices base .. base + 255, 4 per lane): whole rows of the current shape on the fast
    // path; a row that reaches past it vertex by vertex, walking the shapes forward (each lane to the shape
    // of its vertex), then the current shape moves on
    auto count_row = [&](int64_t row, const float (&sv)[4], uint32_t g) {
        const int64_t base = row * OV_ROW;
        const int64_t v0 = base + 4 * lane;
        const int64_t last = min(base + OV_ROW, total) - 1;
        if (base >= cur_lo && last < cur_hi) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (v0 + e <= last) {
                    const bool pos = sv[e] > thr, t = ((g >> (8 * e)) & 0xffu) != 0u;
                    c[pos ? (t ? 0 : 1) : (t ? 2 : 3)] += 1u;
                }
            }
        } else {
            flush();
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t v = v0 + e;
                if (v <= last) {
                    int s = cur;
                    while (s + 1 < S && off[s + 1] <= v) ++s;
                    if (v >= off[s] && v < off[s + 1]) {
                        const bool pos = sv[e] > thr, t = ((g >> (8 * e)) & 0xffu) != 0u;
                        atomicAdd(&counts[4 * (int64_t)s + (pos ? (t ? 0 : 1) : (t ? 2 : 3))], 1ull);
                    }
                }
            }
            const int64_t nb = base + OV_ROW;  // first vertex of the next row
            while (cur + 1 < S && off[cur + 1] <= nb) ++cur;
            cur_lo = off[cur];
            cur_hi = off[cur + 1];
        }
    };
    // rows in chunks of OV_DEPTH, the next chunk's loads in flight while one is counted (two register
    // buffers alternating by unrolling; loads past the run re-read its last row and are not counted)
    float sa[OV_DEPTH][4], sb[OV_DEPTH][4];
    uint32_t ga[OV_DEPTH], gb[OV_DEPTH];
    auto load_chunk = [&](int64_t r0, float (&sv)[OV_DEPTH][4], uint32_t (&g)[OV_DEPTH]) {
#pragma unroll
        for (int u = 0; u < OV_DEPTH; ++u) load(min(r0 + u, row1 - 1), sv[u], g[u]);
    };
    load_chunk(row0, sa, ga);
    for (int64_t row = row0; row < row1; row += 2 * OV_DEPTH) {
        load_chunk(row + OV_DEPTH, sb, gb);
#pragma unroll
        for (int u = 0; u < OV_DEPTH; ++u)
            if (row + u < row1) count_row(row + u, sa[u], ga[u]);
        if (row + OV_DEPTH >= row1) break;
        load_chunk(row + 2 * OV_DEPTH, sa, ga);
#pragma unroll
        for (int u = 0; u < OV_DEPTH; ++u)
            if (row + OV_DEPTH + u < row1) count_row(row + OV_DEPTH + u, sb[u], gb[u]);
    }
    flush();
}

// metrics [S][7]: accuracy, precision, recall, specificity, IoU, F1, balanced accuracy (float64 arithmetic
// on the exact counts, rounded once to float32; a ratio with a zero denominator is 0; balanced accuracy
// averages the class recalls that are defined)
__global__ __launch_bounds__(256) void overlap_metrics_kernel(const unsigned long long *__restrict__ counts, int S,
                                                              float *__restrict__ metrics)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    const double tp = (double)counts[4 * (int64_t)s], fp = (double)counts[4 * (int64_t)s + 1];
    const double fn = (double)counts[4 * (int64_t)s + 2], tn = (double)counts[4 * (int64_t)s + 3];
    auto ratio = [](double a, double b) { return b != 0.0 ? a / b : 0.0; };
    const double sens = ratio(tp, tp + fn), spec = ratio(tn, tn + fp);
    const bool ds = tp + fn != 0.0, dsp = tn + fp != 0.0;
    const double bal = (ds && dsp) ? (sens + spec) / 2.0 : (ds ? sens : (dsp ? spec : 0.0));
    float *m = metrics + 7 * (int64_t)s;
    m[0] = (float)ratio(tp + tn, tp + fp + fn + tn);
    m[1] = (float)ratio(tp, tp + fp);
    m[2] = (float)sens;
    m[3] = (float)spec;
    m[4] = (float)ratio(tp, tp + fp + fn);
    m[5] = (float)ratio(2.0 * tp, 2.0 * tp + fp + fn);
    m[6] = (float)bal;
}

hipError_t launch_overlap(const float *score, const uint8_t *truth, const int64_t *offsets, int64_t S, int64_t total,
                          float thr, int64_t *counts, float *metrics, hipStream_t st)
{
    unsigned long long *cnt = (unsigned long long *)counts;
    const int64_t nc = 4 * S;
    hipLaunchKernelGGL(overlap_clear_kernel, dim3((unsigned)std::min<int64_t>((nc + 255) / 256, 1024)), dim3(256), 0,
                       st, cnt, nc);
    if (total > 0) {
        // each wave a contiguous run of rows: about 16 waves per CU, at least 8 rows each
        const int64_t nrows = (total + OV_ROW - 1) / OV_ROW;
        const int64_t waves = 16 * (int64_t)device_cus();
        const int64_t rpw = std::max<int64_t>(8, (nrows + waves - 1) / waves);
        const int64_t nw = (nrows + rpw - 1) / rpw;
        const unsigned grid = (unsigned)((nw + OV_THREADS / 64 - 1) / (OV_THREADS / 64));
        const bool vec = (((uintptr_t)score) & 15) == 0 && (((uintptr_t)truth) & 3) == 0;
        if (vec)
            hipLaunchKernelGGL(overlap_count_kernel<true>, dim3(grid), dim3(OV_THREADS), 0, st, score, truth, offsets,
                               (int)S, total, thr, rpw, cnt);
        else
            hipLaunchKernelGGL(overlap_count_kernel<false>, dim3(grid), dim3(OV_THREADS), 0, st, score, truth,
                               offsets, (int)S, total, thr, rpw, cnt);
    }
    hipLaunchKernelGGL(overlap_metrics_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st, cnt, (int)S,
                       metrics);
    return hipGetLastError();
}

}  // namespace fmap

extern "C" fmap_status fmap_overlap_metrics(const float *scores, const uint8_t *truth, const int64_t *offsets,
                                            int64_t shapes, int64_t total, float threshold, int64_t *counts,
                                            float *metrics, void *stream)
{
    if (!offsets || !counts || !metrics) return FMAP_ERR_NULL;
    if (total > 0 && (!scores || !truth)) return FMAP_ERR_NULL;
    if (shapes < 1 || shapes >= ((int64_t)1 << 30) || total < 0 || total >= ((int64_t)1 << 40)) return FMAP_ERR_SHAPE;
    if (threshold != threshold) return FMAP_ERR_VALUE;  // NaN threshold
    return fmap::launch_overlap(scores, truth, offsets, shapes, total, threshold, counts, metrics,
                                (hipStream_t)stream) == hipSuccess
               ? FMAP_OK
               : FMAP_ERR_HIP;
}

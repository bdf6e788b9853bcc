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
// walks rows of 256 consecutive vertices, four per lane, keeping per-lane
// counts for the shape it is in; when it leaves a shape it adds the counts of
// the wave to that shape's slot with 64-bit integer atomics, so the totals do
// not depend on the order in which workgroups finish.  Rows that cross a shape
// boundary are counted vertex by vertex.  The slots are cleared by a kernel
// (no memset node under graph capture), and a last kernel turns the counts
// into the metrics in float64.
#include "../../include/fmap.h"

#include <algorithm>

#include "fmap_launch.h"

namespace fmap {

namespace {

constexpr int OV_THREADS = 256;
constexpr int OV_ROW = 256;  // vertices per wave row (4 per lane)

// Largest s in [0, S) with off[s] <= v (off nondecreasing; clamps for any contents).
__device__ __forceinline__ int shape_of(const int64_t *__restrict__ off, int S, int64_t v)
{
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= v) lo = mid;
        else hi = mid - 1;
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

// counts [S][4] = TP, FP, FN, TN
__global__ __launch_bounds__(OV_THREADS) void overlap_count_kernel(const float *__restrict__ score,
                                                                   const uint8_t *__restrict__ truth,
                                                                   const int64_t *__restrict__ off, int S,
                                                                   int64_t total, float thr, int64_t rows_per_wg,
                                                                   unsigned long long *__restrict__ counts)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t nrows = (total + OV_ROW - 1) / OV_ROW;
    const int64_t row1 = min(row0 + rows_per_wg, nrows);
    int cur = -1;                 // shape of the per-lane counts (wave-uniform)
    int64_t cur_lo = 0, cur_hi = -1;  // its vertex range [cur_lo, cur_hi)
    unsigned c[4] = {0u, 0u, 0u, 0u};
    auto flush = [&]() {
        if (cur >= 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const unsigned t = wave_sum_u32(c[q]);
                if (lane == 0 && t) atomicAdd(&counts[4 * (int64_t)cur + q], (unsigned long long)t);
                c[q] = 0u;
            }
        }
    };
    for (int64_t row = row0 + wave; row < row1; row += OV_THREADS / 64) {
        const int64_t base = row * OV_ROW;
        const int64_t v0 = base + 4 * lane;
        const int64_t last = min(base + OV_ROW, total) - 1;
        // the four vertices of this lane: unconditional loads from clamped indices, masked afterwards
        float sc[4];
        uint8_t gt[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t v = min(v0 + e, total - 1);
            sc[e] = score[v];
            gt[e] = truth[v];
        }
        if (!(base >= cur_lo && last < cur_hi)) {
            // the row leaves the current shape: find the shape of its first vertex
            const int s0 = shape_of(off, S, base);
            const int64_t lo = off[s0], hi = off[s0 + 1];
            flush();
            if (base >= lo && last < hi) {
                cur = s0;
                cur_lo = lo;
                cur_hi = hi;
            } else {
                // the row crosses a shape boundary (or lies outside the offsets): vertex by vertex
                cur = -1;
                cur_hi = -1;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t v = v0 + e;
                    if (v <= last) {
                        const int s = shape_of(off, S, v);
                        if (v >= off[s] && v < off[s + 1]) {
                            const bool pos = sc[e] > thr, t = gt[e] != 0;
                            atomicAdd(&counts[4 * (int64_t)s + (pos ? (t ? 0 : 1) : (t ? 2 : 3))], 1ull);
                        }
                    }
                }
                continue;
            }
        }
        // the whole row lies in shape cur
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (v0 + e <= last) {
                const bool pos = sc[e] > thr, t = gt[e] != 0;
                c[pos ? (t ? 0 : 1) : (t ? 2 : 3)] += 1u;
            }
        }
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
        // about 8 workgroups per CU, at least 4 rows per wave
        const int64_t nrows = (total + OV_ROW - 1) / OV_ROW;
        const int64_t want = 8 * (int64_t)device_cus();
        int64_t rows = std::max<int64_t>(16, (nrows + want - 1) / want);
        const int64_t grid = (nrows + rows - 1) / rows;
        hipLaunchKernelGGL(overlap_count_kernel, dim3((unsigned)grid), dim3(OV_THREADS), 0, st, score, truth, offsets,
                           (int)S, total, thr, rows, cnt);
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

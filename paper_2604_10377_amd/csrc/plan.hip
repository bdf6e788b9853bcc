// Plans for uneven batches of shape pairs (different n and k per pair).
//
// fmap_plan_create groups the pairs by k (the rows of all pairs of a group are
// one batch dimension, Eq. (8)), allocates the group buffers, and builds device
// tables of work items:
//   - forward projection items: (shape, vertex chunk, 64-row k block, 256-column
//     d block).  Shapes the emulated float32 kernel takes (k even, d % 4 == 0,
//     16-byte aligned rows) run their whole 32-vertex stages on it, one
//     workgroup per item (one launch for k <= 64, one for k > 64); the last
//     n % 32 vertices, and all other shapes, are items of ONE persistent launch
//     of the general kernel;
//   - reduction items: the fixed-order sum of each shape's chunk partials;
//   - backward projection items: (shape, 256-vertex tiles, column block) on the
//     emulated kernels, one launch per k group; (shape, rows, d block) items of
//     one persistent launch of the general kernel for the rest;
//   - copy items: gather eigenvalues / lambda / dC into the group buffers and
//     scatter C / info back to the pairs.
// It then autotunes (vertices per item, persistent grid size, row systems per
// workgroup, backward rows per item) by timing candidates on the caller's
// stream, or takes them from the cache file, and captures the forward and the
// backward pass as HIP graphs on a private stream, the k groups' solves as
// parallel branches between the projections.  fmap_plan_forward /
// _backward replay the graphs on the caller's stream: no host work, no
// allocation, no per-pair launches.
#include "../../include/fmap.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "fmap_launch.h"

namespace fmap {

struct CopyItem {
    const uint32_t *src;  // 4-byte words, copied bit for bit (floats and int32 info alike)
    uint32_t *dst;
    int n;
};

__global__ __launch_bounds__(256) void copy_items_kernel(const CopyItem *__restrict__ items, int nitems)
{
    for (int it = blockIdx.y; it < nitems; it += gridDim.y) {
        const CopyItem w = items[it];
        for (int e = blockIdx.x * 256 + threadIdx.x; e < w.n; e += gridDim.x * 256) w.dst[e] = w.src[e];
    }
}

static hipError_t launch_copies(const CopyItem *items, int nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_items_kernel, dim3(4, (unsigned)std::min(nitems, 65535)), dim3(256), 0, st, items, nitems);
    return hipGetLastError();
}

// Graph branches for the per-group solves, at most HIP's default number of hardware queues per process.
constexpr int kLanes = 4;

}  // namespace fmap

using namespace fmap;

struct Bucket {
    int64_t k = 0;
    std::vector<int> pairs;
    int waves = 4;             // row systems per workgroup of the register row solve (k <= kSmallK)
    int mc_off = 0, mc_n = 0;  // this group's backward items in the emulated-kernel table
    float *AB = nullptr, *dAB = nullptr, *C = nullptr, *factors = nullptr, *evx = nullptr, *evy = nullptr,
          *lam = nullptr, *dC = nullptr;
    int32_t *info = nullptr;
    void *ws = nullptr;
};

struct fmap_plan {
    std::vector<fmap_pair> pairs;
    int64_t d = 0;
    int mask_kind = 0;
    float gamma = 0.5f;
    bool recompute = false, has_bwd = false;
    int64_t kmax = 0;
    std::vector<Bucket> buckets;
    std::vector<void *> allocs;
    float *partials = nullptr;
    FwdItem *d_fwd = nullptr, *d_x3 = nullptr, *d_x3s = nullptr;
    int nfwd = 0, nx3 = 0, nx3s = 0;
    McItem *d_mc = nullptr;
    int nmc = 0;
    RedItem *d_red = nullptr;
    int nred = 0;
    BwdItem *d_bwd = nullptr;
    int nbwd = 0;
    CopyItem *d_gf = nullptr, *d_sf = nullptr, *d_gb = nullptr;
    int ngf = 0, nsf = 0, ngb = 0;
    int chunk = 1024, grid_fwd = 512, grid_bwd = 512, rb = 2, from_cache = 0;
    hipStream_t cap = nullptr;
    // k groups solve on up to kLanes graph branches: lane 0 is the capturing stream, lanes 1.. these streams
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    hipGraph_t gf = nullptr, gb = nullptr;
    hipGraphExec_t ef = nullptr, eb = nullptr;
};

namespace {

template <typename T>
hipError_t dev_alloc(fmap_plan *pl, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    pl->allocs.push_back(q);
    *p = (T *)q;
    return hipSuccess;
}

template <typename T>
hipError_t upload(fmap_plan *pl, T **dptr, const std::vector<T> &v, hipStream_t st)
{
    hipError_t e = dev_alloc(pl, dptr, v.size());
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    e = hipMemcpyAsync(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

template <typename S, typename D>
CopyItem words(const S *src, D *dst, int64_t n)
{
    static_assert(sizeof(S) == 4 && sizeof(D) == 4, "4-byte elements");
    return CopyItem{(const uint32_t *)src, (uint32_t *)dst, (int)n};
}

struct Shape {
    const float *phi, *mass, *feat;
    float *A_user, *dF;
    int64_t n, k;
    int bucket, slot;  // slot within the bucket's [2P] shape array
};

bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// the forward of this shape runs its whole stages on the emulated float32 kernel
bool x3r_shape(const Shape &s, int64_t d)
{
    return x3r_item_shape_ok(s.k, d) && aligned(s.phi, 16) && aligned(s.feat, 16) && s.n >= 32;
}

// the backward of every shape of this group runs on the emulated float32 kernels
bool mc_bucket(const fmap_plan *pl, int b)
{
    const Bucket &B = pl->buckets[b];
    if (!mc_item_shape_ok(B.k)) return false;
    for (int q : B.pairs) {
        const fmap_pair &p = pl->pairs[q];
        if (!aligned(p.phi_x, 8) || !aligned(p.phi_y, 8) ||
            (pl->d % 4 == 0 && (!aligned(p.dF_x, 16) || !aligned(p.dF_y, 16))))
            return false;
    }
    return true;
}

std::vector<Shape> shapes_of(const fmap_plan *pl)
{
    std::vector<Shape> sh;
    for (int b = 0; b < (int)pl->buckets.size(); ++b) {
        const Bucket &B = pl->buckets[b];
        const int P = (int)B.pairs.size();
        for (int q = 0; q < P; ++q) {
            const fmap_pair &pr = pl->pairs[B.pairs[q]];
            sh.push_back({pr.phi_x, pr.mass_x, pr.feat_x, pr.A, pr.dF_x, pr.n_x, B.k, b, q});
            sh.push_back({pr.phi_y, pr.mass_y, pr.feat_y, pr.B, pr.dF_y, pr.n_y, B.k, b, P + q});
        }
    }
    return sh;
}

// One workgroup per item, workgroup ids dealt round-robin to the 8 XCDs: reorder an emulated-kernel
// item list so that the items of one vertex chunk (its k and d blocks, which read the same feature
// rows) share an XCD and that XCD's L2.  Chunks, longest first, go to the least loaded XCD queue;
// table slot r * 8 + x is item r of queue x, or an empty item (v0 == v1) that returns at once.
static void deal_to_xcds(std::vector<FwdItem> &v)
{
    if (v.empty()) return;
    std::vector<std::vector<FwdItem>> q(8);
    std::vector<int64_t> load(8, 0);
    for (size_t i = 0; i < v.size();) {
        size_t j = i + 1;  // the items of one chunk are adjacent (pushed together, stable sort)
        while (j < v.size() && v[j].phi == v[i].phi && v[j].v0 == v[i].v0 && v[j].v1 == v[i].v1) ++j;
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (size_t t = i; t < j; ++t) q[x].push_back(v[t]);
        load[x] += (int64_t)(j - i) * (v[i].v1 - v[i].v0);
        i = j;
    }
    size_t rounds = 0;
    for (const auto &qx : q) rounds = std::max(rounds, qx.size());
    std::vector<FwdItem> out;
    out.reserve(8 * rounds);
    for (size_t r = 0; r < rounds; ++r)
        for (int x = 0; x < 8; ++x) {
            FwdItem w = r < q[x].size() ? q[x][r] : v[0];
            if (r >= q[x].size()) w.v1 = w.v0;
            out.push_back(w);
        }
    v.swap(out);
}

// Forward and reduction items for a given chunk size (a multiple of 32); partial slots are laid out shape
// after shape.  fx / fxs: emulated-kernel items (k <= 64 / k > 64), fi: general-kernel items.
void build_fwd_items(const fmap_plan *pl, int chunk, std::vector<FwdItem> &fi, std::vector<FwdItem> &fx,
                     std::vector<FwdItem> &fxs, std::vector<RedItem> &ri, size_t *partial_floats)
{
    fi.clear();
    fx.clear();
    fxs.clear();
    ri.clear();
    size_t off = 0;
    const int64_t d = pl->d;
    for (const Shape &s : shapes_of(pl)) {
        const Bucket &B = pl->buckets[s.bucket];
        const bool fast = x3r_shape(s, d);
        const int64_t nfast = fast ? s.n - s.n % 32 : 0;  // vertices in whole stages, on the emulated kernel
        const int nchf = (int)((nfast + chunk - 1) / chunk);
        const int nchg = (int)((s.n - nfast + chunk - 1) / chunk);
        const int nch = nchf + nchg;
        const int kb = (int)((s.k + 63) / 64), db = (int)((d + 255) / 256);
        float *part = pl->partials ? pl->partials + off : nullptr;
        for (int c = 0; c < nch; ++c) {
            const bool cf = c < nchf;
            const int64_t v0 = cf ? (int64_t)c * chunk : nfast + (int64_t)(c - nchf) * chunk;
            const int64_t v1 = std::min<int64_t>(cf ? nfast : s.n, v0 + chunk);
            for (int kk = 0; kk < kb; ++kk)
                for (int dd = 0; dd < db; ++dd) {
                    FwdItem w;
                    w.phi = s.phi;
                    w.mass = s.mass;
                    w.feat = s.feat;
                    w.out = part ? part + (size_t)c * s.k * d : nullptr;
                    w.n = (int)s.n;
                    w.k = (int)s.k;
                    w.d = (int)d;
                    w.v0 = (int)v0;
                    w.v1 = (int)v1;
                    w.kbase = kk * 64;
                    w.dbase = dd * 256;
                    (cf ? (s.k > 64 ? fxs : fx) : fi).push_back(w);
                }
        }
        RedItem r;
        r.part = part;
        r.A = B.AB + (size_t)s.slot * s.k * d;
        r.A_user = s.A_user;
        r.nchunks = nch;
        r.kd = (int)(s.k * d);
        ri.push_back(r);
        off += (size_t)nch * s.k * d;
    }
    // longest items first: the workgroup scheduler (or the persistent grid's static round-robin) then
    // balances the tails
    auto longer = [](const FwdItem &a, const FwdItem &b) { return a.v1 - a.v0 > b.v1 - b.v0; };
    std::stable_sort(fi.begin(), fi.end(), longer);
    std::stable_sort(fx.begin(), fx.end(), longer);
    std::stable_sort(fxs.begin(), fxs.end(), longer);
    deal_to_xcds(fx);
    deal_to_xcds(fxs);
    *partial_floats = off;
}

// Backward items: groups on the emulated kernels get McItems of 2 rb 256-vertex tiles (bucket by bucket,
// with each bucket's offset and count recorded), the rest general-kernel items of 128 rb rows.
void build_bwd_items(fmap_plan *pl, int rb, std::vector<BwdItem> &bi, std::vector<McItem> &mi)
{
    bi.clear();
    mi.clear();
    const int64_t d = pl->d;
    for (int b = 0; b < (int)pl->buckets.size(); ++b) {
        Bucket &B = pl->buckets[b];
        B.mc_off = (int)mi.size();
        B.mc_n = 0;
        if (!mc_bucket(pl, b)) continue;
        const int cols = mc_item_cols(B.k);
        const int tpi = 2 * rb;
        std::vector<McItem> ranges;  // (shape, tile range) tasks, column block still open
        for (const Shape &s : shapes_of(pl)) {
            if (s.bucket != b) continue;
            const int ntile = (int)((s.n + 255) / 256);
            for (int t0 = 0; t0 < ntile; t0 += tpi) {
                McItem w;
                w.phi = s.phi;
                w.mass = s.mass;
                w.dA = B.dAB + (size_t)s.slot * s.k * d;
                w.dF = s.dF;
                w.n = (int)s.n;
                w.k = (int)s.k;
                w.d = (int)d;
                w.t0 = t0;
                w.t1 = std::min(ntile, t0 + tpi);
                w.dbase = 0;
                ranges.push_back(w);
            }
        }
        // Workgroup ids go round-robin to the 8 XCDs: slot q * 8 + x holds column block q % nb of tile
        // range (q / nb) * 8 + x, so the column blocks of one range run on one XCD and read its basis
        // rows from HBM once (from that XCD's L2 afterwards).  Slots past the last range are empty
        // items (t0 == t1, pointers of a real range) that return at once.
        const int nr = (int)ranges.size();
        const int nb = (int)((d + cols - 1) / cols);
        const int slots = nr > 0 ? 8 * nb * ((nr + 7) / 8) : 0;
        for (int bid = 0; bid < slots; ++bid) {
            const int x = bid & 7, q = bid >> 3;
            const int j = (q / nb) * 8 + x;
            McItem w = ranges[std::min(j, nr - 1)];
            w.dbase = (q % nb) * cols;
            if (j >= nr) w.t1 = w.t0;
            mi.push_back(w);
        }
        B.mc_n = (int)mi.size() - B.mc_off;
    }
    for (const Shape &s : shapes_of(pl)) {
        const Bucket &B = pl->buckets[s.bucket];
        if (B.mc_n > 0) continue;
        const int db = (int)((d + 255) / 256);
        for (int64_t r0 = 0; r0 < s.n; r0 += 128 * rb)
            for (int dd = 0; dd < db; ++dd) {
                BwdItem w;
                w.phi = s.phi;
                w.mass = s.mass;
                w.dA = B.dAB + (size_t)s.slot * s.k * d;
                w.dF = s.dF;
                w.n = (int)s.n;
                w.k = (int)s.k;
                w.d = (int)d;
                w.r0 = (int)r0;
                w.rb = rb;
                w.dbase = dd * 256;
                bi.push_back(w);
            }
    }
}

// The forward projection items of all shapes, then the fixed-order chunk sums.
hipError_t launch_projections_fwd(fmap_plan *pl, int grid, hipStream_t st)
{
    hipError_t e = launch_fwd_x3r_items(pl->d_x3, pl->nx3, false, st);
    if (e == hipSuccess) e = launch_fwd_x3r_items(pl->d_x3s, pl->nx3s, true, st);
    if (e == hipSuccess && pl->nfwd > 0) e = launch_fwd_items(pl->d_fwd, pl->nfwd, (int)pl->kmax, grid, st);
    if (e == hipSuccess) e = launch_reduce_items(pl->d_red, pl->nred, st);
    return e;
}

hipError_t launch_projections_bwd(fmap_plan *pl, int grid, hipStream_t st)
{
    hipError_t e = hipSuccess;
    for (const Bucket &B : pl->buckets)
        if (e == hipSuccess && B.mc_n > 0) e = launch_bwd_mc_items(pl->d_mc + B.mc_off, B.mc_n, B.k, st);
    if (e == hipSuccess && pl->nbwd > 0) e = launch_bwd_items(pl->d_bwd, pl->nbwd, (int)pl->kmax, grid, st);
    return e;
}

// The per-group solves of one pass.  Groups share no buffer (each has its own blocks of A, B, C, factors,
// info and workspace) and the solve kernels have no inter-workgroup waits, so with `branch` the groups run on
// separate streams forked from st and joined back into it: under capture, parallel branches of the graph, so
// that one group's latency-bound kernels run beside another group's.  With `tiled_in_line` the groups of the
// tiled row solve (k > kSmallK) stay in sequence on st: each is a persistent grid sized to the whole chip, and
// two side by side contend for it; only the other groups branch off beside them.
template <typename Fn>
hipError_t record_groups(fmap_plan *pl, hipStream_t st, bool branch, bool tiled_in_line, Fn fn)
{
    const int nb = (int)pl->buckets.size();
    const int nside = branch ? std::min<int>((int)pl->side.size(), nb - 1) : 0;
    std::vector<int> lane(nb, 0);
    int next = 0, used = 0;  // lanes 1..used receive work
    for (int i = 0; i < nb && nside > 0; ++i) {
        if (tiled_in_line && pl->buckets[i].k > kSmallK) continue;
        // round robin over all lanes, or over the side lanes when st carries the tiled groups
        const int span = tiled_in_line ? nside : nside + 1;
        const int l = (tiled_in_line ? 1 : 0) + (next++ % span);
        lane[i] = l;
        used = std::max(used, l);
    }
    hipError_t e = hipSuccess;
    if (used > 0) {
        e = hipEventRecord(pl->fork, st);
        for (int l = 1; l <= used && e == hipSuccess; ++l) e = hipStreamWaitEvent(pl->side[l - 1], pl->fork, 0);
    }
    for (int i = 0; i < nb && e == hipSuccess; ++i) e = fn(pl->buckets[i], lane[i] == 0 ? st : pl->side[lane[i] - 1]);
    // join every forked lane, also after an error, so that the capture ends with no unjoined work
    for (int l = 1; l <= used; ++l) {
        hipError_t j = hipEventRecord(pl->join[l - 1], pl->side[l - 1]);
        if (j == hipSuccess) j = hipStreamWaitEvent(st, pl->join[l - 1], 0);
        if (e == hipSuccess) e = j;
    }
    return e;
}

hipError_t record_forward(fmap_plan *pl, hipStream_t st, bool branch = false)
{
    hipError_t e = launch_copies(pl->d_gf, pl->ngf, st);
    if (e == hipSuccess) e = launch_projections_fwd(pl, pl->grid_fwd, st);
    if (e == hipSuccess)
        e = record_groups(pl, st, branch, true, [&](Bucket &B, hipStream_t s) {
            const int64_t P = (int64_t)B.pairs.size();
            return launch_solve(B.AB, B.AB + (size_t)P * B.k * pl->d, B.evx, B.evy, B.lam, pl->mask_kind, pl->gamma,
                                P, B.k, B.k, pl->d, 0, 0.f, B.C, pl->recompute ? nullptr : B.factors, B.info, nullptr,
                                B.ws, s, B.waves);
        });
    if (e == hipSuccess) e = launch_copies(pl->d_sf, pl->nsf, st);
    return e;
}

hipError_t record_backward(fmap_plan *pl, hipStream_t st, bool branch = false)
{
    hipError_t e = launch_copies(pl->d_gb, pl->ngb, st);
    if (e == hipSuccess)
        e = record_groups(pl, st, branch, false, [&](Bucket &B, hipStream_t s) {
            const int64_t P = (int64_t)B.pairs.size();
            const size_t half = (size_t)P * B.k * pl->d;
            return launch_solve_backward(B.dC, B.AB, B.AB + half, B.C, B.evx, B.evy, B.lam, pl->mask_kind, pl->gamma,
                                         P, B.k, B.k, pl->d, pl->recompute ? nullptr : B.factors, B.dAB, B.dAB + half,
                                         nullptr, nullptr, B.ws, s, B.waves);
        });
    if (e == hipSuccess) e = launch_projections_bwd(pl, pl->grid_bwd, st);
    return e;
}

// Median time (ms) of `reps` runs of fn on st.
template <typename Fn>
float time_ms(hipStream_t st, Fn fn, int reps = 3)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return 1e30f;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return 1e30f;
    }
    (void)hipGetLastError();
    fn();  // warm-up
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();  // a candidate that cannot launch is skipped, and its error cleared
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return 1e30f;
    }
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(a, st);
        fn();
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

#ifndef FMAP_BUILD_ID
#define FMAP_BUILD_ID "unversioned"
#endif

// Cache key: the library build (a hash of its kernel sources), the pass set (forward only, or with a
// backward pass storing or recomputing the factors) and the workload (d, mask, vertex total, k histogram).
std::string signature(const fmap_plan *pl)
{
    int64_t verts = 0;
    for (const fmap_pair &p : pl->pairs) verts += p.n_x + p.n_y;
    char buf[320];
    std::string ks;
    for (const Bucket &B : pl->buckets) ks += std::to_string(B.k) + "x" + std::to_string(B.pairs.size()) + ",";
    const int pass = !pl->has_bwd ? 0 : (pl->recompute ? 2 : 1);
    std::snprintf(buf, sizeof buf, "gfx950 build=%s f32 d=%lld mask=%d pass=%d verts=%lldk pairs=%zu k=",
                  FMAP_BUILD_ID, (long long)pl->d, pl->mask_kind, pass, (long long)(verts / 1000), pl->pairs.size());
    return std::string(buf) + ks;
}

// Line format: "<signature>|chunk grid_fwd rb grid_bwd w_0 w_1 ..." with one row-solve width per k group.
bool cache_lookup(const char *path, const std::string &sig, fmap_plan *pl)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[2048];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        std::string s(line);
        const size_t bar = s.find('|');
        if (bar == std::string::npos || s.substr(0, bar) != sig) continue;
        int c, gfm, rb, gbm, used = 0;
        const char *q = s.c_str() + bar + 1;
        // only values the tuner itself can produce: the partial slots are sized for the smallest chunk
        if (std::sscanf(q, "%d %d %d %d%n", &c, &gfm, &rb, &gbm, &used) != 4 ||
            !(c == 512 || c == 1024 || c == 2048) || gfm < 1 || gfm > 65535 ||
            !(rb == 1 || rb == 2 || rb == 4 || rb == 8) || gbm < 1 || gbm > 65535)
            continue;
        q += used;
        std::vector<int> w(pl->buckets.size());
        bool ok = true;
        for (size_t b = 0; b < w.size() && ok; ++b) {
            ok = std::sscanf(q, "%d%n", &w[b], &used) == 1 && (w[b] == 1 || w[b] == 2 || w[b] == 4);
            q += ok ? used : 0;
        }
        if (!ok) continue;
        pl->chunk = c;
        pl->grid_fwd = gfm;
        pl->rb = rb;
        pl->grid_bwd = gbm;
        for (size_t b = 0; b < w.size(); ++b) pl->buckets[b].waves = w[b];
        found = true;  // the last matching line wins
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &sig, const fmap_plan *pl)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s|%d %d %d %d", sig.c_str(), pl->chunk, pl->grid_fwd, pl->rb, pl->grid_bwd);
    for (const Bucket &B : pl->buckets) std::fprintf(f, " %d", B.waves);
    std::fprintf(f, "\n");
    std::fclose(f);
}

void plan_free(fmap_plan *pl)
{
    if (!pl) return;
    if (pl->ef) (void)hipGraphExecDestroy(pl->ef);
    if (pl->eb) (void)hipGraphExecDestroy(pl->eb);
    if (pl->gf) (void)hipGraphDestroy(pl->gf);
    if (pl->gb) (void)hipGraphDestroy(pl->gb);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    for (hipStream_t q : pl->side) (void)hipStreamDestroy(q);
    for (hipEvent_t ev : pl->join) (void)hipEventDestroy(ev);
    if (pl->fork) (void)hipEventDestroy(pl->fork);
    for (void *p : pl->allocs) (void)hipFree(p);
    delete pl;
}

}  // namespace

extern "C" {

fmap_status fmap_plan_create(const fmap_pair *pairs, int32_t npairs, int64_t d, int32_t mask_kind, float gamma,
                             int32_t bwd_recompute, const char *tune_cache_path, void *stream, fmap_plan **out)
{
    if (!pairs || !out) return FMAP_ERR_NULL;
    *out = nullptr;
    if (npairs < 1 || d < 1 || d > (1 << 20)) return FMAP_ERR_SHAPE;
    if (mask_kind != FMAP_MASK_LAPLACIAN && mask_kind != FMAP_MASK_RESOLVENT) return FMAP_ERR_VALUE;
    if (mask_kind == FMAP_MASK_RESOLVENT && !(gamma > 0.f && gamma < 1e30f)) return FMAP_ERR_VALUE;
    const bool bwd = pairs[0].dC != nullptr;
    for (int i = 0; i < npairs; ++i) {
        const fmap_pair &p = pairs[i];
        if (!p.phi_x || !p.phi_y || !p.mass_x || !p.mass_y || !p.feat_x || !p.feat_y || !p.evals_x || !p.evals_y ||
            !p.lambda || !p.C || !p.info)
            return FMAP_ERR_NULL;
        if ((p.dC != nullptr) != bwd) return FMAP_ERR_NULL;  // all pairs or none take part in the backward
        if (bwd && (!p.dF_x || !p.dF_y)) return FMAP_ERR_NULL;
        if (p.k < 1 || p.n_x < 1 || p.n_y < 1 || p.n_x * p.k >= ((int64_t)1 << 31) || p.n_x * d >= ((int64_t)1 << 31) ||
            p.n_y * p.k >= ((int64_t)1 << 31) || p.n_y * d >= ((int64_t)1 << 31))
            return FMAP_ERR_SHAPE;
        if (p.k > kMaxK) return FMAP_ERR_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    fmap_plan *pl = new fmap_plan();
    pl->pairs.assign(pairs, pairs + npairs);
    pl->d = d;
    pl->mask_kind = mask_kind;
    pl->gamma = gamma;
    pl->recompute = bwd_recompute != 0;
    pl->has_bwd = bwd;
    std::map<int64_t, std::vector<int>> byk;
    for (int i = 0; i < npairs; ++i) byk[pairs[i].k].push_back(i);
    for (auto &kv : byk) {
        Bucket B;
        B.k = kv.first;
        B.pairs = kv.second;
        pl->buckets.push_back(B);
        pl->kmax = std::max(pl->kmax, kv.first);
    }
#define FMAP_TRY(x)                  \
    do {                             \
        if ((x) != hipSuccess) {     \
            plan_free(pl);           \
            return FMAP_ERR_HIP;     \
        }                            \
    } while (0)
    // group buffers
    std::vector<CopyItem> gf, sf, gb;
    for (Bucket &B : pl->buckets) {
        const int64_t P = (int64_t)B.pairs.size(), k = B.k;
        FMAP_TRY(dev_alloc(pl, &B.AB, (size_t)2 * P * k * d));
        FMAP_TRY(dev_alloc(pl, &B.C, (size_t)P * k * k));
        FMAP_TRY(dev_alloc(pl, &B.info, (size_t)P * k));
        FMAP_TRY(dev_alloc(pl, &B.evx, (size_t)P * k));
        FMAP_TRY(dev_alloc(pl, &B.evy, (size_t)P * k));
        FMAP_TRY(dev_alloc(pl, &B.lam, (size_t)P));
        if (!pl->recompute) FMAP_TRY(dev_alloc(pl, &B.factors, (size_t)P * k * (k * (k + 1) / 2)));
        if (bwd) {
            FMAP_TRY(dev_alloc(pl, &B.dC, (size_t)P * k * k));
            FMAP_TRY(dev_alloc(pl, &B.dAB, (size_t)2 * P * k * d));
        }
        FMAP_TRY(dev_alloc(pl, (char **)&B.ws, solve_workspace_layout(P, k, k, d).total));
        for (int q = 0; q < (int)P; ++q) {
            const fmap_pair &p = pairs[B.pairs[q]];
            gf.push_back(words(p.evals_x, B.evx + (size_t)q * k, k));
            gf.push_back(words(p.evals_y, B.evy + (size_t)q * k, k));
            gf.push_back(words(p.lambda, B.lam + q, 1));
            sf.push_back(words(B.C + (size_t)q * k * k, p.C, k * k));
            sf.push_back(words(B.info + (size_t)q * k, p.info, k));
            if (bwd) gb.push_back(words(p.dC, B.dC + (size_t)q * k * k, k * k));
        }
    }
    pl->ngf = (int)gf.size();
    pl->nsf = (int)sf.size();
    pl->ngb = (int)gb.size();
    FMAP_TRY(upload(pl, &pl->d_gf, gf, st));
    FMAP_TRY(upload(pl, &pl->d_sf, sf, st));
    FMAP_TRY(upload(pl, &pl->d_gb, gb, st));

    // partial slots sized for the smallest candidate chunk
    const int chunks[3] = {512, 1024, 2048};
    {
        std::vector<FwdItem> fi, fx, fxs;
        std::vector<RedItem> ri;
        size_t pf = 0;
        build_fwd_items(pl, chunks[0], fi, fx, fxs, ri, &pf);
        FMAP_TRY(dev_alloc(pl, &pl->partials, pf));
    }
    const std::string sig = signature(pl);
    const int cus = device_cus();
    pl->from_cache = cache_lookup(tune_cache_path, sig, pl) ? 1 : 0;

    auto set_fwd = [&](int chunk) -> hipError_t {
        std::vector<FwdItem> fi, fx, fxs;
        std::vector<RedItem> ri;
        size_t pf = 0;
        build_fwd_items(pl, chunk, fi, fx, fxs, ri, &pf);
        pl->nfwd = (int)fi.size();
        pl->nx3 = (int)fx.size();
        pl->nx3s = (int)fxs.size();
        pl->nred = (int)ri.size();
        hipError_t e = upload(pl, &pl->d_fwd, fi, st);
        if (e == hipSuccess) e = upload(pl, &pl->d_x3, fx, st);
        if (e == hipSuccess) e = upload(pl, &pl->d_x3s, fxs, st);
        if (e == hipSuccess) e = upload(pl, &pl->d_red, ri, st);
        return e;
    };
    auto set_bwd = [&](int rb) -> hipError_t {
        std::vector<BwdItem> bi;
        std::vector<McItem> mi;
        build_bwd_items(pl, rb, bi, mi);
        pl->nbwd = (int)bi.size();
        pl->nmc = (int)mi.size();
        hipError_t e = upload(pl, &pl->d_bwd, bi, st);
        if (e == hipSuccess) e = upload(pl, &pl->d_mc, mi, st);
        return e;
    };

    if (!pl->from_cache) {
        // forward projection: vertices per item x persistent grid
        float best = 1e30f;
        int bc = 1024, bg = 2 * cus;
        for (int c : chunks) {
            FMAP_TRY(set_fwd(c));
            for (int gm : {1, 2, 4}) {
                const int g = std::max(1, std::min(gm * cus, pl->nfwd));
                const float t = time_ms(st, [&]() { (void)launch_projections_fwd(pl, g, st); });
                if (t < best) {
                    best = t;
                    bc = c;
                    bg = g;
                }
            }
        }
        pl->chunk = bc;
        pl->grid_fwd = bg;
        // row systems per workgroup of the register row solve, per k group (k <= 64; the tiled solve of
        // larger k runs one system per workgroup)
        FMAP_TRY(set_fwd(pl->chunk));
        FMAP_TRY(launch_copies(pl->d_gf, pl->ngf, st));
        FMAP_TRY(launch_projections_fwd(pl, pl->grid_fwd, st));
        for (Bucket &B : pl->buckets) {
            if (B.k > kSmallK) continue;
            const int64_t P = (int64_t)B.pairs.size();
            best = 1e30f;
            int bw = 4;
            for (int w : {1, 2, 4}) {
                const float t = time_ms(st, [&]() {
                    (void)launch_solve(B.AB, B.AB + (size_t)P * B.k * d, B.evx, B.evy, B.lam, mask_kind, gamma, P, B.k,
                                       B.k, d, 0, 0.f, B.C, B.factors, B.info, nullptr, B.ws, st, w);
                });
                if (t < best) {
                    best = t;
                    bw = w;
                }
            }
            B.waves = bw;
        }
        // backward projection: rows per item x persistent grid
        if (bwd) {
            best = 1e30f;
            int brb = 2, bgb = 2 * cus;
            for (int rb : {1, 2, 4, 8}) {
                FMAP_TRY(set_bwd(rb));
                for (int gm : {1, 2, 4}) {
                    const int g = std::max(1, std::min(gm * cus, std::max(pl->nbwd, 1)));
                    const float t = time_ms(st, [&]() { (void)launch_projections_bwd(pl, g, st); });
                    if (t < best) {
                        best = t;
                        brb = rb;
                        bgb = g;
                    }
                }
            }
            pl->rb = brb;
            pl->grid_bwd = bgb;
        }
        cache_store(tune_cache_path, sig, pl);
    }
    FMAP_TRY(set_fwd(pl->chunk));
    if (bwd) FMAP_TRY(set_bwd(pl->rb));

    // one eager pass (sets up every kernel), then capture both passes
    FMAP_TRY(record_forward(pl, st));
    if (bwd) FMAP_TRY(record_backward(pl, st));
    FMAP_TRY(hipStreamSynchronize(st));
    FMAP_TRY(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking));
    if (pl->buckets.size() > 1) {
        FMAP_TRY(hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming));
        const int nside = std::min<int>((int)pl->buckets.size(), kLanes) - 1;
        for (int l = 0; l < nside; ++l) {
            hipStream_t q = nullptr;
            hipEvent_t ev = nullptr;
            FMAP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
            pl->side.push_back(q);
            FMAP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            pl->join.push_back(ev);
        }
    }
    FMAP_TRY(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
    hipError_t rec = record_forward(pl, pl->cap, true);
    hipError_t endc = hipStreamEndCapture(pl->cap, &pl->gf);
    FMAP_TRY(rec);
    FMAP_TRY(endc);
    FMAP_TRY(hipGraphInstantiate(&pl->ef, pl->gf, nullptr, nullptr, 0));
    if (bwd) {
        FMAP_TRY(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
        rec = record_backward(pl, pl->cap, true);
        endc = hipStreamEndCapture(pl->cap, &pl->gb);
        FMAP_TRY(rec);
        FMAP_TRY(endc);
        FMAP_TRY(hipGraphInstantiate(&pl->eb, pl->gb, nullptr, nullptr, 0));
    }
#undef FMAP_TRY
    *out = pl;
    return FMAP_OK;
}

fmap_status fmap_plan_forward(fmap_plan *plan, void *stream)
{
    if (!plan || !plan->ef) return FMAP_ERR_NULL;
    return hipGraphLaunch(plan->ef, (hipStream_t)stream) == hipSuccess ? FMAP_OK : FMAP_ERR_HIP;
}

fmap_status fmap_plan_backward(fmap_plan *plan, void *stream)
{
    if (!plan) return FMAP_ERR_NULL;
    if (!plan->eb) return FMAP_ERR_UNSUPPORTED;  // created without dC
    return hipGraphLaunch(plan->eb, (hipStream_t)stream) == hipSuccess ? FMAP_OK : FMAP_ERR_HIP;
}

fmap_status fmap_plan_tuning(const fmap_plan *plan, int32_t *chunk, int32_t *grid, int32_t *systems_per_wg,
                             int32_t *from_cache)
{
    if (!plan) return FMAP_ERR_NULL;
    if (chunk) *chunk = plan->chunk;
    if (grid) *grid = plan->grid_fwd;
    if (systems_per_wg) {
        *systems_per_wg = 4;
        for (const Bucket &B : plan->buckets)
            if (B.k <= kSmallK) {
                *systems_per_wg = B.waves;
                break;
            }
    }
    if (from_cache) *from_cache = plan->from_cache;
    return FMAP_OK;
}

fmap_status fmap_plan_groups(const fmap_plan *plan, int32_t *groups)
{
    if (!plan) return FMAP_ERR_NULL;
    if (groups) *groups = (int32_t)plan->buckets.size();
    return FMAP_OK;
}

fmap_status fmap_plan_group(const fmap_plan *plan, int32_t g, int32_t *k, int32_t *npairs, int32_t *systems_per_wg)
{
    if (!plan) return FMAP_ERR_NULL;
    if (g < 0 || g >= (int32_t)plan->buckets.size()) return FMAP_ERR_VALUE;
    const Bucket &B = plan->buckets[(size_t)g];
    if (k) *k = (int32_t)B.k;
    if (npairs) *npairs = (int32_t)B.pairs.size();
    if (systems_per_wg) *systems_per_wg = B.k <= kSmallK ? B.waves : 1;
    return FMAP_OK;
}

fmap_status fmap_plan_destroy(fmap_plan *plan)
{
    if (!plan) return FMAP_ERR_NULL;
    plan_free(plan);
    return FMAP_OK;
}

}  // extern "C"

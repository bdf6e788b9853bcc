// fmap_project without any allocation: the split-K partial sums go to a
// file-scope device array instead of a caller workspace, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// `scratch` is a device symbol: in host code its name is only a stand-in, so
// its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and that address, never the name, is handed to
// the kernels.  Every call on one device shares that device's array, and the
// array keeps the last call's contents; the projection writes every partial
// slot before the fixed-order reduction reads it, so nothing has to start at
// zero.  Calls that overlap in time on one device (different streams or host
// threads) race on the array.
#include "../../include/fmap.h"

#include <mutex>

#include "fmap_launch.h"

namespace {

constexpr size_t kScratchBytes = (size_t)FMAP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

std::mutex g_mutex;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's `scratch` (looked up on the first call per device).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" fmap_status fmap_project_noalloc(const void *phi, const float *mass, const void *feat, int32_t in_dtype,
                                            int64_t batch, int64_t n, int64_t k, int64_t d, float *A, void *stream)
{
    if (!phi || !mass || !feat || !A) return FMAP_ERR_NULL;
    if (in_dtype != FMAP_F32 && in_dtype != FMAP_BF16) return FMAP_ERR_DTYPE;
    const int64_t lim = (int64_t)1 << 30;
    if (batch < 1 || n < 1 || k < 1 || d < 1 || batch >= lim || n >= lim || k >= lim || d >= lim)
        return FMAP_ERR_SHAPE;
    if (n * k > ((int64_t)1 << 31) || n * d > ((int64_t)1 << 31)) return FMAP_ERR_SHAPE;
    const size_t need = fmap::project_workspace_bytes(batch, n, k, d, in_dtype);
    if (need > kScratchBytes) return FMAP_ERR_WORKSPACE;
    void *ws = nullptr;
    if (need > 0 && scratch_address(&ws) != hipSuccess) return FMAP_ERR_HIP;
    return fmap::launch_project(phi, mass, feat, in_dtype, batch, n, k, d, A, ws, (hipStream_t)stream) == hipSuccess
               ? FMAP_OK
               : FMAP_ERR_HIP;
}

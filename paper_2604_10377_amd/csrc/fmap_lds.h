// Helpers of the direct global->LDS load pipelines (gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace fmap {

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

__device__ __forceinline__ void dma16(const float *g, float *lds_base)
{
    __builtin_amdgcn_global_load_lds((glb_void_t *)g, (lds_void_t *)lds_base, 16, 0, 0);
}

// The same with the streaming (non-temporal) cache policy, for data read once.
__device__ __forceinline__ void dma16_stream(const float *g, float *lds_base)
{
    __builtin_amdgcn_global_load_lds((glb_void_t *)g, (lds_void_t *)lds_base, 16, 0, 2);
}

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Workgroup barrier for the LDS pipelines: waits for this wave's LDS operations
// only (lgkmcnt), not for the direct global->LDS loads still in flight for later
// stages (a __syncthreads() would drain vmcnt and serialise the pipeline).  The
// loads of the stage about to be read were retired by an explicit vmcnt wait
// before the barrier.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt unconstrained
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

}  // namespace fmap

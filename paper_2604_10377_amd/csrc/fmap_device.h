// Device-side helpers shared by the libfmap kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmap {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// A pointer read from a work-item table in device memory carries no address
// space, so accesses through it compile to flat instructions, which count on
// both the vector-memory and the LDS counters and make every use of a load wait
// for all outstanding memory operations.  The tables hold global addresses
// only: rebuilding them as global pointers (from the integer address, which the
// compiler cannot fold back into the generic pointer) restores global loads and
// stores, and with them per-load waits.
template <typename T> __device__ __forceinline__ T *global_ptr(T *p)
{
    return (T *)((__attribute__((address_space(1))) T *)(uintptr_t)p);
}

// One 32x32x2 float32 matrix-core step.  Operand layout (lane l, wave64):
//   a = X[m = l % 32][kk = l / 32],  b = Y[kk = l / 32][n = l % 32],
//   accumulator register r of lane l holds D[acc32_row(r, l)][l % 32].
__device__ __forceinline__ f32x16 mfma32x32x2(float a, float b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int acc32_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ f32x16 zero16()
{
    f32x16 z;
#pragma unroll
    for (int i = 0; i < 16; ++i) z[i] = 0.f;
    return z;
}

// Strided loop e = start, start + stride, ... < end whose body loads one value
// and consumes it (e.g. staging into LDS).  Written as a plain loop, the
// compiler waits for each load before the next one is issued, one memory round
// trip per iteration.  Here U loads are issued from clamped indices before any
// is consumed, so a loop of N iterations costs N / U round trips.
template <int U, typename Load, typename Use>
__device__ __forceinline__ void batched_for(int start, int end, int stride, Load load, Use use)
{
    for (int e0 = start; e0 < end; e0 += U * stride) {
        decltype(load(0)) v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = load(min(e0 + u * stride, end - 1));
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u * stride < end) use(e0 + u * stride, v[u]);
    }
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the 64 lanes, returned wave-uniform.  Within each 16-lane row the DPP steps
// (xor 1, xor 2 via quad permutes, then rotations by 4 and 8) leave the row sum in every lane;
// the four row sums are combined with readlanes.  No LDS round trips, unlike a shuffle butterfly.
__device__ __forceinline__ float wave_sum_uniform(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xF, 0xF, false));  // row_ror:4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, false));  // row_ror:8
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float readlane(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// v_writelane: lane `lane` of `old` takes the wave-uniform `src`, the other lanes keep theirs (the LLVM
// intrinsic, which this compiler exposes under no builtin name)
__device__ int amdgcn_writelane_i32(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ float writelane(float src, int lane, float old)
{
    return __int_as_float(amdgcn_writelane_i32(__float_as_int(src), lane, __float_as_int(old)));
}

// bfloat16 bit pattern -> float (exact).
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Penalty mask entry for one (target i, source j) eigenvalue pair.
//   kind 0 (Laplacian): (mu_y - mu_x)^2
//   kind 1 (resolvent): |r(mu_y) - r(mu_x)|^2 with r(mu) = 1/(a - i),
//   a = (max(mu,0) * inv_scale)^gamma.
struct MaskParams {
    int kind;
    float gamma;
    float inv_scale;
};

__device__ __forceinline__ void resolvent_point(float mu, const MaskParams &m, float &re, float &im)
{
    const float t = fmaxf(mu, 0.f) * m.inv_scale;
    const float a = (m.gamma == 0.5f) ? sqrtf(t) : powf(t, m.gamma);
    const float den = 1.f / (1.f + a * a);
    re = a * den;
    im = den;
}

__device__ __forceinline__ float mask_entry(float mu_y, float mu_x, const MaskParams &m)
{
    if (m.kind == 0) {
        const float t = mu_y - mu_x;
        return t * t;
    }
    float ry, iy, rx, ix;
    resolvent_point(mu_y, m, ry, iy);
    resolvent_point(mu_x, m, rx, ix);
    const float a = ry - rx, b = iy - ix;
    return a * a + b * b;
}

}  // namespace fmap

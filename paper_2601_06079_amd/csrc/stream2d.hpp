// stream2d.hpp -- helpers of the row-streaming 2-D kernels (one 64-lane
// wavefront per strip of columns, rows marched through registers).
#pragma once
#include "device.hpp"

namespace pfk {
namespace {

// raw buffer access: the row offset is a scalar (one SGPR), the column offset
// a per-lane VGPR set once, so no per-row address arithmetic runs on the VALU.
// Out-of-range addresses read 0 and drop stores (the launcher keeps every
// access in range; this is the hardware's own bounds check on top).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __hiloint2double((int)v.y, (int)v.x);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    v2u w;
    w.x = (unsigned)__double2loint(v);
    w.y = (unsigned)__double2hiint(v);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, voff, soff, 0);
}

// wave index made provably uniform so that all row bookkeeping stays scalar
__device__ __forceinline__ int uniform_wave()
{
    return (int)(blockIdx.x * (blockDim.x / WAVE)) +
           __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
}

}  // namespace
}  // namespace pfk

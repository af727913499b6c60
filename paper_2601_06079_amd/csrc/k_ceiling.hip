// k_ceiling.hip -- the two practical ceilings the stencil kernels are measured
// against:
//   - pf_stream_copy: a device-to-device copy with one 16-byte load and store per
//     thread over a grid that covers the buffer (every wave has its loads in flight
//     at once; on MI355X this beat grid-stride loops of 1-4 vectors per thread and
//     8-vector blocks: 6.25 TB/s for 1 GiB);
//   - pf_fma_probe: independent non-packed FP32 FMA chains, the VALU issue rate a
//     kernel of plain FP32 arithmetic can reach.
#include <hip/hip_runtime.h>

#include "api_internal.hpp"

namespace {

constexpr int CB = 256;  // threads per block

__global__ __launch_bounds__(CB) void k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    long long n4)
{
    const long long i = (long long)blockIdx.x * CB + threadIdx.x;
    if (i < n4) dst[i] = src[i];
}

// Eight independent FMA chains per thread, `iters` rounds: 16 * iters flops per
// thread.  Each thread writes the sum of its chains, so nothing is dead code.
constexpr int FMA_CHAINS = 8;
__global__ __launch_bounds__(CB) void k_fma_probe(float* __restrict__ out, float a, float b, int iters)
{
    float x[FMA_CHAINS];
#pragma unroll
    for (int c = 0; c < FMA_CHAINS; ++c) x[c] = threadIdx.x * 1e-3f + c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < FMA_CHAINS; ++c) x[c] = __builtin_fmaf(x[c], a, b);
    }
    float s = 0;
#pragma unroll
    for (int c = 0; c < FMA_CHAINS; ++c) s += x[c];
    out[(long long)blockIdx.x * CB + threadIdx.x] = s;
}

}  // namespace

using namespace pfapi;

extern "C" int pf_stream_copy(pf_ctx* ctx, const void* src, void* dst, size_t bytes, void* stream)
{
    return guarded("pf_stream_copy", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (!src || !dst) return fail(PF_EINVAL, "NULL pointer argument");
        if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || bytes % 16)
            return fail(PF_EINVAL, "src, dst and bytes must be multiples of 16");
        const char* s0 = static_cast<const char*>(src);
        const char* d0 = static_cast<const char*>(dst);
        if (s0 < d0 + bytes && d0 < s0 + bytes) return fail(PF_EINVAL, "src and dst overlap");
        const long long n4 = (long long)(bytes / 16);
        const long long blocks = (n4 + CB - 1) / CB;
        if (blocks > 0x7fffffffLL) return fail(PF_EINVAL, "copy of %zu bytes exceeds one launch", bytes);
        if (int rc = require_device(ctx)) return rc;
        if (n4 == 0) return PF_OK;
        k_stream_copy<<<(unsigned)blocks, CB, 0, (hipStream_t)stream>>>(static_cast<const float4*>(src),
                                                                       static_cast<float4*>(dst), n4);
        return check_launch("pf_stream_copy");
    });
}

extern "C" int pf_fma_probe(pf_ctx* ctx, int blocks, int iters, float* out, void* stream)
{
    return guarded("pf_fma_probe", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (!out || reinterpret_cast<uintptr_t>(out) % 4) return fail(PF_EINVAL, "out is NULL or misaligned");
        if (blocks < 1 || iters < 1) return fail(PF_EINVAL, "blocks and iters must be positive");
        if (int rc = require_device(ctx)) return rc;
        k_fma_probe<<<blocks, CB, 0, (hipStream_t)stream>>>(out, 0.999f, 1e-4f, iters);
        return check_launch("pf_fma_probe");
    });
}

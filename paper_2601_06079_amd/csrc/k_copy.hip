// k_copy.hip -- device-to-device copy with 16-byte loads and stores: the
// practical HBM ceiling the stencil kernels' bandwidth is compared with.
//
// Each thread moves four 16-byte vectors per round, loads issued before stores,
// over a grid of a few resident blocks per CU that strides through the buffer.
#include <hip/hip_runtime.h>

#include "api_internal.hpp"

namespace {

constexpr int CB = 256;  // threads per block

__global__ __launch_bounds__(CB) void k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    long long n4)
{
    const long long stride = (long long)gridDim.x * CB;
    long long i = (long long)blockIdx.x * CB + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n4; i += stride) dst[i] = src[i];
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
        if (int rc = require_device(ctx)) return rc;
        const long long n4 = (long long)(bytes / 16);
        if (n4 == 0) return PF_OK;
        const long long want = (n4 + CB - 1) / CB;
        const long long cap = 8LL * ctx->cus;  // eight resident blocks per CU
        const unsigned blocks = (unsigned)(want < cap ? want : cap);
        k_stream_copy<<<blocks, CB, 0, (hipStream_t)stream>>>(static_cast<const float4*>(src),
                                                              static_cast<float4*>(dst), n4);
        return check_launch("pf_stream_copy");
    });
}

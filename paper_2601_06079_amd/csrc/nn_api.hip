// nn_api.hip -- C ABI of the convolutional surrogate and of its residual check.
#include <cmath>
#include <cstring>

#include "api_internal.hpp"
#include "krylov.hpp"
#include "nn.hpp"

namespace pfapi {
namespace {

inline size_t al(size_t b) { return (b + 255) & ~size_t(255); }

struct NNWS {
    unsigned short *a0, *a1, *a2, *a3, *ga, *gb, *frag, *w4;
    float *d, *chat, *g, *r2, *part, *partb, *tile;
    double *spart, *mean, *mean2;
    size_t bytes;
};

NNWS nn_layout(int B, int H, int W, void* base)
{
    NNWS L{};
    char* c = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t b) {
        char* r = c ? c + off : nullptr;
        off += al(b);
        return r;
    };
    const size_t P = (size_t)B * H * W;
    const pfk::NNFragOffsets fo = pfk::nn_frag_offsets();
    L.a0 = (unsigned short*)take(P * 16 * 2);
    L.a1 = (unsigned short*)take(P * 32 * 2);
    L.a2 = (unsigned short*)take(P * 32 * 2);
    L.a3 = (unsigned short*)take(P * 32 * 2);
    L.ga = (unsigned short*)take(P * 32 * 2);
    L.gb = (unsigned short*)take(P * 32 * 2);
    L.frag = (unsigned short*)take((size_t)fo.total * 2);
    L.w4 = (unsigned short*)take(9 * 32 * 2);
    L.d = (float*)take(P * 4);
    L.chat = (float*)take(P * 4);
    L.g = (float*)take(P * 4);
    L.r2 = (float*)take(P * 4);
    const size_t nwg = (size_t)pfk::nn_wgrad_blocks(B, H, W), nog = (size_t)pfk::nn_out_wgrad_blocks(B, H, W);
    L.part = (float*)take(std::max(nwg * 9 * 32 * 32, nog * 289) * 4);
    L.partb = (float*)take(nwg * 32 * 4);
    L.tile = (float*)take(9 * 32 * 32 * 4);
    const size_t nbs = ((size_t)H * W + 255) / 256;
    L.spart = (double*)take((size_t)B * nbs * 3 * 8);
    L.mean = (double*)take((size_t)B * 8);
    L.mean2 = (double*)take((size_t)B * 8);
    L.bytes = off;
    return L;
}

int check_shape(int B, int H, int W)
{
    if (B < 1 || H < 1 || W < 32) return fail(PF_EINVAL, "need B >= 1, H >= 1, W >= 32");
    if (W % 32) return fail(PF_EINVAL, "W must be a multiple of 32 (got %d)", W);
    if ((long long)B * H * W >= (1ll << 31) / 64) return fail(PF_EINVAL, "batch too large");
    return PF_OK;
}

// the forward pass (the weight fragments already prepared in L.frag, L.w4) into
// chat; training (keep_a0) leaves a0..a3 and d in the workspace
void forward(const float* params, int B, int H, int W, const float* c, const float* M,
             const float* kappa, const float* target, float* chat, NNWS& L, hipStream_t s, bool keep_a0)
{
    const pfk::NNOffsets o = pfk::nn_offsets();
    const pfk::NNFragOffsets fo = pfk::nn_frag_offsets();
    const int HW = H * W;
    if (keep_a0) {  // training: the weight gradients read a0, a1, a2 and a3
        pfk::nn_pack_input(c, M, kappa, L.a0, B, HW, s);
        pfk::nn_conv(1, 0, L.a0, L.frag + fo.f1, params + o.b1, nullptr, L.a1, B, H, W, s);
        pfk::nn_conv(2, 0, L.a1, L.frag + fo.f2, params + o.b2, nullptr, L.a2, B, H, W, s);
        pfk::nn_conv(3, 0, L.a2, L.frag + fo.f3, params + o.b3, nullptr, L.a3, B, H, W, s);
        pfk::nn_out_fwd(L.a3, L.w4, params, L.d, B, H, W, s);
        pfk::nn_sample_mean(L.d, L.spart, L.mean, B, HW, s);
    } else {
        // inference: the first layer runs inside the second's tiles (a1 is never
        // stored), and the output layer's channel sums leave the third as 9 tap planes
        pfk::nn_conv12_planes(c, M, kappa, params + o.w1, params + o.b1, L.frag + fo.f2, params + o.b2, L.a2, B,
                              H, W, s);
        float* P = reinterpret_cast<float*>(L.a3);  // 36 of a3's 64 bytes per pixel
        pfk::nn_conv3_taps(L.a2, L.frag + fo.f3, params + o.b3, L.w4, P, B, H, W, s);
        pfk::nn_out_taps_project(P, params, c, L.d, L.spart, L.mean, chat, B, H, W, s);
        return;
    }
    pfk::nn_project(c, L.d, L.mean, target, chat, L.g, L.r2, B, HW, s);
}

}  // namespace
}  // namespace pfapi

using namespace pfapi;

extern "C" {

int pf_nn_param_count(void) { return pfk::nn_offsets().total; }

int pf_nn_workspace_size(int B, int H, int W, size_t* bytes)
{
    return guarded("pf_nn_workspace_size", [&]() -> int {
        if (int rc = check_shape(B, H, W)) return rc;
        if (!bytes) return fail(PF_EINVAL, "bytes is NULL");
        *bytes = nn_layout(B, H, W, nullptr).bytes;
        return PF_OK;
    });
}

int pf_nn_forward(const float* params, int B, int H, int W, const float* c, const float* M,
                  const float* kappa, float* chat, void* ws, void* stream)
{
    return guarded("pf_nn_forward", [&]() -> int {
        if (int rc = check_shape(B, H, W)) return rc;
        if (!params || !c || !M || !kappa || !chat || !ws) return fail(PF_EINVAL, "NULL pointer argument");
        if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws must be 256-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        NNWS L = nn_layout(B, H, W, ws);
        // Groups of samples whose 32-channel BF16 activation (64 B per pixel) stays
        // within 128 MiB, so that a layer's input and output share the 256 MB Infinity
        // Cache (measured on MI355X for 16 x 512^2: 0.477 ms in groups of 8 against
        // 0.495 ms in one; groups of 4 or fewer leave the matrix cores short of work).
        // Every group runs the same per-sample kernels, so the result does not depend
        // on the grouping.
        const long long HW = (long long)H * W;
        int G = pfk::tune_nn_group();
        if (G <= 0) G = (int)std::max<long long>(1, (128ll << 20) / (HW * 64));
        G = std::min(G, B);
        pfk::nn_prep_weights(params, L.frag, L.w4, s);
        for (int b0 = 0; b0 < B; b0 += G) {
            const int nb = std::min(G, B - b0);
            const long long o = (long long)b0 * HW;
            // c and chat are B x H x W; M and kappa hold one value per sample
            forward(params, nb, H, W, c + o, M + b0, kappa + b0, nullptr, chat + o, L, s, false);
        }
        return check_launch("pf_nn_forward");
    });
}

int pf_nn_backward(const float* params, int B, int H, int W, const float* c, const float* M,
                   const float* kappa, const float* target, double* loss, float* grad, void* ws,
                   void* stream)
{
    return guarded("pf_nn_backward", [&]() -> int {
        if (int rc = check_shape(B, H, W)) return rc;
        if (!params || !c || !M || !kappa || !target || !grad || !ws)
            return fail(PF_EINVAL, "NULL pointer argument");
        if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws must be 256-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        NNWS L = nn_layout(B, H, W, ws);
        const pfk::NNOffsets o = pfk::nn_offsets();
        const pfk::NNFragOffsets fo = pfk::nn_frag_offsets();
        const int HW = H * W;
        pfk::nn_prep_weights(params, L.frag, L.w4, s);
        forward(params, B, H, W, c, M, kappa, target, L.chat, L, s, true);
        if (loss) pfk::nn_sample_mean(L.r2, L.spart, loss, B, HW, s);  // per-sample MSE
        // backward of the mass projection: g <- g - mean(g)
        pfk::nn_sample_mean(L.g, L.spart, L.mean2, B, HW, s);
        pfk::nn_center(L.g, L.mean2, B, HW, s);
        // output layer
        pfk::nn_out_bwd(L.a3, L.w4, L.g, L.ga, L.part, B, H, W, s);
        pfk::nn_sum_partials(L.part, pfk::nn_out_wgrad_blocks(B, H, W), 289, grad + o.w4, s);
        const int nwg = pfk::nn_wgrad_blocks(B, H, W);
        // layer 3: ga = d pre3
        pfk::nn_wgrad(3, L.a2, L.ga, L.part, L.partb, B, H, W, s);
        pfk::nn_sum_partials(L.part, nwg, 9 * 32 * 32, grad + o.w3, s);
        pfk::nn_sum_partials(L.partb, nwg, 32, grad + o.b3, s);
        pfk::nn_conv(3, 1, L.ga, L.frag + fo.d3, nullptr, L.a2, L.gb, B, H, W, s);  // gb = d pre2
        // layer 2
        pfk::nn_wgrad(2, L.a1, L.gb, L.part, L.partb, B, H, W, s);
        pfk::nn_sum_partials(L.part, nwg, 9 * 32 * 32, grad + o.w2, s);
        pfk::nn_sum_partials(L.partb, nwg, 32, grad + o.b2, s);
        pfk::nn_conv(2, 1, L.gb, L.frag + fo.d2, nullptr, L.a1, L.ga, B, H, W, s);  // ga = d pre1
        // layer 1 (input channels padded 3 -> 16)
        pfk::nn_wgrad(1, L.a0, L.ga, L.part, L.partb, B, H, W, s);
        pfk::nn_sum_partials(L.part, nwg, 9 * 32 * 32, L.tile, s);
        pfk::nn_extract_w1(L.tile, grad + o.w1, s);
        pfk::nn_sum_partials(L.partb, nwg, 32, grad + o.b1, s);
        return check_launch("pf_nn_backward");
    });
}

int pf_nn_check(int B, int H, int W, const float* chat, const float* c_prev, const float* c_step,
                double K_dt, double dt, double* out, void* ws, void* stream)
{
    return guarded("pf_nn_check", [&]() -> int {
        if (int rc = check_shape(B, H, W)) return rc;
        if (!chat || !c_prev || !c_step || !out || !ws) return fail(PF_EINVAL, "NULL pointer argument");
        if (!(K_dt > 0.0) || !(dt > 0.0)) return fail(PF_EINVAL, "K_dt and dt must be > 0");
        NNWS L = nn_layout(B, H, W, ws);
        pfk::nn_check(chat, c_prev, c_step, B, H * W, K_dt, dt, L.spart, out, (hipStream_t)stream);
        return check_launch("pf_nn_check");
    });
}

int pf_nn_adam(float* params, float* m, float* v, const float* grad, int t, double lr, double beta1,
               double beta2, double eps, void* stream)
{
    return guarded("pf_nn_adam", [&]() -> int {
        if (!params || !m || !v || !grad) return fail(PF_EINVAL, "NULL pointer argument");
        if (t < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
            !(eps > 0.0))
            return fail(PF_EINVAL, "bad Adam hyper-parameters");
        pfk::nn_adam(params, m, v, grad, pfk::nn_offsets().total, t, lr, beta1, beta2, eps,
                     (hipStream_t)stream);
        return check_launch("pf_nn_adam");
    });
}

}  // extern "C"

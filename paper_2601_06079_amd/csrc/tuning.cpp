// tuning.cpp -- launch-shape choices for the fused 2-D explicit kernel.
//
// The kernel's cost is VALU issue on each SIMD: a wave marching ty rows costs
// about (ty + 2H) row-steps, and waves that land on the same SIMD serialise.
// With W waves spread over the S SIMDs of the device, the busiest SIMD runs
// ceil(W / S) waves, so the step time is proportional to
//     ceil(W(ty) / S) * (ty + 2H),   W(ty) = strips * ceil(ny / ty).
// The chooser minimises that over ty; pf_tune_set overrides it.
#include <atomic>
#include <mutex>

#include "api_internal.hpp"

namespace pfapi {
namespace {
std::atomic<int> g_rows_override{0};
std::atomic<int> g_depth_override{0};
int g_simds = -1;
std::mutex g_mu;

int device_simds()
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_simds < 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                v > 0)
                cus = v;
        }
        g_simds = 4 * cus;
    }
    return g_simds;
}
}  // namespace

int stream2d_rows(const pf_problem* p)
{
    const int ov = g_rows_override.load();
    if (ov > 0) return ov;
    const int H = p->model == PF_CAHN_HILLIARD ? 2 : 1;
    const long long nx = p->n[0], ny = p->n[1];
    const long long strips = (nx + (64 - 2 * H) - 1) / (64 - 2 * H);
    const long long S = device_simds();
    long long best_ty = 32, best_cost = -1;
    for (long long ty = 8; ty <= ny; ++ty) {
        const long long W = strips * ((ny + ty - 1) / ty);
        const long long cost = ((W + S - 1) / S) * (ty + 2 * H);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best_ty = ty;
        }
        if (ty > 8 && (ny + ty - 1) / ty == 1) break;
    }
    if (ny < 8) best_ty = ny;
    return (int)best_ty;
}

int stream2d_depth(const pf_problem* p)
{
    (void)p;
    const int ov = g_depth_override.load();
    return ov > 0 ? ov : 32;
}

}  // namespace pfapi

using namespace pfapi;
extern "C" {
int pf_tune_set(int key, int value)
{
    if (value < 0) return fail(PF_EINVAL, "tuning value must be >= 0");
    if (key == PF_TUNE_STREAM2D_ROWS)
        g_rows_override.store(value);
    else if (key == PF_TUNE_STREAM2D_DEPTH)
        g_depth_override.store(value);
    else
        return fail(PF_EINVAL, "unknown tuning key %d", key);
    return PF_OK;
}
int pf_tune_get(int key, int* value)
{
    if (!value) return fail(PF_EINVAL, "value is NULL");
    if (key == PF_TUNE_STREAM2D_ROWS)
        *value = g_rows_override.load();
    else if (key == PF_TUNE_STREAM2D_DEPTH)
        *value = g_depth_override.load();
    else
        return fail(PF_EINVAL, "unknown tuning key %d", key);
    return PF_OK;
}
}

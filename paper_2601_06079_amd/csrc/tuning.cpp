// tuning.cpp -- launch-shape choices for the fused 2-D explicit kernel:
// rows per wavefront (chunk length) and prefetch depth.  Defaults come from
// measurements on MI355X; pf_tune_set overrides them (the autotuner uses it).
#include <algorithm>
#include <atomic>

#include "api_internal.hpp"

namespace pfapi {
namespace {
std::atomic<int> g_rows_override{0};
std::atomic<int> g_depth_override{0};
std::atomic<int> g_fuse_override{0};
std::atomic<int> g_jvp3d_planes{0};
std::atomic<int> g_el_planes{0};
std::atomic<int> g_el_mg{0};
std::atomic<int> g_seam{0};
std::atomic<int> g_nn_group{0};
std::atomic<int> g_gs_reorth{0};
std::atomic<int> g_gg_stream{0};
std::atomic<int> g_jvp2d_stream{0};
}  // namespace

int stream2d_fuse(const pf_problem* p)
{
    const int ov = g_fuse_override.load();
    if (ov > 0) return std::min(ov, 4);
    // Measured on MI355X: four fused steps are fastest for Allen-Cahn from 128^2 to
    // 2048^2 (128^2 FP64: 1.9 against 2.4 us/step for two; 2048^2: 5.8 against 6.8) and
    // for Cahn-Hilliard below 2048^2, where launches dominate; at 2048^2 and above
    // Cahn-Hilliard on the seam-sharing kernel is fastest with three or four (7.7
    // us/step at 2048^2; two: 8.1, and 10% slower than three at 8192^2).  With nodal
    // quadrature the step is a third of the arithmetic and four are fastest there too
    // (2048^2: 3.9 us/step; three 4.1, two 4.9).
    if (p->model == PF_CAHN_HILLIARD && p->quad == PF_QUAD_GAUSS && p->n[0] * p->n[1] >= (1ll << 22))
        return 3;
    return 4;
}

int stream2d_rows(const pf_problem* p, int ks, int cus)
{
    const int ov = g_rows_override.load();
    if (ov > 0) return ov;
    const int HK = (p->model == PF_ALLEN_CAHN ? 1 : 2) * ks;  // Cahn-Hilliard and coupled: 2 per step
    const long long nx = p->n[0], ny = p->n[1];
    const long long strips = (nx + (64 - 2 * HK) - 1) / (64 - 2 * HK);
    const long long S = 4LL * (cus > 0 ? cus : 256);  // SIMDs
    // The launch splits each strip into balanced chunks (sizes differ by at most
    // one row).  Measured on MI355X: enough chunks for about four waves per SIMD
    // hide latency, and stopping just below a whole number of waves per SIMD
    // avoids a partly filled last round.  Chunks are never shorter than 8 rows.
    // Longer chunks mean a grid of many rounds, where the measured best is 32
    // rows for single steps and 48 for fused ones.
    // (coupled model: six, measured at 512^2..2048^2; its pipeline is VALU-bound and
    // light on registers)
    const long long waves = p->model == PF_COUPLED ? 6 : 4;
    long long nch = std::max<long long>(1, waves * S / strips);
    // periodic fused launches run on the seam-sharing kernel, which rounds the chunks
    // up to whole workgroups of 4: round down here so that the total stays in one round
    if (!p->bc && ks >= 2 && p->model != PF_COUPLED) nch = std::max<long long>(4, nch / 4 * 4);
    nch = std::min(nch, std::max<long long>(1, ny / 8));
    long long ty = (ny + nch - 1) / nch;
    const long long tmax = ks == 1 ? 32 : 48;
    if (ty > tmax) ty = tmax;
    return (int)std::max<long long>(ty, 1);
}

int stream2d_depth(const pf_problem* p)
{
    (void)p;
    const int ov = g_depth_override.load();
    return ov > 0 ? ov : 4;
}

}  // namespace pfapi

namespace pfk {
int tune_jvp3d_planes() { return pfapi::g_jvp3d_planes.load(); }
int tune_el_planes() { return pfapi::g_el_planes.load(); }
int tune_el_mg() { return pfapi::g_el_mg.load(); }
int tune_stream2d_seam() { return pfapi::g_seam.load(); }
int tune_nn_group() { return pfapi::g_nn_group.load(); }
int tune_gs_reorth() { return pfapi::g_gs_reorth.load(); }
int tune_gg_stream() { return pfapi::g_gg_stream.load(); }
int tune_jvp2d_stream() { return pfapi::g_jvp2d_stream.load(); }
int tune_stream2d_rows() { return pfapi::g_rows_override.load(); }
}  // namespace pfk

using namespace pfapi;
extern "C" {
int pf_tune_set(int key, int value)
{
    if (value < 0) return fail(PF_EINVAL, "tuning value must be >= 0");
    if (key == PF_TUNE_STREAM2D_ROWS)
        g_rows_override.store(value);
    else if (key == PF_TUNE_STREAM2D_DEPTH)
        g_depth_override.store(value);
    else if (key == PF_TUNE_STREAM2D_FUSE)
        g_fuse_override.store(value);
    else if (key == PF_TUNE_JVP3D_PLANES)
        g_jvp3d_planes.store(value);
    else if (key == PF_TUNE_EL_PLANES)
        g_el_planes.store(value);
    else if (key == PF_TUNE_EL_MG)
        g_el_mg.store(value);
    else if (key == PF_TUNE_STREAM2D_SEAM)
        g_seam.store(value);
    else if (key == PF_TUNE_NN_GROUP)
        g_nn_group.store(value);
    else if (key == PF_TUNE_GS_REORTH)
        g_gs_reorth.store(value);
    else if (key == PF_TUNE_GG_STREAM)
        g_gg_stream.store(value);
    else if (key == PF_TUNE_JVP2D_STREAM)
        g_jvp2d_stream.store(value);
    else
        return fail(PF_EINVAL, "unknown tuning key %d", key);
    return PF_OK;
}
int pf_launch_shape(const pf_ctx* ctx, const pf_problem* p, int* ks, int* ty, int* depth)
{
    return guarded("pf_launch_shape", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (!ks || !ty || !depth) return fail(PF_EINVAL, "NULL output pointer");
        *ks = stream2d_fuse(p);
        *ty = stream2d_rows(p, *ks, ctx->cus);
        *depth = stream2d_depth(p);
        return PF_OK;
    });
}

int pf_tune_get(int key, int* value)
{
    if (!value) return fail(PF_EINVAL, "value is NULL");
    if (key == PF_TUNE_STREAM2D_ROWS)
        *value = g_rows_override.load();
    else if (key == PF_TUNE_STREAM2D_DEPTH)
        *value = g_depth_override.load();
    else if (key == PF_TUNE_STREAM2D_FUSE)
        *value = g_fuse_override.load();
    else if (key == PF_TUNE_JVP3D_PLANES)
        *value = g_jvp3d_planes.load();
    else if (key == PF_TUNE_EL_PLANES)
        *value = g_el_planes.load();
    else if (key == PF_TUNE_EL_MG)
        *value = g_el_mg.load();
    else if (key == PF_TUNE_STREAM2D_SEAM)
        *value = g_seam.load();
    else if (key == PF_TUNE_NN_GROUP)
        *value = g_nn_group.load();
    else if (key == PF_TUNE_GS_REORTH)
        *value = g_gs_reorth.load();
    else if (key == PF_TUNE_GG_STREAM)
        *value = g_gg_stream.load();
    else if (key == PF_TUNE_JVP2D_STREAM)
        *value = g_jvp2d_stream.load();
    else
        return fail(PF_EINVAL, "unknown tuning key %d", key);
    return PF_OK;
}
}

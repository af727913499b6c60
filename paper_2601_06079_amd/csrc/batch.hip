// batch.hip -- ragged batches of independent 2-D problems in one launch, the
// batched explicit-step adjoint, and the launch-shape autotuner.
//
// A batch packs the fields of `count` samples (each its own grid size and
// theta = (mobility, kappa, W)) into one array at caller-chosen offsets.  The
// host turns the sample list into a device plan:
//   BatchSample[count]  per-sample geometry and coefficients,
//   BatchItem[n_items]  one (sample, strip, chunk) work item per wavefront of the
//                       fused explicit kernel (strips and chunks as for a single
//                       problem, so tail items of uneven sizes are just shorter).
// One launch then advances every sample by ks fused steps.  The adjoint kernel
// streams the same work items backwards in time, one step per launch, and adds
// each item's FP64 sensitivity sums to its own slot; a final fixed-order
// reduction turns the slots into per-sample gradients.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "api_internal.hpp"
#include "kernels.hpp"

namespace pfapi {
namespace {

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int validate_base(const pf_problem* p)
{
    if (!p) return fail(PF_EINVAL, "base problem is NULL");
    if (p->dim != 2) return fail(PF_EUNSUPPORTED, "batches support 2-D problems only");
    if (p->model == PF_COUPLED || p->model == PF_GRAIN)
        return fail(PF_EUNSUPPORTED, "batches: Allen-Cahn and Cahn-Hilliard only");
    if (p->model != PF_ALLEN_CAHN && p->model != PF_CAHN_HILLIARD)
        return fail(PF_EINVAL, "unknown model %d", p->model);
    if (p->fe != PF_F_SYM && p->fe != PF_F_01) return fail(PF_EINVAL, "unknown free energy %d", p->fe);
    if (p->dtype != PF_F32 && p->dtype != PF_F64) return fail(PF_EINVAL, "unknown dtype %d", p->dtype);
    if (p->bc != PF_PERIODIC) return fail(PF_EUNSUPPORTED, "batches support periodic grids only");
    if (p->mass != PF_MASS_LUMPED) return fail(PF_EUNSUPPORTED, "batches use the lumped mass only");
    if (p->quad != PF_QUAD_GAUSS) return fail(PF_EUNSUPPORTED, "batches use Gauss quadrature only");
    return PF_OK;
}

int strips_of(long long nx, int HK) { return (int)((nx + (64 - 2 * HK) - 1) / (64 - 2 * HK)); }

struct Counts {
    long long n_items = 0, total = 0;
};

int count_plan(const pf_problem* base, const pf_batch_sample* s, int count, int ks, int ty,
               Counts* c)
{
    if (count < 1) return fail(PF_EINVAL, "count must be >= 1");
    if (count > PF_BATCH_MAX_COUNT) return fail(PF_EINVAL, "count %d exceeds PF_BATCH_MAX_COUNT", count);
    if (!s) return fail(PF_EINVAL, "samples is NULL");
    if (ks < 1 || ks > 4) return fail(PF_EINVAL, "ks must be in 1..4");
    if (ty < 1) return fail(PF_EINVAL, "ty must be >= 1");
    const int HK = (base->model == PF_CAHN_HILLIARD ? 2 : 1) * ks;
    const size_t es = base->dtype == PF_F64 ? 8 : 4;
    std::vector<std::pair<long long, long long>> ranges;
    for (int i = 0; i < count; ++i) {
        const pf_batch_sample& q = s[i];
        if (q.n[0] < 2 || q.n[1] < 2 || q.n[0] > (1 << 20) || q.n[1] > (1 << 20))
            return fail(PF_EINVAL, "sample %d: n must be in 2..2^20", i);
        const long long N = q.n[0] * q.n[1];
        if ((size_t)N * es >= (size_t(1) << 31)) return fail(PF_EINVAL, "sample %d exceeds 2 GiB", i);
        if (q.offset < 0) return fail(PF_EINVAL, "sample %d: negative offset", i);
        if (!(q.h > 0.0) || !std::isfinite(q.h) || !std::isfinite(q.W) || !std::isfinite(q.kappa) ||
            !std::isfinite(q.mobility))
            return fail(PF_EINVAL, "sample %d: h must be > 0 and parameters finite", i);
        ranges.push_back({q.offset, q.offset + N});
        c->n_items += (long long)strips_of(q.n[0], HK) * ((q.n[1] + ty - 1) / ty);
        c->total = std::max(c->total, q.offset + N);
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].second) return fail(PF_EINVAL, "sample ranges overlap");
    if (c->n_items > (1ll << 30)) return fail(PF_EINVAL, "batch too large");
    return PF_OK;
}

size_t plan_bytes_of(int count, const Counts& c)
{
    return align256(sizeof(pfk::BatchSample) * count) + align256(sizeof(pfk::BatchItem) * c.n_items);
}

int auto_ty(const pf_problem* base, const pf_batch_sample* s, int count, int ks)
{
    // as for a single problem: up to 48 rows, shortened to about four waves per SIMD
    long long items48 = 0;
    const int HK = (base->model == PF_CAHN_HILLIARD ? 2 : 1) * ks;
    int ty = 48;
    while ((ty + 2 * HK) % 4) --ty;  // chunk + halo fills whole prefetch groups
    for (;;) {
        items48 = 0;
        for (int i = 0; i < count; ++i)
            items48 += (long long)strips_of(s[i].n[0], HK) * ((s[i].n[1] + ty - 1) / ty);
        if (ty - 4 < 8 || items48 >= 4 * 1024) break;  // never below 8 rows (plan size bound)
        ty -= 4;
    }
    return ty;
}

// the signature of a batch shape under which the autotuner files its result
BatchShapeKey key_of(const pf_problem* base, const pf_batch_sample* s, int count)
{
    BatchShapeKey k{base->model, base->dtype, count, 0, 0};
    for (int i = 0; i < count; ++i) {
        k.cells += s[i].n[0] * s[i].n[1];
        k.maxn = std::max<long long>(k.maxn, std::max(s[i].n[0], s[i].n[1]));
    }
    return k;
}

}  // namespace
}  // namespace pfapi

using namespace pfapi;

extern "C" {

int pf_batch_plan_size(const pf_problem* base, const pf_batch_sample* samples, int count, int ks,
                       int ty, size_t* bytes)
{
    return guarded("pf_batch_plan_size", [&]() -> int {
        if (int rc = validate_base(base)) return rc;
        if (!bytes) return fail(PF_EINVAL, "bytes is NULL");
        if (ks == 0) ks = 4;  // narrowest strips: the worst case of the automatic choice
        if (ty == 0) ty = 8;  // shortest chunks
        Counts c;
        if (int rc = count_plan(base, samples, count, ks, ty, &c)) return rc;
        *bytes = plan_bytes_of(count, c);
        return PF_OK;
    });
}

int pf_batch_plan(pf_ctx* ctx, const pf_problem* base, const pf_batch_sample* samples, int count, double dt,
                  int ks, int ty, int depth, void* plan_dev, size_t plan_bytes, pf_batch_info* info,
                  void* stream)
{
    return guarded("pf_batch_plan", [&]() -> int {
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = validate_base(base)) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PF_EINVAL, "dt must be finite and > 0");
    if (!plan_dev || reinterpret_cast<uintptr_t>(plan_dev) % 256)
        return fail(PF_EINVAL, "plan must be a 256-byte aligned device pointer");
    if (!info) return fail(PF_EINVAL, "info is NULL");
    if (depth < 0 || ks < 0 || ty < 0) return fail(PF_EINVAL, "negative launch-shape value");
    if (count > PF_BATCH_MAX_COUNT) return fail(PF_EINVAL, "count %d exceeds PF_BATCH_MAX_COUNT", count);
    if ((ks == 0 || ty == 0 || depth == 0) && samples && count >= 1) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->tuned.find(key_of(base, samples, count));
        if (it != ctx->tuned.end()) {
            if (ks == 0) ks = it->second[0];
            if (ty == 0) ty = it->second[1];
            if (depth == 0) depth = it->second[2];
        }
    }
    if (ks == 0) ks = 2;
    if (depth == 0) depth = 4;
    if (ty == 0) ty = auto_ty(base, samples, count, ks);
    Counts c;
    if (int rc = count_plan(base, samples, count, ks, ty, &c)) return rc;
    const size_t need = plan_bytes_of(count, c);
    if (plan_bytes < need) return fail(PF_EINVAL, "plan buffer holds %zu bytes, %zu needed", plan_bytes, need);

    std::vector<pfk::BatchSample> smp(count);
    std::vector<pfk::BatchItem> items;
    items.reserve(c.n_items);
    const int H = base->model == PF_CAHN_HILLIARD ? 2 : 1;
    const int HK = H * ks;
    for (int i = 0; i < count; ++i) {
        const pf_batch_sample& q = samples[i];
        pfk::BatchSample& b = smp[i];
        std::memset(&b, 0, sizeof b);
        b.offset = q.offset;
        b.nx = (int)q.n[0];
        b.ny = (int)q.n[1];
        b.nstrips = strips_of(q.n[0], HK);
        b.first_item = (int)items.size();
        b.fe = base->fe;
        const pfk::FreeEnergy f = pfk::make_free_energy(base->fe, q.W);
        const double m = q.h * q.h, detJ = 0.25 * q.h * q.h;
        if (base->model == PF_ALLEN_CAHN) {
            const double sc = dt * q.mobility * detJ / m;
            b.a1 = sc * f.a1; b.a2 = sc * f.a2; b.a3 = sc * f.a3;
            b.beta = dt * q.mobility * q.kappa / (3.0 * m);
        } else {
            const double sc = detJ / m;
            b.a1 = sc * f.a1; b.a2 = sc * f.a2; b.a3 = sc * f.a3;
            b.beta = q.kappa / (3.0 * m);
            b.gamma = dt * q.mobility / (3.0 * m);
        }
        b.W = q.W;
        b.kappa = q.kappa;
        b.mob = q.mobility;
        b.h = q.h;
        b.dt = dt;
        const int chunks = (int)((q.n[1] + ty - 1) / ty);
        for (int ch = 0; ch < chunks; ++ch)
            for (int st = 0; st < b.nstrips; ++st) items.push_back({i, st, ch, 0});
    }
    std::vector<unsigned char> host(need, 0);
    const size_t o_s = 0, o_i = align256(sizeof(pfk::BatchSample) * count);
    std::memcpy(host.data() + o_s, smp.data(), sizeof(pfk::BatchSample) * count);
    std::memcpy(host.data() + o_i, items.data(), sizeof(pfk::BatchItem) * items.size());
    if (int rc = require_device(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(plan_dev, host.data(), need, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return check_launch("batch plan upload");
    pf_batch_info I{};
    I.count = count;
    I.n_items = (int32_t)items.size();
    I.ks = ks;
    I.ty = ty;
    I.depth = depth;
    I.model = base->model;
    I.fe = base->fe;
    I.dtype = base->dtype;
    I.total = c.total;
    I.plan_bytes = (int64_t)need;
    I.dt = dt;
    I.off_samples = (int64_t)o_s;
    I.off_items = (int64_t)o_i;
    *info = I;
    return PF_OK;
    });
}

int pf_batch_workspace_size(const pf_batch_info* info, int op, size_t* bytes)
{
    if (!info || !bytes) return fail(PF_EINVAL, "info or bytes is NULL");
    if (info->total < 1 || info->n_items < 0) return fail(PF_EINVAL, "info does not describe a plan");
    const size_t es = info->dtype == PF_F64 ? 8 : 4;
    const size_t field = align256((size_t)info->total * es);
    if (op == PF_OP_STEP_EXPLICIT)
        *bytes = field;
    else if (op == PF_OP_VJP)
        *bytes = field + align256((size_t)info->n_items * 2 * sizeof(double));
    else
        return fail(PF_EINVAL, "batches support PF_OP_STEP_EXPLICIT and PF_OP_VJP");
    return PF_OK;
}

}  // extern "C"

namespace {

int check_info(const pf_batch_info* info, const void* plan)
{
    if (!info) return fail(PF_EINVAL, "info is NULL");
    if (!plan || reinterpret_cast<uintptr_t>(plan) % 256) return fail(PF_EINVAL, "plan is NULL or misaligned");
    if (info->count < 1 || info->n_items < 1 || info->ks < 1 || info->ks > 4 || info->total < 1 ||
        (info->dtype != PF_F32 && info->dtype != PF_F64) || info->off_items <= 0)
        return fail(PF_EINVAL, "info does not describe a plan built by pf_batch_plan");
    return PF_OK;
}

template <typename T>
int batched_steps_t(const pf_batch_info* info, const void* plan, int64_t nsteps, T* U, T* ws,
                    T* traj, hipStream_t s)
{
    const char* pb = static_cast<const char*>(plan);
    const auto* smp = reinterpret_cast<const pfk::BatchSample*>(pb + info->off_samples);
    const auto* items = reinterpret_cast<const pfk::BatchItem*>(pb + info->off_items);
    const long long total = info->total;
    if (traj) {
        // pairs of steps fused where the plan's strips leave room (ks >= 2), each
        // launch writing both states; a lone last step runs alone (the plan's
        // narrower strips cover every column for a single-step launch too)
        const pfk::Stream2DConfig one{info->ty, info->depth, 1};
        int64_t k = 0;
        for (; info->ks >= 2 && k + 2 <= nsteps; k += 2) {
            const T* in = k == 0 ? U : traj + (k - 1) * total;
            pfk::launch_explicit2d_batched<T>(info->model, in, traj + (k + 1) * total, smp, items,
                                              info->n_items, one, s, traj + k * total);
        }
        for (; k < nsteps; ++k) {
            const T* in = k == 0 ? U : traj + (k - 1) * total;
            pfk::launch_explicit2d_batched<T>(info->model, in, traj + k * total, smp, items,
                                              info->n_items, one, s);
        }
        return check_launch("pf_step_explicit_batched");
    }
    const pfk::Stream2DConfig cfg{info->ty, info->depth, info->ks};
    T* cur = U;
    T* other = ws;
    for (int64_t k = 0; k < nsteps; k += info->ks) {
        pfk::launch_explicit2d_batched<T>(info->model, cur, other, smp, items, info->n_items, cfg, s);
        std::swap(cur, other);
    }
    if (int rc = check_launch("pf_step_explicit_batched")) return rc;
    if (cur != U && hipMemcpyAsync(U, cur, (size_t)total * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return check_launch("batched copy-back");
    return PF_OK;
}

template <typename T>
int batched_vjp_t(const pf_batch_info* info, const void* plan, int64_t nsteps, const T* states,
                  T* lam, double* theta_bar, void* ws, int flags, hipStream_t s)
{
    const char* pb = static_cast<const char*>(plan);
    const auto* smp = reinterpret_cast<const pfk::BatchSample*>(pb + info->off_samples);
    const auto* items = reinterpret_cast<const pfk::BatchItem*>(pb + info->off_items);
    const long long total = info->total;
    T* other = static_cast<T*>(ws);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + align256((size_t)total * sizeof(T)));
    if ((flags & PF_VJP_BEGIN) &&
        hipMemsetAsync(part, 0, (size_t)info->n_items * 2 * sizeof(double), s) != hipSuccess)
        return check_launch("batched vjp init");
    const int hk = info->ks;  // Allen-Cahn: strip halo H ks with H = 1
    // two adjoint steps per launch where the plan's strips leave room (hk >= 2),
    // paired from the last step down; a lone first step runs alone
    T* cur = lam;
    for (int64_t k = nsteps - 1; k >= 0;) {
        const int two = hk >= 2 && k >= 1;
        pfk::launch_vjp2d_batched<T>(states + k * total, states + (two ? k - 1 : k) * total, cur,
                                     other, smp, items, info->n_items, info->ty, hk, info->depth,
                                     two ? 2 : 1, info->fe == PF_F_SYM, part, s);
        std::swap(cur, other);
        k -= two ? 2 : 1;
    }
    if (flags & PF_VJP_END) pfk::launch_vjp2d_reduce(part, smp, info->count, info->ty, theta_bar, s);
    if (int rc = check_launch("pf_vjp_explicit_batched")) return rc;
    if (cur != lam && hipMemcpyAsync(lam, cur, (size_t)total * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return check_launch("batched vjp copy-back");
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_step_explicit_batched(pf_ctx* ctx, const pf_batch_info* info, const void* plan, int64_t nsteps, void* U,
                             void* ws, void* traj, void* stream)
{
    return guarded("pf_step_explicit_batched", [&]() -> int {
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = check_info(info, plan)) return rc;
    if (nsteps < 0) return fail(PF_EINVAL, "nsteps must be >= 0");
    if (!U) return fail(PF_EINVAL, "U is NULL");
    if (traj) {
        if (nsteps < 1) return fail(PF_EINVAL, "trajectory mode needs nsteps >= 1");
    } else {
        if (nsteps % info->ks) return fail(PF_EINVAL, "nsteps must be a multiple of the plan's ks (%d)", info->ks);
        if (!ws) return fail(PF_EINVAL, "ws is NULL");
    }
    if (int rc = require_device(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (info->dtype == PF_F32)
        return batched_steps_t<float>(info, plan, nsteps, (float*)U, (float*)ws, (float*)traj, s);
    return batched_steps_t<double>(info, plan, nsteps, (double*)U, (double*)ws, (double*)traj, s);
    });
}

int pf_vjp_explicit_batched(pf_ctx* ctx, const pf_batch_info* info, const void* plan, int64_t nsteps,
                            const void* states, void* lam, double* theta_bar, void* ws, int flags,
                            void* stream)
{
    return guarded("pf_vjp_explicit_batched", [&]() -> int {
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = check_info(info, plan)) return rc;
    if (info->model != PF_ALLEN_CAHN)
        return fail(PF_EUNSUPPORTED, "batched adjoint is implemented for Allen-Cahn");
    if (nsteps < 0) return fail(PF_EINVAL, "nsteps must be >= 0");
    if (!states || !lam || !ws || !theta_bar) return fail(PF_EINVAL, "NULL pointer argument");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws must be 256-byte aligned");
    if (flags & ~(PF_VJP_BEGIN | PF_VJP_END)) return fail(PF_EINVAL, "unknown flags");
    if (int rc = require_device(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (info->dtype == PF_F32)
        return batched_vjp_t<float>(info, plan, nsteps, (const float*)states, (float*)lam, theta_bar,
                                    ws, flags, s);
    return batched_vjp_t<double>(info, plan, nsteps, (const double*)states, (double*)lam, theta_bar,
                                 ws, flags, s);
    });
}

int pf_batch_autotune(pf_ctx* ctx, const pf_problem* base, const pf_batch_sample* samples, int count, double dt,
                      void* U_scratch, void* ws, void* plan_dev, size_t plan_bytes,
                      pf_batch_info* best, double* best_us_per_step, void* stream)
{
    return guarded("pf_batch_autotune", [&]() -> int {
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = validate_base(base)) return rc;
    if (!U_scratch || !ws || !best) return fail(PF_EINVAL, "NULL pointer argument");
    if (count < 1 || count > PF_BATCH_MAX_COUNT || !samples)
        return fail(PF_EINVAL, "count must be in 1..PF_BATCH_MAX_COUNT with samples given");
    if (int rc = require_device(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return check_launch("autotune events");
    const int kss[] = {1, 2, 3, 4};
    const int tys[] = {16, 24, 32, 48};
    const int depths[] = {4, 8};
    double best_t = -1.0;
    int bk = 2, bt = 24, bd = 4;
    int status = PF_OK;
    for (int ks : kss)
        for (int ty : tys)
            for (int depth : depths) {
                // rounded down so that chunk + halo fills whole prefetch groups
                const int HK = (base->model == PF_CAHN_HILLIARD ? 2 : 1) * ks;
                const int tya = ty - (ty + 2 * HK) % 4;
                pf_batch_info I;
                int rc = pf_batch_plan(ctx, base, samples, count, dt, ks, tya, depth, plan_dev, plan_bytes, &I,
                                       stream);
                if (rc == PF_EINVAL) continue;  // this candidate's plan does not fit the buffer
                if (rc) { status = rc; goto done; }
                const int64_t steps = 2 * ks;
                if ((rc = pf_step_explicit_batched(ctx, &I, plan_dev, steps, U_scratch, ws, nullptr, stream))) { status = rc; goto done; }
                hipEventRecord(e0, s);
                const int reps = 3;
                for (int r = 0; r < reps; ++r)
                    if ((rc = pf_step_explicit_batched(ctx, &I, plan_dev, steps, U_scratch, ws, nullptr, stream))) { status = rc; goto done; }
                hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) { status = check_launch("autotune timing"); goto done; }
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                const double t = ms / (reps * steps);
                if (best_t < 0 || t < best_t) {
                    best_t = t;
                    bk = ks;
                    bt = tya;
                    bd = depth;
                }
            }
    if (best_t < 0) { status = fail(PF_EINVAL, "plan buffer too small for every candidate"); goto done; }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tuned[key_of(base, samples, count)] = {bk, bt, bd};
    }
    status = pf_batch_plan(ctx, base, samples, count, dt, bk, bt, bd, plan_dev, plan_bytes, best, stream);
    if (best_us_per_step) *best_us_per_step = best_t * 1e3;
done:
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return status;
    });
}

}  // extern "C"

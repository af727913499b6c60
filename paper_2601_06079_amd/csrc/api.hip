// api.hip -- the extern "C" boundary of libpfhip.so (declared in include/pf.h).
//
// Every entry point validates its arguments on the host before anything is
// enqueued, converts the problem statement into kernel parameters and
// launches on the caller's stream.  No exception crosses the ABI (each body runs
// inside guarded()); errors are reported as pf_status plus a thread-local
// message held in a fixed buffer, so reporting an error never allocates.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>

#include "../../include/pf.h"
#include "api_internal.hpp"
#include "kernels.hpp"

namespace pfapi {

thread_local char g_last_error[512];

int fail(int status, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return status;
}

int check_ctx(const pf_ctx* ctx)
{
    if (!ctx) return fail(PF_EINVAL, "ctx is NULL (make one with pf_create)");
    return PF_OK;
}

int require_device(const pf_ctx* ctx)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (ctx->device < 0) return fail(PF_EINVAL, "a host-only context cannot enqueue device work");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return check_launch("hipGetDevice");
    if (cur != ctx->device)
        return fail(PF_EINVAL, "the context belongs to device %d but device %d is current", ctx->device, cur);
    return PF_OK;
}

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return PF_OK;
}

int validate(const pf_problem* p)
{
    if (!p) return fail(PF_EINVAL, "problem is NULL");
    if (p->dim != 2 && p->dim != 3) return fail(PF_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->model != PF_ALLEN_CAHN && p->model != PF_CAHN_HILLIARD && p->model != PF_COUPLED &&
        p->model != PF_GRAIN)
        return fail(PF_EINVAL, "unknown model %d", p->model);
    if (p->quad != PF_QUAD_GAUSS && p->quad != PF_QUAD_LOBATTO)
        return fail(PF_EINVAL, "unknown quadrature %d", p->quad);
    if (p->quad == PF_QUAD_LOBATTO && p->model != PF_ALLEN_CAHN && p->model != PF_CAHN_HILLIARD)
        return fail(PF_EUNSUPPORTED, "Gauss-Lobatto quadrature: Allen-Cahn and Cahn-Hilliard only");
    if (p->model == PF_GRAIN) {
        const int pmax = p->dtype == PF_F64 ? 12 : 32;  // LDS of the tile kernel <= 64 KB
        if (p->nfields < 1 || p->nfields > pmax)
            return fail(PF_EINVAL, "grain growth: nfields must be in [1, %d] (got %d)", pmax, p->nfields);
        if (!std::isfinite(p->gamma)) return fail(PF_EINVAL, "gamma must be finite");
        if (p->dim != 2) return fail(PF_EUNSUPPORTED, "grain growth: 2-D grids only");
        if (p->mass != PF_MASS_LUMPED) return fail(PF_EUNSUPPORTED, "grain growth: lumped mass only");
    }
    if (p->model == PF_COUPLED && !std::isfinite(p->mobility_eta))
        return fail(PF_EINVAL, "mobility_eta must be finite");
    if (p->model != PF_COUPLED && p->model != PF_GRAIN && p->fe != PF_F_SYM && p->fe != PF_F_01)
        return fail(PF_EINVAL, "unknown free energy %d", p->fe);
    if (p->dtype != PF_F32 && p->dtype != PF_F64) return fail(PF_EINVAL, "unknown dtype %d", p->dtype);
    if (p->mass != PF_MASS_LUMPED && p->mass != PF_MASS_CONSISTENT)
        return fail(PF_EINVAL, "unknown mass matrix %d", p->mass);
    if (p->mass == PF_MASS_CONSISTENT && p->model == PF_COUPLED)
        return fail(PF_EUNSUPPORTED, "the coupled model uses the lumped mass only");
    long long N = 1;
    for (int k = 0; k < p->dim; ++k) {
        if (p->n[k] < 2) return fail(PF_EINVAL, "n[%d] = %lld must be >= 2", k, (long long)p->n[k]);
        if (p->n[k] > (1ll << 30)) return fail(PF_EINVAL, "n[%d] too large", k);
        N *= p->n[k];
        if (N > (1ll << 40)) return fail(PF_EINVAL, "grid too large");
    }
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail(PF_EINVAL, "h must be finite and > 0");
    if (!std::isfinite(p->W) || !std::isfinite(p->kappa) || !std::isfinite(p->mobility))
        return fail(PF_EINVAL, "W, kappa and mobility must be finite");
    if (p->bc != PF_PERIODIC && p->bc != PF_NOFLUX)
        return fail(PF_EINVAL, "unknown boundary condition %d", p->bc);
    return PF_OK;
}

int check_ptr(const void* ptr, const pf_problem* p, const char* name)
{
    if (!ptr) return fail(PF_EINVAL, "%s is NULL", name);
    const size_t al = p->dtype == PF_F64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(ptr) % al)
        return fail(PF_EINVAL, "%s is not %zu-byte aligned", name, al);
    return PF_OK;
}

pfk::Geom geom_of(const pf_problem* p)
{
    pfk::Geom g{};
    g.dim = p->dim;
    g.N = 1;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = k < p->dim ? (int)p->n[k] : 1;
        g.N *= g.n[k];
    }
    g.h = p->h;
    g.bc = p->bc == PF_NOFLUX ? 1 : 0;
    g.quad = p->quad == PF_QUAD_LOBATTO ? 1 : 0;
    // nodal quadrature makes the Gauss-integrated mass the lumped one
    g.cm = p->mass == PF_MASS_CONSISTENT && !g.quad ? 1 : 0;
    return g;
}

long long ndof(const pf_problem* p)
{
    const pfk::Geom g = geom_of(p);
    if (p->model == PF_GRAIN) return (long long)p->nfields * g.N;
    return (p->model == PF_COUPLED ? 3 : p->model == PF_CAHN_HILLIARD ? 2 : 1) * g.N;
}

size_t elem_size(const pf_problem* p) { return p->dtype == PF_F64 ? 8 : 4; }

// the grain-growth Jacobian product stages two sets of fields in LDS (<= 64 KB)
int grain_implicit_ok(const pf_problem* p)
{
    const int pmax = p->dtype == PF_F64 ? 12 : 24;
    if (p->nfields > pmax)
        return fail(PF_EUNSUPPORTED, "grain growth: the implicit path takes at most %d order parameters", pmax);
    return PF_OK;
}

}  // namespace pfapi

using namespace pfapi;

namespace {

// coupled model: node-centric path, ws = [c ping-pong field | eta ping-pong field]
template <typename T>
int step_coupled_t(const pf_problem* p, int cus, double dt, int64_t nsteps, T* U, T* ws, hipStream_t s)
{
    const pfk::Geom g = geom_of(p);
    T* c = U;
    T* mu = U + g.N;
    T* eta = U + 2 * g.N;
    T *cc = c, *co = ws, *ec = eta, *eo = ws + g.N;
    // 2-D: the fused streaming kernel (32-bit buffer offsets); else node-centric kernels
    const bool fused2d = p->dim == 2 && (size_t)g.N * sizeof(T) < (size_t(1) << 31);
    const int rows = stream2d_rows(p, 1, cus);
    for (int64_t st = 0; st < nsteps; ++st) {
        if (fused2d) {
            pfk::launch_cp_explicit2d<T>(g, p->kappa, p->mobility, p->mobility_eta, dt, cc, ec, co, eo,
                                         rows, s);
        } else {
            pfk::launch_cp_mu_eta<T>(g, p->kappa, dt * p->mobility_eta, cc, ec, mu, eo, s);
            pfk::launch_ch_update<T>(g, dt * p->mobility, cc, mu, co, s);
        }
        std::swap(cc, co);
        std::swap(ec, eo);
    }
    if (cc != c) {
        if (hipMemcpyAsync(c, cc, (size_t)g.N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(eta, ec, (size_t)g.N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return check_launch("coupled step copy-back");
    }
    pfk::launch_cp_mu_eta<T>(g, p->kappa, 0.0, c, eta, mu, (T*)nullptr, s);
    return check_launch("coupled explicit step");
}

// grain growth: all order parameters per launch, ping-pong between U and ws
template <typename T>
int step_grain_t(const pf_problem* p, int cus, double dt, int64_t nsteps, T* U, T* ws, hipStream_t s)
{
    const pfk::Geom g = geom_of(p);
    T *cur = U, *other = ws;
    for (int64_t st = 0; st < nsteps; ++st) {
        if (!pfk::launch_gg_stream2d<T>(g, p->nfields, p->mobility, p->kappa, p->gamma, dt, cur, other, cus, s))
            pfk::launch_gg_tile2d<T>(g, p->nfields, p->mobility, p->kappa, p->gamma, dt, cur, other, 0, s);
        std::swap(cur, other);
    }
    if (int rc = check_launch("grain step")) return rc;
    if (cur != U &&
        hipMemcpyAsync(U, cur, (size_t)p->nfields * g.N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return check_launch("grain step copy-back");
    return check_launch("grain step");
}

template <typename T>
int step_explicit_t(const pf_problem* p, int cus, double dt, int64_t nsteps, T* U, T* ws, hipStream_t s)
{
    if (p->model == PF_COUPLED) return step_coupled_t<T>(p, cus, dt, nsteps, U, ws, s);
    if (p->model == PF_GRAIN) return step_grain_t<T>(p, cus, dt, nsteps, U, ws, s);
    const pfk::Geom g = geom_of(p);
    const pfk::FreeEnergy f = pfk::make_free_energy(p->fe, p->W);
    T* c = U;
    T* other = ws;
    T* cur = c;
    // the fused 2-D kernel addresses a field with 32-bit buffer offsets
    const bool fused2d = p->dim == 2 && (size_t)g.N * sizeof(T) < (size_t(1) << 31);
    if (fused2d) {
        // launches of ks fused steps, then the remainder one step at a time
        const int ks = stream2d_fuse(p);
        pfk::Stream2DConfig cfg{stream2d_rows(p, ks, cus), stream2d_depth(p), ks};
        pfk::Stream2DConfig one{stream2d_rows(p, 1, cus), stream2d_depth(p), 1};
        int64_t st = 0;
        for (; ks > 1 && st + ks <= nsteps; st += ks) {
            pfk::launch_explicit2d<T>(g, p->model, f, p->kappa, p->mobility, dt, cur, other, cfg, s);
            std::swap(cur, other);
        }
        for (; st < nsteps; ++st) {
            pfk::launch_explicit2d<T>(g, p->model, f, p->kappa, p->mobility, dt, cur, other, one, s);
            std::swap(cur, other);
        }
    } else if (p->model == PF_ALLEN_CAHN) {
        // node-centric path: 3-D, and 2-D fields of 2 GiB or more
        for (int64_t st = 0; st < nsteps; ++st) {
            pfk::launch_ac_step<T>(g, f, p->kappa, dt * p->mobility, cur, other, s);
            std::swap(cur, other);
        }
    } else {
        T* mu = U + g.N;
        for (int64_t st = 0; st < nsteps; ++st) {
            pfk::launch_chem<T>(g, f, p->kappa, cur, mu, s);
            pfk::launch_ch_update<T>(g, dt * p->mobility, cur, mu, other, s);
            std::swap(cur, other);
        }
    }
    if (int rc = check_launch("explicit step")) return rc;
    if (cur != c) {
        if (hipMemcpyAsync(c, cur, (size_t)g.N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return check_launch("explicit step copy-back");
    }
    if (p->model == PF_CAHN_HILLIARD) pfk::launch_chem<T>(g, f, p->kappa, c, U + g.N, s);
    return check_launch("explicit step");
}

// energy and sum m c of U, partial sums in `part` (energy_blocks(g) pairs)
int energy_t(const pf_problem* p, const void* U, double* out, double* part, hipStream_t s)
{
    const pfk::Geom g = geom_of(p);
    if (p->model == PF_GRAIN) {
        if (p->dtype == PF_F32)
            pfk::launch_gg_energy2d<float>(g, p->nfields, p->kappa, p->gamma, (const float*)U, part, out, s);
        else
            pfk::launch_gg_energy2d<double>(g, p->nfields, p->kappa, p->gamma, (const double*)U, part, out, s);
        return check_launch("pf_energy");
    }
    const pfk::FreeEnergy f = pfk::make_free_energy(p->fe, p->W);
    if (p->model == PF_COUPLED) {
        if (p->dtype == PF_F32)
            pfk::launch_cp_energy<float>(g, p->kappa, (const float*)U, part, out, s);
        else
            pfk::launch_cp_energy<double>(g, p->kappa, (const double*)U, part, out, s);
        return check_launch("pf_energy");
    }
    if (p->dtype == PF_F32)
        pfk::launch_energy<float>(g, f, p->kappa, (const float*)U, part, out, s);
    else
        pfk::launch_energy<double>(g, f, p->kappa, (const double*)U, part, out, s);
    return check_launch("pf_energy");
}

}  // namespace

namespace {

// Device scratch of pf_energy_noalloc: the per-block FP64 partial sums of the
// energy reduction (a pair per block of 256 nodes), for callers that cannot
// allocate.  Each device the library runs on holds its own copy until the
// process ends; pf_create looks up its address on that device.  Calls that
// overlap on one device race on it.  Every partial is written before it is read,
// so nothing needs clearing between calls.
constexpr size_t NOALLOC_ENERGY_DOUBLES = size_t(1) << 17;  // 1 MiB: up to 2^24 nodes
static __device__ __align__(256) double scratch[NOALLOC_ENERGY_DOUBLES];

int make_slots(pfapi::PinnedSlots* sl, size_t doubles, int events)
{
    double* h = nullptr;
    hipError_t e = hipHostMalloc((void**)&h, doubles * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return fail(PF_EDEVICE, "pinned host slots: %s", hipGetErrorString(e));
    sl->host = h;
    std::memset(h, 0, doubles * sizeof(double));
    e = hipHostGetDevicePointer((void**)&sl->dev, h, 0);
    if (e != hipSuccess) return fail(PF_EDEVICE, "pinned host slots mapping: %s", hipGetErrorString(e));
    for (int i = 0; i < events; ++i) {
        e = hipEventCreateWithFlags(&sl->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return fail(PF_EDEVICE, "readback event: %s", hipGetErrorString(e));
    }
    return PF_OK;
}

void free_slots(pfapi::PinnedSlots* sl)
{
    for (hipEvent_t& ev : sl->ev)
        if (ev) {
            (void)hipEventDestroy(ev);
            ev = nullptr;
        }
    if (sl->host) (void)hipHostFree(sl->host);
    sl->host = sl->dev = nullptr;
}

void free_ctx(pf_ctx* c)
{
    if (!c) return;
    if (c->device >= 0) {
        int prev = -1;
        const bool had = hipGetDevice(&prev) == hipSuccess;
        if (hipSetDevice(c->device) == hipSuccess) {
            free_slots(&c->gmres);
            free_slots(&c->cg);
        }
        if (had) (void)hipSetDevice(prev);
        (void)hipGetLastError();
    }
    delete c;
}

}  // namespace

extern "C" {

const char* pf_last_error(void) { return g_last_error; }

int pf_version(void) { return 200; }

int pf_create(int device, pf_ctx** out)
{
    return guarded("pf_create", [&]() -> int {
        if (!out) return fail(PF_EINVAL, "out is NULL");
        *out = nullptr;
        std::unique_ptr<pf_ctx> c(new pf_ctx());
        if (device == PF_HOST_ONLY) {
            *out = c.release();
            return PF_OK;
        }
        if (device < 0) return fail(PF_EINVAL, "device must be >= 0 or PF_HOST_ONLY (got %d)", device);
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess) count = 0;
        (void)hipGetLastError();
        if (device >= count) return fail(PF_EDEVICE, "device %d is not available (%d visible)", device, count);
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) return check_launch("hipGetDevice");
        if (hipSetDevice(device) != hipSuccess) return check_launch("hipSetDevice");
        c->device = device;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            c->cus = cus;
        int rc = make_slots(&c->gmres, newton_pinned_doubles(), 3);
        if (rc == PF_OK) rc = make_slots(&c->cg, elastic_pinned_doubles(), 2);
        if (rc == PF_OK) {  // this device's copy of the static scratch (device current here)
            void* sp = nullptr;
            const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !sp)
                rc = fail(PF_EDEVICE, "static scratch address: %s", hipGetErrorString(e));
            c->scratch = static_cast<double*>(sp);
        }
        (void)hipSetDevice(prev);
        if (rc != PF_OK) {
            free_ctx(c.release());
            return rc;
        }
        *out = c.release();
        return PF_OK;
    });
}

int pf_destroy(pf_ctx* ctx)
{
    return guarded("pf_destroy", [&]() -> int {
        free_ctx(ctx);
        return PF_OK;
    });
}

int pf_ctx_device(const pf_ctx* ctx, int* device)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (!device) return fail(PF_EINVAL, "device is NULL");
    *device = ctx->device;
    return PF_OK;
}

int pf_workspace_size(const pf_ctx* ctx, const pf_problem* p, int op, size_t* bytes)
{
    return guarded("pf_workspace_size", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (!bytes) return fail(PF_EINVAL, "bytes is NULL");
        const pfk::Geom g = geom_of(p);
        const size_t es = elem_size(p);
        size_t b = 0;
        switch (op) {
            case PF_OP_RESIDUAL:
            case PF_OP_JVP: b = 0; break;
            case PF_OP_STEP_EXPLICIT:
                if (p->mass != PF_MASS_LUMPED) return fail(PF_EUNSUPPORTED, "explicit steps need the lumped mass");
                b = (size_t)g.N * es * (p->model == PF_COUPLED ? 2 : p->model == PF_GRAIN ? p->nfields : 1);
                break;
            case PF_OP_ENERGY: b = (size_t)pfk::energy_blocks(g) * 2 * sizeof(double); break;
            case PF_OP_NEWTON:
                if (p->model == PF_GRAIN)
                    if (int rc = grain_implicit_ok(p)) return rc;
                b = newton_workspace_bytes(p, 30);
                break;
            case PF_OP_VJP:
                if (p->model == PF_GRAIN) return fail(PF_EUNSUPPORTED, "grain growth: the adjoint is not implemented");
                if (p->model == PF_COUPLED) return fail(PF_EUNSUPPORTED, "coupled model: the adjoint is not implemented");
                b = vjp_workspace_bytes(p);
                break;
            default: return fail(PF_EINVAL, "unknown op %d", op);
        }
        *bytes = b;
        return PF_OK;
    });
}

int pf_residual(pf_ctx* ctx, const pf_problem* p, const void* U, void* r, void* ws, void* stream)
{
    (void)ws;  // the residual needs no scratch (pf_workspace_size(PF_OP_RESIDUAL) is 0)
    return guarded("pf_residual", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (int rc = check_ptr(U, p, "U")) return rc;
        if (int rc = check_ptr(r, p, "r")) return rc;
        if (U == r) return fail(PF_EINVAL, "U and r must not alias");
        if (int rc = require_device(ctx)) return rc;
        const pfk::Geom g = geom_of(p);
        hipStream_t s = (hipStream_t)stream;
        if (p->model == PF_GRAIN) {
            if (p->dtype == PF_F32)
                pfk::launch_gg_tile2d<float>(g, p->nfields, p->mobility, p->kappa, p->gamma, 0.0, (const float*)U,
                                             (float*)r, 1, s);
            else
                pfk::launch_gg_tile2d<double>(g, p->nfields, p->mobility, p->kappa, p->gamma, 0.0,
                                              (const double*)U, (double*)r, 1, s);
            return check_launch("pf_residual");
        }
        const pfk::FreeEnergy f = pfk::make_free_energy(p->fe, p->W);
        if (p->model == PF_COUPLED) {
            if (p->dtype == PF_F32)
                pfk::launch_cp_residual<float>(g, p->kappa, p->mobility, p->mobility_eta, (const float*)U,
                                               (float*)r, s);
            else
                pfk::launch_cp_residual<double>(g, p->kappa, p->mobility, p->mobility_eta,
                                                (const double*)U, (double*)r, s);
            return check_launch("pf_residual");
        }
        if (p->dtype == PF_F32)
            pfk::launch_residual<float>(g, p->model, f, p->kappa, p->mobility, (const float*)U,
                                        (float*)r, s);
        else
            pfk::launch_residual<double>(g, p->model, f, p->kappa, p->mobility, (const double*)U,
                                         (double*)r, s);
        return check_launch("pf_residual");
    });
}

int pf_step_explicit(pf_ctx* ctx, const pf_problem* p, double dt, int64_t nsteps, void* U, void* ws,
                     void* stream)
{
    return guarded("pf_step_explicit", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PF_EINVAL, "dt must be finite and > 0");
        if (nsteps < 0) return fail(PF_EINVAL, "nsteps must be >= 0");
        if (int rc = check_ptr(U, p, "U")) return rc;
        if (int rc = check_ptr(ws, p, "ws")) return rc;
        if (p->mass != PF_MASS_LUMPED)
            return fail(PF_EUNSUPPORTED, "explicit steps need the lumped mass (a consistent mass needs a solve)");
        if (int rc = require_device(ctx)) return rc;
        hipStream_t s = (hipStream_t)stream;
        if (p->dtype == PF_F32) return step_explicit_t<float>(p, ctx->cus, dt, nsteps, (float*)U, (float*)ws, s);
        return step_explicit_t<double>(p, ctx->cus, dt, nsteps, (double*)U, (double*)ws, s);
    });
}

int pf_energy(pf_ctx* ctx, const pf_problem* p, const void* U, double* out, void* ws, void* stream)
{
    return guarded("pf_energy", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (int rc = check_ptr(U, p, "U")) return rc;
        if (!out || reinterpret_cast<uintptr_t>(out) % 8) return fail(PF_EINVAL, "out is NULL or misaligned");
        if (!ws || reinterpret_cast<uintptr_t>(ws) % 8) return fail(PF_EINVAL, "ws is NULL or misaligned");
        if (int rc = require_device(ctx)) return rc;
        return energy_t(p, U, out, (double*)ws, (hipStream_t)stream);
    });
}

int pf_energy_noalloc(pf_ctx* ctx, const pf_problem* p, const void* U, double* out, void* stream)
{
    return guarded("pf_energy_noalloc", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (int rc = check_ptr(U, p, "U")) return rc;
        if (!out || reinterpret_cast<uintptr_t>(out) % 8) return fail(PF_EINVAL, "out is NULL or misaligned");
        const pfk::Geom g = geom_of(p);
        const size_t need = (size_t)pfk::energy_blocks(g) * 2;
        if (need > NOALLOC_ENERGY_DOUBLES)
            return fail(PF_EINVAL, "pf_energy_noalloc: %lld nodes exceed the static scratch (at most %lld)",
                        (long long)g.N, (long long)(NOALLOC_ENERGY_DOUBLES / 2 * 256));
        if (int rc = require_device(ctx)) return rc;
        if (!ctx->scratch) return fail(PF_EDEVICE, "the context has no static scratch address");
        return energy_t(p, U, out, ctx->scratch, (hipStream_t)stream);
    });
}

int pf_jvp(pf_ctx* ctx, const pf_problem* p, double inv_dt, const void* U, const void* v, void* Jv,
           void* stream)
{
    return guarded("pf_jvp", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (!std::isfinite(inv_dt) || inv_dt < 0.0) return fail(PF_EINVAL, "inv_dt must be finite and >= 0");
        if (int rc = check_ptr(U, p, "U")) return rc;
        if (int rc = check_ptr(v, p, "v")) return rc;
        if (int rc = check_ptr(Jv, p, "Jv")) return rc;
        if (Jv == U || Jv == v) return fail(PF_EINVAL, "Jv must not alias U or v");
        if (p->model == PF_GRAIN)
            if (int rc = grain_implicit_ok(p)) return rc;
        if (int rc = require_device(ctx)) return rc;
        const pfk::Geom g = geom_of(p);
        hipStream_t s = (hipStream_t)stream;
        if (p->model == PF_GRAIN) {
            if (p->dtype == PF_F32)
                pfk::launch_gg_jvp2d<float>(g, p->nfields, p->mobility, p->kappa, p->gamma, inv_dt, (const float*)U,
                                            (const float*)v, (float*)Jv, s);
            else
                pfk::launch_gg_jvp2d<double>(g, p->nfields, p->mobility, p->kappa, p->gamma, inv_dt,
                                             (const double*)U, (const double*)v, (double*)Jv, s);
            return check_launch("pf_jvp");
        }
        const pfk::FreeEnergy f = pfk::make_free_energy(p->fe, p->W);
        if (p->model == PF_COUPLED) {
            if (p->dtype == PF_F32)
                pfk::launch_cp_jvp<float>(g, p->kappa, p->mobility, p->mobility_eta, inv_dt, (const float*)U,
                                          (const float*)v, (float*)Jv, s);
            else
                pfk::launch_cp_jvp<double>(g, p->kappa, p->mobility, p->mobility_eta, inv_dt,
                                           (const double*)U, (const double*)v, (double*)Jv, s);
            return check_launch("pf_jvp");
        }
        if (p->dtype == PF_F32)
            pfk::launch_jvp<float>(g, p->model, f, p->kappa, p->mobility, inv_dt, (const float*)U,
                                   (const float*)v, (float*)Jv, s);
        else
            pfk::launch_jvp<double>(g, p->model, f, p->kappa, p->mobility, inv_dt, (const double*)U,
                                    (const double*)v, (double*)Jv, s);
        return check_launch("pf_jvp");
    });
}

}  // extern "C"

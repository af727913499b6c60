// newton.hip -- backward-Euler step by Newton-Raphson with matrix-free GMRES
// (Eqs. 13-14, Sec. 2.3), and the adjoint solve of that step (Supp. Note 2).
//
// Host loop, device data.  All vectors (residual, correction, the Krylov basis,
// the preconditioner) live in the caller's workspace on the device; every
// matrix-vector product is the matrix-free Jacobian kernel; every dot product
// and norm is an FP64 device reduction.  Per Arnoldi step the host reads back
// one Hessenberg column (<= 2 m + 3 doubles) to apply its Givens rotation and
// test convergence; the (m+1) x m Hessenberg matrix and the small triangular
// solve stay on the host in FP64.  The read is pipelined: the next Arnoldi step
// is queued before the host waits for the current column, so the device never
// idles on the round trip; a step queued past convergence is discarded.
//
// GMRES(m) variant: right preconditioning (the residual it monitors is the true
// one), classical Gram-Schmidt with one re-orthogonalisation, x0 = 0, restart
// from the true residual b - J x.  Inexact Newton: the linear tolerance is
// clamp(0.1 ||R_k|| / ||R_0||, lin_rtol_min, lin_rtol_max) relative to ||R_k||.
#include <cmath>
#include <array>
#include <cstring>

#include "api_internal.hpp"
#include "kernels.hpp"
#include "krylov.hpp"

namespace pfapi {
namespace {

constexpr int MAXM = 32;  // largest restart length

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Workspace layout shared by the forward Newton step and the adjoint solve.
template <typename T>
struct NWS {
    T *R, *x, *w, *z, *b, *V, *pinv;
    long long ld;
    double *part, *dev;  // dev: [h1(MAXM+1) | h2(MAXM+1) | nrm(2) | y(MAXM) | misc(8)]
    long long part_len;  // doubles in part
    double* theta;       // device copy of a host theta_bar (pf_vjp with PF_VJP_THETA_HOST)
    size_t bytes;
};

template <typename T>
NWS<T> layout(const pf_problem* p, void* base)
{
    const pfk::Geom g = geom_of(p);
    const long long n = ndof(p);
    NWS<T> L{};
    // basis columns 256-byte aligned and 1280 bytes off a power-of-two stride, so that
    // the k streams of a Gram-Schmidt sweep do not start on the same HBM channel
    L.ld = (n + 63) / 64 * 64 + 1280 / (long long)sizeof(T);
    char* c = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t b) {
        char* r = c ? c + off : nullptr;
        off += align256(b);
        return r;
    };
    L.R = (T*)take(n * sizeof(T));
    L.x = (T*)take(n * sizeof(T));
    L.w = (T*)take(n * sizeof(T));
    L.z = (T*)take(n * sizeof(T));
    L.b = (T*)take(n * sizeof(T));
    L.V = (T*)take((size_t)(MAXM + 1) * L.ld * sizeof(T));
    L.pinv = (T*)take((size_t)(p->model == PF_COUPLED ? 9 : p->model == PF_CAHN_HILLIARD ? 4
                               : p->model == PF_GRAIN ? p->nfields : 1) * g.N * sizeof(T));
    const long long nbp = std::max<long long>(pfk::krylov_blocks(n), (g.N + 255) / 256);
    L.part = (double*)take((size_t)(MAXM + 2) * nbp * sizeof(double) + 64);
    L.part_len = (long long)(MAXM + 2) * nbp;
    L.dev = (double*)take(4 * (MAXM + 8) * sizeof(double));
    L.theta = (double*)take(4 * sizeof(double));
    L.bytes = off;
    return L;
}

enum { DEV_H1 = 0, DEV_H2 = MAXM + 1, DEV_NRM = 2 * (MAXM + 1), DEV_Y = 2 * (MAXM + 1) + 2,
       DEV_MISC = 3 * (MAXM + 1) + 2 };

// Pinned host slots for the Hessenberg columns (two, used alternately) and the
// scalars the kernels store directly, with the events that mark each slot's step.
// The memory belongs to the context (made by pf_create); this is a view of it.
// Layout (doubles): [slot 0: DEV_Y | slot 1: DEV_Y | y: MAXM | scalars: 8].
struct ColReadback {
    double* host = nullptr;      // host address of the slots
    double* host_dev = nullptr;  // the same memory as the device addresses it
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // slot 0, slot 1, scalars
    double* y() const { return host + 2 * DEV_Y; }
    double* scal() const { return host + 2 * DEV_Y + MAXM; }
    double* scal_dev() const { return host_dev + 2 * DEV_Y + MAXM; }
    // wait for the scalars written by kernels queued so far on s
    int wait_scalars(hipStream_t s) const
    {
        if (hipEventRecord(ev[2], s) != hipSuccess || hipEventSynchronize(ev[2]) != hipSuccess)
            return check_launch("scalar readback");
        return PF_OK;
    }
};
constexpr size_t RB_DOUBLES = 2 * DEV_Y + MAXM + 8;

ColReadback col_readback(const pf_ctx* ctx)
{
    static_assert(MAXM <= pfk::KR_MAXK, "restart length beyond the Gram-Schmidt kernels");
    ColReadback r;
    r.host = ctx->gmres.host;
    r.host_dev = ctx->gmres.dev;
    for (int i = 0; i < 3; ++i) r.ev[i] = ctx->gmres.ev[i];
    return r;
}

struct Opts {
    double rtol, atol, lmin, lmax;
    int max_newton, m, max_its, precond, stagnation, krylov;
};

Opts resolve(const pf_newton_opts* o)
{
    pf_newton_opts d;
    pf_newton_default_opts(&d);
    if (!o) o = &d;
    Opts r{};
    r.rtol = o->rtol;
    r.atol = o->atol;
    r.lmin = o->lin_rtol_min;
    r.lmax = o->lin_rtol_max;
    r.max_newton = o->max_newton;
    r.m = o->gmres_restart;
    r.max_its = o->gmres_max_its;
    r.precond = o->precond;
    r.stagnation = o->stagnation;
    r.krylov = o->krylov;
    return r;
}

int check_opts(const Opts& o)
{
    if (!(o.rtol >= 0.0) || !(o.atol >= 0.0) || !std::isfinite(o.rtol) || !std::isfinite(o.atol))
        return fail(PF_EINVAL, "rtol/atol must be finite and >= 0");
    if (o.max_newton < 0 || o.max_newton > 1000) return fail(PF_EINVAL, "max_newton out of range");
    if (o.m < 1 || o.m > MAXM) return fail(PF_EINVAL, "gmres_restart must be in 1..%d", MAXM);
    if (o.max_its < 1) return fail(PF_EINVAL, "gmres_max_its must be >= 1");
    if (o.precond != PF_PRECOND_NONE && o.precond != PF_PRECOND_JACOBI)
        return fail(PF_EINVAL, "unknown preconditioner");
    if (!(o.lmin > 0.0) || !(o.lmax >= o.lmin) || !(o.lmax < 1.0))
        return fail(PF_EINVAL, "need 0 < lin_rtol_min <= lin_rtol_max < 1");
    if (o.krylov != PF_KRYLOV_GMRES && o.krylov != PF_KRYLOV_CG) return fail(PF_EINVAL, "unknown krylov solver");
    return PF_OK;
}

// CG needs a symmetric positive definite Jacobian.  Allen-Cahn's is
// (m/dt) M + L (N'(eta) + kappa K) with N'(eta) >= -W M_c (f'' >= -W for both
// double wells) and M_c <= the lumped mass, so dt L W < 1 makes it positive
// definite for every eta; the other models are not symmetric (or not definite).
int check_cg(const pf_problem* p, double dt, const Opts& o)
{
    if (o.krylov != PF_KRYLOV_CG) return PF_OK;
    if (p->model != PF_ALLEN_CAHN) return fail(PF_EINVAL, "krylov = CG needs the Allen-Cahn model");
    // positive definiteness below rests on L > 0, kappa >= 0 (K is positive
    // semi-definite) and W >= 0 (f'' >= -W for both double wells)
    if (!(p->mobility > 0.0)) return fail(PF_EINVAL, "krylov = CG needs mobility > 0 (got %g)", p->mobility);
    if (!(p->kappa >= 0.0)) return fail(PF_EINVAL, "krylov = CG needs kappa >= 0 (got %g)", p->kappa);
    if (!(p->W >= 0.0)) return fail(PF_EINVAL, "krylov = CG needs W >= 0 (got %g)", p->W);
    if (!(dt * p->mobility * p->W < 1.0))
        return fail(PF_EINVAL, "krylov = CG needs dt L W < 1 (got %g): the Jacobian may be indefinite",
                    dt * p->mobility * p->W);
    return PF_OK;
}

int d2h(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return check_launch("device-to-host read");
    return PF_OK;
}

// The linear operator handed to GMRES: J = dR/dU at U (or its transpose).
template <typename T>
struct LinOp {
    const pf_problem* p;
    pfk::Geom g;
    pfk::FreeEnergy f;
    double inv_dt;
    const T* U;
    int trans;
    void apply(const T* v, T* out, hipStream_t s) const
    {
        if (p->model == PF_COUPLED)
            pfk::launch_cp_jvp<T>(g, p->kappa, p->mobility, p->mobility_eta, inv_dt, U, v, out, s);
        else if (p->model == PF_GRAIN)
            pfk::launch_gg_jvp2d<T>(g, p->nfields, p->mobility, p->kappa, p->gamma, inv_dt, U, v, out, s);
        else
            pfk::launch_jvp<T>(g, p->model, f, p->kappa, p->mobility, inv_dt, U, v, out, s, trans, 0);
    }
    // out = J v with the per-block partial sums of v . out in part2 (at most max_blocks),
    // their count in *nb; false (nothing launched) where the operator has no such fused
    // form (then apply and a separate sum are needed)
    bool apply_pq(const T* v, T* out, double* part2, int* nb, int max_blocks, hipStream_t s) const
    {
        if (p->model != PF_ALLEN_CAHN) return false;
        return pfk::launch_jvp2d_stream<T>(g, p->model, f, p->kappa, p->mobility, inv_dt, U, v, out, s, part2, nb,
                                           max_blocks);
    }
};

// Solve J x = b (x overwritten, starting from 0) to ||b - J x|| <= tol_abs.
// The preconditioner (if any) must already be in L.pinv.  Returns PF status;
// *its receives the Arnoldi steps taken, *res the last residual estimate.
template <typename T>
int gmres(const ColReadback* rb, const LinOp<T>& A, NWS<T>& L, long long n, int m, int max_its, bool prec,
          double bnorm, double tol_abs, int* its, double* res, hipStream_t s)
{
    // grain growth: point Jacobi over all p N unknowns (the Krylov kernels' point model)
    const bool grain = A.p->model == PF_GRAIN;
    const int model = grain ? 0 : A.p->model;
    const long long Nn = grain ? n : A.g.N;
    const T* pinv = prec ? L.pinv : nullptr;
    const int tr = A.trans;
    double* dh1 = L.dev + DEV_H1;
    double* dh2 = L.dev + DEV_H2;
    double* dnrm = L.dev + DEV_NRM;
    double* dy = L.dev + DEV_Y;
    if (hipMemsetAsync(L.x, 0, (size_t)n * sizeof(T), s) != hipSuccess) return check_launch("gmres init");
    std::array<double, (MAXM + 1) * MAXM> H{};
    std::array<double, MAXM> cs{}, sn{}, y{};
    std::array<double, MAXM + 1> gv{};
    int total = 0;
    double beta = bnorm;
    bool first = true;
    *res = bnorm;
    if (bnorm <= tol_abs) {
        *its = 0;
        return PF_OK;
    }
    for (;;) {
        // v0 = r / ||r||, z = P^-1 v0 with r = b - J x (= b on the first cycle)
        if (first) {
            pfk::kr_norm2<T>(L.b, nullptr, n, L.part, dnrm, s);
        } else {
            A.apply(L.x, L.w, s);
            pfk::kr_rsub<T>(L.b, L.w, n, s);
            pfk::kr_norm2<T>(L.w, nullptr, n, L.part, dnrm, s, rb->scal_dev());
            if (int rc = rb->wait_scalars(s)) return rc;
            beta = std::sqrt(rb->scal()[0]);
            *res = beta;
            if (!std::isfinite(beta)) return fail(PF_ENONFINITE, "GMRES residual is not finite");
            if (beta <= tol_abs || total >= max_its) break;
        }
        pfk::kr_normalize_prec<T>(model, first ? L.b : L.w, dnrm, L.V, L.z, pinv, Nn, 1.0, s, tr);
        first = false;
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        // Arnoldi step i: w = J z_i, orthogonalise, v_{i+1} and z_{i+1}; its
        // column goes to pinned slot i % 2
        auto enqueue = [&](int i) -> int {
            A.apply(L.z, L.w, s);
            double* slot = rb->host_dev + (i & 1) * DEV_Y;
            const pfk::KrOut out{dh1, dh2, dnrm, slot + DEV_H1, slot + DEV_H2, slot + DEV_NRM};
            if (pfk::kr_cgs2<T>(model, L.V, L.ld, i + 1, L.w, L.V + (long long)(i + 1) * L.ld, L.z, pinv,
                                Nn, L.part, out, s, tr))
                return fail(PF_EINVAL, "Gram-Schmidt basis of %d vectors", i + 1);
            if (hipEventRecord(rb->ev[i & 1], s) != hipSuccess) return check_launch("GMRES column readback");
            return PF_OK;
        };
        int j = 0;
        bool done = false;
        const int steps = std::min(m, max_its - total);
        if (steps > 0)
            if (int rc = enqueue(0)) return rc;
        for (; j < steps; ++j) {
            if (j + 1 < steps)
                if (int rc = enqueue(j + 1)) return rc;
            if (hipEventSynchronize(rb->ev[j & 1]) != hipSuccess) return check_launch("GMRES column wait");
            const double* col = rb->host + (j & 1) * DEV_Y;
            ++total;
            for (int i = 0; i <= j; ++i) H[i * MAXM + j] = col[DEV_H1 + i] + col[DEV_H2 + i];
            const double hn = std::sqrt(std::max(col[DEV_NRM], 0.0));
            H[(j + 1) * MAXM + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * MAXM + j] + sn[i] * H[(i + 1) * MAXM + j];
                H[(i + 1) * MAXM + j] = -sn[i] * H[i * MAXM + j] + cs[i] * H[(i + 1) * MAXM + j];
                H[i * MAXM + j] = t;
            }
            const double a = H[j * MAXM + j], bb = H[(j + 1) * MAXM + j];
            const double rr = std::hypot(a, bb);
            if (!std::isfinite(rr)) {
                hipStreamSynchronize(s);
                return fail(PF_ENONFINITE, "GMRES Hessenberg is not finite");
            }
            cs[j] = rr > 0.0 ? a / rr : 1.0;
            sn[j] = rr > 0.0 ? bb / rr : 0.0;
            H[j * MAXM + j] = rr;
            H[(j + 1) * MAXM + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            *res = std::fabs(gv[j + 1]);
            if (*res <= tol_abs || hn == 0.0) {
                ++j;
                done = true;
                break;
            }
        }
        // y = H^-1 g (upper triangular j x j), x += P^-1 V y
        for (int i = j - 1; i >= 0; --i) {
            double sum = gv[i];
            for (int k = i + 1; k < j; ++k) sum -= H[i * MAXM + k] * y[k];
            y[i] = H[i * MAXM + i] != 0.0 ? sum / H[i * MAXM + i] : 0.0;
        }
        if (j > 0) {
            // pinned source: the copy is asynchronous; the host rewrites y only after
            // waiting on work queued behind it
            std::copy(y.begin(), y.begin() + j, rb->y());
            if (hipMemcpyAsync(dy, rb->y(), (size_t)j * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
                return check_launch("GMRES solution coefficients");
            pfk::kr_update<T>(model, L.V, L.ld, j, dy, pinv, L.x, Nn, s, tr);
        }
        if (done || total >= max_its) break;
    }
    *its = total;
    return check_launch("gmres");
}

// Preconditioned CG on J x = b (x overwritten, starting from 0) to
// ||b - J x|| <= tol_abs, for a symmetric positive definite J (check_cg).  The
// scalars stay on the device; the host reads the pinned mirror one iteration
// behind the GPU.  Returns PF status; *its: iterations, *res: ||r||.
template <typename T>
int pcg(const ColReadback* rb, const LinOp<T>& A, NWS<T>& L, long long n, int max_its, bool prec, double bnorm,
        double tol_abs, int* its, double* res, hipStream_t s)
{
    *its = 0;
    *res = bnorm;
    const T* pinv = prec ? L.pinv : nullptr;
    T* r = L.V;
    T* pdir = L.V + L.ld;
    T* q = L.V + 2 * L.ld;
    double* part = L.part;
    double* part2 = L.part + 2 * pfk::cg_blocks(n);
    // room for part2 in the workspace's partial-sum area (MAXM + 2 rows of nbp)
    const int pq_max = (int)std::min<long long>(INT_MAX, L.part_len - 2 * pfk::cg_blocks(n));
    double* st = L.dev + DEV_MISC;
    double* hdev = rb->scal_dev();
    const double* h = rb->scal();
    pfk::cg_start<T>(L.b, pinv, r, L.z, pdir, L.x, n, part, st, hdev, tol_abs * tol_abs, max_its, s);
    if (bnorm <= tol_abs) return check_launch("CG start");
    int enq = 0, slot = 0;
    bool pending = false;
    for (;;) {
        pfk::cg_dir<T>(L.z, pdir, n, part, st, hdev, s);
        int nb2 = 0;  // the Jacobian product may leave the p . q partials itself
        if (!A.apply_pq(pdir, q, part2, &nb2, pq_max, s)) {
            A.apply(pdir, q, s);
            pfk::cg_pq<T>(pdir, q, n, part2, st, s);
            nb2 = 0;
        }
        pfk::cg_alpha<T>(L.x, r, L.z, pdir, q, pinv, n, part2, part, st, hdev, s, nb2);
        ++enq;
        if (int rc = check_launch("CG iteration")) return rc;
        if (hipEventRecord(rb->ev[slot], s) != hipSuccess) return check_launch("CG event");
        if (pending) {
            if (hipEventSynchronize(rb->ev[slot ^ 1]) != hipSuccess) return check_launch("CG wait");
            if (*(volatile const double*)&h[pfk::CG_H_DONE] != 0.0) break;
        }
        pending = true;
        slot ^= 1;
        if (enq > max_its) break;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return check_launch("CG sync");
    const double done = *(volatile const double*)&h[pfk::CG_H_DONE];
    *its = (int)*(volatile const double*)&h[pfk::CG_H_ITS];
    *res = std::sqrt(std::max((double)*(volatile const double*)&h[pfk::CG_H_RR], 0.0));
    if (done == pfk::CG_NONFINITE) return fail(PF_ENONFINITE, "CG met a non-finite value");
    if (done == pfk::CG_BREAKDOWN)
        return fail(PF_ENOCONV, "CG breakdown after %d iterations (Jacobian not positive definite)", *its);
    return PF_OK;  // converged, or the iteration limit (an inexact correction, as GMRES)
}

template <typename T>
double eps_of()
{
    return sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
}

template <typename T>
int newton_t(const pf_ctx* ctx, const pf_problem* p, double dt, const T* Uold, T* U, const Opts& o,
             pf_newton_report* rep, void* ws, hipStream_t s)
{
    const pfk::Geom g = geom_of(p);
    const pfk::FreeEnergy f = pfk::make_free_energy(p->fe, p->W);
    const long long n = ndof(p);
    NWS<T> L = layout<T>(p, ws);
    const double inv_dt = 1.0 / dt;
    double* dnrm = L.dev + DEV_NRM;
    double* dmisc = L.dev + DEV_MISC;
    pf_newton_report R{};
    const ColReadback rbv = col_readback(ctx);
    const ColReadback* rb = &rbv;
    // ||R(U)||, read back together with whatever scalars were queued before it
    auto residual_norm = [&](double* out) -> int {
        if (p->model == PF_COUPLED)
            pfk::launch_cp_residual<T>(g, p->kappa, p->mobility, p->mobility_eta, U, L.R, s, Uold, inv_dt);
        else if (p->model == PF_GRAIN)
            pfk::launch_gg_tile2d<T>(g, p->nfields, p->mobility, p->kappa, p->gamma, 0.0, U, L.R, 1, s, Uold,
                                     inv_dt);
        else
            pfk::launch_residual<T>(g, p->model, f, p->kappa, p->mobility, U, L.R, s, Uold, inv_dt);
        pfk::kr_norm2<T>(L.R, nullptr, n, L.part, dnrm, s, rb->scal_dev());
        if (int rc = rb->wait_scalars(s)) return rc;
        *out = std::sqrt(rb->scal()[0]);
        return PF_OK;
    };
    double r0;
    if (int rc = residual_norm(&r0)) return rc;
    R.res_norm[0] = r0;
    R.reason = -1;
    int status = PF_OK;
    double rk = r0, rprev = r0;
    if (!std::isfinite(r0)) {
        R.reason = -2;
        status = fail(PF_ENONFINITE, "initial residual is not finite");
    }
    const LinOp<T> A{p, g, f, inv_dt, U, 0};
    int k = 0;
    double dmax = 0.0, umax = 0.0;
    while (status == PF_OK) {
        if (rk <= o.rtol * r0) { R.converged = 1; R.reason = 0; break; }
        if (rk <= o.atol) { R.converged = 1; R.reason = 1; break; }
        // rounding floor: the residual stopped falling, and either the last correction
        // was within a few units in the last place of the field, or it left the
        // residual where it was (within 10%) although it was too small (at most
        // sqrt(eps) of the field) for the nonlinearity to undo a converged linear
        // solve -- the residual was rounding noise, whose correction can stay well
        // above the field's last place
        if (o.stagnation && k >= 2 && rk > 0.5 * rprev &&
            (dmax <= 8.0 * eps_of<T>() * umax ||
             (rk > 0.9 * rprev && dmax <= std::sqrt(eps_of<T>()) * umax))) {
            R.converged = 1;
            R.reason = 2;  // rounding floor of the field precision reached
            break;
        }
        if (k >= o.max_newton) break;
        if (o.precond == PF_PRECOND_JACOBI) {
            if (p->model == PF_COUPLED)
                pfk::launch_cp_prec<T>(g, p->kappa, p->mobility, p->mobility_eta, inv_dt, U, L.pinv, s);
            else if (p->model == PF_GRAIN)
                pfk::launch_gg_tile2d<T>(g, p->nfields, p->mobility, p->kappa, p->gamma, 0.0, U, L.pinv, 2, s,
                                         nullptr, inv_dt);
            else
                pfk::launch_prec<T>(g, p->model, f, p->kappa, p->mobility, inv_dt, U, L.pinv, s);
        }
        pfk::kr_scale<T>(L.R, L.b, -1.0, n, s);  // b = -R
        const double lin = std::min(o.lmax, std::max(o.lmin, 0.1 * rk / r0));
        int its = 0;
        double lres = 0.0;
        const bool jac = o.precond == PF_PRECOND_JACOBI;
        if (int rc = o.krylov == PF_KRYLOV_CG ? pcg<T>(rb, A, L, n, o.max_its, jac, rk, lin * rk, &its, &lres, s)
                                              : gmres<T>(rb, A, L, n, o.m, o.max_its, jac, rk, lin * rk, &its,
                                                         &lres, s)) {
            status = rc;
            R.reason = -2;
            break;
        }
        R.gmres_its += its;
        pfk::kr_add_maxabs<T>(U, L.x, n, L.part, dmisc, s, rb->scal_dev() + 1);
        rprev = rk;
        if (int rc = residual_norm(&rk)) return rc;
        dmax = rb->scal()[1];
        umax = rb->scal()[2];
        ++k;
        if (k <= 32) R.res_norm[k] = rk;
        if (!std::isfinite(rk)) {
            R.reason = -2;
            status = fail(PF_ENONFINITE, "Newton residual is not finite");
        }
    }
    R.newton_its = k;
    if (rep) *rep = R;
    if (status != PF_OK) return status;
    if (!R.converged)
        return fail(PF_ENOCONV, "Newton stopped after %d corrections at ||R|| = %.3e (||R0|| = %.3e)",
                    k, rk, r0);
    return check_launch("pf_newton_step");
}

}  // namespace

size_t newton_workspace_bytes(const pf_problem* p, int)
{
    return p->dtype == PF_F64 ? layout<double>(p, nullptr).bytes : layout<float>(p, nullptr).bytes;
}

size_t vjp_workspace_bytes(const pf_problem* p) { return newton_workspace_bytes(p, MAXM); }

template <typename T>
int vjp_simple_t(const pf_problem* p, int kind, double dt, bool be, const T* U, const T* vbar, T* Ubar,
                 double* theta_bar, void* ws, hipStream_t s)
{
    const pfk::Geom g = geom_of(p);
    const pfk::FreeEnergy f = pfk::make_free_energy(p->fe, p->W);
    NWS<T> L = layout<T>(p, ws);
    if (kind == PF_VJP_RESIDUAL) {
        // Ubar += (dr/dU)^T vbar : the transpose Jacobian product with no time term
        pfk::launch_jvp<T>(g, p->model, f, p->kappa, p->mobility, 0.0, U, vbar, Ubar, s, 1, 1);
        // backward-Euler residual R = M (U - U_old)/dt + r (Eq. 14): M is symmetric,
        // so its transposed time term adds (M/dt) vbar on the mass rows
        if (be) pfk::launch_mass_axpy<T>(g, 1.0 / dt, vbar, Ubar, s);
        pfk::launch_dtheta<T>(g, p->model, f, p->kappa, p->mobility, U, vbar, 1.0, L.part,
                              theta_bar, s);
    } else {
        pfk::launch_vjp_explicit<T>(g, p->model, f, p->kappa, p->mobility, dt, U, vbar, Ubar, L.V,
                                    L.part, theta_bar, s);
    }
    return check_launch("pf_vjp");
}

// Adjoint of one backward-Euler step at its root U (II.5-II.6):
// solve (dR/dU)^T lambda = vbar, then Uold_bar += (M/dt) lambda on the mass
// rows and theta_bar -= (dr/dtheta)^T lambda.  lambda is left in the
// workspace's x vector.
template <typename T>
int newton_adjoint_t(const pf_ctx* ctx, const pf_problem* p, double dt, const T* U, const T* vbar, T* Ubar,
                     double* theta_bar, const Opts& o, void* ws, hipStream_t s)
{
    const ColReadback rbv = col_readback(ctx);
    const pfk::Geom g = geom_of(p);
    const pfk::FreeEnergy f = pfk::make_free_energy(p->fe, p->W);
    const long long n = ndof(p);
    NWS<T> L = layout<T>(p, ws);
    const double inv_dt = 1.0 / dt;
    if (o.precond == PF_PRECOND_JACOBI)
        pfk::launch_prec<T>(g, p->model, f, p->kappa, p->mobility, inv_dt, U, L.pinv, s);
    if (hipMemcpyAsync(L.b, vbar, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return check_launch("adjoint rhs copy");
    pfk::kr_norm2<T>(L.b, nullptr, n, L.part, L.dev + DEV_NRM, s);
    double nn;
    if (int rc = d2h(&nn, L.dev + DEV_NRM, sizeof(double), s)) return rc;
    const double bn = std::sqrt(nn);
    if (!std::isfinite(bn)) return fail(PF_ENONFINITE, "adjoint right-hand side is not finite");
    const LinOp<T> At{p, g, f, inv_dt, U, 1};
    int its = 0;
    double res = 0.0;
    // the adjoint solve is taken to the field-precision floor, not an inexact-Newton tolerance
    const double tol = (sizeof(T) == 4 ? 1e-6 : 1e-12) * bn;
    const bool jac = o.precond == PF_PRECOND_JACOBI;
    // (Allen-Cahn's Jacobian is symmetric: CG solves the transposed system as well)
    if (int rc = o.krylov == PF_KRYLOV_CG ? pcg<T>(&rbv, At, L, n, o.max_its * 4, jac, bn, tol, &its, &res, s)
                                          : gmres<T>(&rbv, At, L, n, o.m, o.max_its * 4, jac, bn, tol, &its, &res,
                                                     s))
        return rc;
    // Ubar (mass rows) += (m/dt) lambda ; theta_bar -= (dr/dtheta)^T lambda
    pfk::launch_mass_axpy<T>(g, inv_dt, L.x, Ubar, s);
    pfk::launch_dtheta<T>(g, p->model, f, p->kappa, p->mobility, U, L.x, -1.0, L.part, theta_bar, s);
    return check_launch("newton adjoint");
}

int newton_adjoint(const pf_ctx* ctx, const pf_problem* p, double dt, const void* U, const void* vbar, void* Ubar,
                   double* theta_bar, void* ws, hipStream_t s)
{
    const Opts o = resolve(nullptr);
    if (p->dtype == PF_F32)
        return newton_adjoint_t<float>(ctx, p, dt, (const float*)U, (const float*)vbar, (float*)Ubar,
                                       theta_bar, o, ws, s);
    return newton_adjoint_t<double>(ctx, p, dt, (const double*)U, (const double*)vbar, (double*)Ubar,
                                    theta_bar, o, ws, s);
}

size_t newton_pinned_doubles() { return RB_DOUBLES; }

}  // namespace pfapi

using namespace pfapi;

extern "C" {

void pf_newton_default_opts(pf_newton_opts* o)
{
    if (!o) return;
    *o = pf_newton_opts{};
    o->rtol = 1e-8;
    o->atol = 0.0;
    o->max_newton = 20;
    o->gmres_restart = 30;
    o->gmres_max_its = 600;
    o->precond = PF_PRECOND_JACOBI;
    o->lin_rtol_max = 1e-2;
    o->lin_rtol_min = 1e-6;
    o->stagnation = 1;
}

int pf_newton_step(pf_ctx* ctx, const pf_problem* p, double dt, const void* U_old, void* U,
                   const pf_newton_opts* opts, pf_newton_report* rep, void* ws, void* stream)
{
    return guarded("pf_newton_step", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (p->model == PF_GRAIN)
            if (int rc = grain_implicit_ok(p)) return rc;
        if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PF_EINVAL, "dt must be finite and > 0");
        if (int rc = check_ptr(U_old, p, "U_old")) return rc;
        if (int rc = check_ptr(U, p, "U")) return rc;
        if (U == U_old) return fail(PF_EINVAL, "U and U_old must not alias");
        if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws must be 256-byte aligned");
        const Opts o = resolve(opts);
        if (int rc = check_opts(o)) return rc;
        if (int rc = check_cg(p, dt, o)) return rc;
        if (int rc = require_device(ctx)) return rc;
        hipStream_t s = (hipStream_t)stream;
        if (p->dtype == PF_F32)
            return newton_t<float>(ctx, p, dt, (const float*)U_old, (float*)U, o, rep, ws, s);
        return newton_t<double>(ctx, p, dt, (const double*)U_old, (double*)U, o, rep, ws, s);
    });
}

int pf_vjp(pf_ctx* ctx, const pf_problem* p, int kind, double dt, const void* U, const void* U_old,
           const void* vbar, void* Ubar, double* theta_bar, int flags, void* ws, void* stream)
{
    return guarded("pf_vjp", [&]() -> int {
        if (int rc = check_ctx(ctx)) return rc;
        if (int rc = validate(p)) return rc;
        if (p->model == PF_COUPLED) return fail(PF_EUNSUPPORTED, "pf_vjp: coupled model not implemented");
        if (p->model == PF_GRAIN) return fail(PF_EUNSUPPORTED, "pf_vjp: grain growth not implemented");
        if (p->quad != PF_QUAD_GAUSS) return fail(PF_EUNSUPPORTED, "pf_vjp: Gauss-Lobatto quadrature not implemented");
        if (kind != PF_VJP_RESIDUAL && kind != PF_VJP_EXPLICIT_STEP && kind != PF_VJP_NEWTON_STEP)
            return fail(PF_EINVAL, "unknown vjp kind %d", kind);
        if (flags & ~PF_VJP_THETA_HOST) return fail(PF_EINVAL, "unknown flags 0x%x", flags);
        const bool be = kind == PF_VJP_RESIDUAL && U_old != nullptr;
        if ((kind != PF_VJP_RESIDUAL || be) && (!(dt > 0.0) || !std::isfinite(dt)))
            return fail(PF_EINVAL, "dt must be finite and > 0");
        if (kind == PF_VJP_EXPLICIT_STEP && p->mass != PF_MASS_LUMPED)
            return fail(PF_EUNSUPPORTED, "explicit steps need the lumped mass");
        if (int rc = check_ptr(U, p, "U")) return rc;
        if (U_old)
            if (int rc = check_ptr(U_old, p, "U_old")) return rc;
        if (int rc = check_ptr(vbar, p, "vbar")) return rc;
        if (int rc = check_ptr(Ubar, p, "Ubar")) return rc;
        if (Ubar == U || Ubar == vbar) return fail(PF_EINVAL, "Ubar must not alias U or vbar");
        if (!theta_bar || reinterpret_cast<uintptr_t>(theta_bar) % 8)
            return fail(PF_EINVAL, "theta_bar is NULL or misaligned");
        if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws must be 256-byte aligned");
        if (int rc = require_device(ctx)) return rc;
        hipStream_t s = (hipStream_t)stream;
        const bool host_theta = (flags & PF_VJP_THETA_HOST) != 0;
        double* tb = theta_bar;
        if (host_theta) {  // accumulate into a device copy, then return it to the host
            tb = p->dtype == PF_F32 ? layout<float>(p, ws).theta : layout<double>(p, ws).theta;
            if (hipMemcpyAsync(tb, theta_bar, 3 * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
                return check_launch("theta_bar upload");
        }
        int rc;
        if (kind == PF_VJP_NEWTON_STEP)
            rc = newton_adjoint(ctx, p, dt, U, vbar, Ubar, tb, ws, s);
        else if (p->dtype == PF_F32)
            rc = vjp_simple_t<float>(p, kind, dt, be, (const float*)U, (const float*)vbar, (float*)Ubar, tb, ws, s);
        else
            rc = vjp_simple_t<double>(p, kind, dt, be, (const double*)U, (const double*)vbar, (double*)Ubar, tb,
                                      ws, s);
        if (rc != PF_OK || !host_theta) return rc;
        if (hipMemcpyAsync(theta_bar, tb, 3 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return check_launch("theta_bar download");
        return PF_OK;
    });
}

}  // extern "C"

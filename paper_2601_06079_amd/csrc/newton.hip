// newton.hip -- backward-Euler Newton step and sensitivities (filled in below).
#include "api_internal.hpp"

namespace pfapi {
size_t newton_workspace_bytes(const pf_problem* p, int restart) { (void)p; (void)restart; return 0; }
size_t vjp_workspace_bytes(const pf_problem* p) { (void)p; return 0; }
}  // namespace pfapi

using namespace pfapi;
extern "C" {
void pf_newton_default_opts(pf_newton_opts* o)
{
    if (!o) return;
    *o = pf_newton_opts{};
    o->rtol = 1e-8; o->atol = 0.0; o->max_newton = 20; o->gmres_restart = 30;
    o->gmres_max_its = 600; o->precond = PF_PRECOND_JACOBI; o->lin_rtol_max = 1e-2;
    o->lin_rtol_min = 1e-6; o->stagnation = 1;
}
int pf_newton_step(const pf_problem* p, double, const void*, void*, const pf_newton_opts*,
                   pf_newton_report*, void*, void*)
{
    if (int rc = validate(p)) return rc;
    return fail(PF_EUNSUPPORTED, "pf_newton_step: not built yet");
}
int pf_vjp(const pf_problem* p, int, double, const void*, const void*, void*, double*, void*, void*)
{
    if (int rc = validate(p)) return rc;
    return fail(PF_EUNSUPPORTED, "pf_vjp: not built yet");
}
}

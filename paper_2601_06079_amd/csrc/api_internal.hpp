// api_internal.hpp -- helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <exception>
#include <new>

#include "../../include/pf.h"
#include "ctx.hpp"
#include "kernels.hpp"

namespace pfapi {

int fail(int status, const char* fmt, ...);
int check_launch(const char* what);
int validate(const pf_problem* p);
int check_ptr(const void* ptr, const pf_problem* p, const char* name);
pfk::Geom geom_of(const pf_problem* p);
long long ndof(const pf_problem* p);
size_t elem_size(const pf_problem* p);
int grain_implicit_ok(const pf_problem* p);

// Runs an entry point's body; a C++ exception (a host allocation that failed, an
// internal error) becomes PF_EDEVICE with a message instead of crossing the ABI.
template <class F>
int guarded(const char* name, F&& body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(PF_EDEVICE, "%s: host memory exhausted", name);
    } catch (const std::exception& e) {
        return fail(PF_EDEVICE, "%s: %s", name, e.what());
    } catch (...) {
        return fail(PF_EDEVICE, "%s: unexpected internal error", name);
    }
}

// launch shape of the fused 2-D explicit kernel for this problem (tuning table):
// steps fused per launch, rows per wave for a given fusion depth on a device of
// `cus` compute units, prefetch depth
int stream2d_fuse(const pf_problem* p);
int stream2d_rows(const pf_problem* p, int ks, int cus);
int stream2d_depth(const pf_problem* p);

size_t newton_workspace_bytes(const pf_problem* p, int restart);
size_t vjp_workspace_bytes(const pf_problem* p);

}  // namespace pfapi

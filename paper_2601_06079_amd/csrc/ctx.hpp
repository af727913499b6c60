// ctx.hpp -- the per-device context behind the opaque pf_ctx of include/pf.h.
//
// A context owns what the library keeps between calls on one device: the device
// properties the launchers size their grids with, the pinned host slots the
// Newton/GMRES and elasticity CG kernels store their scalars into (made once at
// pf_create, never inside a compute call), the smoother eigenvalue cache of the
// elasticity multigrid and the batch autotuner's results.  Calls that share a
// context must not run concurrently on different host threads (one context per
// thread, or external locking); the mutex only guards the two caches.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "../../include/pf.h"

namespace pfapi {

// Pinned, device-mapped host memory that kernels store into and the host polls.
struct PinnedSlots {
    double* host = nullptr;  // host address
    double* dev = nullptr;   // the same memory as the device addresses it
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};

// signature of a batch shape, the key of the autotuner's results
struct BatchShapeKey {
    int model, dtype, count;
    long long cells, maxn;
    bool operator<(const BatchShapeKey& o) const
    {
        return std::tie(model, dtype, count, cells, maxn) < std::tie(o.model, o.dtype, o.count, o.cells, o.maxn);
    }
};

// sizes of the pinned slots (doubles), defined by their users
size_t newton_pinned_doubles();
size_t elastic_pinned_doubles();

}  // namespace pfapi

struct pf_ctx {
    int device = -1;  // PF_HOST_ONLY: sizing and validation only
    int cus = 256;    // compute units (4 SIMDs each)
    pfapi::PinnedSlots gmres;  // Hessenberg columns and CG scalars (pf_newton_step, pf_vjp)
    pfapi::PinnedSlots cg;     // elasticity CG / PCG scalars and stop flag
    std::mutex mu;
    std::map<std::pair<int, double>, double> el_lmax;  // lambda_max(D^-1 K) per (dim, nu)
    std::map<pfapi::BatchShapeKey, std::array<int, 3>> tuned;  // (ks, ty, depth) per batch shape
    double* scratch = nullptr;  // this device's address of the library's static energy scratch
};

namespace pfapi {
// PF_EINVAL unless ctx is non-NULL (any context: sizing and validation)
int check_ctx(const pf_ctx* ctx);
// PF_EINVAL unless ctx is a device context and its device is the current one
int require_device(const pf_ctx* ctx);
}  // namespace pfapi

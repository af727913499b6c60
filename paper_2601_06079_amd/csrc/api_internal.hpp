// api_internal.hpp -- helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/pf.h"
#include "kernels.hpp"

namespace pfapi {

int fail(int status, const char* fmt, ...);
int check_launch(const char* what);
int validate(const pf_problem* p);
int check_ptr(const void* ptr, const pf_problem* p, const char* name);
pfk::Geom geom_of(const pf_problem* p);
long long ndof(const pf_problem* p);
size_t elem_size(const pf_problem* p);

// rows per wave of the 2-D streaming kernel for this problem (tuning table)
int stream2d_rows(const pf_problem* p);
int stream2d_depth(const pf_problem* p);

size_t newton_workspace_bytes(const pf_problem* p, int restart);
size_t vjp_workspace_bytes(const pf_problem* p);

}  // namespace pfapi

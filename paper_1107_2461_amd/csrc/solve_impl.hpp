// Host-side solve sequence shared by the C entry points helm_solve and helm_solve_noalloc.
#pragma once

#include "../../include/helm.h"

namespace helm {

// Runs one solve with the caller's (or the library's static) workspace `ws`.  noalloc = true
// refuses (EINVAL) the two paths that allocate on demand: adaptive refinement (ir_tol > 0 on a
// refined plan) and stage timing.
helm_status solve_impl(helm_plan* p, const double* f, double* u, int nrhs, const double* sigma_per_rhs, void* ws,
                       void* stream, helm_info* info, bool noalloc);

// The HIP device a plan lives on (-1 for a null plan).
int plan_device(const helm_plan* p);

}  // namespace helm

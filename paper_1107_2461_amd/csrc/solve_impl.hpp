// Host-side solve sequence shared by the C entry points helm_solve and helm_solve_noalloc.
#pragma once

#include "../../include/helm.h"

namespace helm {

// Device tables of a grouped solve (the right-hand sides of several plans of one shape solved
// together, one launch per stage): for every RHS, the operands and eigenvalues of its own plan.
// The tables live in the solve's workspace, after the plan's own layout.
struct GroupTabs {
  const void* const* msw[3][2] = {};     // [axis][forward, inverse]: swizzled operand per RHS
  const double* const* lam[3] = {};      // eigenvalues per axis and RHS
  const double* const* lamxy = nullptr;  // split-BF16 lambda_x + lambda_y table per RHS
  const double* const* coef[3] = {};     // 7-point operator rows per axis and RHS
  const helm_plan* const* rhs_plan = nullptr;  // host: the plan of every RHS
};

// Runs one solve with the caller's (or the library's static) workspace `ws`.  noalloc = true
// refuses (EINVAL) the two paths that allocate on demand: adaptive refinement (ir_tol > 0 on a
// refined plan) and stage timing.  grp: a grouped solve (p is the group's first plan, which
// fixes the shape, precision and options).
helm_status solve_impl(helm_plan* p, const double* f, double* u, int nrhs, const double* sigma_per_rhs, void* ws,
                       void* stream, helm_info* info, bool noalloc, const GroupTabs* grp = nullptr);

// The HIP device a plan lives on (-1 for a null plan).
int plan_device(const helm_plan* p);

// Whether right-hand sides of plans a and b can always share a grouped solve: the conditions
// of helm_solve_group, and a shape whose per-RHS extents (ny nz, nz nx, nx ny) are multiples of
// 512, which every stage's tiling divides.
bool plans_groupable(const helm_plan* a, const helm_plan* b);
// Frees a plan without the device-wide synchronization of helm_destroy, for an owner that has
// already waited for every solve it enqueued with the plan (the solve server: a plan's last
// reference is dropped after the worker's stream wait).
void release_plan(helm_plan* p);

}  // namespace helm

// pf_batched.hpp -- many-disk forward map and launch-shape tuning.
#pragma once
#include <vector>

#include "pf_common.hpp"

namespace pf {

// Forward map for several plans of one precision as grouped launches (pass
// A, B, C of every disk, one launch per class of transform length and
// launch shape).
int batched_forces(const std::vector<const Plan *> &plans, const void *const *sigma,
                   void *const *f_r, void *const *f_phi, hipStream_t st);
// The same without allocating: the batch's tables go to a static device
// array of the library (at most 256 disks); see pf_forces_batched_noalloc.
int batched_forces_noalloc(const Plan *const *plans, int n, const void *const *sigma,
                           void *const *f_r, void *const *f_phi, hipStream_t st);
// Drop cached batch state that refers to plan `uid`.
void batched_forget(int64_t uid);
// Choose launch shapes for the plan's sizes (timed on the device, cached).
// A failed HIP call or launch returns its status (message in pf_last_error)
// and leaves the plan's shapes as they were.
int autotune_plan(Plan &p, hipStream_t st);

}  // namespace pf

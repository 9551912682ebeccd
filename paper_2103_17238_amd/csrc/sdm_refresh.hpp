// sdm_refresh.hpp -- device-side refresh of a launch plan after the cell
// layout of its simulation changed (libsdm internal).
#pragma once

#include "sdm_internal.hpp"

namespace sdm {

// Rewrites every workgroup-per-cell task of the plan (both dispatch-order
// lists of the adaptive cells included) from the new offsets `off` of its
// single simulation, whose state now starts at xi / v.  Word w[0] gets bit 1
// if the offsets are not a valid layout of n_slots, bit 2 if a cell no longer
// fits its class; w[1] the sum of the task cells' new sizes (equal to
// n_slots exactly when no slot sits in a cell without a task).  w: two
// device words, cleared here.
hipError_t launch_refresh(const PlanDev& p, const int64_t* off, int n_cells, int64_t n_slots,
                          int64_t* xi, double* v, unsigned long long* w, hipStream_t st);

}  // namespace sdm

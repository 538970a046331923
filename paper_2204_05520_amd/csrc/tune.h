// Tile autotuner: opts.tile_chunk == ODP_TILE_AUTOTUNE.
#pragma once

#include <vector>

#include "plan.h"

namespace odp {

// Device bytes a plan of these items needs for any chunk the tuner may pick.
size_t tune_workspace_bytes(const std::vector<PlanItem> &items, const odp_solve_opts &opts);

// The cached chunk for these items, if they have been tuned before.
bool tune_cached(const std::vector<PlanItem> &items, const odp_solve_opts &opts, int *chunk);

// The chunk (planes of axis 0 per block, to plan_build with round4) for
// these items: from the process-wide cache, else by timing the stage
// launches of step 0 for each candidate in the workspace `base` (at least
// tune_workspace_bytes).  Runs before the real plan's prologue: it leaves
// the workspace and the items' output arrays holding garbage, which the
// start copy and the steps overwrite.
int tune_tile_chunk(const std::vector<PlanItem> &items, const odp_solve_opts &opts, unsigned char *base,
                    hipStream_t st, int *chunk);

}  // namespace odp

// Stage launches of one (precision, dynamics) slice.  Each slice is compiled
// from stage_inst.hip as its own translation unit (ODP_PREC 32 or 64,
// ODP_DYN 0..4), so the template instantiations build in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "odp_dev.h"

namespace odp {

#define ODP_STAGE_SLICE_ARGS                                                                      \
    int ndim, int vec, int kind, const SolveDesc *d, const uint32_t *ts, const uint32_t *tl,     \
        uint32_t nblocks, int stage, int from_desc, int64_t step, int xgroup, hipStream_t st

hipError_t launch_stage_f32_d0(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f32_d1(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f32_d2(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f32_d3(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f32_d4(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f64_d0(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f64_d1(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f64_d2(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f64_d3(ODP_STAGE_SLICE_ARGS);
hipError_t launch_stage_f64_d4(ODP_STAGE_SLICE_ARGS);

}  // namespace odp

// One (precision, dynamics) slice of the stage kernels: compiled once per
// slice with ODP_PREC (32 or 64) and ODP_DYN (0..4) defined.
#include "kernels_dev.h"
#include "stage_inst.h"

#if !defined(ODP_PREC) || !defined(ODP_DYN)
#error "stage_inst.hip needs ODP_PREC and ODP_DYN"
#endif

#define ODP_SLICE_NAME2(p, d) launch_stage_f##p##_d##d
#define ODP_SLICE_NAME(p, d) ODP_SLICE_NAME2(p, d)

namespace odp {

hipError_t ODP_SLICE_NAME(ODP_PREC, ODP_DYN)(ODP_STAGE_SLICE_ARGS) {
    using T = std::conditional_t<ODP_PREC == 32, float, double>;
    constexpr int D = ODP_DYN;
    if constexpr (D == 1) {
        return launch_stage_v<T, 1, 3>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
    } else if constexpr (D == 2) {
        return launch_stage_v<T, 2, 4>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
    } else if constexpr (D == 3) {
        return launch_stage_v<T, 3, 6>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
    } else if constexpr (D == 4) {
        return launch_stage_v<T, 4, 3>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
    } else {
        switch (ndim) {
        case 1: return launch_stage_v<T, 0, 1>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
        case 2: return launch_stage_v<T, 0, 2>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
        case 3: return launch_stage_v<T, 0, 3>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
        case 4: return launch_stage_v<T, 0, 4>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
        case 5: return launch_stage_v<T, 0, 5>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
        case 6: return launch_stage_v<T, 0, 6>(vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
        }
        return hipErrorInvalidValue;
    }
}

}  // namespace odp

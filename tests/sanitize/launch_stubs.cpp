// Stand-ins for the device launchers, so that the host runtime links in a
// CPU-only sanitizer build; none of them is reached by the driver.
#include "runtime.h"

namespace odp {

hipError_t launch_stage(int, int, int, int, int, const SolveDesc *, const uint32_t *, const uint32_t *, uint32_t,
                        int, int, int64_t, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_alpha(int, int, const SolveDesc *, int, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_init(const SolveDesc *, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_sched(const SolveDesc *, int, int64_t *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_advance(const SolveDesc *, const int32_t *, const int32_t *, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_ttr(int, int, int, const SolveDesc *, uint32_t, int, int, const void *, void *, const void *,
                      unsigned long long *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_ttr_init(int, const void *, void *, int64_t, double, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_ttr_zero(unsigned long long *, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_box_dt(const SolveDesc *, const int32_t *, int, int, int, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_box_finish(int, const SolveDesc *, const uint32_t *, const uint32_t *, uint32_t, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_box_save(int, const SolveDesc *, int64_t, void *, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_box_slice(int, SolveDesc *, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_set_slice(int, SolveDesc *, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_finish_copy(int, const SolveDesc *, const uint32_t *, const uint32_t *, uint32_t, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_start_copy(int, const SolveDesc *, const uint32_t *, const uint32_t *, uint32_t, hipStream_t) {
    return hipErrorInvalidValue;
}

}  // namespace odp

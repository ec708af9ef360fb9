// ssa_wave.hip -- wavefront-per-walker direct-method SSA (placeholder until
// the wave kernel lands: reports that no network fits).
#include "we_common.h"

hipError_t launch_ssa_wave(const SimArgs &, int32_t *, uint32_t, hipStream_t) {
    return hipErrorNotSupported;
}
bool wave_kernel_fits(int32_t, int32_t) { return false; }

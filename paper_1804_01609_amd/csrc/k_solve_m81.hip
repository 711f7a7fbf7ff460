// Solver instantiation for systems of size M <= 81: 3 wave(s) per stencil,
// 2 lane-column(s), 41 register slots per lane.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<3, 2, 41>() == 81, "capacity");
hipError_t solve_m81(const SolveArgs &a, hipStream_t s) { return launch_solve_variant<3, 2, 41>(a, s); }
}  // namespace rbfsl

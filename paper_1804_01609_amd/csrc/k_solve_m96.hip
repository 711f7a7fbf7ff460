// Solver instantiation for systems of size M <= 96: 3 wave(s) per stencil,
// 2 lane-column(s), 49 register slots per lane.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<3, 2, 49>() == 96, "capacity");
hipError_t solve_m96(const SolveArgs &a, hipStream_t s) { return launch_solve_variant<3, 2, 49>(a, s); }
}  // namespace rbfsl

// Solver instantiation for systems of size M <= 47: 1 wave(s) per stencil,
// 1 lane-column(s), 48 register slots per lane.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<1, 1, 48>() == 47, "capacity");
hipError_t solve_m47(const SolveArgs &a, hipStream_t s) { return launch_solve_variant<1, 1, 48>(a, s); }
}  // namespace rbfsl

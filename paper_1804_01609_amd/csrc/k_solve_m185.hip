// Solver instantiation for systems of size M <= 185: 8 wave(s) per stencil,
// 2 lane-column(s), 93 register slots per lane.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<8, 2, 93>() == 185, "capacity");
hipError_t solve_m185(const SolveArgs &a, hipStream_t s) { return launch_solve_variant<8, 2, 93>(a, s); }
}  // namespace rbfsl

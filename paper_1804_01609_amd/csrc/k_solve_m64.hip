// Solver instantiation for systems of size M <= 64: 1 wave(s) per stencil,
// 1 lane-column(s), 65 register slots per lane.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<1, 1, 65>() == 64, "capacity");
hipError_t solve_m64(const SolveArgs &a, hipStream_t s) { return launch_solve_variant<1, 1, 65>(a, s); }
}  // namespace rbfsl

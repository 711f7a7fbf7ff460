// Solver instantiation for systems of size M <= 128: 4 wave(s) per stencil,
// 2 lane-column(s), 65 register slots per lane.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<4, 2, 65>() == 128, "capacity");
hipError_t solve_m128(const SolveArgs &a, hipStream_t s) { return launch_solve_variant<4, 2, 65>(a, s); }
}  // namespace rbfsl

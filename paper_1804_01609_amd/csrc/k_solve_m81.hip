// Solver instantiation for systems of size M <= 81: 3 wave(s) per stencil,
// 2 row slot(s) per lane, 3 blocks of 9 column slots per wave, 3 waves per SIMD.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<3, 2, 3, 9>() == 81, "capacity");
hipError_t solve_m81(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<3, 2, 3, 9, 3>(a, s);
}
hipError_t factor_m81(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<3, 2, 3, 9, 3>(a, s);
}
}  // namespace rbfsl

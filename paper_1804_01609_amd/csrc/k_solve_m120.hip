// Solver instantiation for systems of size M <= 120: 4 wave(s) per stencil,
// 2 row slot(s) per lane, 10 blocks of 3 column slots per wave, 3 waves per SIMD.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<4, 2, 10, 3>() == 120, "capacity");
hipError_t solve_m120(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<4, 2, 10, 3, 3>(a, s);
}
hipError_t factor_m120(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<4, 2, 10, 3, 3>(a, s);
}
}  // namespace rbfsl

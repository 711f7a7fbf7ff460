// Solver instantiation for systems of size M <= 128: 4 wave(s) per stencil,
// 2 row slot(s) per lane, 4 blocks of 8 column slots per wave, 3 waves per SIMD.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<4, 2, 4, 8>() == 128, "capacity");
hipError_t solve_m128(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<4, 2, 4, 8, 3>(a, s);
}
hipError_t factor_m128(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<4, 2, 4, 8, 3>(a, s);
}
}  // namespace rbfsl

// Solver instantiation for systems of size M <= 192: 8 wave(s) per stencil,
// 3 row slot(s) per lane, 3 blocks of 8 column slots per wave, 2 waves per SIMD;
// LDS base opaque to the compiler (no scratch spills).
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<8, 3, 3, 8>() == 192, "capacity");
hipError_t solve_m192(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<8, 3, 3, 8, 2, true>(a, s);
}
hipError_t factor_m192(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<8, 3, 3, 8, 2, true>(a, s);
}
}  // namespace rbfsl

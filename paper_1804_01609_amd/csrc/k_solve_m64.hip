// Solver instantiation for systems of size M <= 64: 1 wave(s) per stencil,
// 1 row slot(s) per lane, 8 blocks of 8 column slots per wave, 3 waves per SIMD.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<1, 1, 8, 8>() == 64, "capacity");
hipError_t solve_m64(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<1, 1, 8, 8, 3>(a, s);
}
hipError_t factor_m64(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<1, 1, 8, 8, 3>(a, s);
}
}  // namespace rbfsl

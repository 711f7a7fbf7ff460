// Solver instantiation for systems of size M <= 48: 1 wave(s) per stencil,
// 1 row slot(s) per lane, 6 blocks of 8 column slots per wave, 4 waves per SIMD.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<1, 1, 6, 8>() == 48, "capacity");
hipError_t solve_m48(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<1, 1, 6, 8, 4>(a, s);
}
hipError_t factor_m48(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<1, 1, 6, 8, 4>(a, s);
}
}  // namespace rbfsl

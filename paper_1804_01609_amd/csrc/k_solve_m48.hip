// Solver instantiations for systems of size M <= 48: 1 wave per stencil, 1 row
// slot per lane, 6 blocks of 8 column slots per wave, 4 waves per SIMD; and,
// for launches of few systems, 4 waves per stencil (2 blocks of 6 column slots
// per wave), which spreads each system's columns over four SIMDs.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<1, 1, 6, 8>() == 48, "capacity");
hipError_t solve_m48(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<1, 1, 6, 8, 4>(a, s);
}
static_assert(variant_mcap<4, 1, 2, 6>() == 48, "capacity");
hipError_t solve_m48_wide(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<4, 1, 2, 6, 4>(a, s);
}
hipError_t factor_m48(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<1, 1, 6, 8, 4>(a, s);
}
}  // namespace rbfsl

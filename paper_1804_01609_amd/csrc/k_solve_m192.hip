// Solver instantiation for systems of size M <= 192: 16 waves per stencil,
// 3 row slots per lane, 3 blocks of 4 column slots per wave (110 VGPRs, 4
// waves per SIMD: the pivot-row broadcasts by readlane cost each wave ~16
// cycles of latency, hidden only when several waves share a SIMD); LDS base
// opaque to the compiler (no scratch spills).  The factor-only kernel keeps 8
// waves per stencil.
#include "k_solve.h"

namespace rbfsl {
static_assert(variant_mcap<16, 3, 3, 4>() == 192, "capacity");
static_assert(variant_mcap<8, 3, 3, 8>() == 192, "capacity");
hipError_t solve_m192(const SolveArgs &a, hipStream_t s) {
    return launch_solve_variant<16, 3, 3, 4, 4, true>(a, s);
}
hipError_t factor_m192(const FactorArgs &a, hipStream_t s) {
    return launch_factor_variant<8, 3, 3, 8, 2, true>(a, s);
}
}  // namespace rbfsl

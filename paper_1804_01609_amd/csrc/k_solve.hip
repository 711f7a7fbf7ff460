// Dispatch of the stencil solver over its compiled capacities (the kernel
// itself is in k_solve.h; each capacity is compiled in its own unit).
#include "rbfsl_impl.h"

namespace rbfsl {

hipError_t solve_m48(const SolveArgs &a, hipStream_t s);
hipError_t solve_m48_wide(const SolveArgs &a, hipStream_t s);
hipError_t solve_m64(const SolveArgs &a, hipStream_t s);
hipError_t solve_m81(const SolveArgs &a, hipStream_t s);
hipError_t solve_m96(const SolveArgs &a, hipStream_t s);
hipError_t solve_m120(const SolveArgs &a, hipStream_t s);
hipError_t solve_m128(const SolveArgs &a, hipStream_t s);
hipError_t solve_m192(const SolveArgs &a, hipStream_t s);
hipError_t factor_m48(const FactorArgs &a, hipStream_t s);
hipError_t factor_m64(const FactorArgs &a, hipStream_t s);
hipError_t factor_m81(const FactorArgs &a, hipStream_t s);
hipError_t factor_m96(const FactorArgs &a, hipStream_t s);
hipError_t factor_m120(const FactorArgs &a, hipStream_t s);
hipError_t factor_m128(const FactorArgs &a, hipStream_t s);
hipError_t factor_m192(const FactorArgs &a, hipStream_t s);

struct Variant {
    int mcap;
    hipError_t (*fn)(const SolveArgs &, hipStream_t);
    hipError_t (*factor)(const FactorArgs &, hipStream_t);
};

static const Variant kVariants[] = {
    {48, solve_m48, factor_m48},
    {64, solve_m64, factor_m64},
    {81, solve_m81, factor_m81},
    {96, solve_m96, factor_m96},
    {120, solve_m120, factor_m120},
    {128, solve_m128, factor_m128},
    {192, solve_m192, factor_m192},
};

static const Variant *pick(int M) {
    for (const Variant &v : kVariants)
        if (M <= v.mcap) return &v;
    return nullptr;
}

int solve_variant_capacity(int M) {
    const Variant *v = pick(M);
    return v ? v->mcap : 0;
}

// a launch of at most this many systems of the smallest capacity uses four
// waves per system: with one wave per system, 1,024 systems occupy one wave
// slot of each SIMD and every system's elimination runs serially in its wave
constexpr int64_t SMALL_LAUNCH = 1024;

hipError_t launch_solve(const SolveArgs &a, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    const Variant *v = pick(a.n + (a.L + 1) * (a.L + 1));
    if (!v) return hipErrorInvalidValue;
    if (v->mcap == 48 && a.count <= SMALL_LAUNCH) return solve_m48_wide(a, s);
    return v->fn(a, s);
}

hipError_t launch_factor(const FactorArgs &a, hipStream_t s) {
    if (a.s.count <= 0) return hipSuccess;
    const Variant *v = pick(a.s.n + (a.s.L + 1) * (a.s.L + 1));
    if (!v) return hipErrorInvalidValue;
    return v->factor(a, s);
}

}  // namespace rbfsl

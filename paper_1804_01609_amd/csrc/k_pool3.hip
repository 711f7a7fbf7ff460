// Pooled step kernel, family 2: workgroups of 3 waves, one stencil each, for
// systems of up to 90 unknowns: with three waves per stencil four workgroups
// share a compute unit (twelve waves), one more stencil in flight per CU than
// with four waves per stencil.
#include "k_pool.h"

namespace rbfsl {

//                      W  R NCB B     capacity  W  G  B
#define POOL3_VARIANTS                                          \
    PV<3, 2, 3, 9>,    /* 81                    3  1  9 */      \
        PV<3, 2, 4, 7>, /* 84                   3  1  7 */      \
        PV<3, 2, 7, 4>, /* 84                   3  1  4 */      \
        PV<3, 2, 5, 6>  /* 90                   3  1  6 */
#define POOL3_KERNEL k_pool<3, 3, POOL3_VARIANTS>

static_assert(PV<3, 2, 3, 9>::MCAP == 81 && PV<3, 2, 4, 7>::MCAP == 84 && PV<3, 2, 7, 4>::MCAP == 84 &&
                  PV<3, 2, 5, 6>::MCAP == 90,
              "variant capacities");

extern const PoolVariantInfo kPool3Variants[];
extern const int kPool3NumVariants;
const PoolVariantInfo kPool3Variants[] = {
    {2, 0, 81, 3, 1, 9, "w3b9"}, {2, 1, 84, 3, 1, 7, "w3b7"}, {2, 2, 84, 3, 1, 4, "w3b4"}, {2, 3, 90, 3, 1, 6, "w3b6"},
};
const int kPool3NumVariants = sizeof(kPool3Variants) / sizeof(kPool3Variants[0]);

hipError_t pool3_launch(const PoolArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((POOL3_KERNEL), dim3((unsigned)blocks), dim3(192), 0, s, a);
    return hipGetLastError();
}

int pool3_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&POOL3_KERNEL), 192, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace rbfsl

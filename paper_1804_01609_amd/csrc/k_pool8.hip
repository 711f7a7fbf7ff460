// Pooled step kernel, family 1: workgroups of 8 waves, one stencil each, for
// systems of up to 192 unknowns (three row slots per lane).
#include "k_pool.h"

namespace rbfsl {

#define POOL8_KERNEL k_pool<8, 2, PV<8, 3, 3, 8>>

static_assert(PV<8, 3, 3, 8>::MCAP == 192, "variant capacity");

extern const PoolVariantInfo kPool8Variants[];
extern const int kPool8NumVariants;
const PoolVariantInfo kPool8Variants[] = {{1, 0, 192, 8, 1, 8, "w8b8"}};
const int kPool8NumVariants = 1;

hipError_t pool8_launch(const PoolArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((POOL8_KERNEL), dim3((unsigned)blocks), dim3(512), 0, s, a);
    return hipGetLastError();
}

int pool8_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&POOL8_KERNEL), 512, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace rbfsl

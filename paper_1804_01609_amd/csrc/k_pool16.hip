// Pooled step kernel, family 3: workgroups of 16 waves, one stencil each, for
// systems of up to 192 unknowns (three row slots per lane, blocks of four
// column slots per wave, four waves per SIMD): the single-run kernel's layout
// for M <= 192, where the pivot-row broadcasts by readlane need several waves
// per SIMD to hide their latency.  One system per compute unit.
#include "k_pool.h"

namespace rbfsl {

#define POOL16_KERNEL k_pool<16, 4, PV<16, 3, 3, 4>>

static_assert(PV<16, 3, 3, 4>::MCAP == 192, "variant capacity");

extern const PoolVariantInfo kPool16Variants[];
extern const int kPool16NumVariants;
const PoolVariantInfo kPool16Variants[] = {{3, 0, 192, 16, 1, 4, "w16b4"}};
const int kPool16NumVariants = 1;

hipError_t pool16_launch(const PoolArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((POOL16_KERNEL), dim3((unsigned)blocks), dim3(1024), 0, s, a);
    return hipGetLastError();
}

int pool16_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&POOL16_KERNEL), 1024, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace rbfsl

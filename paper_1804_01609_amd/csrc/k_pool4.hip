// Pooled step kernel, family 0: workgroups of 4 waves; systems of up to 128
// unknowns.  The variants differ in waves per stencil W (stencils per
// workgroup G = 4 / W) and in panel width B; the pool's tuner picks one per
// system size by timing them.
#include "k_pool.h"

namespace rbfsl {

//                       W  R NCB  B  (CM)   capacity  W  G  B
#define POOL4_VARIANTS                                                   \
    PV<1, 1, 6, 8, 8>,   /* 48                        1  4  8 */          \
        PV<2, 1, 3, 8>,  /* 48                        2  2  8 */          \
        PV<4, 1, 2, 6>,  /* 48                        4  1  6 */          \
        PV<4, 2, 3, 7>,  /* 84                        4  1  7 */          \
        PV<4, 2, 7, 3>,  /* 84                        4  1  3 */          \
        PV<4, 2, 5, 6>,  /* 120                       4  1  6 */          \
        PV<4, 2, 3, 10>, /* 120                       4  1 10 */          \
        PV<4, 2, 6, 5>   /* 120                       4  1  5 */
#define POOL4_KERNEL k_pool<4, 3, POOL4_VARIANTS>

static_assert(PV<1, 1, 6, 8, 8>::MCAP == 48 && PV<2, 1, 3, 8>::MCAP == 48 && PV<4, 1, 2, 6>::MCAP == 48 &&
                  PV<4, 2, 3, 7>::MCAP == 84 && PV<4, 2, 7, 3>::MCAP == 84 && PV<4, 2, 5, 6>::MCAP == 120 &&
                  PV<4, 2, 3, 10>::MCAP == 120 && PV<4, 2, 6, 5>::MCAP == 120,
              "variant capacities");

extern const PoolVariantInfo kPool4Variants[];
extern const int kPool4NumVariants;
const PoolVariantInfo kPool4Variants[] = {
    {0, 0, 48, 1, 4, 8, "w1b8"},  {0, 1, 48, 2, 2, 8, "w2b8"},   {0, 2, 48, 4, 1, 6, "w4b6"},
    {0, 3, 84, 4, 1, 7, "w4b7"},  {0, 4, 84, 4, 1, 3, "w4b3"},   {0, 5, 120, 4, 1, 6, "w4b6"},
    {0, 6, 120, 4, 1, 10, "w4b10"}, {0, 7, 120, 4, 1, 5, "w4b5"},
};
const int kPool4NumVariants = sizeof(kPool4Variants) / sizeof(kPool4Variants[0]);

hipError_t pool4_launch(const PoolArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((POOL4_KERNEL), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

int pool4_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&POOL4_KERNEL), 256, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace rbfsl

// Search pass of a pooled step: for every node of every run with steps left,
// the departure point (RK4, Section 3.2) and the exact n-nearest-node stencil
// of it (Sections 2.2 and 3.3.2), written to the run's xi / S / s2 buffers.
// One wave per node, grid-stride over the search queue (items = nodes); the
// search does not depend on q, so it runs ahead of the solves at the high
// occupancy a latency-bound search needs.
#include "k_knn.h"
#include "k_trace.h"
#include "pool_impl.h"

namespace rbfsl {

constexpr int POOL_KNN_CAP = 512;

__global__ void __launch_bounds__(64) k_pool_search(PoolArgs P) {
    __shared__ KnnSmem<POOL_KNN_CAP> sh;
    const int lane = threadIdx.x;
    const PoolQueue *Q = P.queue;
    const int64_t nitems = Q->nitems;
    const int nseg = Q->nseg;
    int lo = 0;
    int64_t s_lo = 0, s_hi = 0;  // item range of segment lo, searched only when an item leaves it
    for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        if (!(item >= s_lo && item < s_hi)) {
            int l = 0, hi = nseg - 1;  // last segment with item0 <= item
            while (l < hi) {
                const int mid = (l + hi + 1) >> 1;
                if (Q->seg[mid].item0 <= item) l = mid;
                else hi = mid - 1;
            }
            lo = l;
            s_lo = Q->seg[lo].item0;
            s_hi = (lo + 1 < nseg) ? Q->seg[lo + 1].item0 : nitems;
        }
        const int slot = __builtin_amdgcn_readfirstlane(Q->seg[lo].slot);
        const int64_t j = item - s_lo;
        const PoolRunDev &r = P.runs[slot];
        const int64_t step = P.state[slot].step;
        if (step >= r.nsteps || r.status[ST_FAILSTEP] <= step) continue;
        const int64_t N = r.N;
        const double x[3] = {r.nx[j], r.ny[j], r.nz[j]};
        double xi[3];
        trace_point(r.coef[step], x, xi);
        const GridView gv{r.G, r.invh, r.cell_start, r.sx, r.sy, r.sz, r.perm};
        if (!knn_wave<POOL_KNN_CAP>(sh, lane, gv, xi[0], xi[1], xi[2], r.n, r.R0)) {
            if (lane == 0) {
                atomicAdd(&r.status[ST_SEARCH], 1);
                atomicMin(&r.status[ST_FAILSTEP], (int)step);
            }
            continue;
        }
        int32_t *Sj = r.S + j * r.n;
        for (int a = lane; a < r.n; a += 64) Sj[a] = sh.ki[a];
        if (lane == 0) {
            r.xi[j] = xi[0];
            r.xi[N + j] = xi[1];
            r.xi[2 * N + j] = xi[2];
            r.s2[j] = sh.kd[r.n - 1];
        }
        wave_lds_sync();  // the stencil is read before the next search reuses the buffers
    }
}

hipError_t pool_launch_search(const PoolArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_pool_search, dim3((unsigned)blocks), dim3(64), 0, s, a);
    return hipGetLastError();
}

int pool_search_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_pool_search), 64, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace rbfsl

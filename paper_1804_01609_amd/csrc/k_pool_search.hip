// Trace and search passes of a pooled step: for every node of every run with
// steps left, the departure point (RK4, Section 3.2; one thread per node)
// and then the exact n-nearest-node stencil of it (Sections 2.2 and 3.3.2;
// one wave per node), written to the run's xi / S / s2 buffers, for every item
// of the search queue (items = nodes), launched outside the step's graph
// with one thread or one wave per node.  Neither depends on q, so they run
// ahead of the solves; as two plain kernels (no tracer inlined, no loop over
// nodes) the search keeps the registers of the search alone and the
// occupancy a latency-bound search needs.
#include "k_knn.h"
#include "k_trace.h"
#include "pool_impl.h"

namespace rbfsl {

// The candidate store of the single-run search for the same n: a quarter of
// the full store up to n = KNN_SMALL_N / 2, else half (the pool's systems hold
// n < MAX_SYSTEM <= KNN_SMALL_N), so that both paths sort the same number of
// keys and fail on the same node clusters.  One LDS area serves both sizes.
static_assert(MAX_SYSTEM <= KNN_SMALL_N, "pooled stencils fit the half-size store");
union PoolKnnSmem {
    KnnSmem<KNN_CAP / 4> q;
    KnnSmem<KNN_CAP / 2> h;
};

// the segment of queue item `item`: the last with item0 <= item
__device__ __forceinline__ int pool_segment(const PoolQueue *Q, int64_t item) {
    int l = 0, hi = Q->nseg - 1;
    while (l < hi) {
        const int mid = (l + hi + 1) >> 1;
        if (Q->seg[mid].item0 <= item) l = mid;
        else hi = mid - 1;
    }
    return l;
}

// one thread per queue item (node)
__global__ void __launch_bounds__(256) k_pool_trace(PoolArgs P) {
    const PoolQueue *Q = P.queue;
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= Q->nitems) return;
    const PoolSeg &sg = Q->seg[pool_segment(Q, item)];
    const int64_t j = item - sg.item0;
    const PoolRunDev &r = P.runs[sg.slot];
    const int64_t step = P.state[sg.slot].step;
    if (step >= r.nsteps || r.status[ST_FAILSTEP] <= step) return;
    const int64_t N = r.N;
    const double x[3] = {r.nx[j], r.ny[j], r.nz[j]};
    double xi[3];
    trace_point(r.coef[step], x, xi);
    r.xi[j] = xi[0];
    r.xi[N + j] = xi[1];
    r.xi[2 * N + j] = xi[2];
}

// one wave per queue item (node)
__global__ void __launch_bounds__(64) k_pool_search(PoolArgs P) {
    __shared__ PoolKnnSmem sh;
    const int lane = threadIdx.x;
    const PoolQueue *Q = P.queue;
    const int64_t item = blockIdx.x;
    if (item >= Q->nitems) return;
    const int lo = pool_segment(Q, item);
    const int slot = __builtin_amdgcn_readfirstlane(Q->seg[lo].slot);
    const int64_t j = item - Q->seg[lo].item0;
    const PoolRunDev &r = P.runs[slot];
    const int64_t step = P.state[slot].step;
    if (step >= r.nsteps || r.status[ST_FAILSTEP] <= step) return;
    const int64_t N = r.N;
    const double xi[3] = {r.xi[j], r.xi[N + j], r.xi[2 * N + j]};
    const GridView gv{r.G, r.invh, r.cell_start, r.sx, r.sy, r.sz, r.perm};
    const bool quarter = r.n <= KNN_SMALL_N / 2;
    const bool found = quarter ? knn_wave<KNN_CAP / 4>(sh.q, lane, gv, xi[0], xi[1], xi[2], r.n, r.R0)
                               : knn_wave<KNN_CAP / 2>(sh.h, lane, gv, xi[0], xi[1], xi[2], r.n, r.R0);
    if (!found) {
        if (lane == 0) {
            atomicAdd(&r.status[ST_SEARCH], 1);
            atomicMin(&r.status[ST_FAILSTEP], (int)step);
        }
        return;
    }
    const int *ki = quarter ? sh.q.ki : sh.h.ki;
    const double *kd = quarter ? sh.q.kd : sh.h.kd;
    int32_t *Sj = r.S + j * r.n;
    for (int a = lane; a < r.n; a += 64) Sj[a] = ki[a];
    if (lane == 0) r.s2[j] = kd[r.n - 1];
}

hipError_t pool_launch_search(const PoolArgs &a, int64_t items, hipStream_t s) {
    if (items <= 0) return hipSuccess;
    if (items > 0x7fffffffLL) return hipErrorInvalidConfiguration;  // one workgroup per node
    hipLaunchKernelGGL(k_pool_trace, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pool_search, dim3((unsigned)items), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace rbfsl

// Batched transport: many independent runs advanced together, one persistent
// launch per step and kernel family.  Declarations shared by the kernels and
// the host side (pool_api.hip).
//
// Every device-side table lives at a fixed address for the life of the pool,
// so one captured HIP graph (reset -> step kernels -> commit) serves every
// step: what changes between steps (which runs take part, their step
// counters) is data in those tables, not kernel arguments.
#pragma once

#include "rbfsl_impl.h"

namespace rbfsl {

// One run slot as the kernels read it.
struct PoolRunDev {
    const double *nx, *ny, *nz;  // nodes, original order
    int G;                       // spatial hash of the nodes
    double invh;
    double R0;                   // first search radius
    const int *cell_start;
    const double *sx, *sy, *sz;
    const int *perm;
    double *q[2];                // q^m / q^{m+1}, n_tracers x N each
    const StepCoef *coef;        // tracer coefficients of steps 0 .. nsteps-1
    double *xi;                  // this step's departure points, x[N] y[N] z[N]
    int32_t *S;                  // ... their stencils, N x n
    double *s2;                  // ... squared distance of the n-th stencil node
    int *status;                 // ST_WORDS failure words of the run
    int64_t N;
    int64_t nsteps;              // 0: slot unused
    int n, L, k, ntr;
};

// Mutable step state of a slot (written only by the commit kernel and the host
// while no step is in flight).
struct PoolState {
    int64_t step;  // steps committed: q^step is in q[cur]
    int cur;
    int pad;
};

// A run's share of one kernel family's work queue: ceil(N / G) items of G
// consecutive nodes, items item0 .. item0 + nitems - 1 of the queue.
struct PoolSeg {
    int slot;
    int var;   // solver variant inside the family's kernel
    int G;     // stencil groups per workgroup for that variant
    int pad;
    int64_t N;
    int64_t item0;
};

constexpr int POOL_MAX_SEG = 4096;

// Work queue of one kernel family.
struct PoolQueue {
    int64_t nitems;
    int nseg;
    int pad;
    unsigned long long next;  // claim counter, cleared before every step
    PoolSeg seg[POOL_MAX_SEG];
};

struct PoolArgs {
    const PoolRunDev *runs;
    const PoolState *state;
    PoolQueue *queue;
};

// The tracer and stencil search of a step, for every node of every run
// (queue items = nodes; `items` is the search queue's item count): the
// departure points, one thread per node, then the stencils, one wave per node.
hipError_t pool_launch_search(const PoolArgs &a, int64_t items, hipStream_t s);

// Kernel families, by waves per workgroup: 4 (systems up to 128 unknowns,
// one, two or four waves per stencil), 8 (up to 192 unknowns), 3 (up to 90
// unknowns, three waves per stencil) and 16 (up to 192 unknowns).
constexpr int POOL_FAMILIES = 4;
struct PoolVariantInfo {
    int family;
    int var;     // index inside the family's kernel
    int mcap;    // largest system
    int W;       // waves per stencil
    int G;       // stencils per workgroup
    int B;       // panel width
    const char *name;
};
int pool_variants(const PoolVariantInfo **out);  // table of every compiled variant

// launchers
hipError_t pool_launch_family(int family, const PoolArgs &a, int blocks, hipStream_t s);
int pool_family_blocks_per_cu(int family);       // occupancy of the family's kernel (0: error)

}  // namespace rbfsl

// Host side of the pooled transport API (rbfsl_pool_* in rbfsl.h): many
// independent runs advanced together, one persistent launch per kernel family
// and step, optionally replayed from one captured HIP graph.
//
// Memory: the pool reserves its HBM budget once, as an arena, and carves each
// run's state out of it (nodes, hash grid, q ping-pong, per-step tracer
// coefficients, scratch of the grid build), so admitting and retiring runs
// never calls the HIP allocator and never blocks the device.
//
// Streams (all at the default priority): `main` carries the steps, `side[]`
// the other kernel families inside the captured step (so that one family's
// workgroups fill the compute units another's tail leaves idle), `admit` the
// uploads and grid builds of new runs, which the next step waits for through
// an event.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "pool_impl.h"

namespace rbfsl {

extern const PoolVariantInfo kPool4Variants[];
extern const int kPool4NumVariants;
extern const PoolVariantInfo kPool8Variants[];
extern const int kPool8NumVariants;
extern const PoolVariantInfo kPool3Variants[];
extern const int kPool3NumVariants;
extern const PoolVariantInfo kPool16Variants[];
extern const int kPool16NumVariants;
hipError_t pool4_launch(const PoolArgs &a, int blocks, hipStream_t s);
hipError_t pool8_launch(const PoolArgs &a, int blocks, hipStream_t s);
hipError_t pool3_launch(const PoolArgs &a, int blocks, hipStream_t s);
hipError_t pool16_launch(const PoolArgs &a, int blocks, hipStream_t s);
int pool4_blocks_per_cu();
int pool8_blocks_per_cu();
int pool3_blocks_per_cu();
int pool16_blocks_per_cu();

struct QueueSet {
    PoolQueue *q[POOL_FAMILIES];
};

__global__ void k_pool_reset(QueueSet qs) {
    if (threadIdx.x < POOL_FAMILIES) qs.q[threadIdx.x]->next = 0;
}

// advance every slot whose step went through: not finished, no failure at or
// before the step
// The step tables (every queue's used part and the commit's slot list) from
// pinned staging to the device in one launch on the main stream: per-table
// copy-engine transfers cost tens of microseconds of hand-over each, at every
// step whose set of stepping runs changed.
constexpr int STAGE_TABLES = POOL_FAMILIES + 2;
struct StageList {
    const uint64_t *src[STAGE_TABLES];
    uint64_t *dst[STAGE_TABLES];
    int64_t nwords[STAGE_TABLES];
};
__global__ void k_stage_tables(StageList L) {
    const int e = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.nwords[e];
         i += (int64_t)gridDim.x * blockDim.x)
        L.dst[e][i] = L.src[e][i];
}

// on[s]: slot s took part in the step (its nodes were in the queues)
__global__ void k_pool_commit(const PoolRunDev *runs, PoolState *state, const int *on, int nslots) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    const PoolRunDev &r = runs[s];
    PoolState &st = state[s];
    if (on[s] && r.nsteps > 0 && st.step < r.nsteps && r.status[ST_FAILSTEP] > st.step) {
        st.step += 1;
        st.cur ^= 1;
    }
}

hipError_t pool_launch_family(int family, const PoolArgs &a, int blocks, hipStream_t s) {
    switch (family) {
        case 0: return pool4_launch(a, blocks, s);
        case 1: return pool8_launch(a, blocks, s);
        case 2: return pool3_launch(a, blocks, s);
        default: return pool16_launch(a, blocks, s);
    }
}

int pool_family_blocks_per_cu(int family) {
    switch (family) {
        case 0: return pool4_blocks_per_cu();
        case 1: return pool8_blocks_per_cu();
        case 2: return pool3_blocks_per_cu();
        default: return pool16_blocks_per_cu();
    }
}

int pool_variants(const PoolVariantInfo **out) {
    static std::vector<PoolVariantInfo> all;
    if (all.empty()) {
        // the 16-wave variant before the 8-wave one: the default for systems
        // of 129..192 unknowns (M = 184: 840 against 881 ns per node)
        for (int i = 0; i < kPool4NumVariants; ++i) all.push_back(kPool4Variants[i]);
        for (int i = 0; i < kPool16NumVariants; ++i) all.push_back(kPool16Variants[i]);
        for (int i = 0; i < kPool8NumVariants; ++i) all.push_back(kPool8Variants[i]);
        for (int i = 0; i < kPool3NumVariants; ++i) all.push_back(kPool3Variants[i]);
    }
    *out = all.data();
    return (int)all.size();
}

}  // namespace rbfsl

using namespace rbfsl;

namespace {

constexpr size_t ALIGN = 256;
size_t al(size_t b) { return (b + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit allocator over one device reservation.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> busy_;
    void *alloc(size_t bytes) {
        bytes = al(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            busy_[off] = bytes;
            used += bytes;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p) {
        if (!p) return;
        const size_t off = (size_t)((char *)p - base);
        auto b = busy_.find(off);
        if (b == busy_.end()) return;
        size_t o = off, len = b->second;
        busy_.erase(b);
        used -= len;
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && o + len == nx->first) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == o) {
                o = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[o] = len;
    }
};

// Device bytes of one run, carved as one block (see RunLayout).
struct RunLayout {
    size_t nodes, sorted, cstart, perm, q, coef, xi, S, s2, cell, count, aos, total;
    int G;
    double invh, R0;
};

RunLayout run_layout(int64_t N, int n, int ntr, int64_t nsteps) {
    RunLayout L{};
    grid_dims(N, n, &L.G, &L.invh, &L.R0);
    const size_t ncell = (size_t)L.G * L.G * L.G;
    size_t o = 0;
    L.nodes = o;  o += al(3 * sizeof(double) * N);
    L.sorted = o; o += al(3 * sizeof(double) * N);
    L.cstart = o; o += al(sizeof(int) * (ncell + 1));
    L.perm = o;   o += al(sizeof(int) * N);
    L.q = o;      o += 2 * al(sizeof(double) * N * ntr);
    L.coef = o;   o += al(sizeof(StepCoef) * (size_t)nsteps);
    L.xi = o;     o += al(3 * sizeof(double) * N);
    L.S = o;      o += al(sizeof(int32_t) * N * n);
    L.s2 = o;     o += al(sizeof(double) * N);
    L.cell = o;   o += al(sizeof(int) * N);
    L.count = o;  o += al(sizeof(int) * ncell);
    L.aos = o;    o += al(3 * sizeof(double) * N);
    L.total = o;
    return L;
}

struct Run {
    bool used = false;
    int64_t id = -1;
    int64_t N = 0, nsteps = 0;
    int64_t h_step = 0;   // steps enqueued (= committed unless the run failed)
    bool failed = false;
    int fail_code = 0;
    int n = 0, L = 0, k = 0, M = 0, ntr = 1;
    int family = 0, var = 0, G = 1;
    rbfsl_params p{};
    char *block = nullptr;
    size_t bytes = 0;
    RunLayout lay{};
    bool hold = false;  // left out of the next steps (the served form's scheduler)
    bool in_table() const { return used && !failed && h_step < nsteps; }
    bool stepping() const { return in_table() && !hold; }
};

}  // namespace

struct rbfsl_pool {
    int device = 0, ncu = 0;
    hipStream_t main = nullptr, admit = nullptr;
    hipStream_t side[POOL_FAMILIES - 1] = {};
    hipEvent_t admitted = nullptr, fork = nullptr;
    hipEvent_t join[POOL_FAMILIES - 1] = {};
    bool admit_pending = false;
    int max_runs = 0;
    bool use_graph = true;
    bool log_requests = false;
    Arena arena;
    std::vector<Run> runs;
    int64_t next_id = 0;
    std::map<int64_t, int> slot_of;  // run id -> slot
    PoolRunDev *d_runs = nullptr, *h_runs = nullptr;   // h_*: pinned mirrors
    PoolState *d_state = nullptr, *h_state = nullptr;
    int *d_on = nullptr, *h_on[2] = {};                // slots taking part in the step (ring as the queues)
    int *d_status = nullptr, *h_status = nullptr;      // max_runs x ST_WORDS
    // queues: one per kernel family, and the search pass's (index SEARCH)
    PoolQueue *d_queue[POOL_FAMILIES + 1] = {};
    PoolQueue *h_queue[POOL_FAMILIES + 1][2] = {};     // pinned staging, and its device address
    const PoolQueue *m_queue[POOL_FAMILIES + 1][2] = {};
    const int *m_on[2] = {};
    hipEvent_t tev[2] = {};                            // the staging of ring slot r has been read
    int64_t search_items = 0;  // nodes in the search queue
    int qring = 0;
    bool dirty = true;
    int blocks[POOL_FAMILIES] = {};
    std::map<int, int> tuned;  // system size M -> global variant index
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t steps_launched = 0;
    int64_t items_last[POOL_FAMILIES] = {};
    std::string err;
};

namespace {

int pfail(rbfsl_pool *pl, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int pfail(rbfsl_pool *pl, int code, const char *fmt, ...) {
    if (pl) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        pl->err = buf;
    }
    return code;
}

#define PHIP(pl, call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return pfail((pl), e_ == hipErrorOutOfMemory ? RBFSL_E_NOMEM : RBFSL_E_DEVICE,    \
                         "%s: %s", #call, hipGetErrorString(e_));                             \
    } while (0)

int code_of(const int *st) {
    if (st[ST_SEARCH]) return RBFSL_E_SEARCH;
    if (st[ST_SINGULAR]) return RBFSL_E_SINGULAR;
    if (st[ST_NONFINITE]) return RBFSL_E_NONFINITE;
    return RBFSL_OK;
}

// default variant for a system of M unknowns: the smallest capacity, first
// listed (or the tuned choice)
int pick_variant(const rbfsl_pool *pl, int M) {
    auto t = pl->tuned.find(M);
    if (t != pl->tuned.end()) return t->second;
    const PoolVariantInfo *v;
    const int nv = pool_variants(&v);
    int best = -1;
    for (int i = 0; i < nv; ++i)
        if (v[i].mcap >= M && (best < 0 || v[i].mcap < v[best].mcap)) best = i;
    return best;
}

void set_variant(Run &r, int gi) {
    const PoolVariantInfo *v;
    pool_variants(&v);
    r.family = v[gi].family;
    r.var = v[gi].var;
    r.G = v[gi].G;
}

// the queues of the runs stepping (costliest systems first) and the commit's
// slot list, to the device on the main stream through a ring of two pinned
// staging areas
int upload_tables(rbfsl_pool *pl) {
    const int ring = pl->qring;
    pl->qring ^= 1;
    std::vector<int> order;
    for (int s = 0; s < pl->max_runs; ++s)
        if (pl->runs[s].stepping()) order.push_back(s);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pl->runs[a].M > pl->runs[b].M; });
    PHIP(pl, hipEventSynchronize(pl->tev[ring]));  // the staging area is free again
    StageList L{};
    for (int f = 0; f <= POOL_FAMILIES; ++f) {
        const bool search = (f == POOL_FAMILIES);  // every run, one item per node
        PoolQueue *h = pl->h_queue[f][ring];
        int64_t item = 0;
        int ns = 0;
        for (int s : order) {
            const Run &r = pl->runs[s];
            if (!search && r.family != f) continue;
            if (ns >= POOL_MAX_SEG) return pfail(pl, RBFSL_E_STATE, "too many runs in one queue");
            const int G = search ? 1 : r.G;
            PoolSeg &sg = h->seg[ns++];
            sg.slot = s;
            sg.var = search ? 0 : r.var;
            sg.G = G;
            sg.pad = 0;
            sg.N = r.N;
            sg.item0 = item;
            item += (r.N + G - 1) / G;
        }
        h->nitems = item;
        h->nseg = ns;
        h->pad = 0;
        h->next = 0;
        if (!search) pl->items_last[f] = item;
        else pl->search_items = item;
        static_assert(offsetof(PoolQueue, seg) % 8 == 0 && sizeof(PoolSeg) % 8 == 0, "staged as 64-bit words");
        L.src[f] = reinterpret_cast<const uint64_t *>(pl->m_queue[f][ring]);
        L.dst[f] = reinterpret_cast<uint64_t *>(pl->d_queue[f]);
        L.nwords[f] = (int64_t)((offsetof(PoolQueue, seg) + sizeof(PoolSeg) * (size_t)ns) / 8);
    }
    int *on = pl->h_on[ring];
    for (int s = 0; s < pl->max_runs; ++s) on[s] = pl->runs[s].stepping() ? 1 : 0;
    L.src[POOL_FAMILIES + 1] = reinterpret_cast<const uint64_t *>(pl->m_on[ring]);
    L.dst[POOL_FAMILIES + 1] = reinterpret_cast<uint64_t *>(pl->d_on);
    L.nwords[POOL_FAMILIES + 1] = (pl->max_runs + 1) / 2;  // the lists hold an even count of ints
    hipLaunchKernelGGL(k_stage_tables, dim3(8, STAGE_TABLES), dim3(256), 0, pl->main, L);
    PHIP(pl, hipGetLastError());
    PHIP(pl, hipEventRecord(pl->tev[ring], pl->main));
    pl->dirty = false;
    return RBFSL_OK;
}

PoolArgs family_args(rbfsl_pool *pl, int f) {
    PoolArgs a;
    a.runs = pl->d_runs;
    a.state = pl->d_state;
    a.queue = pl->d_queue[f];
    return a;
}

// the trace and search passes of a step, sized by the current search queue
// (outside the captured graph, whose launch sizes are fixed)
hipError_t enqueue_search(rbfsl_pool *pl) {
    return pool_launch_search(family_args(pl, POOL_FAMILIES), pl->search_items, pl->main);
}

// the rest of a step: reset the claim counters, the solve families (all but
// the first on side streams, joined back), commit
hipError_t enqueue_step_kernels(rbfsl_pool *pl, bool commit) {
    QueueSet qs;
    for (int f = 0; f < POOL_FAMILIES; ++f) qs.q[f] = pl->d_queue[f];
    hipLaunchKernelGGL(k_pool_reset, dim3(1), dim3(64), 0, pl->main, qs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(pl->fork, pl->main)) != hipSuccess) return e;
    for (int f = 1; f < POOL_FAMILIES; ++f)
        if ((e = hipStreamWaitEvent(pl->side[f - 1], pl->fork, 0)) != hipSuccess) return e;
    if ((e = pool_launch_family(0, family_args(pl, 0), pl->blocks[0], pl->main)) != hipSuccess) return e;
    for (int f = 1; f < POOL_FAMILIES; ++f) {
        if ((e = pool_launch_family(f, family_args(pl, f), pl->blocks[f], pl->side[f - 1])) != hipSuccess) return e;
        if ((e = hipEventRecord(pl->join[f - 1], pl->side[f - 1])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(pl->main, pl->join[f - 1], 0)) != hipSuccess) return e;
    }
    if (commit) {
        const int nb = (pl->max_runs + 255) / 256;
        hipLaunchKernelGGL(k_pool_commit, dim3(nb), dim3(256), 0, pl->main, pl->d_runs, pl->d_state, pl->d_on,
                           pl->max_runs);
        e = hipGetLastError();
    }
    return e;
}

int launch_one_step(rbfsl_pool *pl) {
    if (pl->admit_pending) {
        PHIP(pl, hipStreamWaitEvent(pl->main, pl->admitted, 0));
        pl->admit_pending = false;
    }
    if (pl->dirty) {
        int r = upload_tables(pl);
        if (r != RBFSL_OK) return r;
    }
    PHIP(pl, enqueue_search(pl));
    if (pl->use_graph) {
        if (!pl->exec) {
            PHIP(pl, hipStreamBeginCapture(pl->main, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_step_kernels(pl, true);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(pl->main, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return pfail(pl, RBFSL_E_DEVICE, "step capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
            }
            pl->graph = g;
            PHIP(pl, hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0));
        }
        PHIP(pl, hipGraphLaunch(pl->exec, pl->main));
    } else {
        PHIP(pl, enqueue_step_kernels(pl, true));
    }
    pl->steps_launched += 1;
    for (Run &r : pl->runs)
        if (r.stepping()) {
            r.h_step += 1;
            if (r.h_step == r.nsteps) pl->dirty = true;
        }
    return RBFSL_OK;
}

// device truth after a synchronisation: step counters and failures
int reconcile(rbfsl_pool *pl) {
    PHIP(pl, hipStreamSynchronize(pl->main));
    PHIP(pl, hipStreamSynchronize(pl->admit));
    PHIP(pl, hipMemcpy(pl->h_state, pl->d_state, sizeof(PoolState) * pl->max_runs, hipMemcpyDeviceToHost));
    PHIP(pl, hipMemcpy(pl->h_status, pl->d_status, sizeof(int) * ST_WORDS * pl->max_runs, hipMemcpyDeviceToHost));
    for (int s = 0; s < pl->max_runs; ++s) {
        Run &r = pl->runs[s];
        if (!r.used) continue;
        const int *st = pl->h_status + ST_WORDS * s;
        if (st[ST_FAILSTEP] != NO_FAIL && !r.failed) {
            r.failed = true;
            r.fail_code = code_of(st);
            pl->dirty = true;
        }
        r.h_step = pl->h_state[s].step;
    }
    return RBFSL_OK;
}

int active_runs(const rbfsl_pool *pl) {
    int a = 0;
    for (const Run &r : pl->runs) a += r.in_table() ? 1 : 0;
    return a;
}

void pool_free(rbfsl_pool *pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    for (int f = 0; f <= POOL_FAMILIES; ++f) {
        if (pl->d_queue[f]) (void)hipFree(pl->d_queue[f]);
        for (int r = 0; r < 2; ++r)
            if (pl->h_queue[f][r]) (void)hipHostFree(pl->h_queue[f][r]);
    }
    void *dev[] = {pl->d_runs, pl->d_state, pl->d_status, pl->d_on, pl->arena.base};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    void *host[] = {pl->h_runs, pl->h_state, pl->h_status, pl->h_on[0], pl->h_on[1]};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    hipEvent_t evs[] = {pl->admitted, pl->fork, pl->tev[0], pl->tev[1]};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->join)
        if (e) (void)hipEventDestroy(e);
    hipStream_t ss[] = {pl->main, pl->admit};
    for (hipStream_t s : ss)
        if (s) (void)hipStreamDestroy(s);
    for (hipStream_t s : pl->side)
        if (s) (void)hipStreamDestroy(s);
}

// descriptor of slot s (pinned mirror) to the device, on the main stream
int upload_slot(rbfsl_pool *pl, int s) {
    PHIP(pl, hipMemcpyAsync(pl->d_runs + s, pl->h_runs + s, sizeof(PoolRunDev), hipMemcpyHostToDevice, pl->main));
    PHIP(pl, hipMemcpyAsync(pl->d_state + s, pl->h_state + s, sizeof(PoolState), hipMemcpyHostToDevice, pl->main));
    return RBFSL_OK;
}

__global__ void k_status_init(int *st) {
    if (threadIdx.x < ST_WORDS) st[threadIdx.x] = (threadIdx.x == ST_FAILSTEP) ? NO_FAIL : 0;
}

int pool_add_impl(rbfsl_pool *pl, const double *nodes_xyz, int64_t N, int nodes_on_device,
                  const rbfsl_params *p, const double *q0, int q_on_device, int64_t nsteps, int64_t *run_id) {
    if (!pl || !nodes_xyz || !p || !q0 || !run_id || nsteps < 1) return pfail(pl, RBFSL_E_INVAL, "invalid argument");
    int L, k;
    char msg[256];
    if (validate_params(N, p, &L, &k, msg, sizeof msg) != RBFSL_OK) return pfail(pl, RBFSL_E_INVAL, "%s", msg);
    if (p->stencil_mode != 0) return pfail(pl, RBFSL_E_INVAL, "pooled runs search the stencil of every departure point (stencil_mode 0)");
    const int M = p->n + (L + 1) * (L + 1);
    const int gi = pick_variant(pl, M);
    if (gi < 0) return pfail(pl, RBFSL_E_INVAL, "system size %d exceeds every pooled solver variant", M);
    int s = -1;
    for (int i = 0; i < pl->max_runs; ++i)
        if (!pl->runs[i].used) {
            s = i;
            break;
        }
    if (s < 0) return pfail(pl, RBFSL_E_BUDGET, "all %d run slots are busy", pl->max_runs);
    const RunLayout lay = run_layout(N, p->n, p->n_tracers, nsteps);
    char *blk = (char *)pl->arena.alloc(lay.total);
    if (!blk)
        return pfail(pl, RBFSL_E_BUDGET, "run needs %zu bytes, %zu of %zu in use", lay.total, pl->arena.used,
                     pl->arena.size);
    Run &r = pl->runs[s];
    r = Run();
    r.used = true;
    r.hold = false;
    r.id = pl->next_id++;
    r.N = N;
    r.nsteps = nsteps;
    r.n = p->n; r.L = L; r.k = k; r.M = M; r.ntr = p->n_tracers;
    r.p = *p;
    r.p.L = L;
    r.p.k = k;
    r.block = blk;
    r.bytes = lay.total;
    r.lay = lay;
    set_variant(r, gi);

    double *nodes = (double *)(blk + lay.nodes);
    double *sorted = (double *)(blk + lay.sorted);
    Grid g;
    g.G = lay.G;
    g.invh = lay.invh;
    g.R0 = lay.R0;
    g.cell_start = (int *)(blk + lay.cstart);
    g.sx = sorted;
    g.sy = sorted + N;
    g.sz = sorted + 2 * N;
    g.perm = (int *)(blk + lay.perm);
    double *q0d = (double *)(blk + lay.q);
    double *q1d = (double *)(blk + lay.q + al(sizeof(double) * N * r.ntr));
    StepCoef *coef = (StepCoef *)(blk + lay.coef);
    std::vector<StepCoef> hc((size_t)nsteps);
    for (int64_t m = 0; m < nsteps; ++m) hc[(size_t)m] = step_coef(r.p, m);

    hipStream_t a = pl->admit;
    hipError_t e = upload_points_via(nodes_xyz, N, nodes_on_device, nodes, nodes + N, nodes + 2 * N,
                                     (double *)(blk + lay.aos), a);
    if (e == hipSuccess) e = grid_build_in(nodes, nodes + N, nodes + 2 * N, N, &g, (int *)(blk + lay.cell),
                                           (int *)(blk + lay.count), a);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q0d, q0, sizeof(double) * N * r.ntr,
                           q_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, a);
    if (e == hipSuccess)
        e = hipMemcpyAsync(coef, hc.data(), sizeof(StepCoef) * (size_t)nsteps, hipMemcpyHostToDevice, a);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, a, pl->d_status + ST_WORDS * s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(pl->admitted, a);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(a);
        pl->arena.release(blk);
        r = Run();
        return pfail(pl, RBFSL_E_DEVICE, "run upload: %s", hipGetErrorString(e));
    }
    // the coefficient copy reads hc: it must have left host memory
    (void)hipStreamSynchronize(a);
    pl->admit_pending = true;
    PoolRunDev &d = pl->h_runs[s];
    d.nx = nodes; d.ny = nodes + N; d.nz = nodes + 2 * N;
    d.G = g.G; d.invh = g.invh; d.R0 = g.R0;
    d.cell_start = g.cell_start;
    d.sx = g.sx; d.sy = g.sy; d.sz = g.sz;
    d.perm = g.perm;
    d.q[0] = q0d; d.q[1] = q1d;
    d.coef = coef;
    d.xi = (double *)(blk + lay.xi);
    d.S = (int32_t *)(blk + lay.S);
    d.s2 = (double *)(blk + lay.s2);
    d.status = pl->d_status + ST_WORDS * s;
    d.N = N;
    d.nsteps = nsteps;
    d.n = r.n; d.L = L; d.k = k; d.ntr = r.ntr;
    pl->h_state[s].step = 0;
    pl->h_state[s].cur = 0;
    pl->h_state[s].pad = 0;
    // the main stream must see the grid before the descriptor goes live
    PHIP(pl, hipStreamWaitEvent(pl->main, pl->admitted, 0));
    pl->admit_pending = false;
    int rc = upload_slot(pl, s);
    if (rc != RBFSL_OK) return rc;
    pl->slot_of[r.id] = s;
    pl->dirty = true;
    *run_id = r.id;
    return RBFSL_OK;
}

int slot_for(rbfsl_pool *pl, int64_t id) {
    auto it = pl->slot_of.find(id);
    return it == pl->slot_of.end() ? -1 : it->second;
}

int release_run(rbfsl_pool *pl, int s) {
    Run &r = pl->runs[s];
    pl->arena.release(r.block);
    pl->slot_of.erase(r.id);
    r = Run();
    memset(&pl->h_runs[s], 0, sizeof(PoolRunDev));
    pl->h_state[s].step = 0;
    pl->h_state[s].cur = 0;
    int rc = upload_slot(pl, s);
    pl->dirty = true;
    return rc;
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

int rbfsl_pool_create(const rbfsl_pool_config *cfg, rbfsl_pool **out) {
    if (!out) return RBFSL_E_INVAL;
    *out = nullptr;
    if (!cfg || cfg->max_runs < 1 || cfg->max_runs > POOL_MAX_SEG || cfg->hbm_budget < 0) return RBFSL_E_INVAL;
    rbfsl_pool *pl = new (std::nothrow) rbfsl_pool();
    if (!pl) return RBFSL_E_NOMEM;
    pl->max_runs = cfg->max_runs;
    pl->use_graph = cfg->use_graph != 0;
    pl->log_requests = cfg->log_requests != 0;
    pl->runs.assign((size_t)pl->max_runs, Run());
    hipError_t e = hipGetDevice(&pl->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&pl->ncu, hipDeviceAttributeMultiprocessorCount, pl->device);
    size_t budget = (size_t)cfg->hbm_budget;
    if (e == hipSuccess && budget == 0) {
        size_t fr = 0, tot = 0;
        e = hipMemGetInfo(&fr, &tot);
        budget = fr / 2;
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->main, hipStreamNonBlocking);
    for (int f = 0; f + 1 < POOL_FAMILIES && e == hipSuccess; ++f) {
        e = hipStreamCreateWithFlags(&pl->side[f], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join[f], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->admit, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->admitted, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&pl->d_runs, sizeof(PoolRunDev) * pl->max_runs);
    if (e == hipSuccess) e = hipMalloc(&pl->d_state, sizeof(PoolState) * pl->max_runs);
    if (e == hipSuccess) e = hipMalloc(&pl->d_status, sizeof(int) * ST_WORDS * pl->max_runs);
    if (e == hipSuccess) e = hipHostMalloc(&pl->h_runs, sizeof(PoolRunDev) * pl->max_runs, 0);
    if (e == hipSuccess) e = hipHostMalloc(&pl->h_state, sizeof(PoolState) * pl->max_runs, 0);
    const size_t on_bytes = sizeof(int) * (size_t)((pl->max_runs + 1) & ~1);
    if (e == hipSuccess) e = hipMalloc(&pl->d_on, on_bytes);
    for (int r = 0; r < 2 && e == hipSuccess; ++r) {
        e = hipHostMalloc(&pl->h_on[r], on_bytes, hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&pl->m_on[r], pl->h_on[r], 0);
        if (e == hipSuccess) memset(pl->h_on[r], 0, on_bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->tev[r], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipHostMalloc(&pl->h_status, sizeof(int) * ST_WORDS * pl->max_runs, 0);
    for (int f = 0; f <= POOL_FAMILIES && e == hipSuccess; ++f) {
        e = hipMalloc(&pl->d_queue[f], sizeof(PoolQueue));
        for (int r = 0; r < 2 && e == hipSuccess; ++r) {
            e = hipHostMalloc(&pl->h_queue[f][r], sizeof(PoolQueue), hipHostMallocMapped);
            if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&pl->m_queue[f][r], pl->h_queue[f][r], 0);
        }
    }
    if (e == hipSuccess) e = hipMalloc(&pl->arena.base, budget);
    if (e == hipSuccess) {
        pl->arena.size = budget;
        pl->arena.free_[0] = budget;
        memset(pl->h_runs, 0, sizeof(PoolRunDev) * pl->max_runs);
        memset(pl->h_state, 0, sizeof(PoolState) * pl->max_runs);
        e = hipMemcpy(pl->d_runs, pl->h_runs, sizeof(PoolRunDev) * pl->max_runs, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl->d_state, pl->h_state, sizeof(PoolState) * pl->max_runs, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(pl->d_status, 0, sizeof(int) * ST_WORDS * pl->max_runs);
        if (e == hipSuccess) e = hipMemset(pl->d_on, 0, on_bytes);
        for (int f = 0; f <= POOL_FAMILIES && e == hipSuccess; ++f) e = hipMemset(pl->d_queue[f], 0, sizeof(PoolQueue));
    }
    for (int f = 0; f < POOL_FAMILIES && e == hipSuccess; ++f) {
        const int bpc = pool_family_blocks_per_cu(f);
        if (bpc < 1) e = hipErrorInvalidConfiguration;
        pl->blocks[f] = bpc * pl->ncu;
    }
    if (e != hipSuccess) {
        const int code = (e == hipErrorOutOfMemory) ? RBFSL_E_NOMEM : RBFSL_E_DEVICE;
        pool_free(pl);
        delete pl;
        return code;
    }
    *out = pl;
    return RBFSL_OK;
}

int64_t rbfsl_pool_run_bytes(int64_t N, const rbfsl_params *p, int64_t nsteps) {
    if (!p || N < 1 || nsteps < 1 || p->n < 1 || p->n_tracers < 1) return -1;
    return (int64_t)al(run_layout(N, p->n, p->n_tracers, nsteps).total);
}

int rbfsl_pool_add(rbfsl_pool *pl, const double *nodes_xyz, int64_t N, int nodes_on_device,
                   const rbfsl_params *p, const double *q0, int q_on_device, int64_t nsteps, int64_t *run_id) {
    return pool_add_impl(pl, nodes_xyz, N, nodes_on_device, p, q0, q_on_device, nsteps, run_id);
}

int rbfsl_pool_step(rbfsl_pool *pl, int64_t nsteps) {
    if (!pl || nsteps < 0) return RBFSL_E_INVAL;
    for (int64_t i = 0; i < nsteps; ++i) {
        if (active_runs(pl) == 0) break;
        const int r = launch_one_step(pl);
        if (r != RBFSL_OK) return r;
    }
    return reconcile(pl);
}

int rbfsl_pool_run_info(rbfsl_pool *pl, int64_t run_id, int64_t *step, int64_t *nsteps, int *status) {
    if (!pl) return RBFSL_E_INVAL;
    const int s = slot_for(pl, run_id);
    if (s < 0) return pfail(pl, RBFSL_E_INVAL, "unknown run %lld", (long long)run_id);
    const int rc = reconcile(pl);
    if (rc != RBFSL_OK) return rc;
    const Run &r = pl->runs[s];
    if (step) *step = r.h_step;
    if (nsteps) *nsteps = r.nsteps;
    if (status) *status = r.failed ? r.fail_code : RBFSL_OK;
    return RBFSL_OK;
}

int rbfsl_pool_get_q(rbfsl_pool *pl, int64_t run_id, double *out, int on_device) {
    if (!pl || !out) return RBFSL_E_INVAL;
    const int s = slot_for(pl, run_id);
    if (s < 0) return pfail(pl, RBFSL_E_INVAL, "unknown run %lld", (long long)run_id);
    const int rc = reconcile(pl);
    if (rc != RBFSL_OK) return rc;
    const Run &r = pl->runs[s];
    const double *q = pl->h_runs[s].q[pl->h_state[s].cur];
    PHIP(pl, hipMemcpy(out, q, sizeof(double) * r.N * r.ntr, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return RBFSL_OK;
}

int rbfsl_pool_remove(rbfsl_pool *pl, int64_t run_id) {
    if (!pl) return RBFSL_E_INVAL;
    const int s = slot_for(pl, run_id);
    if (s < 0) return pfail(pl, RBFSL_E_INVAL, "unknown run %lld", (long long)run_id);
    PHIP(pl, hipStreamSynchronize(pl->main));
    PHIP(pl, hipStreamSynchronize(pl->admit));
    int rc = release_run(pl, s);
    if (rc != RBFSL_OK) return rc;
    PHIP(pl, hipStreamSynchronize(pl->main));
    return RBFSL_OK;
}

static_assert(sizeof(rbfsl_pool_stats::blocks) / sizeof(int32_t) == POOL_FAMILIES &&
                  sizeof(rbfsl_pool_stats::items_per_step) / sizeof(int64_t) == POOL_FAMILIES,
              "one entry per kernel family");

int rbfsl_pool_info(rbfsl_pool *pl, rbfsl_pool_stats *st) {
    if (!pl || !st) return RBFSL_E_INVAL;
    memset(st, 0, sizeof(*st));
    for (const Run &r : pl->runs) {
        st->runs += r.used ? 1 : 0;
        st->active += r.in_table() ? 1 : 0;
    }
    st->bytes_used = (int64_t)pl->arena.used;
    st->bytes_budget = (int64_t)pl->arena.size;
    st->steps_launched = pl->steps_launched;
    for (int f = 0; f < POOL_FAMILIES; ++f) {
        st->items_per_step[f] = pl->items_last[f];
        st->blocks[f] = pl->blocks[f];
    }
    st->graph = pl->use_graph ? 1 : 0;
    return RBFSL_OK;
}

int rbfsl_pool_variants(int32_t *mcap, int32_t *waves, int32_t *group, int32_t *panel, int32_t cap) {
    const PoolVariantInfo *v;
    const int nv = pool_variants(&v);
    for (int i = 0; i < nv && i < cap; ++i) {
        if (mcap) mcap[i] = v[i].mcap;
        if (waves) waves[i] = v[i].W;
        if (group) group[i] = v[i].G;
        if (panel) panel[i] = v[i].B;
    }
    return nv;
}

int rbfsl_pool_set_variant(rbfsl_pool *pl, int32_t M, int32_t variant) {
    if (!pl) return RBFSL_E_INVAL;
    const PoolVariantInfo *v;
    const int nv = pool_variants(&v);
    if (variant < -1 || variant >= nv || (variant >= 0 && v[variant].mcap < M))
        return pfail(pl, RBFSL_E_INVAL, "variant %d cannot solve systems of size %d", variant, M);
    const int rc = reconcile(pl);
    if (rc != RBFSL_OK) return rc;
    if (variant < 0) pl->tuned.erase(M);
    else pl->tuned[M] = variant;
    const int gi = pick_variant(pl, M);
    for (Run &r : pl->runs)
        if (r.used && r.M == M) set_variant(r, gi);
    pl->dirty = true;
    return RBFSL_OK;
}

int rbfsl_pool_tune(rbfsl_pool *pl, int32_t trials, rbfsl_tune_result *res, int32_t cap, int32_t *count) {
    if (!pl || trials < 1) return RBFSL_E_INVAL;
    if (count) *count = 0;
    int rc = reconcile(pl);
    if (rc != RBFSL_OK) return rc;
    const PoolVariantInfo *v;
    const int nv = pool_variants(&v);
    std::vector<int> sizes;
    for (const Run &r : pl->runs)
        if (r.in_table() && std::find(sizes.begin(), sizes.end(), r.M) == sizes.end()) sizes.push_back(r.M);
    std::sort(sizes.begin(), sizes.end());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PHIP(pl, hipEventCreate(&e0));
    PHIP(pl, hipEventCreate(&e1));
    int nres = 0;
    std::vector<int> saved_var(pl->max_runs);
    for (int M : sizes) {
        int best = -1;
        float best_ms = 0.f;
        for (int gi = 0; gi < nv; ++gi) {
            if (v[gi].mcap < M) continue;
            // only the runs of this size, all on candidate gi; dry steps
            // (no commit): q^{m+1} lands in the idle buffer and is discarded
            std::vector<Run> keep = pl->runs;
            for (Run &r : pl->runs) {
                if (r.in_table() && r.M == M) set_variant(r, gi);
                else if (r.used) r.failed = true;  // hidden from the queues
            }
            rc = upload_tables(pl);
            float ms = 0.f;
            hipError_t e = hipSuccess;
            if (rc == RBFSL_OK) {
                e = enqueue_search(pl);  // warm-up
                if (e == hipSuccess) e = enqueue_step_kernels(pl, false);
                if (e == hipSuccess) e = hipEventRecord(e0, pl->main);
                for (int t = 0; t < trials && e == hipSuccess; ++t) {
                    e = enqueue_search(pl);
                    if (e == hipSuccess) e = enqueue_step_kernels(pl, false);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, pl->main);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            }
            pl->runs = keep;
            pl->dirty = true;
            if (rc != RBFSL_OK || e != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc != RBFSL_OK ? rc : pfail(pl, RBFSL_E_DEVICE, "tuning step: %s", hipGetErrorString(e));
            }
            ms /= (float)trials;
            if (res && nres < cap) {
                res[nres].M = M;
                res[nres].variant = gi;
                res[nres].ms_per_step = ms;
                res[nres].chosen = 0;
            }
            const int idx = nres++;
            if (best < 0 || ms < best_ms) {
                best = gi;
                best_ms = ms;
                for (int i = 0; i < idx && res && i < cap; ++i)
                    if (res[i].M == M) res[i].chosen = 0;
                if (res && idx < cap) res[idx].chosen = 1;
            }
        }
        pl->tuned[M] = best;
        for (Run &r : pl->runs)
            if (r.used && r.M == M) set_variant(r, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (count) *count = nres;
    pl->dirty = true;
    // a run that a dry step found failing fails the same way in its real step
    return reconcile(pl);
}

int rbfsl_pool_serve(rbfsl_pool *pl, const rbfsl_request *req, int64_t nreq, rbfsl_request_result *res,
                     double *wall_seconds) {
    if (!pl || (nreq > 0 && (!req || !res))) return RBFSL_E_INVAL;
    for (int64_t i = 0; i < nreq; ++i) {
        res[i].admitted = res[i].finished = -1.0;
        res[i].status = RBFSL_E_STATE;
        res[i].steps = 0;
    }
    std::vector<int64_t> order((size_t)nreq);
    for (int64_t i = 0; i < nreq; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return req[a].arrival < req[b].arrival; });
    std::map<int64_t, int64_t> req_of;  // run id -> request
    std::vector<int64_t> pending;       // FIFO of arrived requests
    size_t next = 0, head = 0;
    int64_t done = 0;
    const double t0 = now_s();
    std::vector<hipEvent_t> ev(3, nullptr);
    for (auto &e : ev) PHIP(pl, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int64_t s = 0;
    int rc = RBFSL_OK;
    // Shortest remaining work first, in batches: a step takes the admitted
    // runs whose estimated remaining device time, divided by 1 + (time since
    // admission) / SERVE_AGING_S, is at most SERVE_BATCH times the smallest.
    // Runs of similar remaining work step together; a small request is not
    // held to the pace of the largest one admitted, and the division lets a
    // long-admitted run's turn come even while short requests keep arriving.
    constexpr double SERVE_BATCH = 2.0, SERVE_AGING_S = 30.0;
    std::vector<double> admitted_at((size_t)pl->max_runs, 0.0);
    auto step_cost_us = [](const Run &r) {  // per-node cost ~ 0.03 us x (M / 47)^2.5, plus a step's floor
        return 300.0 + 0.03 * (double)r.N * pow((double)r.M / 47.0, 2.5);
    };
    auto finish = [&](int slot, double tnow) -> int {
        Run &r = pl->runs[slot];
        const int64_t i = req_of[r.id];
        const int *st = pl->h_status + ST_WORDS * slot;
        res[i].status = r.failed ? code_of(st) : RBFSL_OK;
        res[i].steps = pl->h_state[slot].step;
        const double *q = pl->h_runs[slot].q[pl->h_state[slot].cur];
        hipError_t e = hipMemcpy(req[i].q_out, q, sizeof(double) * r.N * r.ntr, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return pfail(pl, RBFSL_E_DEVICE, "result copy: %s", hipGetErrorString(e));
        res[i].finished = now_s() - tnow;
        req_of.erase(r.id);
        ++done;
        if (pl->log_requests)
            fprintf(stderr, "serve: request %lld done at %.2f s (%lld of %lld), status %d, %lld steps\n", (long long)i,
                    res[i].finished, (long long)done, (long long)nreq, res[i].status, (long long)res[i].steps);
        return release_run(pl, slot);
    };
    while (done < nreq && rc == RBFSL_OK) {
        const double now = now_s() - t0;
        while (next < order.size() && req[order[next]].arrival <= now) pending.push_back(order[next++]);
        // admission, first come first served, while a slot and HBM are free
        while (head < pending.size()) {
            const int64_t i = pending[head];
            int64_t id = -1;
            const int a = pool_add_impl(pl, req[i].nodes_xyz, req[i].N, 0, &req[i].params, req[i].q0, 0,
                                        req[i].nsteps, &id);
            if (a == RBFSL_E_BUDGET) break;
            ++head;
            res[i].admitted = now_s() - t0;
            if (a != RBFSL_OK) {  // rejected outright
                res[i].status = a;
                res[i].finished = res[i].admitted;
                ++done;
                continue;
            }
            req_of[id] = i;
            admitted_at[(size_t)pl->slot_of[id]] = res[i].admitted;
        }
        if (active_runs(pl) == 0) {
            if (head == pending.size() && next < order.size()) {
                const double wait = req[order[next]].arrival - (now_s() - t0);
                if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait < 1e-3 ? wait : 1e-3));
                continue;
            }
            if (head < pending.size() && req_of.empty()) {  // the head request can never fit
                const int64_t i = pending[head++];
                res[i].status = RBFSL_E_BUDGET;
                res[i].admitted = res[i].finished = now_s() - t0;
                ++done;
                continue;
            }
            if (req_of.empty()) continue;
        } else {
            const double tq = now_s() - t0;
            std::vector<double> rem((size_t)pl->max_runs, -1.0);
            double least = -1.0;
            for (int q = 0; q < pl->max_runs; ++q) {
                const Run &r = pl->runs[q];
                if (!r.in_table()) continue;
                const double age = tq - admitted_at[(size_t)q];
                rem[(size_t)q] = (double)(r.nsteps - r.h_step) * step_cost_us(r) / (1.0 + age / SERVE_AGING_S);
                if (least < 0.0 || rem[(size_t)q] < least) least = rem[(size_t)q];
            }
            for (int q = 0; q < pl->max_runs; ++q) {
                Run &r = pl->runs[q];
                if (!r.in_table()) continue;
                const bool h = rem[(size_t)q] > SERVE_BATCH * least;
                if (h != r.hold) {
                    r.hold = h;
                    pl->dirty = true;
                }
            }
            rc = launch_one_step(pl);
            if (rc != RBFSL_OK) break;
            hipError_t e = hipEventRecord(ev[s % 3], pl->main);
            if (e == hipSuccess && s >= 1) e = hipEventSynchronize(ev[(s - 1) % 3]);  // two steps in flight
            if (e != hipSuccess) {
                rc = pfail(pl, RBFSL_E_DEVICE, "serve step: %s", hipGetErrorString(e));
                break;
            }
            ++s;
        }
        // runs whose last step has been enqueued: collect once it is done
        bool any = false;
        for (const Run &r : pl->runs)
            if (r.used && req_of.count(r.id) && !r.in_table()) any = true;
        if (!any) continue;
        rc = reconcile(pl);
        const double tnow = t0;
        for (int slot = 0; slot < pl->max_runs && rc == RBFSL_OK; ++slot) {
            const Run &r = pl->runs[slot];
            if (r.used && req_of.count(r.id) && !r.in_table()) rc = finish(slot, tnow);
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    for (Run &r : pl->runs)
        if (r.hold) {
            r.hold = false;
            pl->dirty = true;
        }
    if (wall_seconds) *wall_seconds = now_s() - t0;
    if (rc == RBFSL_OK) rc = reconcile(pl);
    return rc;
}

const char *rbfsl_pool_last_error(const rbfsl_pool *pl) { return pl ? pl->err.c_str() : ""; }

void rbfsl_pool_destroy(rbfsl_pool *pl) {
    if (!pl) return;
    (void)hipStreamSynchronize(pl->main);
    for (hipStream_t s : pl->side) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(pl->admit);
    pool_free(pl);
    delete pl;
}

}  // extern "C"

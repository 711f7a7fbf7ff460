#pragma once
// Persistent step kernel of the pooled (batched) transport: one launch moves
// every run of one kernel family by one step, after the search pass has
// found the departure point and stencil of every node (Algorithm 1 for each
// node of each run; the search does not depend on q and runs at its own,
// higher occupancy).
//
// Workgroups of NW waves claim items from the family's queue, two per atomic
// (k_pool below).  An item is G consecutive nodes of one run, G = NW / W for a solver
// variant with W waves per stencil: the G stencil groups of the workgroup
// work side by side, each on its own node.  Per node: the q^m values of the
// stencil are fetched into LDS (their latency hides behind the assembly),
// the saddle system (eq. rbf_poly_linsys) is assembled and solved, and
// q^{m+1}_j = sum_a w_a q^m[S_a] for every tracer.  Nothing per node goes to
// HBM but q^{m+1}.  The arithmetic is the same code as the single-run
// kernels (solve_system and the fma chain of the apply), so the two paths
// agree bit for bit.
//
// Groups of one workgroup share its barriers; they always solve systems of
// one size (same run), and solve_system's lockstep mode keeps their barrier
// sequences identical even when one of them meets a singular system.
#include "k_solve.h"
#include "pool_impl.h"

namespace rbfsl {

template <int W_, int R_, int NCB_, int B_, int CM_ = 24>
struct PV {
    static constexpr int W = W_, R = R_, NCB = NCB_, B = B_, CM = CM_;
    static constexpr int MCAP = Cfg<W_, R_, NCB_, B_, 1, CM_>::MCAP;
    using Smem = SolveSmem<W_, R_, NCB_, B_, CM_>;
};

// LDS of one stencil group: the solver's, and the q^m values of the stencil
// for up to QT tracers (more tracers are gathered after the solve).
constexpr int POOL_QT = 4;
template <class V>
struct GroupSmem {
    typename V::Smem sol;
    double qp[POOL_QT * V::MCAP];
};

template <int NW, class V>
constexpr size_t pool_smem_bytes() {
    return (size_t)(NW / V::W) * sizeof(GroupSmem<V>);
}
template <int NW, class V0, class... Vs>
constexpr size_t pool_smem_max() {
    if constexpr (sizeof...(Vs) == 0) return pool_smem_bytes<NW, V0>();
    else {
        constexpr size_t a = pool_smem_bytes<NW, V0>(), b = pool_smem_max<NW, Vs...>();
        return a > b ? a : b;
    }
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(unsigned)hi << 32) | (unsigned)lo);
}

// sum_a w[a] q[a] as one fma chain in stencil order, both operands in LDS;
// the loads of eight terms are issued together ahead of their fmas
__device__ __forceinline__ double lds_dot_chain(const double *w, const double *q, const int n) {
    double acc = 0.0;
    int a = 0;
    for (; a + 8 <= n; a += 8) {
        double wv[8], qv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            wv[u] = w[a + u];
            qv[u] = q[a + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(wv[u], qv[u], acc);
    }
    for (; a < n; ++a) acc = fma(w[a], q[a], acc);
    return acc;
}

struct ItemInfo {
    int64_t j0, step;
    int slot, var, cnt, cur, valid, skip;
};

template <int NW, class V>
__device__ __forceinline__ void pool_item(const PoolArgs &P, const ItemInfo &I, unsigned char *smem,
                                          const int t) {
    constexpr int W = V::W, G = NW / W;
    static_assert(NW % W == 0, "groups must tile the workgroup");
    GroupSmem<V> *gsm = reinterpret_cast<GroupSmem<V> *>(smem);
    const int wave = t >> 6, lane = t & 63;
    const int grp = wave / W, gw = wave - grp * W, gt = t - grp * 64 * W;
    GroupSmem<V> &S = gsm[grp];
    const PoolRunDev &r = P.runs[I.slot];
    const int n = r.n;
    const int64_t N = r.N;
    const int64_t j = I.j0 + grp;
    const bool mine = grp < I.cnt;

    // the stencil's q^m values: issued now, consumed after the solve (whose
    // barriers order the LDS writes before the reads)
    const int32_t *Sj = r.S + j * n;
    const bool pre = r.ntr * n <= POOL_QT * V::MCAP;
    if (gw == 0 && mine && pre) {
        const double *qin = r.q[I.cur];
        for (int idx = lane; idx < r.ntr * n; idx += 64) {
            const int tr = idx / n, a = idx - tr * n;
            const int g = Sj[a];
            S.qp[idx] = ((unsigned)g < (unsigned)N) ? qin[(int64_t)tr * N + g] : 0.0;
        }
    }

    // a group without a node solves a stand-in system (node 0's) in lockstep
    // with the others; its result is dropped
    const int64_t js = mine ? j : 0;
    SysIn in;
    in.nx = r.nx; in.ny = r.ny; in.nz = r.nz; in.N = N;
    in.S = r.S + js * n;
    in.xe[0] = r.xi[js]; in.xe[1] = r.xi[N + js]; in.xe[2] = r.xi[2 * N + js];
    in.ctr[0] = in.xe[0]; in.ctr[1] = in.xe[1]; in.ctr[2] = in.xe[2];
    in.s2 = r.s2[js];
    in.n = n; in.L = r.L; in.k = r.k;
    in.status = r.status; in.step = I.step;
    const bool solved = solve_system<W, V::R, V::NCB, V::B, (G > 1), V::CM>(S.sol, gt, in);

    // q^{m+1} of node j, by the first wave of the group: lane tr runs tracer
    // tr's fma chain in stencil order over the fetched values
    if (gw == 0 && mine) {
        const double *zb = S.sol.zb;
        if (!solved) {
            if (lane == 0) {
                atomicAdd(&r.status[ST_SINGULAR], 1);
                atomicMin(&r.status[ST_FAILSTEP], (int)I.step);
            }
            return;
        }
        bool bad = false;
        for (int a = lane; a < n; a += 64)
            if (!isfinite(zb[a])) bad = true;
        if (__ballot(bad)) {
            if (lane == 0) {
                atomicAdd(&r.status[ST_NONFINITE], 1);
                atomicMin(&r.status[ST_FAILSTEP], (int)I.step);
            }
            return;
        }
        double *qout = r.q[1 - I.cur];
        if (pre) {
            for (int tr = lane; tr < r.ntr; tr += 64) {
                qout[(int64_t)tr * N + j] = lds_dot_chain(zb, S.qp + tr * n, n);
            }
            return;
        }
        // many tracers: gather them in chunks through the (now free) stage
        double *qg = S.sol.stage;
        const double *qin = r.q[I.cur];
        constexpr int STAGE = Cfg<W, V::R, V::NCB, V::B, 1, V::CM>::STAGE;
        const int tchunk = (STAGE / n < 64) ? STAGE / n : 64;  // >= 1
        for (int t0 = 0; t0 < r.ntr; t0 += tchunk) {
            const int tc = (r.ntr - t0 < tchunk) ? r.ntr - t0 : tchunk;
            for (int idx = lane; idx < tc * n; idx += 64) {
                const int tr = idx / n, a = idx - tr * n;
                const int g = Sj[a];
                qg[idx] = ((unsigned)g < (unsigned)N) ? qin[(int64_t)(t0 + tr) * N + g] : 0.0;
            }
            wave_lds_sync();
            if (lane < tc) {
                qout[(int64_t)(t0 + lane) * N + j] = lds_dot_chain(zb, qg + lane * n, n);
            }
            wave_lds_sync();
        }
    }
}

template <int NW, int I0, class V0, class... Vs>
__device__ __forceinline__ void pool_dispatch(const int var, const PoolArgs &P, const ItemInfo &I,
                                              unsigned char *smem, const int t) {
    if (var == I0) {
        pool_item<NW, V0>(P, I, smem, t);
    } else if constexpr (sizeof...(Vs) > 0) {
        pool_dispatch<NW, I0 + 1, Vs...>(var, P, I, smem, t);
    }
}

// Thread 0's claim state, kept in LDS (not in registers, which the solver
// needs): the claimed but unprocessed items, and the last decoded segment
// with everything about it that is fixed during the step.
struct ClaimCache {
    int64_t nxt, end;    // claimed items not yet processed: [nxt, end)
    int64_t s_lo, s_hi;  // item range of the cached segment
    int64_t nitems, item0, N, step, nsteps;
    const int *status;
    int slot, var, G, cur;
};

// Claims items until the queue is empty.  Thread 0 claims POOL_CLAIM items
// per atomic and decodes them, searching the segment table only when an
// item leaves the cached segment; the item record is double-buffered so one
// barrier per item suffices.
constexpr int POOL_CLAIM = 2;
template <int NW, int WPE, class... V>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_pool(PoolArgs P) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[pool_smem_max<NW, V...>()];
    __shared__ ItemInfo info[2];
    __shared__ ClaimCache cc;
    const int t = threadIdx.x;
    PoolQueue *Q = P.queue;
    if (t == 0) {
        cc.nxt = cc.end = 0;
        cc.s_lo = cc.s_hi = 0;
        cc.nitems = Q->nitems;
    }
    for (int it = 0;; ++it) {
        ItemInfo &I = info[it & 1];
        if (t == 0) {
            if (cc.nxt >= cc.end) {
                const int64_t b = (int64_t)atomicAdd(&Q->next, (unsigned long long)POOL_CLAIM);
                cc.nxt = b;
                cc.end = b + POOL_CLAIM;
            }
            const int64_t item = cc.nxt++;
            I.valid = item < cc.nitems;
            if (I.valid) {
                if (!(item >= cc.s_lo && item < cc.s_hi)) {
                    const int nseg = Q->nseg;
                    int lo = 0, hi = nseg - 1;  // last segment with item0 <= item
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (Q->seg[mid].item0 <= item) lo = mid;
                        else hi = mid - 1;
                    }
                    const PoolSeg &sg = Q->seg[lo];
                    cc.s_lo = sg.item0;
                    cc.s_hi = (lo + 1 < nseg) ? Q->seg[lo + 1].item0 : cc.nitems;
                    cc.item0 = sg.item0;
                    cc.N = sg.N;
                    cc.G = sg.G;
                    cc.slot = sg.slot;
                    cc.var = sg.var;
                    cc.step = P.state[sg.slot].step;
                    cc.cur = P.state[sg.slot].cur;
                    const PoolRunDev &r = P.runs[sg.slot];
                    cc.nsteps = r.nsteps;
                    cc.status = r.status;
                }
                const int64_t j0 = (item - cc.item0) * cc.G;
                I.slot = cc.slot;
                I.var = cc.var;
                I.j0 = j0;
                I.cnt = (int)((cc.N - j0 < cc.G) ? cc.N - j0 : cc.G);
                I.step = cc.step;
                I.cur = cc.cur;
                // finished, or failed at this or an earlier step
                I.skip = (cc.step >= cc.nsteps) || (cc.status[ST_FAILSTEP] <= cc.step);
            }
        }
        __syncthreads();
        if (!I.valid) break;
        if (I.skip) continue;
        // the item is the same for the whole workgroup: keep it in scalar
        // registers (the run's pointers are then scalar loads)
        ItemInfo U;
        U.j0 = uniform64(I.j0);
        U.step = uniform64(I.step);
        U.slot = __builtin_amdgcn_readfirstlane(I.slot);
        U.var = __builtin_amdgcn_readfirstlane(I.var);
        U.cnt = __builtin_amdgcn_readfirstlane(I.cnt);
        U.cur = __builtin_amdgcn_readfirstlane(I.cur);
        U.valid = 1;
        U.skip = 0;
        // the thread index, made opaque per item: otherwise the compiler
        // hoists the solver's per-slot LDS addresses out of the item loop and
        // keeps them all live (spilling the matrix registers)
        int tl = t;
        __asm__ volatile("" : "+v"(tl));
        pool_dispatch<NW, 0, V...>(U.var, P, U, smem, tl);
    }
}

}  // namespace rbfsl

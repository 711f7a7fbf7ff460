// Weights from stored factorizations: the paper's centre-point stencils
// (Section 3.3.2), whose systems depend only on the centre node, are factored
// once; every step then only builds the right-hand side [phi(|y_a - y_xi|);
// p(xi)] of each departure point and replays the stored elimination on it.
//
// The replay is the exact operation sequence the full elimination applies to
// the right-hand side: for step k with pivot row p_k, every row i takes
// y_i = fma(-l_ik, y_pk, y_i) with l_ik = a_ik r_k for rows not yet pivoted
// (a_ik: column k as step k found it, which is what the stored matrix holds
// there) and l_ik = 0 for the others; then back substitution from the last
// unknown, z_k = y_pk r_k, y_i = fma(-u_ik, z_k, y_i) for rows pivoted before
// step k.  The weights are therefore bit for bit those of refactoring.
//
// One wave per evaluation point, positions in pivot order on lanes (R slots),
// the replay itself in k_replay.h: the stored matrix keeps its rows in pivot
// order, so step k's multipliers are the positions below k of column k and
// its U entries the positions above it; each stored element is read once,
// and the kernel is bound by HBM bandwidth: 8 M^2 bytes per point.
#include "dev_util.h"
#include "k_replay.h"
#include "k_solve.h"

namespace rbfsl {

// the largest harmonic basis a system can carry: (L+1)^2 <= n and
// n + (L+1)^2 <= MAX_SYSTEM, so (L+1)^2 <= MAX_SYSTEM / 2
constexpr int MAX_BASIS = MAX_SYSTEM / 2;

template <int R>
__global__ void __launch_bounds__(64) k_solve_cached(CachedArgs A) {
    __shared__ double peb[MAX_BASIS];  // basis values at the evaluation point
    const int64_t j = blockIdx.x;
    const int lane = threadIdx.x;
    if (__builtin_amdgcn_readfirstlane(A.status[ST_FAILSTEP]) <= A.step) return;
    const int n = A.n, L = A.L, k = A.k;
    const int mL = (L + 1) * (L + 1);
    const int M = n + mL;
    const int64_t K = A.cidx[j];
    if (A.fstat[K] != 0) {
        if (lane == 0) {
            atomicAdd(&A.status[ST_SINGULAR], 1);
            atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
        }
        return;
    }
    const double ctr[3] = {A.nx[K], A.ny[K], A.nz[K]};
    const double s2 = A.s2[K];
    const double s = (s2 > 0.0) ? sqrt(s2) : 1.0;
    const double inv_s = 1.0 / s;
    double e1[3], e2[3];
    frame3(ctr, e1, e2);
    const double xe[3] = {A.ex[j], A.ey[j], A.ez[j]};
    double yx[3], al, be, u;
    local3(xe, ctr, e1, e2, inv_s, yx, al, be, u);
    if (lane == 0) basis_all(L, al, be, u, peb);
    wave_lds_sync();

    // right-hand side, as the assembly builds it, moved to pivot order
    __shared__ double yl[MAX_SYSTEM];
    const int32_t *Srow = A.S + K * n;
    const int32_t *stepof = A.stepof + K * M;
    sfor<0, R>([&](auto RI) SI {
        constexpr int r = RI;
        const int i = lane + 64 * r;
        double rhs = 0.0;
        if (i < n) {
            int g = Srow[i];
            if (g < 0 || (int64_t)g >= A.N) {  // not a node index: flag the stencil, read node 0
                atomicAdd(&A.status[ST_SEARCH], 1);
                atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
                g = 0;
            }
            const double x[3] = {A.nx[g], A.ny[g], A.nz[g]};
            double yi[3], ai, bi, ui;
            local3(x, ctr, e1, e2, inv_s, yi, ai, bi, ui);
            const double d0 = yi[0] - yx[0], d1 = yi[1] - yx[1], d2 = yi[2] - yx[2];
            rhs = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
        } else if (i < M) {
            rhs = peb[i - n];
        }
        if (i < M) yl[stepof[i]] = rhs;
    });
    wave_lds_sync();
    double y[R];  // y at position q = lane + 64 r (the row pivoted at step q)
    sfor<0, R>([&](auto RI) SI {
        constexpr int r = RI;
        const int q = lane + 64 * r;
        y[r] = (q < M) ? yl[q] : 0.0;
    });

    // the stored elimination replayed; z_k for k < n are the weights
    bool bad = false;
    replay_solve<R>(A.F + K * (int64_t)M * M, A.rinv + K * M, M, lane, y, [&](int kk, double zk) SI {
        if (kk < n) {
            if (lane == 0) A.w[j * n + kk] = zk;
            if (!isfinite(zk)) bad = true;
        }
    });
    if (bad && lane == 0) {
        atomicAdd(&A.status[ST_NONFINITE], 1);
        atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
    }
}

hipError_t launch_solve_cached(const CachedArgs &a, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    const int M = a.n + (a.L + 1) * (a.L + 1);
    const dim3 grid((unsigned)a.count), block(64);
    if (M <= 64) hipLaunchKernelGGL(k_solve_cached<1>, grid, block, 0, s, a);
    else if (M <= 128) hipLaunchKernelGGL(k_solve_cached<2>, grid, block, 0, s, a);
    else if (M <= 192) hipLaunchKernelGGL(k_solve_cached<3>, grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace rbfsl

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
// One wave per evaluation point, rows on lanes (R row slots); the stored
// matrix streams from HBM column by column (read twice), so the kernel is
// bound by HBM bandwidth: 16 M^2 bytes per point.
#include "dev_util.h"
#include "k_solve.h"

namespace rbfsl {

template <int R>
__global__ void __launch_bounds__(64) k_solve_cached(CachedArgs A) {
    __shared__ double peb[64];  // basis values at the evaluation point
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

    // right-hand side, as the assembly builds it
    const int32_t *Srow = A.S + K * n;
    double y[R];
    int stp[R];
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
        y[r] = rhs;
        stp[r] = (i < M) ? stepof[i] : -1;  // padding rows count as pivoted from the start
    });

    const double *F = A.F + K * (int64_t)M * M;
    const int32_t *piv = A.piv + K * M;
    const double *rinv = A.rinv + K * M;
    // forward: the elimination's updates of the right-hand side
    for (int kk = 0; kk < M; ++kk) {
        const int p = __builtin_amdgcn_readfirstlane(piv[kk]);
        const double rk = rinv[kk];
        const int pl = p & 63, pr = p >> 6;
        double yp = bcast_d(y[0], pl);
        sfor<1, R>([&](auto RI) SI {
            constexpr int r = RI;
            const double yr = bcast_d(y[r], pl);
            yp = (pr == r) ? yr : yp;
        });
        sfor<0, R>([&](auto RI) SI {
            constexpr int r = RI;
            const int i = lane + 64 * r;
            const double a = (i < M) ? F[(int64_t)kk * M + i] : 0.0;
            const double l = (stp[r] <= kk) ? 0.0 : a * rk;
            y[r] = fma(-l, yp, y[r]);
        });
    }
    // back substitution; z_k for k < n are the weights
    bool bad = false;
    for (int kk = M - 1; kk >= 0; --kk) {
        const int p = __builtin_amdgcn_readfirstlane(piv[kk]);
        const double rk = rinv[kk];
        const int pl = p & 63, pr = p >> 6;
        double yk = bcast_d(y[0], pl);
        sfor<1, R>([&](auto RI) SI {
            constexpr int r = RI;
            const double yr = bcast_d(y[r], pl);
            yk = (pr == r) ? yr : yk;
        });
        const double zk = yk * rk;
        if (kk < n) {
            if (lane == 0) A.w[j * n + kk] = zk;
            if (!isfinite(zk)) bad = true;
        }
        sfor<0, R>([&](auto RI) SI {
            constexpr int r = RI;
            const int i = lane + 64 * r;
            const double uik = (i < M) ? F[(int64_t)kk * M + i] : 0.0;
            const double yn = fma(-uik, zk, y[r]);
            y[r] = (stp[r] < kk) ? yn : y[r];
        });
    }
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

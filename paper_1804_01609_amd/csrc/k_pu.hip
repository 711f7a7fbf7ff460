// RBF-PU interpolation in the SL step (Sections 2.3 and 3.3.3): patches are
// spherical caps of one radius R around given centres; each patch's
// augmented interpolant (eq. rbf_poly) is solved for the tracer values at its
// nodes, and the departure point's value is the B-spline partition of unity
// (eq. wght_func, eq. bspline, eq. pu_func) over the patches that contain it
// (eq. PU_interp).
//
// The patch systems do not change between steps: they are factored once
// (k_factor with per-patch node counts).  Per step:
//   k_pu_search  one thread per departure point: the containing patches,
//              through the spatial hash of the centres;
//   k_pu_coef  one wave per (patch, tracer): the right-hand side [q(X_l); 0]
//              in pivot order and the stored elimination replayed on it
//              (k_replay.h), giving the coefficients [c; d];
//   k_pu_patch_eval  one thread per (containing patch, departure point): the
//              patch's interpolant sum_b c_b phi(|y_b - y_xi|) + sum_q d_q p_q(xi)
//              in the patch's frame (one fma chain);
//   k_pu_blend one thread per departure point: the containing patches in
//              (d^2, l) order blended by phi_l = B(sqrt(d^2) / R): numerator by
//              fma, denominator by add, q = numerator / denominator.
// Every expression follows the same operation order as the patch assembly
// of k_solve.h, so the results are bit for bit those of the plain definition.
#include "dev_util.h"
#include "k_replay.h"
#include "k_solve.h"

namespace rbfsl {

// the cubic B-spline of eq. bspline
__device__ __forceinline__ double pu_bspline(double r) {
    if (r < 0.5) {
        double v = 4.0 * (r - 1.0);
        v = v * r;
        v = v * r;
        return (2.0 / 3.0) + v;
    }
    if (r < 1.0) {
        const double t = r - 1.0;
        double v = t * t;
        v = v * t;
        return (-4.0 / 3.0) * v;
    }
    return 0.0;
}

__global__ void k_pu_count(PuArgs A, int nallow, int32_t *cnt, int *nmax) {
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= A.Mp) return;
    const double *d2 = A.pd2 + l * A.ncap;
    int c = 0;
    while (c < A.ncap && d2[c] < A.R2) ++c;
    // a full list may miss nodes of the cap (unless it holds every node); an
    // empty or too large patch has no usable system
    if ((c == A.ncap && (int64_t)A.ncap < A.N) || c == 0 || c > nallow) {
        atomicAdd(&A.status[ST_SEARCH], 1);
        atomicMin(&A.status[ST_FAILSTEP], 0);
    }
    cnt[l] = c;
    atomicMax(nmax, c);
}

hipError_t launch_pu_count(const PuArgs &a, int nmax_allowed, int32_t *cnt, int *nmax, hipStream_t s) {
    if (a.Mp <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pu_count, dim3((unsigned)((a.Mp + 255) / 256)), dim3(256), 0, s, a, nmax_allowed,
                       cnt, nmax);
    return hipGetLastError();
}

// cell of coordinate v in the spatial hash (the formula of its build)
__device__ __forceinline__ int pu_cell(double v, double invh, int G) {
    const double f = floor((v + 1.0) * invh);
    if (!(f >= 0.0)) return 0;  // also NaN
    return (f > (double)(G - 1)) ? G - 1 : (int)f;
}

// One thread per departure point: every centre with d^2 < R2, found in the
// hash cells that cover the cube of half-width R (1 + 1e-9) around the point
// (a centre with computed d^2 < R2 differs from the point by less than
// R (1 + 2^-52) in each coordinate, and the cell index is monotone in the
// coordinate, so the enlargement, far above any rounding of the cube's faces,
// loses none), kept in ascending (d^2, l) order -- the prefix of the sorted
// list of all centres.  d^2 = (dx*dx + dy*dy) + dz*dz with d = centre - point.
__global__ void __launch_bounds__(256) k_pu_search(PuArgs A, int G, double invh, const int *cell_start,
                                                  const double *sx, const double *sy, const double *sz,
                                                  const int *perm) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= A.N) return;
    if (A.status[ST_FAILSTEP] <= A.step) return;
    const double q0 = A.ex[j], q1 = A.ey[j], q2 = A.ez[j];
    int32_t *si = A.sidx + j * A.pcap;
    double *sd = A.sd2 + j * A.pcap;
    int lo[3], hi[3];
    const double qv[3] = {q0, q1, q2};
    const double Re = A.R * (1.0 + 1e-9);
    for (int a = 0; a < 3; ++a) {
        lo[a] = pu_cell(qv[a] - Re, invh, G);
        hi[a] = pu_cell(qv[a] + Re, invh, G);
    }
    int cnt = 0;
    bool over = false;
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
        for (int cy = lo[1]; cy <= hi[1]; ++cy)
            for (int cx = lo[0]; cx <= hi[0]; ++cx) {
                const int c = (cz * G + cy) * G + cx;
                for (int p = cell_start[c]; p < cell_start[c + 1]; ++p) {
                    const double d0 = sx[p] - q0, d1 = sy[p] - q1, d2 = sz[p] - q2;
                    const double dist = (d0 * d0 + d1 * d1) + d2 * d2;
                    if (!(dist < A.R2)) continue;
                    const int32_t l = perm[p];
                    if (cnt == A.pcap) {
                        over = true;
                        continue;
                    }
                    // insertion in (d^2, l) order
                    int pos = cnt;
                    while (pos > 0 && (sd[pos - 1] > dist || (sd[pos - 1] == dist && si[pos - 1] > l))) {
                        sd[pos] = sd[pos - 1];
                        si[pos] = si[pos - 1];
                        --pos;
                    }
                    sd[pos] = dist;
                    si[pos] = l;
                    ++cnt;
                }
            }
    for (int c = cnt; c < A.pcap; ++c) {
        sd[c] = __builtin_inf();
        si[c] = 0;
    }
    if (over) {
        atomicAdd(&A.status[ST_SEARCH], 1);
        atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
    }
}

hipError_t launch_pu_search(const PuArgs &a, const Grid &cg, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pu_search, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s, a, cg.G, cg.invh,
                       cg.cell_start, cg.sx, cg.sy, cg.sz, cg.perm);
    return hipGetLastError();
}

// one thread per (patch, node slot): the node's coordinates in the patch's
// frame, y = (x - c) / s with s = sqrt(R2), as the patch's assembly and
// every evaluation compute them
__global__ void __launch_bounds__(256) k_pu_local(PuArgs A) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= A.Mp * A.ncap) return;
    const int64_t l = t / A.ncap;
    const int b = (int)(t - l * A.ncap);
    if (b >= A.cnt[l]) return;
    const double ctr[3] = {A.cx[l], A.cy[l], A.cz[l]};
    const double s = (A.R2 > 0.0) ? sqrt(A.R2) : 1.0;
    const double inv_s = 1.0 / s;
    double e1[3], e2[3];
    frame3(ctr, e1, e2);
    const int g = A.pidx[l * A.ncap + b];
    const double x[3] = {A.nx[g], A.ny[g], A.nz[g]};
    double y[3], al, be, u;
    local3(x, ctr, e1, e2, inv_s, y, al, be, u);
    double *o = A.ploc + t * 3;
    o[0] = y[0];
    o[1] = y[1];
    o[2] = y[2];
}

hipError_t launch_pu_local(const PuArgs &a, hipStream_t s) {
    const int64_t n = a.Mp * a.ncap;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pu_local, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int R>
__global__ void __launch_bounds__(64) k_pu_coef(PuArgs A) {
    __shared__ double yl[64 * R];
    const int64_t l = blockIdx.x;
    const int tr = blockIdx.y;
    const int lane = threadIdx.x;
    if (__builtin_amdgcn_readfirstlane(A.status[ST_FAILSTEP]) <= A.step) return;
    if (A.fstat[l] != 0) return;  // a singular patch: reported where it is used
    const int mL = (A.L + 1) * (A.L + 1);
    const int Ms = A.nmax + mL;   // slot size
    const int n = A.cnt[l];
    const int M = n + mL;
    const int32_t *S = A.pidx + l * A.ncap;
    const int32_t *stepof = A.stepof + l * Ms;
    const double *q = A.qin + (int64_t)tr * A.N;
    // right-hand side [q(X_l); 0], moved to pivot order
    sfor<0, R>([&](auto RI) SI {
        constexpr int r = RI;
        const int i = lane + 64 * r;
        if (i < M) yl[stepof[i]] = (i < n) ? q[S[i]] : 0.0;
    });
    wave_lds_sync();
    double y[R];
    sfor<0, R>([&](auto RI) SI {
        constexpr int r = RI;
        const int p = lane + 64 * r;
        y[r] = (p < M) ? yl[p] : 0.0;
    });
    double *coef = A.coef + ((int64_t)l * A.ntr + tr) * Ms;
    // few waves (one per patch and tracer): a deeper prefetch than the
    // cached-factor kernel's keeps more of HBM busy
    replay_solve<R, 16>(A.F + l * (int64_t)Ms * Ms, A.rinv + l * Ms, M, lane, y, [&](int kk, double zk) SI {
        if (lane == 0) coef[kk] = zk;
    });
}

hipError_t launch_pu_coef(const PuArgs &a, hipStream_t s) {
    if (a.Mp <= 0) return hipSuccess;
    const int Ms = a.nmax + (a.L + 1) * (a.L + 1);
    const dim3 grid((unsigned)a.Mp, (unsigned)a.ntr), block(64);
    if (Ms <= 64) hipLaunchKernelGGL(k_pu_coef<1>, grid, block, 0, s, a);
    else if (Ms <= 128) hipLaunchKernelGGL(k_pu_coef<2>, grid, block, 0, s, a);
    else if (Ms <= 192) hipLaunchKernelGGL(k_pu_coef<3>, grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

constexpr int PU_TB = 4;  // tracers evaluated together

// one thread per (containing-patch slot c, departure point j), slot-major so
// that the threads of a wave share c and are mostly all active: s_l(xi_j) of
// every tracer to sval[(c * ntr + t) * N + j]
__global__ void __launch_bounds__(256) k_pu_patch_eval(PuArgs A) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= A.N) return;
    if (A.status[ST_FAILSTEP] <= A.step) return;
    if (!(A.sd2[j * A.pcap + c] < A.R2)) return;  // not a containing patch
    const int64_t l = A.sidx[j * A.pcap + c];
    if (A.fstat[l] != 0) return;                 // reported by the blend
    const int L = A.L, k = A.k;
    const int Ms = A.nmax + (L + 1) * (L + 1);
    const double xe[3] = {A.ex[j], A.ey[j], A.ez[j]};
    const double ctr[3] = {A.cx[l], A.cy[l], A.cz[l]};
    const double s = (A.R2 > 0.0) ? sqrt(A.R2) : 1.0;
    const double inv_s = 1.0 / s;
    double e1[3], e2[3];
    frame3(ctr, e1, e2);
    double yx[3], al, be, u;
    local3(xe, ctr, e1, e2, inv_s, yx, al, be, u);
    const int n = A.cnt[l];
    const double *yl = A.ploc + l * A.ncap * 3;  // the nodes' local coordinates
    for (int t0 = 0; t0 < A.ntr; t0 += PU_TB) {
        const int tb = (A.ntr - t0 < PU_TB) ? A.ntr - t0 : PU_TB;
        const double *cf = A.coef + (l * A.ntr + t0) * Ms;
        double acc[PU_TB] = {0.0, 0.0, 0.0, 0.0};
        // unrolled so that several nodes' loads and square roots are in
        // flight; the fma chain keeps its order
#pragma unroll 4
        for (int b = 0; b < n; ++b) {
            const double *yb = yl + 3 * b;
            const double d0 = yb[0] - yx[0], d1 = yb[1] - yx[1], d2 = yb[2] - yx[2];
            const double ph = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
            for (int t = 0; t < tb; ++t) acc[t] = fma(cf[t * Ms + b], ph, acc[t]);
        }
        // the polynomial part: the basis of basis_all, value by value
        int col = n;
        double hc = 1.0, hs = 0.0;
        for (int m = 0; m <= L; ++m) {
            if (m > 0) {
                const double nc = al * hc - be * hs;
                const double ns = al * hs + be * hc;
                hc = nc;
                hs = ns;
            }
            for (int sg = 0; sg < (m == 0 ? 1 : 2); ++sg) {
                double v = (sg == 0) ? hc : hs;
                for (int i = 0; i <= L - m; ++i) {
                    for (int t = 0; t < tb; ++t) acc[t] = fma(cf[t * Ms + col], v, acc[t]);
                    ++col;
                    v = v * u;
                }
            }
        }
        for (int t = 0; t < tb; ++t) A.sval[((int64_t)c * A.ntr + t0 + t) * A.N + j] = acc[t];
    }
}

// one thread per departure point: the blend over its containing patches in
// (d^2, l) order
__global__ void __launch_bounds__(256) k_pu_blend(PuArgs A) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= A.N) return;
    if (A.status[ST_FAILSTEP] <= A.step) return;
    const int32_t *sidx = A.sidx + j * A.pcap;
    const double *sd2 = A.sd2 + j * A.pcap;
    int c_end = 0;  // containing patches: the prefix with d^2 < R^2
    while (c_end < A.pcap && sd2[c_end] < A.R2) ++c_end;
    int fail = -1;
    for (int c = 0; c < c_end && fail < 0; ++c)
        if (A.fstat[sidx[c]] != 0) fail = ST_SINGULAR;
    double den = 0.0;
    for (int c = 0; c < c_end; ++c) den = den + pu_bspline(sqrt(sd2[c]) / A.R);
    if (fail < 0 && !(den > 0.0)) fail = ST_SEARCH;  // in no patch
    if (fail >= 0) {
        atomicAdd(&A.status[fail], 1);
        atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
        return;
    }
    for (int t = 0; t < A.ntr; ++t) {
        double num = 0.0;
        for (int c = 0; c < c_end; ++c) {
            const double phi = pu_bspline(sqrt(sd2[c]) / A.R);
            num = fma(phi, A.sval[((int64_t)c * A.ntr + t) * A.N + j], num);
        }
        A.qout[(int64_t)t * A.N + j] = num / den;
    }
}

hipError_t launch_pu_eval(const PuArgs &a, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    const unsigned bx = (unsigned)((a.N + 255) / 256);
    hipLaunchKernelGGL(k_pu_patch_eval, dim3(bx, (unsigned)a.pcap), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pu_blend, dim3(bx), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace rbfsl

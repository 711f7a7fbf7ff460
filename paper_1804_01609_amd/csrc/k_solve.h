#pragma once
// Assembly and solution of the local saddle-point systems (eq. rbf_poly_linsys,
// Sections 2.2, 2.4 and 3.3.2): one workgroup per stencil, the augmented
// M x (M+1) matrix [A~ | b; p(xi)] held in VGPRs, Gaussian elimination with
// partial pivoting, back substitution, cardinal weights w = first n unknowns.
//
// Layout.  The workgroup's 64*W lanes form RR = 64W/CC lane-rows times CC
// lane-columns.  Matrix row i lives in lane-row i; column j lives in
// lane-column j % CC, register slot j / CC (cyclic, so the shrinking trailing
// matrix stays balanced across lane-columns).  Register slots are indexed only
// by compile-time constants: the step loop is unrolled over the slot of the
// pivot column, so "columns right of the pivot" is a static slot range.
//
// Pivoting is implicit: rows never move; a row is marked used once it has been
// a pivot row and is then left alone (its multiplier is 0).  Per step k:
//   1. the lanes owning column k reduce max |a_ik| over unused rows (ties to
//      the lowest row) within each wave, then across waves through LDS;
//   2. r = 1/a_pk; each unused row's multiplier l_i = a_ik * r is broadcast
//      through LDS; the pivot row's entries right of the pivot slot are
//      appended to the U store in LDS (kept for the back substitution);
//   3. every lane updates its slots right of the pivot slot with
//      a_ij = fma(-l_i, u_j, a_ij).
// Each matrix element therefore sees exactly the same sequence of correctly
// rounded operations as in textbook right-looking elimination: the result
// does not depend on the lane layout.
//
// Back substitution: one wave, unknowns from the last one down, each lane
// holding the right-hand sides of two or three pivot rows; z_k = y_k r_k, then
// y_i = fma(-u_ik, z_k, y_i) for the pivot rows of earlier steps.
#include <float.h>

#include <type_traits>
#include <utility>

#include "rbfsl_impl.h"

namespace rbfsl {

template <int B, typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, B + Is>{}), ...);
}
// compile-time loop over B..E-1 (f receives an integral_constant)
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    if constexpr (E > B) sfor_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}

template <int W, int CC, int NC>
struct Cfg {
    static constexpr int NT = 64 * W;
    static constexpr int RR = NT / CC;
    static constexpr int MCAP = (RR < NC * CC - 1) ? RR : NC * CC - 1;
    static constexpr int YT = (MCAP + 63) / 64;  // back-substitution slots per lane
    // offset of step k's pivot-row record in the U store
    static constexpr __host__ __device__ int base(int k) {
        int sk = k / CC, c = k % CC;
        return CC * CC * (sk * NC - sk * (sk - 1) / 2) + c * CC * (NC - sk);
    }
    static constexpr int US = base(MCAP);
};

__device__ __forceinline__ double phs(double r2, int k) {
    double p = sqrt(r2);
    for (int t = 0; t < k; ++t) p = p * r2;
    return p;
}

__device__ __forceinline__ void proj3(double v[3]) {
    double r = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    v[0] = v[0] / r;
    v[1] = v[1] / r;
    v[2] = v[2] / r;
}

// e1: axis with the smallest |c_i| (ties: lowest i), made tangent and unit;
// e2 = c x e1
__device__ __forceinline__ void frame3(const double c[3], double e1[3], double e2[3]) {
    int im = 0;
    double am = fabs(c[0]);
    if (fabs(c[1]) < am) { am = fabs(c[1]); im = 1; }
    if (fabs(c[2]) < am) { am = fabs(c[2]); im = 2; }
    double t = c[im];
#pragma unroll
    for (int i = 0; i < 3; ++i) e1[i] = (i == im) ? (1.0 - t * c[i]) : (0.0 - t * c[i]);
    proj3(e1);
    e2[0] = c[1] * e1[2] - c[2] * e1[1];
    e2[1] = c[2] * e1[0] - c[0] * e1[2];
    e2[2] = c[0] * e1[1] - c[1] * e1[0];
}

__device__ __forceinline__ void local3(const double x[3], const double c[3], const double e1[3],
                                       const double e2[3], double inv_s, double y[3], double &al,
                                       double &be, double &u) {
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = (x[i] - c[i]) * inv_s;
    al = (e1[0] * y[0] + e1[1] * y[1]) + e1[2] * y[2];
    be = (e2[0] * y[0] + e2[1] * y[1]) + e2[2] * y[2];
    double g = (c[0] * y[0] + c[1] * y[1]) + c[2] * y[2];
    u = -(g * inv_s);
}

// basis value number `want` (or all of them into out[]) at (al, be, u):
// m = 0..L, cos (and sin for m>0), i = 0..L-m: H_m^sigma(al,be) u^i
__device__ __forceinline__ double basis_one(int L, double al, double be, double u, int want) {
    int col = 0;
    double hc = 1.0, hs = 0.0, res = 0.0;
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            double nc = al * hc - be * hs;
            double ns = al * hs + be * hc;
            hc = nc;
            hs = ns;
        }
        for (int sg = 0; sg < (m == 0 ? 1 : 2); ++sg) {
            double v = (sg == 0) ? hc : hs;
            for (int i = 0; i <= L - m; ++i) {
                if (col == want) res = v;
                ++col;
                v = v * u;
            }
        }
    }
    return res;
}

__device__ __forceinline__ void basis_all(int L, double al, double be, double u, double *out) {
    int col = 0;
    double hc = 1.0, hs = 0.0;
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            double nc = al * hc - be * hs;
            double ns = al * hs + be * hc;
            hc = nc;
            hs = ns;
        }
        for (int sg = 0; sg < (m == 0 ? 1 : 2); ++sg) {
            double v = (sg == 0) ? hc : hs;
            for (int i = 0; i <= L - m; ++i) {
                out[col++] = v;
                v = v * u;
            }
        }
    }
}

__device__ __forceinline__ double shfl_d(double v, int src) {
    return __shfl(v, src, 64);
}

template <int W, int CC, int NC>
__global__ void __launch_bounds__(64 * W) k_solve(SolveArgs A) {
    using C = Cfg<W, CC, NC>;
    constexpr int NT = C::NT, RR = C::RR, MCAP = C::MCAP;
    __shared__ double us[C::US];     // U store; holds the basis table during assembly
    __shared__ double yb[3 * MCAP];  // scaled local coordinates of the stencil nodes
    __shared__ double lb[2][RR];     // multipliers (double buffered by step parity)
    __shared__ double rinvb[MCAP];
    __shared__ double cval[2][W], csig[2][W];
    __shared__ int crow[2][W];

    __shared__ int skip;
    const int64_t j = blockIdx.x;
    const int t = threadIdx.x;
    // one read for the whole workgroup: this or an earlier step already failed
    if (t == 0) skip = (A.status[ST_FAILSTEP] <= A.step);
    __syncthreads();
    if (skip) return;
    const int lr = t % RR, lc = t / RR;
    const int lane = t & 63, wv = t >> 6;
    const int n = A.n, L = A.L, k = A.k;
    const int mL = (L + 1) * (L + 1);
    const int M = n + mL;

    // ---- stencil, centre, scale, frame ----
    const int64_t row = A.cidx ? (int64_t)A.cidx[j] : j;
    const int32_t *Srow = A.S + row * n;
    const double xe[3] = {A.ex[j], A.ey[j], A.ez[j]};
    double ctr[3];
    if (A.cx) {
        ctr[0] = A.cx[row]; ctr[1] = A.cy[row]; ctr[2] = A.cz[row];
    } else {
        ctr[0] = xe[0]; ctr[1] = xe[1]; ctr[2] = xe[2];
    }
    const double s2 = A.s2[row];
    const double s = (s2 > 0.0) ? sqrt(s2) : 1.0;
    const double inv_s = 1.0 / s;
    double e1[3], e2[3];
    frame3(ctr, e1, e2);
    double yx[3], alx, bex, ux;
    local3(xe, ctr, e1, e2, inv_s, yx, alx, bex, ux);

    // ---- assembly 1: local coordinates and basis table of the stencil nodes ----
    double *Pb = us;  // n x mL basis values (aliases the U store until elimination)
    if (t < n) {
        int g = Srow[t];
        if (g < 0 || (int64_t)g >= A.N) {  // not a node index: flag the stencil, read node 0
            atomicAdd(&A.status[ST_SEARCH], 1);
            atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
            g = 0;
        }
        const double x[3] = {A.nx[g], A.ny[g], A.nz[g]};
        double y[3], al, be, u;
        local3(x, ctr, e1, e2, inv_s, y, al, be, u);
        yb[3 * t] = y[0];
        yb[3 * t + 1] = y[1];
        yb[3 * t + 2] = y[2];
        basis_all(L, al, be, u, Pb + t * mL);
    }
    __syncthreads();

    // ---- assembly 2: my row, my columns ----
    const int i = lr;
    double a[NC];
    double pe_i = 0.0;  // p(xi) entry of rows n..M-1
    if (i >= n && i < M) pe_i = basis_one(L, alx, bex, ux, i - n);
    double yi[3] = {0.0, 0.0, 0.0}, bi = 0.0;
    if (i < n) {
        yi[0] = yb[3 * i]; yi[1] = yb[3 * i + 1]; yi[2] = yb[3 * i + 2];
        double d0 = yi[0] - yx[0], d1 = yi[1] - yx[1], d2 = yi[2] - yx[2];
        bi = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
    }
    sfor<0, NC>([&](auto S) {
        constexpr int sl = S;
        const int jc = lc + CC * sl;
        double v = 0.0;
        if (i < n) {
            if (jc < n) {
                double d0 = yi[0] - yb[3 * jc], d1 = yi[1] - yb[3 * jc + 1], d2 = yi[2] - yb[3 * jc + 2];
                v = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
            } else if (jc < M) {
                v = Pb[i * mL + (jc - n)];
            } else if (jc == M) {
                v = bi;
            }
        } else if (i < M) {
            if (jc < n) v = Pb[jc * mL + (i - n)];
            else if (jc == M) v = pe_i;
        }
        a[sl] = v;
    });
    bool used = (i >= M);
    __syncthreads();  // the basis table is dead from here on

    // ---- elimination ----
    bool fail = false;
    sfor<0, NC>([&](auto SK) {
        constexpr int sk = SK;
        if (fail || sk * CC >= M) return;
        for (int c = 0; c < CC; ++c) {
            const int kk = sk * CC + c;
            if (kk >= M) break;
            const int par = kk & 1;
            // 1. pivot search in column kk
            const bool own = (lc == c);
            const double av = a[sk];
            double cand = (own && !used) ? fabs(av) : -1.0;
            double m = cand;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
            unsigned long long bal = __ballot(cand == m);
            int first = __ffsll((long long)bal) - 1;
            int prow = __shfl(lr, first, 64);
            double psig = shfl_d(av, first);
            if (lane == 0) {
                cval[par][wv] = m;
                csig[par][wv] = psig;
                crow[par][wv] = prow;
            }
            __syncthreads();
            double best = cval[par][0], pval = csig[par][0];
            int p = crow[par][0];
#pragma unroll
            for (int q = 1; q < W; ++q) {
                double v = cval[par][q];
                int r = crow[par][q];
                if (v > best || (v == best && r < p)) {
                    best = v;
                    pval = csig[par][q];
                    p = r;
                }
            }
            if (!(best > 0.0)) {
                fail = true;
                break;
            }
            // 2. multipliers and the pivot row
            if (i == p) used = true;
            const double r = 1.0 / pval;
            if (own) lb[par][i] = used ? 0.0 : av * r;
            const int rb = C::base(kk) + lc * (NC - sk);
            if (i == p) {
                sfor<sk, NC>([&](auto S) {
                    constexpr int sl = S;
                    us[rb + (sl - sk)] = a[sl];
                });
            }
            if (t == 0) rinvb[kk] = r;
            __syncthreads();
            // 3. rank-1 update of the slots right of the pivot slot
            const double l = lb[par][i];
            sfor<sk, NC>([&](auto S) {
                constexpr int sl = S;
                a[sl] = fma(-l, us[rb + (sl - sk)], a[sl]);
            });
        }
    });
    if (fail) {
        if (t == 0) {
            atomicAdd(&A.status[ST_SINGULAR], 1);
            atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
        }
        if (A.st_out && t == 0) A.st_out[j] = RBFSL_E_SINGULAR;
        return;
    }
    __syncthreads();

    // ---- back substitution (wave 0) ----
    if (wv != 0) return;
    double y[C::YT], z[C::YT];
#pragma unroll
    for (int q = 0; q < C::YT; ++q) {
        int kk = lane + 64 * q;
        y[q] = 0.0;
        z[q] = 0.0;
        if (kk < M) {
            int skk = kk / CC;
            y[q] = us[C::base(kk) + (M % CC) * (NC - skk) + (M / CC - skk)];
        }
    }
    for (int kk = M - 1; kk >= 0; --kk) {
        const int q = kk >> 6, src = kk & 63;
        double yk = 0.0;
#pragma unroll
        for (int qq = 0; qq < C::YT; ++qq)
            if (qq == q) yk = shfl_d(y[qq], src);
        const double zk = yk * rinvb[kk];
        const int col_l = kk % CC, col_s = kk / CC;
#pragma unroll
        for (int qq = 0; qq < C::YT; ++qq) {
            int rr = lane + 64 * qq;
            if (qq == q && lane == src) z[qq] = zk;
            if (rr < kk) {
                int srr = rr / CC;
                double u = us[C::base(rr) + col_l * (NC - srr) + (col_s - srr)];
                y[qq] = fma(-u, zk, y[qq]);
            }
        }
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < C::YT; ++q) {
        int aidx = lane + 64 * q;
        if (aidx < n) {
            A.w[j * n + aidx] = z[q];
            if (!isfinite(z[q])) bad = true;
        }
    }
    unsigned long long bb = __ballot(bad);
    if (lane == 0) {
        if (bb) {
            atomicAdd(&A.status[ST_NONFINITE], 1);
            atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
        }
        if (A.st_out) A.st_out[j] = bb ? RBFSL_E_NONFINITE : 0;
    }
}

template <int W, int CC, int NC>
hipError_t launch_solve_variant(const SolveArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_solve<W, CC, NC>), dim3((unsigned)a.count), dim3(64 * W), 0, s, a);
    return hipGetLastError();
}

template <int W, int CC, int NC>
constexpr int variant_mcap() { return Cfg<W, CC, NC>::MCAP; }

}  // namespace rbfsl

#pragma once
// Assembly and solution of the local saddle-point systems (eq. rbf_poly_linsys,
// Sections 2.2, 2.4 and 3.3.2): one workgroup of W waves per stencil, the
// M x M matrix held in VGPRs, Gaussian elimination with partial pivoting,
// back substitution, cardinal weights w = first n unknowns.
//
// Layout.  Matrix row i lives in lane i % 64, row slot i / 64 (R slots).
// Columns are dealt to the waves in blocks of B: column j belongs to block
// g = j / B, owned by wave g % W, at column slot (g / W) * B + j % B.  Each
// wave holds all rows of its columns, so the pivot search of a column is a
// reduction inside one wave.  The right-hand side is kept, identically, in
// every wave.  Register slots are indexed only by compile-time constants.
//
// Elimination (right-looking, blocked, implicit partial pivoting: rows never
// move; a row is marked used once it has been a pivot row and its multiplier
// is 0 from then on).  For each block g of B columns:
//   1. the owner wave factors the panel: for each of its B columns k, the
//      pivot p = the unused row with the largest |a_pk| (ties to the lowest
//      row), r_k = 1/a_pk, multipliers l_ik = a_ik * r_k, and the update of the
//      panel's remaining columns; p, r_k and the l_ik go to LDS;
//   2. one barrier;
//   3. every wave applies the B rank-1 updates, in step order, to its columns
//      right of the panel and to the right-hand side:
//      a_ij = fma(-l_ik, a_pj, a_ij), y_i = fma(-l_ik, y_p, y_i), where a_pj
//      is row p's current value in this wave (it already carries the updates
//      of the earlier steps of the block).
// Every matrix element therefore sees exactly the sequence of correctly
// rounded operations of textbook unblocked right-looking elimination.
//
// Back substitution: unknowns from the last one down (z_k = y_pk r_k, then
// y_i = fma(-u_ik, z_k, y_i) for the rows pivoted before step k), by wave 0,
// with the U columns streamed from the waves through LDS in chunks.
#include <float.h>

#include <type_traits>
#include <utility>

#include "dev_util.h"
#include "rbfsl_impl.h"

namespace rbfsl {

template <int W, int R, int NCB, int B, int WPE_, int CM = 24>
struct Cfg {
    static constexpr int NT = 64 * W;
    static constexpr int ROWS = 64 * R;
    static constexpr int NC = NCB * B;                      // column slots per wave
    static constexpr int NBLK = W * NCB;                    // column blocks
    static constexpr int MCAP = (ROWS < W * NC) ? ROWS : W * NC;
    static constexpr int CSB0 = (CM / (W * B)) > 0 ? (CM / (W * B)) : 1;  // slot-blocks per chunk
    static constexpr int CSB = (CSB0 > NCB) ? NCB : CSB0;
    static constexpr int NCHUNK = (NCB + CSB - 1) / CSB;
    static constexpr int UBN = CSB * W * B * ROWS;          // doubles of one U chunk
    static constexpr int ASM = 4 * MCAP + 8 + (MCAP * MCAP + 3) / 4;  // assembly tables (n*mL <= M^2/4)
    static constexpr int LBN = 2 * B * ROWS;                // panel multipliers, two buffers
    static constexpr int STAGE0 = (UBN > ASM) ? UBN : ASM;
    static constexpr int STAGE = (STAGE0 > LBN) ? STAGE0 : LBN;
    static constexpr int UBW = (NC + 3) & ~1;               // per-wave pivot-row buffer (even)
    // waves per SIMD the kernel is compiled for: the compiler may use
    // 512/WPE VGPRs per lane and must not spill to reach a higher occupancy
    static constexpr int WPE = WPE_;
};

// LDS of one stencil group (W waves).  stage: assembly tables, then the panel
// multipliers (elimination), then the U chunks (back substitution).
template <int W, int R, int NCB, int B, int CM = 24>
struct SolveSmem {
    using C = Cfg<W, R, NCB, B, 1, CM>;
    double stage[C::STAGE];
    double rinvb[C::MCAP];
    double zb[C::MCAP];   // the solution; its first n entries are the weights
    int pivb[C::MCAP];
    int stepb[C::ROWS];   // the step at which each row was the pivot row (16-wave layout)
    int failk[2];         // failing step of a panel, by block parity
};

// One stencil system: node indices S[0..n), evaluation point, centre of the
// local frame, squared scale.  Node indices outside [0, N) are reported in
// status (as a failed search of `step`) and read as node 0.
struct SysIn {
    const double *nx, *ny, *nz;
    int64_t N;
    const int32_t *S;
    double xe[3], ctr[3];
    double s2;
    int n, L, k;
    int *status;
    int64_t step;
};

// Where a factorization goes (factor-only mode): the eliminated matrix,
// column-major M x M with the rows in pivot order (row i at position
// stepof[i]), so that column k holds below position k the values step k
// divided by the pivot and above it U; the pivot row and reciprocal of every
// step, and the step at which every row was pivoted.
struct FactorOut {
    double *F;
    int32_t *piv;
    double *rinv;
    int32_t *stepof;
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

// the (L+1)^2 basis values at (al, be, u): m = 0..L, cos (and sin for m>0),
// i = 0..L-m: H_m^sigma(al,be) u^i with H_m = Re/Im (al + i be)^m
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


// lane value moved by a DPP control (CTRL, row and bank masks); lanes the
// control does not write read 0, the identity of an unsigned maximum
template <int CTRL, int ROWM, int BANKM>
__device__ __forceinline__ unsigned dpp_u(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWM, BANKM, false);
}

// maximum over the wave of 32-bit unsigned values, returned to every lane:
// quad swaps, row shifts, row broadcasts (the classic DPP reduction, each
// stage one v_max_u32 with a DPP operand), then lane 63 holds the result
__device__ __forceinline__ unsigned wave_max_u(unsigned v) {
    v = max(v, dpp_u<0xB1, 0xF, 0xF>(v));   // quad_perm [1,0,3,2]
    v = max(v, dpp_u<0x4E, 0xF, 0xF>(v));   // quad_perm [2,3,0,1]
    v = max(v, dpp_u<0x114, 0xF, 0xE>(v));  // row_shr:4
    v = max(v, dpp_u<0x118, 0xF, 0xC>(v));  // row_shr:8
    v = max(v, dpp_u<0x142, 0xA, 0xF>(v));  // row_bcast:15
    v = max(v, dpp_u<0x143, 0xC, 0xF>(v));  // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// maximum over the wave of doubles that are >= +0 and not NaN: for such
// values the numeric order is the unsigned order of the bit patterns, so the
// high words are reduced first, then the low words of the lanes that hold the
// largest high word
__device__ __forceinline__ double wave_max_nonneg(double v) {
    const unsigned hi = (unsigned)__double2hiint(v), lo = (unsigned)__double2loint(v);
    const unsigned H = wave_max_u(hi);
    const unsigned Lw = wave_max_u(hi == H ? lo : 0u);
    return __hiloint2double((int)H, (int)Lw);
}


// Assembly tables of one system (eq. rbf_poly_linsys in the local graded
// basis): the scaled local coordinates of the stencil nodes (3 x MCAP), the
// evaluation point's (3) and its basis values, and the n x mL basis values of
// the nodes, all in stage; NT threads; the caller puts a barrier between
// filling and reading them.
struct SysTables {
    const double *yb, *yxb, *peb, *Pb;
};
template <int NT, int MCAP>
__device__ __forceinline__ SysTables assembly_tables(double *const stage, const int t, const SysIn &A) {
    const int n = A.n, L = A.L;
    const int mL = (L + 1) * (L + 1);

    // ---- stencil, centre, scale, frame ----
    const int32_t *Srow = A.S;
    const double xe[3] = {A.xe[0], A.xe[1], A.xe[2]};
    const double ctr[3] = {A.ctr[0], A.ctr[1], A.ctr[2]};
    const double s2 = A.s2;
    const double s = (s2 > 0.0) ? sqrt(s2) : 1.0;
    const double inv_s = 1.0 / s;
    double e1[3], e2[3];
    frame3(ctr, e1, e2);

    double *yb = stage;                 // 3 x MCAP scaled local coordinates
    double *yxb = stage + 3 * MCAP;     // evaluation point (3) ...
    double *peb = yxb + 4;              // ... and its basis values (mL <= MCAP)
    double *Pb = peb + MCAP;            // n x mL basis values of the stencil nodes
    for (int a = t; a <= n; a += NT) {
        double x[3];
        if (a < n) {
            int g = Srow[a];
            if (g < 0 || (int64_t)g >= A.N) {  // not a node index: flag the stencil, read node 0
                atomicAdd(&A.status[ST_SEARCH], 1);
                atomicMin(&A.status[ST_FAILSTEP], (int)A.step);
                g = 0;
            }
            x[0] = A.nx[g]; x[1] = A.ny[g]; x[2] = A.nz[g];
        } else {
            x[0] = xe[0]; x[1] = xe[1]; x[2] = xe[2];
        }
        double yl[3], al, be, u;
        local3(x, ctr, e1, e2, inv_s, yl, al, be, u);
        if (a < n) {
            yb[3 * a] = yl[0]; yb[3 * a + 1] = yl[1]; yb[3 * a + 2] = yl[2];
            basis_all(L, al, be, u, Pb + a * mL);
        } else {
            yxb[0] = yl[0]; yxb[1] = yl[1]; yxb[2] = yl[2];
            basis_all(L, al, be, u, peb);
        }
    }
    return SysTables{yb, yxb, peb, Pb};
}

// Entry (i, jc) of the saddle-point matrix, i a row below M whose scaled
// local coordinates are yi (rows i >= n: any); 0 outside M x M
__device__ __forceinline__ double system_entry(const SysTables &tb, int i, int jc, double yi0, double yi1,
                                               double yi2, int n, int M, int mL, int k) {
    double v = 0.0;
    if (i < n) {
        if (jc < n) {
            double d0 = yi0 - tb.yb[3 * jc], d1 = yi1 - tb.yb[3 * jc + 1], d2 = yi2 - tb.yb[3 * jc + 2];
            v = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
        } else if (jc < M) {
            v = tb.Pb[i * mL + (jc - n)];
        }
    } else if (i < M) {
        if (jc < n) v = tb.Pb[jc * mL + (i - n)];
    }
    return v;
}

// Entry i of the right-hand side [b; p(xi)]: the kernel between node i and the
// evaluation point, or the evaluation point's basis value i - n; 0 from M on
__device__ __forceinline__ double system_rhs(const SysTables &tb, int i, double yi0, double yi1, double yi2, int n,
                                             int M, int k) {
    double rhs = 0.0;
    if (i < n) {
        double d0 = yi0 - tb.yxb[0], d1 = yi1 - tb.yxb[1], d2 = yi2 - tb.yxb[2];
        rhs = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
    } else if (i < M) {
        rhs = tb.peb[i - n];
    }
    return rhs;
}

// Assembly of one system: this lane's rows (i = lane + 64 r) of this wave's
// columns go to a, the right-hand side of the same rows to y.
template <int W, int R, int NCB, int B, int CM = 24>
__device__ __forceinline__ void assemble_system(double *const stage, const int t, const SysIn &A,
                                                double (&a)[R][Cfg<W, R, NCB, B, 1, CM>::NC], double (&y)[R]) {
    using C = Cfg<W, R, NCB, B, 1, CM>;
    constexpr int NT = C::NT, MCAP = C::MCAP, NC = C::NC;
    const int lane = t & 63, wv = t >> 6;
    const int n = A.n, L = A.L, k = A.k;
    const int mL = (L + 1) * (L + 1);
    const int M = n + mL;
    const SysTables tb = assembly_tables<NT, MCAP>(stage, t, A);
    __syncthreads();
    sfor<0, R>([&](auto RI) SI {
        constexpr int r = RI;
        const int i = lane + 64 * r;
        double yi0 = 0.0, yi1 = 0.0, yi2 = 0.0;
        if (i < n) { yi0 = tb.yb[3 * i]; yi1 = tb.yb[3 * i + 1]; yi2 = tb.yb[3 * i + 2]; }
        y[r] = system_rhs(tb, i, yi0, yi1, yi2, n, M, k);
        sfor<0, NC>([&](auto S) SI {
            constexpr int sl = S;
            const int jc = ((sl / B) * W + wv) * B + sl % B;
            a[r][sl] = system_entry(tb, i, jc, yi0, yi1, yi2, n, M, mL, k);
        });
    });
}

// Back substitution (after the elimination of solve_system or
// solve_system_df), chunks of CSB slot-blocks from the right: slot-blocks
// [sb1, sb2) of every wave cover columns [sb1*W*B, sb2*W*B); wave 0 holds the
// pivot rows in registers (lane k % 64, slot k / 64) and, for each of its
// rows, the reciprocal of the pivot of the step at which the row was the
// pivot row.  Unknown k is z_k = y_p * r_k with p the pivot row of step k: it
// is formed in row p's lane and broadcast.  A row's y is final once its own
// step is reached, so every unknown is again y_p * r_k at the end, where
// wave 0 writes them all to zb at once.  Ends with a barrier.
template <int W, int R, int NCB, int B, int CM = 24>
__device__ __forceinline__ void back_substitute(double *const stage, const double *const rinvb,
                                                const int *const pivb, double *const zb, const int (&stepof)[R],
                                                const double (&a)[R][Cfg<W, R, NCB, B, 1, CM>::NC],
                                                double (&y)[R], const int t, const int M) {
    using C = Cfg<W, R, NCB, B, 1, CM>;
    constexpr int ROWS = C::ROWS, MCAP = C::MCAP;
    const int lane = t & 63, wv = t >> 6;
    constexpr int KT = (MCAP + 63) / 64;
    int pivr[KT];
    sfor<0, KT>([&](auto TI) SI {
        constexpr int tt = TI;
        const int kk = lane + 64 * tt;
        pivr[tt] = (kk < M) ? pivb[kk] : 0;
    });
    double rrow[R];
    sfor<0, R>([&](auto RI) SI {
        constexpr int r = RI;
        rrow[r] = (stepof[r] < M) ? rinvb[stepof[r]] : 0.0;
    });
    double *UB = stage;
    sfor<0, C::NCHUNK>([&](auto CI) SI {
        constexpr int ch = C::NCHUNK - 1 - CI;
        constexpr int sb1 = ch * C::CSB;
        constexpr int sb2 = (sb1 + C::CSB < NCB) ? sb1 + C::CSB : NCB;
        constexpr int c0 = sb1 * W * B;
        if (c0 >= M) return;  // chunk lies beyond the last column
        __syncthreads();      // previous chunk consumed
        sfor<sb1 * B, sb2 * B>([&](auto S) SI {
            constexpr int sl = S;
            const int col = ((sl / B) * W + wv) * B + sl % B - c0;
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                UB[col * ROWS + lane + 64 * r] = a[r][sl];
            });
        });
        __syncthreads();
        if (wv == 0) {
            const int khi = (sb2 * W * B < M) ? sb2 * W * B : M;
            double un[R];
            sfor<0, R>([&](auto RI) SI { un[RI] = UB[(khi - 1 - c0) * ROWS + lane + 64 * RI]; });
            for (int kk = khi - 1; kk >= c0; --kk) {
                double u[R];
                sfor<0, R>([&](auto RI) SI { u[RI] = un[RI]; });
                const int kn = (kk > c0) ? kk - 1 : c0;
                sfor<0, R>([&](auto RI) SI { un[RI] = UB[(kn - c0) * ROWS + lane + 64 * RI]; });
                const int kl = kk & 63, kt = kk >> 6;
                // pivot row of step kk (register slot kt, lane kl)
                int pk = __builtin_amdgcn_readlane(pivr[0], kl);
                sfor<1, KT>([&](auto TI) SI {
                    constexpr int tt = TI;
                    const int pt = __builtin_amdgcn_readlane(pivr[tt], kl);
                    pk = (kt == tt) ? pt : pk;
                });
                const int pl = pk & 63, pr = pk >> 6;
                double ysel = y[0], rsel = rrow[0];
                sfor<1, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    ysel = (pr == r) ? y[r] : ysel;
                    rsel = (pr == r) ? rrow[r] : rsel;
                });
                const double zk = bcast_d(ysel * rsel, pl);
                sfor<0, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    const double yn = fma(-u[r], zk, y[r]);
                    y[r] = (stepof[r] < kk) ? yn : y[r];
                });
            }
        }
    });
    if (wv == 0) {
        sfor<0, R>([&](auto RI) SI {
            constexpr int r = RI;
            if (stepof[r] < M) zb[stepof[r]] = y[r] * rrow[r];
        });
    }
    __syncthreads();
}

// Assembles and solves one system with the W waves of a stencil group;
// t = thread index inside the group (0 .. 64W-1), block-wide barriers.
// Returns false when elimination met a column with no usable pivot (the
// system is singular to working precision); else the solution is in sh.zb.
// LOCK: several groups of one workgroup run this in lockstep on systems of
// the same size, so every group passes every barrier: a singular group keeps
// going (on values that are then discarded) instead of leaving early.
template <int W, int R, int NCB, int B, bool LOCK, int CM = 24, bool FACT = false>
__device__ __forceinline__ bool solve_system(SolveSmem<W, R, NCB, B, CM> &sh, const int t, const SysIn &A,
                                             const FactorOut *fo = nullptr) {
    using C = Cfg<W, R, NCB, B, 1, CM>;
    constexpr int NT = C::NT, ROWS = C::ROWS, MCAP = C::MCAP, NC = C::NC;
    // the 16-wave layout (M <= 192) records each row's pivot step once after
    // the elimination instead of in every wave at every step (1% of its time;
    // the layouts near their register limit keep the per-step form)
    constexpr bool LATE = (R >= 3 && W >= 16);
    double *const stage = sh.stage;
    double *const rinvb = sh.rinvb;
    double *const zb = sh.zb;
    int *const pivb = sh.pivb;
    int *const failk = sh.failk;
    double(*lb)[B][ROWS] = reinterpret_cast<double(*)[B][ROWS]>(stage);  // [2][B][ROWS]
    constexpr int NOFAIL = 0x7fffffff;

    const int lane = t & 63, wv = t >> 6;
    if (t == 0) {  // read after the assembly barriers
        failk[0] = NOFAIL;
        failk[1] = NOFAIL;
    }

    const int n = A.n, L = A.L;
    const int mL = (L + 1) * (L + 1);
    const int M = n + mL;
    double a[R][NC];
    double y[R];
    assemble_system<W, R, NCB, B, CM>(stage, t, A, a, y);
    bool used[R];
    int stepof[R];
    sfor<0, R>([&](auto RI) SI {
        used[RI] = (lane + 64 * RI >= M);
        stepof[RI] = MCAP;
    });

    __syncthreads();  // the assembly tables are dead; stage now holds multipliers

    // ---- elimination, one block of B columns at a time ----
    // The block loop is a runtime loop (the code must fit the instruction
    // cache); per block, a runtime slot-block index is dispatched once to code
    // whose register slots are all static.
    // factor panel g (its owner wave only; panel = slot-block PSB): pivots,
    // reciprocals and multipliers of the panel's columns, in-panel updates
    auto factor = [&](auto PSBC, int g) SI {
        constexpr int PSB = PSBC;
        constexpr int ps0 = PSB * B;
        const int k0 = g * B;
        const int cnt = (k0 + B < M) ? B : M - k0;
        bool stop = false;
        sfor<0, B>([&](auto CI) SI {
            constexpr int c = CI;
            if (c >= cnt || stop) return;
            const int kk = k0 + c;
            double best = 0.0;  // NaN entries never win (v > best is false)
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                const double v = fabs(a[r][ps0 + c]);
                if (!used[r] && v > best) best = v;
            });
            const double m = wave_max_nonneg(best);
            if (!(m > 0.0)) {
                if (lane == 0) failk[g & 1] = kk;
                stop = true;
                return;
            }
            const double rm = 1.0 / m;  // |pivot| = m: the reciprocal can start now
            int p = -1;
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                const unsigned long long msk = __ballot(!used[r] && fabs(a[r][ps0 + c]) == m);
                if (p < 0 && msk) p = 64 * r + __ffsll((long long)msk) - 1;
            });
            const int pl = p & 63, pr = p >> 6;
            double pvsel = a[0][ps0 + c];
            sfor<1, R>([&](auto RI) SI {
                constexpr int r = RI;
                pvsel = (pr == r) ? a[r][ps0 + c] : pvsel;
            });
            const double pv = bcast_d(pvsel, pl);
            const double rinv = (pv < 0.0) ? -rm : rm;  // = 1 / pv exactly
            double l[R];
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                if (pr == r && lane == pl) { used[r] = true; if constexpr (!LATE) stepof[r] = kk; }
                l[r] = used[r] ? 0.0 : a[r][ps0 + c] * rinv;
                lb[g & 1][c][lane + 64 * r] = l[r];
            });
            if (lane == 0) {
                pivb[kk] = p;
                rinvb[kk] = rinv;
            }
            sfor<c + 1, B>([&](auto CC) SI {
                constexpr int cc = CC;
                double usel = a[0][ps0 + cc];
                sfor<1, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    usel = (pr == r) ? a[r][ps0 + cc] : usel;
                });
                const double u = bcast_d(usel, pl);
                sfor<0, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    a[r][ps0 + cc] = fma(-l[r], u, a[r][ps0 + cc]);
                });
            });
        });
    };
    // apply the rank-1 updates of block g's steps, in step order, to this
    // wave's slots S0 .. NC-1 and mark the pivot rows as used.  Row p's
    // entries reach every lane by readlane.  Only wave 0 carries the
    // right-hand side (the back substitution is its alone).
    auto upd = [&](auto S0C, auto S1C, int g, int cnt) SI {
        constexpr int S0 = S0C, S1 = S1C;
        const bool doY = (wv == 0);
        const int k0 = g * B;
        for (int c = 0; c < cnt; ++c) {
            const int kk = k0 + c;
            const int p = pivb[kk];
            const int pl = p & 63, pr = p >> 6;
            double l[R];
            sfor<0, R>([&](auto RI) SI { l[RI] = lb[g & 1][c][lane + 64 * RI]; });
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                if (pr == r && lane == pl) { used[r] = true; if constexpr (!LATE) stepof[r] = kk; }
            });
            sfor<0, R>([&](auto PRI) SI {
                constexpr int prr = PRI;
                if (pr == prr) {
                    sfor<S0, S1>([&](auto S) SI {
                        constexpr int sl = S;
                        const double u = bcast_d(a[prr][sl], pl);
                        sfor<0, R>([&](auto RI) SI {
                            constexpr int r = RI;
                            a[r][sl] = fma(-l[r], u, a[r][sl]);
                        });
                        // keep each broadcast next to its use (the scheduler would
                        // otherwise hoist them all and run out of registers)
                        if constexpr ((sl - S0) % 4 == 3) __builtin_amdgcn_sched_barrier(0);
                    });
                    if (doY) {
                        const double yp = bcast_d(y[prr], pl);
                        sfor<0, R>([&](auto RI) SI {
                            constexpr int r = RI;
                            y[r] = fma(-l[r], yp, y[r]);
                        });
                    }
                }
            });
        }
    };
    bool dead = false;
    // blocks g = sb * W + ow: the slot-block sb is a compile-time loop, the
    // owner wave ow a runtime loop, so every register slot stays static
    sfor<0, NCB>([&](auto SBC) SI {
        constexpr int sb = SBC;
        for (int ow = 0; ow < W; ++ow) {
            const int g = sb * W + ow;
            const int k0 = g * B;
            if ((!LOCK && dead) || k0 >= M) break;
            if (wv == ow) {
                __builtin_amdgcn_s_setprio(2);
                factor(SBC, g);
                __builtin_amdgcn_s_setprio(0);
            }
            __syncthreads();
            const int fa = failk[g & 1];
            const int kend = (k0 + B < M) ? k0 + B : M;
            const int cnt = ((kend < fa) ? kend : fa) - k0;
            if (wv > ow) upd(std::integral_constant<int, sb * B>{}, std::integral_constant<int, NC>{}, g, cnt);
            else upd(std::integral_constant<int, (sb + 1) * B>{}, std::integral_constant<int, NC>{}, g, cnt);
            dead = dead || (fa != NOFAIL);
        }
    });
    if (!LOCK && dead) return false;
    if constexpr (LATE) {  // the step at which each row was pivoted, from the pivot list
        int *const stepb = sh.stepb;
        for (int i = t; i < C::ROWS; i += NT) stepb[i] = MCAP;
        __syncthreads();
        for (int kk = t; kk < M; kk += NT) stepb[pivb[kk]] = kk;
        __syncthreads();
        sfor<0, R>([&](auto RI) SI { stepof[RI] = stepb[lane + 64 * RI]; });
    }

    if constexpr (FACT) {
        // factor-only mode: store the factorization instead of solving
        sfor<0, NC>([&](auto S) SI {
            constexpr int sl = S;
            const int jc = ((sl / B) * W + wv) * B + sl % B;
            if (jc < M) {
                sfor<0, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    const int i = lane + 64 * r;
                    if (i < M) fo->F[(int64_t)jc * M + stepof[r]] = a[r][sl];
                });
            }
        });
        if (wv == 0) {
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                const int i = lane + 64 * r;
                if (i < M) fo->stepof[i] = stepof[r];
            });
        }
        for (int kk = t; kk < M; kk += NT) {
            fo->piv[kk] = pivb[kk];
            fo->rinv[kk] = rinvb[kk];
        }
        return true;
    }

    back_substitute<W, R, NCB, B, CM>(stage, rinvb, pivb, zb, stepof, a, y, t, M);

    return !dead;
}

// The solver's LDS.  With OPQ the base address is made opaque to the
// compiler (an offset of zero that it cannot see through): with a constant
// base it precomputes the per-slot LDS addresses of the largest variant and
// keeps them all live, which pushes matrix registers to scratch.
template <class SM, bool OPQ>
__device__ __forceinline__ SM &solver_smem(unsigned char *raw) {
    if constexpr (OPQ) {
        int zero = 0;
        __asm__ volatile("" : "+v"(zero));
        return *reinterpret_cast<SM *>(raw + zero);
    } else {
        return *reinterpret_cast<SM *>(raw);
    }
}

// One workgroup of W waves per stencil (plain path): weights to w, failures
// counted in status.
template <int W, int R, int NCB, int B, int WPE, bool OPQ = false>
__global__ void __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(WPE, WPE))) k_solve(SolveArgs A) {
    __shared__ __attribute__((aligned(16))) unsigned char sh_raw[sizeof(SolveSmem<W, R, NCB, B>)];
    SolveSmem<W, R, NCB, B> &sh = solver_smem<SolveSmem<W, R, NCB, B>, OPQ>(sh_raw);
    __shared__ int skip;
    const int64_t j = blockIdx.x;
    const int t = threadIdx.x;
    constexpr int NT = 64 * W;
    const int64_t step = A.step + (A.step_count ? j / A.step_count : 0);
    // one read for the whole workgroup: this or an earlier step already failed
    if (t == 0) skip = (A.status[ST_FAILSTEP] <= step);
    __syncthreads();
    if (skip) return;
    const int n = A.n;
    const int64_t row = A.cidx ? (int64_t)A.cidx[j] : j;
    SysIn in;
    in.nx = A.nx; in.ny = A.ny; in.nz = A.nz; in.N = A.N;
    in.S = A.S + row * n;
    in.xe[0] = A.ex[j]; in.xe[1] = A.ey[j]; in.xe[2] = A.ez[j];
    if (A.cx) {
        in.ctr[0] = A.cx[row]; in.ctr[1] = A.cy[row]; in.ctr[2] = A.cz[row];
    } else {
        in.ctr[0] = in.xe[0]; in.ctr[1] = in.xe[1]; in.ctr[2] = in.xe[2];
    }
    in.s2 = A.s2[row];
    in.n = n; in.L = A.L; in.k = A.k;
    in.status = A.status; in.step = step;
    if (!solve_system<W, R, NCB, B, false>(sh, t, in)) {
        if (t == 0) {
            atomicAdd(&A.status[ST_SINGULAR], 1);
            atomicMin(&A.status[ST_FAILSTEP], (int)step);
            if (A.st_out) A.st_out[j] = RBFSL_E_SINGULAR;
        }
        return;
    }
    // ---- weights ----
    bool bad = false;
    for (int aidx = t; aidx < n; aidx += NT) {
        const double z = sh.zb[aidx];
        A.w[j * n + aidx] = z;
        if (!isfinite(z)) bad = true;
    }
    const int anybad = __syncthreads_or(bad ? 1 : 0);
    if (t == 0) {
        if (anybad) {
            atomicAdd(&A.status[ST_NONFINITE], 1);
            atomicMin(&A.status[ST_FAILSTEP], (int)step);
        }
        if (A.st_out) A.st_out[j] = anybad ? RBFSL_E_NONFINITE : 0;
    }
}

// One workgroup per stencil: assemble and eliminate, store the factorization
// (row t of FactorArgs' arrays) instead of solving; fstat[t] = 0, or
// RBFSL_E_SINGULAR when the system has no usable pivot.
template <int W, int R, int NCB, int B, int WPE, bool OPQ = false>
__global__ void __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(WPE, WPE))) k_factor(FactorArgs FA) {
    __shared__ __attribute__((aligned(16))) unsigned char sh_raw[sizeof(SolveSmem<W, R, NCB, B>)];
    SolveSmem<W, R, NCB, B> &sh = solver_smem<SolveSmem<W, R, NCB, B>, OPQ>(sh_raw);
    const SolveArgs &A = FA.s;
    const int64_t j = blockIdx.x;
    const int t = threadIdx.x;
    // slots sized for the largest system; this system has nvar[row] nodes
    const int M = A.n + (A.L + 1) * (A.L + 1);
    const int64_t row = A.cidx ? (int64_t)A.cidx[j] : j;
    const int n = A.nvar ? A.nvar[row] : A.n;
    SysIn in;
    in.nx = A.nx; in.ny = A.ny; in.nz = A.nz; in.N = A.N;
    in.S = A.S + row * (A.sstride ? A.sstride : (int64_t)A.n);
    in.xe[0] = A.ex[j]; in.xe[1] = A.ey[j]; in.xe[2] = A.ez[j];
    if (A.cx) {
        in.ctr[0] = A.cx[row]; in.ctr[1] = A.cy[row]; in.ctr[2] = A.cz[row];
    } else {
        in.ctr[0] = in.xe[0]; in.ctr[1] = in.xe[1]; in.ctr[2] = in.xe[2];
    }
    in.s2 = A.s2[row];
    in.n = n; in.L = A.L; in.k = A.k;
    in.status = A.status; in.step = A.step;
    FactorOut fo;
    fo.F = FA.F + j * (int64_t)M * M;
    fo.piv = FA.piv + j * M;
    fo.rinv = FA.rinv + j * M;
    fo.stepof = FA.stepof + j * M;
    const bool ok = solve_system<W, R, NCB, B, false, 24, true>(sh, t, in, &fo);
    if (t == 0) FA.fstat[j] = ok ? 0 : RBFSL_E_SINGULAR;
}

template <int W, int R, int NCB, int B, int WPE, bool OPQ = false>
hipError_t launch_factor_variant(const FactorArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_factor<W, R, NCB, B, WPE, OPQ>), dim3((unsigned)a.s.count), dim3(64 * W), 0, s, a);
    return hipGetLastError();
}

template <int W, int R, int NCB, int B, int WPE, bool OPQ = false>
hipError_t launch_solve_variant(const SolveArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_solve<W, R, NCB, B, WPE, OPQ>), dim3((unsigned)a.count), dim3(64 * W), 0, s, a);
    return hipGetLastError();
}

template <int W, int R, int NCB, int B>
constexpr int variant_mcap() { return Cfg<W, R, NCB, B, 1>::MCAP; }

}  // namespace rbfsl

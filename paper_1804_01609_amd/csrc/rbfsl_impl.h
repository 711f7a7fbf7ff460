// Internal declarations shared by the HIP kernels and the host API.
//
// Floating-point contract: everything is compiled with -ffp-contract=off, so
// every expression rounds exactly as written; fused multiply-adds appear only
// as explicit fma() calls.  Sums are written with their association made
// explicit.  This fixes the result of every step bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbfsl.h"

namespace rbfsl {

// Velocity coefficients at one time: u(x) = c R u0(R^T x) + w x x.
struct VelCoef {
    double c;
    double R[9];  // row-major
    double w[3];
    double cw, sw;  // NL2010 flow: cos and sin of (2 pi/T) t
};

// Everything one step's tracer needs: the velocity coefficients at the stage
// times (RK4: t_{m+1}, t_{m+1} - dt/2, t_m; RK5: t_{m+1} + c_s h, s = 0..5)
// and the step h = -dt with RK4's fractions of it.
struct StepCoef {
    VelCoef v[6];
    double h, hh, h6;
    int vel_id;
    int rk;  // RBFSL_RK4 or RBFSL_RK5_FEHLBERG
};

// Fehlberg's fifth-order formula (Section 3.2): stage fractions c_s of the
// step, stage coefficients a_sj and fifth-order weights b_j, each written as
// the rational number it is (folded to the nearest double at compile time).
constexpr double kRk5C[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
struct Rk5Tableau {
    double a[6][5];
    double b[6];
};
constexpr Rk5Tableau kRk5 = {
    {{0.0, 0.0, 0.0, 0.0, 0.0},
     {1.0 / 4.0, 0.0, 0.0, 0.0, 0.0},
     {3.0 / 32.0, 9.0 / 32.0, 0.0, 0.0, 0.0},
     {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0.0, 0.0},
     {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0.0},
     {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}},
    {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0}};

// Spatial hash over the cube [-1,1]^3 with G cells per axis.
struct Grid {
    int G = 0;
    double invh = 0.0;   // G / 2
    double R0 = 0.0;     // first search radius for n-point stencils
    int *cell_start = nullptr;  // G^3 + 1 offsets into the cell-sorted arrays
    double *sx = nullptr, *sy = nullptr, *sz = nullptr;  // cell-sorted coordinates
    int *perm = nullptr;        // cell-sorted position -> node index
};

// Device status words of a run.
enum { ST_SINGULAR = 0, ST_NONFINITE = 1, ST_SEARCH = 2, ST_FAILSTEP = 3, ST_WORDS = 4 };
constexpr int NO_FAIL = 0x7fffffff;

// kNN capacity: candidates kept per query inside the search ball; searches
// for n <= KNN_SMALL_N / 2 keep a quarter of it, for n <= KNN_SMALL_N half.
constexpr int KNN_CAP = 1024;
constexpr int KNN_SMALL_N = 256;
constexpr int MAX_SYSTEM = 192;

// ---- launchers (return hipSuccess or the launch error) ----
hipError_t launch_trace(const double *nx, const double *ny, const double *nz, int64_t N,
                        const StepCoef &sc, double *ex, double *ey, double *ez,
                        const int *status, int64_t step, hipStream_t s);
// the departure points of steps m0 .. m0 + K - 1 (sc: K device coefficients),
// step s's to ex[s N ..]
hipError_t launch_trace_steps(const double *nx, const double *ny, const double *nz, int64_t N,
                              const StepCoef *sc, int K, double *ex, double *ey, double *ez,
                              const int *status, int64_t m0, hipStream_t s);

hipError_t grid_build(const double *nx, const double *ny, const double *nz, int64_t N, int n,
                      Grid *g, hipStream_t s);
// grid size, cell scale and first search radius for N nodes and n-point stencils
void grid_dims(int64_t N, int n, int *G, double *invh, double *R0);
// build into caller-owned arrays (g->G, invh, R0 and all pointers set;
// cell: N ints, count: G^3 ints of scratch); enqueued only, no synchronisation
hipError_t grid_build_in(const double *nx, const double *ny, const double *nz, int64_t N, Grid *g,
                         int *cell, int *count, hipStream_t s);
void grid_free(Grid *g);

// n nearest nodes of Q query points (SoA qx,qy,qz).  idx: Q x n; d2: Q x n or
// null; s2: Q (squared distance of the n-th neighbour) or null.
hipError_t launch_knn(const Grid &g, int64_t N, const double *qx, const double *qy,
                      const double *qz, int64_t Q, int n, int32_t *idx, double *d2, double *s2,
                      int *status, int64_t step, hipStream_t s, int64_t per = 0);
// (per > 0: the queries of consecutive steps step, step + 1, ..., per each)

// Weights of `count` stencils.  Stencil t uses node indices S[row(t)*n..],
// squared scale s2[row(t)], centre c[row(t)] (or its own evaluation point when
// no centres are given) and evaluation point t; row(t) = cidx ? cidx[t] : t.
struct SolveArgs {
    const double *nx, *ny, *nz;
    int64_t N;                   // node count (stencil indices are checked against it)
    const double *ex, *ey, *ez;  // evaluation points (departure points)
    const double *cx, *cy, *cz;  // stencil centres by row; null: centre = evaluation point
    const int32_t *S;
    const double *s2;
    const int32_t *cidx;         // row of stencil t; null: row = t
    int64_t count;
    int n, L, k;
    double *w;                   // count x n
    int32_t *st_out;             // optional per-stencil status
    int *status;
    int64_t step;
    int64_t step_count;          // > 0: stencils of consecutive steps, step_count per step
    // factor-only use with stencils of different sizes (RBF-PU patches):
    // stencil t has nvar[row(t)] <= n nodes, stored with row stride sstride
    // (null / 0: every stencil has n nodes, stride n)
    const int32_t *nvar;
    int64_t sstride;
};
hipError_t launch_solve(const SolveArgs &a, hipStream_t s);

// Factorizations of `count` systems (as SolveArgs describes them), stored
// for reuse: system t's eliminated matrix (column-major M x M), pivot rows,
// reciprocals and the step at which each row was pivoted; fstat[t] = 0 or
// RBFSL_E_SINGULAR.
struct FactorArgs {
    SolveArgs s;
    double *F;        // count x M x M (M = s.n + (L+1)^2: the largest system;
                      // a smaller one is stored column-major in its slot's start)
    int32_t *piv;     // count x M
    double *rinv;     // count x M
    int32_t *stepof;  // count x M
    int32_t *fstat;   // count
};
hipError_t launch_factor(const FactorArgs &a, hipStream_t s);

// Weights from stored factorizations (the paper's centre-point stencils,
// Section 3.3.2): for each evaluation point j, the system of centre node
// cidx[j] (stencil S[cidx[j]], scale s2[cidx[j]]) with the right-hand side
// [phi(|y_a - y_xi|); p(xi)] of xi_j, replayed through the stored
// elimination and back substitution.  w: count x n.
struct CachedArgs {
    const double *nx, *ny, *nz;
    int64_t N;
    const double *ex, *ey, *ez;
    const int32_t *S, *cidx;
    const double *s2;
    const double *F, *rinv;
    const int32_t *piv, *stepof, *fstat;
    int64_t count;
    int n, L, k;
    double *w;
    int *status;
    int64_t step;
};
hipError_t launch_solve_cached(const CachedArgs &a, hipStream_t s);
int solve_variant_capacity(int M);  // capacity of the variant chosen for M (0: unsupported)

// RBF-PU (Sections 2.3 and 3.3.3).  Patch l holds the cnt[l] nodes
// pidx[l*ncap ..] (its stencil, in (d^2, index) order), its system factored
// as FactorArgs stores it (slots of Mmax = nmax + (L+1)^2), centre c[l],
// squared radius R2.
struct PuArgs {
    const double *nx, *ny, *nz;
    int64_t N;
    const double *cx, *cy, *cz;  // patch centres
    int64_t Mp;                  // patch count
    double R, R2;                // radius, R * R
    const int32_t *pidx;         // Mp x ncap node lists
    const double *pd2;           // Mp x ncap squared distances (counting only)
    const int32_t *cnt;          // Mp node counts
    double *ploc;                // Mp x ncap x 3: the nodes' local coordinates in their patch's frame
    int ncap, nmax, L, k, ntr;
    const double *F, *rinv;
    const int32_t *stepof, *fstat;
    double *coef;                // Mp x ntr x Mmax: [c; d] of every patch and tracer
    // departure points and the patches that contain them
    const double *ex, *ey, *ez;
    int32_t *sidx;               // N x pcap patch indices, (d^2, l) order
    double *sd2;                 // N x pcap squared distances (+inf past the last)
    int pcap;
    const double *qin;           // ntr x N
    double *qout;                // ntr x N
    double *sval;                // pcap x ntr x N: each containing patch's value
    int *status;
    int64_t step;
};
// node counts of the patches (d^2 < R2 among the ncap nearest); a full
// list, a count over nmax_allowed or an empty patch is reported in status
// as a failed search; *nmax (device int) receives the largest count
hipError_t launch_pu_count(const PuArgs &a, int nmax_allowed, int32_t *cnt, int *nmax, hipStream_t s);
// the patches containing each departure point (d^2 < R2), through the
// spatial hash of the centres `cg`; more than pcap is a failed search
hipError_t launch_pu_search(const PuArgs &a, const Grid &cg, hipStream_t s);
// the local coordinates of every patch's nodes (fixed: computed at create)
hipError_t launch_pu_local(const PuArgs &a, hipStream_t s);
// every patch's coefficients for every tracer, from the stored factorizations
hipError_t launch_pu_coef(const PuArgs &a, hipStream_t s);
// q at the departure points: the B-spline partition of unity over the
// patches that contain each point (eq. PU_interp)
hipError_t launch_pu_eval(const PuArgs &a, hipStream_t s);

hipError_t launch_apply(const double *w, const int32_t *S, const int32_t *cidx, int64_t N, int n,
                        int ntr, const double *qin, double *qout, const int *status,
                        int64_t step, hipStream_t s);
hipError_t launch_status_reset(int *status, hipStream_t s);

// ---- host helpers shared by the single-run and the pooled API (api.hip) ----
// validated (n, L, k) of a parameter set for N nodes; RBFSL_E_INVAL with a
// message otherwise
int validate_params(int64_t N, const rbfsl_params *p, int *L, int *k, char *msg, size_t msz);
// validated (n, L, k) alone (L = -1 / k = -1 select the paper's rule)
int resolve_stencil(int64_t N, int n, int L, int k, int *Lo, int *ko, char *msg, size_t msz);
StepCoef step_coef(const rbfsl_params &p, int64_t m);  // p with resolved L, k
// N x 3 AoS (host or device) -> SoA device arrays, through `tmp` (3N doubles)
hipError_t upload_points_via(const double *xyz, int64_t N, int on_device, double *x, double *y,
                             double *z, double *tmp, hipStream_t s);

}  // namespace rbfsl

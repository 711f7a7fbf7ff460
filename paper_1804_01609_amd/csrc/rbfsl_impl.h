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
};

// Everything one step's tracer needs: coefficients at t_{m+1}, the midpoint
// t_{m+1} - dt/2 and t_m, and the RK4 step fractions of h = -dt.
struct StepCoef {
    VelCoef c1, ch, c0;
    double h, hh, h6;
    int vel_id;
};

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

// kNN capacity: candidates kept per query inside the search ball.
constexpr int KNN_CAP = 1024;
constexpr int MAX_SYSTEM = 192;

// ---- launchers (return hipSuccess or the launch error) ----
hipError_t launch_trace(const double *nx, const double *ny, const double *nz, int64_t N,
                        const StepCoef &sc, double *ex, double *ey, double *ez,
                        const int *status, int64_t step, hipStream_t s);

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
                      int *status, int64_t step, hipStream_t s);

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
};
hipError_t launch_solve(const SolveArgs &a, hipStream_t s);
int solve_variant_capacity(int M);  // capacity of the variant chosen for M (0: unsupported)

hipError_t launch_apply(const double *w, const int32_t *S, const int32_t *cidx, int64_t N, int n,
                        int ntr, const double *qin, double *qout, const int *status,
                        int64_t step, hipStream_t s);

hipError_t launch_status_reset(int *status, hipStream_t s);

// ---- host helpers shared by the single-run and the pooled API (api.hip) ----
// validated (n, L, k) of a parameter set for N nodes; RBFSL_E_INVAL with a
// message otherwise
int validate_params(int64_t N, const rbfsl_params *p, int *L, int *k, char *msg, size_t msz);
StepCoef step_coef(const rbfsl_params &p, int64_t m);  // p with resolved L, k
// N x 3 AoS (host or device) -> SoA device arrays, through `tmp` (3N doubles)
hipError_t upload_points_via(const double *xyz, int64_t N, int on_device, double *x, double *y,
                             double *z, double *tmp, hipStream_t s);

}  // namespace rbfsl

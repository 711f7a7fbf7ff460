/*
 * rbfsl.h -- C ABI of the MI355X (gfx950) local-stencil RBF semi-Lagrangian
 * transport library.
 *
 * The method is the local RBF interpolation scheme of Shankar & Wright,
 * "Mesh-free semi-Lagrangian methods for transport on a sphere using radial
 * basis functions" (arXiv:1804.01609):
 *   - Algorithm 1 (Section 3): each step traces every Eulerian node x_j back
 *     to its departure point xi_j and sets q^{m+1}_j = s(xi_j);
 *   - Section 3.2: the departure point solves the trajectory ODE (eq. sl_ode)
 *     backward over one step, here with RK4 and an orthogonal projection onto
 *     the sphere at every stage;
 *   - Sections 2.2 and 3.3.2: s is the augmented local interpolant (eq.
 *     rbf_poly) on an n-node stencil, with PHS phi(r) = r^(2k+1) and the
 *     spherical harmonics of degree <= L (Section 2.4), whose coefficients
 *     solve the saddle-point system (eq. rbf_poly_linsys) by LU with partial
 *     pivoting.
 *
 * Every step runs on the GPU in hand-written HIP kernels; the host only
 * evaluates the time-dependent coefficients of the velocity field (cosines and
 * sines of the stage times) and enqueues work.
 *
 * Conventions for every function below:
 *   - all return an int status (RBFSL_OK or a negative RBFSL_E_* code) unless
 *     stated; none throws, aborts or returns memory the caller must free;
 *   - arrays are plain pointers; a flag `*_on_device` says whether a pointer
 *     is device memory (HIP/torch allocation on the context's device) or host
 *     memory; inputs are copied, the caller keeps ownership;
 *   - work is enqueued on the context's HIP stream (NULL = the default
 *     stream); functions that return data to the caller synchronise that
 *     stream first;
 *   - a context is used by one host thread at a time; different contexts are
 *     independent.
 */
#ifndef RBFSL_H
#define RBFSL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbfsl_ctx rbfsl_ctx; /* opaque; owns all of its device buffers */

enum {
    RBFSL_OK = 0,
    RBFSL_E_INVAL = -1,     /* invalid argument or parameter combination */
    RBFSL_E_NOMEM = -2,     /* a device or host allocation failed */
    RBFSL_E_DEVICE = -3,    /* a HIP runtime call failed */
    RBFSL_E_SINGULAR = -4,  /* a stencil system had a zero pivot (e.g. duplicate nodes) */
    RBFSL_E_NONFINITE = -5, /* a stencil produced non-finite weights */
    RBFSL_E_STATE = -6,     /* call not valid in the current state (e.g. q not set) */
    RBFSL_E_SEARCH = -7,    /* the neighbour search could not bound a stencil */
    RBFSL_E_BUDGET = -8,    /* a pool has no free run slot or HBM for the run */
    RBFSL_E_CAPACITY = -9   /* input larger than rbfsl_weights_noalloc's fixed scratch */
};

/* Velocity fields u(x,t) (tangent to the sphere, divergence free).
 * vel[0] = T (period), vel[1..3] = unit axis a, vel[4] = amplitude kappa.
 *   ZERO:       u = 0
 *   SOLID_BODY: u = (2 pi/T) a x x                       (Section 4.1)
 *   DEFORM:     u = x x grad psi + (2 pi/T) a x x with
 *               psi = kappa cos(pi t/T) psi0(R(t)^T x), psi0 = xyz + z^2 x/2,
 *               R(t) the rotation about a by 2 pi t/T; the flow reverses and
 *               every parcel returns to its start at t = T.
 *   NL2010:     the deformational flow of Section 4.2 (vel[0] = T only):
 *               u_lambda = (10/T) cos(pi t/T) sin^2(lambda') sin(2 theta)
 *                          + (2 pi/T) cos(theta),
 *               u_theta  = (10/T) cos(pi t/T) sin(2 lambda') cos(theta),
 *               lambda' = lambda - 2 pi t/T, evaluated in Cartesian form. */
enum { RBFSL_VEL_ZERO = 0, RBFSL_VEL_SOLID_BODY = 1, RBFSL_VEL_DEFORM = 2, RBFSL_VEL_NL2010 = 3 };

/* Departure-point integrators (Section 3.2): classical RK4, or Fehlberg's
 * fifth-order formula; every stage point and the result are projected onto
 * the sphere. */
enum { RBFSL_RK4 = 0, RBFSL_RK5_FEHLBERG = 1 };

typedef struct {
    int32_t n;            /* stencil size, 1 <= n <= N                                    */
    int32_t L;            /* harmonic degree; -1 selects L = floor((sqrt(n)-1)/2) (Sec 2.4) */
    int32_t k;            /* PHS order, phi = r^(2k+1), 0 <= k <= L; -1 selects k = L      */
    int32_t stencil_mode; /* 0: n nearest nodes of xi_j, centred at xi_j;
                             1: the paper's centre-point stencils: the n nearest nodes
                                of the node nearest to xi_j (Section 3.3.2);
                             RBFSL_STENCIL_PU (2): RBF-PU, rbfsl_create_pu only; n is
                                the nominal number of nodes per patch                 */
    int32_t velocity_id;  /* RBFSL_VEL_*                                                  */
    int32_t n_tracers;    /* number of fields sharing each step's weights, >= 1           */
    int32_t integrator;   /* RBFSL_RK4 (0) or RBFSL_RK5_FEHLBERG (1)                      */
    int32_t cache_factors; /* stencil_mode 1 only: 1 = factor every node's system once at
                              create and reuse the factorizations each step (Section
                              3.3.2; N (n+(L+1)^2)^2 doubles of device memory, results
                              unchanged); 0 = assemble and factor every step          */
    double vel[8];        /* velocity parameters, see above                               */
    double dt;            /* time step, > 0                                               */
    double t0;            /* time of step 0                                               */
} rbfsl_params;

/* Create a transport context: the inputs of Algorithm 1 (Section 3) -- the
 * node set X on the sphere, the velocity u (velocity_id, vel), the time step
 * dt and start t0 -- and the local method's stencil size n with its harmonic
 * degree L and PHS order k (Sections 2.2 and 2.4).
 * nodes_xyz: N x 3 row-major (x, y, z) of nodes on the unit sphere (copied).
 * Builds the spatial hash of the nodes (and, in stencil_mode 1, every node's
 * stencil) on the device.  (n + (L+1)^2) must not exceed rbfsl_max_system().
 * On failure *out is NULL. */
int rbfsl_create(const double *nodes_xyz, int64_t N, int nodes_on_device,
                 const rbfsl_params *p, void *hip_stream, rbfsl_ctx **out);

/* RBF-PU interpolation (Sections 2.3 and 3.3.3) in place of the local
 * stencils.  Patch l is the spherical cap |x - c_l| < R around
 * centers_xyz[l] (Mp x 3, copied; the paper's choice: a quasi-uniform set of
 * ceil(a N / n) points and R = 2 sqrt(n/N), eq. rad_patches and
 * eq. num_patches); its nodes are every node inside it, in ascending
 * (distance^2, index) order.  Each patch's augmented interpolant (eq. rbf_poly
 * in the patch's frame, squared scale R * R) is factored once here; a step
 * solves it for the tracer values at the patch's nodes and evaluates, at each
 * departure point, the blend (eq. PU_interp) of the interpolants of the
 * patches containing it (ascending (distance^2, patch index)) with the cubic
 * B-spline weights phi_l = B(|xi - c_l| / R) (eq. bspline, eq. pu_func):
 * q = (sum_l phi_l s_l(xi)) / (sum_l phi_l).
 * p->stencil_mode must be RBFSL_STENCIL_PU and cache_factors 0; 0 < R <= 2.
 * Fails with RBFSL_E_SEARCH when a patch is empty, holds more nodes than a
 * system of rbfsl_max_system() unknowns allows, or more than its node list
 * (about 2n + 64 nodes); a step fails with RBFSL_E_SEARCH when a departure
 * point lies in no patch or in more patches than its list holds (twice the
 * mean overlap Mp R^2 / 4 plus 3, at least 8, at most 32), and with
 * RBFSL_E_SINGULAR when a patch it uses has a singular system.  rbfsl_debug_stencils and
 * rbfsl_debug_weights do not apply (RBFSL_E_INVAL). */
enum { RBFSL_STENCIL_PU = 2 };
int rbfsl_create_pu(const double *nodes_xyz, int64_t N, int nodes_on_device, const double *centers_xyz,
                    int64_t Mp, double R, const rbfsl_params *p, void *hip_stream, rbfsl_ctx **out);
/* Patch geometry of an RBF-PU context: patch count, node-list capacity ncap,
 * largest patch (any output may be NULL).  RBFSL_E_INVAL for other contexts. */
int rbfsl_pu_info(const rbfsl_ctx *ctx, int64_t *npatch, int32_t *ncap, int32_t *nmax, double *R);
/* Parity tap: every patch's node count (Mp) and node list (Mp x ncap, the
 * first count entries of each row are the patch's nodes). */
int rbfsl_debug_patches(rbfsl_ctx *ctx, int32_t *counts, int32_t *idx);

/* Set q^m, the field values at the nodes (Algorithm 1's q^0 = q(X, 0) when
 * called before the first step): n_tracers x N row-major, copied.  Does not
 * change the step index. */
int rbfsl_set_q(rbfsl_ctx *ctx, const double *q, int on_device);

/* One pass of Algorithm 1's loop, q^m -> q^{m+1}: trace every node back over
 * [t_m, t_{m+1}] (eq. sl_ode, Section 3.2), interpolate q^m at the departure
 * points with the local interpolant (eq. rbf_poly, Section 3.3.2) and assign
 * the values to the nodes.  Synchronises and commits only if every stencil
 * solved: on RBFSL_E_SINGULAR / _NONFINITE / _SEARCH the state stays at m. */
int rbfsl_step(rbfsl_ctx *ctx);

/* nsteps passes of Algorithm 1's loop (each as rbfsl_step), enqueued without
 * host synchronisation between them; one synchronisation at the end.  If step
 * f fails, later steps do nothing and the state is left at step f (q^f), with
 * the failure code returned.  The results are those of nsteps rbfsl_step
 * calls, bit for bit.  In stencil modes 0 and 1 without cached factors and
 * for N <= 65,536, a run of two or more steps goes in chunks: a step's departure points,
 * stencils and weights do not depend on q (the velocity is prescribed, eq.
 * sl_ode), so the tracer, search and solve of the K steps of a chunk each run
 * as one launch over K N points (K = rbfsl_steps_per_launch), then the
 * chunk's K field updates follow in step order.  Chunks
 * hold K steps (a last chunk of more than K/2 steps in two halves when
 * K >= 8); a chunk's tracer and search run on one stream of the library's
 * and its solve on another, overlapping the solve of the chunk before and
 * the field updates (on hip_stream) of the one before that.  The buffers of
 * two chunks (departure points, stencils, weights) are allocated by the
 * first such run and kept until rbfsl_destroy; when they do not fit, runs go
 * step by step.  In that mode the failure
 * counts of rbfsl_get_failures may include stencils of steps after the first
 * failing one (their launch had already started); the failing step, the
 * state and q are as above.  After the run, the debug taps show the run's
 * last step. */
int rbfsl_run(rbfsl_ctx *ctx, int64_t nsteps);

/* Steps per launch that rbfsl_run(ctx, nsteps) takes at most: 1 for the
 * step-by-step path (N > 65,536 among others), else K >= 2: half of nsteps
 * rounded up, at least 2, at most 131,072 / N and 128. */
int64_t rbfsl_steps_per_launch(const rbfsl_ctx *ctx, int64_t nsteps);

/* Copy q^m, Algorithm 1's state after m steps, out (n_tracers x N).
 * Synchronises. */
int rbfsl_get_q(rbfsl_ctx *ctx, double *out, int on_device);

/* Current step index m and time t0 + m dt. */
int rbfsl_get_state(const rbfsl_ctx *ctx, int64_t *step, double *t);

/* Number of stencils of the last step whose system was singular, non-finite,
 * or whose neighbour search failed (each may be NULL). */
int rbfsl_get_failures(const rbfsl_ctx *ctx, int64_t *singular, int64_t *nonfinite,
                       int64_t *search);

/* Measurement taps.  While profiling is enabled, every step records HIP
 * events around each of its four phases on the context's stream; the
 * accumulated device time per phase (ms: [0] trace, [1] stencil search,
 * [2] assembly + elimination + back substitution, [3] apply) and the number of
 * steps recorded are read (synchronising) by rbfsl_phase_times.  Enabling
 * resets the totals. */
int rbfsl_profile(rbfsl_ctx *ctx, int enable);
int rbfsl_phase_times(rbfsl_ctx *ctx, double *ms, int64_t *steps);

/* Parity taps: quantities of the last executed step (host outputs).
 * departure: N x 3 departure points; stencils: N x n node indices in the
 * order used (ascending (distance^2, index)); weights: N x n. */
int rbfsl_debug_departure(rbfsl_ctx *ctx, double *xi);
int rbfsl_debug_stencils(rbfsl_ctx *ctx, int32_t *idx);
int rbfsl_debug_weights(rbfsl_ctx *ctx, double *w);
/* The same taps for J selected nodes jl[0..J) (host int64 indices in [0, N)),
 * gathered on the device: xi J x 3, idx J x n, w J x n (any may be NULL;
 * idx and w are RBFSL_E_INVAL for RBF-PU contexts).  An index outside [0, N)
 * is RBFSL_E_INVAL and nothing is written. */
int rbfsl_debug_sample(rbfsl_ctx *ctx, const int64_t *jl, int64_t J, double *xi, int32_t *idx,
                       double *w);

/* Stateless exact neighbour search through the spatial hash: for each of Q
 * query points (Q x 3), the n nodes with the smallest keys (d^2, index),
 * d^2 = (dx*dx + dy*dy) + dz*dz, ascending.  idx: Q x n, d2: Q x n (may be
 * NULL).  All arrays host or all device per `on_device`. */
int rbfsl_knn(const double *nodes_xyz, int64_t N, const double *queries, int64_t Q, int32_t n,
              int32_t *idx, double *d2, int on_device, void *hip_stream);

/* Stateless batched weights for `count` stencils (Section 3.3.2 with the
 * system of eq. rbf_poly_linsys): stencil t has node indices idx[t*n ..],
 * centre centers[t], squared scale s2[t] and evaluation point evals[t]
 * (all points x 3 row-major).  w: count x n, status: count (0, or the
 * RBFSL_E_* code of that stencil; may be NULL). */
int rbfsl_weights(const double *nodes_xyz, int64_t N, const int32_t *idx, const double *centers,
                  const double *s2, const double *evals, int64_t count, int32_t n, int32_t L,
                  int32_t k, double *w, int32_t *status, int on_device, void *hip_stream);

/* rbfsl_weights for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same weights, bit for bit, computed without any allocation.  Every
 * array is device memory on the current device (nodes_xyz N x 3, idx count x n,
 * centers and evals count x 3, s2 count; outputs w count x n and status count,
 * status may be NULL); a host pointer is RBFSL_E_INVAL.  The work is only
 * enqueued on hip_stream (NULL = default stream): the outputs are valid once
 * the stream has reached this point; nothing is synchronised.  The library's
 * scratch for it (the coordinates as separate x, y, z arrays and the status
 * words) is one fixed device array per GPU, held until the process ends, of
 * 3 (N + 2 count) doubles at most: N + 2 count <= rbfsl_weights_noalloc_capacity()
 * (2,097,152; 48 MiB), else RBFSL_E_CAPACITY and nothing is enqueued.  Calls
 * that overlap on one GPU (other streams, other host threads) share that
 * array and race; serialise them. */
int rbfsl_weights_noalloc(const double *nodes_xyz, int64_t N, const int32_t *idx, const double *centers,
                          const double *s2, const double *evals, int64_t count, int32_t n, int32_t L,
                          int32_t k, double *w, int32_t *status, void *hip_stream);
/* The largest N + 2 count rbfsl_weights_noalloc accepts. */
int64_t rbfsl_weights_noalloc_capacity(void);

/* Largest supported system size n + (L+1)^2. */
int rbfsl_max_system(void);

/* sha256 (hex) of the sources this library was built from, as the build
 * computes it; a binding compares it with the sources next to it to refuse a
 * stale library.  Static string. */
const char *rbfsl_source_hash(void);

const char *rbfsl_strerror(int code);
/* Message of the last failure on this context (owned by the context, valid
 * until the next call on it). */
const char *rbfsl_last_error(const rbfsl_ctx *ctx);
void rbfsl_destroy(rbfsl_ctx *ctx);

/* ------------------------------------------------------------------------
 * Pooled runs: the batched and served forms.
 *
 * A pool holds many independent transport runs (each: its own nodes, flow,
 * stencil size n, degree L, PHS order k, tracers and step count) resident in
 * HBM and advances all of them together.  Each step is one persistent launch
 * per kernel family in which every node of every run goes through the whole
 * of Algorithm 1 (departure point, stencil search, assembly and solution of
 * the system of eq. rbf_poly_linsys, new value of q); the launches of one
 * step are captured once as a HIP graph and replayed.  Results are bit for
 * bit those of rbfsl_run on the same run (stencil_mode 0).
 *
 * Memory: the pool reserves `hbm_budget` bytes of device memory at creation
 * and places every admitted run inside it (rbfsl_pool_run_bytes says how
 * much one run takes); admission fails with RBFSL_E_BUDGET when no slot or no
 * contiguous space is left.  The pool works on streams of its own; calls that
 * return data synchronise them.  One host thread at a time per pool.
 * ------------------------------------------------------------------------ */
typedef struct rbfsl_pool rbfsl_pool;

typedef struct {
    int32_t max_runs;   /* run slots, 1 .. 4096                                   */
    int32_t use_graph;  /* 1: every step is one replay of a captured HIP graph;   *
                         * 0: the same kernels launched one by one                */
    int64_t hbm_budget; /* bytes reserved for run state; 0: half the free memory  */
    int32_t log_requests; /* 1: rbfsl_pool_serve writes one line per completed    *
                           * request to stderr (index, time, status)              */
    int32_t reserved;     /* 0                                                    */
} rbfsl_pool_config;

int rbfsl_pool_create(const rbfsl_pool_config *cfg, rbfsl_pool **out);

/* Device bytes one run of N nodes with these parameters and nsteps steps
 * occupies in a pool (-1 on invalid input). */
int64_t rbfsl_pool_run_bytes(int64_t N, const rbfsl_params *p, int64_t nsteps);

/* Admit a run: N x 3 nodes, q0 (n_tracers x N), nsteps steps from p->t0.
 * p->stencil_mode must be 0.  The run starts with the next step; *run_id
 * names it.  RBFSL_E_BUDGET: no free slot or HBM (nothing was changed). */
int rbfsl_pool_add(rbfsl_pool *pool, const double *nodes_xyz, int64_t N, int nodes_on_device,
                   const rbfsl_params *p, const double *q0, int q_on_device, int64_t nsteps,
                   int64_t *run_id);

/* Up to nsteps steps of every run that has steps left; a run stops at its
 * own step count, or at a failing step (singular/non-finite/search), which is
 * then not committed: its q stays at that step (as rbfsl_run).  Synchronises
 * at the end; per-run outcome through rbfsl_pool_run_info. */
int rbfsl_pool_step(rbfsl_pool *pool, int64_t nsteps);

/* Steps done, steps requested, and RBFSL_OK or the failure code of a run. */
int rbfsl_pool_run_info(rbfsl_pool *pool, int64_t run_id, int64_t *step, int64_t *nsteps, int *status);

/* q of a run at its current step (n_tracers x N). */
int rbfsl_pool_get_q(rbfsl_pool *pool, int64_t run_id, double *out, int on_device);

/* Retire a run and give its slot and memory back. */
int rbfsl_pool_remove(rbfsl_pool *pool, int64_t run_id);

typedef struct {
    int32_t runs, active;         /* admitted runs; runs with steps left */
    int64_t bytes_used, bytes_budget;
    int64_t steps_launched;
    int64_t items_per_step[4];    /* queue items of the last step, per kernel family */
    int32_t blocks[4];            /* persistent workgroups per launch, per family    */
    int32_t graph;
} rbfsl_pool_stats;
int rbfsl_pool_info(rbfsl_pool *pool, rbfsl_pool_stats *st);

/* The compiled solver variants of the pooled kernels: for variant i, the
 * largest system, waves per stencil, stencils per workgroup and panel width.
 * Returns the number of variants (fills at most cap entries). */
int rbfsl_pool_variants(int32_t *mcap, int32_t *waves, int32_t *group, int32_t *panel, int32_t cap);

/* Use variant `variant` (-1: the default) for every run with n + (L+1)^2 = M. */
int rbfsl_pool_set_variant(rbfsl_pool *pool, int32_t M, int32_t variant);

/* Autotuner: for every system size among the runs with steps left, time
 * `trials` uncommitted steps of those runs with each variant that can solve
 * them and keep the fastest (results do not depend on the choice).  One entry
 * per (size, variant) tried goes to res (at most cap; count = entries). */
typedef struct {
    int32_t M, variant;
    float ms_per_step;
    int32_t chosen;
} rbfsl_tune_result;
int rbfsl_pool_tune(rbfsl_pool *pool, int32_t trials, rbfsl_tune_result *res, int32_t cap, int32_t *count);

/* Served form: run a stream of requests through the pool with continuous
 * batching.  Request i arrives `arrival` seconds after the call starts; it is
 * admitted first come first served as soon as a slot and HBM are free (while
 * other runs are stepping), steps alongside the other admitted runs on the
 * device, and its final q (n_tracers x N, host) is written to q_out.  Each
 * pool step takes the admitted runs with the least remaining work: those
 * whose estimated remaining device time, divided by 1 + (seconds since
 * admission) / 30, is within twice the smallest; the others wait for that
 * step (their state is untouched).  The schedule changes when runs step, not
 * what a run computes: every result is the one the request gets alone.  Host
 * arrays are read during the call only.  res[i]: admission and completion
 * times (seconds after the start), RBFSL_OK or the failure code, steps done.
 * A request that cannot fit an empty pool gets RBFSL_E_BUDGET. */
typedef struct {
    double arrival;
    const double *nodes_xyz;  /* N x 3, host */
    int64_t N;
    rbfsl_params params;
    const double *q0;         /* n_tracers x N, host */
    int64_t nsteps;
    double *q_out;            /* n_tracers x N, host */
} rbfsl_request;
typedef struct {
    double admitted, finished;
    int32_t status;
    int32_t pad;
    int64_t steps;
} rbfsl_request_result;
int rbfsl_pool_serve(rbfsl_pool *pool, const rbfsl_request *req, int64_t nreq, rbfsl_request_result *res,
                     double *wall_seconds);

const char *rbfsl_pool_last_error(const rbfsl_pool *pool);
void rbfsl_pool_destroy(rbfsl_pool *pool);

#ifdef __cplusplus
}
#endif
#endif

// Host side of the C ABI declared in rbfsl.h: parameter validation, buffer
// ownership, the per-step velocity coefficients (the only transcendental
// functions evaluated anywhere: cos/sin of the stage times) and the enqueueing
// of the step kernels (Algorithm 1: trace -> stencils -> weights -> apply).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rbfsl_impl.h"

using namespace rbfsl;

struct rbfsl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    rbfsl_params p{};
    int n = 0, L = 0, k = 0, M = 0, ntr = 1, mode = 0;
    int64_t N = 0;
    double *nx = nullptr, *ny = nullptr, *nz = nullptr;
    Grid grid;
    double *ex = nullptr, *ey = nullptr, *ez = nullptr;  // departure points
    int32_t *S = nullptr;                                // stencils (mode 1: of every node)
    double *s2 = nullptr;
    int32_t *cidx = nullptr;                             // mode 1: nearest node of xi_j
    double *w = nullptr;
    // mode 1 with cached factors: every node's factorization (Section 3.3.2)
    bool cached = false;
    double *F = nullptr, *frinv = nullptr;
    int32_t *fpiv = nullptr, *fstep = nullptr, *fstat = nullptr;
    // RBF-PU (mode RBFSL_STENCIL_PU): patches, their factorizations (the
    // fields above) and coefficients, and the centres' spatial hash
    int64_t Mp = 0;
    double R = 0.0;
    int ncap = 0, pcap = 0, nmax = 0;
    double *cx = nullptr, *cy = nullptr, *cz = nullptr, *pd2 = nullptr, *pr2 = nullptr;
    double *coef = nullptr, *sd2 = nullptr, *sval = nullptr, *ploc = nullptr;
    int32_t *pidx = nullptr, *pcnt = nullptr, *sidx = nullptr;
    Grid cgrid;
    double *q[2] = {nullptr, nullptr};
    int cur = 0;
    // runs in chunks of steps: two sets, by chunk parity, of the departure
    // points, stencils and weights of up to ahead_cap steps with their tracer
    // coefficients (device, and pinned staging).  A chunk's tracer and search
    // run on sstream, its solve on wstream, while the solve of the chunk
    // before and the field updates of the one before that run.
    struct AheadSet {
        double *ex = nullptr, *ey = nullptr, *ez = nullptr, *s2 = nullptr, *w = nullptr;
        int32_t *S = nullptr, *cidx = nullptr;
        StepCoef *sc = nullptr, *sc_host = nullptr;
        const StepCoef *sc_mapped = nullptr;  // sc_host's device address
        hipEvent_t staged = nullptr;   // the coefficients' staging has run
        hipEvent_t searched = nullptr; // the chunk's departure points and stencils are written
        hipEvent_t solved = nullptr;   // the chunk's weights are written
        hipEvent_t applied = nullptr;  // the chunk's field updates have run
        bool used = false;
    };
    int64_t ahead_cap = 0;
    AheadSet aset[2];
    hipStream_t wstream = nullptr, sstream = nullptr;
    hipEvent_t run_start = nullptr;
    bool ahead_off = false;  // the chunk sets did not fit: step by step
    // what the debug taps read: the single-step buffers, or after a run of
    // several steps per launch, its last step's slice of an ahead set
    const double *tex = nullptr, *tey = nullptr, *tez = nullptr, *tw = nullptr;
    const int32_t *tS = nullptr, *tcidx = nullptr;
    int *status = nullptr;
    int64_t step = 0;
    bool q_set = false, ran = false;
    int64_t f_sing = 0, f_nonf = 0, f_search = 0;
    // profiling: per-step events around the four phases (trace, search and
    // solve back to back on one stream, the field update on its own pair)
    bool prof = false;
    std::vector<hipEvent_t> ev;  // 7 per recorded step
    int64_t ev_used = 0, prof_steps = 0;
    std::vector<int64_t> ev_steps;  // steps covered by each recorded group of 6
    double prof_ms[4] = {0, 0, 0, 0};
    std::string err;
};

namespace {

int fail(rbfsl_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(rbfsl_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIP_TRY(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), e_ == hipErrorOutOfMemory ? RBFSL_E_NOMEM : RBFSL_E_DEVICE,   \
                        "%s: %s", #call, hipGetErrorString(e_));                             \
    } while (0)

// libm cos and sin, each called on its own (a merged sincos() call can differ
// in the last bit)
__attribute__((noinline)) double cos_of(double x) { return cos(x); }
__attribute__((noinline)) double sin_of(double x) { return sin(x); }

// velocity coefficients at time t (see rbfsl.h); evaluated term by term in a
// fixed order
void vel_coef_at(int vel_id, const double *vp, double t, VelCoef *vc) {
    memset(vc, 0, sizeof(*vc));
    vc->R[0] = 1.0;
    vc->R[4] = 1.0;
    vc->R[8] = 1.0;
    if (vel_id == RBFSL_VEL_ZERO) return;
    const double T = vp[0];
    const double a[3] = {vp[1], vp[2], vp[3]};
    const double Om = (2.0 * M_PI) / T;
    if (vel_id == RBFSL_VEL_NL2010) {
        vc->w[2] = Om;
        vc->c = (10.0 / T) * cos_of((M_PI * t) / T);
        vc->cw = cos_of(Om * t);
        vc->sw = sin_of(Om * t);
        return;
    }
    for (int i = 0; i < 3; ++i) vc->w[i] = Om * a[i];
    if (vel_id != RBFSL_VEL_DEFORM) return;
    const double th = Om * t;
    const double ct = cos_of(th), st = sin_of(th);
    const double omc = 1.0 - ct;
    const double K[9] = {0.0, -a[2], a[1], a[2], 0.0, -a[0], -a[1], a[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double d = (i == j) ? 1.0 : 0.0;
            vc->R[3 * i + j] = ((ct * d) + (st * K[3 * i + j])) + (omc * (a[i] * a[j]));
        }
    vc->c = vp[4] * cos_of((M_PI * t) / T);
}

StepCoef make_step_coef(const rbfsl_params &p, int64_t m) {
    StepCoef sc;
    memset(&sc, 0, sizeof sc);
    const double t1 = p.t0 + (double)(m + 1) * p.dt;
    sc.h = -p.dt;
    sc.hh = 0.5 * sc.h;
    sc.h6 = sc.h / 6.0;
    sc.vel_id = p.velocity_id;
    sc.rk = p.integrator;
    if (p.integrator == RBFSL_RK4) {
        vel_coef_at(p.velocity_id, p.vel, t1, &sc.v[0]);
        vel_coef_at(p.velocity_id, p.vel, t1 - 0.5 * p.dt, &sc.v[1]);
        vel_coef_at(p.velocity_id, p.vel, p.t0 + (double)m * p.dt, &sc.v[2]);
    } else {
        for (int s = 0; s < 6; ++s) vel_coef_at(p.velocity_id, p.vel, t1 + kRk5C[s] * sc.h, &sc.v[s]);
    }
    return sc;
}

__global__ void k_aos_to_soa(const double *aos, int64_t N, double *x, double *y, double *z) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    x[i] = aos[3 * i];
    y[i] = aos[3 * i + 1];
    z[i] = aos[3 * i + 2];
}

__global__ void k_soa_to_aos(const double *x, const double *y, const double *z, int64_t N, double *aos) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    aos[3 * i] = x[i];
    aos[3 * i + 1] = y[i];
    aos[3 * i + 2] = z[i];
}

// A chunk's tracer coefficients from pinned host memory to the device, read by
// a kernel on the weights stream itself (a copy-engine transfer there cost
// 15-80 us of hand-over between engines at every chunk): one 8-byte word per
// thread, so that every read of host memory is in flight at once.
__global__ void k_stage_words(const uint64_t *src, uint64_t *dst, int64_t nwords) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) dst[i] = src[i];
}

__global__ void k_gather_rows(const int32_t *S, const int32_t *cidx, int64_t N, int n, int32_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * n) return;
    int64_t j = i / n, a = i % n;
    out[i] = S[(int64_t)cidx[j] * n + a];
}

// rows jl[0..J) of the last step's departure points, stencils and weights
// (stencils of node K = cidx[j] in the centre-point mode)
__global__ void k_gather_sample(const int64_t *jl, int64_t J, const double *ex, const double *ey,
                                const double *ez, const int32_t *S, const int32_t *cidx, const double *w,
                                int n, double *xi, int32_t *Sout, double *wout) {
    const int64_t t = (int64_t)blockIdx.x;
    if (t >= J) return;
    const int64_t j = jl[t];
    if (threadIdx.x == 0 && xi) {
        xi[3 * t] = ex[j];
        xi[3 * t + 1] = ey[j];
        xi[3 * t + 2] = ez[j];
    }
    const int64_t row = cidx ? (int64_t)cidx[j] : j;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        if (Sout) Sout[t * n + a] = S[row * n + a];
        if (wout) wout[t * n + a] = w[j * n + a];
    }
}

// upload an N x 3 AoS array (host or device) as SoA device arrays
hipError_t upload_points(const double *xyz, int64_t N, int on_device, double *x, double *y,
                         double *z, hipStream_t s) {
    if (N == 0) return hipSuccess;
    double *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, sizeof(double) * 3 * N);
    if (e != hipSuccess) return e;
    e = rbfsl::upload_points_via(xyz, N, on_device, x, y, z, tmp, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return e;
}

hipError_t download_points(const double *x, const double *y, const double *z, int64_t N,
                           double *xyz_host, hipStream_t s) {
    if (N == 0) return hipSuccess;
    double *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, sizeof(double) * 3 * N);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soa_to_aos, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, x, y, z,
                       N, tmp);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(xyz_host, tmp, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return e;
}

int paper_L(int n) {
    int L = 0;
    while ((2 * (L + 1) + 1) * (2 * (L + 1) + 1) <= n) ++L;
    return L;
}

// validated (n, L, k) or an error message
int resolve_nlk(int64_t N, int n, int L, int k, int *Lo, int *ko, char *msg, size_t msz) {
    if (n < 1 || (int64_t)n > N) {
        snprintf(msg, msz, "stencil size n=%d must be in [1, N=%lld]", n, (long long)N);
        return RBFSL_E_INVAL;
    }
    if (L < 0) L = paper_L(n);
    if (k < 0) k = L;
    if (k > L) {
        snprintf(msg, msz, "PHS order k=%d must not exceed the harmonic degree L=%d", k, L);
        return RBFSL_E_INVAL;
    }
    if ((L + 1) * (L + 1) > n) {
        snprintf(msg, msz, "n=%d nodes cannot determine the (L+1)^2=%d harmonics of degree L=%d", n,
                 (L + 1) * (L + 1), L);
        return RBFSL_E_INVAL;
    }
    const int M = n + (L + 1) * (L + 1);
    if (solve_variant_capacity(M) == 0) {
        snprintf(msg, msz, "system size n+(L+1)^2=%d exceeds the supported maximum %d", M, MAX_SYSTEM);
        return RBFSL_E_INVAL;
    }
    *Lo = L;
    *ko = k;
    return RBFSL_OK;
}

void ahead_free(rbfsl_ctx *c) {
    if (c->sstream) (void)hipStreamSynchronize(c->sstream);  // nothing of them still uses the sets
    if (c->wstream) (void)hipStreamSynchronize(c->wstream);
    for (rbfsl_ctx::AheadSet &A : c->aset) {
        void *bufs[] = {A.ex, A.ey, A.ez, A.s2, A.w, A.S, A.cidx, A.sc};
        for (void *b : bufs)
            if (b) (void)hipFree(b);
        if (A.sc_host) (void)hipHostFree(A.sc_host);
        hipEvent_t evs[] = {A.staged, A.searched, A.solved, A.applied};
        for (hipEvent_t e : evs)
            if (e) (void)hipEventDestroy(e);
        A = rbfsl_ctx::AheadSet{};
    }
    if (c->run_start) (void)hipEventDestroy(c->run_start);
    if (c->wstream) (void)hipStreamDestroy(c->wstream);
    if (c->sstream) (void)hipStreamDestroy(c->sstream);
    c->run_start = nullptr;
    c->wstream = c->sstream = nullptr;
    c->ahead_cap = 0;
}

void taps_single(rbfsl_ctx *c) {
    c->tex = c->ex; c->tey = c->ey; c->tez = c->ez; c->tw = c->w;
    c->tS = c->S; c->tcidx = c->cidx;
}

void ctx_free(rbfsl_ctx *c) {
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    ahead_free(c);
    void *bufs[] = {c->nx, c->ny, c->nz, c->ex, c->ey, c->ez, c->S, c->s2, c->cidx, c->w,
                    c->q[0], c->q[1], c->status, c->F, c->frinv, c->fpiv, c->fstep, c->fstat,
                    c->cx, c->cy, c->cz, c->pd2, c->pr2, c->coef, c->sd2, c->sval, c->ploc, c->pidx, c->pcnt, c->sidx};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    grid_free(&c->grid);
    grid_free(&c->cgrid);
}

int read_status(rbfsl_ctx *c, int st[ST_WORDS]) {
    HIP_TRY(c, hipMemcpyAsync(st, c->status, sizeof(int) * ST_WORDS, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RBFSL_OK;
}

int status_code(const int st[ST_WORDS]) {
    if (st[ST_SEARCH]) return RBFSL_E_SEARCH;
    if (st[ST_SINGULAR]) return RBFSL_E_SINGULAR;
    if (st[ST_NONFINITE]) return RBFSL_E_NONFINITE;
    return RBFSL_OK;
}

// One group of seven events per profiled step (or chunk of steps): marks 0, 1
// open the trace and search phases and 6 closes the search, 2 and 3 bracket
// the solve, 4 and 5 the field update.  prof_group reserves a group (-1 when not
// profiling); prof_mark records one of its marks on stream s.
hipError_t prof_group(rbfsl_ctx *c, int64_t steps, int64_t *g) {
    *g = -1;
    if (!c->prof) return hipSuccess;
    const int64_t need = c->ev_used + 7;
    while ((int64_t)c->ev.size() < need) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        c->ev.push_back(e);
    }
    *g = c->ev_used;
    c->ev_used += 7;
    c->ev_steps.push_back(steps);
    return hipSuccess;
}
hipError_t prof_mark(rbfsl_ctx *c, int64_t g, int mark, hipStream_t s) {
    return (g < 0) ? hipSuccess : hipEventRecord(c->ev[g + mark], s);
}
hipError_t prof_mark(rbfsl_ctx *c, int64_t g, int mark) { return prof_mark(c, g, mark, c->stream); }

// fold recorded events into the per-phase totals (after a synchronisation)
void prof_collect(rbfsl_ctx *c) {
    for (int64_t b = 0; b + 7 <= c->ev_used; b += 7) {
        static const int from[4] = {0, 1, 2, 4}, to[4] = {1, 6, 3, 5};
        for (int ph = 0; ph < 4; ++ph) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev[b + from[ph]], c->ev[b + to[ph]]) == hipSuccess) c->prof_ms[ph] += ms;
        }
        const size_t gi = (size_t)(b / 7);
        c->prof_steps += (gi < c->ev_steps.size()) ? c->ev_steps[gi] : 1;
    }
    c->ev_used = 0;
    c->ev_steps.clear();
}

PuArgs pu_args(const rbfsl_ctx *c, int64_t m) {
    PuArgs a{};
    a.nx = c->nx; a.ny = c->ny; a.nz = c->nz; a.N = c->N;
    a.cx = c->cx; a.cy = c->cy; a.cz = c->cz; a.Mp = c->Mp;
    a.R = c->R; a.R2 = c->R * c->R;
    a.pidx = c->pidx; a.pd2 = c->pd2; a.cnt = c->pcnt; a.ploc = c->ploc;
    a.ncap = c->ncap; a.nmax = c->nmax; a.L = c->L; a.k = c->k; a.ntr = c->ntr;
    a.F = c->F; a.rinv = c->frinv; a.stepof = c->fstep; a.fstat = c->fstat;
    a.coef = c->coef;
    a.ex = c->ex; a.ey = c->ey; a.ez = c->ez;
    a.sidx = c->sidx; a.sd2 = c->sd2; a.pcap = c->pcap;
    a.qin = c->q[c->cur]; a.qout = c->q[1 - c->cur]; a.sval = c->sval;
    a.status = c->status; a.step = m;
    return a;
}

hipError_t enqueue_step(rbfsl_ctx *c, int64_t m) {
    const StepCoef sc = make_step_coef(c->p, m);
    int64_t g;
    hipError_t e = prof_group(c, 1, &g);
    if (e == hipSuccess) e = prof_mark(c, g, 0);
    if (e != hipSuccess) return e;
    e = launch_trace(c->nx, c->ny, c->nz, c->N, sc, c->ex, c->ey, c->ez, c->status, m, c->stream);
    if (e != hipSuccess) return e;
    if ((e = prof_mark(c, g, 1)) != hipSuccess) return e;
    if (c->mode == RBFSL_STENCIL_PU) {
        // the patches containing each departure point, the patches'
        // coefficients, the partition-of-unity blend
        const PuArgs a = pu_args(c, m);
        if ((e = launch_pu_search(a, c->cgrid, c->stream)) != hipSuccess) return e;
        if ((e = prof_mark(c, g, 6)) != hipSuccess || (e = prof_mark(c, g, 2)) != hipSuccess) return e;
        if ((e = launch_pu_coef(a, c->stream)) != hipSuccess) return e;
        if ((e = prof_mark(c, g, 3)) != hipSuccess || (e = prof_mark(c, g, 4)) != hipSuccess) return e;
        if ((e = launch_pu_eval(a, c->stream)) != hipSuccess) return e;
        return prof_mark(c, g, 5);
    }
    if (c->mode == 0)
        e = launch_knn(c->grid, c->N, c->ex, c->ey, c->ez, c->N, c->n, c->S, nullptr, c->s2, c->status, m, c->stream);
    else
        e = launch_knn(c->grid, c->N, c->ex, c->ey, c->ez, c->N, 1, c->cidx, nullptr, nullptr, c->status, m, c->stream);
    if (e != hipSuccess) return e;
    if ((e = prof_mark(c, g, 6)) != hipSuccess || (e = prof_mark(c, g, 2)) != hipSuccess) return e;
    SolveArgs a{};
    a.nx = c->nx; a.ny = c->ny; a.nz = c->nz; a.N = c->N;
    a.ex = c->ex; a.ey = c->ey; a.ez = c->ez;
    if (c->mode == 1) {
        a.cx = c->nx; a.cy = c->ny; a.cz = c->nz;
        a.cidx = c->cidx;
    }
    a.S = c->S; a.s2 = c->s2;
    a.count = c->N; a.n = c->n; a.L = c->L; a.k = c->k;
    a.w = c->w; a.st_out = nullptr; a.status = c->status; a.step = m;
    if (c->cached) {
        CachedArgs ca{};
        ca.nx = c->nx; ca.ny = c->ny; ca.nz = c->nz; ca.N = c->N;
        ca.ex = c->ex; ca.ey = c->ey; ca.ez = c->ez;
        ca.S = c->S; ca.cidx = c->cidx; ca.s2 = c->s2;
        ca.F = c->F; ca.rinv = c->frinv; ca.piv = c->fpiv; ca.stepof = c->fstep; ca.fstat = c->fstat;
        ca.count = c->N; ca.n = c->n; ca.L = c->L; ca.k = c->k;
        ca.w = c->w; ca.status = c->status; ca.step = m;
        e = launch_solve_cached(ca, c->stream);
    } else {
        e = launch_solve(a, c->stream);
    }
    if (e != hipSuccess) return e;
    if ((e = prof_mark(c, g, 3)) != hipSuccess || (e = prof_mark(c, g, 4)) != hipSuccess) return e;
    e = launch_apply(c->w, c->S, c->mode == 1 ? c->cidx : nullptr, c->N, c->n, c->ntr,
                     c->q[c->cur], c->q[1 - c->cur], c->status, m, c->stream);
    if (e != hipSuccess) return e;
    return prof_mark(c, g, 5);
}

// Runs of small problems take several steps per launch: the departure points,
// stencils and weights of a step do not depend on the transported field (the
// velocity is prescribed), so K steps' tracer, search and solve run as one
// launch each, and then the K field updates in step order.  Every step's
// arithmetic is the step-by-step path's.  A run is cut into about AHEAD_CHUNKS
// chunks so that the search of one chunk, the solve of the one before and the
// field updates of the one before that overlap.  Problems too large for two
// steps per launch (N > AHEAD_STENCILS / 2) go step by step: with chunks of
// one step, the next step's search running beside the solve slowed it by more
// than the search and update time it hid (N = 655,362, n = 120: 548.8 against
// 545.5 ms per step).
constexpr int64_t AHEAD_STENCILS = 131072;  // stencils per launch at most
constexpr int64_t AHEAD_MAX = 128;
constexpr int64_t AHEAD_CHUNKS = 2;  // N = 1,024, 128 steps: 2, 3, 4, 6 chunks 0.029, 0.0296, 0.0298, 0.0308 ms/step

// the most steps per chunk this context takes
int64_t ahead_max(const rbfsl_ctx *c) {
    const int64_t K = std::min(AHEAD_MAX, AHEAD_STENCILS / c->N);
    return (K < 1) ? 1 : K;
}

// runs of this many steps go in chunks (not the cached, RBF-PU or single-step
// forms, nor problems of more than AHEAD_STENCILS / 2 nodes)
bool chunked(const rbfsl_ctx *c, int64_t nsteps) {
    return c->mode != RBFSL_STENCIL_PU && !c->cached && !c->ahead_off && nsteps >= 2 && ahead_max(c) >= 2;
}

int64_t ahead_steps(const rbfsl_ctx *c, int64_t nsteps) {
    if (!chunked(c, nsteps)) return 1;
    return std::min(ahead_max(c), std::max<int64_t>(2, (nsteps + AHEAD_CHUNKS - 1) / AHEAD_CHUNKS));
}

// both sets at the context's largest chunk, once (a run never reallocates)
hipError_t ahead_alloc(rbfsl_ctx *c) {
    if (c->ahead_cap > 0) return hipSuccess;
    const int64_t K = ahead_max(c), KN = K * c->N;
    hipError_t e = hipStreamCreateWithFlags(&c->wstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->sstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->run_start, hipEventDisableTiming);
#define ALLOC(ptr, bytes) if (e == hipSuccess) e = hipMalloc(&(ptr), (bytes))
#define EVENT(ev) if (e == hipSuccess) e = hipEventCreateWithFlags(&(ev), hipEventDisableTiming)
    for (rbfsl_ctx::AheadSet &A : c->aset) {
        ALLOC(A.ex, sizeof(double) * KN);
        ALLOC(A.ey, sizeof(double) * KN);
        ALLOC(A.ez, sizeof(double) * KN);
        ALLOC(A.w, sizeof(double) * KN * c->n);
        if (c->mode == 0) {
            ALLOC(A.s2, sizeof(double) * KN);
            ALLOC(A.S, sizeof(int32_t) * KN * c->n);
        } else {
            ALLOC(A.cidx, sizeof(int32_t) * KN);
        }
        ALLOC(A.sc, sizeof(StepCoef) * K);
        if (e == hipSuccess) e = hipHostMalloc((void **)&A.sc_host, sizeof(StepCoef) * K, hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&A.sc_mapped, A.sc_host, 0);
        EVENT(A.staged);
        EVENT(A.searched);
        EVENT(A.solved);
        EVENT(A.applied);
    }
#undef EVENT
#undef ALLOC
    if (e != hipSuccess) {
        ahead_free(c);
        return e;
    }
    c->ahead_cap = K;
    return hipSuccess;
}

// the debug taps show step s of set cb
void taps_ahead(rbfsl_ctx *c, int cb, int64_t s) {
    const rbfsl_ctx::AheadSet &A = c->aset[cb];
    const int64_t N = c->N, n = c->n;
    c->tex = A.ex + s * N; c->tey = A.ey + s * N; c->tez = A.ez + s * N;
    c->tw = A.w + s * N * n;
    if (c->mode == 0) {
        c->tS = A.S + s * N * n;
        c->tcidx = nullptr;
    } else {
        c->tS = c->S;
        c->tcidx = A.cidx + s * N;
    }
}

// The departure points and stencils of steps m .. m + K - 1 into set cb on
// sstream, after the field updates that last read the set; their weights on
// wstream, after that search.
hipError_t enqueue_weights(rbfsl_ctx *c, int64_t m, int K, int cb, int64_t g) {
    rbfsl_ctx::AheadSet &A = c->aset[cb];
    const hipStream_t ss = c->sstream, ws = c->wstream;
    hipError_t e;
    if (A.used && (e = hipEventSynchronize(A.staged)) != hipSuccess) return e;
    for (int s = 0; s < K; ++s) A.sc_host[s] = make_step_coef(c->p, m + s);
    if (A.used && (e = hipStreamWaitEvent(ss, A.applied, 0)) != hipSuccess) return e;
    static_assert(sizeof(StepCoef) % sizeof(uint64_t) == 0, "StepCoef is staged as 64-bit words");
    const int64_t nwords = (int64_t)(sizeof(StepCoef) / sizeof(uint64_t)) * K;
    hipLaunchKernelGGL(k_stage_words, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, ss,
                       (const uint64_t *)A.sc_mapped, (uint64_t *)A.sc, nwords);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(A.staged, ss)) != hipSuccess) return e;
    A.used = true;
    const int64_t N = c->N, KN = (int64_t)K * N;
    if ((e = prof_mark(c, g, 0, ss)) != hipSuccess) return e;
    if ((e = launch_trace_steps(c->nx, c->ny, c->nz, N, A.sc, K, A.ex, A.ey, A.ez, c->status, m, ss)) != hipSuccess)
        return e;
    if ((e = prof_mark(c, g, 1, ss)) != hipSuccess) return e;
    if (c->mode == 0)
        e = launch_knn(c->grid, N, A.ex, A.ey, A.ez, KN, c->n, A.S, nullptr, A.s2, c->status, m, ss, N);
    else
        e = launch_knn(c->grid, N, A.ex, A.ey, A.ez, KN, 1, A.cidx, nullptr, nullptr, c->status, m, ss, N);
    if (e != hipSuccess) return e;
    if ((e = prof_mark(c, g, 6, ss)) != hipSuccess) return e;
    if ((e = hipEventRecord(A.searched, ss)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(ws, A.searched, 0)) != hipSuccess) return e;
    if ((e = prof_mark(c, g, 2, ws)) != hipSuccess) return e;
    SolveArgs a{};
    a.nx = c->nx; a.ny = c->ny; a.nz = c->nz; a.N = N;
    a.ex = A.ex; a.ey = A.ey; a.ez = A.ez;
    if (c->mode == 1) {
        a.cx = c->nx; a.cy = c->ny; a.cz = c->nz;
        a.cidx = A.cidx;
        a.S = c->S; a.s2 = c->s2;
    } else {
        a.S = A.S; a.s2 = A.s2;
    }
    a.count = KN; a.n = c->n; a.L = c->L; a.k = c->k;
    a.w = A.w; a.st_out = nullptr; a.status = c->status; a.step = m; a.step_count = N;
    if ((e = launch_solve(a, ws)) != hipSuccess) return e;
    if ((e = prof_mark(c, g, 3, ws)) != hipSuccess) return e;
    return hipEventRecord(A.solved, ws);
}

// The K field updates of steps m .. m + K - 1 from set cb, one launch each, on
// the context's stream after that set's solve; q^m is in q[par].  (One
// workgroup holding the field in LDS across the steps measured 3x slower at
// N = 1,024: a single compute unit cannot stream the steps' weights fast
// enough.)
hipError_t enqueue_applies(rbfsl_ctx *c, int64_t m, int K, int par, int cb, int64_t g) {
    rbfsl_ctx::AheadSet &A = c->aset[cb];
    const int64_t N = c->N;
    hipError_t e;
    if ((e = hipStreamWaitEvent(c->stream, A.solved, 0)) != hipSuccess) return e;
    if ((e = prof_mark(c, g, 4)) != hipSuccess) return e;
    const int32_t *Sb = (c->mode == 0) ? A.S : c->S;
    const int64_t sstride = (c->mode == 0) ? N * c->n : 0;
    for (int s = 0; s < K && e == hipSuccess; ++s)
        e = launch_apply(A.w + (int64_t)s * N * c->n, Sb + s * sstride,
                         (c->mode == 1) ? A.cidx + s * N : nullptr, N, c->n, c->ntr, c->q[par ^ (s & 1)],
                         c->q[par ^ ((s + 1) & 1)], c->status, m + s, c->stream);
    if (e != hipSuccess) return e;
    if ((e = prof_mark(c, g, 5)) != hipSuccess) return e;
    return hipEventRecord(A.applied, c->stream);
}

// A run of nsteps steps in chunks of K from step m0 (q^m0 in q[cur0]): each
// chunk's weights are enqueued before the previous chunk's field updates, so
// that the host never holds the weights stream back behind a row of updates.
// The last chunk's updates run after every solve has ended; when chunks are
// long (K >= 8) a last chunk of more than K/2 steps is cut in two halves, so
// that fewer of them wait.
hipError_t enqueue_chunks(rbfsl_ctx *c, int64_t m0, int64_t nsteps, int64_t K, int cur0, int64_t *mfail) {
    std::vector<int64_t> size;
    for (int64_t left = nsteps; left > 0;) {
        const int64_t k = std::min(K, left);
        if (k == left && K >= 8 && 2 * k > K) {
            size.push_back((k + 1) / 2);
            size.push_back(k / 2);
        } else {
            size.push_back(k);
        }
        left -= k;
    }
    const size_t nch = size.size();
    std::vector<int64_t> first(nch), grp(nch, -1);
    for (size_t j = 0, m = 0; j < nch; m += (size_t)size[j], ++j) first[j] = (int64_t)m;
    hipError_t e = hipSuccess;
    for (size_t j = 0; j <= nch && e == hipSuccess; ++j) {
        if (j < nch) {
            *mfail = m0 + first[j];
            e = prof_group(c, size[j], &grp[j]);
            if (e == hipSuccess) e = enqueue_weights(c, m0 + first[j], (int)size[j], (int)(j & 1), grp[j]);
        }
        if (j > 0 && e == hipSuccess) {
            const size_t i = j - 1;
            *mfail = m0 + first[i];
            e = enqueue_applies(c, m0 + first[i], (int)size[i], cur0 ^ (int)(first[i] & 1), (int)(i & 1), grp[i]);
        }
    }
    if (e == hipSuccess) taps_ahead(c, (int)((nch - 1) & 1), size[nch - 1] - 1);
    return e;
}

}  // namespace

namespace rbfsl {

StepCoef step_coef(const rbfsl_params &p, int64_t m) { return make_step_coef(p, m); }

int resolve_stencil(int64_t N, int n, int L, int k, int *Lo, int *ko, char *msg, size_t msz) {
    return resolve_nlk(N, n, L, k, Lo, ko, msg, msz);
}

int validate_params(int64_t N, const rbfsl_params *p, int *L, int *k, char *msg, size_t msz) {
    msg[0] = 0;
    if (N < 1 || N > 0x7fffffffLL) {
        snprintf(msg, msz, "node count N=%lld out of range", (long long)N);
        return RBFSL_E_INVAL;
    }
    if (!(p->dt > 0.0) || !isfinite(p->dt) || !isfinite(p->t0) || p->n_tracers < 1) {
        snprintf(msg, msz, "dt must be positive and finite, t0 finite, n_tracers >= 1");
        return RBFSL_E_INVAL;
    }
    if (p->velocity_id < RBFSL_VEL_ZERO || p->velocity_id > RBFSL_VEL_NL2010) {
        snprintf(msg, msz, "unknown velocity_id %d", p->velocity_id);
        return RBFSL_E_INVAL;
    }
    if (p->velocity_id != RBFSL_VEL_ZERO && (!(p->vel[0] != 0.0) || !isfinite(p->vel[0]))) {
        snprintf(msg, msz, "the flow period vel[0] must be finite and non-zero");
        return RBFSL_E_INVAL;
    }
    if (p->stencil_mode != 0 && p->stencil_mode != 1) {
        snprintf(msg, msz, "stencil_mode must be 0 or 1");
        return RBFSL_E_INVAL;
    }
    if (p->integrator != RBFSL_RK4 && p->integrator != RBFSL_RK5_FEHLBERG) {
        snprintf(msg, msz, "integrator must be RBFSL_RK4 or RBFSL_RK5_FEHLBERG");
        return RBFSL_E_INVAL;
    }
    if (p->cache_factors != 0 && (p->cache_factors != 1 || p->stencil_mode != 1)) {
        snprintf(msg, msz, "cache_factors = 1 needs stencil_mode 1 (fixed per-node systems)");
        return RBFSL_E_INVAL;
    }
    return resolve_nlk(N, p->n, p->L, p->k, L, k, msg, msz);
}

hipError_t upload_points_via(const double *xyz, int64_t N, int on_device, double *x, double *y,
                             double *z, double *tmp, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(tmp, xyz, sizeof(double) * 3 * N,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_aos_to_soa, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, tmp, N, x, y, z);
    return hipGetLastError();
}

}  // namespace rbfsl

extern "C" {

int rbfsl_max_system(void) { return MAX_SYSTEM; }

const char *rbfsl_strerror(int code) {
    switch (code) {
        case RBFSL_OK: return "ok";
        case RBFSL_E_INVAL: return "invalid argument";
        case RBFSL_E_NOMEM: return "out of memory";
        case RBFSL_E_DEVICE: return "HIP runtime error";
        case RBFSL_E_SINGULAR: return "singular stencil system";
        case RBFSL_E_NONFINITE: return "non-finite stencil weights";
        case RBFSL_E_STATE: return "invalid state";
        case RBFSL_E_SEARCH: return "neighbour search failed";
        case RBFSL_E_BUDGET: return "no free run slot or HBM budget";
        case RBFSL_E_CAPACITY: return "input larger than the fixed scratch of the no-allocation entry point";
        default: return "unknown status";
    }
}

const char *rbfsl_last_error(const rbfsl_ctx *c) { return c ? c->err.c_str() : ""; }

int rbfsl_create(const double *nodes_xyz, int64_t N, int nodes_on_device, const rbfsl_params *p,
                 void *hip_stream, rbfsl_ctx **out) {
    if (!out) return RBFSL_E_INVAL;
    *out = nullptr;
    if (!p || !nodes_xyz) return RBFSL_E_INVAL;
    int L, k;
    char msg[256];
    if (validate_params(N, p, &L, &k, msg, sizeof msg) != RBFSL_OK) return RBFSL_E_INVAL;
    rbfsl_ctx *c = new (std::nothrow) rbfsl_ctx();
    if (!c) return RBFSL_E_NOMEM;
    c->p = *p;
    c->p.L = L;
    c->p.k = k;
    c->n = p->n; c->L = L; c->k = k; c->M = p->n + (L + 1) * (L + 1);
    c->ntr = p->n_tracers; c->mode = p->stencil_mode; c->N = N;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    const size_t d = sizeof(double);
#define ALLOC(ptr, bytes) if (e == hipSuccess) e = hipMalloc(&(ptr), (bytes))
    ALLOC(c->nx, d * N); ALLOC(c->ny, d * N); ALLOC(c->nz, d * N);
    ALLOC(c->ex, d * N); ALLOC(c->ey, d * N); ALLOC(c->ez, d * N);
    ALLOC(c->S, sizeof(int32_t) * N * c->n);
    ALLOC(c->s2, d * N);
    ALLOC(c->w, d * N * c->n);
    ALLOC(c->q[0], d * N * c->ntr); ALLOC(c->q[1], d * N * c->ntr);
    ALLOC(c->status, sizeof(int) * ST_WORDS);
    if (c->mode == 1) ALLOC(c->cidx, sizeof(int32_t) * N);
#undef ALLOC
    if (e == hipSuccess) e = upload_points(nodes_xyz, N, nodes_on_device, c->nx, c->ny, c->nz, c->stream);
    if (e == hipSuccess) e = grid_build(c->nx, c->ny, c->nz, N, c->n, &c->grid, c->stream);
    if (e == hipSuccess) e = launch_status_reset(c->status, c->stream);
    if (e == hipSuccess && c->mode == 1) {
        // every node's own stencil, found once (the nodes do not move)
        e = launch_knn(c->grid, N, c->nx, c->ny, c->nz, N, c->n, c->S, nullptr, c->s2, c->status, 0, c->stream);
        if (e == hipSuccess && p->cache_factors) {
            // every node's system depends only on the node: factor each once
            c->cached = true;
            const size_t M = (size_t)c->M;
            void **fb[] = {(void **)&c->F, (void **)&c->frinv, (void **)&c->fpiv, (void **)&c->fstep,
                           (void **)&c->fstat};
            const size_t fs[] = {d * N * M * M, d * N * M, sizeof(int32_t) * N * M, sizeof(int32_t) * N * M,
                                 sizeof(int32_t) * N};
            for (int b = 0; b < 5 && e == hipSuccess; ++b) e = hipMalloc(fb[b], fs[b]);
            if (e == hipSuccess) {
                FactorArgs fa{};
                fa.s.nx = c->nx; fa.s.ny = c->ny; fa.s.nz = c->nz; fa.s.N = N;
                fa.s.ex = c->nx; fa.s.ey = c->ny; fa.s.ez = c->nz;
                fa.s.cx = c->nx; fa.s.cy = c->ny; fa.s.cz = c->nz;
                fa.s.S = c->S; fa.s.s2 = c->s2; fa.s.cidx = nullptr;
                fa.s.count = N; fa.s.n = c->n; fa.s.L = c->L; fa.s.k = c->k;
                fa.s.w = nullptr; fa.s.st_out = nullptr; fa.s.status = c->status; fa.s.step = 0;
                fa.F = c->F; fa.piv = c->fpiv; fa.rinv = c->frinv; fa.stepof = c->fstep; fa.fstat = c->fstat;
                e = launch_factor(fa, c->stream);
            }
        }
        int st[ST_WORDS];
        if (e == hipSuccess) e = hipMemcpyAsync(st, c->status, sizeof st, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess && st[ST_SEARCH]) {
            ctx_free(c);
            delete c;
            return RBFSL_E_SEARCH;
        }
    }
    if (e != hipSuccess) {
        int code = (e == hipErrorOutOfMemory) ? RBFSL_E_NOMEM : RBFSL_E_DEVICE;
        ctx_free(c);
        delete c;
        return code;
    }
    taps_single(c);
    *out = c;
    return RBFSL_OK;
}

int rbfsl_create_pu(const double *nodes_xyz, int64_t N, int nodes_on_device, const double *centers_xyz,
                    int64_t Mp, double R, const rbfsl_params *p, void *hip_stream, rbfsl_ctx **out) {
    if (!out) return RBFSL_E_INVAL;
    *out = nullptr;
    if (!p || !nodes_xyz || !centers_xyz) return RBFSL_E_INVAL;
    if (p->stencil_mode != RBFSL_STENCIL_PU || p->cache_factors != 0 || Mp < 1 || Mp > 0x7fffffffLL ||
        !(R > 0.0) || !(R < 2.0 + 1e-12) || !isfinite(R))
        return RBFSL_E_INVAL;
    rbfsl_params q = *p;
    q.stencil_mode = 0;
    int L, k;
    char msg[256];
    if (validate_params(N, &q, &L, &k, msg, sizeof msg) != RBFSL_OK) return RBFSL_E_INVAL;
    const int mL = (L + 1) * (L + 1);
    rbfsl_ctx *c = new (std::nothrow) rbfsl_ctx();
    if (!c) return RBFSL_E_NOMEM;
    c->p = *p;
    c->p.L = L;
    c->p.k = k;
    c->n = p->n; c->L = L; c->k = k;
    c->ntr = p->n_tracers; c->mode = RBFSL_STENCIL_PU; c->N = N;
    c->Mp = Mp; c->R = R;
    // node lists hold up to ncap nodes (about twice the nominal patch size);
    // a departure point may lie in up to pcap patches: about twice the mean
    // overlap Mp R^2 / 4 (area of the caps over the sphere's) plus 3, 8..32
    c->ncap = (int)std::min<int64_t>(N, std::min<int64_t>(2 * (int64_t)p->n + 64, KNN_CAP));
    const double overlap = (double)Mp * R * R / 4.0;
    c->pcap = (int)std::min<int64_t>(Mp, std::max(8, std::min(32, (int)ceil(2.0 * overlap) + 3)));
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    const size_t d = sizeof(double);
    const int64_t nc = c->ncap;
#define ALLOC(ptr, bytes) if (e == hipSuccess) e = hipMalloc(&(ptr), (bytes))
    ALLOC(c->nx, d * N); ALLOC(c->ny, d * N); ALLOC(c->nz, d * N);
    ALLOC(c->ex, d * N); ALLOC(c->ey, d * N); ALLOC(c->ez, d * N);
    ALLOC(c->cx, d * Mp); ALLOC(c->cy, d * Mp); ALLOC(c->cz, d * Mp);
    ALLOC(c->pidx, sizeof(int32_t) * Mp * nc); ALLOC(c->pd2, d * Mp * nc); ALLOC(c->ploc, d * Mp * nc * 3);
    ALLOC(c->pcnt, sizeof(int32_t) * (Mp + 1)); ALLOC(c->pr2, d * Mp);
    ALLOC(c->sidx, sizeof(int32_t) * N * c->pcap); ALLOC(c->sd2, d * N * c->pcap);
    ALLOC(c->sval, d * N * c->pcap * c->ntr);
    ALLOC(c->q[0], d * N * c->ntr); ALLOC(c->q[1], d * N * c->ntr);
    ALLOC(c->status, sizeof(int) * ST_WORDS);
#undef ALLOC
    int code = RBFSL_OK;
    if (e == hipSuccess) e = upload_points(nodes_xyz, N, nodes_on_device, c->nx, c->ny, c->nz, c->stream);
    if (e == hipSuccess) e = upload_points(centers_xyz, Mp, nodes_on_device, c->cx, c->cy, c->cz, c->stream);
    if (e == hipSuccess) e = grid_build(c->nx, c->ny, c->nz, N, c->ncap, &c->grid, c->stream);
    if (e == hipSuccess) e = grid_build(c->cx, c->cy, c->cz, Mp, c->pcap, &c->cgrid, c->stream);
    if (e == hipSuccess) e = launch_status_reset(c->status, c->stream);
    // each patch: the ncap nodes nearest its centre, the cap's prefix counted
    if (e == hipSuccess)
        e = launch_knn(c->grid, N, c->cx, c->cy, c->cz, Mp, c->ncap, c->pidx, c->pd2, nullptr, c->status, 0,
                       c->stream);
    int *dmax = c->pcnt + Mp;  // scratch word for the largest count
    if (e == hipSuccess) e = hipMemsetAsync(dmax, 0, sizeof(int), c->stream);
    PuArgs a = pu_args(c, 0);
    if (e == hipSuccess) e = launch_pu_count(a, MAX_SYSTEM - mL, c->pcnt, dmax, c->stream);
    int st[ST_WORDS] = {0, 0, 0, NO_FAIL};
    int nmax = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(st, c->status, sizeof st, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&nmax, dmax, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && (st[ST_SEARCH] || nmax < 1 || solve_variant_capacity(nmax + mL) == 0)) code = RBFSL_E_SEARCH;
    if (e == hipSuccess && code == RBFSL_OK) {
        // every patch's system, factored once (slots of the largest system)
        c->nmax = nmax;
        const size_t Ms = (size_t)(nmax + mL);
        void **fb[] = {(void **)&c->F, (void **)&c->frinv, (void **)&c->fpiv, (void **)&c->fstep,
                       (void **)&c->fstat, (void **)&c->coef};
        const size_t fs[] = {d * Mp * Ms * Ms, d * Mp * Ms, sizeof(int32_t) * Mp * Ms, sizeof(int32_t) * Mp * Ms,
                             sizeof(int32_t) * Mp, d * Mp * c->ntr * Ms};
        for (int b = 0; b < 6 && e == hipSuccess; ++b) e = hipMalloc(fb[b], fs[b]);
        std::vector<double> r2((size_t)Mp, R * R);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->pr2, r2.data(), d * Mp, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) {
            FactorArgs fa{};
            fa.s.nx = c->nx; fa.s.ny = c->ny; fa.s.nz = c->nz; fa.s.N = N;
            fa.s.ex = c->cx; fa.s.ey = c->cy; fa.s.ez = c->cz;
            fa.s.cx = c->cx; fa.s.cy = c->cy; fa.s.cz = c->cz;
            fa.s.S = c->pidx; fa.s.s2 = c->pr2; fa.s.cidx = nullptr;
            fa.s.count = Mp; fa.s.n = nmax; fa.s.L = c->L; fa.s.k = c->k;
            fa.s.nvar = c->pcnt; fa.s.sstride = nc;
            fa.s.w = nullptr; fa.s.st_out = nullptr; fa.s.status = c->status; fa.s.step = 0;
            fa.F = c->F; fa.piv = c->fpiv; fa.rinv = c->frinv; fa.stepof = c->fstep; fa.fstat = c->fstat;
            e = launch_factor(fa, c->stream);
        }
        if (e == hipSuccess) e = launch_pu_local(pu_args(c, 0), c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) code = (e == hipErrorOutOfMemory) ? RBFSL_E_NOMEM : RBFSL_E_DEVICE;
    if (code != RBFSL_OK) {
        ctx_free(c);
        delete c;
        return code;
    }
    taps_single(c);
    *out = c;
    return RBFSL_OK;
}

int rbfsl_pu_info(const rbfsl_ctx *c, int64_t *npatch, int32_t *ncap, int32_t *nmax, double *R) {
    if (!c || c->mode != RBFSL_STENCIL_PU) return RBFSL_E_INVAL;
    if (npatch) *npatch = c->Mp;
    if (ncap) *ncap = c->ncap;
    if (nmax) *nmax = c->nmax;
    if (R) *R = c->R;
    return RBFSL_OK;
}

int rbfsl_debug_patches(rbfsl_ctx *c, int32_t *counts, int32_t *idx) {
    if (!c || c->mode != RBFSL_STENCIL_PU || !counts || !idx) return RBFSL_E_INVAL;
    HIP_TRY(c, hipMemcpyAsync(counts, c->pcnt, sizeof(int32_t) * c->Mp, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(idx, c->pidx, sizeof(int32_t) * c->Mp * c->ncap, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RBFSL_OK;
}

int rbfsl_set_q(rbfsl_ctx *c, const double *q, int on_device) {
    if (!c || !q) return RBFSL_E_INVAL;
    HIP_TRY(c, hipMemcpyAsync(c->q[c->cur], q, sizeof(double) * c->N * c->ntr,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->q_set = true;
    return RBFSL_OK;
}

int rbfsl_run(rbfsl_ctx *c, int64_t nsteps) {
    if (!c || nsteps < 0) return RBFSL_E_INVAL;
    if (!c->q_set) return fail(c, RBFSL_E_STATE, "q has not been set");
    if (nsteps == 0) return RBFSL_OK;
    HIP_TRY(c, launch_status_reset(c->status, c->stream));
    const int64_t m0 = c->step;
    const int cur0 = c->cur;
    if (chunked(c, nsteps) && c->ahead_cap == 0) {
        const hipError_t ea = ahead_alloc(c);
        if (ea == hipErrorOutOfMemory) {  // the chunk sets do not fit: step by step from now on
            (void)hipGetLastError();
            c->ahead_off = true;
        } else if (ea != hipSuccess) {
            return fail(c, RBFSL_E_DEVICE, "chunk buffers: %s", hipGetErrorString(ea));
        }
    }
    if (chunked(c, nsteps)) {
        const int64_t K = ahead_steps(c, nsteps);
        // the search stream starts after the status reset
        HIP_TRY(c, hipEventRecord(c->run_start, c->stream));
        HIP_TRY(c, hipStreamWaitEvent(c->sstream, c->run_start, 0));
        int64_t m = m0;
        const hipError_t e = enqueue_chunks(c, m0, nsteps, K, cur0, &m);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(c->sstream);
            (void)hipStreamSynchronize(c->wstream);
            (void)hipStreamSynchronize(c->stream);
            c->cur = cur0;
            return fail(c, RBFSL_E_DEVICE, "steps %lld.. launch: %s", (long long)m, hipGetErrorString(e));
        }
    } else {
        taps_single(c);
        for (int64_t m = m0; m < m0 + nsteps; ++m) {
            c->cur = cur0 ^ (int)((m - m0) & 1);  // buffer holding q^m
            hipError_t e = enqueue_step(c, m);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(c->stream);
                c->cur = cur0;
                return fail(c, RBFSL_E_DEVICE, "step %lld launch: %s", (long long)m, hipGetErrorString(e));
            }
        }
    }
    int st[ST_WORDS];
    int r = read_status(c, st);
    if (r != RBFSL_OK) {
        c->cur = cur0;
        return r;
    }
    prof_collect(c);
    c->ran = true;
    c->f_sing = st[ST_SINGULAR];
    c->f_nonf = st[ST_NONFINITE];
    c->f_search = st[ST_SEARCH];
    if (st[ST_FAILSTEP] != NO_FAIL) {
        // steps f, f+1, ... did nothing: the state is q^f
        const int64_t f = st[ST_FAILSTEP];
        c->cur = cur0 ^ (int)((f - m0) & 1);
        c->step = f;
        return fail(c, status_code(st), "step %lld: %d singular, %d non-finite, %d search failures",
                    (long long)f, st[ST_SINGULAR], st[ST_NONFINITE], st[ST_SEARCH]);
    }
    c->cur = cur0 ^ (int)(nsteps & 1);
    c->step = m0 + nsteps;
    return RBFSL_OK;
}

int rbfsl_step(rbfsl_ctx *c) { return rbfsl_run(c, 1); }

int64_t rbfsl_steps_per_launch(const rbfsl_ctx *c, int64_t nsteps) {
    if (!c || nsteps < 1) return 1;
    return ahead_steps(c, nsteps);
}

int rbfsl_get_q(rbfsl_ctx *c, double *out, int on_device) {
    if (!c || !out) return RBFSL_E_INVAL;
    if (!c->q_set) return fail(c, RBFSL_E_STATE, "q has not been set");
    HIP_TRY(c, hipMemcpyAsync(out, c->q[c->cur], sizeof(double) * c->N * c->ntr,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RBFSL_OK;
}

int rbfsl_get_state(const rbfsl_ctx *c, int64_t *step, double *t) {
    if (!c) return RBFSL_E_INVAL;
    if (step) *step = c->step;
    if (t) *t = c->p.t0 + (double)c->step * c->p.dt;
    return RBFSL_OK;
}

int rbfsl_get_failures(const rbfsl_ctx *c, int64_t *singular, int64_t *nonfinite, int64_t *search) {
    if (!c) return RBFSL_E_INVAL;
    if (singular) *singular = c->f_sing;
    if (nonfinite) *nonfinite = c->f_nonf;
    if (search) *search = c->f_search;
    return RBFSL_OK;
}

int rbfsl_profile(rbfsl_ctx *c, int enable) {
    if (!c) return RBFSL_E_INVAL;
    c->prof = enable != 0;
    c->ev_used = 0;
    c->prof_steps = 0;
    for (double &v : c->prof_ms) v = 0.0;
    return RBFSL_OK;
}

int rbfsl_phase_times(rbfsl_ctx *c, double *ms, int64_t *steps) {
    if (!c || !ms) return RBFSL_E_INVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    for (int i = 0; i < 4; ++i) ms[i] = c->prof_ms[i];
    if (steps) *steps = c->prof_steps;
    return RBFSL_OK;
}

int rbfsl_debug_departure(rbfsl_ctx *c, double *xi) {
    if (!c || !xi) return RBFSL_E_INVAL;
    if (!c->ran) return fail(c, RBFSL_E_STATE, "no step has run");
    HIP_TRY(c, download_points(c->tex, c->tey, c->tez, c->N, xi, c->stream));
    return RBFSL_OK;
}

int rbfsl_debug_stencils(rbfsl_ctx *c, int32_t *idx) {
    if (!c || !idx || c->mode == RBFSL_STENCIL_PU) return RBFSL_E_INVAL;
    if (!c->ran) return fail(c, RBFSL_E_STATE, "no step has run");
    const size_t bytes = sizeof(int32_t) * c->N * c->n;
    if (c->mode == 0) {
        HIP_TRY(c, hipMemcpyAsync(idx, c->tS, bytes, hipMemcpyDeviceToHost, c->stream));
    } else {
        int32_t *tmp = nullptr;
        HIP_TRY(c, hipMalloc(&tmp, bytes));
        hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((c->N * c->n + 255) / 256)), dim3(256), 0,
                           c->stream, c->tS, c->tcidx, c->N, c->n, tmp);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(idx, tmp, bytes, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return fail(c, RBFSL_E_DEVICE, "stencil gather: %s", hipGetErrorString(e));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RBFSL_OK;
}

int rbfsl_debug_weights(rbfsl_ctx *c, double *w) {
    if (!c || !w || c->mode == RBFSL_STENCIL_PU) return RBFSL_E_INVAL;
    if (!c->ran) return fail(c, RBFSL_E_STATE, "no step has run");
    HIP_TRY(c, hipMemcpyAsync(w, c->tw, sizeof(double) * c->N * c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RBFSL_OK;
}

int rbfsl_debug_sample(rbfsl_ctx *c, const int64_t *jl, int64_t J, double *xi, int32_t *idx, double *w) {
    if (!c || J < 0 || (J > 0 && !jl)) return RBFSL_E_INVAL;
    if ((idx || w) && c->mode == RBFSL_STENCIL_PU) return RBFSL_E_INVAL;
    if (!c->ran) return fail(c, RBFSL_E_STATE, "no step has run");
    for (int64_t t = 0; t < J; ++t)
        if (jl[t] < 0 || jl[t] >= c->N) return fail(c, RBFSL_E_INVAL, "node index %lld out of range", (long long)jl[t]);
    if (J == 0) return RBFSL_OK;
    const size_t d = sizeof(double), nn = (size_t)c->n;
    int64_t *djl = nullptr;
    double *dxi = nullptr, *dw = nullptr;
    int32_t *dS = nullptr;
    hipError_t e = hipMalloc(&djl, sizeof(int64_t) * J);
    if (e == hipSuccess) e = hipMalloc(&dxi, d * 3 * J);
    if (e == hipSuccess && idx) e = hipMalloc(&dS, sizeof(int32_t) * J * nn);
    if (e == hipSuccess && w) e = hipMalloc(&dw, d * J * nn);
    if (e == hipSuccess) e = hipMemcpyAsync(djl, jl, sizeof(int64_t) * J, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gather_sample, dim3((unsigned)J), dim3(64), 0, c->stream, djl, J, c->tex, c->tey,
                           c->tez, c->tS, c->mode == 1 ? c->tcidx : nullptr, c->tw, c->n, dxi, dS, dw);
        e = hipGetLastError();
    }
    if (e == hipSuccess && xi) e = hipMemcpyAsync(xi, dxi, d * 3 * J, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && idx) e = hipMemcpyAsync(idx, dS, sizeof(int32_t) * J * nn, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && w) e = hipMemcpyAsync(w, dw, d * J * nn, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    void *bufs[] = {djl, dxi, dS, dw};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (e != hipSuccess) return fail(c, RBFSL_E_DEVICE, "sample gather: %s", hipGetErrorString(e));
    return RBFSL_OK;
}

#ifndef RBFSL_SOURCE_HASH
#define RBFSL_SOURCE_HASH "unknown"
#endif
const char *rbfsl_source_hash(void) { return RBFSL_SOURCE_HASH; }

void rbfsl_destroy(rbfsl_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    ctx_free(c);
    delete c;
}

int rbfsl_knn(const double *nodes_xyz, int64_t N, const double *queries, int64_t Q, int32_t n,
              int32_t *idx, double *d2, int on_device, void *hip_stream) {
    if (!nodes_xyz || !queries || !idx || N < 1 || N > 0x7fffffffLL || Q < 0 || n < 1 || n > N ||
        n > KNN_CAP)
        return RBFSL_E_INVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t d = sizeof(double);
    double *nx = nullptr, *ny = nullptr, *nz = nullptr, *qx = nullptr, *qy = nullptr, *qz = nullptr, *dd = nullptr;
    int32_t *ii = nullptr;
    int *status = nullptr;
    Grid g;
    int code = RBFSL_OK;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes) if (e == hipSuccess) e = hipMalloc(&(ptr), (bytes))
    ALLOC(nx, d * N); ALLOC(ny, d * N); ALLOC(nz, d * N);
    ALLOC(qx, d * (Q + 1)); ALLOC(qy, d * (Q + 1)); ALLOC(qz, d * (Q + 1));
    ALLOC(ii, sizeof(int32_t) * (Q * n + 1));
    ALLOC(dd, d * (Q * n + 1));
    ALLOC(status, sizeof(int) * ST_WORDS);
#undef ALLOC
    if (e == hipSuccess) e = upload_points(nodes_xyz, N, on_device, nx, ny, nz, s);
    if (e == hipSuccess) e = upload_points(queries, Q, on_device, qx, qy, qz, s);
    if (e == hipSuccess) e = grid_build(nx, ny, nz, N, n, &g, s);
    if (e == hipSuccess) e = launch_status_reset(status, s);
    if (e == hipSuccess) e = launch_knn(g, N, qx, qy, qz, Q, n, ii, dd, nullptr, status, 0, s);
    int st[ST_WORDS] = {0, 0, 0, NO_FAIL};
    if (e == hipSuccess) e = hipMemcpyAsync(st, status, sizeof st, hipMemcpyDeviceToHost, s);
    const hipMemcpyKind out = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (e == hipSuccess && Q > 0) e = hipMemcpyAsync(idx, ii, sizeof(int32_t) * Q * n, out, s);
    if (e == hipSuccess && Q > 0 && d2) e = hipMemcpyAsync(d2, dd, d * Q * n, out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) code = (e == hipErrorOutOfMemory) ? RBFSL_E_NOMEM : RBFSL_E_DEVICE;
    else if (st[ST_SEARCH]) code = RBFSL_E_SEARCH;
    void *bufs[] = {nx, ny, nz, qx, qy, qz, ii, dd, status};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    grid_free(&g);
    return code;
}

int rbfsl_weights(const double *nodes_xyz, int64_t N, const int32_t *idx, const double *centers,
                  const double *s2, const double *evals, int64_t count, int32_t n, int32_t L,
                  int32_t k, double *w, int32_t *status_out, int on_device, void *hip_stream) {
    if (!nodes_xyz || !idx || !centers || !s2 || !evals || !w || N < 1 || count < 0) return RBFSL_E_INVAL;
    int Lr, kr;
    char msg[256];
    if (resolve_nlk(N, n, L, k, &Lr, &kr, msg, sizeof msg) != RBFSL_OK) return RBFSL_E_INVAL;
    if (count == 0) return RBFSL_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t d = sizeof(double);
    const hipMemcpyKind in = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    double *nx = nullptr, *ny = nullptr, *nz = nullptr, *cx = nullptr, *cy = nullptr, *cz = nullptr;
    double *ex = nullptr, *ey = nullptr, *ez = nullptr, *ss = nullptr, *ww = nullptr;
    int32_t *SS = nullptr, *so = nullptr;
    int *status = nullptr;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes) if (e == hipSuccess) e = hipMalloc(&(ptr), (bytes))
    ALLOC(nx, d * N); ALLOC(ny, d * N); ALLOC(nz, d * N);
    ALLOC(cx, d * count); ALLOC(cy, d * count); ALLOC(cz, d * count);
    ALLOC(ex, d * count); ALLOC(ey, d * count); ALLOC(ez, d * count);
    ALLOC(ss, d * count); ALLOC(ww, d * count * n);
    ALLOC(SS, sizeof(int32_t) * count * n); ALLOC(so, sizeof(int32_t) * count);
    ALLOC(status, sizeof(int) * ST_WORDS);
#undef ALLOC
    if (e == hipSuccess) e = upload_points(nodes_xyz, N, on_device, nx, ny, nz, s);
    if (e == hipSuccess) e = upload_points(centers, count, on_device, cx, cy, cz, s);
    if (e == hipSuccess) e = upload_points(evals, count, on_device, ex, ey, ez, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ss, s2, d * count, in, s);
    if (e == hipSuccess) e = hipMemcpyAsync(SS, idx, sizeof(int32_t) * count * n, in, s);
    if (e == hipSuccess) e = launch_status_reset(status, s);
    if (e == hipSuccess) {
        SolveArgs a{};
        a.nx = nx; a.ny = ny; a.nz = nz; a.N = N;
        a.ex = ex; a.ey = ey; a.ez = ez;
        a.cx = cx; a.cy = cy; a.cz = cz;
        a.S = SS; a.s2 = ss; a.cidx = nullptr;
        a.count = count; a.n = n; a.L = Lr; a.k = kr;
        a.w = ww; a.st_out = so; a.status = status; a.step = 0;
        e = launch_solve(a, s);
    }
    const hipMemcpyKind out = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (e == hipSuccess) e = hipMemcpyAsync(w, ww, d * count * n, out, s);
    if (e == hipSuccess && status_out) e = hipMemcpyAsync(status_out, so, sizeof(int32_t) * count, out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int code = RBFSL_OK;
    if (e != hipSuccess) code = (e == hipErrorOutOfMemory) ? RBFSL_E_NOMEM : RBFSL_E_DEVICE;
    void *bufs[] = {nx, ny, nz, cx, cy, cz, ex, ey, ez, ss, ww, SS, so, status};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    return code;
}

}  // extern "C"

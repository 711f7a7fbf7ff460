/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the local-stencil RBF
 * semi-Lagrangian transport step of Shankar & Wright, "Mesh-free
 * semi-Lagrangian methods for transport on a sphere using radial basis
 * functions" (arXiv:1804.01609).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, import or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP implementation.
 *
 * What it computes, per time step m -> m+1 (Algorithm 1, Section 3):
 *   1. departure points: the trajectory ODE (eq. sl_ode, Section 3.2) solved
 *      backward over [t_m, t_{m+1}] with classical RK4 or Fehlberg's RK5,
 *      projecting every stage point and the result orthogonally back onto
 *      the unit sphere;
 *   2. stencils: the n nearest nodes of each departure point, by brute force
 *      (all N keys formed, the n smallest kept);  the kd-tree of Section 2.2
 *      only accelerates this;
 *   3. the augmented local interpolant (eq. rbf_poly) with PHS phi = r^(2k+1)
 *      (Section 2.4) and the degree-L spherical-harmonic space, whose moment
 *      conditions give the saddle-point system (eq. rbf_poly_linsys);
 *   4. that system solved by Gaussian elimination with partial pivoting (the
 *      LU route of Section 3.3.2);
 *   5. q^{m+1}_j = s(xi_j), evaluated in cardinal form as sum_a w_a q_a.
 * and, as the second interpolation method of Section 3.3, the RBF-PU step:
 * the augmented interpolants of the patches (spherical caps) solved for the
 * right-hand side [q; 0] and blended with the B-spline partition of unity
 * at every departure point (the functions orc_bspline ... orc_pu_step).
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - the basis of the degree-L harmonic space is the graded local basis
 *     H_m(alpha,beta) u^i (m+i <= L) in a frame centred on the stencil centre;
 *     it spans exactly the same space as the spherical harmonics of degree
 *     <= L, so the weights are the same; the PHS block is evaluated on
 *     coordinates scaled by 1/s, which leaves the weights unchanged because
 *     r^(2k+1) is homogeneous;
 *   - the cardinal weights w = first n entries of inv(A~) [b; p(xi)], which by
 *     the symmetry of A~ equal the paper's "solve for coefficients, then
 *     evaluate" route;
 *   - GE pivot: largest |a_ik| over rows not yet used, ties to the lowest row
 *     index; rows are not moved (implicit pivoting);  multipliers a_ik * r with
 *     r = 1/a_pk;  updates a_ij = fma(-l, a_pj, a_ij);  back substitution
 *     column by column from the last unknown, z_k = y_k * r_k.
 * Every floating-point expression is written with its evaluation order made
 * explicit and is compiled with -ffp-contract=off; fma() appears only where
 * a fused multiply-add is meant.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_SINGULAR 1
#define ORC_NONFINITE 2
#define ORC_INVAL 3

#define VEL_ZERO 0
#define VEL_SOLID 1
#define VEL_DEFORM 2
#define VEL_NL2010 3

#define INT_RK4 0
#define INT_RK5F 1

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads used by later parallel regions (timing on one core or all) */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Velocity fields (Section 4.1 solid body; the time-reversing stream-       */
/* function flow of the transport problem).                                   */
/*                                                                            */
/* vp[0] = T (period), vp[1..3] = unit rotation axis a, vp[4] = amplitude kap */
/*   solid body:   u(x)   = Omega a x x,                  Omega = 2 pi / T    */
/*   deformation:  u(x,t) = kap cos(pi t/T) R(t) u0(R(t)^T x) + Omega a x x   */
/*                 R(t) = rotation about a by Omega t,                        */
/*                 u0(y) = y x grad psi0(y),  psi0 = y0 y1 y2 + y2^2 y0 / 2   */
/*   NL2010 deformational flow (Section 4.2), given there in longitude /      */
/*   latitude components with T = vp[0], Omega = 2 pi / T,                   */
/*   lambda' = lambda - Omega t:                                              */
/*     u_lambda = (10/T) cos(pi t/T) sin^2(lambda') sin(2 theta)              */
/*                + Omega cos(theta)                                          */
/*     u_theta  = (10/T) cos(pi t/T) sin(2 lambda') cos(theta)                */
/*   (the printed u_theta has sin(2 lambda - Omega t); read as sin(2 lambda'),*/
/*   the cited test case's form: only then is the flow divergence free and    */
/*   time independent in the rotating frame up to cos(pi t/T), so that it     */
/*   returns every parcel at t = T as the section states).  Cartesian form    */
/*   (x on the unit sphere, rho^2 = x^2 + y^2, e_lambda = (-y, x, 0)/rho,     */
/*   e_theta = (-z x, -z y, rho^2)/rho):                                      */
/*     u = A (-y, x, 0) + B (-z x, -z y, rho^2) + Omega e_z x x,              */
/*     s1 = y cos(Omega t) - x sin(Omega t)   (= rho sin lambda'),            */
/*     c1 = x cos(Omega t) + y sin(Omega t)   (= rho cos lambda'),            */
/*     A = c 2z s1^2 / rho^2,  B = c 2 s1 c1 / rho^2,                         */
/*     c = (10/T) cos(pi t/T).                                                */
/* ------------------------------------------------------------------------ */

/* libm cos and sin, each called on its own: a compiler may otherwise merge a
 * cos/sin pair into one sincos() call, whose last bit can differ */
static __attribute__((noinline)) double cos_of(double x) { return cos(x); }
static __attribute__((noinline)) double sin_of(double x) { return sin(x); }

typedef struct {
    double c;      /* time factor of the deformation part */
    double R[9];   /* row-major rotation matrix R(t) */
    double w[3];   /* angular velocity Omega a */
    double cw, sw; /* NL2010: cos and sin of Omega t */
} vel_coef;

static void vel_coef_at(int vel_id, const double *vp, double t, vel_coef *vc) {
    memset(vc, 0, sizeof(*vc));
    vc->R[0] = 1.0; vc->R[4] = 1.0; vc->R[8] = 1.0;
    if (vel_id == VEL_ZERO) return;
    double T = vp[0];
    double a[3] = {vp[1], vp[2], vp[3]};
    double Om = (2.0 * M_PI) / T;
    if (vel_id == VEL_NL2010) {
        vc->w[2] = Om;
        vc->c = (10.0 / T) * cos_of((M_PI * t) / T);
        vc->cw = cos_of(Om * t);
        vc->sw = sin_of(Om * t);
        return;
    }
    vc->w[0] = Om * a[0];
    vc->w[1] = Om * a[1];
    vc->w[2] = Om * a[2];
    if (vel_id != VEL_DEFORM) return;
    double th = Om * t;
    double ct = cos_of(th), st = sin_of(th);
    double omc = 1.0 - ct;
    /* Rodrigues: R = cos I + sin [a]x + (1 - cos) a a^T, term by term */
    double K[9] = {0.0, -a[2], a[1],
                   a[2], 0.0, -a[0],
                   -a[1], a[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double d = (i == j) ? 1.0 : 0.0;
            vc->R[3 * i + j] = ((ct * d) + (st * K[3 * i + j])) + (omc * (a[i] * a[j]));
        }
    vc->c = vp[4] * cos_of((M_PI * t) / T);
}

static void cross(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* u0(y) = y x grad psi0(y) */
static void u0_deform(const double y[3], double u[3]) {
    double g[3];
    g[0] = y[1] * y[2] + 0.5 * (y[2] * y[2]);
    g[1] = y[0] * y[2];
    g[2] = y[0] * y[1] + y[2] * y[0];
    cross(y, g, u);
}

static void velocity(int vel_id, const vel_coef *vc, const double x[3], double u[3]) {
    if (vel_id == VEL_ZERO) { u[0] = u[1] = u[2] = 0.0; return; }
    double wx[3];
    cross(vc->w, x, wx);
    if (vel_id == VEL_SOLID) { u[0] = wx[0]; u[1] = wx[1]; u[2] = wx[2]; return; }
    if (vel_id == VEL_NL2010) {
        double rho2 = x[0] * x[0] + x[1] * x[1];
        double s1 = x[1] * vc->cw - x[0] * vc->sw;
        double c1 = x[0] * vc->cw + x[1] * vc->sw;
        double A = (vc->c * ((2.0 * x[2]) * (s1 * s1))) / rho2;
        double B = (vc->c * ((2.0 * s1) * c1)) / rho2;
        u[0] = (-(A * x[1]) - B * (x[2] * x[0])) + wx[0];
        u[1] = (A * x[0] - B * (x[2] * x[1])) + wx[1];
        u[2] = B * rho2 + wx[2];
        return;
    }
    const double *R = vc->R;
    double y[3], v[3];
    for (int i = 0; i < 3; ++i)  /* y = R^T x */
        y[i] = (R[0 * 3 + i] * x[0] + R[1 * 3 + i] * x[1]) + R[2 * 3 + i] * x[2];
    u0_deform(y, v);
    for (int i = 0; i < 3; ++i) {  /* u = c R v + w x x */
        double rv = (R[3 * i + 0] * v[0] + R[3 * i + 1] * v[1]) + R[3 * i + 2] * v[2];
        u[i] = vc->c * rv + wx[i];
    }
}

void orc_velocity(int vel_id, const double *vp, double t, const double *x, double *u) {
    vel_coef vc;
    vel_coef_at(vel_id, vp, t, &vc);
    velocity(vel_id, &vc, x, u);
}

/* orthogonal projection onto the unit sphere */
static void project(double v[3]) {
    double nn = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    double r = sqrt(nn);
    v[0] = v[0] / r;
    v[1] = v[1] / r;
    v[2] = v[2] / r;
}

/* Fehlberg's fifth-order Runge-Kutta formula (the higher-order member of
 * his 4(5) pair, the integrator the paper settles on in Section 3.2): stage
 * fractions c_s, coefficients a_sj and fifth-order weights b_j, each written
 * as the rational number it is. */
static const double RKF_C[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
static const double RKF_A[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 4.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 32.0, 9.0 / 32.0, 0.0, 0.0, 0.0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0.0, 0.0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0.0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
static const double RKF_B[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0,
                                2.0 / 55.0};

/* velocity coefficients of every stage time of step m -> m+1 */
typedef struct {
    int rk;
    vel_coef v[6];
} step_coefs;

static void step_coefs_at(int vel_id, const double *vp, int rk, double t0, double dt, int64_t m,
                          step_coefs *sc) {
    double t1 = t0 + (double)(m + 1) * dt;
    sc->rk = rk;
    if (rk == INT_RK4) {
        vel_coef_at(vel_id, vp, t1, &sc->v[0]);
        vel_coef_at(vel_id, vp, t1 - 0.5 * dt, &sc->v[1]);
        vel_coef_at(vel_id, vp, t0 + (double)m * dt, &sc->v[2]);
    } else {
        double h = -dt;
        for (int st = 0; st < 6; ++st) vel_coef_at(vel_id, vp, t1 + RKF_C[st] * h, &sc->v[st]);
    }
}

/* Departure point of node x for step m -> m+1: eq. sl_ode backward over
 * [t_m, t_{m+1}] (h = -dt from t_{m+1}), with classical RK4 or Fehlberg's
 * RK5, every stage point and the result projected onto the sphere. */
static void departure(int vel_id, const step_coefs *sc, double dt, const double x[3], double xi[3]) {
    double h = -dt;
    if (sc->rk == INT_RK4) {
        double hh = 0.5 * h, h6 = h / 6.0;
        double k1[3], k2[3], k3[3], k4[3], y[3];
        velocity(vel_id, &sc->v[0], x, k1);
        for (int i = 0; i < 3; ++i) y[i] = x[i] + hh * k1[i];
        project(y);
        velocity(vel_id, &sc->v[1], y, k2);
        for (int i = 0; i < 3; ++i) y[i] = x[i] + hh * k2[i];
        project(y);
        velocity(vel_id, &sc->v[1], y, k3);
        for (int i = 0; i < 3; ++i) y[i] = x[i] + h * k3[i];
        project(y);
        velocity(vel_id, &sc->v[2], y, k4);
        for (int i = 0; i < 3; ++i) {
            double s = ((k1[i] + 2.0 * k2[i]) + 2.0 * k3[i]) + k4[i];
            xi[i] = x[i] + h6 * s;
        }
        project(xi);
        return;
    }
    double k[6][3], y[3];
    velocity(vel_id, &sc->v[0], x, k[0]);
    for (int st = 1; st < 6; ++st) {
        for (int i = 0; i < 3; ++i) {
            double acc = RKF_A[st][0] * k[0][i];
            for (int j = 1; j < st; ++j) acc = acc + RKF_A[st][j] * k[j][i];
            y[i] = x[i] + h * acc;
        }
        project(y);
        velocity(vel_id, &sc->v[st], y, k[st]);
    }
    for (int i = 0; i < 3; ++i) {
        double acc = RKF_B[0] * k[0][i];
        for (int j = 1; j < 6; ++j) acc = acc + RKF_B[j] * k[j][i];
        xi[i] = x[i] + h * acc;
    }
    project(xi);
}

void orc_trace(int64_t N, const double *nodes, int vel_id, const double *vp, int rk,
               double t0, double dt, int64_t m, double *xi) {
    step_coefs sc;
    step_coefs_at(vel_id, vp, rk, t0, dt, m, &sc);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) departure(vel_id, &sc, dt, nodes + 3 * j, xi + 3 * j);
}

/* ------------------------------------------------------------------------ */
/* Brute-force nearest neighbours (stencils X_k, Section 2.2).               */
/* Key of node i for query q: (d2, i) with d2 = (dx*dx + dy*dy) + dz*dz.     */
/* ------------------------------------------------------------------------ */

typedef struct { double d2; int32_t i; } key_t_;

static int key_cmp(const void *pa, const void *pb) {
    const key_t_ *a = (const key_t_ *)pa, *b = (const key_t_ *)pb;
    if (a->d2 < b->d2) return -1;
    if (a->d2 > b->d2) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

static double dist2(const double *x, const double *q) {
    double d0 = x[0] - q[0], d1 = x[1] - q[1], d2 = x[2] - q[2];
    return (d0 * d0 + d1 * d1) + d2 * d2;
}

static int key_less(const key_t_ *a, const key_t_ *b) { return key_cmp(a, b) < 0; }

/* restore the max-heap order of h[0..cnt) below position r (the largest key
 * at the root) */
static void heap_sift_down(key_t_ *h, int cnt, int r) {
    for (;;) {
        int c = 2 * r + 1;
        if (c >= cnt) return;
        if (c + 1 < cnt && key_less(&h[c], &h[c + 1])) c = c + 1;
        if (!key_less(&h[r], &h[c])) return;
        key_t_ t = h[r]; h[r] = h[c]; h[c] = t;
        r = c;
    }
}

/* The n smallest of all N keys (d2, i), in ascending key order.  Brute force:
 * every key is formed; a max-heap keeps the n smallest seen so far (a key
 * enters when it is smaller than the largest kept one), and the kept keys are
 * sorted at the end.  The keys are all distinct (distinct i), so the result
 * is the first n entries of the fully sorted key list. */
static void knn_one(int64_t N, const double *nodes, const double *q, int n, key_t_ *heap,
                    int32_t *idx, double *d2) {
    int cnt = 0;
    for (int64_t i = 0; i < N; ++i) {
        key_t_ k;
        k.d2 = dist2(nodes + 3 * i, q);
        k.i = (int32_t)i;
        if (cnt < n) {
            /* grow the heap: put k last and move it up to its place */
            int c = cnt++;
            heap[c] = k;
            while (c > 0 && key_less(&heap[(c - 1) / 2], &heap[c])) {
                key_t_ t = heap[c]; heap[c] = heap[(c - 1) / 2]; heap[(c - 1) / 2] = t;
                c = (c - 1) / 2;
            }
        } else if (key_less(&k, &heap[0])) {
            heap[0] = k;
            heap_sift_down(heap, cnt, 0);
        }
    }
    qsort(heap, (size_t)cnt, sizeof(key_t_), key_cmp);
    for (int a = 0; a < n; ++a) {
        idx[a] = heap[a].i;
        if (d2) d2[a] = heap[a].d2;
    }
}

void orc_knn(int64_t N, const double *nodes, int64_t Q, const double *queries, int n,
             int32_t *idx, double *d2) {
#pragma omp parallel
    {
        key_t_ *scratch = (key_t_ *)malloc(sizeof(key_t_) * (size_t)N);
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < Q; ++q)
            knn_one(N, nodes, queries + 3 * q, n, scratch, idx + (int64_t)n * q, d2 ? d2 + (int64_t)n * q : NULL);
        free(scratch);
    }
}

/* ------------------------------------------------------------------------ */
/* Gaussian elimination with partial pivoting (Section 3.3.2: LU, because   */
/* the augmented PHS matrix is not positive definite).                       */
/* A is M x M row-major and is overwritten; rhs (M) is overwritten by z.     */
/* ------------------------------------------------------------------------ */

int orc_gauss_solve(int M, double *A, double *rhs) {
    int *used = (int *)calloc((size_t)M, sizeof(int));
    int *piv = (int *)malloc(sizeof(int) * (size_t)M);
    double *rinv = (double *)malloc(sizeof(double) * (size_t)M);
    double *z = (double *)malloc(sizeof(double) * (size_t)M);
    int status = ORC_OK;
    for (int k = 0; k < M && status == ORC_OK; ++k) {
        int p = -1;
        double best = -1.0;
        for (int i = 0; i < M; ++i) {
            if (used[i]) continue;
            double v = fabs(A[(int64_t)i * M + k]);
            if (v > best) { best = v; p = i; }
        }
        if (!(best > 0.0)) { status = ORC_SINGULAR; break; }
        used[p] = 1;
        piv[k] = p;
        double r = 1.0 / A[(int64_t)p * M + k];
        rinv[k] = r;
        const double *ap = A + (int64_t)p * M;
        for (int i = 0; i < M; ++i) {
            if (used[i]) continue;
            double *ai = A + (int64_t)i * M;
            double l = ai[k] * r;
            for (int j = k + 1; j < M; ++j) ai[j] = fma(-l, ap[j], ai[j]);
            rhs[i] = fma(-l, rhs[p], rhs[i]);
        }
    }
    if (status == ORC_OK) {
        /* back substitution, unknown k from the last one down; rows are
         * addressed through the pivot order */
        for (int k = M - 1; k >= 0; --k) {
            double zk = rhs[piv[k]] * rinv[k];
            z[k] = zk;
            for (int kk = 0; kk < k; ++kk) {
                int i = piv[kk];
                rhs[i] = fma(-A[(int64_t)i * M + k], zk, rhs[i]);
            }
        }
        for (int k = 0; k < M; ++k) {
            rhs[k] = z[k];
            if (!isfinite(z[k])) status = ORC_NONFINITE;
        }
    }
    free(used); free(piv); free(rinv); free(z);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Assembly of the augmented local system (eq. rbf_poly_linsys).             */
/* ------------------------------------------------------------------------ */

/* phi(r) = r^(2k+1) from r^2: r = sqrt(r2); then k multiplications by r2 */
static double phs(double r2, int k) {
    double p = sqrt(r2);
    for (int t = 0; t < k; ++t) p = p * r2;
    return p;
}

/* local frame at centre c: e1 from the coordinate axis with the smallest
 * |c_i| (ties to the lowest i), projected onto the tangent plane and
 * normalised; e2 = c x e1 */
static void frame(const double c[3], double e1[3], double e2[3]) {
    int im = 0;
    double am = fabs(c[0]);
    for (int i = 1; i < 3; ++i)
        if (fabs(c[i]) < am) { am = fabs(c[i]); im = i; }
    double t = c[im];
    for (int i = 0; i < 3; ++i) e1[i] = (i == im) ? (1.0 - t * c[i]) : (0.0 - t * c[i]);
    project(e1);
    cross(c, e1, e2);
}

/* local coordinates of point x: y = (x - c)/s, alpha = e1.y, beta = e2.y,
 * u = -(c.y)/s */
static void local_coords(const double x[3], const double c[3], const double e1[3],
                         const double e2[3], double inv_s, double y[3], double *al,
                         double *be, double *u) {
    for (int i = 0; i < 3; ++i) y[i] = (x[i] - c[i]) * inv_s;
    *al = (e1[0] * y[0] + e1[1] * y[1]) + e1[2] * y[2];
    *be = (e2[0] * y[0] + e2[1] * y[1]) + e2[2] * y[2];
    double g = (c[0] * y[0] + c[1] * y[1]) + c[2] * y[2];
    *u = -(g * inv_s);
}

/* the (L+1)^2 basis values at (alpha, beta, u): for m = 0..L, sigma = cos
 * (and sin for m > 0), i = 0..L-m: H^sigma_m(alpha, beta) * u^i, where
 * H_m = Re/Im (alpha + i beta)^m by the recurrence
 * H_m = (alpha Hc - beta Hs, alpha Hs + beta Hc) */
static void basis(int L, double al, double be, double u, double *out) {
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

/* Assemble A~ (M x M row-major) and the right-hand side [b; p(xi)] for one
 * stencil.  xs: n x 3 stencil nodes in stencil order; c: centre; s2: squared
 * scale; xi: evaluation point. */
void orc_assemble(int n, int L, int k, const double *xs, const double *c, double s2,
                  const double *xi, double *A, double *rhs) {
    int mL = (L + 1) * (L + 1);
    int M = n + mL;
    double s = (s2 > 0.0) ? sqrt(s2) : 1.0;
    double inv_s = 1.0 / s;
    double e1[3], e2[3];
    frame(c, e1, e2);
    double *y = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *P = (double *)malloc(sizeof(double) * (size_t)n * (size_t)mL);
    for (int a = 0; a < n; ++a) {
        double al, be, u;
        local_coords(xs + 3 * a, c, e1, e2, inv_s, y + 3 * a, &al, &be, &u);
        basis(L, al, be, u, P + (int64_t)a * mL);
    }
    double yx[3], alx, bex, ux;
    local_coords(xi, c, e1, e2, inv_s, yx, &alx, &bex, &ux);
    memset(A, 0, sizeof(double) * (size_t)M * (size_t)M);
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) {
            double d0 = y[3 * a] - y[3 * b], d1 = y[3 * a + 1] - y[3 * b + 1], d2 = y[3 * a + 2] - y[3 * b + 2];
            A[(int64_t)a * M + b] = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
        }
        for (int q = 0; q < mL; ++q) {
            A[(int64_t)a * M + n + q] = P[(int64_t)a * mL + q];
            A[(int64_t)(n + q) * M + a] = P[(int64_t)a * mL + q];
        }
        double d0 = y[3 * a] - yx[0], d1 = y[3 * a + 1] - yx[1], d2 = y[3 * a + 2] - yx[2];
        rhs[a] = phs((d0 * d0 + d1 * d1) + d2 * d2, k);
    }
    basis(L, alx, bex, ux, rhs + n);
    free(y);
    free(P);
}

/* weights of one stencil; returns ORC_* status */
int orc_weights(int n, int L, int k, const double *xs, const double *c, double s2,
                const double *xi, double *w) {
    int M = n + (L + 1) * (L + 1);
    double *A = (double *)malloc(sizeof(double) * (size_t)M * (size_t)M);
    double *r = (double *)malloc(sizeof(double) * (size_t)M);
    orc_assemble(n, L, k, xs, c, s2, xi, A, r);
    int st = orc_gauss_solve(M, A, r);
    for (int a = 0; a < n; ++a) w[a] = r[a];
    free(A);
    free(r);
    return st;
}

/* ------------------------------------------------------------------------ */
/* One SL step for a set of target nodes (Algorithm 1 + Section 3.3.2).      */
/* mode 0: stencil = n nearest nodes of xi_j, centre xi_j.                   */
/* mode 1: K = nearest node of xi_j; stencil = n nearest nodes of x_K,       */
/*         centre x_K (the paper's centre-point stencils).                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, L, k, mode, vel_id, ntr;
    int rk; /* INT_RK4 or INT_RK5F */
    int reserved;
    double vp[8];
    double dt, t0;
} orc_params;

static int step_one(int64_t N, const double *nodes, const orc_params *p, const step_coefs *sc,
                    int64_t j, key_t_ *scratch, double *xs, double *xi, int32_t *S, double *w) {
    int n = p->n;
    departure(p->vel_id, sc, p->dt, nodes + 3 * j, xi);
    double ctr[3], s2;
    double *d2 = (double *)malloc(sizeof(double) * (size_t)n);
    if (p->mode == 0) {
        knn_one(N, nodes, xi, n, scratch, S, d2);
        ctr[0] = xi[0]; ctr[1] = xi[1]; ctr[2] = xi[2];
    } else {
        int32_t K;
        knn_one(N, nodes, xi, 1, scratch, &K, NULL);
        const double *xk = nodes + 3 * (int64_t)K;
        knn_one(N, nodes, xk, n, scratch, S, d2);
        ctr[0] = xk[0]; ctr[1] = xk[1]; ctr[2] = xk[2];
    }
    s2 = d2[n - 1];
    free(d2);
    for (int a = 0; a < n; ++a)
        for (int i = 0; i < 3; ++i) xs[3 * a + i] = nodes[3 * (int64_t)S[a] + i];
    return orc_weights(n, p->L, p->k, xs, ctr, s2, xi, w);
}

static double apply_one(int n, const double *w, const int32_t *S, const double *q) {
    double acc = 0.0;
    for (int a = 0; a < n; ++a) acc = fma(w[a], q[S[a]], acc);
    return acc;
}

/* Step m for the J target nodes in jl.  q_in: ntr x N.  Outputs (any may be
 * NULL): xi (J x 3), S (J x n), w (J x n), q_out (ntr x J), status (J). */
int orc_step_sample(int64_t N, const double *nodes, const orc_params *p, int64_t m,
                    int64_t J, const int64_t *jl, const double *q_in, double *xi_out,
                    int32_t *S_out, double *w_out, double *q_out, int32_t *st_out) {
    step_coefs sc;
    step_coefs_at(p->vel_id, p->vp, p->rk, p->t0, p->dt, m, &sc);
    int n = p->n;
    int bad = 0;
#pragma omp parallel reduction(+ : bad)
    {
        key_t_ *scratch = (key_t_ *)malloc(sizeof(key_t_) * (size_t)N);
        double *xs = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 8)
        for (int64_t t = 0; t < J; ++t) {
            double xi[3];
            int st = step_one(N, nodes, p, &sc, jl[t], scratch, xs, xi, S, w);
            if (st) bad += 1;
            if (st_out) st_out[t] = st;
            if (xi_out) memcpy(xi_out + 3 * t, xi, sizeof(xi));
            if (S_out) memcpy(S_out + (int64_t)n * t, S, sizeof(int32_t) * (size_t)n);
            if (w_out) memcpy(w_out + (int64_t)n * t, w, sizeof(double) * (size_t)n);
            if (q_out && q_in)
                for (int r = 0; r < p->ntr; ++r)
                    q_out[r * J + t] = apply_one(n, w, S, q_in + (int64_t)r * N);
        }
        free(scratch); free(xs); free(w); free(S);
    }
    return bad;
}

/* Full run of nsteps steps from step index m0, q (ntr x N) updated in place.
 * Returns ORC_OK, or the status of the first failing step, whose index is
 * stored in *fail_step (q then holds the state before that step). */
int orc_run(int64_t N, const double *nodes, const orc_params *p, int64_t m0, int64_t nsteps,
            double *q, int64_t *fail_step) {
    int64_t *jl = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    for (int64_t j = 0; j < N; ++j) jl[j] = j;
    double *qn = (double *)malloc(sizeof(double) * (size_t)N * (size_t)p->ntr);
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int status = ORC_OK;
    if (fail_step) *fail_step = -1;
    for (int64_t m = m0; m < m0 + nsteps; ++m) {
        int bad = orc_step_sample(N, nodes, p, m, N, jl, q, NULL, NULL, NULL, qn, st);
        if (bad) {
            for (int64_t j = 0; j < N; ++j)
                if (st[j]) { status = st[j]; break; }
            if (fail_step) *fail_step = m;
            break;
        }
        memcpy(q, qn, sizeof(double) * (size_t)N * (size_t)p->ntr);
    }
    free(jl); free(qn); free(st);
    return status;
}

/* ------------------------------------------------------------------------ */
/* RBF-PU interpolation (Section 2.3: patches, the weight functions          */
/* eq. wght_func with the cubic B-spline eq. bspline, the PU weights         */
/* eq. pu_func and the interpolant eq. PU_interp) in the SL step             */
/* (Section 3.3.3: one radius R = 2 sqrt(n/N), eq. rad_patches, and          */
/* ceil(aN/n) patches, eq. num_patches).                                     */
/* Readings: the patch centres are an input (a quasi-uniform point set);     */
/* patch l holds every node with |x - omega_l|^2 < R^2, in (d^2, index)      */
/* order; its interpolant is eq. rbf_poly in the frame centred on omega_l    */
/* with squared scale R^2; the patches containing a point are taken in       */
/* (d^2, l) order, and s(x) = (sum_l phi_l s_l(x)) / (sum_l phi_l) with the  */
/* numerator (fma) and the denominator (add) accumulated in that order;      */
/* phi_l = B(|x - omega_l| / R), the distance as sqrt(d^2).                  */
/* ------------------------------------------------------------------------ */

/* the cubic B-spline of eq. bspline */
double orc_bspline(double r) {
    if (r < 0.5) {
        double v = 4.0 * (r - 1.0);
        v = v * r;
        v = v * r;
        return (2.0 / 3.0) + v;
    }
    if (r < 1.0) {
        double t = r - 1.0;
        double v = t * t;
        v = v * t;
        return (-4.0 / 3.0) * v;
    }
    return 0.0;
}

/* nodes of one patch: returns how many x_i have |x_i - omega|^2 < R2 and
 * writes the first min(count, cap) of them, in (d^2, i) order, to idx */
int64_t orc_patch_nodes(int64_t N, const double *nodes, const double *omega, double R2, int64_t cap,
                        int32_t *idx) {
    key_t_ *keys = (key_t_ *)malloc(sizeof(key_t_) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        keys[i].d2 = dist2(nodes + 3 * i, omega);
        keys[i].i = (int32_t)i;
    }
    qsort(keys, (size_t)N, sizeof(key_t_), key_cmp);
    int64_t cnt = 0;
    while (cnt < N && keys[cnt].d2 < R2) {
        if (cnt < cap) idx[cnt] = keys[cnt].i;
        ++cnt;
    }
    free(keys);
    return cnt;
}

/* coefficients [c; d] of one patch's interpolant (eq. rbf_poly): the system
 * eq. rbf_poly_linsys of its nodes xs (n x 3) solved for [qv; 0] */
int orc_patch_coef(int n, int L, int k, const double *xs, const double *omega, double R2,
                   const double *qv, double *coef) {
    int mL = (L + 1) * (L + 1);
    int M = n + mL;
    double *A = (double *)malloc(sizeof(double) * (size_t)M * (size_t)M);
    double *r = (double *)malloc(sizeof(double) * (size_t)M);
    orc_assemble(n, L, k, xs, omega, R2, omega, A, r);  /* the right-hand side is replaced */
    for (int a = 0; a < n; ++a) r[a] = qv[a];
    for (int q = 0; q < mL; ++q) r[n + q] = 0.0;
    int st = orc_gauss_solve(M, A, r);
    memcpy(coef, r, sizeof(double) * (size_t)M);
    free(A);
    free(r);
    return st;
}

/* one patch's interpolant at x: sum_b c_b phi(|y_b - y_x|) + sum_q d_q p_q(x),
 * one fma chain in that order, in the patch's local coordinates */
double orc_patch_eval(int n, int L, int k, const double *xs, const double *omega, double R2,
                      const double *coef, const double *x) {
    int mL = (L + 1) * (L + 1);
    double s = (R2 > 0.0) ? sqrt(R2) : 1.0;
    double inv_s = 1.0 / s;
    double e1[3], e2[3];
    frame(omega, e1, e2);
    double yx[3], alx, bex, ux;
    local_coords(x, omega, e1, e2, inv_s, yx, &alx, &bex, &ux);
    double acc = 0.0;
    for (int b = 0; b < n; ++b) {
        double yb[3], al, be, u;
        local_coords(xs + 3 * b, omega, e1, e2, inv_s, yb, &al, &be, &u);
        double d0 = yb[0] - yx[0], d1 = yb[1] - yx[1], d2 = yb[2] - yx[2];
        acc = fma(coef[b], phs((d0 * d0 + d1 * d1) + d2 * d2, k), acc);
    }
    double *px = (double *)malloc(sizeof(double) * (size_t)mL);
    basis(L, alx, bex, ux, px);
    for (int q = 0; q < mL; ++q) acc = fma(coef[n + q], px[q], acc);
    free(px);
    return acc;
}

/* patch membership of all Mp patches: counts (Mp) and, when idx is given,
 * the concatenated node lists (offsets from the running sum of counts) */
void orc_pu_patches(int64_t N, const double *nodes, int64_t Mp, const double *centers, double R,
                    int64_t *counts, int32_t *idx) {
    const double R2 = R * R;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Mp + 1));
    if (idx) {
        off[0] = 0;
        for (int64_t l = 0; l < Mp; ++l) off[l + 1] = off[l] + counts[l];
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t l = 0; l < Mp; ++l) {
        if (idx)
            orc_patch_nodes(N, nodes, centers + 3 * l, R2, counts[l], idx + off[l]);
        else
            counts[l] = orc_patch_nodes(N, nodes, centers + 3 * l, R2, 0, NULL);
    }
    free(off);
}

/* One RBF-PU SL step m for the J target nodes jl (Algorithm 1 with the
 * interpolant eq. PU_interp).  p gives L, k, the flow, the integrator, dt,
 * t0 and the tracer count; the patches are given by counts/idx (from
 * orc_pu_patches).  q_in: ntr x N; outputs (may be NULL): xi (J x 3), q_out
 * (ntr x J), st_out (J: ORC_OK, ORC_SINGULAR for a singular patch system
 * used at the point, ORC_INVAL for a point in no patch).  Returns the number
 * of failing points. */
int orc_pu_step(int64_t N, const double *nodes, int64_t Mp, const double *centers, double R,
                const int64_t *counts, const int32_t *idx, const orc_params *p, int64_t m,
                int64_t J, const int64_t *jl, const double *q_in, double *xi_out, double *q_out,
                int32_t *st_out) {
    const int L = p->L, k = p->k, ntr = p->ntr;
    const int mL = (L + 1) * (L + 1);
    const double R2 = R * R;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Mp + 1));
    int64_t *coff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Mp + 1));
    off[0] = 0;
    coff[0] = 0;
    for (int64_t l = 0; l < Mp; ++l) {
        off[l + 1] = off[l] + counts[l];
        coff[l + 1] = coff[l] + (counts[l] + mL) * ntr;
    }
    double *coef = (double *)malloc(sizeof(double) * (size_t)coff[Mp]);
    int *pst = (int *)malloc(sizeof(int) * (size_t)Mp);
    /* the patches' interpolants of every tracer */
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t l = 0; l < Mp; ++l) {
        const int n = (int)counts[l];
        double *xs = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        double *qv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) xs[3 * a + i] = nodes[3 * (int64_t)idx[off[l] + a] + i];
        pst[l] = ORC_OK;
        for (int t = 0; t < ntr && pst[l] == ORC_OK; ++t) {
            for (int a = 0; a < n; ++a) qv[a] = q_in[(int64_t)t * N + idx[off[l] + a]];
            pst[l] = orc_patch_coef(n, L, k, xs, centers + 3 * l, R2, qv, coef + coff[l] + (int64_t)t * (n + mL));
        }
        free(xs);
        free(qv);
    }
    step_coefs sc;
    step_coefs_at(p->vel_id, p->vp, p->rk, p->t0, p->dt, m, &sc);
    int bad = 0;
#pragma omp parallel reduction(+ : bad)
    {
        key_t_ *keys = (key_t_ *)malloc(sizeof(key_t_) * (size_t)Mp);
        double *num = (double *)malloc(sizeof(double) * (size_t)ntr);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < J; ++t) {
            double xi[3];
            departure(p->vel_id, &sc, p->dt, nodes + 3 * jl[t], xi);
            for (int64_t l = 0; l < Mp; ++l) {
                keys[l].d2 = dist2(centers + 3 * l, xi);
                keys[l].i = (int32_t)l;
            }
            qsort(keys, (size_t)Mp, sizeof(key_t_), key_cmp);
            int st = ORC_OK;
            double den = 0.0;
            for (int r = 0; r < ntr; ++r) num[r] = 0.0;
            for (int64_t c = 0; c < Mp && keys[c].d2 < R2; ++c) {
                const int64_t l = keys[c].i;
                if (pst[l] != ORC_OK) { st = pst[l]; continue; }
                const int n = (int)counts[l];
                double *xs = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
                for (int a = 0; a < n; ++a)
                    for (int i = 0; i < 3; ++i) xs[3 * a + i] = nodes[3 * (int64_t)idx[off[l] + a] + i];
                const double phi = orc_bspline(sqrt(keys[c].d2) / R);
                for (int r = 0; r < ntr; ++r) {
                    const double sv = orc_patch_eval(n, L, k, xs, centers + 3 * l, R2,
                                                     coef + coff[l] + (int64_t)r * (n + mL), xi);
                    num[r] = fma(phi, sv, num[r]);
                }
                den = den + phi;
                free(xs);
            }
            if (st == ORC_OK && !(den > 0.0)) st = ORC_INVAL;
            if (st != ORC_OK) bad += 1;
            if (st_out) st_out[t] = st;
            if (xi_out) memcpy(xi_out + 3 * t, xi, sizeof(xi));
            if (q_out)
                for (int r = 0; r < ntr; ++r) q_out[(int64_t)r * J + t] = num[r] / den;
        }
        free(keys);
        free(num);
    }
    free(off); free(coff); free(coef); free(pst);
    return bad;
}

/*
 * sanitize_driver.c -- calls every entry point of the oracle on small inputs,
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer:
 *
 *   gcc -O1 -g -std=gnu11 -fopenmp -ffp-contract=off -fsanitize=address,undefined \
 *       -fno-omit-frame-pointer -fno-sanitize-recover=all oracle/sanitize_driver.c -o driver -lm
 *
 * The oracle is included as one translation unit (it has no header).  Exit
 * status 0 when every call returned the expected status; the sanitizers abort
 * on the first memory error or undefined operation.  Test infrastructure only.
 */
#include <stdio.h>

#include "oracle.c"

static void fib_nodes(int64_t N, double *X) {
    const double ga = M_PI * (3.0 - sqrt(5.0));
    for (int64_t i = 0; i < N; ++i) {
        double z = 1.0 - (2.0 * (double)i + 1.0) / (double)N;
        double rho = sqrt((1.0 - z) * (1.0 + z));
        double ph = fmod((double)i * ga, 2.0 * M_PI);
        X[3 * i] = rho * cos(ph);
        X[3 * i + 1] = rho * sin(ph);
        X[3 * i + 2] = z;
    }
}

static int fails = 0;
#define EXPECT(cond, what)                                        \
    do {                                                          \
        if (!(cond)) {                                            \
            fprintf(stderr, "unexpected result: %s\n", (what));   \
            ++fails;                                              \
        }                                                         \
    } while (0)

static orc_params params(int n, int L, int k, int mode, int vel, int rk, int ntr, double dt) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.n = n; p.L = L; p.k = k; p.mode = mode; p.vel_id = vel; p.ntr = ntr; p.rk = rk;
    p.vp[0] = 5.0; p.vp[1] = 0.0; p.vp[2] = 0.6; p.vp[3] = 0.8; p.vp[4] = 1.0;
    p.dt = dt; p.t0 = 0.0;
    return p;
}

int main(void) {
    const int64_t N = 1500;
    double *X = malloc(sizeof(double) * 3 * (N + 1));
    fib_nodes(N, X);

    /* velocities and departure points, every flow and both integrators */
    double vp[8] = {5.0, 0.0, 0.6, 0.8, 1.0, 0, 0, 0}, u[3];
    for (int v = 0; v <= VEL_NL2010; ++v) orc_velocity(v, vp, 0.3, X + 30, u);
    double *xi = malloc(sizeof(double) * 3 * N);
    for (int rk = 0; rk <= INT_RK5F; ++rk)
        for (int v = 0; v <= VEL_NL2010; ++v) orc_trace(N, X, v, vp, rk, 0.0, 0.1, 3, xi);

    /* neighbour search, n from 1 to N */
    int32_t *idx = malloc(sizeof(int32_t) * N * 4);
    double *d2 = malloc(sizeof(double) * N * 4);
    const int ns[4] = {1, 31, 184, (int)N};
    for (int t = 0; t < 4; ++t) orc_knn(N, X, 4, xi, ns[t], idx, d2);

    /* elimination: a saddle system and a singular one */
    {
        int M = 47;
        double *A = calloc((size_t)M * M, sizeof(double)), *b = calloc((size_t)M, sizeof(double));
        orc_knn(N, X, 1, X, 31, idx, d2);
        double xs[3 * 31];
        for (int a = 0; a < 31; ++a) memcpy(xs + 3 * a, X + 3 * (int64_t)idx[a], sizeof(double) * 3);
        orc_assemble(31, 3, 2, xs, X, d2[30], X + 3, A, b);
        EXPECT(orc_gauss_solve(M, A, b) == ORC_OK, "saddle solve");
        memset(A, 0, sizeof(double) * (size_t)M * M);
        EXPECT(orc_gauss_solve(M, A, b) == ORC_SINGULAR, "zero matrix is singular");
        free(A);
        free(b);
    }

    /* weights for every solver size the library supports, degree 0 to 8 */
    const int cases[][3] = {{1, 0, 0}, {4, 1, 1}, {31, 3, 2}, {56, 4, 2}, {84, 5, 3}, {120, 7, 4}, {90, 8, 4}};
    for (size_t c = 0; c < sizeof cases / sizeof cases[0]; ++c) {
        int n = cases[c][0], L = cases[c][1], k = cases[c][2];
        orc_knn(N, X, 1, xi, n, idx, d2);
        double *xs = malloc(sizeof(double) * 3 * (size_t)n), *w = malloc(sizeof(double) * (size_t)n);
        for (int a = 0; a < n; ++a) memcpy(xs + 3 * a, X + 3 * (int64_t)idx[a], sizeof(double) * 3);
        EXPECT(orc_weights(n, L, k, xs, xi, d2[n - 1], xi, w) == ORC_OK, "weights");
        free(xs);
        free(w);
    }

    /* steps and runs: both stencil modes, RK4 and RK5, two tracers */
    {
        double *q = malloc(sizeof(double) * 2 * (N + 1));
        for (int64_t j = 0; j < 2 * (N + 1); ++j) q[j] = sin(0.01 * (double)j);
        int64_t jl[5] = {0, 7, 700, 1200, N - 1};
        double qo[10], xo[15], wo[5 * 31];
        int32_t So[5 * 31], st[5];
        for (int mode = 0; mode <= 1; ++mode) {
            orc_params p = params(31, 3, 2, mode, VEL_DEFORM, mode, 2, 0.25);
            EXPECT(orc_step_sample(N, X, &p, 2, 5, jl, q, xo, So, wo, qo, st) == 0, "step sample");
            int64_t fs = 0;
            EXPECT(orc_run(N, X, &p, 0, 3, q, &fs) == ORC_OK && fs == -1, "run");
        }
        /* a duplicated node: its stencils are singular and the run stops */
        memcpy(X + 3 * N, X + 3 * 5, sizeof(double) * 3);
        orc_params p = params(17, 1, 1, 0, VEL_SOLID, INT_RK4, 1, 0.1);
        int64_t fs = 0;
        EXPECT(orc_run(N + 1, X, &p, 0, 2, q, &fs) == ORC_SINGULAR && fs == 0, "singular run");
        free(q);
    }

    /* RBF-PU: patches, one step */
    {
        const int64_t Mp = 160;
        const double R = 2.0 * sqrt(31.0 / (double)N) * 1.2;
        double *C = malloc(sizeof(double) * 3 * Mp);
        fib_nodes(Mp, C);
        int64_t *cnt = malloc(sizeof(int64_t) * Mp);
        orc_pu_patches(N, X, Mp, C, R, cnt, NULL);
        int64_t tot = 0;
        for (int64_t l = 0; l < Mp; ++l) tot += cnt[l];
        int32_t *pidx = malloc(sizeof(int32_t) * (size_t)tot);
        orc_pu_patches(N, X, Mp, C, R, cnt, pidx);
        double *q = malloc(sizeof(double) * N);
        for (int64_t j = 0; j < N; ++j) q[j] = cos(0.02 * (double)j);
        orc_params p = params(31, 3, 2, 0, VEL_NL2010, INT_RK5F, 1, 0.1);
        int64_t jl[4] = {0, 300, 901, N - 1};
        double xo[12], qo[4];
        int32_t st[4];
        EXPECT(orc_pu_step(N, X, Mp, C, R, cnt, pidx, &p, 1, 4, jl, q, xo, qo, st) == 0, "pu step");
        (void)orc_bspline(0.3);
        (void)orc_bspline(0.7);
        free(C); free(cnt); free(pidx); free(q);
    }

    free(X); free(xi); free(idx); free(d2);
    if (fails) return 1;
    printf("oracle sanitizer driver: all calls ok\n");
    return 0;
}

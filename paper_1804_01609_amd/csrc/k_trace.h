// Departure-point tracer (Section 3.2, eq. sl_ode): RK4 or Fehlberg's RK5
// backward over [t_m, t_{m+1}] with the stage points and the result projected
// orthogonally onto the unit sphere.  The time-dependent coefficients of the
// velocity (cos/sin of the stage times, rotation matrices) arrive from the
// host, so the kernel itself uses only +, -, *, / and sqrt, each correctly
// rounded.
#pragma once
#include "dev_util.h"
#include "rbfsl_impl.h"

namespace rbfsl {

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// u(x) for one stage: solid body w x x; c R u0(R^T x) + w x x with
// u0(y) = y x grad(y0 y1 y2 + y2^2 y0 / 2); or the NL2010 flow of Section 4.2
// in Cartesian form, A (-y, x, 0) + B (-z x, -z y, rho^2) + w x x with
// rho^2 = x^2 + y^2, s1 = rho sin(lambda'), c1 = rho cos(lambda'),
// A = c 2z s1^2 / rho^2, B = c 2 s1 c1 / rho^2, lambda' = lambda - (2 pi/T) t.
__device__ __forceinline__ void vel(int vel_id, const VelCoef &v, const double x[3], double u[3]) {
    if (vel_id == RBFSL_VEL_ZERO) {
        u[0] = 0.0; u[1] = 0.0; u[2] = 0.0;
        return;
    }
    double wx[3];
    cross3(v.w, x, wx);
    if (vel_id == RBFSL_VEL_SOLID_BODY) {
        u[0] = wx[0]; u[1] = wx[1]; u[2] = wx[2];
        return;
    }
    if (vel_id == RBFSL_VEL_NL2010) {
        const double rho2 = x[0] * x[0] + x[1] * x[1];
        const double s1 = x[1] * v.cw - x[0] * v.sw;
        const double c1 = x[0] * v.cw + x[1] * v.sw;
        const double A = (v.c * ((2.0 * x[2]) * (s1 * s1))) / rho2;
        const double B = (v.c * ((2.0 * s1) * c1)) / rho2;
        u[0] = (-(A * x[1]) - B * (x[2] * x[0])) + wx[0];
        u[1] = (A * x[0] - B * (x[2] * x[1])) + wx[1];
        u[2] = B * rho2 + wx[2];
        return;
    }
    double y[3], g[3], u0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = (v.R[i] * x[0] + v.R[3 + i] * x[1]) + v.R[6 + i] * x[2];
    g[0] = y[1] * y[2] + 0.5 * (y[2] * y[2]);
    g[1] = y[0] * y[2];
    g[2] = y[0] * y[1] + y[2] * y[0];
    cross3(y, g, u0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double rv = (v.R[3 * i] * u0[0] + v.R[3 * i + 1] * u0[1]) + v.R[3 * i + 2] * u0[2];
        u[i] = v.c * rv + wx[i];
    }
}

__device__ __forceinline__ void proj(double v[3]) {
    double r = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    v[0] = v[0] / r;
    v[1] = v[1] / r;
    v[2] = v[2] / r;
}

// departure point of node x over one step (coefficients sc): RK4, or
// Fehlberg's RK5 with the stage sums accumulated term by term in j order
__device__ __forceinline__ void trace_point(const StepCoef &sc, const double x[3], double xi[3]) {
    if (sc.rk == RBFSL_RK4) {
        double k1[3], k2[3], k3[3], k4[3], y[3];
        vel(sc.vel_id, sc.v[0], x, k1);
#pragma unroll
        for (int i = 0; i < 3; ++i) y[i] = x[i] + sc.hh * k1[i];
        proj(y);
        vel(sc.vel_id, sc.v[1], y, k2);
#pragma unroll
        for (int i = 0; i < 3; ++i) y[i] = x[i] + sc.hh * k2[i];
        proj(y);
        vel(sc.vel_id, sc.v[1], y, k3);
#pragma unroll
        for (int i = 0; i < 3; ++i) y[i] = x[i] + sc.h * k3[i];
        proj(y);
        vel(sc.vel_id, sc.v[2], y, k4);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s = ((k1[i] + 2.0 * k2[i]) + 2.0 * k3[i]) + k4[i];
            xi[i] = x[i] + sc.h6 * s;
        }
        proj(xi);
        return;
    }
    double k[6][3], y[3];
    vel(sc.vel_id, sc.v[0], x, k[0]);
    sfor<1, 6>([&](auto SI_) SI {
        constexpr int st = SI_;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double acc = kRk5.a[st][0] * k[0][i];
            sfor<1, st>([&](auto JI) SI {
                constexpr int j = JI;
                acc = acc + kRk5.a[st][j] * k[j][i];
            });
            y[i] = x[i] + sc.h * acc;
        }
        proj(y);
        vel(sc.vel_id, sc.v[st], y, k[st]);
    });
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double acc = kRk5.b[0] * k[0][i];
        sfor<1, 6>([&](auto JI) SI {
            constexpr int j = JI;
            acc = acc + kRk5.b[j] * k[j][i];
        });
        xi[i] = x[i] + sc.h * acc;
    }
    proj(xi);
}

}  // namespace rbfsl

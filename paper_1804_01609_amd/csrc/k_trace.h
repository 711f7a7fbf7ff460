// Departure-point tracer (Section 3.2, eq. sl_ode): one lane per node, RK4
// backward over [t_m, t_{m+1}] with the stage points and the result projected
// orthogonally onto the unit sphere.  The time-dependent coefficients of the
// velocity (cos/sin of the stage times, rotation matrices) arrive from the
// host, so the kernel itself uses only +, -, *, / and sqrt, each correctly
// rounded.
#pragma once
#include "rbfsl_impl.h"

namespace rbfsl {

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// u(x) for one stage: solid body w x x, or c R u0(R^T x) + w x x with
// u0(y) = y x grad(y0 y1 y2 + y2^2 y0 / 2).
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

// departure point of node x over one step (coefficients sc)
__device__ __forceinline__ void trace_point(const StepCoef &sc, const double x[3], double xi[3]) {
    double k1[3], k2[3], k3[3], k4[3], y[3];
    vel(sc.vel_id, sc.c1, x, k1);
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = x[i] + sc.hh * k1[i];
    proj(y);
    vel(sc.vel_id, sc.ch, y, k2);
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = x[i] + sc.hh * k2[i];
    proj(y);
    vel(sc.vel_id, sc.ch, y, k3);
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = x[i] + sc.h * k3[i];
    proj(y);
    vel(sc.vel_id, sc.c0, y, k4);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double s = ((k1[i] + 2.0 * k2[i]) + 2.0 * k3[i]) + k4[i];
        xi[i] = x[i] + sc.h6 * s;
    }
    proj(xi);
}

}  // namespace rbfsl

// Tracer kernel: one lane per node (the RK4 step itself is trace_point in
// k_trace.h).
#include "k_trace.h"

namespace rbfsl {

__global__ void __launch_bounds__(256) k_trace(const double *__restrict__ nx,
                                               const double *__restrict__ ny,
                                               const double *__restrict__ nz, int64_t N,
                                               StepCoef sc, double *__restrict__ ex,
                                               double *__restrict__ ey, double *__restrict__ ez,
                                               const int *__restrict__ status, int64_t step) {
    if (status[ST_FAILSTEP] < step) return;  // an earlier step of this run failed
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const double x[3] = {nx[j], ny[j], nz[j]};
    double xi[3];
    trace_point(sc, x, xi);
    ex[j] = xi[0];
    ey[j] = xi[1];
    ez[j] = xi[2];
}

hipError_t launch_trace(const double *nx, const double *ny, const double *nz, int64_t N,
                        const StepCoef &sc, double *ex, double *ey, double *ez,
                        const int *status, int64_t step, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    unsigned blocks = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_trace, dim3(blocks), dim3(256), 0, s, nx, ny, nz, N, sc, ex, ey, ez,
                       status, step);
    return hipGetLastError();
}

// The departure points of K consecutive steps m0 .. m0 + K - 1 at once
// (their tracer does not depend on the transported field): point j of step s
// goes to j + s N; sc[s] holds step m0 + s's coefficients.
__global__ void __launch_bounds__(256) k_trace_steps(const double *__restrict__ nx,
                                                     const double *__restrict__ ny,
                                                     const double *__restrict__ nz, int64_t N,
                                                     const StepCoef *__restrict__ sc, int64_t KN,
                                                     double *__restrict__ ex, double *__restrict__ ey,
                                                     double *__restrict__ ez,
                                                     const int *__restrict__ status, int64_t m0) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= KN) return;
    const int64_t s = id / N, j = id - s * N;
    if (status[ST_FAILSTEP] < m0 + s) return;  // an earlier step of this run failed
    const double x[3] = {nx[j], ny[j], nz[j]};
    double xi[3];
    trace_point(sc[s], x, xi);
    ex[id] = xi[0];
    ey[id] = xi[1];
    ez[id] = xi[2];
}

hipError_t launch_trace_steps(const double *nx, const double *ny, const double *nz, int64_t N,
                              const StepCoef *sc, int K, double *ex, double *ey, double *ez,
                              const int *status, int64_t m0, hipStream_t s) {
    const int64_t KN = N * (int64_t)K;
    if (KN <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trace_steps, dim3((unsigned)((KN + 255) / 256)), dim3(256), 0, s, nx, ny, nz, N, sc,
                       KN, ex, ey, ez, status, m0);
    return hipGetLastError();
}

__global__ void k_status_reset(int *status) {
    if (threadIdx.x < ST_WORDS) status[threadIdx.x] = (threadIdx.x == ST_FAILSTEP) ? NO_FAIL : 0;
}

hipError_t launch_status_reset(int *status, hipStream_t s) {
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, s, status);
    return hipGetLastError();
}

}  // namespace rbfsl

// Gather-and-dot: q^{m+1}[t][j] = sum_a w_ja q^m[t][S_ja] (Algorithm 1: the
// interpolant evaluated at the departure point becomes the new nodal value),
// accumulated as a chain of fma in stencil order.  One lane per (node,
// tracer), the tracer index fastest: the lanes of one node read the same
// weights and indices (one cache line serves them all) and their tracers'
// values at the same node indices.
#include "rbfsl_impl.h"

namespace rbfsl {

__global__ void __launch_bounds__(256) k_apply(const double *__restrict__ w,
                                               const int32_t *__restrict__ S,
                                               const int32_t *__restrict__ cidx, int64_t N, int n,
                                               int ntr, const double *__restrict__ qin,
                                               double *__restrict__ qout,
                                               const int *__restrict__ status, int64_t step) {
    if (status[ST_FAILSTEP] <= step) return;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N * ntr) return;
    const int64_t j = id / ntr;
    const int t = (int)(id - j * ntr);
    const int64_t row = cidx ? (int64_t)cidx[j] : j;
    const double *wj = w + j * n;
    const int32_t *Sj = S + row * n;
    const double *q = qin + (int64_t)t * N;
    double acc = 0.0;
    int a = 0;
    // eight terms per iteration: their index, weight and value loads are in
    // flight together ahead of the fmas (the chain order is unchanged)
    for (; a + 8 <= n; a += 8) {
        int32_t s8[8];
        double w8[8], q8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s8[u] = Sj[a + u];
            w8[u] = wj[a + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) q8[u] = q[s8[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(w8[u], q8[u], acc);
    }
    for (; a < n; ++a) acc = fma(wj[a], q[Sj[a]], acc);
    qout[(int64_t)t * N + j] = acc;
}

hipError_t launch_apply(const double *w, const int32_t *S, const int32_t *cidx, int64_t N, int n,
                        int ntr, const double *qin, double *qout, const int *status,
                        int64_t step, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    unsigned blocks = (unsigned)((N * ntr + 255) / 256);
    hipLaunchKernelGGL(k_apply, dim3(blocks), dim3(256), 0, s, w, S, cidx, N, n, ntr, qin, qout,
                       status, step);
    return hipGetLastError();
}

}  // namespace rbfsl

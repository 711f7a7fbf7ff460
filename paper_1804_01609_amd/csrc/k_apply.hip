// Gather-and-dot: q^{m+1}[t][j] = sum_a w_ja q^m[t][S_ja] (Algorithm 1: the
// interpolant evaluated at the departure point becomes the new nodal value),
// accumulated as a chain of fma in stencil order.  One lane per (node,
// tracer), the tracer index fastest: the lanes of one node read the same
// weights and indices (one cache line serves them all) and their tracers'
// values at the same node indices.  Small fields take eight lanes per (node,
// tracer) instead (k_apply8).
#include "rbfsl_impl.h"

namespace rbfsl {

__global__ void __launch_bounds__(64) k_apply(const double *__restrict__ w,
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

// Eight lanes per (node, tracer): lane u loads the terms u, u + 8, ... (the
// lanes of a node read neighbouring indices and weights, so a load touches a
// few cache lines instead of one per lane), the values meet in LDS and the
// first lane of the eight runs the same fma chain in stencil order.  For
// fields of a few thousand (node, tracer) pairs, where one lane per pair
// would leave most compute units idle and each busy one bound by address
// processing (N = 1,024, n = 31: 3.3 against 7.4 us per launch).
constexpr int64_t APPLY8_MAX = 8192;  // (node, tracer) pairs

__global__ void __launch_bounds__(64) k_apply8(const double *__restrict__ w,
                                              const int32_t *__restrict__ S,
                                              const int32_t *__restrict__ cidx, int64_t N, int n,
                                              int ntr, const double *__restrict__ qin,
                                              double *__restrict__ qout,
                                              const int *__restrict__ status, int64_t step) {
    if (status[ST_FAILSTEP] <= step) return;
    extern __shared__ double sh[];
    const int p = threadIdx.x >> 3, u = threadIdx.x & 7;
    const int64_t id = (int64_t)blockIdx.x * 8 + p;
    const bool live = id < N * ntr;
    const int64_t j = live ? id / ntr : 0;
    const int t = live ? (int)(id - j * ntr) : 0;
    const int64_t row = cidx ? (int64_t)cidx[j] : j;
    const double *wj = w + j * n;
    const int32_t *Sj = S + row * n;
    const double *q = qin + (int64_t)t * N;
    double *const sw = sh + (int64_t)p * 2 * n, *const sq = sw + n;
    for (int a0 = 0; a0 < n; a0 += 32) {
        // four terms per lane in flight together; loads past the last
        // term repeat it and are not stored
        int32_t s4[4];
        double w4[4], q4[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = min(a0 + u + 8 * r, n - 1);
            s4[r] = Sj[a];
            w4[r] = wj[a];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) q4[r] = q[s4[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = a0 + u + 8 * r;
            if (a < n) {
                sw[a] = w4[r];
                sq[a] = q4[r];
            }
        }
    }
    __syncthreads();
    if (u == 0 && live) {
        double acc = 0.0;
        for (int a = 0; a < n; ++a) acc = fma(sw[a], sq[a], acc);
        qout[(int64_t)t * N + j] = acc;
    }
}

hipError_t launch_apply(const double *w, const int32_t *S, const int32_t *cidx, int64_t N, int n,
                        int ntr, const double *qin, double *qout, const int *status,
                        int64_t step, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const int64_t pairs = N * ntr;
    if (pairs <= APPLY8_MAX) {
        const size_t lds = sizeof(double) * 16 * (size_t)n;  // 8 pairs x (weights, values)
        hipLaunchKernelGGL(k_apply8, dim3((unsigned)((pairs + 7) / 8)), dim3(64), lds, s, w, S, cidx, N, n,
                           ntr, qin, qout, status, step);
    } else {
        hipLaunchKernelGGL(k_apply, dim3((unsigned)((pairs + 63) / 64)), dim3(64), 0, s, w, S, cidx, N, n,
                           ntr, qin, qout, status, step);
    }
    return hipGetLastError();
}

}  // namespace rbfsl

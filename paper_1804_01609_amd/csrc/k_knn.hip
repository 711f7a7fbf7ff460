// Stencil search kernel: one wavefront per query point (the search itself is
// knn_wave in k_knn.h).
#include "k_knn.h"

namespace rbfsl {

template <int CAP>
__global__ void __launch_bounds__(64) k_knn(GridView g, const double *__restrict__ qx,
                                            const double *__restrict__ qy,
                                            const double *__restrict__ qz, int n, double R_init,
                                            int32_t *__restrict__ idx, double *__restrict__ d2out,
                                            double *__restrict__ s2out, int *status, int64_t step0,
                                            int64_t per) {
    __shared__ KnnSmem<CAP> sh;
    const int64_t q = blockIdx.x;
    const int64_t step = step0 + (per ? q / per : 0);  // queries of several steps: per a step
    if (status[ST_FAILSTEP] < step) return;
    const int lane = threadIdx.x;
    if (!knn_wave<CAP>(sh, lane, g, qx[q], qy[q], qz[q], n, R_init)) {
        if (lane == 0) {
            atomicAdd(&status[ST_SEARCH], 1);
            atomicMin(&status[ST_FAILSTEP], (int)step);
        }
        return;
    }
    int32_t *orow = idx + q * n;
    for (int a = lane; a < n; a += 64) {
        orow[a] = sh.ki[a];
        if (d2out) d2out[q * n + a] = sh.kd[a];
    }
    if (s2out && lane == 0) s2out[q] = sh.kd[n - 1];
}

double knn_first_radius(int n, int64_t N) {
    double R = 2.0 * sqrt(1.4 * (double)n / (double)N);
    return (R > 2.0) ? 2.0 : R;
}

hipError_t launch_knn(const Grid &g, int64_t N, const double *qx, const double *qy,
                      const double *qz, int64_t Q, int n, int32_t *idx, double *d2, double *s2,
                      int *status, int64_t step, hipStream_t s, int64_t per) {
    if (Q <= 0) return hipSuccess;
    const GridView gv{g.G, g.invh, g.cell_start, g.sx, g.sy, g.sz, g.perm};
    // the first radius keeps about 1.4 n nodes: for small n a quarter- or
    // half-size candidate store suffices (the radius adapts when it does not),
    // and its smaller LDS footprint lets more searches share a compute unit
    const double R0 = knn_first_radius(n, N);
    if (n <= KNN_SMALL_N / 2)
        hipLaunchKernelGGL(k_knn<KNN_CAP / 4>, dim3((unsigned)Q), dim3(64), 0, s, gv, qx, qy, qz, n, R0, idx, d2,
                           s2, status, step, per);
    else if (n <= KNN_SMALL_N)
        hipLaunchKernelGGL(k_knn<KNN_CAP / 2>, dim3((unsigned)Q), dim3(64), 0, s, gv, qx, qy, qz, n, R0, idx, d2,
                           s2, status, step, per);
    else
        hipLaunchKernelGGL(k_knn<KNN_CAP>, dim3((unsigned)Q), dim3(64), 0, s, gv, qx, qy, qz, n, R0, idx, d2,
                           s2, status, step, per);
    return hipGetLastError();
}

}  // namespace rbfsl

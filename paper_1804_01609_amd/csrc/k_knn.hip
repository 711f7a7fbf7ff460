// Exact n-nearest-neighbour search through the spatial hash: one wavefront
// per query point.  The stencils of Section 2.2 / 3.3.2 are the n nodes with
// the smallest keys (d^2, node index), d^2 = (dx*dx + dy*dy) + dz*dz, in
// ascending key order -- the same total order as a brute-force sort.
//
// Exactness: the kernel gathers every node of every cell that meets the cube
// of half-width R around the query and keeps those with d^2 < Rt^2,
// Rt = R (1 - 1e-9).  If at least n are kept, the n-th smallest kept key is
// below Rt^2 while every node outside the cell box is farther than R - O(ulp)
// from the query, hence has a larger key: the kept set contains the true n
// nearest.  Otherwise R grows (or shrinks when more than KNN_CAP are kept) and
// the search repeats.  The kept keys are ordered by a bitonic sort in LDS.
#include <float.h>
#include <limits.h>

#include "rbfsl_impl.h"

namespace rbfsl {

__device__ __forceinline__ int cellc(double v, double invh, int G) {
    const double f = floor((v + 1.0) * invh);
    if (!(f >= 0.0)) return 0;  // also NaN
    return (f > (double)(G - 1)) ? G - 1 : (int)f;
}

__global__ void __launch_bounds__(64) k_knn(int G, double invh, const int *__restrict__ cstart,
                                            const double *__restrict__ sx, const double *__restrict__ sy,
                                            const double *__restrict__ sz, const int *__restrict__ perm,
                                            const double *__restrict__ qx, const double *__restrict__ qy,
                                            const double *__restrict__ qz, int n, double R_init,
                                            int32_t *__restrict__ idx, double *__restrict__ d2out,
                                            double *__restrict__ s2out, int *status, int64_t step) {
    __shared__ double kd[KNN_CAP];
    __shared__ int ki[KNN_CAP];
    __shared__ int cnt;
    if (status[ST_FAILSTEP] < step) return;
    const int64_t q = blockIdx.x;
    const int lane = threadIdx.x;
    const double q0 = qx[q], q1 = qy[q], q2 = qz[q];
    double R = R_init, Rlo = 0.0, Rhi = 0.0;
    int F = 0;
    bool ok = false;
    for (int it = 0; it < 64; ++it) {
        const double Rt = R * (1.0 - 1e-9);
        const double Rt2 = Rt * Rt;
        const int lx = cellc(q0 - R, invh, G), hx = cellc(q0 + R, invh, G);
        const int ly = cellc(q1 - R, invh, G), hy = cellc(q1 + R, invh, G);
        const int lz = cellc(q2 - R, invh, G), hz = cellc(q2 + R, invh, G);
        const int nbx = hx - lx + 1, nby = hy - ly + 1, nbz = hz - lz + 1;
        const int nb = nbx * nby * nbz;
        if (lane == 0) cnt = 0;
        __syncthreads();
        for (int cb = lane; cb < nb; cb += 64) {
            int cx = lx + cb % nbx;
            int r = cb / nbx;
            int cy = ly + r % nby;
            int cz = lz + r / nby;
            int c = (cz * G + cy) * G + cx;
            int b = cstart[c], e = cstart[c + 1];
            for (int p = b; p < e; ++p) {
                double d0 = sx[p] - q0, d1 = sy[p] - q1, dd = sz[p] - q2;
                double dist = (d0 * d0 + d1 * d1) + dd * dd;
                if (dist < Rt2) {
                    int slot = atomicAdd(&cnt, 1);
                    if (slot < KNN_CAP) {
                        kd[slot] = dist;
                        ki[slot] = perm[p];
                    }
                }
            }
        }
        __syncthreads();
        F = cnt;
        __syncthreads();
        if (F > KNN_CAP) {
            Rhi = R;
            R = (Rlo > 0.0) ? 0.5 * (Rlo + R) : 0.7 * R;
        } else if (F < n) {
            if (R >= 4.0) break;
            Rlo = R;
            R = (Rhi > 0.0) ? 0.5 * (R + Rhi) : 1.5 * R;
            if (R > 4.0) R = 4.0;
        } else {
            ok = true;
            break;
        }
    }
    if (!ok) {
        if (lane == 0) {
            atomicAdd(&status[ST_SEARCH], 1);
            atomicMin(&status[ST_FAILSTEP], (int)step);
        }
        return;
    }
    int P = 64;
    while (P < F) P <<= 1;
    for (int t = F + lane; t < P; t += 64) {
        kd[t] = DBL_MAX;
        ki[t] = INT_MAX;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < (P >> 1); t += 64) {
                int i = 2 * t - (t & (stride - 1));
                int j = i + stride;
                double di = kd[i], dj = kd[j];
                int ii = ki[i], ij = ki[j];
                bool gt = (di > dj) || (di == dj && ii > ij);
                bool asc = (i & size) == 0;
                if (gt == asc) {
                    kd[i] = dj; kd[j] = di;
                    ki[i] = ij; ki[j] = ii;
                }
            }
            __syncthreads();
        }
    }
    int32_t *orow = idx + q * n;
    for (int a = lane; a < n; a += 64) {
        orow[a] = ki[a];
        if (d2out) d2out[q * n + a] = kd[a];
    }
    if (s2out && lane == 0) s2out[q] = kd[n - 1];
}

hipError_t launch_knn(const Grid &g, int64_t N, const double *qx, const double *qy,
                      const double *qz, int64_t Q, int n, int32_t *idx, double *d2, double *s2,
                      int *status, int64_t step, hipStream_t s) {
    if (Q <= 0) return hipSuccess;
    double R = 2.0 * sqrt(1.4 * (double)n / (double)N);
    if (R > 2.0) R = 2.0;
    hipLaunchKernelGGL(k_knn, dim3((unsigned)Q), dim3(64), 0, s, g.G, g.invh, g.cell_start, g.sx,
                       g.sy, g.sz, g.perm, qx, qy, qz, n, R, idx, d2, s2, status, step);
    return hipGetLastError();
}

}  // namespace rbfsl

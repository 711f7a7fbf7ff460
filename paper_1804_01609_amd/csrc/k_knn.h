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
#pragma once
#include <float.h>
#include <limits.h>

#include "dev_util.h"
#include "rbfsl_impl.h"

namespace rbfsl {

__device__ __forceinline__ int cellc(double v, double invh, int G) {
    const double f = floor((v + 1.0) * invh);
    if (!(f >= 0.0)) return 0;  // also NaN
    return (f > (double)(G - 1)) ? G - 1 : (int)f;
}

// the spatial hash as the search reads it
struct GridView {
    int G;
    double invh;
    const int *cell_start;
    const double *sx, *sy, *sz;
    const int *perm;
};

// LDS of one search: up to CAP kept keys
template <int CAP>
struct KnnSmem {
    double kd[CAP];
    int ki[CAP];
    int cnt;
};

// ordering of the search's LDS traffic among its NWV waves: the wave itself,
// or the whole workgroup (NWV waves = the workgroup)
template <int NWV>
__device__ __forceinline__ void knn_sync() {
    if constexpr (NWV == 1) wave_lds_sync();
    else __syncthreads();
}

// The n nearest nodes of (q0, q1, q2), searched by NWV waves (tid =
// 0 .. 64 NWV - 1; NWV > 1 only when they form the whole workgroup).  On
// success kd[0..n) / ki[0..n) hold the keys in ascending (d^2, index) order;
// false when no radius gave between n and CAP candidates.  The result is the
// same for every NWV (the key order is total).
template <int CAP, int NWV = 1>
__device__ __forceinline__ bool knn_wave(KnnSmem<CAP> &sh, const int tid, const GridView &g,
                                         const double q0, const double q1, const double q2,
                                         const int n, const double R_init) {
    constexpr int NT = 64 * NWV;
    const int lane = tid;
    double *const kd = sh.kd;
    int *const ki = sh.ki;
    const int G = g.G;
    const double invh = g.invh;
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
        if (lane == 0) sh.cnt = 0;
        knn_sync<NWV>();
        for (int cb = lane; cb < nb; cb += NT) {
            int cx = lx + cb % nbx;
            int r = cb / nbx;
            int cy = ly + r % nby;
            int cz = lz + r / nby;
            int c = (cz * G + cy) * G + cx;
            const int b = g.cell_start[c], e = g.cell_start[c + 1];
            // four nodes per iteration: their loads are in flight together
            int p = b;
            for (; p + 4 <= e; p += 4) {
                double x[4], y[4], z[4];
                int id[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    x[u] = g.sx[p + u];
                    y[u] = g.sy[p + u];
                    z[u] = g.sz[p + u];
                    id[u] = g.perm[p + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    double d0 = x[u] - q0, d1 = y[u] - q1, dd = z[u] - q2;
                    double dist = (d0 * d0 + d1 * d1) + dd * dd;
                    if (dist < Rt2) {
                        int slot = atomicAdd(&sh.cnt, 1);
                        if (slot < CAP) {
                            kd[slot] = dist;
                            ki[slot] = id[u];
                        }
                    }
                }
            }
            for (; p < e; ++p) {
                double d0 = g.sx[p] - q0, d1 = g.sy[p] - q1, dd = g.sz[p] - q2;
                double dist = (d0 * d0 + d1 * d1) + dd * dd;
                if (dist < Rt2) {
                    int slot = atomicAdd(&sh.cnt, 1);
                    if (slot < CAP) {
                        kd[slot] = dist;
                        ki[slot] = g.perm[p];
                    }
                }
            }
        }
        knn_sync<NWV>();
        F = sh.cnt;
        knn_sync<NWV>();
        if (F > CAP) {
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
    if (!ok) return false;
    if (n == 1) {
        // the nearest node alone: the smallest key, no sort
        if (lane == 0) {
            double bd = kd[0];
            int bi = ki[0];
            for (int t = 1; t < F; ++t) {
                const double d = kd[t];
                const int i = ki[t];
                if (d < bd || (d == bd && i < bi)) {
                    bd = d;
                    bi = i;
                }
            }
            kd[0] = bd;
            ki[0] = bi;
        }
        knn_sync<NWV>();
        return true;
    }
    int P = 64;
    while (P < F) P <<= 1;
    for (int t = F + lane; t < P; t += NT) {
        kd[t] = DBL_MAX;
        ki[t] = INT_MAX;
    }
    knn_sync<NWV>();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < (P >> 1); t += NT) {
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
            knn_sync<NWV>();
        }
    }
    return true;
}

}  // namespace rbfsl

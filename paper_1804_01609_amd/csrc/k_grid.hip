// Spatial hash of the nodes: a dense G^3 grid over [-1,1]^3 filled by a
// counting sort (count -> exclusive scan -> scatter), then each cell's entries
// ordered by node index so the layout is deterministic.  It plays the role of
// the kd-tree of Sections 2.2 and 3.3.2: built once per node set, then
// searched every step.
#include "rbfsl_impl.h"

namespace rbfsl {

__device__ __forceinline__ int cell1(double v, double invh, int G) {
    const double f = floor((v + 1.0) * invh);
    if (!(f >= 0.0)) return 0;  // also NaN
    return (f > (double)(G - 1)) ? G - 1 : (int)f;
}

__global__ void k_cell_count(const double *nx, const double *ny, const double *nz, int64_t N,
                             int G, double invh, int *cell, int *count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int cx = cell1(nx[i], invh, G), cy = cell1(ny[i], invh, G), cz = cell1(nz[i], invh, G);
    int c = (cz * G + cy) * G + cx;
    cell[i] = c;
    atomicAdd(&count[c], 1);
}

// Exclusive scan of `n` counts into start[0..n] by one 1024-thread block:
// each thread scans a contiguous chunk, then the chunk totals are scanned.
__global__ void __launch_bounds__(1024) k_scan(const int *count, int64_t n, int *start) {
    __shared__ int part[1024];
    int t = threadIdx.x;
    int64_t chunk = (n + 1023) / 1024;
    int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
    int s = 0;
    for (int64_t i = b; i < e; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;  // exclusive prefix of this chunk
    for (int64_t i = b; i < e; ++i) {
        start[i] = run;
        run += count[i];
    }
    if (t == 1023) start[n] = part[1023];
}

__global__ void k_scatter(const int *cell, int64_t N, const int *start, int *fill, int *perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int c = cell[i];
    int pos = start[c] + atomicAdd(&fill[c], 1);
    perm[pos] = (int)i;
}

// order each cell by node index (insertion sort; cells hold a few nodes)
__global__ void k_sort_cells(int64_t ncell, const int *start, int *perm) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int b = start[c], e = start[c + 1];
    for (int i = b + 1; i < e; ++i) {
        int v = perm[i];
        int j = i - 1;
        while (j >= b && perm[j] > v) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

__global__ void k_gather_sorted(const double *nx, const double *ny, const double *nz, int64_t N,
                                const int *perm, double *sx, double *sy, double *sz) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    int i = perm[p];
    sx[p] = nx[i];
    sy[p] = ny[i];
    sz[p] = nz[i];
}

void grid_dims(int64_t N, int n, int *G, double *invh, double *R0) {
    // First search radius: the chordal ball of radius R covers the area pi R^2
    // of the unit sphere, i.e. about N R^2 / 4 quasi-uniform nodes; aim for
    // 1.4 n of them.  Cells are R/1.5 wide, so a ball spans at most 4 cells
    // per axis.
    double R = 2.0 * sqrt(1.4 * (double)n / (double)N);
    if (R > 2.0) R = 2.0;
    double h = R / 1.5;
    int g = (int)ceil(2.0 / h);
    if (g < 1) g = 1;
    if (g > 160) g = 160;
    *G = g;
    *invh = (double)g / 2.0;
    *R0 = R;
}

hipError_t grid_build_in(const double *nx, const double *ny, const double *nz, int64_t N, Grid *g,
                         int *cell, int *count, hipStream_t s) {
    const int G = g->G;
    const int64_t ncell = (int64_t)G * G * G;
    hipError_t e = hipMemsetAsync(count, 0, sizeof(int) * ncell, s);
    if (e != hipSuccess) return e;
    const unsigned bn = (unsigned)((N + 255) / 256);
    const unsigned bc = (unsigned)((ncell + 255) / 256);
    hipLaunchKernelGGL(k_cell_count, dim3(bn), dim3(256), 0, s, nx, ny, nz, N, G, g->invh, cell, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, count, ncell, g->cell_start);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemsetAsync(count, 0, sizeof(int) * ncell, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter, dim3(bn), dim3(256), 0, s, cell, N, g->cell_start, count, g->perm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_cells, dim3(bc), dim3(256), 0, s, ncell, g->cell_start, g->perm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_sorted, dim3(bn), dim3(256), 0, s, nx, ny, nz, N, g->perm, g->sx, g->sy, g->sz);
    return hipGetLastError();
}

hipError_t grid_build(const double *nx, const double *ny, const double *nz, int64_t N, int n,
                      Grid *g, hipStream_t s) {
    grid_dims(N, n, &g->G, &g->invh, &g->R0);
    const int64_t ncell = (int64_t)g->G * g->G * g->G;
    int *cell = nullptr, *count = nullptr;
    hipError_t e;
#define TRY(x) do { e = (x); if (e != hipSuccess) goto fail; } while (0)
    TRY(hipMalloc(&cell, sizeof(int) * N));
    TRY(hipMalloc(&count, sizeof(int) * ncell));
    TRY(hipMalloc(&g->cell_start, sizeof(int) * (ncell + 1)));
    TRY(hipMalloc(&g->perm, sizeof(int) * N));
    TRY(hipMalloc(&g->sx, sizeof(double) * N));
    TRY(hipMalloc(&g->sy, sizeof(double) * N));
    TRY(hipMalloc(&g->sz, sizeof(double) * N));
    TRY(grid_build_in(nx, ny, nz, N, g, cell, count, s));
    TRY(hipStreamSynchronize(s));
    (void)hipFree(cell);
    (void)hipFree(count);
    return hipSuccess;
fail:
    if (cell) (void)hipFree(cell);
    if (count) (void)hipFree(count);
    grid_free(g);
    return e;
#undef TRY
}

void grid_free(Grid *g) {
    if (g->cell_start) (void)hipFree(g->cell_start);
    if (g->perm) (void)hipFree(g->perm);
    if (g->sx) (void)hipFree(g->sx);
    if (g->sy) (void)hipFree(g->sy);
    if (g->sz) (void)hipFree(g->sz);
    g->cell_start = g->perm = nullptr;
    g->sx = g->sy = g->sz = nullptr;
}

}  // namespace rbfsl

// rbfsl_weights_noalloc: the stencil weights of rbfsl_weights (the same
// solver kernels, so the same weights bit for bit) for callers that cannot
// allocate device memory.  Its scratch -- the node, centre and evaluation
// coordinates as separate x, y, z arrays and the status words the solver
// checks and counts failures in -- is the file-scope device array below, of
// a fixed size; every other array is the caller's.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per GPU (hipGetSymbolAddress, with that
// GPU current) and only that address is used.  All calls on one GPU share
// the array: calls that overlap there race, and every call clears the status
// words it uses (with a kernel, not a memset, so that the call can be
// captured in a HIP graph).
#include <mutex>

#include "rbfsl_impl.h"

namespace rbfsl {

// N + 2 count coordinate triples at most: 3 (N + 2 count) doubles
constexpr int64_t NOALLOC_POINTS = 1 << 21;
constexpr int64_t NOALLOC_DOUBLES = 3 * NOALLOC_POINTS;
// the coordinates, then the status words (ST_WORDS ints in 2 doubles)
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES + 2];
static_assert(ST_WORDS * sizeof(int) <= 2 * sizeof(double), "status words fit the tail");

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[NOALLOC_MAX_DEVICES] = {};

// device address of `scratch` on the current device `dev` (looked up once)
hipError_t scratch_address(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

bool on_device(const void *p) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // the query's error is not the caller's
        return false;
    }
    return at.type == hipMemoryTypeDevice;
}

__global__ void k_split_xyz(const double *aos, int64_t count, double *x, double *y, double *z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    x[i] = aos[3 * i];
    y[i] = aos[3 * i + 1];
    z[i] = aos[3 * i + 2];
}

hipError_t split_xyz(const double *aos, int64_t count, double *x, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_xyz, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, aos, count, x,
                       x + count, x + 2 * count);
    return hipGetLastError();
}

}  // namespace
}  // namespace rbfsl

using namespace rbfsl;

extern "C" {

int64_t rbfsl_weights_noalloc_capacity(void) { return NOALLOC_POINTS; }

int rbfsl_weights_noalloc(const double *nodes_xyz, int64_t N, const int32_t *idx, const double *centers,
                          const double *s2, const double *evals, int64_t count, int32_t n, int32_t L,
                          int32_t k, double *w, int32_t *status, void *hip_stream) {
    if (!nodes_xyz || !idx || !centers || !s2 || !evals || !w || N < 1 || count < 0) return RBFSL_E_INVAL;
    int Lr, kr;
    char msg[256];
    if (resolve_stencil(N, n, L, k, &Lr, &kr, msg, sizeof msg) != RBFSL_OK) return RBFSL_E_INVAL;
    if (N > NOALLOC_POINTS || count > NOALLOC_POINTS || N + 2 * count > NOALLOC_POINTS) return RBFSL_E_CAPACITY;
    if (count == 0) return RBFSL_OK;
    const void *arrays[] = {nodes_xyz, idx, centers, s2, evals, w};
    for (const void *a : arrays)
        if (!on_device(a)) return RBFSL_E_INVAL;
    if (status && !on_device(status)) return RBFSL_E_INVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return RBFSL_E_DEVICE;
    double *base = nullptr;
    if (scratch_address(dev, &base) != hipSuccess) return RBFSL_E_DEVICE;
    hipStream_t s = (hipStream_t)hip_stream;
    double *nx = base, *cx = base + 3 * N, *ex = cx + 3 * count;
    int *st = reinterpret_cast<int *>(base + NOALLOC_DOUBLES);
    hipError_t e = split_xyz(nodes_xyz, N, nx, s);
    if (e == hipSuccess) e = split_xyz(centers, count, cx, s);
    if (e == hipSuccess) e = split_xyz(evals, count, ex, s);
    if (e == hipSuccess) e = launch_status_reset(st, s);
    if (e == hipSuccess) {
        SolveArgs a{};
        a.nx = nx; a.ny = nx + N; a.nz = nx + 2 * N; a.N = N;
        a.ex = ex; a.ey = ex + count; a.ez = ex + 2 * count;
        a.cx = cx; a.cy = cx + count; a.cz = cx + 2 * count;
        a.S = idx; a.s2 = s2; a.cidx = nullptr;
        a.count = count; a.n = n; a.L = Lr; a.k = kr;
        a.w = w; a.st_out = status; a.status = st; a.step = 0;
        e = launch_solve(a, s);
    }
    return (e == hipSuccess) ? RBFSL_OK : RBFSL_E_DEVICE;
}

}  // extern "C"

// generate.hip -- synthetic workload on the device: the (2d+1)-point grid
// Laplacians and uniform right-hand sides of the benchmarks, built directly in
// HBM (a serving loop that receives thousands of matrices of up to millions of
// rows cannot build them on the host).  Every value is bit-identical to the host
// generator of the Python package: the same counter-based SplitMix64 draws, the
// same slot order of each row, the diagonal summed in that order, and every
// product and sum rounded on its own (no contraction into fused multiply-adds).
#include "amg.h"
#include "amg_internal.h"

#include <mutex>

// hipcc contracts a * b + c into fused multiply-adds by default; every expression
// of this file must round each product and sum on its own.
#pragma clang fp contract(off)

namespace amg {
namespace {

__device__ inline uint64_t splitmix64_dev(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (k + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// u in [0, 1) with a 53-bit mantissa (exact conversions)
__device__ inline double uniform_dev(uint64_t seed, uint64_t k)
{
    return (double)(splitmix64_dev(seed, k) >> 11) * 0x1.0p-53;
}

struct Grid {
    int d;
    int dims[3];
    int64_t stride[3], ext_stride[3];
    double jitter;
    uint64_t seed;
};

// weight of the grid edge whose lower endpoint has index `lower` on the extended
// grid, in direction a: 1 + jitter (2u - 1)
__device__ inline double edge_weight(const Grid &g, int64_t lower, int a)
{
    if (g.jitter == 0.0) return 1.0;
    const double u = uniform_dev(g.seed, (uint64_t)(lower * g.d + a));
    return 1.0 + g.jitter * (2.0 * u - 1.0);
}

__device__ inline void coords_of(const Grid &g, int64_t i, int (&c)[3], int64_t &ext)
{
    int64_t r = i;
    ext = 0;
    for (int a = 0; a < g.d; a++) {
        c[a] = (int)(r % g.dims[a]);
        r /= g.dims[a];
        ext += (int64_t)(c[a] + 1) * g.ext_stride[a];
    }
}

__global__ void __launch_bounds__(kBlock) k_grid_counts(Grid g, int64_t n, int *__restrict__ cnt)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int c[3];
        int64_t ext;
        coords_of(g, i, c, ext);
        int k = 1;
        for (int a = 0; a < g.d; a++) k += (c[a] > 0) + (c[a] < g.dims[a] - 1);
        cnt[i] = k;
    }
}

__global__ void __launch_bounds__(kBlock) k_grid_fill(Grid g, int64_t n, const int *__restrict__ rp,
                                                      int *__restrict__ ci, double *__restrict__ va)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int c[3];
        int64_t ext;
        coords_of(g, i, c, ext);
        // slots in ascending column order: -z, -y, -x, diagonal, +x, +y, +z
        double wm[3], wp[3];
        for (int a = 0; a < g.d; a++) {
            wm[a] = edge_weight(g, ext - g.ext_stride[a], a);
            wp[a] = edge_weight(g, ext, a);
        }
        double diag = 0.0;  // every incident edge (boundary ones too), in slot order
        for (int a = g.d - 1; a >= 0; a--) diag += wm[a];
        for (int a = 0; a < g.d; a++) diag += wp[a];
        int p = rp[i];
        for (int a = g.d - 1; a >= 0; a--) {
            if (c[a] > 0) {
                ci[p] = (int)(i - g.stride[a]);
                va[p] = -wm[a];
                p++;
            }
        }
        ci[p] = (int)i;
        va[p] = diag;
        p++;
        for (int a = 0; a < g.d; a++) {
            if (c[a] < g.dims[a] - 1) {
                ci[p] = (int)(i + g.stride[a]);
                va[p] = -wp[a];
                p++;
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_uniform_rhs(int64_t n, uint64_t seed, double *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = 2.0 * uniform_dev(seed, (uint64_t)i) - 1.0;
}

int blocks_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

int64_t grid_nnz(int d, const int *dims)
{
    int64_t n = 1;
    for (int a = 0; a < d; a++) n *= dims[a];
    int64_t nnz = n;
    for (int a = 0; a < d; a++) nnz += 2 * (n / dims[a]) * (dims[a] - 1);
    return nnz;
}

void launch_grid_laplacian(int d, const int *dims, double jitter, uint64_t seed, int *rp, int *ci, double *va,
                           int *scan_tmp, hipStream_t s)
{
    Grid g{};
    g.d = d;
    int64_t n = 1, e = 1;
    for (int a = 0; a < d; a++) {
        g.dims[a] = dims[a];
        g.stride[a] = n;
        g.ext_stride[a] = e;
        n *= dims[a];
        e *= dims[a] + 2;
    }
    g.jitter = jitter;
    g.seed = seed;
    k_grid_counts<<<blocks_for(n), kBlock, 0, s>>>(g, n, rp);
    AMG_HIP(hipGetLastError());
    scan_exclusive(rp, rp, n, rp + n, scan_tmp, s);
    k_grid_fill<<<blocks_for(n), kBlock, 0, s>>>(g, n, rp, ci, va);
    AMG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ no-allocation variant
// The scan of the row pointers needs scan_tmp_ints(n) ints of scratch (one block
// total per 2048 rows).  The variant for callers that cannot allocate takes them
// from this array, which every GPU holds for the life of the process: grids of up
// to kNoAllocMaxRows unknowns.  Host code never passes the array's name to a
// kernel (in host code it is a host-side stand-in, not a device address); it
// uses the device address looked up once per GPU below.
constexpr int64_t kNoAllocScratchInts = 65537;  // 256 KiB + 4 B
static_assert(kNoAllocMaxRows == (kNoAllocScratchInts - 1) * 2048, "one block total per 2048 rows");
static __device__ __align__(256) int scratch[kNoAllocScratchInts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
int *scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (the current device's),
// looked up at the first call on that device.
int *scratch_address()
{
    int dev = 0;
    AMG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(AMG_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            throw Error(AMG_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed");
        }
        scratch_ptr[dev] = static_cast<int *>(ptr);
    }
    return scratch_ptr[dev];
}
}  // namespace

void launch_grid_laplacian_noalloc(int d, const int *dims, double jitter, uint64_t seed, int *rp, int *ci,
                                   double *va, hipStream_t s)
{
    int64_t n = 1;
    for (int a = 0; a < d; a++) n *= dims[a];
    if (n > kNoAllocMaxRows || (int64_t)scan_tmp_ints(n) > kNoAllocScratchInts)
        throw Error(AMG_ERR_UNSUPPORTED, "grid larger than the no-allocation scratch");
    launch_grid_laplacian(d, dims, jitter, seed, rp, ci, va, scratch_address(), s);
}

void launch_uniform_rhs(int64_t n, uint64_t seed, double *out, hipStream_t s)
{
    k_uniform_rhs<<<blocks_for(n), kBlock, 0, s>>>(n, seed, out);
    AMG_HIP(hipGetLastError());
}

}  // namespace amg

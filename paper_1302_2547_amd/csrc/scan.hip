// scan.hip -- device-wide exclusive prefix sum of int32 (Blelloch-style scan, the
// "generalised prefix sum" the paper uses to number aggregates, Sec. 5.1).
//
// Three launches: per-block totals, a single-block scan of the totals, and a
// block-local scan plus the block's offset.  Integer sums are exact, so the result
// does not depend on the schedule.
#include "amg_internal.h"

namespace amg {
namespace {

constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;  // 2048 elements per block

// Exclusive scan of one int per thread over the 256-thread block.
__device__ int block_exclusive(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) sh[wid] = x;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) {
        int t = sh[w];
        if (w < wid) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ void __launch_bounds__(kBlock) k_block_totals(const int *__restrict__ in, int64_t n, int *__restrict__ sums)
{
    __shared__ int sh[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++)
        if (base + k < n) s += in[base + k];
    int total;
    block_exclusive(s, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the nb block totals in place; *total_dev = grand total.
__global__ void __launch_bounds__(kBlock) k_scan_totals(int *__restrict__ sums, int nb, int *__restrict__ total_dev)
{
    __shared__ int sh[kBlock / kWave];
    int carry = 0;
    for (int base = 0; base < nb; base += kTile) {
        int v[kItems];
        int s = 0;
        const int first = base + threadIdx.x * kItems;
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            v[k] = (first + k < nb) ? sums[first + k] : 0;
            s += v[k];
        }
        int total;
        int ex = block_exclusive(s, sh, &total) + carry;
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            if (first + k < nb) sums[first + k] = ex;
            ex += v[k];
        }
        carry += total;
    }
    if (threadIdx.x == 0 && total_dev) *total_dev = carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const int *in, int *out, int64_t n, const int *__restrict__ sums)
{
    __shared__ int sh[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int v[kItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive(s, sh, &total) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

}  // namespace

size_t scan_tmp_ints(int64_t n) { return (size_t)((n + kTile - 1) / kTile) + 1; }

void scan_exclusive(const int *in, int *out, int64_t n, int *total_dev, int *tmp, hipStream_t s)
{
    if (n <= 0) {
        if (total_dev) AMG_HIP(hipMemsetAsync(total_dev, 0, sizeof(int), s));
        return;
    }
    const int nb = (int)((n + kTile - 1) / kTile);
    k_block_totals<<<nb, kBlock, 0, s>>>(in, n, tmp);
    k_scan_totals<<<1, kBlock, 0, s>>>(tmp, nb, total_dev);
    k_scan_apply<<<nb, kBlock, 0, s>>>(in, out, n, tmp);
    AMG_HIP(hipGetLastError());
}

}  // namespace amg

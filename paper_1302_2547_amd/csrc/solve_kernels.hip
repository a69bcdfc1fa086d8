// solve_kernels.hip -- gfx950 kernels of the solve phase (Sec. 4).
//
// All matrices are CSR in the nested aggregate order of their level, so that the
// aggregate of every coarse unknown Q is the contiguous range seg_ptr[Q] ..
// seg_ptr[Q+1] of fine rows and its rows' entries are the contiguous range
// srp[Q] .. srp[Q+1] (a "super-row" of P^T A).  A group of G lanes (G | 64)
// serves one row; G is chosen per level from the mean row length so the column
// and value streams stay coalesced.
//
// Inner products use a fixed grid, per-block partial sums and the last-arriving
// block to add the partials in block order: results are identical run to run and
// never leave the device (the K-cycle reads its scalars from device memory).
#include "amg_internal.h"

namespace amg {
namespace {

inline int grid_for(int64_t threads, int cap = 1 << 20)
{
    int64_t b = (threads + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <int G>
__device__ inline double group_sum(double v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Block partial sums of ND values -> partials[d * gridDim.x + block]; the last
// block to arrive adds the partials in block order and writes out[0..ND).
template <int ND>
__device__ void finish_dots(double (&v)[ND], const DotWork &dw, double *out)
{
    __shared__ double sh[ND][kBlock / kWave];
    __shared__ int last;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = 0; d < ND; d++) {
        const double s = wave_sum(v[d]);
        if (lane == 0) sh[d][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < ND) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; w++) s += sh[threadIdx.x][w];
        __hip_atomic_store(&dw.partials[threadIdx.x * kMaxDotBlocks + blockIdx.x], s, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(dw.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int d = wid; d < ND; d += kBlock / kWave) {
        double s = 0.0;
        for (int b = lane; b < (int)gridDim.x; b += kWave)
            s += __hip_atomic_load(&dw.partials[d * kMaxDotBlocks + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s = wave_sum(s);
        if (lane == 0) out[d] = s;
    }
    if (threadIdx.x == 0) __hip_atomic_store(dw.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int G>
__device__ inline double row_product(const int *__restrict__ rp, const int *__restrict__ ci,
                                     const double *__restrict__ va, const double *__restrict__ x, int row, int sub)
{
    double s = 0.0;
    const int e = rp[row + 1];
    for (int p = rp[row] + sub; p < e; p += G) s += va[p] * x[ci[p]];
    return group_sum<G>(s);
}

// ------------------------------------------------------------------ SpMV family

template <int G>
__global__ void __launch_bounds__(kBlock) k_spmv(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const double *__restrict__ va, const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    for (int row = (blockIdx.x * kBlock + threadIdx.x) / G; row < n; row += ngroups) {
        const double s = row_product<G>(rp, ci, va, x, row, sub);
        if (sub == 0) y[row] = s;
    }
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_spmv_dot2(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                      const double *__restrict__ va, const double *__restrict__ x,
                                                      double *__restrict__ y, const double *__restrict__ w,
                                                      DotWork dw, double *__restrict__ out)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    double d[2] = {0.0, 0.0};
    for (int row = (blockIdx.x * kBlock + threadIdx.x) / G; row < n; row += ngroups) {
        const double s = row_product<G>(rp, ci, va, x, row, sub);
        if (sub == 0) {
            y[row] = s;
            const double xr = x[row];
            d[0] += xr * s;
            if (w) d[1] += xr * w[row];
        }
    }
    finish_dots<2>(d, dw, out);
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_spmv_dot3(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                      const double *__restrict__ va, const double *__restrict__ x,
                                                      const double *__restrict__ w1, const double *__restrict__ w2,
                                                      DotWork dw, double *__restrict__ out)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    double d[3] = {0.0, 0.0, 0.0};
    for (int row = (blockIdx.x * kBlock + threadIdx.x) / G; row < n; row += ngroups) {
        const double s = row_product<G>(rp, ci, va, x, row, sub);
        if (sub == 0) {
            const double xr = x[row];
            d[0] += xr * s;
            d[1] += xr * w1[row];
            d[2] += xr * w2[row];
        }
    }
    finish_dots<3>(d, dw, out);
}

// r = b - A x; out[0] = (b, b), out[1] = (r, r)
template <int G>
__global__ void __launch_bounds__(kBlock) k_residual(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const double *__restrict__ va, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r, DotWork dw,
                                                     double *__restrict__ out)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    double d[2] = {0.0, 0.0};
    for (int row = (blockIdx.x * kBlock + threadIdx.x) / G; row < n; row += ngroups) {
        const double s = row_product<G>(rp, ci, va, x, row, sub);
        if (sub == 0) {
            const double br = b[row], rr = br - s;
            r[row] = rr;
            d[0] += br * br;
            d[1] += rr * rr;
        }
    }
    finish_dots<2>(d, dw, out);
}

// ------------------------------------------------------------------ K-cycle pieces

// Pre-smoothing from zero (x = M^-1 r) fused with residual and restriction:
// rc_Q = sum_{q in G_Q} (r_q - (A x)_q) = sum_{seg} r_q - sum_{super-row} a_e minv_t r_t.
template <int G>
__global__ void __launch_bounds__(kBlock) k_pre_restrict(int nc, const int *__restrict__ seg_ptr,
                                                         const int *__restrict__ srp, const int *__restrict__ ci,
                                                         const double *__restrict__ va,
                                                         const double *__restrict__ minv,
                                                         const double *__restrict__ r, double *__restrict__ rc)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    for (int Q = (blockIdx.x * kBlock + threadIdx.x) / G; Q < nc; Q += ngroups) {
        double s = 0.0;
        const int e = srp[Q + 1];
        for (int p = srp[Q] + sub; p < e; p += G) {
            const int t = ci[p];
            s -= va[p] * (minv[t] * r[t]);
        }
        const int qe = seg_ptr[Q + 1];
        for (int q = seg_ptr[Q] + sub; q < qe; q += G) s += r[q];
        s = group_sum<G>(s);
        if (sub == 0) rc[Q] = s;
    }
}

// K-cycle coefficients.  d = [rho1, alpha1, beta, gamma, alpha2] with
// rho1 = (c1, A c1), alpha1 = (c1, rc), beta = (c2, A c2), gamma = (c2, A c1),
// alpha2 = (c2, rt): two flexible-CG steps from zero give
// e = (alpha1/rho1 - (gamma/rho1)(alpha2/rho2)) c1 + (alpha2/rho2) c2,
// rho2 = beta - gamma^2/rho1.  A non-positive rho means A is not SPD: flag it and
// drop the correction.
__device__ inline void kcycle_coefficients(int mode, const double *__restrict__ d, double &a1, double &a2, bool &bad)
{
    a1 = 0.0;
    a2 = 0.0;
    bad = false;
    if (mode == 0) return;
    const double rho1 = d[0];
    if (!(rho1 > 0.0)) {
        bad = true;
        return;
    }
    const double q1 = d[1] / rho1;
    if (mode == 1) {
        a1 = q1;
        return;
    }
    const double g1 = d[3] / rho1;
    const double rho2 = d[2] - d[3] * g1;
    if (!(rho2 > 0.0)) {
        bad = true;
        a1 = q1;
        return;
    }
    a2 = d[4] / rho2;
    a1 = q1 - g1 * a2;
}

__global__ void __launch_bounds__(kBlock) k_inner_residual(int n, const double *__restrict__ rc,
                                                           const double *__restrict__ v1,
                                                           const double *__restrict__ d, double *__restrict__ rt,
                                                           int *__restrict__ flag)
{
    const double rho1 = d[0];
    const bool bad = !(rho1 > 0.0);
    const double s = bad ? 0.0 : d[1] / rho1;
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) rt[i] = rc[i] - s * v1[i];
}

// Prolongation + post-smoothing (Alg. 1 lines "prolongation", "post-smoothing"):
// x = M^-1 r + P e (the pre-smoothed iterate plus the coarse correction) is formed
// on the fly for every column, then out = x + M^-1 (r - A x).
template <int G, int MODE, bool DOT>
__global__ void __launch_bounds__(kBlock) k_post_smooth(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const double *__restrict__ va,
                                                        const double *__restrict__ minv,
                                                        const double *__restrict__ r,
                                                        const int *__restrict__ agg_pos,
                                                        const double *__restrict__ edirect,
                                                        const double *__restrict__ c1,
                                                        const double *__restrict__ c2, const double *__restrict__ d,
                                                        double *__restrict__ xout, const double *__restrict__ wdot,
                                                        DotWork dw, double *__restrict__ out_dot)
{
    double a1 = 0.0, a2 = 0.0;
    bool bad = false;
    if (MODE != 0) kcycle_coefficients(MODE, d, a1, a2, bad);
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(dw.flag, 1);
    auto corr = [&](int J) -> double {
        if (MODE == 0) return edirect[J];
        if (MODE == 1) return a1 * c1[J];
        return a1 * c1[J] + a2 * c2[J];
    };
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    double dsum[1] = {0.0};
    for (int row = (blockIdx.x * kBlock + threadIdx.x) / G; row < n; row += ngroups) {
        double s = 0.0;
        const int e = rp[row + 1];
        for (int p = rp[row] + sub; p < e; p += G) {
            const int t = ci[p];
            s += va[p] * (minv[t] * r[t] + corr(agg_pos[t]));
        }
        s = group_sum<G>(s);
        if (sub == 0) {
            const double mr = minv[row], rr = r[row];
            const double x = mr * rr + corr(agg_pos[row]);
            const double o = x + mr * (rr - s);
            xout[row] = o;
            if (DOT) dsum[0] += o * wdot[row];
        }
    }
    if (DOT) finish_dots<1>(dsum, dw, out_dot);
}

// y = A x for a dense row-major n x n matrix: one wavefront per row.
__global__ void __launch_bounds__(kBlock) k_dense_gemv(int n, const double *__restrict__ a,
                                                       const double *__restrict__ x, double *__restrict__ y)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int nw = gridDim.x * (kBlock / kWave);
    for (int i = (blockIdx.x * kBlock + threadIdx.x) / kWave; i < n; i += nw) {
        double s = 0.0;
        const double *row = a + (size_t)i * n;
        for (int j = lane; j < n; j += kWave) s += row[j] * x[j];
        s = wave_sum(s);
        if (lane == 0) y[i] = s;
    }
}

// ------------------------------------------------------------------ outer flexible CG

// alpha = (p, r) / (p, A p); x += alpha p; r -= alpha q; out = (r, r)
__global__ void __launch_bounds__(kBlock) k_fcg_update(int n, const double *__restrict__ pq_pr,
                                                       double *__restrict__ x, double *__restrict__ r,
                                                       const double *__restrict__ p, const double *__restrict__ q,
                                                       DotWork dw, double *__restrict__ out)
{
    const double pq = pq_pr[0];
    const bool bad = !(pq > 0.0);
    const double alpha = bad ? 0.0 : pq_pr[1] / pq;
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(dw.flag, 1);
    double d[1] = {0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        d[0] += ri * ri;
    }
    finish_dots<1>(d, dw, out);
}

// beta = -(z, A p) / (p, A p); p = z + beta p
__global__ void __launch_bounds__(kBlock) k_fcg_direction(int n, const double *__restrict__ pq,
                                                          const double *__restrict__ zq,
                                                          const double *__restrict__ z, double *__restrict__ p,
                                                          int *__restrict__ flag)
{
    const bool bad = !(pq[0] > 0.0);
    const double beta = bad ? 0.0 : -zq[0] / pq[0];
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kBlock) k_dot(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                DotWork dw, double *__restrict__ out)
{
    double d[1] = {0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[0] += a[i] * b[i];
    finish_dots<1>(d, dw, out);
}

__global__ void __launch_bounds__(kBlock) k_gather(int n, const double *__restrict__ src, const int *__restrict__ idx,
                                                   double *__restrict__ dst)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = src[idx[i]];
}

__global__ void __launch_bounds__(kBlock) k_scatter(int n, const double *__restrict__ src, const int *__restrict__ idx,
                                                    double *__restrict__ dst)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[idx[i]] = src[i];
}

}  // namespace

// ------------------------------------------------------------------ launchers

int lanes_for(double avg_row_len)
{
    int g = 2;
    while (g < avg_row_len && g < kWave) g <<= 1;
    return g;
}

#define AMG_SWITCH_G(G, BODY)                          \
    switch (G) {                                       \
    case 1: { constexpr int kG = 1; BODY; } break;     \
    case 2: { constexpr int kG = 2; BODY; } break;     \
    case 4: { constexpr int kG = 4; BODY; } break;     \
    case 8: { constexpr int kG = 8; BODY; } break;     \
    case 16: { constexpr int kG = 16; BODY; } break;   \
    case 32: { constexpr int kG = 32; BODY; } break;   \
    default: { constexpr int kG = 64; BODY; } break;   \
    }

void launch_spmv(int n, const int *rp, const int *ci, const double *va, const double *x, double *y, int G,
                 hipStream_t s)
{
    const int grid = grid_for((int64_t)n * G);
    AMG_SWITCH_G(G, (k_spmv<kG><<<grid, kBlock, 0, s>>>(n, rp, ci, va, x, y)));
    AMG_HIP(hipGetLastError());
}

void launch_spmv_dot2(int n, const int *rp, const int *ci, const double *va, const double *x, double *y,
                      const double *w, int G, DotWork dw, double *out, hipStream_t s)
{
    const int grid = grid_for((int64_t)n * G, kMaxDotBlocks);
    AMG_SWITCH_G(G, (k_spmv_dot2<kG><<<grid, kBlock, 0, s>>>(n, rp, ci, va, x, y, w, dw, out)));
    AMG_HIP(hipGetLastError());
}

void launch_spmv_dot3(int n, const int *rp, const int *ci, const double *va, const double *x, const double *w1,
                      const double *w2, int G, DotWork dw, double *out, hipStream_t s)
{
    const int grid = grid_for((int64_t)n * G, kMaxDotBlocks);
    AMG_SWITCH_G(G, (k_spmv_dot3<kG><<<grid, kBlock, 0, s>>>(n, rp, ci, va, x, w1, w2, dw, out)));
    AMG_HIP(hipGetLastError());
}

void launch_residual(int n, const int *rp, const int *ci, const double *va, const double *b, const double *x,
                     double *r, int G, DotWork dw, double *out, hipStream_t s)
{
    const int grid = grid_for((int64_t)n * G, kMaxDotBlocks);
    AMG_SWITCH_G(G, (k_residual<kG><<<grid, kBlock, 0, s>>>(n, rp, ci, va, b, x, r, dw, out)));
    AMG_HIP(hipGetLastError());
}

void launch_pre_restrict(int nc, const int *seg_ptr, const int *srp, const int *ci, const double *va,
                         const double *minv, const double *r, double *rc, int G, hipStream_t s)
{
    const int grid = grid_for((int64_t)nc * G);
    AMG_SWITCH_G(G, (k_pre_restrict<kG><<<grid, kBlock, 0, s>>>(nc, seg_ptr, srp, ci, va, minv, r, rc)));
    AMG_HIP(hipGetLastError());
}

void launch_inner_residual(int n, const double *rc, const double *v1, const double *d, double *rt, int *flag,
                           hipStream_t s)
{
    k_inner_residual<<<grid_for(n, 4096), kBlock, 0, s>>>(n, rc, v1, d, rt, flag);
    AMG_HIP(hipGetLastError());
}

void launch_post_smooth(int n, const int *rp, const int *ci, const double *va, const double *minv, const double *r,
                        const int *agg_pos, int mode, const double *edirect, const double *c1, const double *c2,
                        const double *d, double *xout, const double *wdot, DotWork dw, double *out_dot, int G,
                        hipStream_t s)
{
    const bool dot = wdot != nullptr;
    const int grid = grid_for((int64_t)n * G, dot ? kMaxDotBlocks : (1 << 20));
#define AMG_POST(M, D)                                                                                        \
    AMG_SWITCH_G(G, (k_post_smooth<kG, M, D><<<grid, kBlock, 0, s>>>(n, rp, ci, va, minv, r, agg_pos, edirect, \
                                                                      c1, c2, d, xout, wdot, dw, out_dot)))
    if (mode == 0) {
        if (dot) { AMG_POST(0, true); } else { AMG_POST(0, false); }
    } else if (mode == 1) {
        if (dot) { AMG_POST(1, true); } else { AMG_POST(1, false); }
    } else {
        if (dot) { AMG_POST(2, true); } else { AMG_POST(2, false); }
    }
#undef AMG_POST
    AMG_HIP(hipGetLastError());
}

void launch_dense_gemv(int n, const double *a, const double *x, double *y, hipStream_t s)
{
    k_dense_gemv<<<grid_for((int64_t)n * kWave), kBlock, 0, s>>>(n, a, x, y);
    AMG_HIP(hipGetLastError());
}

void launch_fcg_update(int n, const double *pq_pr, double *x, double *r, const double *p, const double *q,
                       DotWork dw, double *out, hipStream_t s)
{
    k_fcg_update<<<grid_for(n, kMaxDotBlocks), kBlock, 0, s>>>(n, pq_pr, x, r, p, q, dw, out);
    AMG_HIP(hipGetLastError());
}

void launch_fcg_direction(int n, const double *pq, const double *zq, const double *z, double *p, int *flag,
                          hipStream_t s)
{
    k_fcg_direction<<<grid_for(n, 4096), kBlock, 0, s>>>(n, pq, zq, z, p, flag);
    AMG_HIP(hipGetLastError());
}

void launch_dot(int n, const double *a, const double *b, DotWork dw, double *out, hipStream_t s)
{
    k_dot<<<grid_for(n, kMaxDotBlocks), kBlock, 0, s>>>(n, a, b, dw, out);
    AMG_HIP(hipGetLastError());
}

void launch_gather(int n, const double *src, const int *idx, double *dst, hipStream_t s)
{
    k_gather<<<grid_for(n, 4096), kBlock, 0, s>>>(n, src, idx, dst);
    AMG_HIP(hipGetLastError());
}

void launch_scatter(int n, const double *src, const int *idx, double *dst, hipStream_t s)
{
    k_scatter<<<grid_for(n, 4096), kBlock, 0, s>>>(n, src, idx, dst);
    AMG_HIP(hipGetLastError());
}

}  // namespace amg

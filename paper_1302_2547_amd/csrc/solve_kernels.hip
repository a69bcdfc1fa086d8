// solve_kernels.hip -- gfx950 kernels of the solve phase (Sec. 4).
//
// All matrices are CSR in the nested aggregate order of their level, so the
// aggregate of coarse unknown Q is the contiguous range seg_ptr[Q] .. seg_ptr[Q+1]
// of fine rows, and its rows' entries form the contiguous "super-row" srp[Q] ..
// srp[Q+1] of P^T A.
//
// Row mapping.  A group of G lanes (G | 64) serves one ordinary row, G chosen per
// level from the mean row length so the column/value streams stay coalesced.
// Coarse levels of 3D problems contain hub rows with thousands of entries; rows
// longer than R.lim are cut into chunks of at most kChunk entries, one block per
// chunk; the last chunk of a row to finish adds the chunk sums in chunk order and
// runs the row's epilogue.
//
// Inner products.  A producing kernel writes one partial sum per block (plus one
// per hub row) -- no fences; a consumer reduces the partials in a fixed order.  Small
// partial sets are reduced by every consumer block itself; large ones by one
// extra block (k_reduce_partials).  Results are identical run to run and never
// leave the device, so the K-cycle has no host round trip.
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

// Sum over the block; every thread receives the same value (fixed order).
__device__ inline double block_sum(double v)
{
    __shared__ double sh[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) s += sh[w];
    __syncthreads();
    return s;
}

// Sums N values over the block in one synchronisation round; every thread
// receives the sums (fixed order).
template <int N>
__device__ inline void block_sums(double (&v)[N])
{
    __shared__ double sh[N][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = 0; d < N; d++) {
        const double t = wave_sum(v[d]);
        if (lane == 0) sh[d][wid] = t;
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < N; d++) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; w++) t += sh[d][w];
        v[d] = t;
    }
    __syncthreads();
}

// Values of N dot products from their partials (same values in every thread).
template <int N>
__device__ inline void dot_values(const DotRef *refs, double (&out)[N])
{
    bool all_final = true;
#pragma unroll
    for (int d = 0; d < N; d++) all_final = all_final && refs[d].count == 1;
    if (all_final) {
#pragma unroll
        for (int d = 0; d < N; d++) out[d] = refs[d].part[0];
        return;
    }
#pragma unroll
    for (int d = 0; d < N; d++) {
        double t = 0.0;
        for (int b = threadIdx.x; b < refs[d].count; b += kBlock) t += refs[d].part[b];
        out[d] = t;
    }
    block_sums<N>(out);
}

__device__ inline double dot_value(DotRef r)
{
    double v[1];
    dot_values<1>(&r, v);
    return v[0];
}

// Writes this block's partials of ND dot products: part[d * kPartStride + block].
template <int ND>
__device__ inline void store_partials(const double (&v)[ND], double *part)
{
    double t[ND];
#pragma unroll
    for (int d = 0; d < ND; d++) t[d] = v[d];
    block_sums<ND>(t);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < ND; d++) part[d * kPartStride + blockIdx.x] = t[d];
    }
}

// Visits every row of R once and calls epi(row, sum, k) with the row's reduced
// sum; k = -1 for an ordinary row, else the index of the hub row (0 .. nlong).
// range(beg, end, lane, width) returns one lane's share of entries [beg, end).
template <int G, class Range, class Epi>
__device__ inline void visit_rows(const Rows &R, Range range, Epi epi)
{
    const int nlb = R.nchunks < kLongBlocks ? R.nchunks : kLongBlocks;
    if ((int)blockIdx.x < nlb) {
        for (int c = blockIdx.x; c < R.nchunks; c += nlb) {
            const Chunk ch = R.chunks[c];
            const double s = block_sum(range(ch.beg, ch.end, (int)threadIdx.x, kBlock));
            const int first = R.long_first[ch.k], m = R.long_first[ch.k + 1] - first;
            if (threadIdx.x == 0) {
                if (m == 1) {
                    epi(ch.row, s, ch.k);
                } else {
                    __hip_atomic_store(&R.chunk_sum[c], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned prev =
                        __hip_atomic_fetch_add(&R.arrive[ch.k], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                    if (prev == (unsigned)(m - 1)) {  // last chunk of this row to finish
                        double t = 0.0;
                        for (int j = first; j < first + m; j++)
                            t += __hip_atomic_load(&R.chunk_sum[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&R.arrive[ch.k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        epi(ch.row, t, ch.k);
                    }
                }
            }
        }
        return;
    }
    const int sub = threadIdx.x % G;
    const int ngroups = (gridDim.x - nlb) * (kBlock / G);
    for (int row = ((blockIdx.x - nlb) * kBlock + threadIdx.x) / G; row < R.n; row += ngroups) {
        const int b = R.ptr[row], e = R.ptr[row + 1];
        if (e - b > R.lim) continue;  // hub row: served by the chunk blocks (uniform within the group)
        const double s = group_sum<G>(range(b, e, sub, G));
        if (sub == 0) epi(row, s, -1);
    }
}

// ------------------------------------------------------------------ SpMV family

template <int G>
__global__ void __launch_bounds__(kBlock) k_spmv(Rows R, const int *__restrict__ ci, const double *__restrict__ va,
                                                 const double *__restrict__ x, double *__restrict__ y)
{
    visit_rows<G>(
        R,
        [&](int b, int e, int lane, int width) {
            double s = 0.0;
            for (int p = b + lane; p < e; p += width) s += va[p] * x[ci[p]];
            return s;
        },
        [&](int row, double s, int) { y[row] = s; });
}

// y = A x (y may be NULL); dots (x, Ax) and, for each non-NULL w_j, (x, w_j).
template <int G, int ND>
__global__ void __launch_bounds__(kBlock) k_spmv_dots(Rows R, const int *__restrict__ ci,
                                                      const double *__restrict__ va, const double *__restrict__ x,
                                                      double *__restrict__ y, const double *__restrict__ w1,
                                                      const double *__restrict__ w2, double *__restrict__ part)
{
    double d[ND] = {};
    const int nb = gridDim.x;
    visit_rows<G>(
        R,
        [&](int b, int e, int lane, int width) {
            double s = 0.0;
            for (int p = b + lane; p < e; p += width) s += va[p] * x[ci[p]];
            return s;
        },
        [&](int row, double s, int k) {
            if (y) y[row] = s;
            const double xr = x[row];
            double t[ND];
            t[0] = xr * s;
            if (ND > 1) t[1] = xr * w1[row];
            if (ND > 2) t[2] = xr * w2[row];
            if (k < 0) {
#pragma unroll
                for (int j = 0; j < ND; j++) d[j] += t[j];
            } else {
#pragma unroll
                for (int j = 0; j < ND; j++) part[j * kPartStride + nb + k] = t[j];
            }
        });
    store_partials<ND>(d, part);
}

// r = b - A x; partials of (b, b) and (r, r)
template <int G>
__global__ void __launch_bounds__(kBlock) k_residual(Rows R, const int *__restrict__ ci,
                                                     const double *__restrict__ va, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ part)
{
    double d[2] = {0.0, 0.0};
    const int nb = gridDim.x;
    visit_rows<G>(
        R,
        [&](int beg, int end, int lane, int width) {
            double s = 0.0;
            for (int p = beg + lane; p < end; p += width) s += va[p] * x[ci[p]];
            return s;
        },
        [&](int row, double s, int k) {
            const double br = b[row], rr = br - s;
            r[row] = rr;
            if (k < 0) {
                d[0] += br * br;
                d[1] += rr * rr;
            } else {
                part[nb + k] = br * br;
                part[kPartStride + nb + k] = rr * rr;
            }
        });
    store_partials<2>(d, part);
}

// One block of 1024 threads reduces large partial sets (fixed order).
constexpr int kReduceThreads = 1024;
__global__ void __launch_bounds__(kReduceThreads) k_reduce_partials(int nd, const double *__restrict__ part,
                                                                    int count, double *__restrict__ out)
{
    __shared__ double sh[kReduceThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int d = 0; d < nd; d++) {
        const double *src = part + d * kPartStride;
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        int b = threadIdx.x;
        for (; b + 3 * kReduceThreads < count; b += 4 * kReduceThreads) {
#pragma unroll
            for (int u = 0; u < 4; u++) t[u] += src[b + u * kReduceThreads];
        }
        for (; b < count; b += kReduceThreads) t[0] += src[b];
        double v = wave_sum((t[0] + t[1]) + (t[2] + t[3]));
        if (lane == 0) sh[wid] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0;
            for (int w = 0; w < kReduceThreads / kWave; w++) a += sh[w];
            out[d] = a;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ K-cycle pieces

// Pre-smoothing from zero fused with residual and restriction.  With x = M^-1 r,
// rc_Q = sum_{q in G_Q} (r - A x)_q = sum_{e in super-row Q} w_e r_{col(e)} where
// w = P^T (I - A M^-1) is stored per entry (w_e = [diagonal] - a_e minv_col).
template <int G>
__global__ void __launch_bounds__(kBlock) k_restrict(Rows S, const int *__restrict__ ci,
                                                     const double *__restrict__ wv, const double *__restrict__ r,
                                                     double *__restrict__ rc)
{
    visit_rows<G>(
        S,
        [&](int b, int e, int lane, int width) {
            double s = 0.0;
            for (int p = b + lane; p < e; p += width) s += wv[p] * r[ci[p]];
            return s;
        },
        [&](int Q, double s, int) { rc[Q] = s; });
}

// K-cycle coefficients.  rho1 = (c1, A c1), alpha1 = (c1, rc), beta = (c2, A c2),
// gamma = (c2, A c1), alpha2 = (c2, rt): two flexible-CG steps from zero give
// e = (alpha1/rho1 - (gamma/rho1)(alpha2/rho2)) c1 + (alpha2/rho2) c2,
// rho2 = beta - gamma^2/rho1.  A non-positive rho means A is not SPD: the flag is
// raised and the correction dropped.
struct KCoef {
    double a1, a2;
    bool bad;
};

__device__ inline KCoef kcycle_coefficients(int mode, const KDots &kd)
{
    KCoef c{0.0, 0.0, false};
    if (mode == 0 || mode == 3) return c;
    double rho1, alpha1, beta = 0.0, gamma = 0.0, alpha2 = 0.0;
    if (mode == 2) {
        const DotRef refs[5] = {kd.rho1, kd.alpha1, kd.beta, kd.gamma, kd.alpha2};
        double v[5];
        dot_values<5>(refs, v);
        rho1 = v[0];
        alpha1 = v[1];
        beta = v[2];
        gamma = v[3];
        alpha2 = v[4];
    } else {
        const DotRef refs[2] = {kd.rho1, kd.alpha1};
        double v[2];
        dot_values<2>(refs, v);
        rho1 = v[0];
        alpha1 = v[1];
    }
    if (!(rho1 > 0.0)) {
        c.bad = true;
        return c;
    }
    const double q1 = alpha1 / rho1;
    c.a1 = q1;
    if (mode == 1) return c;
    const double g1 = gamma / rho1;
    const double rho2 = beta - gamma * g1;
    if (!(rho2 > 0.0)) {
        c.bad = true;
        return c;
    }
    c.a2 = alpha2 / rho2;
    c.a1 = q1 - g1 * c.a2;
    return c;
}

// Restriction of the inner residual of the parent's first flexible-CG step:
// rt = rcf - (alpha1/rho1) v1 is formed on the fly (and stored for the later
// kernels of the visit), rc = W rt.
template <int G>
__global__ void __launch_bounds__(kBlock) k_restrict_rt(Rows S, int nf, const int *__restrict__ ci,
                                                        const double *__restrict__ wv,
                                                        const double *__restrict__ rcf,
                                                        const double *__restrict__ v1, KDots kd,
                                                        double *__restrict__ rt, double *__restrict__ rc,
                                                        int *__restrict__ flag)
{
    const KCoef c = kcycle_coefficients(1, kd);
    if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    const double a = c.a1;
    for (int q = blockIdx.x * kBlock + threadIdx.x; q < nf; q += gridDim.x * kBlock) rt[q] = rcf[q] - a * v1[q];
    visit_rows<G>(
        S,
        [&](int b, int e, int lane, int width) {
            double s = 0.0;
            for (int p = b + lane; p < e; p += width) {
                const int t = ci[p];
                s += wv[p] * (rcf[t] - a * v1[t]);
            }
            return s;
        },
        [&](int Q, double s, int) { rc[Q] = s; });
}

// rt = rc - (alpha1/rho1) v1
__global__ void __launch_bounds__(kBlock) k_inner_residual(int n, const double *__restrict__ rc,
                                                           const double *__restrict__ v1, KDots kd,
                                                           double *__restrict__ rt, int *__restrict__ flag)
{
    const KCoef c = kcycle_coefficients(1, kd);
    if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) rt[i] = rc[i] - c.a1 * v1[i];
}

// Prolongation + post-smoothing: x = M^-1 r + P e (the pre-smoothed iterate plus
// the coarse correction) is formed on the fly for every column (cagg[p], when
// given, is the coarse unknown of column ci[p] stored per entry: on small,
// latency-bound levels it saves a dependent gather), then
// out = x + M^-1 (r - A x).  mode 0: e = edirect; mode 1: e = a1 c1;
// mode 2: e = a1 c1 + a2 c2; mode 3: e = ainv edirect (small dense coarsest level).
// DOT adds partials of (out, wdot).
template <int G, int MODE, bool DOT, bool CAGG>
__global__ void __launch_bounds__(kBlock) k_post_smooth(Rows R, const int *__restrict__ ci,
                                                        const double *__restrict__ va,
                                                        const double *__restrict__ minv,
                                                        const double *__restrict__ r,
                                                        const int *__restrict__ agg_pos,
                                                        const int *__restrict__ cagg,
                                                        const double *__restrict__ edirect,
                                                        const double *__restrict__ c1,
                                                        const double *__restrict__ c2, KDots kd,
                                                        double *__restrict__ xout, const double *__restrict__ wdot,
                                                        double *__restrict__ part, int *__restrict__ flag,
                                                        const double *__restrict__ ainv, int nc)
{
    const KCoef c = kcycle_coefficients(MODE, kd);
    if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    const double a1 = c.a1, a2 = c.a2;
    __shared__ double e_sh[MODE == 3 ? kInlineCoarse : 1];
    if (MODE == 3) {  // e = A_coarsest^-1 rc, computed by every block into LDS
        for (int i = threadIdx.x; i < nc; i += kBlock) {
            double t = 0.0;
            for (int j = 0; j < nc; j++) t += ainv[i * nc + j] * edirect[j];
            e_sh[i] = t;
        }
        __syncthreads();
    }
    auto corr = [&](int J) -> double {
        if (MODE == 0) return edirect[J];
        if (MODE == 3) return e_sh[J];
        if (MODE == 1) return a1 * c1[J];
        return a1 * c1[J] + a2 * c2[J];
    };
    double dsum[1] = {0.0};
    const int nb = gridDim.x;
    visit_rows<G>(
        R,
        [&](int b, int e, int lane, int width) {
            double s = 0.0;
            for (int p = b + lane; p < e; p += width) {
                const int t = ci[p];
                s += va[p] * (minv[t] * r[t] + corr(CAGG ? cagg[p] : agg_pos[t]));
            }
            return s;
        },
        [&](int row, double s, int k) {
            const double mr = minv[row], rr = r[row];
            const double x = mr * rr + corr(agg_pos[row]);
            const double o = x + mr * (rr - s);
            xout[row] = o;
            if (DOT) {
                if (k < 0) dsum[0] += o * wdot[row];
                else part[nb + k] = o * wdot[row];
            }
        });
    if (DOT) store_partials<1>(dsum, part);
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

// alpha = (p, r) / (p, A p); x += alpha p; r -= alpha q; partials of (r, r)
__global__ void __launch_bounds__(kBlock) k_fcg_update(int n, DotRef pq, DotRef pr, double *__restrict__ x,
                                                       double *__restrict__ r, const double *__restrict__ p,
                                                       const double *__restrict__ q, double *__restrict__ part,
                                                       int *__restrict__ flag)
{
    const double vpq = dot_value(pq), vpr = dot_value(pr);
    const bool bad = !(vpq > 0.0);
    const double alpha = bad ? 0.0 : vpr / vpq;
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    double d[1] = {0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        d[0] += ri * ri;
    }
    store_partials<1>(d, part);
}

// beta = -(z, A p) / (p, A p); p = z + beta p
__global__ void __launch_bounds__(kBlock) k_fcg_direction(int n, DotRef pq, DotRef zq, const double *__restrict__ z,
                                                          double *__restrict__ p, int *__restrict__ flag)
{
    const double vpq = dot_value(pq), vzq = dot_value(zq);
    const bool bad = !(vpq > 0.0);
    const double beta = bad ? 0.0 : -vzq / vpq;
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kBlock) k_dot(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                double *__restrict__ part)
{
    double d[1] = {0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[0] += a[i] * b[i];
    store_partials<1>(d, part);
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

// w_e = [col(e) is the row's diagonal] - a_e minv_col(e) for every entry (solve
// layout); G lanes per row
template <int G>
__global__ void __launch_bounds__(kBlock) k_restriction_weights(int n, const int *__restrict__ rp,
                                                                const int *__restrict__ ci,
                                                                const double *__restrict__ va,
                                                                const double *__restrict__ minv,
                                                                double *__restrict__ wv)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    for (int q = (blockIdx.x * kBlock + threadIdx.x) / G; q < n; q += ngroups) {
        for (int p = rp[q] + sub; p < rp[q + 1]; p += G) {
            const int t = ci[p];
            wv[p] = (t == q ? 1.0 : 0.0) - va[p] * minv[t];
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_entry_coarse_column(int nnz, const int *__restrict__ ci,
                                                                const int *__restrict__ agg_pos,
                                                                int *__restrict__ cagg)
{
    for (int p = blockIdx.x * kBlock + threadIdx.x; p < nnz; p += gridDim.x * kBlock) cagg[p] = agg_pos[ci[p]];
}

inline int rows_grid(const Rows &R, int G, int cap)
{
    const int nlb = R.nchunks < kLongBlocks ? R.nchunks : kLongBlocks;
    return nlb + grid_for((int64_t)R.n * G, cap - nlb);
}

// Partial sets larger than this are reduced by one extra block instead of by
// every consumer block.
constexpr int kConsumerReduceMax = 1024;

void reduce_if_large(int nd, double *part, int count, double *final_out, hipStream_t s)
{
    if (count > kConsumerReduceMax && final_out) {
        k_reduce_partials<<<1, kReduceThreads, 0, s>>>(nd, part, count, final_out);
        AMG_HIP(hipGetLastError());
    }
}

DotRef finished(double *part, int count, double *final_out, int d)
{
    if (count <= kConsumerReduceMax || final_out == nullptr) return DotRef{part + d * kPartStride, count};
    return DotRef{final_out + d, 1};
}

}  // namespace

// ------------------------------------------------------------------ launchers

int lanes_for(double avg_row_len, int n)
{
    // largest power of two not above the mean row length; at least 8 lanes on
    // small (latency-bound) levels so that ordinary rows take one step
    int g = 1;
    while (2 * g <= avg_row_len && g < kWave) g <<= 1;
    if (n < kSmallLevel && g < 8) g = 8;
    if (g < 2) g = 2;
    return g;
}

#define AMG_SWITCH_G(G, BODY)                          \
    switch (G) {                                       \
    case 2: { constexpr int kG = 2; BODY; } break;     \
    case 4: { constexpr int kG = 4; BODY; } break;     \
    case 8: { constexpr int kG = 8; BODY; } break;     \
    case 16: { constexpr int kG = 16; BODY; } break;   \
    case 32: { constexpr int kG = 32; BODY; } break;   \
    default: { constexpr int kG = 64; BODY; } break;   \
    }

void launch_spmv(Rows R, const int *ci, const double *va, const double *x, double *y, int G, hipStream_t s)
{
    const int grid = rows_grid(R, G, 1 << 20);
    AMG_SWITCH_G(G, (k_spmv<kG><<<grid, kBlock, 0, s>>>(R, ci, va, x, y)));
    AMG_HIP(hipGetLastError());
}

DotSet launch_spmv_dots(Rows R, const int *ci, const double *va, const double *x, double *y, const double *w1,
                        const double *w2, int G, DotBuf buf, hipStream_t s)
{
    const int grid = rows_grid(R, G, kMaxDotBlocks);
    const int nd = w2 ? 3 : (w1 ? 2 : 1);
    if (nd == 1) {
        AMG_SWITCH_G(G, (k_spmv_dots<kG, 1><<<grid, kBlock, 0, s>>>(R, ci, va, x, y, w1, w2, buf.part)));
    } else if (nd == 2) {
        AMG_SWITCH_G(G, (k_spmv_dots<kG, 2><<<grid, kBlock, 0, s>>>(R, ci, va, x, y, w1, w2, buf.part)));
    } else {
        AMG_SWITCH_G(G, (k_spmv_dots<kG, 3><<<grid, kBlock, 0, s>>>(R, ci, va, x, y, w1, w2, buf.part)));
    }
    AMG_HIP(hipGetLastError());
    const int count = grid + R.nlong;
    reduce_if_large(nd, buf.part, count, buf.final_out, s);
    DotSet out{};
    for (int d = 0; d < nd; d++) out.d[d] = finished(buf.part, count, buf.final_out, d);
    return out;
}

DotSet launch_residual(Rows R, const int *ci, const double *va, const double *b, const double *x, double *r, int G,
                       DotBuf buf, hipStream_t s)
{
    const int grid = rows_grid(R, G, kMaxDotBlocks);
    AMG_SWITCH_G(G, (k_residual<kG><<<grid, kBlock, 0, s>>>(R, ci, va, b, x, r, buf.part)));
    AMG_HIP(hipGetLastError());
    const int count = grid + R.nlong;
    reduce_if_large(2, buf.part, count, buf.final_out, s);
    DotSet out{};
    for (int d = 0; d < 2; d++) out.d[d] = finished(buf.part, count, buf.final_out, d);
    return out;
}

void launch_reduce(const DotRef &ref, double *out, hipStream_t s)
{
    k_reduce_partials<<<1, kReduceThreads, 0, s>>>(1, ref.part, ref.count, out);
    AMG_HIP(hipGetLastError());
}

void launch_restrict(Rows S, const int *ci, const double *wv, const double *r, double *rc, int G, hipStream_t s)
{
    const int grid = rows_grid(S, G, 1 << 20);
    AMG_SWITCH_G(G, (k_restrict<kG><<<grid, kBlock, 0, s>>>(S, ci, wv, r, rc)));
    AMG_HIP(hipGetLastError());
}

void launch_inner_residual(int n, const double *rc, const double *v1, KDots kd, double *rt, int *flag, hipStream_t s)
{
    k_inner_residual<<<grid_for(n, 4096), kBlock, 0, s>>>(n, rc, v1, kd, rt, flag);
    AMG_HIP(hipGetLastError());
}

DotRef launch_post_smooth(Rows R, const int *ci, const double *va, const double *minv, const double *r,
                          const int *agg_pos, const int *cagg, int mode, const double *edirect, const double *c1, const double *c2,
                          KDots kd, double *xout, const double *wdot, DotBuf buf, int *flag, int G, hipStream_t s,
                          const double *ainv, int nc)
{
    const bool dot = wdot != nullptr;
    const int grid = rows_grid(R, G, dot ? kMaxDotBlocks : (1 << 20));
#define AMG_POST(M, D)                                                                                        \
    do {                                                                                                      \
        if (cagg) {                                                                                           \
            AMG_SWITCH_G(G, (k_post_smooth<kG, M, D, true><<<grid, kBlock, 0, s>>>(                           \
                                R, ci, va, minv, r, agg_pos, cagg, edirect, c1, c2, kd, xout, wdot, buf.part, flag, \
                                ainv, nc)));                                                                  \
        } else {                                                                                              \
            AMG_SWITCH_G(G, (k_post_smooth<kG, M, D, false><<<grid, kBlock, 0, s>>>(                          \
                                R, ci, va, minv, r, agg_pos, cagg, edirect, c1, c2, kd, xout, wdot, buf.part, flag, \
                                ainv, nc)));                                                                  \
        }                                                                                                     \
    } while (0)
    switch (mode) {
    case 0: if (dot) { AMG_POST(0, true); } else { AMG_POST(0, false); } break;
    case 1: if (dot) { AMG_POST(1, true); } else { AMG_POST(1, false); } break;
    case 2: if (dot) { AMG_POST(2, true); } else { AMG_POST(2, false); } break;
    default:
        if (nc < 1 || nc > kInlineCoarse || !ainv) throw Error(4, "inline coarsest solve out of range");
        if (dot) { AMG_POST(3, true); } else { AMG_POST(3, false); }
        break;
    }
#undef AMG_POST
    AMG_HIP(hipGetLastError());
    if (!dot) return DotRef{nullptr, 0};
    const int count = grid + R.nlong;
    reduce_if_large(1, buf.part, count, buf.final_out, s);
    return finished(buf.part, count, buf.final_out, 0);
}

void launch_restrict_rt(Rows S, int nf, const int *ci, const double *wv, const double *rcf, const double *v1,
                        KDots kd, double *rt, double *rc, int *flag, int G, hipStream_t s)
{
    const int grid = rows_grid(S, G, 1 << 20);
    AMG_SWITCH_G(G, (k_restrict_rt<kG><<<grid, kBlock, 0, s>>>(S, nf, ci, wv, rcf, v1, kd, rt, rc, flag)));
    AMG_HIP(hipGetLastError());
}

void launch_dense_gemv(int n, const double *a, const double *x, double *y, hipStream_t s)
{
    k_dense_gemv<<<grid_for((int64_t)n * kWave), kBlock, 0, s>>>(n, a, x, y);
    AMG_HIP(hipGetLastError());
}

DotRef launch_fcg_update(int n, DotRef pq, DotRef pr, double *x, double *r, const double *p, const double *q,
                         DotBuf buf, int *flag, hipStream_t s)
{
    const int grid = grid_for(n, kMaxDotBlocks);
    k_fcg_update<<<grid, kBlock, 0, s>>>(n, pq, pr, x, r, p, q, buf.part, flag);
    AMG_HIP(hipGetLastError());
    reduce_if_large(1, buf.part, grid, buf.final_out, s);
    return finished(buf.part, grid, buf.final_out, 0);
}

void launch_fcg_direction(int n, DotRef pq, DotRef zq, const double *z, double *p, int *flag, hipStream_t s)
{
    k_fcg_direction<<<grid_for(n, 4096), kBlock, 0, s>>>(n, pq, zq, z, p, flag);
    AMG_HIP(hipGetLastError());
}

DotRef launch_dot(int n, const double *a, const double *b, DotBuf buf, hipStream_t s)
{
    const int grid = grid_for(n, kMaxDotBlocks);
    k_dot<<<grid, kBlock, 0, s>>>(n, a, b, buf.part);
    AMG_HIP(hipGetLastError());
    reduce_if_large(1, buf.part, grid, buf.final_out, s);
    return finished(buf.part, grid, buf.final_out, 0);
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

void launch_entry_coarse_column(int nnz, const int *ci, const int *agg_pos, int *cagg, hipStream_t s)
{
    k_entry_coarse_column<<<grid_for(nnz, 8192), kBlock, 0, s>>>(nnz, ci, agg_pos, cagg);
    AMG_HIP(hipGetLastError());
}

void launch_restriction_weights(int n, const int *rp, const int *ci, const double *va, const double *minv, double *wv,
                                hipStream_t s)
{
    if (n < kSmallLevel) k_restriction_weights<kWave><<<grid_for((int64_t)n * kWave), kBlock, 0, s>>>(n, rp, ci, va, minv, wv);
    else k_restriction_weights<8><<<grid_for((int64_t)n * 8), kBlock, 0, s>>>(n, rp, ci, va, minv, wv);
    AMG_HIP(hipGetLastError());
}

}  // namespace amg

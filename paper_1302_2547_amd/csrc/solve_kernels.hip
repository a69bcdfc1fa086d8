// solve_kernels.hip -- gfx950 kernels of the solve phase (Sec. 4).
//
// Coarse matrices are CSR in the nested aggregate order of their level, so the
// aggregate of coarse unknown Q is the contiguous range seg_ptr[Q] .. seg_ptr[Q+1]
// of fine rows, and its rows' entries form the contiguous "super-row" srp[Q] ..
// srp[Q+1] of P^T A.  The finest level keeps the caller's numbering for A; its
// super-rows are a separate copy of the entries grouped by aggregate.
//
// Row mapping.  A group of G lanes (G | 64) serves one ordinary row, G chosen per
// level from the mean row length (or timed, on large levels) so the column/value
// streams stay coalesced.
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
#include "wave_ops.h"

#include <algorithm>

namespace amg {
namespace {

inline int grid_for(int64_t threads, int cap = 1 << 20)
{
    int64_t b = (threads + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// Batched launches: right-hand side c = blockIdx.y; a level's vectors (n rows)
// are stored column after column, and every dot site keeps one kDotCol block per
// column.  Unbatched launches have gridDim.y = 1 and change nothing.
template <class P>
__device__ inline P *colv(P *v, int ld)
{
    return v ? v + (size_t)blockIdx.y * (size_t)ld : v;
}
__device__ inline double *colp(double *part)
{
    return part ? part + (size_t)blockIdx.y * kDotCol : part;
}

// K-cycle threshold (Sec. 4.3): a kernel of a second inner step that the
// threshold test skipped for this right-hand side (gate[column] == 0) returns at
// once.  The whole grid of a column takes the same branch.  gate NULL: always runs.
__device__ inline bool gated_off(const int *gate)
{
    return gate && gate[blockIdx.y] == 0;
}
// The latency-bound small-level kernels take the check as a template switch: without
// it their first loads issue at once (a runtime test of a null gate before them
// measurably delays every launch).
template <bool GATE>
__device__ inline bool gated_off_if(const int *gate)
{
    return GATE && gate[blockIdx.y] == 0;
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
// PREFETCH = true (small, latency-bound levels): the block shares the loads --
// the first kBlock * 4 partials of every product are loaded in one unrolled step
// with clamped indices, so they are all in flight together (and with any row
// loads issued before), then summed through LDS; the barrier waits for LDS
// traffic only.  PREFETCH = false (large levels, whose partial sets are normally
// reduced already) keeps a plain per-wavefront loop and few registers.
template <int N, bool PREFETCH = true>
__device__ inline void dot_values(const DotRef *refs, double (&out)[N])
{
    const size_t col = (size_t)blockIdx.y * kDotCol;  // this right-hand side's dot block
    bool all_final = true;
#pragma unroll
    for (int d = 0; d < N; d++) all_final = all_final && refs[d].count == 1;
    if (all_final) {  // one load each, no reduction
#pragma unroll
        for (int d = 0; d < N; d++) out[d] = refs[d].part[col];
        return;
    }
    if (!PREFETCH) {
        const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
        for (int d = 0; d < N; d++) {
            double t = 0.0;
            for (int b = lane; b < refs[d].count; b += kWave) t += refs[d].part[col + b];
            out[d] = wave_sum(t);
        }
        return;
    }
    const int t = threadIdx.x;
    double v[N][4];
#pragma unroll
    for (int d = 0; d < N; d++) {
        const int last = refs[d].count - 1;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int b = t + u * kBlock;
            v[d][u] = refs[d].part[col + (b < last ? b : last)];
        }
    }
#pragma unroll
    for (int d = 0; d < N; d++) {
        const int count = refs[d].count;
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < 4; u++) a += t + u * kBlock < count ? v[d][u] : 0.0;
        for (int b = t + 4 * kBlock; b < count; b += kBlock) a += refs[d].part[col + b];  // beyond kBlock * 4
        out[d] = a;
    }
    block_sums<N>(out);
}

__device__ inline double dot_value(DotRef r)
{
    double v[1];
    dot_values<1, false>(&r, v);
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

// Consecutive blocks are dispatched to the 8 XCDs in turn, each with its own L2.
// Renumbering blocks so that XCD x serves the x-th eighth of the rows keeps the
// gathers of neighbouring rows in one L2 (a bijection on the first multiple of 8
// blocks, identity on the rest).
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int nb)
{
    const int full = nb - nb % kXcds;
    return b < full ? (b % kXcds) * (full / kXcds) + b / kXcds : b;
}

// Completes chunk c of a hub row after the block has summed it (s in every
// thread): a row of one chunk is finished at once; otherwise the chunk sum is
// published and the last chunk of the row to arrive adds all of them (its first
// wavefront loads them together) and finishes the row.  done(row, sum, k) runs
// in one thread.
template <class Done>
__device__ inline void finish_chunk(const Rows &R, int c, const Chunk &ch, double s, Done done, int col = -1)
{
    if (threadIdx.x >= kWave) return;
    const int lane = threadIdx.x;
    const int first = R.long_first[ch.k], m = R.long_first[ch.k + 1] - first;
    if (m == 1) {
        if (lane == 0) done(ch.row, s, ch.k);
        return;
    }
    // The chunk sums are written and read only with device-coherent atomic
    // accesses, so ordering the sum before the arrival count needs no cache
    // write-back: the store's completion is awaited (vector memory counter) before
    // the count is raised, and the last arrival reads the sums only after its
    // count returned.  Nothing else is read afterwards, so no acquire either.
    // every right-hand side of a batched launch (blockIdx.y, or col) has its own sums and counters
    if (col < 0) col = blockIdx.y;
    double *chunk_sum = R.chunk_sum + (size_t)col * R.nchunks;
    unsigned *arrive = R.arrive + (size_t)col * R.nlong;
    unsigned prev = 0;
    if (lane == 0) {
        __hip_atomic_store(&chunk_sum[c], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        prev = __hip_atomic_fetch_add(&arrive[ch.k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = __shfl(prev, 0, kWave);
    if (prev != (unsigned)(m - 1)) return;  // not the last chunk of this row
    double t = 0.0;
    for (int j = lane; j < m; j += kWave)
        t += __hip_atomic_load(&chunk_sum[first + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t = wave_sum(t);
    if (lane == 0) {
        __hip_atomic_store(&arrive[ch.k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        done(ch.row, t, ch.k);
    }
}

// Visits every row of R once.  The callbacks are ordered for latency:
//   pre(row)            loads that depend only on the row index (issued together
//                       with the row-pointer loads);
//   prologue()          once per thread, after the first row's loads are in flight
//                       (typically the reduction of inner-product partials);
//   late(pv)            loads that need the prologue's results;
//   term(p)             contribution of entry p;
//   fin(row, s, k, lv)  the row's reduced sum; k = -1 for an ordinary row, else
//                       the index of the hub row (0 .. nlong).
// Hub-row chunks take all of their entries in one unrolled step (clamped
// indices, no branches), so every load of a chunk is in flight at once.
//
// LAT = false (large, bandwidth-bound levels) keeps the registers few instead: the
// prologue runs first, entries are taken in a plain loop, and pre / late run at
// the end of each row.
template <int G, bool LAT, class Prologue, class Pre, class Late, class Term, class Fin>
__device__ inline void visit_rows(const Rows &R, Prologue prologue, Pre pre, Late late, Term term, Fin fin)
{
    const int nlb = R.nchunks < kLongBlocks ? R.nchunks : kLongBlocks;
    if (!LAT) {
        prologue();
        if ((int)blockIdx.x < nlb) {
            for (int c = blockIdx.x; c < R.nchunks; c += nlb) {
                const Chunk ch = R.chunks[c];
                double s = 0.0;
                for (int p = ch.beg + (int)threadIdx.x; p < ch.end; p += kBlock) s += term(p);
                s = block_sum(s);
                finish_chunk(R, c, ch, s, [&](int row, double t, int k) { fin(row, t, k, late(pre(row))); });
            }
            return;
        }
        const int sub = threadIdx.x % G;
        const int nrb = gridDim.x - nlb;
        const int ngroups = nrb * (kBlock / G);
        const int rb = xcd_block(blockIdx.x - nlb, nrb);
        for (int row = (rb * kBlock + threadIdx.x) / G; row < R.n; row += ngroups) {
            const int b = R.ptr[row], e = R.ptr[row + 1];
            if (e - b > R.lim) continue;  // hub row: served by the chunk blocks (uniform within the group)
            double s = 0.0;
            for (int p = b + sub; p < e; p += G) s += term(p);
            s = group_sum<G>(s);
            if (sub == 0) fin(row, s, -1, late(pre(row)));
        }
        return;
    }
    if ((int)blockIdx.x < nlb) {
        int c = blockIdx.x;
        Chunk ch = R.chunks[c];
        auto pv = pre(ch.row);
        prologue();
        for (;;) {
            const auto lv = late(pv);
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < kChunk / kBlock; u++) {
                const int p = ch.beg + (int)threadIdx.x + u * kBlock;
                const double t = term(p < ch.end ? p : ch.end - 1);
                s += p < ch.end ? t : 0.0;
            }
            s = block_sum(s);
            finish_chunk(R, c, ch, s, [&](int row, double t, int k) { fin(row, t, k, lv); });
            c += nlb;
            if (c >= R.nchunks) break;
            ch = R.chunks[c];
            pv = pre(ch.row);
        }
        return;
    }
    const int sub = threadIdx.x % G;
    const int ngroups = (gridDim.x - nlb) * (kBlock / G);
    int row = ((blockIdx.x - nlb) * kBlock + threadIdx.x) / G;
    int b = 0, e = 0;
    if (row < R.n) {
        b = R.ptr[row];
        e = R.ptr[row + 1];
    }
    auto pv = pre(row < R.n ? row : R.n - 1);
    prologue();
    while (row < R.n) {
        if (e - b <= R.lim) {  // hub rows are served by the chunk blocks (uniform within the group)
            const auto lv = late(pv);
            double s = 0.0;
            if (b < e) {  // first step without a branch: most rows fit in G lanes
                const int p = b + sub;
                const double t = term(p < e ? p : e - 1);
                s = p < e ? t : 0.0;
                for (int q = p + G; q < e; q += G) s += term(q);
            }
            s = group_sum<G>(s);
            if (sub == 0) fin(row, s, -1, lv);
        }
        row += ngroups;
        if (row < R.n) {
            b = R.ptr[row];
            e = R.ptr[row + 1];
            pv = pre(row);
        }
    }
}

// Callbacks for rows that need nothing before or after their sum.
struct NoRow {};
#define AMG_NO_PRE [&](int) { return NoRow{}; }
#define AMG_NO_PROLOGUE [&]() {}
#define AMG_SAME [&](const auto &v) { return v; }

// ------------------------------------------------------------------ SpMV family

template <int G, bool LAT>
__global__ void __launch_bounds__(kBlock) k_spmv(Rows R, const int *__restrict__ ci, const double *__restrict__ va,
                                                 const double *__restrict__ x, double *__restrict__ y)
{
    visit_rows<G, LAT>(
        R, AMG_NO_PROLOGUE, AMG_NO_PRE, AMG_SAME, [&](int p) { return va[p] * x[ci[p]]; },
        [&](int row, double s, int, const NoRow &) { y[row] = s; });
}

// y = A x (y may be NULL); dots (x, Ax) and, for each non-NULL w_j, (x, w_j);
// OMY adds (om, A x) as the last product.
template <class T, int G, int ND, bool LAT, bool OMY, bool GATE>
__global__ void __launch_bounds__(kBlock) k_spmv_dots(Rows R, const int *__restrict__ ci,
                                                      const T *__restrict__ va, const T *__restrict__ x,
                                                      T *__restrict__ y, const T *__restrict__ w1,
                                                      const T *__restrict__ w2, const double *__restrict__ om,
                                                      double *__restrict__ part, const int *__restrict__ gate)
{
    if (gated_off_if<GATE>(gate)) return;
    constexpr int NT = ND + (OMY ? 1 : 0);
    x = colv(x, R.n);
    y = colv(y, R.n);
    w1 = colv(w1, R.n);
    w2 = colv(w2, R.n);
    part = colp(part);
    double d[NT] = {};
    const int nb = gridDim.x;
    struct Pre {
        double xr, w1r, w2r, omr;
    };
    visit_rows<G, LAT>(
        R, AMG_NO_PROLOGUE,
        [&](int row) {
            Pre v{(double)x[row], 0.0, 0.0, 0.0};
            if (ND > 1) v.w1r = (double)w1[row];
            if (ND > 2) v.w2r = (double)w2[row];
            if (OMY) v.omr = om[row];
            return v;
        },
        AMG_SAME, [&](int p) { return (double)va[p] * (double)x[ci[p]]; },
        [&](int row, double s, int k, const Pre &v) {
            if (y) y[row] = (T)s;
            double t[NT];
            t[0] = v.xr * s;
            if (ND > 1) t[1 % NT] = v.xr * v.w1r;
            if (ND > 2) t[2 % NT] = v.xr * v.w2r;
            if (OMY) t[NT - 1] = v.omr * s;
            if (k < 0) {
#pragma unroll
                for (int j = 0; j < NT; j++) d[j] += t[j];
            } else {
#pragma unroll
                for (int j = 0; j < NT; j++) part[j * kPartStride + nb + k] = t[j];
            }
        });
    store_partials<NT>(d, part);
}

// r = b - A x; partials of (b, b) and (r, r)
template <int G>
__global__ void __launch_bounds__(kBlock) k_residual(Rows R, const int *__restrict__ ci,
                                                     const double *__restrict__ va, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ part, const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    b = colv(b, R.n);
    x = colv(x, R.n);
    r = colv(r, R.n);
    part = colp(part);
    double d[2] = {0.0, 0.0};
    const int nb = gridDim.x;
    visit_rows<G, false>(
        R, AMG_NO_PROLOGUE, [&](int row) { return b[row]; }, AMG_SAME, [&](int p) { return va[p] * x[ci[p]]; },
        [&](int row, double s, int k, double br) {
            const double rr = br - s;
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
                                                                    int count, double *__restrict__ out,
                                                                    int out_stride, const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    part += (size_t)blockIdx.y * kDotCol;
    out += (size_t)blockIdx.y * out_stride;
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
// OM adds partials of (om, rc) (the restriction to a single coarse unknown of
// the next level down, see k_post_direct).
template <class T, int G, bool LAT, bool OM, bool GATE>
__global__ void __launch_bounds__(kBlock) k_restrict(Rows S, int nf, const int *__restrict__ ci,
                                                     const T *__restrict__ wv, const T *__restrict__ r,
                                                     T *__restrict__ rc, const double *__restrict__ om,
                                                     double *__restrict__ part, const int *__restrict__ gate)
{
    if (gated_off_if<GATE>(gate)) return;
    r = colv(r, nf);
    rc = colv(rc, S.n);
    part = colp(part);
    double d[1] = {0.0};
    const int nb = gridDim.x;
    visit_rows<G, LAT>(
        S, AMG_NO_PROLOGUE, [&](int Q) { return OM ? om[Q] : 0.0; }, AMG_SAME,
        [&](int p) { return (double)wv[p] * (double)r[ci[p]]; },
        [&](int Q, double s, int k, double w) {
            rc[Q] = (T)s;
            if (OM) {
                if (k < 0) d[0] += w * s;
                else part[nb + k] = w * s;
            }
        });
    if (OM) store_partials<1>(d, part);
}

// K-cycle coefficients.  rho1 = (c1, A c1), alpha1 = (c1, rc), beta = (c2, A c2),
// gamma = (c2, A c1), alpha2 = (c2, rt): two flexible-CG steps from zero give
// e = (alpha1/rho1 - (gamma/rho1)(alpha2/rho2)) c1 + (alpha2/rho2) c2,
// rho2 = beta - gamma^2/rho1.  A non-positive rho means A is not SPD: the flag is
// raised and the correction dropped.
struct KCoef {
    double a1, a2;
    bool bad;
    bool two;  // the second step's direction c2 enters the correction (it was not skipped)
};

// second (may be NULL): the gate of the second inner step; where it is 0 for this
// right-hand side the threshold test skipped that step and mode 2 reads as mode 1.
template <bool PREFETCH = true, bool SECOND = true>
__device__ inline KCoef kcycle_coefficients(int mode, const KDots &kd, const int *second = nullptr)
{
    KCoef c{0.0, 0.0, false, mode == 2};
    if (mode == 0 || mode == 3) return c;
    if (SECOND && mode == 2 && second && second[blockIdx.y] == 0) {
        mode = 1;  // c2 was never formed for this column: it must not be read
        c.two = false;
    }
    double rho1, alpha1, beta = 0.0, gamma = 0.0, alpha2 = 0.0;
    if (mode == 2) {
        const DotRef refs[5] = {kd.rho1, kd.alpha1, kd.beta, kd.gamma, kd.alpha2};
        double v[5];
        dot_values<5, PREFETCH>(refs, v);
        rho1 = v[0];
        alpha1 = v[1];
        beta = v[2];
        gamma = v[3];
        alpha2 = v[4];
    } else {
        const DotRef refs[2] = {kd.rho1, kd.alpha1};
        double v[2];
        dot_values<2, PREFETCH>(refs, v);
        rho1 = v[0];
        alpha1 = v[1];
    }
    // A zero coarse residual (rc = 0: a converged or empty right-hand side of a
    // batch) gives c1 = 0, rho1 = alpha1 = 0 and a zero correction, not a breakdown;
    // likewise rt = 0 in the second step.
    if (!(rho1 > 0.0)) {
        c.bad = !(rho1 == 0.0 && alpha1 == 0.0);
        return c;
    }
    const double q1 = alpha1 / rho1;
    c.a1 = q1;
    if (mode == 1) return c;
    const double g1 = gamma / rho1;
    const double rho2 = beta - gamma * g1;
    if (!(rho2 > 0.0)) {
        if (beta == 0.0 && alpha2 == 0.0) return c;  // c2 = 0: only the first step counts
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
template <class T, int G, bool OM, bool GATE>
__global__ void __launch_bounds__(kBlock) k_restrict_rt(Rows S, int nf, const int *__restrict__ ci,
                                                        const T *__restrict__ wv,
                                                        const T *__restrict__ rcf,
                                                        const T *__restrict__ v1, KDots kd,
                                                        T *__restrict__ rt, T *__restrict__ rc,
                                                        int *__restrict__ flag, const double *__restrict__ om,
                                                        double *__restrict__ part, const int *__restrict__ gate)
{
    if (gated_off_if<GATE>(gate)) return;
    rcf = colv(rcf, nf);
    v1 = colv(v1, nf);
    rt = colv(rt, nf);
    rc = colv(rc, S.n);
    part = colp(part);
    double d[1] = {0.0};
    const int nb = gridDim.x;
    const int gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    double rq = 0.0, vq = 0.0;  // this thread's first element of rt, loaded before the coefficients
    if (gt < nf) {
        rq = (double)rcf[gt];
        vq = (double)v1[gt];
    }
    double a = 0.0;
    visit_rows<G, true>(
        S,
        [&]() {
            const KCoef c = kcycle_coefficients(1, kd);
            if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
            a = c.a1;
            if (gt < nf) rt[gt] = (T)(rq - a * vq);
            for (int q = gt + gs; q < nf; q += gs) rt[q] = (T)((double)rcf[q] - a * (double)v1[q]);
        },
        [&](int Q) { return OM ? om[Q] : 0.0; }, AMG_SAME,
        [&](int p) {
            const int t = ci[p];
            return (double)wv[p] * ((double)rcf[t] - a * (double)v1[t]);
        },
        [&](int Q, double s, int k, double w) {
            rc[Q] = (T)s;
            if (OM) {
                if (k < 0) d[0] += w * s;
                else part[nb + k] = w * s;
            }
        });
    if (OM) store_partials<1>(d, part);
}

// rt = rc - (alpha1/rho1) v1
template <class T>
__global__ void __launch_bounds__(kBlock) k_inner_residual(int n, const T *__restrict__ rc,
                                                           const T *__restrict__ v1, KDots kd,
                                                           T *__restrict__ rt, int *__restrict__ flag,
                                                           const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    rc = colv(rc, n);
    v1 = colv(v1, n);
    rt = colv(rt, n);
    const KCoef c = kcycle_coefficients<false>(1, kd);  // large levels only
    if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        rt[i] = (T)((double)rc[i] - c.a1 * (double)v1[i]);
}

// The same with the threshold test's inputs: partials of (rc, rc), (rt, rt) and,
// with om, (om, rt) (the restriction of rt when the next level down is a single
// unknown).  Runs under the gate of the enclosing step.
template <class T, bool OM>
__global__ void __launch_bounds__(kBlock) k_inner_residual_theta(int n, const T *__restrict__ rc,
                                                                 const T *__restrict__ v1, KDots kd,
                                                                 T *__restrict__ rt, int *__restrict__ flag,
                                                                 const double *__restrict__ om,
                                                                 double *__restrict__ part,
                                                                 const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    rc = colv(rc, n);
    v1 = colv(v1, n);
    rt = colv(rt, n);
    part = colp(part);
    const KCoef c = kcycle_coefficients<true>(1, kd);
    if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    constexpr int ND = OM ? 3 : 2;
    double d[ND] = {};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double g = (double)rc[i];
        const T t = (T)(g - c.a1 * (double)v1[i]);
        rt[i] = t;
        d[0] += g * g;
        d[1] += (double)t * (double)t;
        if (OM) d[2 % ND] += om[i] * (double)t;
    }
    store_partials<ND>(d, part);
}

// Threshold test of one inner flexible-CG step (Sec. 4.3): the second step runs
// for a right-hand side only if the enclosing step runs and ||rt|| >= theta ||rc||
// (compared as squares, as the oracle does).  One block per right-hand side.
__global__ void __launch_bounds__(kBlock) k_theta_gate(DotRef rcrc, DotRef rtrt, double theta2,
                                                       const int *__restrict__ parent, int *__restrict__ gate)
{
    const bool run = !(parent && parent[blockIdx.y] == 0);
    double v[2] = {0.0, 0.0};
    if (run) {
        const DotRef refs[2] = {rcrc, rtrt};
        dot_values<2>(refs, v);
    }
    if (threadIdx.x == 0) gate[blockIdx.y] = run && !(v[1] < theta2 * v[0]) ? 1 : 0;
}

// Prolongation + post-smoothing: x = M^-1 r + P e (the pre-smoothed iterate plus
// the coarse correction) is formed on the fly for every column (cagg[p], when
// given, is the coarse unknown of column ci[p] stored per entry: on small,
// latency-bound levels it saves a dependent gather), then
// out = x + M^-1 (r - A x).  mode 0: e = edirect; mode 1: e = a1 c1;
// mode 2: e = a1 c1 + a2 c2; mode 3: e = ainv edirect (small dense coarsest level).
// DOT adds partials of (out, wdot).
template <class T, int G, int MODE, bool DOT, bool CAGG, bool GATE>
__global__ void __launch_bounds__(kBlock) k_post_smooth(Rows R, const int *__restrict__ ci,
                                                        const T *__restrict__ va,
                                                        const T *__restrict__ minv,
                                                        const T *__restrict__ r,
                                                        const int *__restrict__ agg_pos,
                                                        const int *__restrict__ cagg,
                                                        const T *__restrict__ edirect,
                                                        const T *__restrict__ c1,
                                                        const T *__restrict__ c2, KDots kd,
                                                        T *__restrict__ xout, const T *__restrict__ wdot,
                                                        double *__restrict__ part, int *__restrict__ flag,
                                                        const double *__restrict__ ainv, int nc,
                                                        const int *__restrict__ gate, const int *__restrict__ second)
{
    if (GATE && gated_off(gate)) return;
    r = colv(r, R.n);
    xout = colv(xout, R.n);
    wdot = colv(wdot, R.n);
    edirect = colv(edirect, nc);
    c1 = colv(c1, nc);
    c2 = colv(c2, nc);
    part = colp(part);
    double a1 = 0.0, a2 = 0.0;
    bool two = MODE == 2;  // a constant unless GATE
    __shared__ double e_sh[MODE == 3 ? kInlineCoarse : 1];
    // rounded step by step, so that the gated and the ungated kernel give the same
    // bits; both loads issue unconditionally (a skipped second step's c2 is not used)
    auto corr = [&](int J) -> double {
        if (MODE == 0) return (double)edirect[J];
        if (MODE == 3) return e_sh[J];
        if (MODE == 1) return __dmul_rn(a1, (double)c1[J]);
        const double v1 = (double)c1[J], v2 = (double)c2[J];
        return two ? __fma_rn(a1, v1, __dmul_rn(a2, v2)) : __dmul_rn(a1, v1);
    };
    struct Pre {
        double mr, rr, wd;
        int J;
    };
    struct Late {
        double mr, rr, wd, cj;
    };
    double dsum[1] = {0.0};
    const int nb = gridDim.x;
    visit_rows<G, CAGG>(
        R,
        [&]() {
            const KCoef c = kcycle_coefficients<CAGG, GATE>(MODE, kd, second);  // CAGG marks small levels
            if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
            a1 = c.a1;
            a2 = c.a2;
            if (GATE) two = c.two;
            if (MODE == 3) {  // e = A_coarsest^-1 rc, computed by every block into LDS
                // wavefront w forms rows w, w + 4, ...; lane j holds column j
                constexpr int kRows = kInlineCoarse / (kBlock / kWave);
                const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
                const double ej = lane < nc ? (double)edirect[lane] : 0.0;
                double aij[kRows];
#pragma unroll
                for (int u = 0; u < kRows; u++) {
                    const int i = w + u * (kBlock / kWave);
                    aij[u] = (i < nc && lane < nc) ? ainv[i * nc + lane] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kRows; u++) {
                    const int i = w + u * (kBlock / kWave);
                    if (i < nc) {  // uniform over the wavefront
                        const double t = wave_sum(aij[u] * ej);
                        if (lane == 0) e_sh[i] = t;
                    }
                }
                __syncthreads();
            }
        },
        [&](int row) { return Pre{(double)minv[row], (double)r[row], DOT ? (double)wdot[row] : 0.0, agg_pos[row]}; },
        [&](const Pre &v) { return Late{v.mr, v.rr, v.wd, corr(v.J)}; },
        [&](int p) {
            const int t = ci[p];
            return (double)va[p] * ((double)minv[t] * (double)r[t] + corr(CAGG ? cagg[p] : agg_pos[t]));
        },
        [&](int row, double s, int k, const Late &v) {
            const double x = v.mr * v.rr + v.cj;
            const double o = x + v.mr * (v.rr - s);
            xout[row] = (T)o;
            if (DOT) {
                if (k < 0) dsum[0] += o * v.wd;
                else part[nb + k] = o * v.wd;
            }
        });
    if (DOT) store_partials<1>(dsum, part);
}

// The prolonged iterate x = M^-1 r + (P e) of one row and its coarse value e, as the
// two-launch and the one-sweep post-smoothing of large levels form it: rounded step
// by step (explicit fused multiply-adds, no contraction left to the compiler), so
// both forms produce the same bits.
template <int MODE, class T>
__device__ inline double coarse_value(const KCoef &c, const T *edirect, const T *c1, const T *c2, int J)
{
    if (MODE == 0) return (double)edirect[J];
    if (MODE == 1) return __dmul_rn(c.a1, (double)c1[J]);
    const double v1 = (double)c1[J], v2 = (double)c2[J];
    return c.two ? __fma_rn(c.a1, v1, __dmul_rn(c.a2, v2)) : __dmul_rn(c.a1, v1);
}
__device__ inline double prolonged_iterate(double minv, double r, double e) { return __fma_rn(minv, r, e); }
__device__ inline double smoothed(double x, double minv, double r, double ax) { return __fma_rn(minv, __dsub_rn(r, ax), x); }

// Large levels split the same step in two launches, so that each entry gathers one
// value instead of five (the fused form recomputes x_t = M^-1 r_t + (P e)_t for every
// entry that references column t, which at 128^3 and above is bound by the gathers):
//   k_smooth_start:  x = M^-1 r + P e, one row per thread, stored in FP64;
//   k_smooth_finish: out = x + M^-1 (r - A x), with the partials of (out, wdot).
template <class T, int MODE>
__global__ void __launch_bounds__(kBlock) k_smooth_start(int n, const T *__restrict__ minv,
                                                         const T *__restrict__ r,
                                                         const int *__restrict__ agg_pos,
                                                         const T *__restrict__ edirect,
                                                         const T *__restrict__ c1,
                                                         const T *__restrict__ c2, KDots kd,
                                                         double *__restrict__ x, int *__restrict__ flag, int nc,
                                                         const int *__restrict__ gate,
                                                         const int *__restrict__ second)
{
    if (gated_off(gate)) return;
    r = colv(r, n);
    x = colv(x, n);
    edirect = colv(edirect, nc);
    c1 = colv(c1, nc);
    c2 = colv(c2, nc);
    const KCoef c = kcycle_coefficients<false>(MODE, kd, second);
    if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double e = coarse_value<MODE>(c, edirect, c1, c2, agg_pos[i]);
        x[i] = prolonged_iterate((double)minv[i], (double)r[i], e);
    }
}

template <class T, int G, bool DOT>
__global__ void __launch_bounds__(kBlock) k_smooth_finish(Rows R, const int *__restrict__ ci,
                                                          const T *__restrict__ va,
                                                          const T *__restrict__ minv,
                                                          const T *__restrict__ r,
                                                          const double *__restrict__ x, T *__restrict__ xout,
                                                          const T *__restrict__ wdot, double *__restrict__ part,
                                                          const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    r = colv(r, R.n);
    x = colv(x, R.n);
    xout = colv(xout, R.n);
    wdot = colv(wdot, R.n);
    part = colp(part);
    struct Pre {
        double mr, rr, xr, wd;
    };
    double dsum[1] = {0.0};
    const int nb = gridDim.x;
    visit_rows<G, false>(
        R, AMG_NO_PROLOGUE,
        [&](int row) { return Pre{(double)minv[row], (double)r[row], x[row], DOT ? (double)wdot[row] : 0.0}; },
        AMG_SAME, [&](int p) { return (double)va[p] * x[ci[p]]; },
        [&](int row, double s, int k, const Pre &v) {
            const double o = v.xr + v.mr * (v.rr - s);
            xout[row] = (T)o;
            if (DOT) {
                if (k < 0) dsum[0] += o * v.wd;
                else part[nb + k] = o * v.wd;
            }
        });
    if (DOT) store_partials<1>(dsum, part);
}


// ------------------------------------------------------------------ batched sweeps (SpMM)
// On large levels a batch of right-hand sides is served CB columns per block
// (blockIdx.y = column group): each entry's column index and value are loaded once
// and applied to every column of the group, so the matrix is read ceil(ncol / CB)
// times instead of ncol times (column-major vectors, leading dimension = the level's
// size).  Rows, lanes (G per row, lane-strided entries, group_sum) and blocks are
// those of the one-column kernels, so every column's sums and partials are formed in
// the same order and the results are the same bits.  Columns past ncol in the last
// group repeat the first column of the group and are discarded.
template <int CB>
__device__ inline int mm_columns(int ncol, int *c0)
{
    *c0 = blockIdx.y * CB;
    const int left = ncol - *c0;
    return left < CB ? left : CB;
}
// which of the block's columns run (inside the batch and not gated off); a block
// with none returns at once
template <int CB>
__device__ inline bool mm_live(int nc, int c0, const int *gate, bool (&live)[CB])
{
    bool any = false;
#pragma unroll
    for (int k = 0; k < CB; k++) {
        live[k] = k < nc && !(gate && gate[c0 + k] == 0);
        any = any || live[k];
    }
    return any;
}

// The row loop of visit_rows (large levels) for CB columns: acc(p, s) adds entry
// p's contribution to the CB sums s; fin(row, s, k) finishes the row for every
// column (k: hub row index, -1 for an ordinary row), called by one lane.
template <int G, int CB, class Acc, class Fin>
__device__ inline void visit_rows_mm(const Rows &R, Acc acc, Fin fin)
{
    const int nlb = R.nchunks < kLongBlocks ? R.nchunks : kLongBlocks;
    if ((int)blockIdx.x < nlb) {
        for (int c = blockIdx.x; c < R.nchunks; c += nlb) {
            const Chunk ch = R.chunks[c];
            double s[CB] = {};
            for (int p = ch.beg + (int)threadIdx.x; p < ch.end; p += kBlock) acc(p, s);
            block_sums<CB>(s);
            fin(c, ch, s);
        }
        return;
    }
    const int sub = threadIdx.x % G;
    const int nrb = gridDim.x - nlb;
    const int ngroups = nrb * (kBlock / G);
    const int rb = xcd_block(blockIdx.x - nlb, nrb);
    for (int row = (rb * kBlock + threadIdx.x) / G; row < R.n; row += ngroups) {
        const int b = R.ptr[row], e = R.ptr[row + 1];
        if (e - b > R.lim) continue;  // hub row: served by the chunk blocks
        double s[CB] = {};
        for (int p = b + sub; p < e; p += G) acc(p, s);
#pragma unroll
        for (int k = 0; k < CB; k++) s[k] = group_sum<G>(s[k]);
        if (sub == 0) fin(row, Chunk{-1, 0, 0, -1}, s);
    }
}

// k_spmv_dots for CB columns: y = A x and the partials of (x, A x), (x, w1), (x, w2)
template <class T, int G, int ND, int CB>
__global__ void __launch_bounds__(kBlock) k_spmm_dots(Rows R, const int *__restrict__ ci,
                                                      const T *__restrict__ va, const T *__restrict__ x,
                                                      T *__restrict__ y, const T *__restrict__ w1,
                                                      const T *__restrict__ w2, double *__restrict__ part, int ncol,
                                                      const int *__restrict__ gate)
{
    int c0;
    const int nc = mm_columns<CB>(ncol, &c0);
    bool live[CB];
    if (!mm_live<CB>(nc, c0, gate, live)) return;
    const size_t n = (size_t)R.n;
    const int nb = gridDim.x;
    auto col = [&](int k) { return (size_t)(c0 + (k < nc ? k : 0)); };
    double d[CB][ND] = {};
    auto row_done = [&](int row, int k, double s, int hub) {
        const size_t o = col(k) * n + row;
        if (y) y[o] = (T)s;
        const double xr = (double)x[o];
        double t[ND];
        t[0] = xr * s;
        if (ND > 1) t[1 % ND] = xr * (double)w1[o];
        if (ND > 2) t[2 % ND] = xr * (double)w2[o];
        if (hub < 0) {
#pragma unroll
            for (int j = 0; j < ND; j++) d[k][j] += t[j];
        } else {
            double *pc = part + col(k) * kDotCol;
#pragma unroll
            for (int j = 0; j < ND; j++) pc[j * kPartStride + nb + hub] = t[j];
        }
    };
    visit_rows_mm<G, CB>(
        R,
        [&](int p, double (&s)[CB]) {
            const int j = ci[p];
            const double a = (double)va[p];
#pragma unroll
            for (int k = 0; k < CB; k++) s[k] += a * (double)x[col(k) * n + j];
        },
        [&](int row, const Chunk &ch, double (&s)[CB]) {
            if (ch.k < 0) {
#pragma unroll
                for (int k = 0; k < CB; k++)
                    if (live[k]) row_done(row, k, s[k], -1);
                return;
            }
#pragma unroll
            for (int k = 0; k < CB; k++)
                if (live[k]) finish_chunk(R, row, ch, s[k], [&](int r, double t, int hub) { row_done(r, k, t, hub); },
                                          c0 + k);
        });
#pragma unroll
    for (int k = 0; k < CB; k++)
        if (live[k]) store_partials<ND>(d[k], part + col(k) * kDotCol);
}

// k_restrict (large levels) for CB columns: rc = W r over the super-rows
template <class T, int G, int CB>
__global__ void __launch_bounds__(kBlock) k_restrict_mm(Rows S, int nf, const int *__restrict__ ci,
                                                        const T *__restrict__ wv, const T *__restrict__ r,
                                                        T *__restrict__ rc, int ncol, const int *__restrict__ gate)
{
    int c0;
    const int nc = mm_columns<CB>(ncol, &c0);
    bool live[CB];
    if (!mm_live<CB>(nc, c0, gate, live)) return;
    auto col = [&](int k) { return (size_t)(c0 + (k < nc ? k : 0)); };
    visit_rows_mm<G, CB>(
        S,
        [&](int p, double (&s)[CB]) {
            const int j = ci[p];
            const double w = (double)wv[p];
#pragma unroll
            for (int k = 0; k < CB; k++) s[k] += w * (double)r[col(k) * nf + j];
        },
        [&](int Q, const Chunk &ch, double (&s)[CB]) {
#pragma unroll
            for (int k = 0; k < CB; k++) {
                if (!live[k]) continue;
                if (ch.k < 0) rc[col(k) * S.n + Q] = (T)s[k];
                else finish_chunk(S, Q, ch, s[k], [&](int q, double t, int) {
                    rc[col(k) * S.n + q] = (T)t;
                }, c0 + k);
            }
        });
}

// k_smooth_finish for CB columns: out = x + M^-1 (r - A x), partials of (out, wdot)
template <class T, int G, bool DOT, int CB>
__global__ void __launch_bounds__(kBlock) k_smooth_finish_mm(Rows R, const int *__restrict__ ci,
                                                             const T *__restrict__ va, const T *__restrict__ minv,
                                                             const T *__restrict__ r, const double *__restrict__ x,
                                                             T *__restrict__ xout, const T *__restrict__ wdot,
                                                             double *__restrict__ part, int ncol,
                                                             const int *__restrict__ gate)
{
    int c0;
    const int nc = mm_columns<CB>(ncol, &c0);
    bool live[CB];
    if (!mm_live<CB>(nc, c0, gate, live)) return;
    const size_t n = (size_t)R.n;
    const int nb = gridDim.x;
    auto col = [&](int k) { return (size_t)(c0 + (k < nc ? k : 0)); };
    double d[CB][1] = {};
    auto row_done = [&](int row, int k, double s, int hub) {
        const size_t o = col(k) * n + row;
        const double out = x[o] + (double)minv[row] * ((double)r[o] - s);
        xout[o] = (T)out;
        if (DOT) {
            const double t = out * (double)wdot[o];
            if (hub < 0) d[k][0] += t;
            else part[col(k) * kDotCol + nb + hub] = t;
        }
    };
    visit_rows_mm<G, CB>(
        R,
        [&](int p, double (&s)[CB]) {
            const int j = ci[p];
            const double a = (double)va[p];
#pragma unroll
            for (int k = 0; k < CB; k++) s[k] += a * x[col(k) * n + j];
        },
        [&](int row, const Chunk &ch, double (&s)[CB]) {
            if (ch.k < 0) {
#pragma unroll
                for (int k = 0; k < CB; k++)
                    if (live[k]) row_done(row, k, s[k], -1);
                return;
            }
#pragma unroll
            for (int k = 0; k < CB; k++)
                if (live[k]) finish_chunk(R, row, ch, s[k], [&](int q, double t, int hub) { row_done(q, k, t, hub); },
                                          c0 + k);
        });
    if (DOT) {
#pragma unroll
        for (int k = 0; k < CB; k++)
            if (live[k]) store_partials<1>(d[k], part + col(k) * kDotCol);
    }
}

// ------------------------------------------------------------------ sliced ELLPACK sweeps
// One lane per row and one slice per wavefront (tiles of kBlock rows start at
// multiples of kWave), so a slice's width is uniform over the wavefront and the
// entry and value loads of each slot are contiguous.  The first kSellUnroll slots
// are loaded together (slots past the width re-read the first one with weight 0),
// then their gathers; the sum runs in slot order, i.e. in the row's CSR order.
constexpr int kSellUnroll = 8;

// sum over the row's slots of a_ij * gx(j)
template <class V, class GX>
__device__ inline double sell_row(const int *__restrict__ sc, const V *__restrict__ sv, int beg, int w, int t,
                                  GX gx)
{
    const int p0 = beg + t;
    int c[kSellUnroll];
    double v[kSellUnroll];
#pragma unroll
    for (int u = 0; u < kSellUnroll; u++) {
        const int p = u < w ? p0 + u * kWave : p0;
        c[u] = sc[p];
        v[u] = u < w ? (double)sv[p] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kSellUnroll; u++) s = __fma_rn(v[u], gx(c[u]), s);
    for (int k = kSellUnroll; k < w; k++) {
        const int p = p0 + k * kWave;
        s = __fma_rn((double)sv[p], gx(sc[p]), s);
    }
    return s;
}

// Row i of tile u of this block (blocks renumbered so that each XCD serves a
// contiguous range of tiles); calls row_fn(i, slice offset, width, lane) for
// every row < n.
template <class RowFn>
__device__ inline void sell_tiles(int n, int tpb, const int *__restrict__ sptr, RowFn row_fn)
{
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int t = threadIdx.x & (kWave - 1);
    for (int u = 0; u < tpb; u++) {
        const int i = (b * tpb + u) * kBlock + (int)threadIdx.x;
        if (i >= n) break;
        const int s = __builtin_amdgcn_readfirstlane(i / kWave);
        const int beg = sptr[s];
        const int w = (sptr[s + 1] - beg) / kWave;
        row_fn(i, beg, w, t);
    }
}

// k_smooth_finish on the sliced copy: out = x + M^-1 (r - A x), with the partials of
// (out, wdot) when DOT.
template <class T, bool DOT>
__global__ void __launch_bounds__(kBlock) k_sell_smooth_finish(int n, int tpb, const int *__restrict__ sptr,
                                                               const int *__restrict__ sc, const T *__restrict__ sv,
                                                               const T *__restrict__ minv, const T *__restrict__ r,
                                                               const double *__restrict__ x, T *__restrict__ xout,
                                                               const T *__restrict__ wdot, double *__restrict__ part,
                                                               const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    r = colv(r, n);
    x = colv(x, n);
    xout = colv(xout, n);
    wdot = colv(wdot, n);
    part = colp(part);
    double d[1] = {0.0};
    sell_tiles(n, tpb, sptr, [&](int i, int beg, int w, int t) {
        const double mr = (double)minv[i], rr = (double)r[i], xr = x[i];
        const double wd = DOT ? (double)wdot[i] : 0.0;
        const double o = smoothed(xr, mr, rr, sell_row(sc, sv, beg, w, t, [&](int j) { return x[j]; }));
        xout[i] = (T)o;
        if (DOT) d[0] += o * wd;
    });
    if (DOT) store_partials<1>(d, part);
}

// Prolongation + post-smoothing of a sliced level in one sweep: every row forms
// its iterate x_i = M^-1 r_i + (P e)_i, and every entry the iterate of its column
// the same way, so x never goes to memory (three gathers per entry -- minv, r and
// the aggregate position -- and the coarse values, instead of one gather of the
// stored iterate and its write and read-back).  The products and their order are
// those of k_smooth_start + k_sell_smooth_finish, so the result is the same.
template <class T, int MODE, bool DOT>
__global__ void __launch_bounds__(kBlock) k_sell_post_fused(int n, int tpb, const int *__restrict__ sptr,
                                                            const int *__restrict__ sc, const T *__restrict__ sv,
                                                            const T *__restrict__ minv, const T *__restrict__ r,
                                                            const int *__restrict__ agg_pos,
                                                            const T *__restrict__ edirect, const T *__restrict__ c1,
                                                            const T *__restrict__ c2, KDots kd, int nc,
                                                            T *__restrict__ xout, const T *__restrict__ wdot,
                                                            double *__restrict__ part, int *__restrict__ flag,
                                                            const int *__restrict__ gate,
                                                            const int *__restrict__ second)
{
    if (gated_off(gate)) return;
    r = colv(r, n);
    xout = colv(xout, n);
    wdot = colv(wdot, n);
    edirect = colv(edirect, nc);
    c1 = colv(c1, nc);
    c2 = colv(c2, nc);
    part = colp(part);
    const KCoef c = kcycle_coefficients<false>(MODE, kd, second);
    if (c.bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    auto xval = [&](int j) -> double {  // as k_smooth_start forms x_j
        const double e = coarse_value<MODE>(c, edirect, c1, c2, agg_pos[j]);
        return prolonged_iterate((double)minv[j], (double)r[j], e);
    };
    double d[1] = {0.0};
    sell_tiles(n, tpb, sptr, [&](int i, int beg, int w, int t) {
        const double mr = (double)minv[i], rr = (double)r[i];
        const double wd = DOT ? (double)wdot[i] : 0.0;
        const double xi = xval(i);
        const double o = smoothed(xi, mr, rr, sell_row(sc, sv, beg, w, t, xval));
        xout[i] = (T)o;
        if (DOT) d[0] += o * wd;
    });
    if (DOT) store_partials<1>(d, part);
}

// k_spmv_dots on the sliced copy: y = A x (y may be NULL), partials of (x, A x),
// (x, w1) if ND > 1, (x, w2) if ND > 2.
template <class T, int ND>
__global__ void __launch_bounds__(kBlock) k_sell_spmv_dots(int n, int tpb, const int *__restrict__ sptr,
                                                           const int *__restrict__ sc, const T *__restrict__ sv,
                                                           const T *__restrict__ x, T *__restrict__ y,
                                                           const T *__restrict__ w1, const T *__restrict__ w2,
                                                           double *__restrict__ part, const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    x = colv(x, n);
    y = colv(y, n);
    w1 = colv(w1, n);
    w2 = colv(w2, n);
    part = colp(part);
    double d[ND] = {};
    sell_tiles(n, tpb, sptr, [&](int i, int beg, int w, int t) {
        const double xr = (double)x[i];
        const double w1r = ND > 1 ? (double)w1[i] : 0.0, w2r = ND > 2 ? (double)w2[i] : 0.0;
        const double sum = sell_row(sc, sv, beg, w, t, [&](int j) { return (double)x[j]; });
        if (y) y[i] = (T)sum;
        d[0] += xr * sum;
        if (ND > 1) d[1 % ND] += xr * w1r;
        if (ND > 2) d[2 % ND] += xr * w2r;
    });
    store_partials<ND>(d, part);
}

// Restriction on a sliced level in two launches.  The pre-smoothing sweep from
// zero gives M^-1 r, and its residual t = r - A M^-1 r is formed row by row
// (t_i = r_i - sum_j a_ij minv_j r_j, FP64, stored in the level's FP64 scratch);
// then rc = P^T t sums t over the members of each aggregate in their nested order
// (Sec. 4.2: the restriction of piecewise-constant P adds the fine values of an
// aggregate).
template <class T>
__global__ void __launch_bounds__(kBlock) k_sell_presmooth_residual(int n, int tpb, const int *__restrict__ sptr,
                                                                    const int *__restrict__ sc,
                                                                    const T *__restrict__ sv,
                                                                    const T *__restrict__ minv,
                                                                    const T *__restrict__ r, double *__restrict__ t,
                                                                    const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    r = colv(r, n);
    t = colv(t, n);
    sell_tiles(n, tpb, sptr, [&](int i, int beg, int w, int lane) {
        const double ri = (double)r[i];
        const double s = sell_row(sc, sv, beg, w, lane, [&](int j) { return (double)minv[j] * (double)r[j]; });
        t[i] = ri - s;
    });
}

// rc_J = sum of t over positions seg[J] .. seg[J+1] (fine row idx[p], or p when
// idx is NULL) in position order, one thread per aggregate.  The first kSegUnroll
// members' indices are loaded together (clamped to the last member), then their
// values; members past the end add 0.
constexpr int kSegUnroll = 8;

template <class T>
__global__ void __launch_bounds__(kBlock) k_segment_sum(int nc, const int *__restrict__ seg,
                                                        const int *__restrict__ idx, int nf,
                                                        const double *__restrict__ t, T *__restrict__ rc,
                                                        const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    t = colv(t, nf);
    rc = colv(rc, nc);
    for (int J = blockIdx.x * kBlock + threadIdx.x; J < nc; J += gridDim.x * kBlock) {
        const int b = seg[J], e = seg[J + 1];
        double s = 0.0;
        if (e > b) {
            int q[kSegUnroll];
#pragma unroll
            for (int u = 0; u < kSegUnroll; u++) {
                const int p = b + u < e ? b + u : e - 1;
                q[u] = idx ? idx[p] : p;
            }
            double v[kSegUnroll];
#pragma unroll
            for (int u = 0; u < kSegUnroll; u++) v[u] = t[q[u]];
#pragma unroll
            for (int u = 0; u < kSegUnroll; u++) s += b + u < e ? v[u] : 0.0;
            for (int p = b + kSegUnroll; p < e; p++) s += t[idx ? idx[p] : p];
        }
        rc[J] = (T)s;
    }
}

// Post-smoothing on a level whose coarse level is a single unknown.  P is then
// the all-ones column and the restriction W = P^T (I - A M^-1) is the row vector
// om^T, om_j = 1 - minv_j sum_i a_ij, so rc = (om, r) is an inner product whose
// partials the producers of r wrote.  e = rc / a_c, x = M^-1 r + e and
// out = x + M^-1 (r - A x).  RT (the second inner step of the parent):
// r = rcf - (alpha1/rho1) v1 is formed on the fly and stored, and
// rc = (om, rcf) - (alpha1/rho1) (om, v1).
template <class T, int G, bool RT, bool GATE>
__global__ void __launch_bounds__(kBlock) k_post_direct(Rows R, const int *__restrict__ ci,
                                                        const T *__restrict__ va,
                                                        const T *__restrict__ minv,
                                                        const T *__restrict__ r, const T *__restrict__ v1,
                                                        KDots kd, DotRef om_r, DotRef om_v1,
                                                        const double *__restrict__ ainv, T *__restrict__ xout,
                                                        T *__restrict__ rt_out, int *__restrict__ flag,
                                                        const int *__restrict__ gate)
{
    if (gated_off_if<GATE>(gate)) return;
    r = colv(r, R.n);
    v1 = colv(v1, R.n);
    xout = colv(xout, R.n);
    rt_out = colv(rt_out, R.n);
    double a = 0.0, e = 0.0;
    struct Pre {
        double mr, rr, vr;
    };
    struct Late {
        double mr, rr;
    };
    visit_rows<G, true>(
        R,
        [&]() {
            const double ac_inv = ainv[0];
            if (RT) {
                const DotRef refs[4] = {kd.rho1, kd.alpha1, om_r, om_v1};
                double v[4];
                dot_values<4>(refs, v);
                const bool zero = v[0] == 0.0 && v[1] == 0.0;
                const bool bad = !(v[0] > 0.0) && !zero;
                if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
                a = (bad || zero) ? 0.0 : v[1] / v[0];
                e = ac_inv * (v[2] - a * v[3]);
            } else {
                double v[1];
                dot_values<1>(&om_r, v);
                e = ac_inv * v[0];
            }
        },
        [&](int row) { return Pre{(double)minv[row], (double)r[row], RT ? (double)v1[row] : 0.0}; },
        [&](const Pre &v) { return Late{v.mr, RT ? v.rr - a * v.vr : v.rr}; },
        [&](int p) {
            const int t = ci[p];
            const double rt = RT ? (double)r[t] - a * (double)v1[t] : (double)r[t];
            return (double)va[p] * ((double)minv[t] * rt + e);
        },
        [&](int row, double s, int, const Late &v) {
            const double x = v.mr * v.rr + e;
            xout[row] = (T)(x + v.mr * (v.rr - s));
            if (RT) rt_out[row] = (T)v.rr;
        });
}

// ------------------------------------------------------------------ small single-aggregate level

// Sum over a block of kTailThreads threads (16 wavefronts); every thread
// receives the sums.
template <int N>
__device__ inline void tail_sums(double (&v)[N])
{
    static_assert(kTailThreads / kWave == 16, "one wavefront sum per lane of a row of 16");
    __shared__ double sh[N][kTailThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = 0; d < N; d++) {
        const double t = wave_sum(v[d]);
        if (lane == 0) sh[d][wid] = t;
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < N; d++) v[d] = lane_value(row16_sum(sh[d][lane & 15]), 0);
    __syncthreads();
}

// The whole coarse correction of a K-cycle visit whose coarse level C is small
// and has a single unknown below it: both flexible-CG steps (Sec. 4.4) on C, each
// preconditioned by the two-grid visit of k_post_direct, in one block per
// right-hand side.  C's entries stay in registers for the four products with A,
// the vector being multiplied is shared through LDS (as are rc and M^-1 of the
// owned rows), and every inner product is a block sum, so the correction takes
// one launch instead of four.  Vectors that the separate kernels store in T are
// rounded to T here at the same points (c1, A c1, rt, c2).
template <class T, bool GATE, bool THETA>
__global__ void __launch_bounds__(kTailThreads) k_tail_visit(TailLayout L, const T *__restrict__ va,
                                                             const T *__restrict__ minv,
                                                             const double *__restrict__ om,
                                                             const double *__restrict__ ainv,
                                                             const T *__restrict__ rc, T *__restrict__ c1,
                                                             T *__restrict__ c2, double *__restrict__ d1,
                                                             double *__restrict__ d2, int *__restrict__ flag,
                                                             const int *__restrict__ gate, double theta2)
{
    if (gated_off_if<GATE>(gate)) return;
    constexpr int R = kTailRows, W = kTailWidth, S = kTailSlots, NL = kTailLong;
    __shared__ double xs[R * kTailThreads];  // the vector being multiplied
    __shared__ double rs[R * kTailThreads];  // rc (first step), then rt (second step)
    __shared__ double ms[R * kTailThreads];  // M^-1
    const int n = L.n, t = threadIdx.x;
    rc = colv(rc, n);
    c1 = colv(c1, n);
    c2 = colv(c2, n);
    d1 = colp(d1);
    d2 = colp(d2);
    // The owned rows' rc, M^-1 and om are loaded first (clamped indices, no
    // branches) and the entries after them, so that the first block sum, which
    // needs only the former, overlaps the arrival of the entries.
    double o[R], rv[R], mv[R];
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads < n ? t + u * kTailThreads : n - 1;
        rv[u] = (double)rc[i];
        mv[u] = (double)minv[i];
        o[u] = om[i];
    }
    int ci[S];
    double a[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        ci[s] = L.ci[s * kTailThreads + t];
        a[s] = (double)va[s * kTailThreads + t];
    }
    // first row index of this wavefront's lanes (row slots of u are all padding
    // for the whole wavefront when u * kTailThreads + wbase >= n)
    const int wbase = __builtin_amdgcn_readfirstlane(t & ~(kWave - 1));
    double q[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads;
        if (i >= n) rv[u] = mv[u] = o[u] = 0.0;
        rs[i] = rv[u];
        ms[i] = mv[u];
        q[0] += o[u] * rv[u];
        if (THETA) q[1] += rv[u] * rv[u];  // (rc, rc) for the threshold test
    }
    const double acinv = ainv[0];
    // y = (A xs) at the owned rows; the sums of long rows are block sums (whose
    // barriers also end every thread's reads of xs)
    auto apply = [&](double (&y)[R]) {
        double p[S];
#pragma unroll
        for (int u = 0; u < R; u++) {
            if (u * kTailThreads + wbase < n) {
#pragma unroll
                for (int k = 0; k < W; k++) p[u * W + k] = a[u * W + k] * xs[ci[u * W + k]];
            } else {
#pragma unroll
                for (int k = 0; k < W; k++) p[u * W + k] = 0.0;
            }
        }
#pragma unroll
        for (int s = R * W; s < S; s++) p[s] = a[s] * xs[ci[s]];
#pragma unroll
        for (int u = 0; u < R; u++) {
            double acc = p[u * W];
#pragma unroll
            for (int k = 1; k < W; k++) acc += p[u * W + k];
            y[u] = acc;
        }
        double l[NL];
#pragma unroll
        for (int m = 0; m < NL; m++) {
            l[m] = 0.0;
            if (m < L.nlong) {
#pragma unroll
                for (int s = R * W; s < S; s++) {
                    const int j = s - R * W;
                    l[m] += (j >= L.long_slot[m] && j < L.long_slot[m + 1]) ? p[s] : 0.0;
                }
            }
        }
        tail_sums<NL>(l);
#pragma unroll
        for (int u = 0; u < R; u++) {
#pragma unroll
            for (int m = 0; m < NL; m++)
                if (t + u * kTailThreads == L.long_row[m]) y[u] = l[m];
        }
    };
    // first step: c1 = K(rc) with e = (om, rc) / a_c
    double om_r[1] = {q[0]}, rcrc = 0.0;
    if (THETA) {
        double v2[2] = {q[0], q[1]};
        tail_sums<2>(v2);
        om_r[0] = v2[0];
        rcrc = v2[1];
    } else {
        tail_sums<1>(om_r);
    }
    const double e1 = acinv * om_r[0];
    double x[R], y[R], c[R];
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads;
        x[u] = ms[i] * rs[i] + e1;
        xs[i] = x[u];
    }
    __syncthreads();
    apply(y);
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads;
        const T cv = (T)(x[u] + ms[i] * (rs[i] - y[u]));
        c[u] = (double)cv;
        if (i < n) c1[i] = cv;
        xs[i] = c[u];
    }
    __syncthreads();
    apply(y);  // A c1
    double v[R];
    q[0] = q[1] = q[2] = 0.0;
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads;
        v[u] = (double)(T)y[u];
        if (i < n) {
            q[0] += c[u] * y[u];
            q[1] += c[u] * rs[i];
            q[2] += o[u] * y[u];
        }
    }
    tail_sums<3>(q);
    const double rho1 = q[0], alpha1 = q[1];
    // a zero coarse residual gives c1 = 0 and no correction; a non-positive rho1
    // otherwise means A is not SPD
    const bool zero = rho1 == 0.0 && alpha1 == 0.0;
    const bool bad = !(rho1 > 0.0) && !zero;
    if (bad && t == 0) atomicOr(flag, 1);
    const double al = (bad || zero) ? 0.0 : alpha1 / rho1;
    // second step: rt = rc - (alpha1/rho1) v1, c2 = K(rt) with e = (om, rt) / a_c
    const double e2 = acinv * (om_r[0] - al * q[2]);
    double rtrt[1] = {0.0};
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads;
        const double rr = rs[i] - al * v[u];
        x[u] = ms[i] * rr + e2;
        rs[i] = rr;
        xs[i] = x[u];
        if (THETA && i < n) rtrt[0] += (double)(T)rr * (double)(T)rr;
    }
    if (THETA) {  // threshold test (Sec. 4.3): skip the second step, c2 = 0
        tail_sums<1>(rtrt);
        if (rtrt[0] < theta2 * rcrc) {
#pragma unroll
            for (int u = 0; u < R; u++) {
                const int i = t + u * kTailThreads;
                if (i < n) c2[i] = (T)0.0;
            }
            if (t == 0) {
                d1[0] = rho1;
                d1[1] = alpha1;
                d2[0] = d2[1] = d2[2] = 0.0;
            }
            return;
        }
    }
    __syncthreads();
    apply(y);  // A x
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads;
        const T cv = (T)(x[u] + ms[i] * (rs[i] - y[u]));
        c[u] = (double)cv;
        if (i < n) c2[i] = cv;
        xs[i] = c[u];
    }
    __syncthreads();
    apply(y);  // A c2
    q[0] = q[1] = q[2] = 0.0;
#pragma unroll
    for (int u = 0; u < R; u++) {
        const int i = t + u * kTailThreads;
        if (i < n) {
            q[0] += c[u] * y[u];
            q[1] += c[u] * v[u];
            q[2] += c[u] * (double)(T)rs[i];
        }
    }
    tail_sums<3>(q);
    if (t == 0) {
        d1[0] = rho1;
        d1[1] = alpha1;
        d2[0] = q[0];
        d2[1] = q[1];
        d2[2] = q[2];
    }
}

// Y = A_c^-1 X on the coarsest level for CB right-hand sides per block (see
// CoarseSolve): the block stages the coupled entries of its columns in LDS, then
// one wavefront per coupled row (lanes across the row) reads the row of the inverse
// once for all CB columns; decoupled rows are a division each.
template <class T, int CB>
__global__ void __launch_bounds__(kBlock) k_coarse_solve(CoarseSolve cs, int ncol, const T *__restrict__ x,
                                                         T *__restrict__ y)
{
    extern __shared__ double xs[];  // CB x m
    const int n = cs.n, m = cs.m;
    const int c0 = blockIdx.y * CB;
    const int nc = ncol - c0 < CB ? ncol - c0 : CB;
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < cs.nd * nc; e += gridDim.x * kBlock) {
        const int c = e / cs.nd, k = e - c * cs.nd;
        const size_t at = (size_t)(c0 + c) * n + cs.didx[k];
        y[at] = (T)((double)x[at] * cs.dinv[k]);
    }
    if (m == 0) return;
    for (int e = threadIdx.x; e < CB * m; e += kBlock) {
        const int c = e / m, j = e - c * m;
        xs[e] = c < nc ? (double)x[(size_t)(c0 + c) * n + (cs.idx ? cs.idx[j] : j)] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int nw = gridDim.x * (kBlock / kWave);
    for (int i = (blockIdx.x * kBlock + threadIdx.x) / kWave; i < m; i += nw) {
        const double *row = cs.ainv + (size_t)i * m;
        double acc[CB];
#pragma unroll
        for (int c = 0; c < CB; c++) acc[c] = 0.0;
        for (int j = lane; j < m; j += kWave) {
            const double a = row[j];
#pragma unroll
            for (int c = 0; c < CB; c++) acc[c] += a * xs[c * m + j];
        }
        const int dst = cs.idx ? cs.idx[i] : i;
#pragma unroll
        for (int c = 0; c < CB; c++) {
            const double t = wave_sum(acc[c]);
            if (lane == 0 && c < nc) y[(size_t)(c0 + c) * n + dst] = (T)t;
        }
    }
}

// Mixed precision: the K-cycle takes r / ||r|| in FP32 (it is positively
// homogeneous, so scaling the argument scales the result) and z = ||r|| z32
// comes back in FP64 with the partials of (z, q).  rr is (r, r) on the device.
__global__ void __launch_bounds__(kBlock) k_to_inner(int n, const double *__restrict__ r,
                                                     const double *__restrict__ rr, float *__restrict__ r32)
{
    r = colv(r, n);
    r32 = colv(r32, n);
    const double nr = sqrt(rr[(size_t)blockIdx.y * kScalCol]);
    const double inv = nr > 0.0 ? 1.0 / nr : 1.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) r32[i] = (float)(r[i] * inv);
}

__global__ void __launch_bounds__(kBlock) k_from_inner(int n, const float *__restrict__ z32,
                                                       const double *__restrict__ rr, double *__restrict__ z,
                                                       const double *__restrict__ q, double *__restrict__ part)
{
    z32 = colv(z32, n);
    z = colv(z, n);
    q = colv(q, n);
    part = colp(part);
    const double nr = sqrt(rr[(size_t)blockIdx.y * kScalCol]);
    const double sc = nr > 0.0 ? nr : 1.0;
    double d[1] = {0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double zi = sc * (double)z32[i];
        z[i] = zi;
        d[0] += zi * q[i];
    }
    store_partials<1>(d, part);
}

template <class S, class D>
__global__ void __launch_bounds__(kBlock) k_convert(int64_t n, const S *__restrict__ src, D *__restrict__ dst)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        dst[i] = (D)src[i];
}

// ------------------------------------------------------------------ outer flexible CG

// alpha = (p, r) / (p, A p); x += alpha p; r -= alpha q; partials of (r, r)
__global__ void __launch_bounds__(kBlock) k_fcg_update(int n, DotRef pq, DotRef pr, double *__restrict__ x,
                                                       double *__restrict__ r, const double *__restrict__ p,
                                                       const double *__restrict__ q, double *__restrict__ part,
                                                       int *__restrict__ flag, const int *__restrict__ gate)
{
    if (gated_off(gate)) return;
    x = colv(x, n);
    r = colv(r, n);
    p = colv(p, n);
    q = colv(q, n);
    part = colp(part);
    const double vpq = dot_value(pq), vpr = dot_value(pr);
    const bool zero = vpq == 0.0 && vpr == 0.0;  // p = 0: a converged or empty right-hand side
    const bool bad = !(vpq > 0.0) && !zero;
    const double alpha = (bad || zero) ? 0.0 : vpr / vpq;
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

// beta = -(z, A p) / (p, A p); p = z + beta p.  A column whose restart flag is set
// (the first step, or after a true residual that did not confirm convergence)
// takes p = z and reads no products.
__global__ void __launch_bounds__(kBlock) k_fcg_direction(int n, DotRef pq, DotRef zq, const double *__restrict__ z,
                                                          double *__restrict__ p, int *__restrict__ flag,
                                                          const int *__restrict__ gate,
                                                          const int *__restrict__ restart)
{
    if (gated_off(gate)) return;
    z = colv(z, n);
    p = colv(p, n);
    if (restart && restart[blockIdx.y]) {
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i];
        return;
    }
    const double vpq = dot_value(pq), vzq = dot_value(zq);
    const bool zero = vpq == 0.0 && vzq == 0.0;
    const bool bad = !(vpq > 0.0) && !zero;
    const double beta = (bad || zero) ? 0.0 : -vzq / vpq;
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kBlock) k_dot(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                double *__restrict__ part)
{
    a = colv(a, n);
    b = colv(b, n);
    part = colp(part);
    double d[1] = {0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[0] += a[i] * b[i];
    store_partials<1>(d, part);
}

__global__ void __launch_bounds__(kBlock) k_gather(int n, const double *__restrict__ src, int ld_src,
                                                   const int *__restrict__ idx, double *__restrict__ dst, int ld_dst)
{
    src = colv(src, ld_src);
    dst = colv(dst, ld_dst);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = src[idx ? idx[i] : i];
}

__global__ void __launch_bounds__(kBlock) k_scatter(int n, const double *__restrict__ src, int ld_src,
                                                    const int *__restrict__ idx, double *__restrict__ dst, int ld_dst)
{
    src = colv(src, ld_src);
    dst = colv(dst, ld_dst);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[idx ? idx[i] : i] = src[i];
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
// every consumer block.  The sliced sweeps pass a limit of 1: their consumers
// (the outer-iteration updates, the next level's smoothers) are grids of
// thousands of blocks, each of which would otherwise load the whole set.
constexpr int kConsumerReduceMax = 1024;

void reduce_if_large(int nd, double *part, int count, double *final_out, hipStream_t s, int ncol,
                     int limit = kConsumerReduceMax, const int *gate = nullptr)
{
    if (count > limit && final_out) {
        k_reduce_partials<<<dim3(1, ncol), kReduceThreads, 0, s>>>(nd, part, count, final_out, kDotCol, gate);
        AMG_HIP(hipGetLastError());
    }
}

DotRef finished(double *part, int count, double *final_out, int d, int limit = kConsumerReduceMax)
{
    if (count <= limit || final_out == nullptr) return DotRef{part + d * kPartStride, count};
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
    if (R.n < kSmallLevel) {
        AMG_SWITCH_G(G, (k_spmv<kG, true><<<grid, kBlock, 0, s>>>(R, ci, va, x, y)));
    } else {
        AMG_SWITCH_G(G, (k_spmv<kG, false><<<grid, kBlock, 0, s>>>(R, ci, va, x, y)));
    }
    AMG_HIP(hipGetLastError());
}

// Blocks of a sliced sweep: tpb tiles each, raised so that a dot site's partial
// set (one per block) fits kMaxDotBlocks.
inline int sell_grid(const Sell &S, bool dot, int *tpb)
{
    const int64_t tiles = ((int64_t)S.n + kBlock - 1) / kBlock;
    int64_t t = S.tpb < 1 ? 1 : S.tpb;
    if (dot && (tiles + t - 1) / t > kMaxDotBlocks) t = (tiles + kMaxDotBlocks - 1) / kMaxDotBlocks;
    *tpb = (int)t;
    return (int)((tiles + t - 1) / t);
}

template <class T>
DotSet launch_spmv_dots(Rows R, const int *ci, const T *va, const T *x, T *y, const T *w1, const T *w2, int G,
                        DotBuf buf, hipStream_t s, const double *omy, int ncol, const Sell *sl, const T *sva,
                        const int *gate)
{
    const int nd = w2 ? 3 : (w1 ? 2 : 1);
    if (sl) {
        if (omy) throw Error(4, "spmv_dots: no (om, A x) on a sliced level");
        int tpb = 1;
        const dim3 grid(sell_grid(*sl, true, &tpb), ncol);
#define AMG_SELL_DOTS(ND) \
    k_sell_spmv_dots<T, ND><<<grid, kBlock, 0, s>>>(sl->n, tpb, sl->ptr, sl->ci, sva, x, y, w1, w2, buf.part, gate)
        if (nd == 1) AMG_SELL_DOTS(1);
        else if (nd == 2) AMG_SELL_DOTS(2);
        else AMG_SELL_DOTS(3);
#undef AMG_SELL_DOTS
        AMG_HIP(hipGetLastError());
        const int count = (int)grid.x;
        reduce_if_large(nd, buf.part, count, buf.final_out, s, ncol, 1, gate);
        DotSet out{};
        for (int d = 0; d < nd; d++) out.d[d] = finished(buf.part, count, buf.final_out, d, 1);
        return out;
    }
    const bool lat = R.n < kSmallLevel;
    if (ncol > 1 && !lat && !omy && R.cb > 1) {  // batched: CB columns per block
        const dim3 gm(rows_grid(R, G, kMaxDotBlocks), (ncol + R.cb - 1) / R.cb);
#define AMG_SPMM(ND, CB)                                                                                             \
    AMG_SWITCH_G(G, (k_spmm_dots<T, kG, ND, CB><<<gm, kBlock, 0, s>>>(R, ci, va, x, y, w1, w2, buf.part, ncol, gate)))
#define AMG_SPMM_CB(ND)                    \
    switch (R.cb) {                        \
    case 2: AMG_SPMM(ND, 2); break;        \
    case 4: AMG_SPMM(ND, 4); break;        \
    default: AMG_SPMM(ND, 8); break;       \
    }
        if (nd == 1) { AMG_SPMM_CB(1) } else if (nd == 2) { AMG_SPMM_CB(2) } else { AMG_SPMM_CB(3) }
#undef AMG_SPMM_CB
#undef AMG_SPMM
        AMG_HIP(hipGetLastError());
        const int count = (int)gm.x + R.nlong;
        reduce_if_large(nd, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
        DotSet out{};
        for (int d = 0; d < nd; d++) out.d[d] = finished(buf.part, count, buf.final_out, d);
        return out;
    }
    const dim3 grid(rows_grid(R, G, kMaxDotBlocks), ncol);
    if (omy && nd == 3) throw Error(4, "spmv_dots: at most three products");
#define AMG_SPMV_DOTS_GATE(ND, LAT, OMY, GT)                                                                  \
    AMG_SWITCH_G(G, (k_spmv_dots<T, kG, ND, LAT, OMY, GT><<<grid, kBlock, 0, s>>>(R, ci, va, x, y, w1, w2, omy, \
                                                                                   buf.part, gate)))
#define AMG_SPMV_DOTS(ND, LAT, OMY)               \
    if (gate) {                                   \
        AMG_SPMV_DOTS_GATE(ND, LAT, OMY, true);   \
    } else {                                      \
        AMG_SPMV_DOTS_GATE(ND, LAT, OMY, false);  \
    }
    if (omy) {
        if (nd == 1) {
            AMG_SPMV_DOTS(1, true, true);
        } else {
            AMG_SPMV_DOTS(2, true, true);
        }
    } else if (nd == 1) {
        if (lat) {
            AMG_SPMV_DOTS(1, true, false);
        } else {
            AMG_SPMV_DOTS(1, false, false);
        }
    } else if (nd == 2) {
        if (lat) {
            AMG_SPMV_DOTS(2, true, false);
        } else {
            AMG_SPMV_DOTS(2, false, false);
        }
    } else {
        if (lat) {
            AMG_SPMV_DOTS(3, true, false);
        } else {
            AMG_SPMV_DOTS(3, false, false);
        }
    }
#undef AMG_SPMV_DOTS
#undef AMG_SPMV_DOTS_GATE
    AMG_HIP(hipGetLastError());
    const int nt = nd + (omy ? 1 : 0);
    const int count = (int)grid.x + R.nlong;
    reduce_if_large(nt, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
    DotSet out{};
    for (int d = 0; d < nt; d++) out.d[d] = finished(buf.part, count, buf.final_out, d);
    return out;
}

DotSet launch_residual(Rows R, const int *ci, const double *va, const double *b, const double *x, double *r, int G,
                       DotBuf buf, hipStream_t s, int ncol, const int *gate)
{
    const dim3 grid(rows_grid(R, G, kMaxDotBlocks), ncol);
    AMG_SWITCH_G(G, (k_residual<kG><<<grid, kBlock, 0, s>>>(R, ci, va, b, x, r, buf.part, gate)));
    AMG_HIP(hipGetLastError());
    const int count = (int)grid.x + R.nlong;
    reduce_if_large(2, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
    DotSet out{};
    for (int d = 0; d < 2; d++) out.d[d] = finished(buf.part, count, buf.final_out, d);
    return out;
}

void launch_reduce(const DotRef &ref, double *out, hipStream_t s, int ncol, int out_stride, const int *gate)
{
    k_reduce_partials<<<dim3(1, ncol), kReduceThreads, 0, s>>>(1, ref.part, ref.count, out, out_stride, gate);
    AMG_HIP(hipGetLastError());
}

template <class T>
DotRef launch_restrict(Rows S, int nf, const int *ci, const T *wv, const T *r, T *rc, int G, hipStream_t s,
                       const double *om, DotBuf buf, int ncol, const int *gate)
{
    if (ncol > 1 && !om && S.n >= kSmallLevel && S.cb > 1) {  // batched: CB columns per block
        const dim3 gm(rows_grid(S, G, 1 << 20), (ncol + S.cb - 1) / S.cb);
#define AMG_RMM(CB) \
    AMG_SWITCH_G(G, (k_restrict_mm<T, kG, CB><<<gm, kBlock, 0, s>>>(S, nf, ci, wv, r, rc, ncol, gate)))
        switch (S.cb) {
        case 2: AMG_RMM(2); break;
        case 4: AMG_RMM(4); break;
        default: AMG_RMM(8); break;
        }
#undef AMG_RMM
        AMG_HIP(hipGetLastError());
        return DotRef{nullptr, 0};
    }
    const dim3 grid(rows_grid(S, G, om ? kMaxDotBlocks : (1 << 20)), ncol);
#define AMG_RESTRICT(LAT, OM)                                                                                        \
    if (gate) {                                                                                                      \
        AMG_SWITCH_G(G, (k_restrict<T, kG, LAT, OM, true><<<grid, kBlock, 0, s>>>(S, nf, ci, wv, r, rc, om, buf.part, \
                                                                                   gate)));                          \
    } else {                                                                                                         \
        AMG_SWITCH_G(G, (k_restrict<T, kG, LAT, OM, false><<<grid, kBlock, 0, s>>>(S, nf, ci, wv, r, rc, om,         \
                                                                                    buf.part, gate)));               \
    }
    if (om) {
        AMG_RESTRICT(true, true)
    } else if (S.n < kSmallLevel) {
        AMG_RESTRICT(true, false)
    } else {
        AMG_RESTRICT(false, false)
    }
#undef AMG_RESTRICT
    AMG_HIP(hipGetLastError());
    if (!om) return DotRef{nullptr, 0};
    const int count = (int)grid.x + S.nlong;
    reduce_if_large(1, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
    return finished(buf.part, count, buf.final_out, 0);
}

template <class T>
void launch_inner_residual(int n, const T *rc, const T *v1, KDots kd, T *rt, int *flag, hipStream_t s, int ncol,
                           const int *gate)
{
    k_inner_residual<T><<<dim3(grid_for(n, 4096), ncol), kBlock, 0, s>>>(n, rc, v1, kd, rt, flag, gate);
    AMG_HIP(hipGetLastError());
}

template <class T>
DotRef launch_inner_residual_theta(int n, const T *rc, const T *v1, KDots kd, T *rt, int *flag, const double *om,
                                   DotBuf buf, double theta2, const int *gate, int *gate_out, hipStream_t s, int ncol)
{
    const dim3 grid(grid_for(n, 4096), ncol);
    if (om) k_inner_residual_theta<T, true><<<grid, kBlock, 0, s>>>(n, rc, v1, kd, rt, flag, om, buf.part, gate);
    else k_inner_residual_theta<T, false><<<grid, kBlock, 0, s>>>(n, rc, v1, kd, rt, flag, om, buf.part, gate);
    AMG_HIP(hipGetLastError());
    const int nd = om ? 3 : 2, count = (int)grid.x;
    reduce_if_large(nd, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
    k_theta_gate<<<dim3(1, ncol), kBlock, 0, s>>>(finished(buf.part, count, buf.final_out, 0),
                                                  finished(buf.part, count, buf.final_out, 1), theta2, gate, gate_out);
    AMG_HIP(hipGetLastError());
    return om ? finished(buf.part, count, buf.final_out, 2) : DotRef{nullptr, 0};
}

template <class T>
DotRef launch_post_smooth(Rows R, const int *ci, const T *va, const T *minv, const T *r, const int *agg_pos,
                          const int *cagg, int mode, const T *edirect, const T *c1, const T *c2, KDots kd, T *xout,
                          const T *wdot, DotBuf buf, int *flag, int G, hipStream_t s, const double *ainv, int nc,
                          int ncol, double *xtmp, const Sell *sl, const T *sva, const int *gate, const int *second)
{
    const bool dot = wdot != nullptr;
    const dim3 grid(rows_grid(R, G, dot ? kMaxDotBlocks : (1 << 20)), ncol);
    if (sl && sl->fused && !cagg && R.n >= kSmallLevel && mode >= 0 && mode <= 2) {  // one sweep
        int tpb = 1;
        const dim3 gs(sell_grid(*sl, dot, &tpb), ncol);
#define AMG_FUSED(M, D)                                                                                            \
    k_sell_post_fused<T, M, D><<<gs, kBlock, 0, s>>>(sl->n, tpb, sl->ptr, sl->ci, sva, minv, r, agg_pos, edirect, c1, \
                                                     c2, kd, nc, xout, wdot, buf.part, flag, gate, second)
        switch (mode) {
        case 0: if (dot) { AMG_FUSED(0, true); } else { AMG_FUSED(0, false); } break;
        case 1: if (dot) { AMG_FUSED(1, true); } else { AMG_FUSED(1, false); } break;
        default: if (dot) { AMG_FUSED(2, true); } else { AMG_FUSED(2, false); } break;
        }
#undef AMG_FUSED
        AMG_HIP(hipGetLastError());
        if (!dot) return DotRef{nullptr, 0};
        reduce_if_large(1, buf.part, (int)gs.x, buf.final_out, s, ncol, 1, gate);
        return finished(buf.part, (int)gs.x, buf.final_out, 0, 1);
    }
    if (xtmp && !cagg && R.n >= kSmallLevel && mode >= 0 && mode <= 2) {  // two launches, see k_smooth_start
        const dim3 g1(grid_for(R.n, 1 << 16), ncol);
#define AMG_START(M) \
    k_smooth_start<T, M><<<g1, kBlock, 0, s>>>(R.n, minv, r, agg_pos, edirect, c1, c2, kd, xtmp, flag, nc, gate, second)
        switch (mode) {
        case 0: AMG_START(0); break;
        case 1: AMG_START(1); break;
        default: AMG_START(2); break;
        }
#undef AMG_START
        AMG_HIP(hipGetLastError());
        if (sl) {
            int tpb = 1;
            const dim3 gs(sell_grid(*sl, dot, &tpb), ncol);
            if (dot) {
                k_sell_smooth_finish<T, true><<<gs, kBlock, 0, s>>>(sl->n, tpb, sl->ptr, sl->ci, sva, minv, r, xtmp,
                                                                    xout, wdot, buf.part, gate);
            } else {
                k_sell_smooth_finish<T, false><<<gs, kBlock, 0, s>>>(sl->n, tpb, sl->ptr, sl->ci, sva, minv, r, xtmp,
                                                                     xout, wdot, buf.part, gate);
            }
            AMG_HIP(hipGetLastError());
            if (!dot) return DotRef{nullptr, 0};
            reduce_if_large(1, buf.part, (int)gs.x, buf.final_out, s, ncol, 1, gate);
            return finished(buf.part, (int)gs.x, buf.final_out, 0, 1);
        }
        if (ncol > 1 && R.cb > 1) {  // batched: CB columns per block
            const dim3 gm(grid.x, (ncol + R.cb - 1) / R.cb);
#define AMG_FMM(D, CB)                                                                                              \
    AMG_SWITCH_G(G, (k_smooth_finish_mm<T, kG, D, CB><<<gm, kBlock, 0, s>>>(R, ci, va, minv, r, xtmp, xout, wdot, \
                                                                            buf.part, ncol, gate)))
            switch (R.cb) {
            case 2: if (dot) { AMG_FMM(true, 2); } else { AMG_FMM(false, 2); } break;
            case 4: if (dot) { AMG_FMM(true, 4); } else { AMG_FMM(false, 4); } break;
            default: if (dot) { AMG_FMM(true, 8); } else { AMG_FMM(false, 8); } break;
            }
#undef AMG_FMM
        } else if (dot) {
            AMG_SWITCH_G(G, (k_smooth_finish<T, kG, true><<<grid, kBlock, 0, s>>>(R, ci, va, minv, r, xtmp, xout, wdot,
                                                                                buf.part, gate)));
        } else {
            AMG_SWITCH_G(G, (k_smooth_finish<T, kG, false><<<grid, kBlock, 0, s>>>(R, ci, va, minv, r, xtmp, xout, wdot,
                                                                                 buf.part, gate)));
        }
        AMG_HIP(hipGetLastError());
        if (!dot) return DotRef{nullptr, 0};
        const int count = (int)grid.x + R.nlong;
        reduce_if_large(1, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
        return finished(buf.part, count, buf.final_out, 0);
    }
#define AMG_POST_G(M, D, CA, GT)                                                                        \
    AMG_SWITCH_G(G, (k_post_smooth<T, kG, M, D, CA, GT><<<grid, kBlock, 0, s>>>(                                \
                        R, ci, va, minv, r, agg_pos, cagg, edirect, c1, c2, kd, xout, wdot, buf.part, flag, ainv, nc, \
                        gate, second)))
#define AMG_POST(M, D)                                                                                   \
    do {                                                                                                 \
        const bool gt = gate || second;                                                                  \
        if (cagg) {                                                                                      \
            if (gt) { AMG_POST_G(M, D, true, true); } else { AMG_POST_G(M, D, true, false); }            \
        } else {                                                                                         \
            if (gt) { AMG_POST_G(M, D, false, true); } else { AMG_POST_G(M, D, false, false); }          \
        }                                                                                                \
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
#undef AMG_POST_G
    AMG_HIP(hipGetLastError());
    if (!dot) return DotRef{nullptr, 0};
    const int count = (int)grid.x + R.nlong;
    reduce_if_large(1, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
    return finished(buf.part, count, buf.final_out, 0);
}

template <class T>
void launch_sell_restrict(const Sell &S, const T *sva, const T *minv, const T *r, double *t, int nc, const int *seg,
                          const int *idx, T *rc, hipStream_t s, int ncol, const int *gate)
{
    int tpb = 1;
    const dim3 grid(sell_grid(S, false, &tpb), ncol);
    k_sell_presmooth_residual<T><<<grid, kBlock, 0, s>>>(S.n, tpb, S.ptr, S.ci, sva, minv, r, t, gate);
    AMG_HIP(hipGetLastError());
    k_segment_sum<T><<<dim3(grid_for(nc), ncol), kBlock, 0, s>>>(nc, seg, idx, S.n, t, rc, gate);
    AMG_HIP(hipGetLastError());
}

template <class T>
DotRef launch_restrict_rt(Rows S, int nf, const int *ci, const T *wv, const T *rcf, const T *v1, KDots kd, T *rt,
                          T *rc, int *flag, int G, hipStream_t s, const double *om, DotBuf buf, int ncol,
                          const int *gate)
{
    const dim3 grid(rows_grid(S, G, om ? kMaxDotBlocks : (1 << 20)), ncol);
#define AMG_RESTRICT_RT(OM, GT)                                                                                 \
    AMG_SWITCH_G(G, (k_restrict_rt<T, kG, OM, GT><<<grid, kBlock, 0, s>>>(S, nf, ci, wv, rcf, v1, kd, rt, rc, flag, \
                                                                           om, buf.part, gate)))
    if (om) {
        if (gate) { AMG_RESTRICT_RT(true, true); } else { AMG_RESTRICT_RT(true, false); }
    } else {
        if (gate) { AMG_RESTRICT_RT(false, true); } else { AMG_RESTRICT_RT(false, false); }
    }
#undef AMG_RESTRICT_RT
    AMG_HIP(hipGetLastError());
    if (!om) return DotRef{nullptr, 0};
    const int count = (int)grid.x + S.nlong;
    reduce_if_large(1, buf.part, count, buf.final_out, s, ncol, kConsumerReduceMax, gate);
    return finished(buf.part, count, buf.final_out, 0);
}

template <class T>
void launch_post_direct(Rows R, const int *ci, const T *va, const T *minv, const T *r, const T *v1, KDots kd,
                        DotRef om_r, DotRef om_v1, const double *ainv, T *xout, T *rt_out, int *flag, int G,
                        bool rt_mode, hipStream_t s, int ncol, const int *gate)
{
    const dim3 grid(rows_grid(R, G, 1 << 20), ncol);
#define AMG_DIRECT(RT, GT)                                                                                \
    AMG_SWITCH_G(G, (k_post_direct<T, kG, RT, GT><<<grid, kBlock, 0, s>>>(R, ci, va, minv, r, v1, kd, om_r, om_v1, \
                                                                           ainv, xout, rt_out, flag, gate)))
    if (rt_mode) {
        if (gate) { AMG_DIRECT(true, true); } else { AMG_DIRECT(true, false); }
    } else {
        if (gate) { AMG_DIRECT(false, true); } else { AMG_DIRECT(false, false); }
    }
#undef AMG_DIRECT
    AMG_HIP(hipGetLastError());
}

template <class T>
void launch_tail_visit(const TailLayout &L, const T *va, const T *minv, const double *om, const double *ainv,
                       const T *rc, T *c1, T *c2, double *d1, double *d2, int *flag, hipStream_t s, int ncol,
                       const int *gate, double theta2)
{
#define AMG_TAIL(GT, TH)                                                                                           \
    k_tail_visit<T, GT, TH><<<dim3(1, ncol), kTailThreads, 0, s>>>(L, va, minv, om, ainv, rc, c1, c2, d1, d2, flag, gate, \
                                                                   theta2)
    if (gate) {
        if (theta2 > 0.0) { AMG_TAIL(true, true); } else { AMG_TAIL(true, false); }
    } else {
        if (theta2 > 0.0) { AMG_TAIL(false, true); } else { AMG_TAIL(false, false); }
    }
#undef AMG_TAIL
    AMG_HIP(hipGetLastError());
}

bool build_tail_layout(int n, const int *rp, const int *ci, const double *va, std::vector<uint16_t> &tci,
                       std::vector<double> &tva, TailLayout &L)
{
    if (n < 1 || n > kTailRows * kTailThreads) return false;
    L = TailLayout{};
    L.n = n;
    for (int m = 0; m < kTailLong; m++) L.long_row[m] = -1;
    tci.assign((size_t)kTailSlots * kTailThreads, 0);  // padding: column 0, value 0
    tva.assign((size_t)kTailSlots * kTailThreads, 0.0);
    constexpr int first_long = kTailRows * kTailWidth;
    int nlong = 0, used = 0;
    for (int i = 0; i < n; i++) {
        const int b = rp[i], len = rp[i + 1] - b;
        if (len <= kTailWidth) {
            const int t = i % kTailThreads, u = i / kTailThreads;
            for (int k = 0; k < len; k++) {
                const size_t at = (size_t)(u * kTailWidth + k) * kTailThreads + t;
                tci[at] = (uint16_t)ci[b + k];
                tva[at] = va[b + k];
            }
            continue;
        }
        const int slots = (len + kTailThreads - 1) / kTailThreads;
        if (nlong == kTailLong || used + slots > kTailLongSlots) return false;
        for (int j = 0; j < len; j++) {
            const size_t at = (size_t)(first_long + used + j / kTailThreads) * kTailThreads + j % kTailThreads;
            tci[at] = (uint16_t)ci[b + j];
            tva[at] = va[b + j];
        }
        L.long_row[nlong] = i;
        used += slots;
        L.long_slot[++nlong] = used;
    }
    for (int m = nlong; m < kTailLong; m++) L.long_slot[m + 1] = used;  // empty ranges
    L.nlong = nlong;
    return true;
}

template <class T>
void launch_coarse_solve(const CoarseSolve &cs, const T *x, T *y, hipStream_t s, int ncol)
{
    // columns per block: the staged columns take at most 64 KiB of LDS
    int cb = 1;
    while (cb < 16 && cb < ncol && (size_t)(2 * cb) * cs.m * sizeof(double) <= 65536) cb *= 2;
    const int rows_blocks = cs.m > 0 ? (cs.m + kBlock / kWave - 1) / (kBlock / kWave) : 1;
    const int dec_blocks = (cs.nd * cb + kBlock - 1) / kBlock;
    const int gx = std::max(1, std::min(1024, std::max(rows_blocks, dec_blocks)));
    const dim3 grid(gx, (ncol + cb - 1) / cb);
    const size_t lds = (size_t)cb * cs.m * sizeof(double);
    switch (cb) {
    case 1: k_coarse_solve<T, 1><<<grid, kBlock, lds, s>>>(cs, ncol, x, y); break;
    case 2: k_coarse_solve<T, 2><<<grid, kBlock, lds, s>>>(cs, ncol, x, y); break;
    case 4: k_coarse_solve<T, 4><<<grid, kBlock, lds, s>>>(cs, ncol, x, y); break;
    case 8: k_coarse_solve<T, 8><<<grid, kBlock, lds, s>>>(cs, ncol, x, y); break;
    default: k_coarse_solve<T, 16><<<grid, kBlock, lds, s>>>(cs, ncol, x, y); break;
    }
    AMG_HIP(hipGetLastError());
}

void launch_to_inner(int n, const double *r, const double *rr, float *r32, hipStream_t s, int ncol)
{
    k_to_inner<<<dim3(grid_for(n, 8192), ncol), kBlock, 0, s>>>(n, r, rr, r32);
    AMG_HIP(hipGetLastError());
}

DotRef launch_from_inner(int n, const float *z32, const double *rr, double *z, const double *q, DotBuf buf,
                         hipStream_t s, int ncol)
{
    const int grid = grid_for(n, kMaxDotBlocks);
    k_from_inner<<<dim3(grid, ncol), kBlock, 0, s>>>(n, z32, rr, z, q, buf.part);
    AMG_HIP(hipGetLastError());
    reduce_if_large(1, buf.part, grid, buf.final_out, s, ncol);
    return finished(buf.part, grid, buf.final_out, 0);
}

void launch_to_float(int64_t n, const double *src, float *dst, hipStream_t s)
{
    k_convert<double, float><<<grid_for(n, 1 << 16), kBlock, 0, s>>>(n, src, dst);
    AMG_HIP(hipGetLastError());
}

#define AMG_INSTANTIATE(T)                                                                                           \
    template DotSet launch_spmv_dots<T>(Rows, const int *, const T *, const T *, T *, const T *, const T *, int,     \
                                        DotBuf, hipStream_t, const double *, int, const Sell *, const T *,          \
                                        const int *);                                                               \
    template DotRef launch_restrict<T>(Rows, int, const int *, const T *, const T *, T *, int, hipStream_t,          \
                                       const double *, DotBuf, int, const int *);                                   \
    template void launch_sell_restrict<T>(const Sell &, const T *, const T *, const T *, double *, int, const int *, \
                                          const int *, T *, hipStream_t, int, const int *);                         \
    template void launch_inner_residual<T>(int, const T *, const T *, KDots, T *, int *, hipStream_t, int,         \
                                           const int *);                                                            \
    template DotRef launch_inner_residual_theta<T>(int, const T *, const T *, KDots, T *, int *, const double *,    \
                                                   DotBuf, double, const int *, int *, hipStream_t, int);           \
    template DotRef launch_post_smooth<T>(Rows, const int *, const T *, const T *, const T *, const int *,          \
                                          const int *, int, const T *, const T *, const T *, KDots, T *, const T *, \
                                          DotBuf, int *, int, hipStream_t, const double *, int, int, double *,      \
                                          const Sell *, const T *, const int *, const int *);                       \
    template DotRef launch_restrict_rt<T>(Rows, int, const int *, const T *, const T *, const T *, KDots, T *, T *, \
                                          int *, int, hipStream_t, const double *, DotBuf, int, const int *);       \
    template void launch_post_direct<T>(Rows, const int *, const T *, const T *, const T *, const T *, KDots,       \
                                        DotRef, DotRef, const double *, T *, T *, int *, int, bool, hipStream_t,    \
                                        int, const int *);                                                          \
    template void launch_coarse_solve<T>(const CoarseSolve &, const T *, T *, hipStream_t, int);                   \
    template void launch_tail_visit<T>(const TailLayout &, const T *, const T *, const double *, const double *,    \
                                       const T *, T *, T *, double *, double *, int *, hipStream_t, int,            \
                                       const int *, double);
AMG_INSTANTIATE(double)
AMG_INSTANTIATE(float)
#undef AMG_INSTANTIATE

DotRef launch_fcg_update(int n, DotRef pq, DotRef pr, double *x, double *r, const double *p, const double *q,
                         DotBuf buf, int *flag, hipStream_t s, int ncol, const int *gate)
{
    const int grid = grid_for(n, kMaxDotBlocks);
    k_fcg_update<<<dim3(grid, ncol), kBlock, 0, s>>>(n, pq, pr, x, r, p, q, buf.part, flag, gate);
    AMG_HIP(hipGetLastError());
    reduce_if_large(1, buf.part, grid, buf.final_out, s, ncol, kConsumerReduceMax, gate);
    return finished(buf.part, grid, buf.final_out, 0);
}

void launch_fcg_direction(int n, DotRef pq, DotRef zq, const double *z, double *p, int *flag, hipStream_t s, int ncol,
                          const int *gate, const int *restart)
{
    k_fcg_direction<<<dim3(grid_for(n, 4096), ncol), kBlock, 0, s>>>(n, pq, zq, z, p, flag, gate, restart);
    AMG_HIP(hipGetLastError());
}

DotRef launch_dot(int n, const double *a, const double *b, DotBuf buf, hipStream_t s, int ncol)
{
    const int grid = grid_for(n, kMaxDotBlocks);
    k_dot<<<dim3(grid, ncol), kBlock, 0, s>>>(n, a, b, buf.part);
    AMG_HIP(hipGetLastError());
    reduce_if_large(1, buf.part, grid, buf.final_out, s, ncol);
    return finished(buf.part, grid, buf.final_out, 0);
}

void launch_gather(int n, const double *src, const int *idx, double *dst, hipStream_t s, int ncol, int ld_src,
                   int ld_dst)
{
    k_gather<<<dim3(grid_for(n, 4096), ncol), kBlock, 0, s>>>(n, src, ld_src > 0 ? ld_src : n, idx, dst,
                                                              ld_dst > 0 ? ld_dst : n);
    AMG_HIP(hipGetLastError());
}

void launch_scatter(int n, const double *src, const int *idx, double *dst, hipStream_t s, int ncol, int ld_src,
                    int ld_dst)
{
    k_scatter<<<dim3(grid_for(n, 4096), ncol), kBlock, 0, s>>>(n, src, ld_src > 0 ? ld_src : n, idx, dst,
                                                               ld_dst > 0 ? ld_dst : n);
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

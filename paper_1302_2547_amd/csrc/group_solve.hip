// group_solve.hip -- grouped solves of small problems (gfx950).
//
// A hierarchy of a small problem spends its solve in latency: every visit of a
// coarse level is a handful of dependent launches over a few thousand rows.  Here
// one workgroup of kGroupBlock threads runs the whole solve of one right-hand side
// -- the outer flexible CG of Sec. 4.4 with the K-cycle of Sec. 4.3 as its
// preconditioner -- with block barriers between the sweeps instead of launches,
// and one launch carries any number of such jobs (different problems, sizes and
// depths), so the small-level work of concurrent requests shares one dispatch.
//
// The method is that of the multi-launch path, step for step:
//   K-cycle on level k (Alg. 1 solve phase): pre-smoothing from zero x = M^-1 r,
//     restriction rc = P^T (r - A x), the coarse problem solved by nu flexible-CG
//     steps preconditioned by the K-cycle one level down (exactly on the coarsest
//     level), prolongation x += P e and post-smoothing x += M^-1 (r - A x);
//   inner steps (Sec. 4.3): c1 = K(rc), v1 = A c1, rho1 = (c1, v1),
//     alpha1 = (c1, rc) / rho1, rt = rc - alpha1 v1; with a second step
//     c2 = K(rt), gamma = (c2, v1), rho2 = (c2, A c2) - gamma^2 / rho1 (the second
//     direction c2 - (gamma / rho1) c1 made A-orthogonal to c1),
//     alpha2 = (c2, rt) / rho2 with (c2, rt) = (c2, rc) - alpha1 gamma,
//     e = (alpha1 - alpha2 gamma / rho1) c1 + alpha2 c2; the second step is skipped
//     when ||rt|| < theta ||rc|| (theta > 0);
//   outer iteration: flexible CG with truncation 1, stopping when the recursive
//     relative residual reaches tol and the true one confirms it (else the
//     iteration continues from the true residual).
// The pre-smoothed iterate is never stored: x_j = M^-1_jj r_j is formed where it is
// read, and the post-smoothing forms the prolonged iterate per entry, so a visit of
// level k reads its input and writes its output only; nor is rt: the second
// visit's input is formed as rc_j - alpha1 v1_j where it is read.  All sums are in
// a fixed order (a job's result does not depend on the other jobs of the launch).
//
// One compute unit's memory pipeline sets the cost here: a sweep is a chain of
// dependent gathers (row pointer, column, gathered value) that one workgroup
// issues for all rows of the level, and every pass ends at a barrier.  Each sweep
// keeps kRows rows per lane group in flight, loads what a row's result needs (its
// own input, diagonal and coarse correction) together with its row pointer, and a
// visit makes four passes: restriction, post-smoothing, and the products of the
// two inner steps.  Measured on MI355X, a job takes 4-10x the time of the
// multi-launch solve of its hierarchy alone (whose sweeps spread over every
// compute unit), so the grouped launch pays off only with many concurrent jobs.
//
// The recursion runs as a loop over a per-level state: bit k of `second` says
// whether the visit of level k in progress is the second inner step's (input rt,
// output c2) or the first's (input rc, output c1); alpha1, rho1 and ||rc||^2 of a
// level's first step wait in LDS for its second.
#include "amg.h"
#include "amg_internal.h"
#include "wave_ops.h"

namespace amg {
namespace {

constexpr int kGB = kGroupBlock;
constexpr int kGW = kGB / kWave;  // wavefronts per workgroup
constexpr int kRows = 2;  // rows (aggregates, elements) per lane group in flight (4 and 8 measured slower)

struct Shared {
    double part[2][kGW][3];  // wavefront partial sums, two sets used in turn
    double a1[kGroupMaxLevels], r1[kGroupMaxLevels], gg[kGroupMaxLevels];
};

// Block-wide reductions: every thread passes its share and gets the totals, each
// thread adding the kGW wavefront partials itself in the same order.  Consecutive
// reductions alternate between two partial sets, so one barrier per reduction
// suffices: a set is written again only two reductions later, after every thread
// has passed the barrier of the reduction in between (and so has read it).
struct Red {
    Shared &sh;
    int phase;
};

// A K-cycle input vector: a[j], or a[j] - alpha b[j] (the inner residual after the
// first step, rt = rc - alpha1 v1, formed where it is read)
struct Input {
    const double *a, *b;
    double alpha;
    __device__ __forceinline__ double operator()(int j) const { return b ? a[j] - alpha * b[j] : a[j]; }
};

// sum over each aligned group of G lanes (G uniform: 1, 2, 4, 8 or 16), received by
// every lane of the group; all lanes of the wavefront must be active
__device__ __forceinline__ double lanes_sum(double v, int G)
{
    if (G >= 2) v += dpp_f64<kDppQuadXor1>(v);
    if (G >= 4) v += dpp_f64<kDppQuadXor2>(v);
    if (G >= 8) v += dpp_f64<kDppRowHalfMirror>(v);
    if (G >= 16) v += dpp_f64<kDppRowMirror>(v);
    return v;
}

template <int ND>
__device__ __forceinline__ void block_sum(double (&v)[ND], Red &red)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double(&part)[kGW][3] = red.sh.part[red.phase];
    red.phase ^= 1;
#pragma unroll
    for (int d = 0; d < ND; d++) {
        const double s = wave_sum(v[d]);
        if (lane == 0) part[w][d] = s;
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < ND; d++) {
        double s = 0.0;
        for (int k = 0; k < kGW; k++) s += part[k][d];
        v[d] = s;
    }
}

// Row sweep of a level with G lanes per row and kRows rows per lane group in
// flight: s_i = sum over the row's entries of entry(e, column), summed in a fixed
// order (lane g takes entries g, g + G, ...; then the group sum), then
// fin(i, s_i, ok, pre(i)) with ok on the group's first lane of a row i < n.  The
// row data pre(i) is loaded with the row pointers, before the entries; rows past
// n are clamped to row n - 1 (and get no entries) so that every load is valid.
template <class EntryF, class PreF, class RowF>
__device__ __forceinline__ void sweep(const GroupLevel &F, Red &red, EntryF entry, PreF pre, RowF fin)
{
    using P = decltype(pre(0));
    const int n = F.n, G = F.G, lim = F.lim;
    const int *rp = F.rp, *ci = F.ci;
    const int g = threadIdx.x & (G - 1), slot = threadIdx.x / G, step = kGB / G;
    for (int i0 = 0; i0 < n; i0 += kRows * step) {
        int e[kRows], end[kRows];
        bool own[kRows];  // a row of this lane group (not a hub row, which the block sums below)
        double s[kRows];
        P pd[kRows];
#pragma unroll
        for (int r = 0; r < kRows; r++) {
            const int raw = i0 + r * step + slot, i = min(raw, n - 1);
            const int b = rp[i], t = rp[i + 1];
            pd[r] = pre(i);
            own[r] = raw < n && t - b <= lim;
            e[r] = b + g;
            end[r] = own[r] ? t : 0;
            s[r] = 0.0;
        }
        for (;;) {
            bool any = false;
#pragma unroll
            for (int r = 0; r < kRows; r++) any |= e[r] < end[r];
            if (!any) break;
#pragma unroll
            for (int r = 0; r < kRows; r++) {
                if (e[r] < end[r]) {
                    s[r] += entry(e[r], ci[e[r]]);
                    e[r] += G;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kRows; r++) {
            const double t = lanes_sum(s[r], G);
            const int raw = i0 + r * step + slot;
            fin(min(raw, n - 1), t, own[r] && g == 0, pd[r]);
        }
    }
    // hub rows: every thread takes a share of the entries, then one block sum
    for (int k = 0; k < F.nlong; k++) {
        const int i = F.chunks[F.long_first[k]].row;
        double v[1] = {0.0};
        for (int p = rp[i] + (int)threadIdx.x; p < rp[i + 1]; p += kGB) v[0] += entry(p, ci[p]);
        block_sum(v, red);
        if (threadIdx.x == 0) fin(i, v[0], true, pre(i));
    }
}

// Element pass with kRows elements per thread in flight: f(i, ok) for
// i = threadIdx.x + k kGB, i clamped to n - 1 (ok false past n).
template <class F>
__device__ __forceinline__ void elements(int n, F f)
{
    for (int i0 = threadIdx.x; i0 < n; i0 += kRows * kGB) {
#pragma unroll
        for (int u = 0; u < kRows; u++) {
            const int raw = i0 + u * kGB;
            f(min(raw, n - 1), raw < n);
        }
    }
}

// y = b - A x on level F; returns (y, y) and (b, b)
__device__ __forceinline__ void residual(const GroupLevel &F, const double *b, const double *x, double *y,
                                         double (&d)[2], Red &red)
{
    d[0] = d[1] = 0.0;
    sweep(
        F, red, [&](int e, int j) { return F.va[e] * x[j]; }, [&](int i) { return b[i]; },
        [&](int i, double s, bool ok, double bi) {
            const double yi = bi - s;
            if (ok) y[i] = yi;
            d[0] += ok ? yi * yi : 0.0;
            d[1] += ok ? bi * bi : 0.0;
        });
    block_sum(d, red);
}

// rc = P^T (in - A M^-1 in) on the coarse level C; returns (rc, rc).  Levels in the
// nested aggregate order (perm NULL) hold an aggregate's rows, and so its entries,
// contiguously: one sweep over the aggregates.  The finest level keeps the
// caller's numbering: its residual goes to tmp first, then the aggregates gather it.
__device__ __forceinline__ double restrict_residual(const GroupLevel &F, const GroupLevel &C, const Input &in,
                                                    double *tmp, Red &red)
{
    const int G = F.Gr, g = threadIdx.x & (G - 1), slot = threadIdx.x / G, step = kGB / G;
    const int nc = C.n;
    double d[1] = {0.0};
    if (F.perm) {
        sweep(
            F, red, [&](int e, int j) { return F.va[e] * (F.minv[j] * in(j)); }, [&](int i) { return in(i); },
            [&](int i, double s, bool ok, double ii) {
                if (ok) tmp[i] = ii - s;
            });
        __syncthreads();
        for (int c0 = 0; c0 < nc; c0 += kRows * step) {
            int k[kRows], end[kRows];
            double s[kRows];
#pragma unroll
            for (int r = 0; r < kRows; r++) {
                const int raw = c0 + r * step + slot, c = min(raw, nc - 1);
                const int b = F.seg[c], t = F.seg[c + 1];
                k[r] = b + g;
                end[r] = raw < nc ? t : 0;
                s[r] = 0.0;
            }
            for (;;) {
                bool any = false;
#pragma unroll
                for (int r = 0; r < kRows; r++) any |= k[r] < end[r];
                if (!any) break;
#pragma unroll
                for (int r = 0; r < kRows; r++) {
                    const bool ok = k[r] < end[r];
                    const double v = tmp[F.perm[ok ? k[r] : 0]];
                    s[r] += ok ? v : 0.0;
                    k[r] += G;
                }
            }
#pragma unroll
            for (int r = 0; r < kRows; r++) {
                const double t = lanes_sum(s[r], G);
                const int raw = c0 + r * step + slot;
                if (raw < nc && g == 0) C.rc[raw] = t;
                d[0] += raw < nc && g == 0 ? t * t : 0.0;
            }
        }
    } else {
        for (int c0 = 0; c0 < nc; c0 += kRows * step) {
            int k[kRows], kend[kRows], e[kRows], eend[kRows];
            bool own[kRows];  // an aggregate of this lane group (not a hub, which the block sums below)
            double s[kRows];
#pragma unroll
            for (int r = 0; r < kRows; r++) {
                const int raw = c0 + r * step + slot, c = min(raw, nc - 1);
                const int k0 = F.seg[c], k1 = F.seg[c + 1];
                const int e0 = F.srp ? F.srp[c] : F.rp[k0], e1 = F.srp ? F.srp[c + 1] : F.rp[k1];
                own[r] = raw < nc && e1 - e0 <= F.slim;
                k[r] = k0 + g;
                kend[r] = own[r] ? k1 : 0;
                e[r] = e0 + g;
                eend[r] = own[r] ? e1 : 0;
                s[r] = 0.0;
            }
            for (;;) {
                bool any = false;
#pragma unroll
                for (int r = 0; r < kRows; r++) any |= (k[r] < kend[r]) | (e[r] < eend[r]);
                if (!any) break;
#pragma unroll
                for (int r = 0; r < kRows; r++) {
                    const bool okr = k[r] < kend[r], oke = e[r] < eend[r];
                    const double a = in(okr ? k[r] : 0);
                    const int ee = oke ? e[r] : 0;
                    const int j = F.ci[ee];
                    const double v = F.va[ee] * (F.minv[j] * in(j));
                    s[r] += okr ? a : 0.0;
                    s[r] -= oke ? v : 0.0;
                    k[r] += G;
                    e[r] += G;
                }
            }
#pragma unroll
            for (int r = 0; r < kRows; r++) {
                const double t = lanes_sum(s[r], G);
                const int raw = c0 + r * step + slot;
                if (own[r] && g == 0) C.rc[raw] = t;
                d[0] += own[r] && g == 0 ? t * t : 0.0;
            }
        }
        // hub aggregates (more than slim entries): every thread takes a share
        for (int h = 0; h < F.snlong; h++) {
            const int c = F.schunks[F.slong_first[h]].row;
            double v[1] = {0.0};
            for (int q = F.seg[c] + (int)threadIdx.x; q < F.seg[c + 1]; q += kGB) v[0] += in(q);
            for (int p = F.srp[c] + (int)threadIdx.x; p < F.srp[c + 1]; p += kGB) {
                const int j = F.ci[p];
                v[0] -= F.va[p] * (F.minv[j] * in(j));
            }
            block_sum(v, red);
            if (threadIdx.x == 0) {
                C.rc[c] = v[0];
                d[0] += v[0] * v[0];
            }
        }
    }
    block_sum(d, red);
    return d[0];
}

// c1 = A_c^-1 rc on the coarsest level: decoupled unknowns by a division, the
// coupled block by its dense inverse (one wavefront per row)
__device__ __forceinline__ void coarsest(const GroupLevel &C, const CoarseSolve &cs)
{
    for (int k = threadIdx.x; k < cs.nd; k += kGB) {
        const int i = cs.didx[k];
        C.c1[i] = C.rc[i] * cs.dinv[k];
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int i0 = 0; i0 < cs.m; i0 += kGW) {
        const int i = i0 + w;
        double s = 0.0;
        if (i < cs.m) {
            const double *row = cs.ainv + (size_t)i * cs.m;
            for (int j = lane; j < cs.m; j += kWave) s += row[j] * C.rc[cs.idx ? cs.idx[j] : j];
        }
        s = wave_sum(s);
        if (i < cs.m && lane == 0) C.c1[cs.idx ? cs.idx[i] : i] = s;
    }
    __syncthreads();
}

struct PostRow {
    double mi, ri, ei;
};

// out = x + P e + M^-1 (in - A (x + P e)) with x = M^-1 in and e = ca c1 + cb c2 of
// the coarse level C (cb = 0: c1 alone, c2 not read); returns (out, q) when q is given
__device__ __forceinline__ double post_smooth(const GroupLevel &F, const GroupLevel &C, const Input &in, double *out,
                                              double ca, double cb, const double *q, Red &red)
{
    const bool two = cb != 0.0;
    auto corr = [&](int a) { return two ? ca * C.c1[a] + cb * C.c2[a] : ca * C.c1[a]; };
    double d[1] = {0.0};
    auto pre = [&](int i) { return PostRow{F.minv[i], in(i), corr(F.agg[i])}; };
    auto fin = [&](int i, double s, bool ok, const PostRow &w) {
        const double o = (w.mi * w.ri + w.ei) + w.mi * (w.ri - s);
        if (ok) out[i] = o;
        if (q) d[0] += ok ? o * q[i] : 0.0;
    };
    if (F.cagg)
        sweep(F, red, [&](int e, int j) { return F.va[e] * (F.minv[j] * in(j) + corr(F.cagg[e])); }, pre, fin);
    else
        sweep(F, red, [&](int e, int j) { return F.va[e] * (F.minv[j] * in(j) + corr(F.agg[j])); }, pre, fin);
    if (q) {
        block_sum(d, red);
        return d[0];
    }
    __syncthreads();
    return 0.0;
}

struct DotRow {
    double x, u, w;
};

// y = A x on level F with (x, y), (x, u) [, (x, w)]; y may be NULL (products only)
template <int ND>
__device__ __forceinline__ void product_dots(const GroupLevel &F, const double *x, double *y, const double *u,
                                             const double *w, double (&d)[ND], Red &red)
{
#pragma unroll
    for (int k = 0; k < ND; k++) d[k] = 0.0;
    sweep(
        F, red, [&](int e, int j) { return F.va[e] * x[j]; },
        [&](int i) { return DotRow{x[i], u[i], ND > 2 ? w[i] : 0.0}; },
        [&](int i, double s, bool ok, const DotRow &v) {
            if (y && ok) y[i] = s;
            d[0] += ok ? v.x * s : 0.0;
            d[1] += ok ? v.x * v.u : 0.0;
            if constexpr (ND > 2) d[2] += ok ? v.x * v.w : 0.0;
        });
    block_sum(d, red);
}

// z = K_0(r) (Sec. 4.3); with q, returns (z, q) in *zq.  Returns false on a
// breakdown of an inner step ((c, A c) <= 0).  z serves as the finest level's
// scratch for the restriction (it is written only by the last post-smoothing).
__device__ __forceinline__ bool kcycle(const GroupJob &J, const double *r, double *z, const double *q, double *zq,
                                       Red &red)
{
    enum { VISIT, POST, STEP1, STEP2 };
    const int L = J.levels - 1;
    unsigned second = 0;  // bit k: the visit of level k in progress is the second inner step's
    int k = 0, act = VISIT;
    double ca = 1.0, cb = 0.0;  // coefficients of the coarse correction the next POST applies
    auto input = [&](int l) -> Input {
        if (l == 0) return Input{r, nullptr, 0.0};
        const GroupLevel &C = J.lev[l];
        return ((second >> l) & 1u) ? Input{C.rc, C.v1, red.sh.a1[l]} : Input{C.rc, nullptr, 0.0};
    };
    auto output = [&](int l) -> double * { return l == 0 ? z : ((second >> l) & 1u) ? J.lev[l].c2 : J.lev[l].c1; };
    for (;;) {
        if (act == VISIT) {
            const GroupLevel &F = J.lev[k], &C = J.lev[k + 1];
            const double gg = restrict_residual(F, C, input(k), z, red);
            if (k + 1 == L) {
                coarsest(C, J.cs);
                ca = 1.0;
                cb = 0.0;
                act = POST;
            } else {
                if (threadIdx.x == 0) red.sh.gg[k + 1] = gg;  // read after the first step's visit
                k++;
                second &= ~(1u << k);
            }
        } else if (act == POST) {
            const double d =
                post_smooth(J.lev[k], J.lev[k + 1], input(k), output(k), ca, cb, k == 0 ? q : nullptr, red);
            if (k == 0) {
                if (q) *zq = d;
                return true;
            }
            act = ((second >> k) & 1u) ? STEP2 : STEP1;
        } else if (act == STEP1) {  // level k is the coarse level of the visit of k - 1
            const GroupLevel &C = J.lev[k];
            double d[2];
            product_dots<2>(C, C.c1, C.v1, C.rc, nullptr, d, red);  // (c1, A c1), (c1, rc)
            const double rho1 = d[0];
            if (!(rho1 > 0.0)) return false;
            const double alpha1 = d[1] / rho1;
            bool more = J.nu > 1;
            if (more && J.theta > 0.0) {  // ||rt||^2 against theta^2 ||rc||^2
                double t[1] = {0.0};
                elements(C.n, [&](int i, bool ok) {
                    const double v = C.rc[i] - alpha1 * C.v1[i];
                    t[0] += ok ? v * v : 0.0;
                });
                block_sum(t, red);
                if (t[0] < J.theta * J.theta * red.sh.gg[k]) more = false;
            }
            if (more) {
                if (threadIdx.x == 0) {
                    red.sh.a1[k] = alpha1;
                    red.sh.r1[k] = rho1;
                }
                __syncthreads();  // the second visit's input reads alpha1
                second |= 1u << k;
                act = VISIT;
            } else {
                ca = alpha1;
                cb = 0.0;
                k--;
                act = POST;
            }
        } else {  // STEP2
            const GroupLevel &C = J.lev[k];
            double d[3];
            product_dots<3>(C, C.c2, nullptr, C.v1, C.rc, d, red);  // (c2, A c2), (c2, v1), (c2, rc)
            const double rho1 = red.sh.r1[k], alpha1 = red.sh.a1[k];
            const double gam = d[1] / rho1;
            const double rho2 = d[0] - d[1] * gam;
            if (!(rho2 > 0.0)) return false;
            const double alpha2 = (d[2] - alpha1 * d[1]) / rho2;  // (c2, rt) / rho2
            ca = alpha1 - alpha2 * gam;
            cb = alpha2;
            k--;
            act = POST;
        }
    }
}

__global__ void __launch_bounds__(kGB) k_group_solve(const GroupJob *__restrict__ jobs, int kcycle_only,
                                                     GroupResult *__restrict__ res)
{
    __shared__ Shared sh;
    Red red{sh, 0};
    const GroupJob &J = jobs[blockIdx.x];
    const GroupLevel &F = J.lev[0];
    const int n = F.n;
    double *x = J.x, *r = J.r, *z = J.z, *p = J.p, *q = J.q;
    const double *kin = r;
    double *kout = z;
    double d[2];
    double bnorm = 1.0, rel = 0.0;
    int it = 0, status = AMG_ERR_NOT_CONVERGED;
    if (kcycle_only) {  // x = K(b): one K-cycle below, nothing else
        kin = J.b;
        kout = x;
    } else {
        residual(F, J.b, x, r, d, red);  // r = b - A x, (r, r), (b, b)
        const double bb = d[1];
        if (!isfinite(bb) || !isfinite(d[0])) {
            if (threadIdx.x == 0) res[blockIdx.x] = GroupResult{AMG_ERR_INVALID_ARGUMENT, 0, 0.0};
            return;
        }
        if (bb == 0.0) {
            elements(n, [&](int i, bool ok) {
                if (ok) x[i] = 0.0;
            });
            if (threadIdx.x == 0) res[blockIdx.x] = GroupResult{AMG_OK, 0, 0.0};
            return;
        }
        bnorm = sqrt(bb);
        rel = sqrt(d[0]) / bnorm;
        if (rel <= J.tol) status = AMG_OK;
    }
    // pass 0: z = K(r), p = z; pass k > 0: outer step k, then z = K(r), p = z + beta p
    // (one call site of the K-cycle, so that it is inlined)
    bool ok = true;
    for (int pass = 0; status != AMG_OK; pass++) {
        double pq = 1.0;
        if (pass > 0) {
            if (it >= J.max_iters) break;
            double e[2];
            product_dots<2>(F, p, q, r, nullptr, e, red);  // q = A p, (p, q), (p, r)
            pq = e[0];
            if (!(pq > 0.0)) {
                ok = false;
                break;
            }
            const double alpha = e[1] / pq;
            double t[1] = {0.0};
            elements(n, [&](int i, bool in) {
                const double xv = x[i], pv = p[i], rv = r[i], qv = q[i];
                const double w = rv - alpha * qv;
                if (in) {
                    x[i] = xv + alpha * pv;
                    r[i] = w;
                }
                t[0] += in ? w * w : 0.0;
            });
            block_sum(t, red);
            it++;
            rel = sqrt(t[0]) / bnorm;
            if (rel <= J.tol) {  // confirm with the true residual; continue from it if it disagrees
                residual(F, J.b, x, r, d, red);
                rel = sqrt(d[0]) / bnorm;
                if (rel <= J.tol) {
                    status = AMG_OK;
                    break;
                }
            }
        }
        double zq = 0.0;
        ok = kcycle(J, kin, kout, pass > 0 ? q : nullptr, &zq, red);
        if (!ok || kcycle_only) break;
        const double beta = pass > 0 ? -zq / pq : 0.0;
        elements(n, [&](int i, bool in) {
            const double zv = z[i], pv = p[i];
            const double v = pass > 0 ? zv + beta * pv : zv;
            if (in) p[i] = v;
        });
        __syncthreads();
    }
    if (kcycle_only) {
        if (threadIdx.x == 0) res[blockIdx.x] = GroupResult{ok ? AMG_OK : AMG_ERR_BREAKDOWN, 0, 0.0};
        return;
    }
    if (!ok) status = AMG_ERR_BREAKDOWN;
    residual(F, J.b, x, r, d, red);  // the reported residual is the true one
    if (threadIdx.x == 0) res[blockIdx.x] = GroupResult{status, it, sqrt(d[0]) / bnorm};
}

}  // namespace

void launch_group_solve(const GroupJob *jobs, int count, int kcycle_only, GroupResult *res, hipStream_t s)
{
    if (count <= 0) return;
    k_group_solve<<<count, kGB, 0, s>>>(jobs, kcycle_only, res);
    AMG_HIP(hipGetLastError());
}

}  // namespace amg

// amg_internal.h -- internal declarations of libamg (gfx950 only).
//
// Kernels live in setup_kernels.hip, solve_kernels.hip and scan.hip; each file
// exports host-side launch functions declared here.  The host engine
// (engine.hip) owns all orchestration.  Every launch takes the stream it runs on.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <vector>

namespace amg {

constexpr int kWave = 64;    // CDNA wavefront width
constexpr int kBlock = 256;  // threads per block for every kernel below
constexpr int kMaxDotBlocks = 1 << 15;  // grid cap of kernels that write dot partials
constexpr int kMaxDots = 5;

struct Error : std::runtime_error {
    int status;
    Error(int s, const char *what) : std::runtime_error(what), status(s) {}
};

void hip_check(hipError_t e, const char *what);
#define AMG_HIP(call) ::amg::hip_check((call), #call)

// Device reduction workspace shared by the kernels of one solve context: per-block
// partial sums, an arrival counter for the last-block pattern, and an error flag.
// Rows of a CSR-like operator: row r has entries ptr[r] .. ptr[r+1].  Rows with
// more than lim entries ("hub" rows) are cut into chunks of at most kChunk
// entries, each served by one block; long_first[k] .. long_first[k+1] are the
// chunks of hub row k.  chunk_sum / arrive are device workspaces, one set of
// nchunks / nlong per right-hand side of a batch (arrive is zero between launches).
constexpr int kChunk = 1024;
constexpr int kLongBlocks = 1024;  // blocks that serve chunks
constexpr int kMaxLong = 2048;     // hub rows per operator (the threshold is raised beyond)
constexpr int kSmallLevel = 100000;  // levels below this are latency-bound
constexpr int kInlineCoarse = 64;    // coarsest levels up to this size are solved inside the post-smoother
constexpr int kPartStride = kMaxDotBlocks + kMaxLong;
// One right-hand side's block of a dot site: 3 partial sets, then 4 reduced values.
// Column c of a batched solve (blockIdx.y = c) finds its block at c * kDotCol.
constexpr int kDotCol = 3 * kPartStride + 4;
constexpr int kScalCol = 8;  // device scalars per right-hand side

struct Chunk {
    int row, beg, end, k;
};

struct Rows {
    int n;
    const int *ptr;
    int lim;
    int nchunks;
    const Chunk *chunks;
    int nlong;
    const int *long_first;
    double *chunk_sum;
    unsigned *arrive;
    // right-hand sides served by one block in batched sweeps of levels of at least
    // kSmallLevel rows (1: one column per block; 2, 4, 8: each entry loaded once for
    // that many columns)
    int cb;
};
constexpr int kMaxColumnsPerBlock = 8;

// Sliced ELLPACK copy of a level's matrix, for the sweeps of levels of at least
// kSmallLevel rows whose row lengths vary little (a 3D stencil: 4..7 entries).
// Slice s holds rows kWave s .. kWave s + kWave - 1 stored column-major: entry k of
// row i (slice s = i / kWave, lane t = i % kWave) is at ptr[s] + kWave k + t for
// k < w_s = (ptr[s+1] - ptr[s]) / kWave, in the row's CSR order; a row shorter than
// w_s (and every slot of the rows past n in the last slice) is padded with column
// min(i, n - 1) and value 0.  Every slice has w_s >= 1.  One lane serves one row, so
// the entry and value loads of a wavefront are contiguous.  tpb: tiles of kBlock rows
// served by one block (the partial sums of a block's inner products are written once
// per block, so fewer, longer blocks amortise that step).
struct Sell {
    int n = 0, nslices = 0, tpb = 1;
    const int *ptr = nullptr;
    const int *ci = nullptr;
    bool fused = false;  // post-smoothing in one sweep (see k_sell_post_fused)
};
constexpr double kSellMaxPadding = 1.25;  // padded / actual entries beyond which a level keeps CSR only
constexpr int kSellMaxWidth = 64;         // widest slice accepted (entries per row)

// A dot product as a set of partial sums (count 1: already reduced).
struct DotRef {
    const double *part;
    int count;
};
struct DotSet {
    DotRef d[3];
};
// Storage of one dot-product site, per right-hand side: partials (3 * kPartStride)
// and up to 4 reduced values (final_out = part + 3 * kPartStride).
struct DotBuf {
    double *part;
    double *final_out;
};
// The five inner products of one K-cycle coarse correction.
struct KDots {
    DotRef rho1, alpha1, beta, gamma, alpha2;
};

// ---------------------------------------------------------------- scan.hip
// out[i] = sum_{k<i} in[i] (in may alias out); *total_dev = sum of all (device).
// tmp must hold scan_tmp_ints(n) ints.
size_t scan_tmp_ints(int64_t n);
void scan_exclusive(const int *in, int *out, int64_t n, int *total_dev, int *tmp, hipStream_t s);

// ---------------------------------------------------------------- setup_kernels.hip
void launch_validate_csr(int n, int nnz, const int *rp, const int *ci, const double *va, int *err, hipStream_t s);
// the smoother's inverse diagonal: l1-Jacobi for weight <= 0, else damped Jacobi weight / a_ii
void launch_inverse_diagonal(int n, const int *rp, const int *ci, const double *va, double weight, double *minv,
                             hipStream_t s);
void launch_priorities(int n, const int *rp, uint32_t s_l, uint64_t *key, int *owner, hipStream_t s);
// one pass of Alg. 2; rows longer than lim (listed in hubs) are served by whole blocks.
// done_counter: kDoneSlots counters kDoneStride apart (block b adds the vertices it
// processed to slot b % kDoneSlots, so that no single address takes every block's
// atomic); launch_sum_slots writes their total to *out.
constexpr int kDoneSlots = 256;
constexpr int kDoneStride = 32;  // one 128-byte line per slot
void launch_mis_pass(int n, const int *rp, const int *ci, uint64_t *key, uint64_t *m1, int *owner, int cap, int G,
                     unsigned *done_counter, const int *hubs, int nhub, int lim, hipStream_t s);
void launch_sum_slots(const unsigned *slots, unsigned *out, hipStream_t s);
void launch_centre_flags(int n, const int *owner, int *flag, hipStream_t s);
void launch_assign_aggregates(int n, const int *owner, const int *cid, int *agg, int *centre_of, hipStream_t s);
void launch_member_counts(int nc, const int *rp, const int *ci, const int *owner, const int *centre_of, int *size,
                          int *pairs, hipStream_t s);
void launch_member_fill(int nc, const int *rp, const int *ci, const int *owner, const int *centre_of,
                        const int *aptr, int *members, hipStream_t s);
// level skipping: size[J] = sum of |G1_I| over the members I of G2_J; then the member
// lists of the composed aggregates (aptr = exclusive scan of size)
void launch_compose_sizes(int nc2, const int *aptr2, const int *members2, const int *aptr1, int *size, hipStream_t s);
void launch_compose_members(int nc2, const int *aptr2, const int *members2, const int *aptr1, const int *members1,
                            const int *aptr, int *members, hipStream_t s);
void launch_coarse_rows(int nc, const int *rp, const int *ci, const double *va, const int *agg, const int *aptr,
                        const int *members, const int *tptr, int *tcol, double *tval, int *cnt, int *big_rows,
                        unsigned *big_count, hipStream_t s);
int coarse_wave_capacity();
// true when the environment sets AMG_TRACE=1 (stage trace on stderr)
bool trace_on();
// Largest coarse level size whose dense accumulator fits in LDS beside the big-row
// kernel's other shared arrays; rows of such levels need no global scratch.
int coarse_acc_capacity();
void launch_coarse_big_rows_acc(int nbig, const int *big_rows, int nc, const int *rp, const int *ci, const double *va,
                                const int *agg, const int *aptr, const int *members, const int *tptr, int *tcol,
                                double *tval, int *cnt, hipStream_t s);
void launch_coarse_big_rows(int nbig, const int *big_rows, const int64_t *scratch_off, uint64_t *skey,
                            const int *rp, const int *ci, const double *va, const int *agg, const int *aptr,
                            const int *members, const int *tptr, int *tcol, double *tval, int *cnt,
                            hipStream_t s);
void launch_coarse_compact(int nc, const int *tptr, const int *tcol, const double *tval, const int *crp, int *cci,
                           double *cva, double weight, double *cminv, hipStream_t s);
void launch_dense_from_csr(int n, const int *rp, const int *ci, const double *va, double *dense, hipStream_t s);
void launch_cholesky_inverse(int n, double *a, double *inv, int *err, hipStream_t s);
// solve-layout permutation
void launch_identity(int n, int *v, hipStream_t s);
void launch_sizes_in_position_order(int nc, const int *aptr_nat, const int *perm_c, int *size_pos, hipStream_t s);
void launch_positions_from_segments(int nc, const int *aptr_nat, const int *members_nat, const int *pos_c,
                                    const int *seg_ptr, int *pos_f, int *perm_f, hipStream_t s);
void launch_permuted_row_lengths(int n, const int *rp_nat, const int *perm, int *len, hipStream_t s);
void launch_permute_rows(int n, const int *rp_nat, const int *ci_nat, const double *va_nat, const double *minv_nat,
                         const int *perm, const int *pos, const int *rp, int *ci, double *va, double *minv,
                         hipStream_t s);
void launch_agg_positions(int n, const int *perm_f, const int *agg_nat, const int *pos_c, int *agg_pos,
                          hipStream_t s);
void launch_gather_int(int n, const int *src, const int *idx, int *dst, hipStream_t s);
// om_t = sum over rows q holding column t of [q == t] - a_qt minv_t: the restriction
// row vector of a level whose coarse level is one unknown
void launch_single_unknown_weights(int n, const int *rp, const int *ci, const double *va, const double *minv,
                                   double *om, hipStream_t s);
// dinv[k] = 1 / va[pos[k]]
void launch_reciprocals(int m, const int *pos, const double *va, double *dinv, hipStream_t s);
// Rows of ptr longer than lim, ascending.  Call first with list == NULL: flags
// (n ints) receive exclusive offsets and *count_dev the count; then call again with
// the same flags and a list of that many ints.
void launch_long_rows(int n, const int *ptr, int lim, int *flags, int *list, int *count_dev, int *scan_tmp,
                      hipStream_t s);

// Sliced ELLPACK build: width[s] = longest row of slice s (at least 1), for the
// ceil(n / kWave) slices; then, with the entry offsets ptr (nslices + 1), the copy.
void launch_sell_widths(int n, const int *rp, int *width, hipStream_t s);
void launch_sell_fill(int n, int nslices, const int *rp, const int *ci, const double *va, const int *ptr, int *sci,
                      double *sva, hipStream_t s);

// ---------------------------------------------------------------- solve_kernels.hip
int lanes_for(double avg_row_len, int n);
// plain y = A x
void launch_spmv(Rows R, const int *ci, const double *va, const double *x, double *y, int G, hipStream_t s);
// The K-cycle launchers take the storage type T of values and vectors (double, or
// float in the mixed-precision mode); arithmetic and inner products are FP64.
// ncol > 1 runs a batch of right-hand sides in one launch (gridDim.y = column):
// each level's vectors are stored column after column (leading dimension = the
// level's size) and every dot site holds one kDotCol block per column.
// gate (device, one int per column, or NULL): with the K-cycle threshold, the
// launchers of a second inner step and of everything nested in it take that step's
// gate, and their kernels do nothing for a column whose gate is 0.
//
// y = A x (y may be NULL); d[0] = (x, A x), d[1] = (x, w1) if w1, d[2] = (x, w2) if w2
// (omy, non-NULL only with at most two other products, adds (omy, A x) last.)
// With sl (and its values sva), the rows are served from the sliced ELLPACK copy
// (omy must then be NULL).
template <class T>
DotSet launch_spmv_dots(Rows R, const int *ci, const T *va, const T *x, T *y, const T *w1, const T *w2, int G,
                        DotBuf buf, hipStream_t s, const double *omy = nullptr, int ncol = 1,
                        const Sell *sl = nullptr, const T *sva = nullptr, const int *gate = nullptr);
// r = b - A x; d[0] = (b, b), d[1] = (r, r)
DotSet launch_residual(Rows R, const int *ci, const double *va, const double *b, const double *x, double *r, int G,
                       DotBuf buf, hipStream_t s, int ncol = 1, const int *gate = nullptr);
// out[c * out_stride] = value of ref for column c (one block per column)
void launch_reduce(const DotRef &ref, double *out, hipStream_t s, int ncol = 1, int out_stride = kScalCol,
                   const int *gate = nullptr);
// rc = W r over the super-rows S (nf fine rows), W = P^T (I - A M^-1) stored per entry.
// With om, also the partials of (om, rc) into buf (returned; else a null reference).
template <class T>
DotRef launch_restrict(Rows S, int nf, const int *ci, const T *wv, const T *r, T *rc, int G, hipStream_t s,
                       const double *om = nullptr, DotBuf buf = DotBuf{}, int ncol = 1, const int *gate = nullptr);
// rc = P^T (r - A M^-1 r) on a level with a sliced copy S (values sva): the
// pre-smoothing residual t (FP64, n per right-hand side, scratch) row by row, then
// the sums of t over the aggregates: rc[J] = sum of t[idx[p]] (t[p] when idx is
// NULL) for positions p in seg[J] .. seg[J+1] of the level's nested order.
template <class T>
void launch_sell_restrict(const Sell &S, const T *sva, const T *minv, const T *r, double *t, int nc, const int *seg,
                          const int *idx, T *rc, hipStream_t s, int ncol = 1, const int *gate = nullptr);
// rc = W r with r = rt formed on the fly as rt = rcf - (alpha1/rho1) v1 (the
// inner residual of the parent's first flexible-CG step), rt also stored
template <class T>
DotRef launch_restrict_rt(Rows S, int nf, const int *ci, const T *wv, const T *rcf, const T *v1, KDots kd, T *rt,
                          T *rc, int *flag, int G, hipStream_t s, const double *om = nullptr, DotBuf buf = DotBuf{},
                          int ncol = 1, const int *gate = nullptr);
// K-cycle visit of a level whose coarse level is one unknown (restriction by the
// inner products om_r and, with rt_mode, om_v1; see k_post_direct).
template <class T>
void launch_post_direct(Rows R, const int *ci, const T *va, const T *minv, const T *r, const T *v1, KDots kd,
                        DotRef om_r, DotRef om_v1, const double *ainv, T *xout, T *rt_out, int *flag, int G,
                        bool rt_mode, hipStream_t s, int ncol = 1, const int *gate = nullptr);
// A small level whose coarse level is one unknown, laid out for a whole coarse
// correction (two flexible-CG steps, Sec. 4.4) in one block of kTailThreads
// threads per right-hand side.  Thread t owns rows t + u kTailThreads
// (u < kTailRows); the entries of an owned ordinary row (at most kTailWidth) sit
// in that thread's slots u kTailWidth .. u kTailWidth + kTailWidth - 1 in CSR
// order, padded with zero values; the entries of at most kTailLong long rows
// (the hub of the single aggregate has every row of the level as a neighbour)
// fill the slots from kTailRows kTailWidth on: entry j of long row m sits in slot
// kTailRows kTailWidth + long_slot[m] + j / kTailThreads of thread
// j % kTailThreads.  ci[s kTailThreads + t] is slot s of thread t (the values are
// a separate array of the same shape, per storage type); padding slots hold
// column 0 and value 0.
constexpr int kTailThreads = 1024;
constexpr int kTailRows = 5;
constexpr int kTailWidth = 2;
constexpr int kTailLong = 2;
constexpr int kTailLongSlots = 6;
constexpr int kTailSlots = kTailRows * kTailWidth + kTailLongSlots;
struct TailLayout {
    int n;
    int nlong;
    int long_row[kTailLong];       // -1 when unused
    int long_slot[kTailLong + 1];  // long row m: slots long_slot[m] .. long_slot[m+1] (after the row slots)
    const uint16_t *ci;  // column indices (n <= kTailRows kTailThreads < 2^16)
};
// Builds the layout of a CSR level on the host; false when the level does not fit.
bool build_tail_layout(int n, const int *rp, const int *ci, const double *va, std::vector<uint16_t> &tci,
                       std::vector<double> &tva, TailLayout &L);
// Both flexible-CG steps of a K-cycle visit of such a level from its restricted
// residual rc: c1 = K(rc), v1 = A c1, rt = rc - (alpha1/rho1) v1, c2 = K(rt), where K
// is the two-grid visit of k_post_direct (pre-smoothing, restriction by om,
// coarse solve, prolongation, post-smoothing).  Writes c1 and c2 and the five
// products as reduced values: d1[0] = rho1 = (c1, A c1), d1[1] = alpha1 = (c1, rc),
// d2[0] = beta = (c2, A c2), d2[1] = gamma = (c2, v1), d2[2] = alpha2 = (c2, rt).
// theta2 > 0 (the squared K-cycle threshold): when (rt, rt) < theta2 (rc, rc) the
// second step is skipped (c2 = 0, d2 = 0, so the caller's coefficients reduce to
// the first step's).
template <class T>
void launch_tail_visit(const TailLayout &L, const T *va, const T *minv, const double *om, const double *ainv,
                       const T *rc, T *c1, T *c2, double *d1, double *d2, int *flag, hipStream_t s, int ncol = 1,
                       const int *gate = nullptr, double theta2 = 0.0);
// rt = rc - (alpha1/rho1) v1
template <class T>
void launch_inner_residual(int n, const T *rc, const T *v1, KDots kd, T *rt, int *flag, hipStream_t s, int ncol = 1,
                           const int *gate = nullptr);
// The same under the K-cycle threshold (Sec. 4.3): also the partials of (rc, rc),
// (rt, rt) and, with om, (om, rt) (returned; else a null reference), then
// gate_out[c] = 1 when column c's enclosing step runs (gate) and
// (rt, rt) >= theta2 (rc, rc), else 0.
template <class T>
DotRef launch_inner_residual_theta(int n, const T *rc, const T *v1, KDots kd, T *rt, int *flag, const double *om,
                                   DotBuf buf, double theta2, const int *gate, int *gate_out, hipStream_t s,
                                   int ncol = 1);
// post-smoothing with the coarse correction folded in (mode 0: e = edirect;
// 1: e = (alpha1/rho1) c1; 2: e = a1 c1 + a2 c2; 3: e = ainv * edirect, a dense
// coarsest solve of size nc <= kInlineCoarse done in the kernel); returns
// (out, wdot) if wdot.  nc is the coarse level's size (the leading dimension of
// edirect, c1, c2).  xtmp (FP64, n per right-hand side, or NULL): on levels of at
// least kSmallLevel rows the step is then split in two launches through it, the
// second served from the sliced ELLPACK copy sl (values sva) when given.  second
// (mode 2, or NULL): the gate of the second inner step; a column whose gate is 0
// takes the mode 1 correction.
template <class T>
DotRef launch_post_smooth(Rows R, const int *ci, const T *va, const T *minv, const T *r, const int *agg_pos,
                          const int *cagg, int mode, const T *edirect, const T *c1, const T *c2, KDots kd, T *xout,
                          const T *wdot, DotBuf buf, int *flag, int G, hipStream_t s, const double *ainv, int nc,
                          int ncol = 1, double *xtmp = nullptr, const Sell *sl = nullptr, const T *sva = nullptr,
                          const int *gate = nullptr, const int *second = nullptr);
// Exact solve on a coarsest level of n unknowns: rows with no off-diagonal entry (and
// no entry in their column) are decoupled, x_i = r_i / a_ii (dinv[k] = 1 / a_ii for
// row didx[k], k < nd); the other m rows idx[0..m) (ascending; NULL: all rows, m = n)
// are coupled only among themselves and use the dense row-major m x m inverse ainv of
// their block.
struct CoarseSolve {
    int n, m, nd;
    const int *idx;
    const double *ainv;
    const int *didx;
    const double *dinv;
};
template <class T>
void launch_coarse_solve(const CoarseSolve &cs, const T *x, T *y, hipStream_t s, int ncol = 1);
// r32 = r / sqrt(rr[c * kScalCol]) (FP32); z = sqrt(rr[c * kScalCol]) z32 with the
// partials of (z, q)
void launch_to_inner(int n, const double *r, const double *rr, float *r32, hipStream_t s, int ncol = 1);
DotRef launch_from_inner(int n, const float *z32, const double *rr, double *z, const double *q, DotBuf buf,
                         hipStream_t s, int ncol = 1);
void launch_to_float(int64_t n, const double *src, float *dst, hipStream_t s);
// alpha = pr/pq; x += alpha p; r -= alpha q; returns (r, r)
DotRef launch_fcg_update(int n, DotRef pq, DotRef pr, double *x, double *r, const double *p, const double *q,
                         DotBuf buf, int *flag, hipStream_t s, int ncol = 1, const int *gate = nullptr);
// beta = -zq/pq; p = z + beta p (p = z for a column whose restart flag is set)
void launch_fcg_direction(int n, DotRef pq, DotRef zq, const double *z, double *p, int *flag, hipStream_t s,
                          int ncol = 1, const int *gate = nullptr, const int *restart = nullptr);
DotRef launch_dot(int n, const double *a, const double *b, DotBuf buf, hipStream_t s, int ncol = 1);
// dst[i] = src[idx[i]] / dst[idx[i]] = src[i]; ld <= 0 means n
void launch_gather(int n, const double *src, const int *idx, double *dst, hipStream_t s, int ncol = 1,
                   int ld_src = 0, int ld_dst = 0);
void launch_scatter(int n, const double *src, const int *idx, double *dst, hipStream_t s, int ncol = 1,
                    int ld_src = 0, int ld_dst = 0);
// cagg[p] = agg_pos[ci[p]]: coarse unknown of every entry's column
void launch_entry_coarse_column(int nnz, const int *ci, const int *agg_pos, int *cagg, hipStream_t s);
void launch_restriction_weights(int n, const int *rp, const int *ci, const double *va, const double *minv, double *wv,
                                hipStream_t s);

// ---------------------------------------------------------------- generate.hip
// Synthetic grid Laplacians and right-hand sides on the device (bit-identical to
// the host generator): rp must hold n + 1 ints, ci / va grid_nnz entries, scan_tmp
// scan_tmp_ints(n) ints.
int64_t grid_nnz(int d, const int *dims);
void launch_grid_laplacian(int d, const int *dims, double jitter, uint64_t seed, int *rp, int *ci, double *va,
                           int *scan_tmp, hipStream_t s);
// The same without allocating: the scan scratch is a static device array of the
// library (grids of at most kNoAllocMaxRows unknowns; larger ones throw
// AMG_ERR_UNSUPPORTED before any launch).  Asynchronous on s.
constexpr int64_t kNoAllocMaxRows = 134217728;  // 2^27
void launch_grid_laplacian_noalloc(int d, const int *dims, double jitter, uint64_t seed, int *rp, int *ci,
                                   double *va, hipStream_t s);
void launch_uniform_rhs(int64_t n, uint64_t seed, double *out, hipStream_t s);

// Grouped solves (group_solve.hip): one workgroup of kGroupBlock threads runs the
// whole outer flexible CG with its K-cycle for one right-hand side of one hierarchy;
// one launch serves any number of such jobs, on different problems.  Level arrays
// are those of the solve layout (level 0 in the caller's numbering).
constexpr int kGroupBlock = 1024;
constexpr int kGroupMaxLevels = 16;
struct GroupLevel {
    int n, nnz;
    int G;   // lanes per row of the row sweeps (1, 2, 4, 8 or 16)
    int Gr;  // lanes per aggregate of the restriction (all but the coarsest)
    const int *rp, *ci;
    const double *va, *minv;
    const int *agg;   // row -> coarse position (all but the coarsest)
    const int *cagg;  // entry -> coarse position of its column (NULL: agg of the column)
    const int *seg;   // rows of coarse position c: positions seg[c] .. seg[c+1]-1
    const int *srp;   // entries of those rows: srp[c] .. srp[c+1]-1 (NULL: from rp and seg)
    const int *perm;  // position -> row (NULL: the identity)
    // hub rows (more than lim entries) of A, summed by the whole workgroup: hub row k
    // is chunks[long_first[k]].row (the level's Rows lists); the same for the
    // aggregates' entry ranges (srp) of the restriction
    int lim, nlong;
    const int *long_first;
    const Chunk *chunks;
    int slim, snlong;
    const int *slong_first;
    const Chunk *schunks;
    // this job's work vectors (levels >= 1): restricted residual, the two inner
    // preconditioned directions, A c1
    double *rc, *c1, *c2, *v1;
};
struct GroupJob {
    int levels, max_iters, nu;
    double tol, theta;
    const double *b;
    double *x;
    double *r, *z, *p, *q;  // finest-level work vectors of this job
    CoarseSolve cs;
    GroupLevel lev[kGroupMaxLevels];
};
struct GroupResult {
    int status, iterations;
    double rel_residual;
};
// kcycle_only: x = K(b) (one K-cycle application per job) instead of the solve
void launch_group_solve(const GroupJob *jobs, int count, int kcycle_only, GroupResult *res, hipStream_t s);

}  // namespace amg

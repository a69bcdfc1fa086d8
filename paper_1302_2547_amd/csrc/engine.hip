// engine.hip -- host engine of libamg: hierarchy construction (Alg. 1 setup),
// K-cycle and outer flexible CG orchestration (Sec. 4), and the C ABI of amg.h.
//
// Device memory is owned by one pool per hierarchy; a failed setup releases
// everything it allocated.  All work is ordered on one HIP stream; the host
// waits on it only where it needs a value: the per-pass count of processed
// vertices, level sizes, the small levels it lays out itself (the coarsest
// level's split solve, the level above a single coarse unknown), the lane-count
// timings of the first solve, and the outer residual norm.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <tuple>
#include <type_traits>
#include <vector>

#include "amg.h"
#include "amg_internal.h"

namespace amg {

void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) throw Error(AMG_ERR_OUT_OF_MEMORY, what);
    throw Error(AMG_ERR_DEVICE, what);
}

namespace {

using amg::DotBuf;
using amg::Rows;

}  // namespace

// Stage trace on stderr when the environment sets AMG_TRACE=1.
bool trace_on()
{
    static const bool on = [] {
        const char *v = std::getenv("AMG_TRACE");
        return v && v[0] == '1';
    }();
    return on;
}
// Milliseconds since the first call (trace time stamps).
double trace_ms()
{
    static const auto t0 = std::chrono::steady_clock::now();
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}
#define AMG_TRACE_MSG(...)                                                \
    do {                                                                  \
        if (::amg::trace_on()) {                                          \
            std::fprintf(stderr, "[amg %10.3f ms] ", ::amg::trace_ms());  \
            std::fprintf(stderr, __VA_ARGS__);                            \
            std::fputc('\n', stderr);                                     \
            std::fflush(stderr);                                          \
        }                                                                 \
    } while (0)

namespace {

// SplitMix64 (Steele, Lea, Flood 2014): k-th output of the stream seeded with seed.
uint64_t splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (k + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Process-wide cache of device blocks.  hipFree synchronises the device and is
// slow, so blocks a hierarchy releases are kept, per device, for later
// allocations: a request takes the smallest cached block of at least its size
// class and at most 1.5 times it.  The cache holds at most an eighth of the
// device's memory (blocks beyond that go back to the driver); an allocation that
// the driver refuses returns the cached blocks first and tries again;
// amg_release_cached_memory() returns them on request.
class BlockCache {
public:
    static BlockCache &get()
    {
        static BlockCache c;
        return c;
    }
    // Bytes actually reserved for a request: 256 B classes up to 1 MiB, 64 KiB
    // classes up to 64 MiB, 2 MiB classes above.
    static size_t size_class(size_t bytes)
    {
        const size_t q = bytes <= (1u << 20) ? 256 : (bytes <= (64u << 20) ? (64u << 10) : (2u << 20));
        return (bytes + q - 1) / q * q;
    }
    // A block of at least cls bytes; *got receives its size (return it with give).
    void *take(size_t cls, size_t *got)
    {
        int dev = 0;
        AMG_HIP(hipGetDevice(&dev));
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(Key{dev, cls});
            if (it != free_.end() && it->first.dev == dev && it->first.cls <= cls + cls / 2) {
                void *p = it->second;
                *got = it->first.cls;
                cached_ -= it->first.cls;
                free_.erase(it);
                return p;
            }
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            release_all();
            e = hipMalloc(&p, cls);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        *got = cls;
        return p;
    }
    void give(void *p, size_t cls, int dev)
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (cached_ + cls <= cap(dev)) {
                free_.emplace(Key{dev, cls}, p);
                cached_ += cls;
                return;
            }
        }
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(dev);
        (void)hipFree(p);
        (void)hipSetDevice(cur);
    }
    void release_all()
    {
        std::multimap<Key, void *> out;
        {
            std::lock_guard<std::mutex> lk(mu_);
            out.swap(free_);
            cached_ = 0;
        }
        int cur = 0;
        (void)hipGetDevice(&cur);
        for (auto &kv : out) {
            (void)hipSetDevice(kv.first.dev);
            (void)hipFree(kv.second);
        }
        (void)hipSetDevice(cur);
    }

private:
    struct Key {
        int dev;
        size_t cls;
        bool operator<(const Key &o) const { return dev != o.dev ? dev < o.dev : cls < o.cls; }
    };
    // an eighth of the device's memory (caller holds mu_)
    size_t cap(int dev)
    {
        if (cap_ == 0) {
            size_t free_b = 0, total = 0;
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(dev);
            if (hipMemGetInfo(&free_b, &total) != hipSuccess) {
                (void)hipGetLastError();
                total = size_t(16) << 30;
            }
            (void)hipSetDevice(cur);
            cap_ = total / 8;
        }
        return cap_;
    }
    std::mutex mu_;
    std::multimap<Key, void *> free_;
    size_t cached_ = 0, cap_ = 0;
};

// Device allocations of one hierarchy, with an optional byte budget (counted in
// requested bytes).  Blocks go back to the process-wide cache.
struct Pool {
    struct Block {
        void *p;
        size_t bytes, cls;
        int dev;
    };
    size_t used = 0, peak = 0, budget = 0;
    std::vector<Block> blocks;

    template <class T>
    T *alloc(size_t count)
    {
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (budget && used + bytes > budget) throw Error(AMG_ERR_OUT_OF_MEMORY, "mem_budget exceeded");
        size_t got = 0;
        void *p = BlockCache::get().take(BlockCache::size_class(bytes), &got);
        if (!p) throw Error(AMG_ERR_OUT_OF_MEMORY, "hipMalloc");
        int dev = 0;
        AMG_HIP(hipGetDevice(&dev));
        blocks.push_back(Block{p, bytes, got, dev});
        used += bytes;
        peak = std::max(peak, used);
        return static_cast<T *>(p);
    }
    void release(void *p)
    {
        if (!p) return;
        for (size_t k = blocks.size(); k-- > 0;) {
            if (blocks[k].p == p) {
                BlockCache::get().give(p, blocks[k].cls, blocks[k].dev);
                used -= blocks[k].bytes;
                blocks.erase(blocks.begin() + (long)k);
                return;
            }
        }
    }
    void release_all()
    {
        for (auto &b : blocks) BlockCache::get().give(b.p, b.cls, b.dev);
        blocks.clear();
        used = 0;
    }
};

// K-cycle values and work vectors of one level in storage type T (FP64, or FP32 in
// the mixed-precision mode; the FP64 set aliases the level's own arrays).
template <class T>
struct KArrays {
    const T *va = nullptr, *minv = nullptr, *wv = nullptr;
    T *rc = nullptr, *rt = nullptr, *c1 = nullptr, *c2 = nullptr, *v1 = nullptr;
    const T *sva = nullptr;  // values of the sliced ELLPACK copy (NULL: none)
};

struct Level {
    int n = 0, nnz = 0, passes = 0;
    // natural numbering (setup result)
    int *rp_nat = nullptr, *ci_nat = nullptr;
    double *va_nat = nullptr, *minv_nat = nullptr;
    int *agg_nat = nullptr, *aptr_nat = nullptr, *members_nat = nullptr;  // all but the coarsest level
    // solve layout (nested aggregate order)
    int *rp = nullptr, *ci = nullptr;
    double *va = nullptr, *minv = nullptr;
    double *wv = nullptr;                                        // restriction weights P^T (I - A M^-1)
    int *perm = nullptr, *pos = nullptr;                        // position -> natural, natural -> position
    int *agg_pos = nullptr, *seg_ptr = nullptr, *srp = nullptr;  // all but the coarsest level
    int *cagg = nullptr;                                         // coarse unknown of each entry's column
    int *sci = nullptr;  // columns of the super-rows of P^T A (the same array as ci unless level 0 is natural)
    double *xs = nullptr;  // FP64 iterate of the split post-smoothing (levels >= kSmallLevel rows), n per column
    Sell sell{};             // sliced ELLPACK copy of A for the large-level sweeps (ptr NULL: none)
    double *sell_va = nullptr;
    size_t sell_slots = 0;
    const Sell *sl() const { return sell.ptr ? &sell : nullptr; }
    int G = 2, Gs = 2;
    Rows A{}, S{};  // rows of A and super-rows of P^T A, each with its hub-row chunks
    // work vectors and dot sites when this level is the coarse level of a visit
    double *rc = nullptr, *rt = nullptr, *c1 = nullptr, *c2 = nullptr, *v1 = nullptr;
    DotBuf d_c1{}, d_c2{};  // (c1, A c1), (c1, rc) [, (om, A c1)] and (c2, A c2), (c2, v1), (c2, rt)
    // K-cycle threshold: (rc, rc), (rt, rt) [, (om, rt)] of the first inner step and
    // the gate of the second (one int per right-hand side; NULL without threshold)
    DotBuf d_th{};
    int *gate2 = nullptr;
    // Level whose coarse level is a single unknown: the restriction is the row
    // vector om^T, applied as inner products written by the producers of rc / v1.
    double *omega = nullptr;
    DotBuf d_om{};
    DotRef om_rc{}, om_v1{};
    // ... and small enough for the one-block coarse correction (tail.n = 0: not laid out)
    TailLayout tail{};
    double *tail_va = nullptr;
    float *tail_va32 = nullptr;
    KArrays<double> k64{};
    KArrays<float> k32{};
    template <class T>
    const KArrays<T> &karr() const;
};
template <>
inline const KArrays<double> &Level::karr<double>() const
{
    return k64;
}
template <>
inline const KArrays<float> &Level::karr<float>() const
{
    return k32;
}

}  // namespace
}  // namespace amg

using amg::DotBuf;
using amg::DotRef;
using amg::Error;
using amg::KDots;
using amg::Level;
using amg::Rows;

struct amg_hierarchy {
    amg_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    amg::Pool pool;
    std::vector<Level> lev;
    double *ainv = nullptr;  // dense inverse of the coarsest matrix (of its coupled block when split)
    amg::CoarseSolve coarse{};  // the coarsest level's exact solve
    // outer iteration vectors (finest level, solve layout)
    double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    DotBuf d_pq{}, d_rr{}, d_zq{}, d_res{};
    DotRef dr_pq{}, dr_pr{}, dr_rr{}, dr_zq{};
    double *scal = nullptr;  // device scalars read by the host: rr, bb, rr0
    // position -> caller's index of the finest level's solve layout (NULL: the
    // finest level keeps the caller's numbering)
    const int *uperm = nullptr;
    bool mixed = false;       // FP32 K-cycle inside the FP64 outer iteration
    float *r32 = nullptr, *z32 = nullptr;
    KDots kd0{};             // dots of the finest visit's coarse correction (for timing)
    int *flag = nullptr;     // bit 0: Krylov breakdown
    struct Graphs {
        hipGraphExec_t k = nullptr, step = nullptr;
    };
    std::map<int, Graphs> graphs;  // per batch width (an entry without graphs: launch eagerly)
    static constexpr int kMaxGraphDepth = 12;
    // Level visits of one K-cycle application: level k is visited nu^k times (nu
    // inner flexible-CG steps per coarse visit), so a deep hierarchy with nu = 2
    // grows as 2^L.  Solves of hierarchies beyond this budget are refused.
    static constexpr double kMaxKcycleVisits = 65536.0;
    double kcycle_visits() const
    {
        double v = 0.0, w = 1.0;
        for (int k = 0; k + 1 < levels(); k++) {
            v += w;
            w *= opt.kcycle_inner;
        }
        return v;
    }
    double *host = nullptr;  // pinned: readbacks
    int *host_i = nullptr;
    // Per right-hand side of the outer iteration (max_rhs ints each, device and a
    // pinned host copy): active (still iterating), restart (the next direction is
    // the preconditioned residual itself), claim (the recursive residual says
    // converged: form the true one).  Every outer kernel and the K-cycle run only for
    // active columns, so a column's iteration is that of its right-hand side alone.
    int *mask = nullptr, *host_mask = nullptr;
    std::vector<int> mask_sent;  // the masks as last copied to the device
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double setup_ms = 0.0;

    ~amg_hierarchy()
    {
        AMG_TRACE_MSG("free: start");
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto &kv : graphs)
            for (hipGraphExec_t g : {kv.second.k, kv.second.step})
                if (g) (void)hipGraphExecDestroy(g);
        AMG_TRACE_MSG("free: graphs destroyed");
        pool.release_all();
        AMG_TRACE_MSG("free: device memory released");
        if (host) (void)hipHostFree(host);
        if (host_mask) (void)hipHostFree(host_mask);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    int levels() const { return (int)lev.size(); }
    // weight of the damped Jacobi smoother, 0 for l1-Jacobi
    double smoother_weight() const { return opt.smoother == AMG_SMOOTHER_JACOBI ? opt.jacobi_weight : 0.0; }
    void sync() { AMG_HIP(hipStreamSynchronize(stream)); }

    template <class T>
    void to_host(T *dst, const T *src, size_t count)
    {
        AMG_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, stream));
        sync();
    }
    // copy of pageable host memory: complete before the source may go
    template <class T>
    void to_dev(T *dst, const T *src, size_t count)
    {
        AMG_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, stream));
        sync();
    }
    int read_int(const int *dev)
    {
        AMG_HIP(hipMemcpyAsync(host_i, dev, sizeof(int), hipMemcpyDeviceToHost, stream));
        sync();
        return host_i[0];
    }
    void scan(const int *in, int *out, int64_t count, int *total_dev, int *tmp)
    {
        amg::scan_exclusive(in, out, count, total_dev, tmp, stream);
    }

    DotBuf dot_buf()
    {
        // one kDotCol block per right-hand side: partials, then the reduced values
        double *base = pool.alloc<double>((size_t)amg::kDotCol * (size_t)opt.max_rhs);
        return DotBuf{base, base + 3 * (size_t)amg::kPartStride};
    }

    // Rows descriptor of a CSR-like operator: rows longer than lim = 8 G entries
    // are hub rows, cut into chunks of at most kChunk entries (raised if there
    // would be more than kMaxLong hub rows).
    Rows make_rows(int n, const int *ptr, int G, int *flags, int *scan_tmp)
    {
        Rows R{};
        R.n = n;
        R.ptr = ptr;
        R.lim = 8 * G;
        for (;;) {
            amg::launch_long_rows(n, ptr, R.lim, flags, nullptr, flags + n, scan_tmp, stream);
            R.nlong = read_int(flags + n);
            if (R.nlong <= amg::kMaxLong) break;
            R.lim *= 2;
        }
        if (R.nlong == 0) return R;
        int *list = pool.alloc<int>(R.nlong);
        amg::launch_long_rows(n, ptr, R.lim, flags, list, nullptr, scan_tmp, stream);
        std::vector<int> rows(R.nlong), beg(R.nlong), end(R.nlong);
        int *bounds = pool.alloc<int>(2 * (size_t)R.nlong);
        amg::launch_gather_int(R.nlong, ptr, list, bounds, stream);
        amg::launch_gather_int(R.nlong, ptr + 1, list, bounds + R.nlong, stream);
        to_host(rows.data(), list, R.nlong);
        to_host(beg.data(), bounds, R.nlong);
        to_host(end.data(), bounds + R.nlong, R.nlong);
        pool.release(bounds);
        pool.release(list);
        std::vector<amg::Chunk> chunks;
        std::vector<int> first(R.nlong + 1, 0);
        for (int k = 0; k < R.nlong; k++) {
            first[k] = (int)chunks.size();
            for (int b0 = beg[k]; b0 < end[k]; b0 += amg::kChunk)
                chunks.push_back(amg::Chunk{rows[k], b0, std::min(end[k], b0 + amg::kChunk), k});
        }
        first[R.nlong] = (int)chunks.size();
        R.nchunks = (int)chunks.size();
        amg::Chunk *dchunks = pool.alloc<amg::Chunk>(chunks.size());
        int *dfirst = pool.alloc<int>(first.size());
        R.chunk_sum = pool.alloc<double>(chunks.size() * (size_t)opt.max_rhs);  // per right-hand side
        R.arrive = pool.alloc<unsigned>((size_t)R.nlong * opt.max_rhs);
        AMG_HIP(hipMemcpyAsync(dchunks, chunks.data(), sizeof(amg::Chunk) * chunks.size(), hipMemcpyHostToDevice,
                               stream));
        AMG_HIP(hipMemcpyAsync(dfirst, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, stream));
        AMG_HIP(hipMemsetAsync(R.arrive, 0, sizeof(unsigned) * R.nlong * opt.max_rhs, stream));
        sync();
        R.chunks = dchunks;
        R.long_first = dfirst;
        return R;
    }

    void build(const amg_csr &A);
    void finalize_layout();
    void build_sell(int l, const int *rp, const int *ci, const double *va);
    // the inner residual rt = rcf - (alpha1/rho1) v1 of a parent's first step
    template <class T>
    struct RtSource {
        const T *rcf, *v1;
        KDots kd;
    };
    template <class T>
    DotRef kcycle(int k, const T *r, T *x, const T *wdot, const RtSource<T> *rts, int ncol,
                  const int *gate = nullptr);
    void run_kcycle(int ncol);
    void run_step(int ncol);
    void upload_masks();
    void capture_graphs(int ncol);
    // lanes per row of the bandwidth-bound levels, by measurement (once per hierarchy)
    bool tuned = false;
    void autotune(int ncol);
    template <class T>
    void autotune_level(int l, int ncol);
    amg_status solve(int ncol, const double *b_user, int ldb, double *x_user, int ldx, double tol,
                     amg_solve_info *info);
};

void amg_hierarchy::build(const amg_csr &A)
{
    using namespace amg;
    AMG_HIP(hipEventCreate(&ev0));
    AMG_HIP(hipEventCreate(&ev1));
    const size_t nscal = (size_t)amg::kScalCol * (size_t)opt.max_rhs;  // per-column device scalars
    AMG_HIP(hipHostMalloc((void **)&host, (nscal + 64) * sizeof(double), hipHostMallocDefault));
    host_i = reinterpret_cast<int *>(host + nscal + 32);
    AMG_HIP(hipHostMalloc((void **)&host_mask, 3 * (size_t)opt.max_rhs * sizeof(int), hipHostMallocDefault));
    AMG_HIP(hipEventRecord(ev0, stream));

    const int n0 = A.n, nnz0 = A.nnz;
    lev.reserve(opt.max_levels);
    lev.emplace_back();
    {
        Level &L0 = lev[0];
        L0.n = n0;
        L0.nnz = nnz0;
        L0.rp_nat = pool.alloc<int>(n0 + 1);
        L0.ci_nat = pool.alloc<int>(nnz0);
        L0.va_nat = pool.alloc<double>(nnz0);
        L0.minv_nat = pool.alloc<double>(n0);
        AMG_HIP(hipMemcpyAsync(L0.rp_nat, A.row_ptr, sizeof(int) * (n0 + 1), hipMemcpyDeviceToDevice, stream));
        AMG_HIP(hipMemcpyAsync(L0.ci_nat, A.col_idx, sizeof(int) * (size_t)nnz0, hipMemcpyDeviceToDevice, stream));
        AMG_HIP(hipMemcpyAsync(L0.va_nat, A.values, sizeof(double) * (size_t)nnz0, hipMemcpyDeviceToDevice, stream));
    }
    // setup scratch, sized by the finest level and released at the end of setup
    int *ibuf = pool.alloc<int>(16);  // 0 err, 2 big_count, 3 nc, 4 total, 5 nnz_c, 8.. pass counts
    uint64_t *key = pool.alloc<uint64_t>(n0);
    uint64_t *m1 = pool.alloc<uint64_t>(n0);
    int *owner = pool.alloc<int>(n0);
    int *cid = pool.alloc<int>(n0 + 1);
    int *centre_of = pool.alloc<int>(n0);
    int *size = pool.alloc<int>(n0);
    int *pairs = pool.alloc<int>(n0);
    int *cnt = pool.alloc<int>(n0);
    int *tptr = pool.alloc<int>(n0 + 1);
    int *tcol = pool.alloc<int>(nnz0);
    double *tval = pool.alloc<double>(nnz0);
    int *big_rows = pool.alloc<int>(n0);
    int *scan_tmp = pool.alloc<int>(scan_tmp_ints((int64_t)nnz0 + 1));
    unsigned *done = pool.alloc<unsigned>((size_t)kDoneSlots * kDoneStride);  // per-block-group counters
    unsigned *big_count = reinterpret_cast<unsigned *>(ibuf + 2);

    AMG_HIP(hipMemsetAsync(ibuf, 0, 16 * sizeof(int), stream));
    launch_validate_csr(n0, nnz0, lev[0].rp_nat, lev[0].ci_nat, lev[0].va_nat, ibuf, stream);
    if (read_int(ibuf) != 0) throw Error(AMG_ERR_INVALID_MATRIX, "invalid CSR");
    launch_inverse_diagonal(n0, lev[0].rp_nat, lev[0].ci_nat, lev[0].va_nat, smoother_weight(), lev[0].minv_nat,
                            stream);

    const int acc_cap = coarse_acc_capacity();
    // One aggregation of level l (Alg. 2, numbering of Sec. 5.1) and its coarse level
    // (eq. (2.4)), appended to the hierarchy; rand() of eq. (3.2) takes the stream of
    // aggregation number `index`.  Returns false, appending nothing, when the
    // aggregation keeps more than stall_ratio * n_l aggregates.
    auto coarsen = [&](int l, int index) -> bool {
        const int n = lev[l].n, nnz = lev[l].nnz;
        const int G = lanes_for((double)nnz / n, n);
        AMG_TRACE_MSG("level %d: n=%d nnz=%d G=%d aggregation", l, n, nnz, G);
        const uint32_t s_l = (uint32_t)splitmix64(opt.seed, (uint64_t)index);
        launch_priorities(n, lev[l].rp_nat, s_l, key, owner, stream);
        AMG_HIP(hipMemsetAsync(done, 0, sizeof(unsigned) * kDoneSlots * kDoneStride, stream));
        // hub rows (longer than 8 G) of this level, served by whole blocks in the passes
        const int lim = 8 * G;
        launch_long_rows(n, lev[l].rp_nat, lim, tptr, nullptr, tptr + n, scan_tmp, stream);
        const int nhub = read_int(tptr + n);
        if (nhub > 0) launch_long_rows(n, lev[l].rp_nat, lim, tptr, big_rows, nullptr, scan_tmp, stream);
        // Passes are launched kPassBatch at a time and the processed count after each
        // is read back once per batch: a pass over a fully processed level changes
        // nothing, so the passes past the last useful one are no-ops, and the count
        // of useful passes is exact.
        constexpr int kPassBatch = 4;
        unsigned *after = reinterpret_cast<unsigned *>(ibuf + 8);
        unsigned after_h[kPassBatch];
        int passes = 0;
        unsigned processed = 0;
        while (processed < (unsigned)n) {
            for (int b = 0; b < kPassBatch; b++) {
                launch_mis_pass(n, lev[l].rp_nat, lev[l].ci_nat, key, m1, owner, opt.max_aggregate, G, done,
                                big_rows, nhub, lim, stream);
                launch_sum_slots(done, after + b, stream);
            }
            to_host(after_h, after, kPassBatch);
            for (int b = 0; b < kPassBatch && processed < (unsigned)n; b++) {
                passes++;
                if (after_h[b] <= processed || after_h[b] > (unsigned)n)
                    throw Error(AMG_ERR_DEVICE, "aggregation made no progress");
                processed = after_h[b];
            }
        }
        AMG_TRACE_MSG("level %d: %d aggregation passes", l, passes);
        // Sec. 5.1: aggregates numbered by increasing coarse-vertex index
        launch_centre_flags(n, owner, cid, stream);
        scan(cid, cid, n, ibuf + 3, scan_tmp);
        const int nc = read_int(ibuf + 3);
        if ((double)nc > opt.stall_ratio * (double)n) return false;  // coarsening stalled
        Level &F = lev[l];
        F.passes = passes;
        F.agg_nat = pool.alloc<int>(n);
        launch_assign_aggregates(n, owner, cid, F.agg_nat, centre_of, stream);
        launch_member_counts(nc, F.rp_nat, F.ci_nat, owner, centre_of, size, pairs, stream);
        F.aptr_nat = pool.alloc<int>(nc + 1);
        scan(size, F.aptr_nat, nc, F.aptr_nat + nc, scan_tmp);
        F.members_nat = pool.alloc<int>(n);
        launch_member_fill(nc, F.rp_nat, F.ci_nat, owner, centre_of, F.aptr_nat, F.members_nat, stream);
        scan(pairs, tptr, nc, tptr + nc, scan_tmp);
        AMG_HIP(hipMemsetAsync(big_count, 0, sizeof(unsigned), stream));
        launch_coarse_rows(nc, F.rp_nat, F.ci_nat, F.va_nat, F.agg_nat, F.aptr_nat, F.members_nat, tptr, tcol, tval,
                           cnt, big_rows, big_count, stream);
        const int nbig = read_int(reinterpret_cast<int *>(big_count));
        AMG_TRACE_MSG("level %d: passes=%d nc=%d big rows=%d", l, passes, nc, nbig);
        if (nbig > 0 && nc <= acc_cap) {  // dense accumulator in LDS, rows listed on the device
            launch_coarse_big_rows_acc(nbig, big_rows, nc, F.rp_nat, F.ci_nat, F.va_nat, F.agg_nat, F.aptr_nat,
                                       F.members_nat, tptr, tcol, tval, cnt, stream);
        } else if (nbig > 0) {
            std::vector<int> rows(nbig), tp(nc + 1);
            to_host(rows.data(), big_rows, nbig);
            to_host(tp.data(), tptr, nc + 1);
            std::vector<int64_t> off(nbig + 1, 0);
            for (int k = 0; k < nbig; k++) {
                int64_t pc = tp[rows[k] + 1] - tp[rows[k]], P = 1;
                while (P < pc) P <<= 1;
                off[k + 1] = off[k] + P;
            }
            int64_t *off_dev = pool.alloc<int64_t>(nbig + 1);
            int *rows_dev = pool.alloc<int>(nbig);
            // per big row: keys, values by position, values in sorted order, segment heads
            uint64_t *scratch = pool.alloc<uint64_t>(4 * off[nbig] + 1);
            AMG_HIP(hipMemcpyAsync(off_dev, off.data(), sizeof(int64_t) * (nbig + 1), hipMemcpyHostToDevice, stream));
            AMG_HIP(hipMemcpyAsync(rows_dev, rows.data(), sizeof(int) * nbig, hipMemcpyHostToDevice, stream));
            launch_coarse_big_rows(nbig, rows_dev, off_dev, scratch, F.rp_nat, F.ci_nat, F.va_nat, F.agg_nat,
                                   F.aptr_nat, F.members_nat, tptr, tcol, tval, cnt, stream);
            sync();
            pool.release(scratch);
            pool.release(rows_dev);
            pool.release(off_dev);
        }
        Level C;
        C.n = nc;
        C.rp_nat = pool.alloc<int>(nc + 1);
        scan(cnt, C.rp_nat, nc, C.rp_nat + nc, scan_tmp);
        C.nnz = read_int(C.rp_nat + nc);
        C.ci_nat = pool.alloc<int>(C.nnz);
        C.va_nat = pool.alloc<double>(C.nnz);
        C.minv_nat = pool.alloc<double>(nc);
        launch_coarse_compact(nc, tptr, tcol, tval, C.rp_nat, C.ci_nat, C.va_nat, smoother_weight(), C.minv_nat,
                              stream);
        lev.push_back(C);
        return true;
    };
    // Alg. 1: coarsen while n_l > n_0 and fewer than L levels exist (a stalled
    // aggregation leaves level l as the coarsest).  With skip_ratio (Sec. 3.3), a level
    // whose aggregation coarsened by less than the ratio is aggregated a second time,
    // from the coarse level just built, and that intermediate level is dropped: level
    // l keeps the composed aggregates P = P1 P2, and A_{l+1} = P2^T (P1^T A_l P1) P2.
    int l = 0, aggregations = 0;
    while (lev[l].n > opt.coarsest_size && l + 1 < opt.max_levels) {
        if (!coarsen(l, aggregations)) break;
        aggregations++;
        const int n = lev[l].n, nc = lev[l + 1].n;
        if (opt.skip_ratio > 0.0 && (double)n < opt.skip_ratio * (double)nc && nc > opt.coarsest_size &&
            l + 2 < opt.max_levels) {
            if (!coarsen(l + 1, aggregations)) {  // the intermediate level stalls: it is the coarsest
                l++;
                break;
            }
            aggregations++;
            Level &F = lev[l], &M = lev[l + 1];
            const int nc2 = lev[l + 2].n;
            AMG_TRACE_MSG("level %d: coarsening ratio %.2f, aggregated twice (%d -> %d -> %d)", l, (double)n / nc, n,
                          nc, nc2);
            int *agg = pool.alloc<int>(n);
            launch_gather_int(n, M.agg_nat, F.agg_nat, agg, stream);  // agg[i] = agg2[agg1[i]]
            int *aptr = pool.alloc<int>(nc2 + 1);
            launch_compose_sizes(nc2, M.aptr_nat, M.members_nat, F.aptr_nat, size, stream);
            scan(size, aptr, nc2, aptr + nc2, scan_tmp);
            int *members = pool.alloc<int>(n);
            launch_compose_members(nc2, M.aptr_nat, M.members_nat, F.aptr_nat, F.members_nat, aptr, members, stream);
            sync();
            for (void *ptr : std::initializer_list<void *>{F.agg_nat, F.aptr_nat, F.members_nat, M.rp_nat, M.ci_nat,
                                                          M.va_nat, M.minv_nat, M.agg_nat, M.aptr_nat, M.members_nat})
                pool.release(ptr);
            F.agg_nat = agg;
            F.aptr_nat = aptr;
            F.members_nat = members;
            F.passes += M.passes;
            lev.erase(lev.begin() + (l + 1));
        }
        l++;
    }
    sync();
    for (void *ptr : std::initializer_list<void *>{key, m1, owner, cid, centre_of, size, pairs, cnt, tptr, tcol, tval,
                                                  big_rows, scan_tmp, done})
        pool.release(ptr);

    // coarsest level: exact solve.  Unknowns with no off-diagonal entry in their row
    // or column (isolated vertices, which also stall the coarsening of random graphs)
    // are a division each; the dense Cholesky factorisation and explicit inverse are
    // formed for the block of the others only (102 of 2,223 unknowns on the 4M-point
    // random graph).  Levels of at most kInlineCoarse unknowns keep the whole inverse
    // (the post-smoother applies it inline).
    Level &Lc = lev.back();
    AMG_TRACE_MSG("coarsest level %d: n=%d", levels() - 1, Lc.n);
    {
        const int n = Lc.n;
        std::vector<int> crp(n + 1), cci, idx, didx, dpos;
        std::vector<double> cva;
        int m = n;
        if (n > kInlineCoarse) {
            std::vector<int> rp(n + 1), ci(Lc.nnz), cnt(n, 0), pos(n, -1);
            std::vector<double> va(Lc.nnz);
            to_host(rp.data(), Lc.rp_nat, n + 1);
            to_host(ci.data(), Lc.ci_nat, Lc.nnz);
            to_host(va.data(), Lc.va_nat, Lc.nnz);
            for (int e = 0; e < Lc.nnz; e++) cnt[ci[e]]++;
            for (int i = 0; i < n; i++) {
                if (rp[i + 1] - rp[i] == 1 && ci[rp[i]] == i && cnt[i] == 1) {
                    if (!(va[rp[i]] > 0.0)) throw Error(AMG_ERR_BREAKDOWN, "coarsest matrix is not positive definite");
                    didx.push_back(i);
                    dpos.push_back(rp[i]);
                } else {
                    pos[i] = (int)idx.size();
                    idx.push_back(i);
                }
            }
            m = (int)idx.size();
            if (!didx.empty()) {  // the coupled block in CSR, columns renumbered
                crp.assign(m + 1, 0);
                for (int k = 0; k < m; k++) {
                    const int i = idx[k];
                    for (int e = rp[i]; e < rp[i + 1]; e++) {
                        cci.push_back(pos[ci[e]]);
                        cva.push_back(va[e]);
                    }
                    crp[k + 1] = (int)cci.size();
                }
            }
        }
        if (m > opt.max_coarsest) throw Error(AMG_ERR_UNSUPPORTED, "coarsest level larger than max_coarsest");
        coarse = CoarseSolve{n, m, (int)didx.size(), nullptr, nullptr, nullptr, nullptr};
        if (!didx.empty()) {  // decoupled unknowns: x_i = r_i / a_ii
            int *d_didx = pool.alloc<int>(didx.size());
            int *d_dpos = pool.alloc<int>(dpos.size());
            double *d_dinv = pool.alloc<double>(didx.size());
            to_dev(d_didx, didx.data(), didx.size());
            to_dev(d_dpos, dpos.data(), dpos.size());
            launch_reciprocals((int)dpos.size(), d_dpos, Lc.va_nat, d_dinv, stream);
            sync();
            pool.release(d_dpos);
            coarse.didx = d_didx;
            coarse.dinv = d_dinv;
        }
        if (m > 0) {
            const size_t nn = (size_t)m * m;
            double *dense = pool.alloc<double>(nn);
            ainv = pool.alloc<double>(nn);
            AMG_HIP(hipMemsetAsync(dense, 0, nn * sizeof(double), stream));
            AMG_HIP(hipMemsetAsync(ibuf, 0, sizeof(int), stream));
            int *b_rp = nullptr, *b_ci = nullptr;
            double *b_va = nullptr;
            if (m == n) {
                launch_dense_from_csr(n, Lc.rp_nat, Lc.ci_nat, Lc.va_nat, dense, stream);
            } else {
                int *d_idx = pool.alloc<int>(m);
                to_dev(d_idx, idx.data(), m);
                coarse.idx = d_idx;
                b_rp = pool.alloc<int>(m + 1);
                b_ci = pool.alloc<int>(cci.size());
                b_va = pool.alloc<double>(cva.size());
                to_dev(b_rp, crp.data(), m + 1);
                to_dev(b_ci, cci.data(), cci.size());
                to_dev(b_va, cva.data(), cva.size());
                launch_dense_from_csr(m, b_rp, b_ci, b_va, dense, stream);
            }
            launch_cholesky_inverse(m, dense, ainv, ibuf, stream);
            const int err = read_int(ibuf);
            pool.release(dense);
            pool.release(b_rp);
            pool.release(b_ci);
            pool.release(b_va);
            if (err) throw Error(AMG_ERR_BREAKDOWN, "coarsest matrix is not positive definite");
            coarse.ainv = ainv;
        }
        AMG_TRACE_MSG("coarsest solve: %d coupled unknowns, %d decoupled", m, (int)didx.size());
    }
    AMG_TRACE_MSG("coarsest inverse done; solve layout");
    mixed = opt.precision == AMG_PREC_FP32_INNER && levels() >= 2;
    finalize_layout();
    AMG_TRACE_MSG("solve layout done");
    AMG_HIP(hipEventRecord(ev1, stream));
    sync();
    pool.release(ibuf);
    float ms = 0.f;
    AMG_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    setup_ms = ms;
}

// Nested aggregate order, built from the coarsest level down (see setup_kernels.hip).
void amg_hierarchy::finalize_layout()
{
    using namespace amg;
    const int L = levels() - 1;
    const size_t nr = (size_t)opt.max_rhs;  // columns of every work vector
    int *tmp = pool.alloc<int>(lev[0].n + 1);
    int *scan_tmp = pool.alloc<int>(scan_tmp_ints((int64_t)lev[0].nnz + 1));
    lev[L].perm = pool.alloc<int>(lev[L].n);
    lev[L].pos = pool.alloc<int>(lev[L].n);
    launch_identity(lev[L].n, lev[L].perm, stream);
    launch_identity(lev[L].n, lev[L].pos, stream);
    for (int l = L - 1; l >= 0; l--) {
        Level &F = lev[l], &C = lev[l + 1];
        launch_sizes_in_position_order(C.n, F.aptr_nat, C.perm, tmp, stream);
        F.seg_ptr = pool.alloc<int>(C.n + 1);
        scan(tmp, F.seg_ptr, C.n, F.seg_ptr + C.n, scan_tmp);
        F.pos = pool.alloc<int>(F.n);
        F.perm = pool.alloc<int>(F.n);
        launch_positions_from_segments(C.n, F.aptr_nat, F.members_nat, C.pos, F.seg_ptr, F.pos, F.perm, stream);
        F.agg_pos = pool.alloc<int>(F.n);
        launch_agg_positions(F.n, F.perm, F.agg_nat, C.pos, F.agg_pos, stream);
    }
    uperm = lev[0].perm;
    std::vector<void *> drained;
    for (int l = 0; l <= L; l++) {
        Level &F = lev[l];
        launch_permuted_row_lengths(F.n, F.rp_nat, F.perm, tmp, stream);
        F.rp = pool.alloc<int>(F.n + 1);
        scan(tmp, F.rp, F.n, F.rp + F.n, scan_tmp);
        F.ci = pool.alloc<int>(F.nnz);
        F.va = pool.alloc<double>(F.nnz);
        F.minv = pool.alloc<double>(F.n);
        launch_permute_rows(F.n, F.rp_nat, F.ci_nat, F.va_nat, F.minv_nat, F.perm, F.pos, F.rp, F.ci, F.va, F.minv,
                            stream);
        F.G = lanes_for((double)F.nnz / F.n, F.n);
        const bool natural = l == 0 && L >= 1;  // see below
        F.A = make_rows(F.n, natural ? F.rp_nat : F.rp, F.G, tmp, scan_tmp);
        F.A.cb = opt.batch_cols > 0 ? opt.batch_cols : 4;
        AMG_TRACE_MSG("layout level %d: G=%d hub rows=%d chunks=%d", l, F.G, F.A.nlong, F.A.nchunks);
        if (l < L) {
            const int nc = lev[l + 1].n;
            // Levels of at least kSmallLevel rows may also hold a sliced ELLPACK copy
            // (not the level above a single coarse unknown, whose visits take another
            // path); their solve sweeps read only that copy, and their restriction is
            // a row sweep plus sums per aggregate -- unless the coarse level below is
            // the one above a single unknown, which restricts by inner products with
            // the weights W.  Only the levels that restrict through W get the
            // aggregate-grouped super-rows and W.
            const bool single_below = [&] {
                return L >= 2 && lev[L].n == 1 && lev[L - 1].nnz <= (1 << 24);
            }();
            const bool omega_here = single_below && l == L - 1;
            const bool omega_below = single_below && l + 1 == L - 1;
            if (!omega_here) {
                if (natural) build_sell(l, F.rp_nat, F.ci_nat, F.va_nat);
                else build_sell(l, F.rp, F.ci, F.va);
            }
            const bool super_rows = !F.sell.ptr || omega_below;
            F.sci = F.ci;
            if (super_rows) {
                F.srp = pool.alloc<int>(nc + 1);
                launch_gather_int(nc + 1, F.rp, F.seg_ptr, F.srp, stream);
                F.Gs = lanes_for((double)F.nnz / nc, nc);
                F.S = make_rows(nc, F.srp, F.Gs, tmp, scan_tmp);
                F.S.cb = F.A.cb;
                AMG_TRACE_MSG("layout level %d: super-rows Gs=%d hub rows=%d chunks=%d", l, F.Gs, F.S.nlong,
                              F.S.nchunks);
                F.wv = pool.alloc<double>(F.nnz);
                launch_restriction_weights(F.n, F.rp, F.ci, F.va, F.minv, F.wv, stream);
            } else {
                AMG_TRACE_MSG("layout level %d: sliced, no super-row copy", l);
            }
            if (natural) {
                // The finest level keeps the caller's numbering for A (the stencil's
                // neighbours stay in nearby cache lines; the nested order scatters them
                // and the finest sweeps fetched ~3x their bytes).  Only the restriction
                // needs the aggregate-grouped super-rows: their entries keep the nested
                // order built above, with the columns mapped back to natural indices.
                int *sci = nullptr;
                if (super_rows) {
                    sci = pool.alloc<int>(F.nnz);
                    launch_gather_int(F.nnz, F.perm, F.ci, sci, stream);  // sci[e] = perm[ci[e]]
                }
                launch_gather_int(F.n, lev[1].pos, F.agg_nat, F.agg_pos, stream);  // natural row -> coarse position
                // released once the stream has drained (another hierarchy's stream
                // may receive the blocks from the shared cache)
                drained.insert(drained.end(), {F.rp, F.ci, F.va, F.minv});
                F.sci = sci;
                F.rp = F.rp_nat;
                F.ci = F.ci_nat;
                F.va = F.va_nat;
                F.minv = F.minv_nat;
                uperm = nullptr;
                AMG_TRACE_MSG("layout level 0: natural numbering, hub rows=%d", F.A.nlong);
            }
            if (F.n >= kSmallLevel) F.xs = pool.alloc<double>((size_t)F.n * nr);
            if (F.n < kSmallLevel) {
                F.cagg = pool.alloc<int>(F.nnz);
                launch_entry_coarse_column(F.nnz, F.ci, F.agg_pos, F.cagg, stream);
            }
        }
        if (l >= 1) {
            F.rc = pool.alloc<double>((size_t)F.n * nr);
            F.rt = pool.alloc<double>((size_t)F.n * nr);
            F.c1 = pool.alloc<double>((size_t)F.n * nr);
            F.c2 = pool.alloc<double>((size_t)F.n * nr);
            F.v1 = pool.alloc<double>((size_t)F.n * nr);
            F.d_c1 = dot_buf();
            F.d_c2 = dot_buf();
            if (opt.kcycle_threshold > 0.0 && l < L) {
                F.d_th = dot_buf();
                F.gate2 = pool.alloc<int>(nr);
                const std::vector<int> ones(nr, 1);
                to_dev(F.gate2, ones.data(), nr);
            }
        }
    }
    // single coarse unknown below level L-1 (L >= 2): the restriction is the row
    // vector om (launch_single_unknown_weights)
    if (L >= 2 && lev[L].n == 1 && lev[L - 1].nnz <= (1 << 24)) {
        Level &F = lev[L - 1];
        F.omega = pool.alloc<double>(F.n);
        launch_single_unknown_weights(F.n, F.rp, F.ci, F.va, F.minv, F.omega, stream);
        F.d_om = dot_buf();
        // the one-block coarse correction's layout is built on the host from the
        // level's pattern (placement only, no arithmetic)
        std::vector<int> rp(F.n + 1), ci(F.nnz);
        std::vector<double> va(F.nnz);
        to_host(rp.data(), F.rp, F.n + 1);
        to_host(ci.data(), F.ci, F.nnz);
        to_host(va.data(), F.va, F.nnz);
        AMG_TRACE_MSG("level %d: single coarse unknown below, restriction by inner products", L - 1);
        std::vector<uint16_t> tci;
        std::vector<double> tva;
        TailLayout tl{};
        if (opt.kcycle_inner == 2 && build_tail_layout(F.n, rp.data(), ci.data(), va.data(), tci, tva, tl)) {
            uint16_t *dci = pool.alloc<uint16_t>(tci.size());
            to_dev(dci, tci.data(), tci.size());
            F.tail_va = pool.alloc<double>(tva.size());
            to_dev(F.tail_va, tva.data(), tva.size());
            if (mixed) {
                const std::vector<float> t32(tva.begin(), tva.end());
                F.tail_va32 = pool.alloc<float>(t32.size());
                to_dev(F.tail_va32, t32.data(), t32.size());
            }
            tl.ci = dci;
            F.tail = tl;
            AMG_TRACE_MSG("level %d: one-block coarse correction (%d long rows)", L - 1, tl.nlong);
        }
    }
    for (int l = 0; l <= L; l++) {
        Level &F = lev[l];
        F.k64 = KArrays<double>{F.va, F.minv, F.wv, F.rc, F.rt, F.c1, F.c2, F.v1, F.sell_va};
    }
    if (mixed) {  // FP32 copies of the K-cycle values and FP32 work vectors
        auto to_float = [&](const double *src, size_t count) -> const float * {
            if (!src) return nullptr;
            float *dst = pool.alloc<float>(count);
            launch_to_float((int64_t)count, src, dst, stream);
            return dst;
        };
        for (int l = 0; l <= L; l++) {
            Level &F = lev[l];
            KArrays<float> &K = F.k32;
            K.va = to_float(F.va, F.nnz);
            K.minv = to_float(F.minv, F.n);
            K.wv = to_float(F.wv, F.nnz);
            K.sva = to_float(F.sell_va, F.sell_slots);
            if (l >= 1) {
                K.rc = pool.alloc<float>((size_t)F.n * nr);
                K.rt = pool.alloc<float>((size_t)F.n * nr);
                K.c1 = pool.alloc<float>((size_t)F.n * nr);
                K.c2 = pool.alloc<float>((size_t)F.n * nr);
                K.v1 = pool.alloc<float>((size_t)F.n * nr);
            }
        }
        r32 = pool.alloc<float>((size_t)lev[0].n * nr);
        z32 = pool.alloc<float>((size_t)lev[0].n * nr);
    }
    const int n = lev[0].n;
    b = pool.alloc<double>((size_t)n * nr);
    x = pool.alloc<double>((size_t)n * nr);
    r = pool.alloc<double>((size_t)n * nr);
    z = pool.alloc<double>((size_t)n * nr);
    p = pool.alloc<double>((size_t)n * nr);
    q = pool.alloc<double>((size_t)n * nr);
    AMG_HIP(hipMemsetAsync(q, 0, sizeof(double) * n * nr, stream));
    AMG_HIP(hipMemsetAsync(p, 0, sizeof(double) * n * nr, stream));
    d_pq = dot_buf();
    d_rr = dot_buf();
    d_zq = dot_buf();
    d_res = dot_buf();
    scal = pool.alloc<double>((size_t)amg::kScalCol * nr);
    flag = pool.alloc<int>(1);
    AMG_HIP(hipMemsetAsync(flag, 0, sizeof(int), stream));
    mask = pool.alloc<int>(3 * nr);
    sync();
    pool.release(tmp);
    pool.release(scan_tmp);
    for (void *p : drained) pool.release(p);
}

// Sliced ELLPACK copies of the levels of at least kSmallLevel rows (not the last
// fine level of a single coarse unknown, whose visits take another path), kept
// where the padding stays within kSellMaxPadding of the entries and no slice is
// wider than kSellMaxWidth; other levels (irregular graphs) keep CSR only.
void amg_hierarchy::build_sell(int l, const int *rp, const int *ci, const double *va)
{
    using namespace amg;
    {
        Level &F = lev[l];
        if (F.n < kSmallLevel || F.n > (1 << 28)) return;
        const int ns = (F.n + kWave - 1) / kWave;
        int *w = pool.alloc<int>(ns);
        launch_sell_widths(F.n, rp, w, stream);
        std::vector<int> hw(ns), ptr(ns + 1);
        to_host(hw.data(), w, ns);
        pool.release(w);
        int64_t slots = 0;
        int wmax = 0;
        for (int k = 0; k < ns; k++) {
            ptr[k] = (int)std::min<int64_t>(slots, INT32_MAX);
            slots += (int64_t)hw[k] * kWave;
            wmax = std::max(wmax, hw[k]);
        }
        ptr[ns] = (int)std::min<int64_t>(slots, INT32_MAX);
        const size_t bytes = sizeof(int) * (ns + 1) + (sizeof(int) + sizeof(double)) * (size_t)slots;
        const bool fits = !pool.budget || pool.used + bytes <= pool.budget;
        if (wmax > kSellMaxWidth || slots > kSellMaxPadding * F.nnz || slots >= INT32_MAX || !fits) {
            AMG_TRACE_MSG("level %d: CSR only (sliced copy %lld slots, widest %d)", l, (long long)slots, wmax);
            return;
        }
        int *dptr = pool.alloc<int>(ns + 1);
        to_dev(dptr, ptr.data(), ns + 1);
        int *sci = pool.alloc<int>((size_t)slots);
        F.sell_va = pool.alloc<double>((size_t)slots);
        launch_sell_fill(F.n, ns, rp, ci, va, dptr, sci, F.sell_va, stream);
        F.sell = Sell{F.n, ns, 1, dptr, sci, opt.post_fused == 1};
        F.sell_slots = (size_t)slots;
        AMG_TRACE_MSG("level %d: sliced copy, %lld slots for %d entries (widest %d)", l, (long long)slots, F.nnz, wmax);
    }
}

// x = K_k(r) on level k (solve layout): pre-smoothing from zero + restriction,
// coarse correction (exact on the coarsest level, else two flexible-CG steps
// preconditioned by K_{k+1}), prolongation + post-smoothing.  When wdot is given
// the returned reference holds (x, wdot).
template <class T>
DotRef amg_hierarchy::kcycle(int k, const T *rr, T *xx, const T *wdot, const RtSource<T> *rts, int ncol,
                             const int *gate)
{
    using namespace amg;
    const int L = levels() - 1;
    Level &F = lev[k];
    const KArrays<T> &FK = F.karr<T>();
    if (k == L) {  // single-level hierarchy (FP64 only): the exact solve is the preconditioner
        launch_coarse_solve<T>(coarse, rr, xx, stream, ncol);
        if constexpr (std::is_same<T, double>::value) {
            if (wdot) return launch_dot(F.n, xx, wdot, d_zq, stream, ncol);
        }
        return DotRef{nullptr, 0};
    }
    if (F.omega) {  // the coarse level is one unknown: restriction by inner products
        // (rts: rr = rt is formed from the parent's first inner step and stored)
        if (rts) {
            launch_post_direct<T>(F.A, F.ci, FK.va, FK.minv, rts->rcf, rts->v1, rts->kd, F.om_rc, F.om_v1, ainv, xx,
                                  const_cast<T *>(rr), flag, F.G, true, stream, ncol, gate);
        } else {
            launch_post_direct<T>(F.A, F.ci, FK.va, FK.minv, rr, nullptr, KDots{}, F.om_rc, DotRef{}, ainv, xx,
                                  nullptr, flag, F.G, false, stream, ncol, gate);
        }
        return DotRef{nullptr, 0};
    }
    Level &C = lev[k + 1];
    const KArrays<T> &CK = C.karr<T>();
    // K-cycle threshold (Sec. 4.3): the second inner step on C runs for a column
    // only while ||rt|| >= theta ||rc||, decided on the device (the launches stay
    // the same, so the cycle is still one static graph)
    const double theta = opt.kcycle_threshold;
    // C small with a single unknown below: the whole coarse correction in one block,
    // which forms (om, rc) itself
    const bool tail = C.tail.n > 0;
    const double *om = tail ? nullptr : C.omega;
    if (rts) {  // rr = rt is formed here from the parent's first inner step (never with a threshold)
        C.om_rc = launch_restrict_rt<T>(F.S, F.n, F.sci, FK.wv, rts->rcf, rts->v1, rts->kd, const_cast<T *>(rr),
                                        CK.rc, flag, F.Gs, stream, om, C.d_om, ncol, gate);
    } else if (F.sell.ptr && !om) {  // sliced level: row sweep, then sums per aggregate
        const int *idx = k == 0 && !uperm ? F.perm : nullptr;  // the finest level's rows are in natural order
        launch_sell_restrict<T>(F.sell, FK.sva, FK.minv, rr, F.xs, C.n, F.seg_ptr, idx, CK.rc, stream, ncol, gate);
        C.om_rc = DotRef{nullptr, 0};
    } else {
        C.om_rc = launch_restrict<T>(F.S, F.n, F.sci, FK.wv, rr, CK.rc, F.Gs, stream, om, C.d_om, ncol, gate);
    }
    KDots kd{};
    int mode;
    const T *edirect = nullptr;
    const int *second = nullptr;  // gate of the second inner step (threshold only)
    if (tail) {
        const T *tva;
        if constexpr (std::is_same<T, double>::value) tva = C.tail_va;
        else tva = C.tail_va32;
        double *d1 = C.d_c1.final_out, *d2 = C.d_c2.final_out;
        launch_tail_visit<T>(C.tail, tva, CK.minv, C.omega, ainv, CK.rc, CK.c1, CK.c2, d1, d2, flag, stream, ncol,
                             gate, theta * theta);
        kd = KDots{DotRef{d1, 1}, DotRef{d1 + 1, 1}, DotRef{d2, 1}, DotRef{d2 + 1, 1}, DotRef{d2 + 2, 1}};
        mode = 2;
    } else if (k + 1 == L) {
        if (C.n <= kInlineCoarse) {
            mode = 3;
            edirect = CK.rc;
        } else {
            launch_coarse_solve<T>(coarse, CK.rc, CK.c1, stream, ncol);
            mode = 0;
            edirect = CK.c1;
        }
    } else {
        kcycle<T>(k + 1, CK.rc, CK.c1, nullptr, nullptr, ncol, gate);
        const DotSet s1 = launch_spmv_dots<T>(C.A, C.ci, CK.va, CK.c1, CK.v1, CK.rc, nullptr, C.G, C.d_c1, stream,
                                              C.omega, ncol, C.sl(), CK.sva, gate);
        kd.rho1 = s1.d[0];
        kd.alpha1 = s1.d[1];
        if (C.omega) C.om_v1 = s1.d[2];
        mode = 1;
        if (opt.kcycle_inner == 2 && theta > 0.0) {
            // rt with the test's products, then the gate of the second step, under
            // which that step and everything nested in it run
            const DotRef om_rt = launch_inner_residual_theta<T>(C.n, CK.rc, CK.v1, kd, CK.rt, flag, C.omega, C.d_th,
                                                                theta * theta, gate, C.gate2, stream, ncol);
            if (C.omega) C.om_rc = om_rt;  // the restriction of rt for C's visit
            kcycle<T>(k + 1, CK.rt, CK.c2, nullptr, nullptr, ncol, C.gate2);
            const DotSet s2 = launch_spmv_dots<T>(C.A, C.ci, CK.va, CK.c2, nullptr, CK.v1, CK.rt, C.G, C.d_c2,
                                                  stream, nullptr, ncol, C.sl(), CK.sva, C.gate2);
            kd.beta = s2.d[0];
            kd.gamma = s2.d[1];
            kd.alpha2 = s2.d[2];
            mode = 2;
            second = C.gate2;
        } else if (opt.kcycle_inner == 2) {
            if (C.n < kSmallLevel || C.omega) {  // fold the inner residual into the next restriction
                const RtSource<T> src{CK.rc, CK.v1, kd};
                kcycle<T>(k + 1, CK.rt, CK.c2, nullptr, &src, ncol, gate);
            } else {
                launch_inner_residual<T>(C.n, CK.rc, CK.v1, kd, CK.rt, flag, stream, ncol, gate);
                kcycle<T>(k + 1, CK.rt, CK.c2, nullptr, nullptr, ncol, gate);
            }
            const DotSet s2 = launch_spmv_dots<T>(C.A, C.ci, CK.va, CK.c2, nullptr, CK.v1, CK.rt, C.G, C.d_c2,
                                                  stream, nullptr, ncol, C.sl(), CK.sva, gate);
            kd.beta = s2.d[0];
            kd.gamma = s2.d[1];
            kd.alpha2 = s2.d[2];
            mode = 2;
        }
    }
    if (k == 0) kd0 = kd;
    return launch_post_smooth<T>(F.A, F.ci, FK.va, FK.minv, rr, F.agg_pos, F.cagg, mode, edirect, CK.c1, CK.c2, kd, xx,
                                 wdot, k == 0 ? d_zq : DotBuf{}, flag, F.G, stream, ainv, C.n, ncol, F.xs, F.sl(),
                                 FK.sva, gate, second);
}

// One outer iteration is split in two replayable pieces, both run for the active
// right-hand sides only (mask[0 .. max_rhs)):
//   K    : z = B r, with (z, A p) for the direction update
//   step : p = z (restart) or p = z + beta p; q = A p, (p, q), (p, r);
//          x += alpha p, r -= alpha q; (r, r)
void amg_hierarchy::run_kcycle(int ncol)
{
    using namespace amg;
    const auto g = graphs.find(ncol);
    // one right-hand side is always active while it iterates: no gate (its load
    // would open every kernel of the cycle)
    const int *active = ncol > 1 ? mask : nullptr;
    if (g != graphs.end() && g->second.k) {
        AMG_HIP(hipGraphLaunch(g->second.k, stream));
    } else if (mixed) {  // scal[c * kScalCol] holds (r, r) of column c
        const int n = lev[0].n;
        launch_to_inner(n, r, scal, r32, stream, ncol);
        kcycle<float>(0, r32, z32, nullptr, nullptr, ncol, active);
        dr_zq = launch_from_inner(n, z32, scal, z, q, d_zq, stream, ncol);
    } else {
        dr_zq = kcycle<double>(0, r, z, q, nullptr, ncol, active);
    }
}

void amg_hierarchy::run_step(int ncol)
{
    using namespace amg;
    const auto g = graphs.find(ncol);
    if (g != graphs.end() && g->second.step) {
        AMG_HIP(hipGraphLaunch(g->second.step, stream));
        return;
    }
    Level &F = lev[0];
    const int *active = ncol > 1 ? mask : nullptr, *restart = mask + opt.max_rhs;
    // before the first step dr_pq is unset; every column restarts then and reads no products
    launch_fcg_direction(F.n, dr_pq, dr_zq, z, p, flag, stream, ncol, active, restart);
    const DotSet s1 = launch_spmv_dots<double>(F.A, F.ci, F.va, p, q, r, nullptr, F.G, d_pq, stream, nullptr, ncol,
                                               F.sl(), F.k64.sva, active);
    dr_pq = s1.d[0];
    dr_pr = s1.d[1];
    dr_rr = launch_fcg_update(F.n, dr_pq, dr_pr, x, r, p, q, d_rr, flag, stream, ncol, active);
    launch_reduce(dr_rr, scal, stream, ncol, kScalCol, active);
}

void amg_hierarchy::upload_masks()
{
    // only when they changed since the last upload (a copy per outer iteration would
    // cost as much as a small kernel)
    const size_t count = 3 * (size_t)opt.max_rhs;
    if (mask_sent.size() == count && std::equal(mask_sent.begin(), mask_sent.end(), host_mask)) return;
    mask_sent.assign(host_mask, host_mask + count);
    AMG_HIP(hipMemcpyAsync(mask, host_mask, count * sizeof(int), hipMemcpyHostToDevice, stream));
}

// Records the three pieces once per hierarchy and batch width; every launch
// argument (buffers, partial-set sizes) is fixed by the level sizes, so the graphs
// stay valid.
// ---------------------------------------------------------------- lane-count autotuner
// On levels of at least kSmallLevel rows (bandwidth-bound) the lanes per row of A (G,
// used by the SpMVs and smoothers) and of the super-rows (Gs, used by the restriction),
// or on a level with a sliced copy the row tiles per block of its sweeps (tpb), are
// chosen by measurement: each candidate launch of the post-smoother and of the
// restriction is timed with HIP events on the hierarchy's stream (one warm-up launch,
// then kTuneReps), and the fastest wins.  The rows table does not depend on the choice
// (rows beyond its hub threshold are served by chunks whatever G is).  Choices are cached
// for the process by (level rows, entries, right-hand sides, storage type, operator), so
// later hierarchies of the same shape skip the measurement.
namespace {
constexpr int kTuneReps = 3;
struct TuneCache {
    std::mutex mu;
    std::map<std::tuple<int, int, int, int, int>, int> best;
    static TuneCache &get()
    {
        static TuneCache c;
        return c;
    }
};
}  // namespace

template <class T>
void amg_hierarchy::autotune_level(int l, int ncol)
{
    using namespace amg;
    Level &F = lev[l], &C = lev[l + 1];
    const KArrays<T> &FK = F.karr<T>();
    const KArrays<T> &CK = C.karr<T>();
    // vectors of this level: the work vectors of a coarse level, the outer ones on level 0
    const T *rv;
    T *out;
    if (l == 0) {
        if constexpr (std::is_same<T, float>::value) {
            rv = r32;
            out = z32;
        } else {
            rv = r;
            out = z;
        }
    } else {
        rv = FK.rt;
        out = FK.v1;
    }
    struct Events {  // the solve's own events time the solve
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    AMG_HIP(hipEventCreate(&ev.a));
    AMG_HIP(hipEventCreate(&ev.b));
    auto timed = [&](auto &&launch) {
        launch();
        AMG_HIP(hipEventRecord(ev.a, stream));
        for (int k = 0; k < kTuneReps; k++) launch();
        AMG_HIP(hipEventRecord(ev.b, stream));
        AMG_HIP(hipEventSynchronize(ev.b));
        float ms = 0.f;
        AMG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        return ms;
    };
    auto pick = [&](int kind, double avg_len, int current, auto &&launch_with) {
        const auto key = std::make_tuple(F.n, F.nnz, ncol, (int)sizeof(T), kind);
        {
            TuneCache &c = TuneCache::get();
            std::lock_guard<std::mutex> lk(c.mu);
            const auto it = c.best.find(key);
            if (it != c.best.end()) return it->second;
        }
        int best = current;
        float best_ms = 0.f;
        for (int g = 2; g <= 32; g *= 2) {
            if (g > 2 * avg_len + 2 && g != current) continue;  // most lanes would idle
            const float ms = timed([&] { launch_with(g); });
            if (best_ms == 0.f || ms < best_ms) {
                best_ms = ms;
                best = g;
            }
        }
        TuneCache &c = TuneCache::get();
        std::lock_guard<std::mutex> lk(c.mu);
        c.best[key] = best;
        return best;
    };
    if (F.sell.ptr) {
        // sliced copy: tiles per block (candidates g = 2..16 give g / 2 = 1..8) of the
        // post-smoother with its inner product; the partials go to a dot site that
        // the solve rewrites before reading it.  The restriction reads the same copy.
        Sell &S = F.sell;
        const DotBuf scratch = l == 0 ? d_zq : F.d_c1;
        const double max_candidate = 8.0;  // pick() skips g > 2 * 8 + 2
        const bool fused = S.fused;
        S.fused = false;
        S.tpb = pick(2, max_candidate, 2 * S.tpb, [&](int g) {
            S.tpb = g / 2;
            launch_post_smooth<T>(F.A, F.ci, FK.va, FK.minv, rv, F.agg_pos, F.cagg, 0, CK.c1, nullptr, nullptr,
                                  KDots{}, out, rv, scratch, flag, F.G, stream, ainv, C.n, ncol, F.xs, &S, FK.sva);
        }) / 2;
        S.fused = fused;
        if (opt.post_fused < 0) {
            // then one sweep (candidate 4) against two launches (2), as the K-cycle runs
            // the step: both coarse directions (the coefficients are read from a reduced
            // dot site whose values do not matter here)
            const DotRef any{scratch.final_out, 1};
            const KDots kd{any, any, any, any, any};
            S.fused = pick(3, 1.0, 2, [&](int g) {
                S.fused = g == 4;
                launch_post_smooth<T>(F.A, F.ci, FK.va, FK.minv, rv, F.agg_pos, F.cagg, 2, nullptr, CK.c1, CK.c2, kd,
                                      out, rv, scratch, flag, F.G, stream, ainv, C.n, ncol, F.xs, &S, FK.sva);
            }) == 4;
        }
    } else {
        // post-smoother with a directly given correction (no inner products read or written)
        F.G = pick(0, (double)F.nnz / F.n, F.G, [&](int g) {
            launch_post_smooth<T>(F.A, F.ci, FK.va, FK.minv, rv, F.agg_pos, F.cagg, 0, CK.c1, nullptr, nullptr,
                                  KDots{}, out, nullptr, DotBuf{}, flag, g, stream, ainv, C.n, ncol, F.xs);
        });
        F.Gs = pick(1, (double)F.nnz / C.n, F.Gs, [&](int g) {
            launch_restrict<T>(F.S, F.n, F.sci, FK.wv, rv, CK.rc, g, stream, nullptr, DotBuf{}, ncol);
        });
        if (ncol > 1 && opt.batch_cols == 0) {
            // columns per block of the batched sweeps (candidates g = 2..16 give g / 2 =
            // 1..8): the post-smoother and the restriction, each reading the matrix once
            // per group of columns
            const int cb = pick(4, 8.0, 2 * F.A.cb, [&](int g) {
                F.A.cb = F.S.cb = g / 2;
                launch_post_smooth<T>(F.A, F.ci, FK.va, FK.minv, rv, F.agg_pos, F.cagg, 0, CK.c1, nullptr, nullptr,
                                      KDots{}, out, nullptr, DotBuf{}, flag, F.G, stream, ainv, C.n, ncol, F.xs);
                launch_restrict<T>(F.S, F.n, F.sci, FK.wv, rv, CK.rc, F.Gs, stream, nullptr, DotBuf{}, ncol);
            }) / 2;
            F.A.cb = F.S.cb = cb;
        }
    }
    AMG_TRACE_MSG("autotune level %d (%d right-hand sides): G=%d Gs=%d tiles per block=%d post-smoothing in %s, "
                  "%d columns per block", l, ncol, F.G, F.Gs, F.sell.tpb, F.sell.fused ? "one sweep" : "two launches",
                  F.A.cb);
}

void amg_hierarchy::autotune(int ncol)
{
    if (tuned || !opt.autotune) return;
    tuned = true;
    for (int l = 0; l + 1 < levels(); l++) {
        if (lev[l].n < amg::kSmallLevel || lev[l].omega) continue;
        if (mixed) autotune_level<float>(l, ncol);
        else autotune_level<double>(l, ncol);
    }
}

void amg_hierarchy::capture_graphs(int ncol)
{
    // The K-cycle visits level k 2^k times, so its graph has about 6 (2^L - 1)
    // nodes; deep hierarchies (small aggregates) are launched eagerly instead.
    if (!opt.use_graph || graphs.count(ncol)) return;
    Graphs &G = graphs[ncol];
    const int L = levels() - 1;
    if (L > kMaxGraphDepth) return;
    // out NULL: record the body's launches and drop them (nothing runs)
    auto capture = [&](auto &&body, hipGraphExec_t *out) {
        hipGraph_t g = nullptr;
        AMG_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            (void)hipStreamEndCapture(stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        AMG_HIP(hipStreamEndCapture(stream, &g));
        const hipError_t e = out ? hipGraphInstantiate(out, g, nullptr, nullptr, 0) : hipSuccess;
        (void)hipGraphDestroy(g);
        AMG_HIP(e);
    };
    hipGraphExec_t gk = nullptr, gs = nullptr;
    AMG_TRACE_MSG("capturing K-cycle graph (%d right-hand sides)", ncol);
    capture([&] { run_kcycle(ncol); }, &gk);
    AMG_TRACE_MSG("capturing outer-iteration graph");
    // the step's direction update reads the products of the previous step, whose
    // partial-sum set its own launch of A p fixes: a first capture (never launched)
    // records that set, the second uses it
    capture([&] { run_step(ncol); }, nullptr);
    capture([&] { run_step(ncol); }, &gs);
    AMG_TRACE_MSG("graphs ready");
    G.k = gk;
    G.step = gs;
}

// Outer flexible CG over ncol right-hand sides at once (column c of b_user at
// b_user + c * ldb).  Each column stops being counted when its recursive and its
// true relative residual are <= tol; it keeps iterating with the others (a zero
// residual gives a zero correction), and any confirmation restarts every column
// from its true residual.
amg_status amg_hierarchy::solve(int ncol, const double *b_user, int ldb, double *x_user, int ldx, double tol,
                                amg_solve_info *info)
{
    using namespace amg;
    Level &F = lev[0];
    const int n = F.n;
    AMG_TRACE_MSG("solve: start (%d right-hand sides)", ncol);
    AMG_HIP(hipEventRecord(ev0, stream));
    autotune(ncol);
    capture_graphs(ncol);
    AMG_HIP(hipMemsetAsync(flag, 0, sizeof(int), stream));
    launch_gather(n, b_user, uperm, b, stream, ncol, ldb, n);
    launch_gather(n, x_user, uperm, x, stream, ncol, ldx, n);
    const int nr = opt.max_rhs;
    int *active = host_mask, *restart = host_mask + nr, *claim = host_mask + 2 * nr;
    // r = b - A x for the columns of `gate` (NULL: all); per column (b, b), (r, r) at
    // scal[c * kScalCol + 1, + 2]
    auto true_residual = [&](const int *gate) {
        const DotSet s0 = launch_residual(F.A, F.ci, F.va, b, x, r, F.G, d_res, stream, ncol, gate);
        launch_reduce(s0.d[0], scal + 1, stream, ncol, kScalCol, gate);
        launch_reduce(s0.d[1], scal + 2, stream, ncol, kScalCol, gate);
        // the mixed K-cycle scales r by sqrt(scal[c * kScalCol])
        if (mixed) launch_reduce(s0.d[1], scal, stream, ncol, kScalCol, gate);
        AMG_HIP(hipMemcpyAsync(host, scal, sizeof(double) * kScalCol * ncol, hipMemcpyDeviceToHost, stream));
        sync();
    };
    std::vector<double> bnorm(ncol), rel(ncol);
    std::vector<int> iters(ncol, 0);
    std::vector<char> done(ncol, 0);
    true_residual(nullptr);
    for (int c = 0; c < nr; c++) active[c] = restart[c] = claim[c] = 0;
    for (int c = 0; c < ncol; c++) {
        const double bb = host[c * kScalCol + 1], rr = host[c * kScalCol + 2];
        if (!std::isfinite(bb) || !std::isfinite(rr)) return AMG_ERR_INVALID_ARGUMENT;
        bnorm[c] = std::sqrt(bb);
        rel[c] = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        done[c] = bb == 0.0 || rel[c] <= tol;
        active[c] = !done[c];
        restart[c] = 1;
    }
    auto all_done = [&]() {
        for (int c = 0; c < ncol; c++)
            if (!done[c]) return false;
        return true;
    };
    // Each column iterates on its own: it stops when its recursive and then its true
    // relative residual are <= tol, and a true residual that does not confirm
    // restarts that column alone; the others are not touched.  So every column goes
    // through the iterates of its right-hand side solved alone.
    int it = 0;
    amg_status st = AMG_ERR_NOT_CONVERGED;
    while (!all_done() && it < opt.max_iters) {
        upload_masks();
        run_kcycle(ncol);  // z = B r
        run_step(ncol);
        AMG_HIP(hipMemcpyAsync(host, scal, sizeof(double) * kScalCol * ncol, hipMemcpyDeviceToHost, stream));
        AMG_HIP(hipMemcpyAsync(host_i, flag, sizeof(int), hipMemcpyDeviceToHost, stream));
        sync();
        it++;
        if (host_i[0]) {
            st = AMG_ERR_BREAKDOWN;
            break;
        }
        bool any = false;
        for (int c = 0; c < ncol; c++) {
            restart[c] = 0;
            claim[c] = active[c] && std::sqrt(host[c * kScalCol]) / bnorm[c] <= tol;
            any = any || claim[c];
        }
        if (any) {  // confirm with the true residual of the claiming columns
            upload_masks();
            true_residual(mask + 2 * nr);
            for (int c = 0; c < ncol; c++) {
                if (!claim[c]) continue;
                if (std::sqrt(host[c * kScalCol + 2]) / bnorm[c] <= tol) {
                    done[c] = 1;
                    active[c] = 0;
                    iters[c] = it;
                } else {
                    restart[c] = 1;  // continue from the true residual
                }
                claim[c] = 0;
            }
        }
    }
    if (st != AMG_ERR_BREAKDOWN) st = all_done() ? AMG_OK : AMG_ERR_NOT_CONVERGED;
    launch_scatter(n, x, uperm, x_user, stream, ncol, n, ldx);
    for (int c = 0; c < ncol; c++)  // b = 0 has the solution 0
        if (bnorm[c] == 0.0) AMG_HIP(hipMemsetAsync(x_user + (size_t)c * ldx, 0, sizeof(double) * n, stream));
    true_residual(nullptr);  // the reported residual is always the true one
    for (int c = 0; c < ncol; c++) {
        const double bb = host[c * kScalCol + 1];
        rel[c] = bb > 0.0 ? std::sqrt(host[c * kScalCol + 2] / bb) : 0.0;
        if (!done[c]) iters[c] = it;
    }
    AMG_HIP(hipEventRecord(ev1, stream));
    sync();
    AMG_TRACE_MSG("solve: done after %d iterations", it);
    float ms = 0.f;
    AMG_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    if (info) {
        for (int c = 0; c < ncol; c++) {
            info[c].iterations = iters[c];
            info[c].rel_residual = rel[c];
            info[c].setup_ms = setup_ms;
            info[c].solve_ms = ms;
        }
    }
    return st;
}

// ====================================================================== C ABI

namespace {

// The ABI takes device arrays.  Memory the GPU cannot address (pageable host
// memory) is rejected here, with AMG_ERR_INVALID_ARGUMENT, instead of faulting
// inside a kernel; device, managed and pinned host memory pass.
bool device_array(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged ||
           (a.type == hipMemoryTypeHost && a.devicePointer != nullptr);
}

template <class F>
amg_status guarded(F &&f)
{
    try {
        return f();
    } catch (const Error &e) {
        return (amg_status)e.status;
    } catch (const std::bad_alloc &) {
        return AMG_ERR_OUT_OF_MEMORY;
    } catch (...) {
        return AMG_ERR_DEVICE;
    }
}

}  // namespace

extern "C" {

void amg_default_options(amg_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->coarsest_size = 64;
    opt->max_levels = 40;
    opt->stall_ratio = 0.9;
    opt->max_aggregate = 0;
    opt->seed = 0x5EED5EEDull;
    opt->kcycle_inner = 2;
    opt->precision = AMG_PREC_FP64;
    opt->max_iters = 200;
    opt->max_coarsest = 4096;
    opt->use_graph = 1;
    opt->mem_budget = 0;
    opt->stream = nullptr;
    opt->max_rhs = 1;
    opt->smoother = AMG_SMOOTHER_L1;
    opt->jacobi_weight = 2.0 / 3.0;
    opt->autotune = 1;
    opt->kcycle_threshold = 0.0;
    opt->skip_ratio = 0.0;
    opt->post_fused = -1;
    opt->batch_cols = 0;
}

amg_status amg_setup(const amg_csr *A, const amg_options *opt_in, amg_hierarchy **out)
{
    if (!out) return AMG_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (!A || !A->row_ptr || !A->col_idx || !A->values || A->n < 1 || A->nnz < A->n) return AMG_ERR_INVALID_ARGUMENT;
    if (!device_array(A->row_ptr) || !device_array(A->col_idx) || !device_array(A->values))
        return AMG_ERR_INVALID_ARGUMENT;
    amg_options opt;
    if (opt_in) opt = *opt_in;
    else amg_default_options(&opt);
    if (opt.coarsest_size < 1 || opt.max_levels < 1 || opt.max_levels > 64 || !(opt.stall_ratio > 0.0) ||
        !(opt.stall_ratio <= 1.0) || opt.max_aggregate < 0 || opt.max_aggregate == 1 || opt.max_iters < 0 ||
        opt.max_coarsest < 1 || opt.max_rhs < 1 || opt.max_rhs > 1024 || !(opt.jacobi_weight > 0.0) ||
        !std::isfinite(opt.jacobi_weight) || !(opt.kcycle_threshold >= 0.0) || !std::isfinite(opt.kcycle_threshold) ||
        !(opt.skip_ratio >= 0.0) || !std::isfinite(opt.skip_ratio) || opt.post_fused < -1 || opt.post_fused > 1 ||
        !(opt.batch_cols == 0 || opt.batch_cols == 1 || opt.batch_cols == 2 || opt.batch_cols == 4 ||
          opt.batch_cols == 8))
        return AMG_ERR_INVALID_ARGUMENT;
    if (opt.smoother != AMG_SMOOTHER_L1 && opt.smoother != AMG_SMOOTHER_JACOBI) return AMG_ERR_UNSUPPORTED;
    if (opt.kcycle_inner != 1 && opt.kcycle_inner != 2) return AMG_ERR_UNSUPPORTED;
    if (opt.precision != AMG_PREC_FP64 && opt.precision != AMG_PREC_FP32_INNER) return AMG_ERR_UNSUPPORTED;
    amg_hierarchy *h = new (std::nothrow) amg_hierarchy();
    if (!h) return AMG_ERR_OUT_OF_MEMORY;
    h->opt = opt;
    h->pool.budget = opt.mem_budget;
    amg_status st = guarded([&]() -> amg_status {
        AMG_TRACE_MSG("setup: start");
        if (opt.stream) {
            h->stream = (hipStream_t)opt.stream;
        } else {
            AMG_HIP(hipStreamCreate(&h->stream));
            h->own_stream = true;
        }
        h->build(*A);
        AMG_TRACE_MSG("setup: done");
        return AMG_OK;
    });
    if (st != AMG_OK) {
        delete h;
        return st;
    }
    *out = h;
    return AMG_OK;
}

amg_status amg_solve(amg_hierarchy *h, const double *b, double *x, double tol, amg_solve_info *info)
{
    if (!h || !b || !x || !(tol > 0.0) || !std::isfinite(tol)) return AMG_ERR_INVALID_ARGUMENT;
    if (!device_array(b) || !device_array(x)) return AMG_ERR_INVALID_ARGUMENT;
    if (h->kcycle_visits() > amg_hierarchy::kMaxKcycleVisits) return AMG_ERR_UNSUPPORTED;
    return guarded([&]() { return h->solve(1, b, h->lev[0].n, x, h->lev[0].n, tol, info); });
}

amg_status amg_solve_batch(amg_hierarchy *h, int32_t nrhs, const double *B, int32_t ldb, double *X, int32_t ldx,
                           double tol, amg_solve_info *info)
{
    if (!h || !B || !X || !(tol > 0.0) || !std::isfinite(tol)) return AMG_ERR_INVALID_ARGUMENT;
    const int n = h->lev[0].n;
    if (nrhs < 1 || nrhs > h->opt.max_rhs || ldb < n || ldx < n) return AMG_ERR_INVALID_ARGUMENT;
    if (!device_array(B) || !device_array(X)) return AMG_ERR_INVALID_ARGUMENT;
    if (h->kcycle_visits() > amg_hierarchy::kMaxKcycleVisits) return AMG_ERR_UNSUPPORTED;
    return guarded([&]() { return h->solve(nrhs, B, ldb, X, ldx, tol, info); });
}

void amg_free(amg_hierarchy *h) { delete h; }

int64_t amg_grid_laplacian_nnz(int32_t dim, const int32_t *dims)
{
    if (!dims || dim < 1 || dim > 3) return -1;
    int64_t n = 1;
    for (int a = 0; a < dim; a++) {
        if (dims[a] < 1) return -1;
        n *= dims[a];
    }
    if (n > INT32_MAX - 1) return -1;
    const int64_t nnz = amg::grid_nnz(dim, dims);
    return nnz > INT32_MAX ? -1 : nnz;
}

amg_status amg_grid_laplacian(int32_t dim, const int32_t *dims, double jitter, uint64_t seed, int32_t *row_ptr,
                              int32_t *col_idx, double *values, void *stream)
{
    if (amg_grid_laplacian_nnz(dim, dims) < 0 || !std::isfinite(jitter) || !(jitter >= 0.0 && jitter < 1.0) ||
        !device_array(row_ptr) || !device_array(col_idx) || !device_array(values))
        return AMG_ERR_INVALID_ARGUMENT;
    return guarded([&]() {
        int64_t n = 1;
        for (int a = 0; a < dim; a++) n *= dims[a];
        const hipStream_t s = (hipStream_t)stream;
        size_t cls = 0;
        void *tmp = amg::BlockCache::get().take(amg::BlockCache::size_class(sizeof(int) * amg::scan_tmp_ints(n)),
                                                &cls);
        if (!tmp) return AMG_ERR_OUT_OF_MEMORY;
        int dev = 0;
        AMG_HIP(hipGetDevice(&dev));
        try {
            amg::launch_grid_laplacian(dim, dims, jitter, seed, row_ptr, col_idx, values, static_cast<int *>(tmp), s);
            AMG_HIP(hipStreamSynchronize(s));
        } catch (...) {
            amg::BlockCache::get().give(tmp, cls, dev);
            throw;
        }
        amg::BlockCache::get().give(tmp, cls, dev);
        return AMG_OK;
    });
}

amg_status amg_grid_laplacian_noalloc(int32_t dim, const int32_t *dims, double jitter, uint64_t seed,
                                      int32_t *row_ptr, int32_t *col_idx, double *values, void *stream)
{
    if (amg_grid_laplacian_nnz(dim, dims) < 0 || !std::isfinite(jitter) || !(jitter >= 0.0 && jitter < 1.0) ||
        !device_array(row_ptr) || !device_array(col_idx) || !device_array(values))
        return AMG_ERR_INVALID_ARGUMENT;
    return guarded([&]() {
        amg::launch_grid_laplacian_noalloc(dim, dims, jitter, seed, row_ptr, col_idx, values, (hipStream_t)stream);
        return AMG_OK;
    });
}

amg_status amg_uniform_rhs(int64_t n, uint64_t seed, double *out, void *stream)
{
    if (n < 1 || !device_array(out)) return AMG_ERR_INVALID_ARGUMENT;
    return guarded([&]() {
        amg::launch_uniform_rhs(n, seed, out, (hipStream_t)stream);
        return AMG_OK;
    });
}

void amg_release_cached_memory(void)
{
    try {
        amg::BlockCache::get().release_all();
    } catch (...) {
    }
}

amg_status amg_memory_bytes(const amg_hierarchy *h, size_t *bytes)
{
    if (!h || !bytes) return AMG_ERR_INVALID_ARGUMENT;
    *bytes = h->pool.used;
    return AMG_OK;
}

amg_status amg_num_levels(const amg_hierarchy *h, int32_t *levels)
{
    if (!h || !levels) return AMG_ERR_INVALID_ARGUMENT;
    *levels = h->levels();
    return AMG_OK;
}

amg_status amg_level_sizes(const amg_hierarchy *h, int32_t level, int32_t *n, int32_t *nnz, int32_t *passes)
{
    if (!h || level < 0 || level >= h->levels()) return AMG_ERR_INVALID_ARGUMENT;
    const Level &L = h->lev[level];
    if (n) *n = L.n;
    if (nnz) *nnz = L.nnz;
    if (passes) *passes = L.passes;
    return AMG_OK;
}

amg_status amg_level_slots(const amg_hierarchy *h, int32_t level, int64_t *slots)
{
    if (!h || !slots || level < 0 || level >= h->levels()) return AMG_ERR_INVALID_ARGUMENT;
    *slots = (int64_t)h->lev[level].sell_slots;
    return AMG_OK;
}

amg_status amg_export_level(const amg_hierarchy *h_c, int32_t level, int32_t *agg_host, int32_t *row_ptr_host,
                            int32_t *col_host, double *val_host)
{
    amg_hierarchy *h = const_cast<amg_hierarchy *>(h_c);
    if (!h || level < 0 || level >= h->levels()) return AMG_ERR_INVALID_ARGUMENT;
    return guarded([&]() {
        const Level &L = h->lev[level];
        if (agg_host) {
            if (L.agg_nat) h->to_host(agg_host, L.agg_nat, L.n);
            else std::fill(agg_host, agg_host + L.n, -1);
        }
        if (row_ptr_host) h->to_host(row_ptr_host, L.rp_nat, L.n + 1);
        if (col_host) h->to_host(col_host, L.ci_nat, L.nnz);
        if (val_host) h->to_host(val_host, L.va_nat, L.nnz);
        return AMG_OK;
    });
}

amg_status amg_spmv(amg_hierarchy *h, int32_t level, const double *x, double *y)
{
    if (!h || !x || !y || level < 0 || level >= h->levels()) return AMG_ERR_INVALID_ARGUMENT;
    if (!device_array(x) || !device_array(y)) return AMG_ERR_INVALID_ARGUMENT;
    return guarded([&]() {
        const Level &L = h->lev[level];
        // natural numbering, no hub-row table: one wavefront per row
        Rows R{};
        R.n = L.n;
        R.ptr = L.rp_nat;
        R.lim = 1 << 30;
        amg::launch_spmv(R, L.ci_nat, L.va_nat, x, y, amg::kWave, h->stream);
        h->sync();
        return AMG_OK;
    });
}

}  // extern "C"

namespace {
amg_status kcycle_columns(amg_hierarchy *h, int ncol, const double *r, int ldr, double *z, int ldz)
{
    if (h->kcycle_visits() > amg_hierarchy::kMaxKcycleVisits) return AMG_ERR_UNSUPPORTED;
    return guarded([&]() {
        const Level &F = h->lev[0];
        h->autotune(ncol);
        h->capture_graphs(ncol);
        AMG_HIP(hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
        for (int c = 0; c < 3 * h->opt.max_rhs; c++) h->host_mask[c] = c < ncol ? 1 : 0;  // every column active
        h->upload_masks();
        amg::launch_gather(F.n, r, h->uperm, h->r, h->stream, ncol, ldr, F.n);
        if (h->mixed) {  // the mixed K-cycle reads (r, r) of column c from scal[c * kScalCol]
            const DotRef rr = amg::launch_dot(F.n, h->r, h->r, h->d_res, h->stream, ncol);
            amg::launch_reduce(rr, h->scal, h->stream, ncol);
        }
        h->run_kcycle(ncol);
        amg::launch_scatter(F.n, h->z, h->uperm, z, h->stream, ncol, F.n, ldz);
        AMG_HIP(hipMemcpyAsync(h->host_i, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        h->sync();
        return h->host_i[0] ? AMG_ERR_BREAKDOWN : AMG_OK;
    });
}
}  // namespace

extern "C" {

amg_status amg_kcycle(amg_hierarchy *h, const double *r, double *z)
{
    if (!h || !r || !z) return AMG_ERR_INVALID_ARGUMENT;
    if (!device_array(r) || !device_array(z)) return AMG_ERR_INVALID_ARGUMENT;
    return kcycle_columns(h, 1, r, h->lev[0].n, z, h->lev[0].n);
}

amg_status amg_kcycle_batch(amg_hierarchy *h, int32_t nrhs, const double *R, int32_t ldr, double *Z, int32_t ldz)
{
    if (!h || !R || !Z) return AMG_ERR_INVALID_ARGUMENT;
    const int n = h->lev[0].n;
    if (nrhs < 1 || nrhs > h->opt.max_rhs || ldr < n || ldz < n) return AMG_ERR_INVALID_ARGUMENT;
    if (!device_array(R) || !device_array(Z)) return AMG_ERR_INVALID_ARGUMENT;
    return kcycle_columns(h, nrhs, R, ldr, Z, ldz);
}

amg_status amg_time_smoother(amg_hierarchy *h, int32_t reps, double *avg_us, double *bytes)
{
    if (!h || reps < 1 || !avg_us) return AMG_ERR_INVALID_ARGUMENT;
    if (h->levels() < 3) return AMG_ERR_UNSUPPORTED;
    if (!h->kd0.rho1.part) return AMG_ERR_UNSUPPORTED;  // the step reads the products of a K-cycle already run
    return guarded([&]() {
        const Level &F = h->lev[0], &C = h->lev[1];
        const int mode = h->opt.kcycle_inner == 1 ? 1 : 2;
        auto launch = [&]() {  // as in the solve: the FP64 step also forms (z, q)
            if (h->mixed) {
                amg::launch_post_smooth<float>(F.A, F.ci, F.k32.va, F.k32.minv, h->r32, F.agg_pos, F.cagg, mode,
                                               nullptr, C.k32.c1, C.k32.c2, h->kd0, h->z32, nullptr, DotBuf{}, h->flag,
                                               F.G, h->stream, h->ainv, C.n, 1, F.xs, F.sl(), F.k32.sva);
            } else {
                amg::launch_post_smooth<double>(F.A, F.ci, F.va, F.minv, h->r, F.agg_pos, F.cagg, mode, nullptr, C.c1,
                                                C.c2, h->kd0, h->z, h->q, h->d_zq, h->flag, F.G, h->stream, h->ainv,
                                                C.n, 1, F.xs, F.sl(), F.k64.sva);
            }
        };
        launch();
        AMG_HIP(hipEventRecord(h->ev0, h->stream));
        for (int k = 0; k < reps; k++) launch();
        AMG_HIP(hipEventRecord(h->ev1, h->stream));
        h->sync();
        float ms = 0.f;
        AMG_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        *avg_us = 1000.0 * ms / reps;
        // per entry: column, value (+ coarse column on small levels); row pointers;
        // per row: minv, r, output (values), the coarse index and (FP64) q; c1, c2 once each
        const double w = h->mixed ? 4.0 : 8.0;
        if (bytes) *bytes = (4.0 + w + (F.cagg ? 4.0 : 0.0)) * F.nnz + 4.0 * (F.n + 1) +
                            ((h->mixed ? 3.0 : 4.0) * w + 4.0) * F.n + 2.0 * w * C.n;
        return AMG_OK;
    });
}

}  // extern "C"

namespace {
// Lanes per row of the one-workgroup sweeps: the power of two nearest below the
// mean row length, at most 16.
int group_lanes(double mean)
{
    int g = 1;
    while (g < 16 && 2.0 * g <= mean) g *= 2;
    return g;
}

amg_status group_call(int32_t count, const amg_group_job *jobs, double tol, void *stream, int kcycle_only,
                      int32_t *status, amg_solve_info *info)
{
    using namespace amg;
    if (count < 0 || (count > 0 && (!jobs || !status))) return AMG_ERR_INVALID_ARGUMENT;
    if (!kcycle_only && (!(tol > 0.0) || !std::isfinite(tol))) return AMG_ERR_INVALID_ARGUMENT;
    if (count == 0) return AMG_OK;
    std::set<std::pair<const amg_hierarchy *, int>> seen;
    std::set<amg_hierarchy *> hs;
    for (int k = 0; k < count; k++) {
        const amg_group_job &j = jobs[k];
        if (!j.h || !device_array(j.b) || !device_array(j.x)) return AMG_ERR_INVALID_ARGUMENT;
        if (j.column < 0 || j.column >= j.h->opt.max_rhs) return AMG_ERR_INVALID_ARGUMENT;
        if (!seen.insert({j.h, j.column}).second) return AMG_ERR_INVALID_ARGUMENT;
        if (j.h->mixed || j.h->levels() < 2 || j.h->levels() > kGroupMaxLevels) return AMG_ERR_UNSUPPORTED;
        if (j.h->kcycle_visits() > amg_hierarchy::kMaxKcycleVisits) return AMG_ERR_UNSUPPORTED;
        hs.insert(j.h);
    }
    return guarded([&]() -> amg_status {
        std::vector<GroupJob> hj((size_t)count);
        for (int k = 0; k < count; k++) {
            const amg_group_job &j = jobs[k];
            const amg_hierarchy &h = *j.h;
            const size_t c = (size_t)j.column;
            GroupJob &g = hj[(size_t)k];
            std::memset(&g, 0, sizeof(g));
            g.levels = h.levels();
            g.max_iters = h.opt.max_iters;
            g.nu = h.opt.kcycle_inner;
            g.tol = tol;
            g.theta = h.opt.kcycle_threshold;
            g.b = j.b;
            g.x = j.x;
            const size_t n0 = (size_t)h.lev[0].n;
            g.r = h.r + c * n0;
            g.z = h.z + c * n0;
            g.p = h.p + c * n0;
            g.q = h.q + c * n0;
            g.cs = h.coarse;
            const int L = h.levels() - 1;
            for (int l = 0; l <= L; l++) {
                const Level &F = h.lev[l];
                GroupLevel &G = g.lev[l];
                G.n = F.n;
                G.nnz = F.nnz;
                G.G = group_lanes((double)F.nnz / F.n);
                // the restriction's lane groups serve one aggregate: its members on the
                // finest level (a gather of the residual), its rows' entries below
                if (l < L) G.Gr = group_lanes((l == 0 ? (double)F.n : (double)F.nnz) / h.lev[l + 1].n);
                G.rp = F.rp;
                G.ci = F.ci;
                G.va = F.va;
                G.minv = F.minv;
                G.lim = F.A.nlong > 0 ? F.A.lim : INT_MAX;
                G.nlong = F.A.nlong;
                G.long_first = F.A.long_first;
                G.chunks = F.A.chunks;
                const bool super_rows = l >= 1 && F.srp != nullptr && F.S.nlong > 0;
                G.slim = super_rows ? F.S.lim : INT_MAX;
                G.snlong = super_rows ? F.S.nlong : 0;
                G.slong_first = super_rows ? F.S.long_first : nullptr;
                G.schunks = super_rows ? F.S.chunks : nullptr;
                if (l < L) {
                    G.agg = F.agg_pos;
                    G.cagg = F.cagg;
                    G.seg = F.seg_ptr;
                    G.srp = l == 0 ? nullptr : F.srp;  // the finest level's super-rows are in another order
                    G.perm = l == 0 ? F.perm : nullptr;  // the finest level keeps the caller's numbering
                }
                if (l >= 1) {
                    const size_t o = c * (size_t)F.n;
                    G.rc = F.rc + o;
                    G.c1 = F.c1 + o;
                    G.c2 = F.c2 + o;
                    G.v1 = F.v1 + o;
                }
            }
        }
        hipStream_t s = stream ? (hipStream_t)stream : jobs[0].h->stream;
        for (amg_hierarchy *h : hs) h->sync();  // each hierarchy's own work is done before the launch
        BlockCache &bc = BlockCache::get();
        int dev = 0;
        AMG_HIP(hipGetDevice(&dev));
        const size_t jb = sizeof(GroupJob) * (size_t)count, rb = sizeof(GroupResult) * (size_t)count;
        size_t got = 0;
        void *blk = bc.take(BlockCache::size_class(jb + rb), &got);
        if (!blk) throw Error(AMG_ERR_OUT_OF_MEMORY, "hipMalloc");
        struct Give {
            BlockCache &bc;
            void *p;
            size_t cls;
            int dev;
            ~Give() { bc.give(p, cls, dev); }
        } give{bc, blk, got, dev};
        GroupJob *d_jobs = static_cast<GroupJob *>(blk);
        GroupResult *d_res = reinterpret_cast<GroupResult *>(static_cast<char *>(blk) + jb);
        std::vector<GroupResult> res((size_t)count);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        AMG_HIP(hipEventCreate(&e0));
        AMG_HIP(hipEventCreate(&e1));
        struct Ev {
            hipEvent_t a, b;
            ~Ev()
            {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } ev{e0, e1};
        AMG_HIP(hipMemcpyAsync(d_jobs, hj.data(), jb, hipMemcpyHostToDevice, s));
        AMG_HIP(hipEventRecord(e0, s));
        launch_group_solve(d_jobs, count, kcycle_only, d_res, s);
        AMG_HIP(hipEventRecord(e1, s));
        AMG_HIP(hipMemcpyAsync(res.data(), d_res, rb, hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        float ms = 0.f;
        AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
        amg_status first = AMG_OK;
        for (int k = 0; k < count; k++) {
            status[k] = res[(size_t)k].status;
            if (first == AMG_OK && res[(size_t)k].status != AMG_OK) first = (amg_status)res[(size_t)k].status;
            if (info) {
                info[k].iterations = res[(size_t)k].iterations;
                info[k].rel_residual = res[(size_t)k].rel_residual;
                info[k].setup_ms = jobs[k].h->setup_ms;
                info[k].solve_ms = ms;
            }
        }
        return first;
    });
}
}  // namespace

extern "C" {

amg_status amg_solve_group(int32_t count, const amg_group_job *jobs, double tol, void *stream, int32_t *status,
                           amg_solve_info *info)
{
    return group_call(count, jobs, tol, stream, 0, status, info);
}

amg_status amg_kcycle_group(int32_t count, const amg_group_job *jobs, void *stream, int32_t *status)
{
    return group_call(count, jobs, 0.0, stream, 1, status, nullptr);
}

const char *amg_status_string(amg_status s)
{
    switch (s) {
    case AMG_OK: return "AMG_OK";
    case AMG_ERR_INVALID_ARGUMENT: return "AMG_ERR_INVALID_ARGUMENT";
    case AMG_ERR_INVALID_MATRIX: return "AMG_ERR_INVALID_MATRIX";
    case AMG_ERR_OUT_OF_MEMORY: return "AMG_ERR_OUT_OF_MEMORY";
    case AMG_ERR_DEVICE: return "AMG_ERR_DEVICE";
    case AMG_ERR_NOT_CONVERGED: return "AMG_ERR_NOT_CONVERGED";
    case AMG_ERR_BREAKDOWN: return "AMG_ERR_BREAKDOWN";
    case AMG_ERR_UNSUPPORTED: return "AMG_ERR_UNSUPPORTED";
    }
    return "AMG_ERR_UNKNOWN";
}

}  // extern "C"

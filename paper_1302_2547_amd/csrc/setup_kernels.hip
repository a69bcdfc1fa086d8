// setup_kernels.hip -- gfx950 kernels of the setup phase (Alg. 1 setup loop).
//
//   priorities (eq. (3.2))            k_priorities
//   parallel aggregation (Alg. 2)     k_mis_max1 + k_mis_select_claim, one pair per pass
//   numbering by coarse vertex (Sec. 5.1)   scan of centre flags, k_assign_aggregates
//   P^T member lists                  k_member_counts / k_member_fill
//   A_c = P^T A P as sums (eq. (2.4))  k_coarse_rows (one wavefront per coarse row,
//                                     LDS bitonic sort + ordered segmented sums),
//                                     k_coarse_big_rows (one block per row beyond
//                                     LDS capacity, LDS-tiled bitonic sort)
//   smoother diagonal (Sec. 4.1)      k_inverse_diagonal / k_coarse_compact
//   coarsest level                    dense Cholesky and explicit inverse
//   solve layout                      nested aggregate order for every level
//
// Coarse levels of 3D problems have hub rows with thousands of entries.  Row
// kernels take a lane count: 1 (a thread per row, regular fine levels) or 64 (a
// wavefront per row, small levels); the MIS passes serve rows longer than `lim`
// with whole blocks.
//
// Every result is independent of the schedule: priorities are unique, a pass
// only claims conflict-free stars, integer counts are exact, and the sums that
// form A_c run in a fixed order.
#include "amg_internal.h"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <vector>

namespace amg {
namespace {

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

inline int grid_for(int64_t threads)
{
    int64_t b = (threads + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > (1 << 20)) b = 1 << 20;
    return (int)b;
}

// MurmurHash3 32-bit finaliser (Appleby): a bijection on 32-bit words.
__device__ inline uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// 64-bit value of another lane of the same row of 16 (DPP move of both halves):
// exchange with lane ^ 1 or lane ^ 2 inside a quad, mirror inside 8 or 16 lanes.
constexpr int kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E, kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;
template <int CTRL>
__device__ inline uint64_t dpp_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Maximum over each aligned group of G lanes, in every lane of the group.  Up to 16
// lanes the partners are reached by DPP inside the group (lanes of other groups may
// be inactive); wider groups add cross-row exchanges.
template <int G>
__device__ inline uint64_t group_max(uint64_t v)
{
    uint64_t w;
    if (G >= 2) { w = dpp_u64<kDppQuadXor1>(v); v = w > v ? w : v; }
    if (G >= 4) { w = dpp_u64<kDppQuadXor2>(v); v = w > v ? w : v; }
    if (G >= 8) { w = dpp_u64<kDppRowHalfMirror>(v); v = w > v ? w : v; }
    if (G >= 16) { w = dpp_u64<kDppRowMirror>(v); v = w > v ? w : v; }
    if (G >= 32) { w = __shfl_xor(v, 16, kWave); v = w > v ? w : v; }
    if (G >= 64) { w = __shfl_xor(v, 32, kWave); v = w > v ? w : v; }
    return v;
}

template <int G>
__device__ inline int group_isum(int v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <int G>
__device__ inline double group_dsum(double v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Block-wide max of a u64 (every thread receives it).
__device__ inline uint64_t block_max(uint64_t v)
{
    __shared__ uint64_t sh[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = group_max<kWave>(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    uint64_t m = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) m = sh[w] > m ? sh[w] : m;
    __syncthreads();
    return m;
}

// ------------------------------------------------------------------ input checks

__global__ void __launch_bounds__(kBlock) k_validate_csr(int n, int nnz, const int *__restrict__ rp,
                                                         const int *__restrict__ ci, const double *__restrict__ va,
                                                         int *__restrict__ err)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(err, 1);
    if (i >= n) return;
    const int b = rp[i], e = rp[i + 1];
    if (b < 0 || e < b || e > nnz) {
        atomicOr(err, 2);
        return;
    }
    int prev = -1;
    bool diag = false;
    for (int p = b; p < e; p++) {
        const int c = ci[p];
        if (c < 0 || c >= n || c <= prev) {
            atomicOr(err, 4);
            return;
        }
        prev = c;
        const double v = va[p];
        if (!isfinite(v)) atomicOr(err, 8);
        if (c == i) {
            diag = true;
            if (!(v > 0.0)) atomicOr(err, 16);
        }
    }
    if (!diag) atomicOr(err, 32);
}

// The smoother's inverse diagonal (Sec. 4.1): with weight <= 0 the l1-Jacobi
// minv_i = 1 / (a_ii + sum_{j != i} |a_ij|) (the row summed in column order),
// else the damped Jacobi minv_i = weight / a_ii.
__device__ inline double smoother_inverse(double diag, double off, double weight)
{
    return weight > 0.0 ? weight / diag : 1.0 / (diag + off);
}

__global__ void __launch_bounds__(kBlock) k_inverse_diagonal(int n, const int *__restrict__ rp,
                                                             const int *__restrict__ ci,
                                                             const double *__restrict__ va, double weight,
                                                             double *__restrict__ minv)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double diag = 0.0, off = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; p++) {
        if (ci[p] == i) diag += va[p];
        else off += fabs(va[p]);
    }
    minv[i] = smoother_inverse(diag, off, weight);
}

// ------------------------------------------------------------------ eq. (3.2)

// key_i = (12 d_i + (i mod 12) + 1) * 2^32 + fmix32(i XOR s_l): 12 * 2^32 * v_i
// shifted by 2^32 so that 0 can mark "processed".  d_i = row length - 1 (the
// diagonal is present in every row of every level).
__global__ void __launch_bounds__(kBlock) k_priorities(int n, const int *__restrict__ rp, uint32_t s_l,
                                                       uint64_t *__restrict__ key, int *__restrict__ owner)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t deg = (uint64_t)(rp[i + 1] - rp[i] - 1);
    const uint64_t whole = 12u * deg + (uint64_t)(i % 12) + 1u;
    key[i] = (whole << 32) | (uint64_t)fmix32((uint32_t)i ^ s_l);
    owner[i] = -1;
}

// ------------------------------------------------------------------ Alg. 2, one pass
//
// Step (2b) with distances measured among unprocessed vertices: i is a coarse
// vertex of the pass iff its key is the maximum over unprocessed vertices within
// distance 2 through unprocessed vertices.  Two sweeps of max-propagation give
// that maximum: m1_i = max over the closed neighbourhood (processed keys are 0),
// m2_i = max over the closed neighbourhood of m1.  A group of G lanes serves an
// ordinary row; rows longer than lim (listed in hubs) are served by whole blocks,
// from the first min(nhub, kLongBlocks) blocks.

template <int G>
__global__ void __launch_bounds__(kBlock) k_mis_max1(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const uint64_t *__restrict__ key, uint64_t *__restrict__ m1,
                                                     const int *__restrict__ hubs, int nhub, int lim)
{
    const int nhb = nhub < kLongBlocks ? nhub : kLongBlocks;
    if ((int)blockIdx.x < nhb) {
        for (int k = blockIdx.x; k < nhub; k += nhb) {
            const int i = hubs[k];
            uint64_t m = 0;
            if (key[i] != 0) {
                for (int p = rp[i] + threadIdx.x; p < rp[i + 1]; p += kBlock) {
                    const uint64_t kj = key[ci[p]];
                    m = kj > m ? kj : m;
                }
            }
            m = block_max(m);
            if (threadIdx.x == 0) m1[i] = m;
        }
        return;
    }
    const int sub = threadIdx.x % G;
    const int ngroups = (gridDim.x - nhb) * (kBlock / G);
    for (int i = ((blockIdx.x - nhb) * kBlock + threadIdx.x) / G; i < n; i += ngroups) {
        const int b = rp[i], e = rp[i + 1];
        if (e - b > lim) continue;
        const uint64_t ki = key[i];
        uint64_t m = 0;
        if (ki != 0) {
            for (int p = b + sub; p < e; p += G) {
                const uint64_t kj = key[ci[p]];
                m = kj > m ? kj : m;
            }
        }
        m = group_max<G>(m);
        if (sub == 0) m1[i] = m;
    }
}

// Step (2b) decision (m2 == key) and step (2c): the coarse vertex takes itself and
// its unprocessed neighbours in ascending order, at most cap-1 of them (cap = 0:
// all).  Coarse vertices of one pass are at distance >= 3 among unprocessed
// vertices, so no two of them touch the same neighbour.  key[i] may be zeroed
// concurrently by a neighbouring coarse vertex that claims i; one lane reads it
// and the group (or block) decides on that one value.  (If i is claimed it cannot
// be a local maximum.)
template <int G>
__global__ void __launch_bounds__(kBlock) k_mis_select_claim(int n, const int *__restrict__ rp,
                                                             const int *__restrict__ ci, uint64_t *key,
                                                             const uint64_t *__restrict__ m1, int *owner, int cap,
                                                             unsigned *__restrict__ done,
                                                             const int *__restrict__ hubs, int nhub, int lim)
{
    __shared__ unsigned block_done;
    __shared__ uint64_t sh_key;
    __shared__ int sh_cnt[kBlock / kWave];
    if (threadIdx.x == 0) block_done = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nhb = nhub < kLongBlocks ? nhub : kLongBlocks;
    if ((int)blockIdx.x < nhb) {
        for (int k = blockIdx.x; k < nhub; k += nhb) {
            const int i = hubs[k];
            if (threadIdx.x == 0) sh_key = key[i];
            __syncthreads();
            const uint64_t ki = sh_key;
            __syncthreads();
            if (ki == 0) continue;  // uniform within the block
            const int b = rp[i], e = rp[i + 1];
            uint64_t m = 0;
            for (int p = b + threadIdx.x; p < e; p += kBlock) {
                const uint64_t v = m1[ci[p]];
                m = v > m ? v : m;
            }
            m = block_max(m);
            if (m != ki) continue;
            int taken = 1;
            for (int p0 = b; p0 < e; p0 += kBlock) {
                if (cap > 0 && taken >= cap) break;
                const int p = p0 + threadIdx.x;
                int j = -1;
                bool cand = false;
                if (p < e) {
                    j = ci[p];
                    cand = (j != i) && (key[j] != 0);
                }
                const uint64_t bal = __ballot(cand);
                if (lane == 0) sh_cnt[wid] = __popcll(bal);
                __syncthreads();
                int before = 0, total = 0;
#pragma unroll
                for (int w = 0; w < kBlock / kWave; w++) {
                    if (w < wid) before += sh_cnt[w];
                    total += sh_cnt[w];
                }
                __syncthreads();
                const int rank = before + __popcll(bal & ((1ull << lane) - 1ull));
                if (cand && (cap == 0 || taken + rank < cap)) {
                    owner[j] = i;
                    key[j] = 0;
                }
                taken += (cap > 0 && taken + total > cap) ? (cap - taken) : total;
            }
            if (threadIdx.x == 0) {
                owner[i] = i;
                key[i] = 0;
                block_done += (unsigned)taken;
            }
            __syncthreads();
        }
    } else {
        const int sub = threadIdx.x % G;
        const int gbase = lane - sub;  // first lane of this group within the wave
        const uint64_t gmask = (G == kWave) ? ~0ull : (((1ull << G) - 1ull) << gbase);
        const int ngroups = (gridDim.x - nhb) * (kBlock / G);
        for (int i = ((blockIdx.x - nhb) * kBlock + threadIdx.x) / G; i < n; i += ngroups) {
            const int b = rp[i], e = rp[i + 1];
            if (e - b > lim) continue;
            uint64_t ki = (sub == 0) ? key[i] : 0;
            ki = __shfl(ki, gbase, kWave);
            if (ki == 0) continue;  // processed (uniform within the group)
            uint64_t m = 0;
            for (int p = b + sub; p < e; p += G) {
                const uint64_t v = m1[ci[p]];
                m = v > m ? v : m;
            }
            m = group_max<G>(m);
            if (m != ki) continue;  // not a local maximum (uniform within the group)
            int taken = 1;
            for (int p0 = b; p0 < e; p0 += G) {
                if (cap > 0 && taken >= cap) break;
                const int p = p0 + sub;
                int j = -1;
                bool cand = false;
                if (p < e) {
                    j = ci[p];
                    cand = (j != i) && (key[j] != 0);
                }
                const uint64_t bal = __ballot(cand) & gmask;
                const int rank = __popcll(bal & ((1ull << lane) - 1ull) & gmask);
                if (cand && (cap == 0 || taken + rank < cap)) {
                    owner[j] = i;
                    key[j] = 0;
                }
                const int c = __popcll(bal);
                taken += (cap > 0 && taken + c > cap) ? (cap - taken) : c;
            }
            if (sub == 0) {
                owner[i] = i;
                key[i] = 0;
                atomicAdd(&block_done, (unsigned)taken);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && block_done) atomicAdd(done + (blockIdx.x % kDoneSlots) * kDoneStride, block_done);
}

// *out = sum of the kDoneSlots counters (one block of kDoneSlots threads).
__global__ void __launch_bounds__(kDoneSlots) k_sum_slots(const unsigned *__restrict__ slots, unsigned *__restrict__ out)
{
    __shared__ unsigned sh[kDoneSlots];
    sh[threadIdx.x] = slots[threadIdx.x * kDoneStride];
    __syncthreads();
    for (int h = kDoneSlots / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// ------------------------------------------------------------------ numbering (Sec. 5.1)

__global__ void __launch_bounds__(kBlock) k_centre_flags(int n, const int *__restrict__ owner, int *__restrict__ flag)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) flag[i] = owner[i] == i ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_assign_aggregates(int n, const int *__restrict__ owner,
                                                              const int *__restrict__ cid, int *__restrict__ agg,
                                                              int *__restrict__ centre_of)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int o = owner[i];
    agg[i] = cid[o];
    if (o == i) centre_of[cid[i]] = i;
}

// Members of aggregate I are its coarse vertex c and the neighbours j of c with
// owner j = c; walking row c (ascending columns, diagonal included) lists them in
// ascending order.  G lanes (1 or 64) serve one aggregate.
template <int G>
__global__ void __launch_bounds__(kBlock) k_member_counts(int nc, const int *__restrict__ rp,
                                                          const int *__restrict__ ci, const int *__restrict__ owner,
                                                          const int *__restrict__ centre_of, int *__restrict__ size,
                                                          int *__restrict__ pairs)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    for (int I = (blockIdx.x * kBlock + threadIdx.x) / G; I < nc; I += ngroups) {
        const int c = centre_of[I];
        int s = 0, pc = 0;
        for (int p = rp[c] + sub; p < rp[c + 1]; p += G) {
            const int j = ci[p];
            if (owner[j] == c) {
                s++;
                pc += rp[j + 1] - rp[j];
            }
        }
        s = group_isum<G>(s);
        pc = group_isum<G>(pc);
        if (sub == 0) {
            size[I] = s;
            pairs[I] = pc;
        }
    }
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_member_fill(int nc, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const int *__restrict__ owner,
                                                        const int *__restrict__ centre_of,
                                                        const int *__restrict__ aptr, int *__restrict__ members)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = threadIdx.x % G;
    const int gbase = lane - sub;
    const uint64_t gmask = (G == kWave) ? ~0ull : (((1ull << G) - 1ull) << gbase);
    const int ngroups = gridDim.x * (kBlock / G);
    for (int I = (blockIdx.x * kBlock + threadIdx.x) / G; I < nc; I += ngroups) {
        const int c = centre_of[I];
        int k = aptr[I];
        for (int p0 = rp[c]; p0 < rp[c + 1]; p0 += G) {
            const int p = p0 + sub;
            int j = -1;
            bool mem = false;
            if (p < rp[c + 1]) {
                j = ci[p];
                mem = owner[j] == c;
            }
            const uint64_t bal = __ballot(mem) & gmask;
            if (mem) members[k + __popcll(bal & ((1ull << lane) - 1ull))] = j;
            k += __popcll(bal);
        }
    }
}

// Level skipping (Sec. 3.3): the aggregates of the composed aggregation P = P1 P2
// are the unions of the first aggregation's groups over each group J of the second.
// Their members are listed group after group, in the second aggregation's member
// order (any order inside an aggregate serves the solve layout).
//
// One wavefront per aggregate J of the second aggregation; lane j takes its middle
// aggregate members2[k0 + j] (64 at a time, k0 = aptr2[J], aptr2[J] + 64, ...).
__global__ void __launch_bounds__(kBlock) k_compose_sizes(int nc2, const int *__restrict__ aptr2,
                                                          const int *__restrict__ members2,
                                                          const int *__restrict__ aptr1, int *__restrict__ size)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t J = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave; J < nc2; J += waves) {
        int s = 0;
        const int ke = aptr2[J + 1];
        for (int k = aptr2[J] + lane; k < ke; k += kWave) {
            const int I = members2[k];
            s += aptr1[I + 1] - aptr1[I];
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
        if (lane == 0) size[J] = s;
    }
}

// The fine members of J: those of its middle aggregates in their order, each one's in
// its own order; a lane copies the members of its middle aggregate at the offset the
// wavefront's prefix of their sizes gives.
__global__ void __launch_bounds__(kBlock) k_compose_members(int nc2, const int *__restrict__ aptr2,
                                                            const int *__restrict__ members2,
                                                            const int *__restrict__ aptr1,
                                                            const int *__restrict__ members1,
                                                            const int *__restrict__ aptr, int *__restrict__ members)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t J = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave; J < nc2; J += waves) {
        int q = aptr[J];
        const int ke = aptr2[J + 1];
        for (int k0 = aptr2[J]; k0 < ke; k0 += kWave) {
            const int k = k0 + lane;
            int b = 0, len = 0;
            if (k < ke) {
                const int I = members2[k];
                b = aptr1[I];
                len = aptr1[I + 1] - b;
            }
            int incl = len;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += y;
            }
            const int at = q + incl - len;
            for (int t = 0; t < len; t++) members[at + t] = members1[b + t];
            q += __shfl(incl, kWave - 1, kWave);
        }
    }
}

// ------------------------------------------------------------------ eq. (2.4)
//
// Coarse row I gathers the pairs (agg[t], a_st) of its members' rows, in member
// order and column order; key = (J << 32) | position makes the sort stable, and
// each segment of equal J is summed sequentially in position order, which is the
// order of a row-by-row accumulation over (s, t).

constexpr int kWaveCap = 256;  // pairs one wavefront sorts in LDS (18 KB of LDS per block: 8 blocks per CU)
constexpr int kWavesPerBlock = kBlock / kWave;

__global__ void __launch_bounds__(kBlock) k_coarse_rows(int nc, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, const double *__restrict__ va,
                                                        const int *__restrict__ agg, const int *__restrict__ aptr,
                                                        const int *__restrict__ members, const int *__restrict__ tptr,
                                                        int *__restrict__ tcol, double *__restrict__ tval,
                                                        int *__restrict__ cnt, int *__restrict__ big_rows,
                                                        unsigned *__restrict__ big_count)
{
    __shared__ uint64_t skey[kWavesPerBlock][kWaveCap];
    __shared__ double sval[kWavesPerBlock][kWaveCap];
    __shared__ int smb[kWavesPerBlock][kWave], smx[kWavesPerBlock][kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint64_t *key = skey[w];
    double *val = sval[w];
    int *mbeg = smb[w], *mexcl = smx[w];
    const int total_waves = gridDim.x * kWavesPerBlock;
    for (int I = blockIdx.x * kWavesPerBlock + w; I < nc; I += total_waves) {
        const int base = tptr[I];
        const int pc = tptr[I + 1] - base;
        if (pc > kWaveCap) {
            if (lane == 0) big_rows[atomicAdd(big_count, 1u)] = I;
            continue;
        }
        // gather: up to 64 members at a time, their rows spread over the lanes
        int fill = 0;
        const int me = aptr[I + 1];
        for (int m0 = aptr[I]; m0 < me; m0 += kWave) {
            const int m = m0 + lane;
            int b = 0, len = 0;
            if (m < me) {
                const int s = members[m];
                b = rp[s];
                len = rp[s + 1] - b;
            }
            int incl = len;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += y;
            }
            mbeg[lane] = b;
            mexcl[lane] = incl - len;
            const int tot = __shfl(incl, kWave - 1, kWave);
            const int nm = (me - m0) < kWave ? (me - m0) : kWave;
            wave_sync();
            for (int k = lane; k < tot; k += kWave) {
                int lo = 0, hi = nm - 1;  // last member with mexcl <= k
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (mexcl[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                const int p = mbeg[lo] + (k - mexcl[lo]);
                const int pos = fill + k;
                key[pos] = ((uint64_t)(uint32_t)agg[ci[p]] << 32) | (uint32_t)pos;
                val[pos] = va[p];
            }
            fill += tot;
            wave_sync();
        }
        int P = 1;
        while (P < pc) P <<= 1;
        for (int k = pc + lane; k < P; k += kWave) key[k] = ~0ull;
        wave_sync();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = lane; t < P / 2; t += kWave) {
                    const int lo = 2 * stride * (t / stride) + (t % stride);
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t a = key[lo], c = key[hi];
                    if ((a > c) == up) {
                        key[lo] = c;
                        key[hi] = a;
                    }
                }
                wave_sync();
            }
        }
        int out = 0;
        for (int q0 = 0; q0 < pc; q0 += kWave) {
            const int q = q0 + lane;
            bool head = false;
            uint32_t J = 0;
            if (q < pc) {
                J = (uint32_t)(key[q] >> 32);
                head = (q == 0) || ((uint32_t)(key[q - 1] >> 32) != J);
            }
            const uint64_t hm = __ballot(head);
            if (head) {
                const int rank = out + __popcll(hm & ((1ull << lane) - 1ull));
                double s = 0.0;
                for (int r = q; r < pc && (uint32_t)(key[r] >> 32) == J; r++) s += val[(uint32_t)key[r]];
                tcol[base + rank] = (int)J;
                tval[base + rank] = s;
            }
            out += __popcll(hm);
        }
        if (lane == 0) cnt[I] = out;
        wave_sync();
    }
}

// Rows with more pairs than one wavefront's LDS holds: one block of kBigThreads
// per row.  Keys live in global scratch; the bitonic network runs its strides
// below kTile inside LDS tiles and only the longer strides as global passes.
constexpr int kBigThreads = 1024;
constexpr int kTile = 4096;

__device__ void tile_steps(uint64_t *t, int64_t base, int64_t size, int stride0, int len)
{
    for (int stride = stride0; stride > 0; stride >>= 1) {
        for (int u = threadIdx.x; u < len / 2; u += kBigThreads) {
            const int lo = 2 * stride * (u / stride) + (u % stride);
            const int hi = lo + stride;
            const bool up = ((base + lo) & size) == 0;
            const uint64_t a = t[lo], c = t[hi];
            if ((a > c) == up) {
                t[lo] = c;
                t[hi] = a;
            }
        }
        __syncthreads();
    }
}

// phase 0: gather every row's pairs; rows of fewer than split_min padded keys are
// then sorted and summed here (one block), the others only gathered.  phase 1:
// the sums of those other rows, whose keys the whole-chip passes below sorted.
__global__ void __launch_bounds__(kBigThreads) k_coarse_big_rows(const int *__restrict__ big_rows,
                                                                 const int64_t *__restrict__ scratch_off,
                                                                 uint64_t *skey, const int *__restrict__ rp,
                                                                 const int *__restrict__ ci,
                                                                 const double *__restrict__ va,
                                                                 const int *__restrict__ agg,
                                                                 const int *__restrict__ aptr,
                                                                 const int *__restrict__ members,
                                                                 const int *__restrict__ tptr, int *__restrict__ tcol,
                                                                 double *__restrict__ tval, int *__restrict__ cnt,
                                                                 int phase, int64_t split_min)
{
    __shared__ uint64_t tile[kTile];
    __shared__ int mbeg[kBigThreads], mexcl[kBigThreads];
    __shared__ int sh_count[kBigThreads / kWave];
    __shared__ int sh_tot, sh_out;
    const int I = big_rows[blockIdx.x];
    uint64_t *key = skey + scratch_off[blockIdx.x];
    double *val = reinterpret_cast<double *>(skey + scratch_off[gridDim.x]) + scratch_off[blockIdx.x];
    const int base = tptr[I];
    const int pc = tptr[I + 1] - base;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int64_t P = 1;
    while (P < pc) P <<= 1;
    const bool split = P >= split_min;
    if (phase == 1 && !split) return;
    if (phase == 0) {
    // gather: up to kBigThreads members at a time, block-wide prefix of row lengths
    int fill = 0;
    const int me = aptr[I + 1];
    for (int m0 = aptr[I]; m0 < me; m0 += kBigThreads) {
        const int m = m0 + threadIdx.x;
        int b = 0, len = 0;
        if (m < me) {
            const int s = members[m];
            b = rp[s];
            len = rp[s + 1] - b;
        }
        int incl = len;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        if (lane == kWave - 1) sh_count[w] = incl;
        __syncthreads();
        int before = 0;
        for (int k = 0; k < w; k++) before += sh_count[k];
        incl += before;
        mbeg[threadIdx.x] = b;
        mexcl[threadIdx.x] = incl - len;
        if (threadIdx.x == kBigThreads - 1) sh_tot = incl;
        __syncthreads();
        const int tot = sh_tot;
        const int nm = (me - m0) < kBigThreads ? (me - m0) : kBigThreads;
        for (int k = threadIdx.x; k < tot; k += kBigThreads) {
            int lo = 0, hi = nm - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (mexcl[mid] <= k) lo = mid;
                else hi = mid - 1;
            }
            const int p = mbeg[lo] + (k - mexcl[lo]);
            const int pos = fill + k;
            key[pos] = ((uint64_t)(uint32_t)agg[ci[p]] << 32) | (uint32_t)pos;
            val[pos] = va[p];
        }
        fill += tot;
        __syncthreads();
    }
    for (int64_t k = pc + threadIdx.x; k < P; k += kBigThreads) key[k] = ~0ull;
    __syncthreads();
    if (split) return;  // sorted by the whole-chip passes, summed in phase 1
    const int tl = P < kTile ? (int)P : kTile;
    // 1) sort every tile completely (bitonic sizes up to the tile length)
    for (int64_t t0 = 0; t0 < P; t0 += tl) {
        for (int k = threadIdx.x; k < tl; k += kBigThreads) tile[k] = key[t0 + k];
        __syncthreads();
        for (int size = 2; size <= tl; size <<= 1) tile_steps(tile, t0, size, size >> 1, tl);
        for (int k = threadIdx.x; k < tl; k += kBigThreads) key[t0 + k] = tile[k];
        __syncthreads();
    }
    // 2) larger sizes: long strides in global memory, the rest inside tiles
    for (int64_t size = 2 * (int64_t)tl; size <= P; size <<= 1) {
        int64_t stride = size >> 1;
        for (; stride >= tl; stride >>= 1) {
            for (int64_t u = threadIdx.x; u < P / 2; u += kBigThreads) {
                const int64_t lo = 2 * stride * (u / stride) + (u % stride);
                const int64_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = key[lo], c = key[hi];
                if ((a > c) == up) {
                    key[lo] = c;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
        for (int64_t t0 = 0; t0 < P; t0 += tl) {
            for (int k = threadIdx.x; k < tl; k += kBigThreads) tile[k] = key[t0 + k];
            __syncthreads();
            tile_steps(tile, t0, size, (int)stride, tl);
            for (int k = threadIdx.x; k < tl; k += kBigThreads) key[t0 + k] = tile[k];
            __syncthreads();
        }
    }
    }  // phase 0
    // 3) values in sorted order, head positions, then every segment of equal J
    //    summed in position order over a contiguous range
    double *sv = reinterpret_cast<double *>(skey + 2 * scratch_off[gridDim.x]) + scratch_off[blockIdx.x];
    int *hp = reinterpret_cast<int *>(skey + 3 * scratch_off[gridDim.x] + scratch_off[blockIdx.x]);
    for (int q = threadIdx.x; q < pc; q += kBigThreads) sv[q] = val[(uint32_t)key[q]];
    if (threadIdx.x == 0) sh_out = 0;
    __syncthreads();
    for (int q0 = 0; q0 < pc; q0 += kBigThreads) {
        const int q = q0 + (int)threadIdx.x;
        bool head = false;
        if (q < pc) head = (q == 0) || ((uint32_t)(key[q - 1] >> 32) != (uint32_t)(key[q] >> 32));
        const uint64_t hm = __ballot(head);
        if (lane == 0) sh_count[w] = __popcll(hm);
        __syncthreads();
        int before = sh_out;
        for (int k = 0; k < w; k++) before += sh_count[k];
        if (head) hp[before + __popcll(hm & ((1ull << lane) - 1ull))] = q;
        __syncthreads();
        if (threadIdx.x == 0) {
            int add = 0;
            for (int k = 0; k < kBigThreads / kWave; k++) add += sh_count[k];
            sh_out += add;
        }
        __syncthreads();
    }
    const int u = sh_out;
    if (threadIdx.x == 0) hp[u] = pc;
    __syncthreads();
    for (int k = threadIdx.x; k < u; k += kBigThreads) {
        const int q = hp[k], qe = hp[k + 1];
        double s = 0.0;
        int r = q;
        for (; r + 16 <= qe; r += 16) {  // loads in flight together, adds in order
            double v[16];
#pragma unroll
            for (int j = 0; j < 16; j++) v[j] = sv[r + j];
#pragma unroll
            for (int j = 0; j < 16; j++) s += v[j];
        }
        for (; r < qe; r++) s += sv[r];
        tcol[base + k] = (int)(uint32_t)(key[q] >> 32);
        tval[base + k] = s;
    }
    if (threadIdx.x == 0) cnt[I] = u;
}

// The sort of the longest big rows as passes over the whole chip (the keys are
// unique, so any correct sort gives the one order the block sort gives): every
// tile of kTile keys sorted in LDS by one block, then for every bitonic size above
// kTile the strides of at least kTile as global compare-exchange passes and the
// shorter ones again inside the tiles.
constexpr int64_t kSplitMin = int64_t(1) << 17;
constexpr int kSplitRows = 32;
struct SplitRows {
    int n;
    int64_t off[kSplitRows];         // first key of the row in the scratch
    int64_t P[kSplitRows];           // padded key count (a power of two >= kSplitMin)
    int64_t tile0[kSplitRows + 1];   // prefix of P / kTile
    int64_t pair0[kSplitRows + 1];   // prefix of P / 2
};

// size 0: sort every tile completely; size > kTile: the strides below kTile of that
// bitonic size, in the tiles of rows of at least size keys
__global__ void __launch_bounds__(kBigThreads) k_big_tile_sort(SplitRows S, uint64_t *skey, int64_t size)
{
    __shared__ uint64_t tile[kTile];
    const int64_t b = blockIdx.x;
    int r = 0;
    while (r + 1 < S.n && S.tile0[r + 1] <= b) r++;
    if (size > S.P[r]) return;
    const int64_t t0 = (b - S.tile0[r]) * kTile;
    uint64_t *key = skey + S.off[r];
    for (int k = threadIdx.x; k < kTile; k += kBigThreads) tile[k] = key[t0 + k];
    __syncthreads();
    if (size == 0) {
        for (int sz = 2; sz <= kTile; sz <<= 1) tile_steps(tile, t0, sz, sz >> 1, kTile);
    } else {
        tile_steps(tile, t0, size, kTile / 2, kTile);
    }
    for (int k = threadIdx.x; k < kTile; k += kBigThreads) key[t0 + k] = tile[k];
}

// one compare-exchange stride of a bitonic size, over every row of at least size keys
__global__ void __launch_bounds__(kBlock) k_big_global_pass(SplitRows S, uint64_t *skey, int64_t size,
                                                            int64_t stride)
{
    const int64_t items = S.pair0[S.n];
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < items; g += (int64_t)gridDim.x * kBlock) {
        int r = 0;
        while (r + 1 < S.n && S.pair0[r + 1] <= g) r++;
        if (size > S.P[r]) continue;
        const int64_t u = g - S.pair0[r];
        const int64_t lo = 2 * stride * (u / stride) + (u % stride);
        const int64_t hi = lo + stride;
        const bool up = (lo & size) == 0;
        uint64_t *key = skey + S.off[r];
        const uint64_t a = key[lo], c = key[hi];
        if ((a > c) == up) {
            key[lo] = c;
            key[hi] = a;
        }
    }
}

// Big rows on coarse levels small enough for a dense accumulator in LDS: one
// block of kBigThreads per row.  The row's pairs are taken in position order
// (members ascending, each member's entries in column order), kBigThreads at a
// time; every batch is sorted by (J, position) -- in registers for strides
// inside a wavefront, through LDS for the longer ones -- and each run of equal J
// is added to acc[J] in position order.  Every coarse entry is therefore summed
// in the order of the sequential definition, and the row never leaves LDS.
constexpr uint64_t kUntouched = 0x7FF4C0A75E000001ull;  // a NaN payload arithmetic never makes
constexpr int kAccStaticBytes = 32 * 1024;              // LDS of the kernel besides acc[]

__device__ inline uint64_t block_sort_keys(uint64_t v, uint64_t *sk)
{
    const int t = threadIdx.x;
    for (int size = 2; size <= kBigThreads; size <<= 1) {
        const bool up = (t & size) == 0;
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            uint64_t o;
            if (stride >= kWave) {  // uniform over the block
                __syncthreads();
                sk[t] = v;
                __syncthreads();
                o = sk[t ^ stride];
            } else {
                o = __shfl_xor(v, stride, kWave);
            }
            const bool lower = (t & stride) == 0;
            v = (lower == up) ? (v < o ? v : o) : (v > o ? v : o);
        }
    }
    return v;
}

__global__ void __launch_bounds__(kBigThreads) k_coarse_big_rows_acc(const int *__restrict__ big_rows, int nc,
                                                                     const int *__restrict__ rp,
                                                                     const int *__restrict__ ci,
                                                                     const double *__restrict__ va,
                                                                     const int *__restrict__ agg,
                                                                     const int *__restrict__ aptr,
                                                                     const int *__restrict__ members,
                                                                     const int *__restrict__ tptr,
                                                                     int *__restrict__ tcol, double *__restrict__ tval,
                                                                     int *__restrict__ cnt)
{
    extern __shared__ double acc[];  // nc entries
    __shared__ uint64_t sk[kBigThreads];
    __shared__ double cv[kBigThreads];
    __shared__ int mbeg[kBigThreads], mexcl[kBigThreads], hp[kBigThreads + 1];
    __shared__ int sh_count[kBigThreads / kWave];
    __shared__ int sh_tot, sh_out;
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const uint64_t below = (1ull << lane) - 1ull;
    const int I = big_rows[blockIdx.x];
    for (int J = t; J < nc; J += kBigThreads) acc[J] = __longlong_as_double((long long)kUntouched);
    const int me = aptr[I + 1];
    for (int m0 = aptr[I]; m0 < me; m0 += kBigThreads) {
        // block-wide prefix of the row lengths of up to kBigThreads members
        const int m = m0 + t;
        int b = 0, len = 0;
        if (m < me) {
            const int sidx = members[m];
            b = rp[sidx];
            len = rp[sidx + 1] - b;
        }
        int incl = len;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        __syncthreads();  // the previous group's readers of mbeg / mexcl / sh_count are done
        if (lane == kWave - 1) sh_count[w] = incl;
        __syncthreads();
        int before = 0;
        for (int k = 0; k < w; k++) before += sh_count[k];
        incl += before;
        mbeg[t] = b;
        mexcl[t] = incl - len;
        if (t == kBigThreads - 1) sh_tot = incl;
        __syncthreads();
        const int tot = sh_tot;
        const int nm = (me - m0) < kBigThreads ? (me - m0) : kBigThreads;
        for (int k0 = 0; k0 < tot; k0 += kBigThreads) {
            const int k = k0 + t;
            uint64_t key = ~0ull;
            double v = 0.0;
            if (k < tot) {
                int lo = 0, hi = nm - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (mexcl[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                const int p = mbeg[lo] + (k - mexcl[lo]);
                key = ((uint64_t)(uint32_t)agg[ci[p]] << 32) | (uint32_t)t;
                v = va[p];
            }
            cv[t] = v;
            key = block_sort_keys(key, sk);
            const bool valid = key != ~0ull;
            const uint32_t J = (uint32_t)(key >> 32);
            __syncthreads();
            const double mv = valid ? cv[(uint32_t)key] : 0.0;
            sk[t] = key;
            __syncthreads();
            cv[t] = mv;  // values in sorted order
            const bool head = valid && (t == 0 || (uint32_t)(sk[t - 1] >> 32) != J);
            const uint64_t hm = __ballot(head);
            if (lane == 0) sh_count[w] = __popcll(hm);
            __syncthreads();
            int hb = 0, nh = 0;
            for (int q = 0; q < kBigThreads / kWave; q++) {
                if (q < w) hb += sh_count[q];
                nh += sh_count[q];
            }
            if (head) hp[hb + __popcll(hm & below)] = t;
            if (t == 0) hp[nh] = (tot - k0) < kBigThreads ? (tot - k0) : kBigThreads;
            __syncthreads();
            if (t < nh) {  // run t: its values in position order onto acc[J]
                const int q = hp[t], qe = hp[t + 1];
                const uint32_t JJ = (uint32_t)(sk[q] >> 32);
                double a = acc[JJ];
                if ((uint64_t)__double_as_longlong(a) == kUntouched) a = 0.0;
                int r = q;
                for (; r + 16 <= qe; r += 16) {  // LDS reads in flight together, adds in order
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; u++) v[u] = cv[r + u];
#pragma unroll
                    for (int u = 0; u < 16; u++) a += v[u];
                }
                for (; r < qe; r++) a += cv[r];
                acc[JJ] = a;
            }
            __syncthreads();
        }
    }
    // the touched columns in ascending order
    const int base = tptr[I];
    if (t == 0) sh_out = 0;
    for (int J0 = 0; J0 < nc; J0 += kBigThreads) {
        const int J = J0 + t;
        double a = 0.0;
        bool on = false;
        if (J < nc) {
            a = acc[J];
            on = (uint64_t)__double_as_longlong(a) != kUntouched;
        }
        const uint64_t hm = __ballot(on);
        __syncthreads();  // sh_out / sh_count of the previous iteration are read
        if (lane == 0) sh_count[w] = __popcll(hm);
        __syncthreads();
        int ob = sh_out, tot = 0;
        for (int q = 0; q < kBigThreads / kWave; q++) {
            if (q < w) ob += sh_count[q];
            tot += sh_count[q];
        }
        if (on) {
            const int o = ob + __popcll(hm & below);
            tcol[base + o] = J;
            tval[base + o] = a;
        }
        __syncthreads();
        if (t == 0) sh_out += tot;
    }
    __syncthreads();
    if (t == 0) cnt[I] = sh_out;
}

// Copy the unique entries of every coarse row into the final CSR and form the
// coarse l1 diagonal.  G = 1: the row is summed in column order; G = 64: lanes
// share the row (used on small levels, whose hub rows are long).
template <int G>
__global__ void __launch_bounds__(kBlock) k_coarse_compact(int nc, const int *__restrict__ tptr,
                                                           const int *__restrict__ tcol,
                                                           const double *__restrict__ tval,
                                                           const int *__restrict__ crp, int *__restrict__ cci,
                                                           double *__restrict__ cva, double weight,
                                                           double *__restrict__ cminv)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    for (int I = (blockIdx.x * kBlock + threadIdx.x) / G; I < nc; I += ngroups) {
        const int src = tptr[I], dst = crp[I], len = crp[I + 1] - crp[I];
        double diag = 0.0, off = 0.0;
        for (int k = sub; k < len; k += G) {
            const int J = tcol[src + k];
            const double v = tval[src + k];
            cci[dst + k] = J;
            cva[dst + k] = v;
            if (J == I) diag += v;
            else off += fabs(v);
        }
        diag = group_dsum<G>(diag);
        off = group_dsum<G>(off);
        if (sub == 0) cminv[I] = smoother_inverse(diag, off, weight);
    }
}

// ------------------------------------------------------------------ coarsest level

__global__ void __launch_bounds__(kBlock) k_dense_from_csr(int n, const int *__restrict__ rp,
                                                           const int *__restrict__ ci, const double *__restrict__ va,
                                                           double *__restrict__ dense)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; p++) dense[(size_t)i * n + ci[p]] = va[p];
}

// One block: right-looking Cholesky A = L L^T in place (lower triangle of a), then
// inv = L^-T L^-1 column by column (forward then backward substitution).
constexpr int kCholThreads = 1024;

constexpr int kSmallDense = 256;  // coarsest levels up to this size: one block factors them
__global__ void __launch_bounds__(kCholThreads) k_cholesky_inverse(int n, double *a, double *inv, int *err)
{
    __shared__ double piv;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < n; k++) {
        if (threadIdx.x == 0) {
            const double d = a[(size_t)k * n + k];
            if (!(d > 0.0)) {
                bad = 1;
                *err = 1;
            } else {
                piv = sqrt(d);
                a[(size_t)k * n + k] = piv;
            }
        }
        __syncthreads();
        if (bad) return;
        for (int i = k + 1 + threadIdx.x; i < n; i += kCholThreads) a[(size_t)i * n + k] /= piv;
        __syncthreads();
        const int m = n - k - 1;
        for (int64_t t = threadIdx.x; t < (int64_t)m * m; t += kCholThreads) {
            const int ii = (int)(t / m), jj = (int)(t % m);
            if (jj <= ii) {
                const int i = k + 1 + ii, j = k + 1 + jj;
                a[(size_t)i * n + j] -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
            }
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < n; j += kCholThreads) {
        // forward: L y = e_j, y_i = 0 for i < j
        for (int i = 0; i < j; i++) inv[(size_t)i * n + j] = 0.0;
        for (int i = j; i < n; i++) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = j; k < i; k++) s -= a[(size_t)i * n + k] * inv[(size_t)k * n + j];
            inv[(size_t)i * n + j] = s / a[(size_t)i * n + i];
        }
        // backward: L^T x = y
        for (int i = n - 1; i >= 0; i--) {
            double s = inv[(size_t)i * n + j];
            for (int k = i + 1; k < n; k++) s -= a[(size_t)k * n + i] * inv[(size_t)k * n + j];
            inv[(size_t)i * n + j] = s / a[(size_t)i * n + i];
        }
    }
}

// Larger coarsest levels: Gauss-Jordan inversion in place, one launch per pivot
// (no pivoting: every pivot is a Schur complement of an SPD matrix, hence > 0).
// Step k reads row k and column k as step k-1 left them from rk / ck and writes
// row and column k+1 of its result to rn / cn for the next step.
__global__ void __launch_bounds__(kBlock) k_gauss_jordan_step(int n, int k, double *__restrict__ a,
                                                              const double *__restrict__ rk,
                                                              const double *__restrict__ ck, double *__restrict__ rn,
                                                              double *__restrict__ cn, int *__restrict__ err)
{
    const double p = rk[k];
    if (!(p > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *err = 1;
        return;
    }
    const double ip = 1.0 / p;
    const int64_t nn = (int64_t)n * n;
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < nn; t += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(t / n), j = (int)(t % n);
        double v;
        if (i == k && j == k) v = ip;
        else if (i == k) v = rk[j] * ip;
        else if (j == k) v = -ck[i] * ip;
        else v = a[t] - ck[i] * (rk[j] * ip);
        a[t] = v;
        if (i == k + 1) rn[j] = v;
        if (j == k + 1) cn[i] = v;
    }
}

__global__ void __launch_bounds__(kBlock) k_row_col(int n, const double *__restrict__ a, double *__restrict__ r0,
                                                    double *__restrict__ c0)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        r0[i] = a[i];
        c0[i] = a[(size_t)i * n];
    }
}

// ------------------------------------------------------------------ solve layout
//
// Every level is stored in nested aggregate order: the coarsest level in its own
// order, and level l as the concatenation of its aggregates in the order their
// coarse unknowns have on level l+1, members ascending inside an aggregate.  Then
// restriction sums contiguous segments and prolongation broadcasts over them.

__global__ void __launch_bounds__(kBlock) k_identity(int n, int *__restrict__ v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = i;
}

__global__ void __launch_bounds__(kBlock) k_sizes_in_position_order(int nc, const int *__restrict__ aptr_nat,
                                                                    const int *__restrict__ perm_c,
                                                                    int *__restrict__ size_pos)
{
    const int Q = blockIdx.x * kBlock + threadIdx.x;
    if (Q >= nc) return;
    const int J = perm_c[Q];
    size_pos[Q] = aptr_nat[J + 1] - aptr_nat[J];
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_positions_from_segments(int nc, const int *__restrict__ aptr_nat,
                                                                    const int *__restrict__ members_nat,
                                                                    const int *__restrict__ pos_c,
                                                                    const int *__restrict__ seg_ptr,
                                                                    int *__restrict__ pos_f, int *__restrict__ perm_f)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    for (int J = (blockIdx.x * kBlock + threadIdx.x) / G; J < nc; J += ngroups) {
        const int start = seg_ptr[pos_c[J]];
        const int b = aptr_nat[J], e = aptr_nat[J + 1];
        for (int k = sub; k < e - b; k += G) {
            const int i = members_nat[b + k];
            pos_f[i] = start + k;
            perm_f[start + k] = i;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_permuted_row_lengths(int n, const int *__restrict__ rp_nat,
                                                                 const int *__restrict__ perm, int *__restrict__ len)
{
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const int i = perm[q];
    len[q] = rp_nat[i + 1] - rp_nat[i];
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_permute_rows(int n, const int *__restrict__ rp_nat,
                                                         const int *__restrict__ ci_nat,
                                                         const double *__restrict__ va_nat,
                                                         const double *__restrict__ minv_nat,
                                                         const int *__restrict__ perm, const int *__restrict__ pos,
                                                         const int *__restrict__ rp, int *__restrict__ ci,
                                                         double *__restrict__ va, double *__restrict__ minv)
{
    const int sub = threadIdx.x % G;
    const int ngroups = gridDim.x * (kBlock / G);
    for (int q = (blockIdx.x * kBlock + threadIdx.x) / G; q < n; q += ngroups) {
        const int i = perm[q];
        const int b = rp_nat[i], len = rp_nat[i + 1] - b, d = rp[q];
        for (int k = sub; k < len; k += G) {
            ci[d + k] = pos[ci_nat[b + k]];
            va[d + k] = va_nat[b + k];
        }
        if (sub == 0) minv[q] = minv_nat[i];
    }
}

__global__ void __launch_bounds__(kBlock) k_agg_positions(int n, const int *__restrict__ perm_f,
                                                          const int *__restrict__ agg_nat,
                                                          const int *__restrict__ pos_c, int *__restrict__ agg_pos)
{
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q < n) agg_pos[q] = pos_c[agg_nat[perm_f[q]]];
}

__global__ void __launch_bounds__(kBlock) k_gather_int(int n, const int *__restrict__ src, const int *__restrict__ idx,
                                                       int *__restrict__ dst)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

__global__ void __launch_bounds__(kBlock) k_long_flags(int n, const int *__restrict__ ptr, int lim,
                                                       int *__restrict__ flags)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) flags[i] = (ptr[i + 1] - ptr[i] > lim) ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_long_compact(int n, const int *__restrict__ ptr, int lim,
                                                         const int *__restrict__ offs, int *__restrict__ list)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n && ptr[i + 1] - ptr[i] > lim) list[offs[i]] = i;
}

// Lanes per row/aggregate for the helper kernels: a wavefront on small levels.
inline bool wide(int n) { return n < kSmallLevel; }

// Sliced ELLPACK build (layout in amg_internal.h).  One wavefront per slice: the
// width is the wavefront's largest row length, at least 1.
__global__ void __launch_bounds__(kBlock) k_sell_widths(int n, const int *__restrict__ rp, int *__restrict__ width)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    int len = i < n ? rp[i + 1] - rp[i] : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o));
    if ((threadIdx.x & (kWave - 1)) == 0 && i < n) width[i / kWave] = max(len, 1);
}

// One thread per slot row (nslices * kWave threads): rows past n are padding rows.
__global__ void __launch_bounds__(kBlock) k_sell_fill(int n, int nslices, const int *__restrict__ rp,
                                                      const int *__restrict__ ci, const double *__restrict__ va,
                                                      const int *__restrict__ ptr, int *__restrict__ sci,
                                                      double *__restrict__ sva)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int s = i / kWave, t = i % kWave;
    if (s >= nslices) return;
    const int b = i < n ? rp[i] : 0, len = i < n ? rp[i + 1] - b : 0;
    const int pad = i < n ? i : n - 1;
    const int beg = ptr[s], w = (ptr[s + 1] - beg) / kWave;
    for (int k = 0; k < w; k++) {
        const int q = beg + k * kWave + t;
        sci[q] = k < len ? ci[b + k] : pad;
        sva[q] = k < len ? va[b + k] : 0.0;
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

#define AMG_LAUNCH_G(G, KERNEL, GRID, STREAM, ...)                                      \
    switch (G) {                                                                        \
    case 1: KERNEL<1><<<GRID, kBlock, 0, STREAM>>>(__VA_ARGS__); break;                 \
    case 2: KERNEL<2><<<GRID, kBlock, 0, STREAM>>>(__VA_ARGS__); break;                 \
    case 4: KERNEL<4><<<GRID, kBlock, 0, STREAM>>>(__VA_ARGS__); break;                 \
    case 8: KERNEL<8><<<GRID, kBlock, 0, STREAM>>>(__VA_ARGS__); break;                 \
    case 16: KERNEL<16><<<GRID, kBlock, 0, STREAM>>>(__VA_ARGS__); break;               \
    case 32: KERNEL<32><<<GRID, kBlock, 0, STREAM>>>(__VA_ARGS__); break;               \
    default: KERNEL<64><<<GRID, kBlock, 0, STREAM>>>(__VA_ARGS__); break;               \
    }

void launch_long_rows(int n, const int *ptr, int lim, int *flags, int *list, int *count_dev, int *scan_tmp,
                      hipStream_t s)
{
    // list == nullptr: count only (flags are left as exclusive offsets)
    if (list == nullptr) {
        k_long_flags<<<grid_for(n), kBlock, 0, s>>>(n, ptr, lim, flags);
        AMG_HIP(hipGetLastError());
        scan_exclusive(flags, flags, n, count_dev, scan_tmp, s);
        return;
    }
    k_long_compact<<<grid_for(n), kBlock, 0, s>>>(n, ptr, lim, flags, list);
    AMG_HIP(hipGetLastError());
}

void launch_validate_csr(int n, int nnz, const int *rp, const int *ci, const double *va, int *err, hipStream_t s)
{
    k_validate_csr<<<grid_for(n), kBlock, 0, s>>>(n, nnz, rp, ci, va, err);
    AMG_HIP(hipGetLastError());
}

void launch_inverse_diagonal(int n, const int *rp, const int *ci, const double *va, double weight, double *minv,
                             hipStream_t s)
{
    k_inverse_diagonal<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, va, weight, minv);
    AMG_HIP(hipGetLastError());
}

void launch_priorities(int n, const int *rp, uint32_t s_l, uint64_t *key, int *owner, hipStream_t s)
{
    k_priorities<<<grid_for(n), kBlock, 0, s>>>(n, rp, s_l, key, owner);
    AMG_HIP(hipGetLastError());
}

void launch_mis_pass(int n, const int *rp, const int *ci, uint64_t *key, uint64_t *m1, int *owner, int cap, int G,
                     unsigned *done_counter, const int *hubs, int nhub, int lim, hipStream_t s)
{
    const int nhb = nhub < kLongBlocks ? nhub : kLongBlocks;
    const int grid = nhb + grid_for((int64_t)n * G);
    AMG_LAUNCH_G(G, k_mis_max1, grid, s, n, rp, ci, key, m1, hubs, nhub, lim);
    AMG_LAUNCH_G(G, k_mis_select_claim, grid, s, n, rp, ci, key, m1, owner, cap, done_counter, hubs, nhub, lim);
    AMG_HIP(hipGetLastError());
}

void launch_sum_slots(const unsigned *slots, unsigned *out, hipStream_t s)
{
    k_sum_slots<<<1, kDoneSlots, 0, s>>>(slots, out);
    AMG_HIP(hipGetLastError());
}

void launch_centre_flags(int n, const int *owner, int *flag, hipStream_t s)
{
    k_centre_flags<<<grid_for(n), kBlock, 0, s>>>(n, owner, flag);
    AMG_HIP(hipGetLastError());
}

void launch_assign_aggregates(int n, const int *owner, const int *cid, int *agg, int *centre_of, hipStream_t s)
{
    k_assign_aggregates<<<grid_for(n), kBlock, 0, s>>>(n, owner, cid, agg, centre_of);
    AMG_HIP(hipGetLastError());
}

void launch_member_counts(int nc, const int *rp, const int *ci, const int *owner, const int *centre_of, int *size,
                          int *pairs, hipStream_t s)
{
    const int G = wide(nc) ? kWave : 1;
    AMG_LAUNCH_G(G, k_member_counts, grid_for((int64_t)nc * G), s, nc, rp, ci, owner, centre_of, size, pairs);
    AMG_HIP(hipGetLastError());
}

void launch_compose_sizes(int nc2, const int *aptr2, const int *members2, const int *aptr1, int *size, hipStream_t s)
{
    k_compose_sizes<<<grid_for((int64_t)nc2 * kWave), kBlock, 0, s>>>(nc2, aptr2, members2, aptr1, size);
    AMG_HIP(hipGetLastError());
}

void launch_compose_members(int nc2, const int *aptr2, const int *members2, const int *aptr1, const int *members1,
                            const int *aptr, int *members, hipStream_t s)
{
    k_compose_members<<<grid_for((int64_t)nc2 * kWave), kBlock, 0, s>>>(nc2, aptr2, members2, aptr1, members1, aptr,
                                                                      members);
    AMG_HIP(hipGetLastError());
}

void launch_member_fill(int nc, const int *rp, const int *ci, const int *owner, const int *centre_of,
                        const int *aptr, int *members, hipStream_t s)
{
    const int G = wide(nc) ? kWave : 1;
    AMG_LAUNCH_G(G, k_member_fill, grid_for((int64_t)nc * G), s, nc, rp, ci, owner, centre_of, aptr, members);
    AMG_HIP(hipGetLastError());
}

int coarse_wave_capacity() { return kWaveCap; }

void launch_coarse_rows(int nc, const int *rp, const int *ci, const double *va, const int *agg, const int *aptr,
                        const int *members, const int *tptr, int *tcol, double *tval, int *cnt, int *big_rows,
                        unsigned *big_count, hipStream_t s)
{
    int64_t blocks = ((int64_t)nc + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    k_coarse_rows<<<(int)blocks, kBlock, 0, s>>>(nc, rp, ci, va, agg, aptr, members, tptr, tcol, tval, cnt, big_rows,
                                                 big_count);
    AMG_HIP(hipGetLastError());
}

void launch_coarse_big_rows(int nbig, const int *big_rows, const int64_t *scratch_off, uint64_t *skey,
                            const int *rp, const int *ci, const double *va, const int *agg, const int *aptr,
                            const int *members, const int *tptr, int *tcol, double *tval, int *cnt, hipStream_t s)
{
    if (nbig <= 0) return;
    // rows of at least kSplitMin padded keys (at most kSplitRows of them, the longest;
    // the threshold is raised otherwise) are sorted by whole-chip passes
    std::vector<int64_t> off(nbig + 1);
    AMG_HIP(hipMemcpyAsync(off.data(), scratch_off, sizeof(int64_t) * (nbig + 1), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> lens;
    for (int k = 0; k < nbig; k++) lens.push_back(off[k + 1] - off[k]);
    std::vector<int64_t> sorted_lens = lens;
    std::sort(sorted_lens.begin(), sorted_lens.end(), std::greater<int64_t>());
    int64_t split_min = kSplitMin;
    // AMG_SPLIT_MIN_KEYS (a power of two >= kTile) lowers the threshold, so that the
    // whole-chip passes can be checked on rows of moderate problems
    if (const char *e = std::getenv("AMG_SPLIT_MIN_KEYS")) {
        const long long v = std::atoll(e);
        if (v >= kTile && (v & (v - 1)) == 0) split_min = v;
    }
    if ((int)sorted_lens.size() > kSplitRows && sorted_lens[kSplitRows] >= split_min)
        split_min = sorted_lens[kSplitRows] * 2;  // powers of two: only lengths above the 33rd
    SplitRows S{};
    int64_t pmax = 0;
    for (int k = 0; k < nbig && S.n < kSplitRows; k++) {
        if (lens[k] < split_min) continue;
        S.off[S.n] = off[k];
        S.P[S.n] = lens[k];
        S.tile0[S.n + 1] = S.tile0[S.n] + lens[k] / kTile;
        S.pair0[S.n + 1] = S.pair0[S.n] + lens[k] / 2;
        pmax = std::max(pmax, lens[k]);
        S.n++;
    }
    if (trace_on())
        std::fprintf(stderr, "[amg] coarse big rows: %d, %d of them (at least %lld keys) by whole-chip passes\n", nbig,
                     S.n, (long long)split_min);
    if (S.n == 0) split_min = INT64_MAX;
    k_coarse_big_rows<<<nbig, kBigThreads, 0, s>>>(big_rows, scratch_off, skey, rp, ci, va, agg, aptr, members, tptr,
                                                   tcol, tval, cnt, 0, split_min);
    AMG_HIP(hipGetLastError());
    if (S.n == 0) return;
    const int64_t tiles = S.tile0[S.n], pairs = S.pair0[S.n];
    const int gp = (int)std::min<int64_t>((pairs + kBlock - 1) / kBlock, 1 << 16);
    k_big_tile_sort<<<(unsigned)tiles, kBigThreads, 0, s>>>(S, skey, 0);
    AMG_HIP(hipGetLastError());
    for (int64_t size = 2 * (int64_t)kTile; size <= pmax; size <<= 1) {
        for (int64_t stride = size >> 1; stride >= kTile; stride >>= 1) {
            k_big_global_pass<<<gp, kBlock, 0, s>>>(S, skey, size, stride);
            AMG_HIP(hipGetLastError());
        }
        k_big_tile_sort<<<(unsigned)tiles, kBigThreads, 0, s>>>(S, skey, size);
        AMG_HIP(hipGetLastError());
    }
    k_coarse_big_rows<<<nbig, kBigThreads, 0, s>>>(big_rows, scratch_off, skey, rp, ci, va, agg, aptr, members, tptr,
                                                   tcol, tval, cnt, 1, split_min);
    AMG_HIP(hipGetLastError());
}

int coarse_acc_capacity()
{
    int dev = 0, lds = 0;
    AMG_HIP(hipGetDevice(&dev));
    AMG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int bytes = lds - kAccStaticBytes;
    return bytes > 0 ? bytes / (int)sizeof(double) : 0;
}

void launch_coarse_big_rows_acc(int nbig, const int *big_rows, int nc, const int *rp, const int *ci, const double *va,
                                const int *agg, const int *aptr, const int *members, const int *tptr, int *tcol,
                                double *tval, int *cnt, hipStream_t s)
{
    if (nbig <= 0) return;
    const size_t lds = sizeof(double) * (size_t)nc;
    k_coarse_big_rows_acc<<<nbig, kBigThreads, lds, s>>>(big_rows, nc, rp, ci, va, agg, aptr, members, tptr, tcol,
                                                         tval, cnt);
    AMG_HIP(hipGetLastError());
}

void launch_coarse_compact(int nc, const int *tptr, const int *tcol, const double *tval, const int *crp, int *cci,
                           double *cva, double weight, double *cminv, hipStream_t s)
{
    const int G = wide(nc) ? kWave : 8;  // coarse rows hold ~10-20 entries
    AMG_LAUNCH_G(G, k_coarse_compact, grid_for((int64_t)nc * G), s, nc, tptr, tcol, tval, crp, cci, cva, weight, cminv);
    AMG_HIP(hipGetLastError());
}

void launch_dense_from_csr(int n, const int *rp, const int *ci, const double *va, double *dense, hipStream_t s)
{
    k_dense_from_csr<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, va, dense);
    AMG_HIP(hipGetLastError());
}

void launch_cholesky_inverse(int n, double *a, double *inv, int *err, hipStream_t s)
{
    if (n <= kSmallDense) {
        k_cholesky_inverse<<<1, kCholThreads, 0, s>>>(n, a, inv, err);
        AMG_HIP(hipGetLastError());
        return;
    }
    // inv <- a, then Gauss-Jordan in place; the row / column buffers follow a.
    const size_t nn = (size_t)n * n;
    AMG_HIP(hipMemcpyAsync(inv, a, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    double *buf = a;  // a (n^2 >= 4n) is free now: two row/column pairs
    double *r[2] = {buf, buf + 2 * (size_t)n}, *c[2] = {buf + n, buf + 3 * (size_t)n};
    k_row_col<<<grid_for(n), kBlock, 0, s>>>(n, inv, r[0], c[0]);
    const int grid = (int)std::min<int64_t>(((int64_t)nn + 4 * kBlock - 1) / (4 * kBlock), 1 << 16);
    for (int k = 0; k < n; k++)
        k_gauss_jordan_step<<<grid, kBlock, 0, s>>>(n, k, inv, r[k & 1], c[k & 1], r[(k + 1) & 1], c[(k + 1) & 1],
                                                     err);
    AMG_HIP(hipGetLastError());
}

namespace {
// om_t = sum over the rows q that hold column t of [q == t] - a_qt minv_t: the row
// vector W = P^T (I - A M^-1) of a level whose coarse level is a single unknown
// (P = all ones).  The rows holding column t are the columns of row t (the pattern
// is symmetric); a_qt is found in row q by bisection.  One block per column: thread
// k takes the entries k, k + kBlock, ... of row t (a hub column has thousands), and
// the block adds the partial sums in a fixed order.
__global__ void __launch_bounds__(kBlock) k_single_unknown_weights(int n, const int *__restrict__ rp,
                                                                   const int *__restrict__ ci,
                                                                   const double *__restrict__ va,
                                                                   const double *__restrict__ minv,
                                                                   double *__restrict__ om)
{
    __shared__ double sh[kBlock];
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const double mt = minv[t];
        double s = 0.0;
        for (int e = rp[t] + (int)threadIdx.x; e < rp[t + 1]; e += kBlock) {
            const int q = ci[e];
            int lo = rp[q], hi = rp[q + 1] - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ci[mid] < t) lo = mid + 1;
                else hi = mid;
            }
            if (lo < rp[q + 1] && ci[lo] == t) s += (q == t ? 1.0 : 0.0) - va[lo] * mt;
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) om[t] = sh[0];
        __syncthreads();
    }
}

// dinv[k] = 1 / va[pos[k]]: the exact solve of the coarsest level's decoupled unknowns
__global__ void __launch_bounds__(kBlock) k_reciprocals(int m, const int *__restrict__ pos,
                                                        const double *__restrict__ va, double *__restrict__ dinv)
{
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < m; k += gridDim.x * kBlock) dinv[k] = 1.0 / va[pos[k]];
}

}  // namespace

void launch_single_unknown_weights(int n, const int *rp, const int *ci, const double *va, const double *minv,
                                   double *om, hipStream_t s)
{
    k_single_unknown_weights<<<n < 65536 ? n : 65536, kBlock, 0, s>>>(n, rp, ci, va, minv, om);
    AMG_HIP(hipGetLastError());
}

void launch_reciprocals(int m, const int *pos, const double *va, double *dinv, hipStream_t s)
{
    if (m <= 0) return;
    k_reciprocals<<<grid_for(m), kBlock, 0, s>>>(m, pos, va, dinv);
    AMG_HIP(hipGetLastError());
}

void launch_identity(int n, int *v, hipStream_t s)
{
    k_identity<<<grid_for(n), kBlock, 0, s>>>(n, v);
    AMG_HIP(hipGetLastError());
}

void launch_sizes_in_position_order(int nc, const int *aptr_nat, const int *perm_c, int *size_pos, hipStream_t s)
{
    k_sizes_in_position_order<<<grid_for(nc), kBlock, 0, s>>>(nc, aptr_nat, perm_c, size_pos);
    AMG_HIP(hipGetLastError());
}

void launch_positions_from_segments(int nc, const int *aptr_nat, const int *members_nat, const int *pos_c,
                                    const int *seg_ptr, int *pos_f, int *perm_f, hipStream_t s)
{
    const int G = wide(nc) ? kWave : 1;
    AMG_LAUNCH_G(G, k_positions_from_segments, grid_for((int64_t)nc * G), s, nc, aptr_nat, members_nat, pos_c,
                 seg_ptr, pos_f, perm_f);
    AMG_HIP(hipGetLastError());
}

void launch_permuted_row_lengths(int n, const int *rp_nat, const int *perm, int *len, hipStream_t s)
{
    k_permuted_row_lengths<<<grid_for(n), kBlock, 0, s>>>(n, rp_nat, perm, len);
    AMG_HIP(hipGetLastError());
}

void launch_permute_rows(int n, const int *rp_nat, const int *ci_nat, const double *va_nat, const double *minv_nat,
                         const int *perm, const int *pos, const int *rp, int *ci, double *va, double *minv,
                         hipStream_t s)
{
    const int G = wide(n) ? kWave : 8;
    AMG_LAUNCH_G(G, k_permute_rows, grid_for((int64_t)n * G), s, n, rp_nat, ci_nat, va_nat, minv_nat, perm, pos, rp,
                 ci, va, minv);
    AMG_HIP(hipGetLastError());
}

void launch_agg_positions(int n, const int *perm_f, const int *agg_nat, const int *pos_c, int *agg_pos,
                          hipStream_t s)
{
    k_agg_positions<<<grid_for(n), kBlock, 0, s>>>(n, perm_f, agg_nat, pos_c, agg_pos);
    AMG_HIP(hipGetLastError());
}

void launch_gather_int(int n, const int *src, const int *idx, int *dst, hipStream_t s)
{
    k_gather_int<<<grid_for(n), kBlock, 0, s>>>(n, src, idx, dst);
    AMG_HIP(hipGetLastError());
}

void launch_sell_widths(int n, const int *rp, int *width, hipStream_t s)
{
    k_sell_widths<<<grid_for(n), kBlock, 0, s>>>(n, rp, width);
    AMG_HIP(hipGetLastError());
}

void launch_sell_fill(int n, int nslices, const int *rp, const int *ci, const double *va, const int *ptr, int *sci,
                      double *sva, hipStream_t s)
{
    k_sell_fill<<<grid_for((int64_t)nslices * kWave), kBlock, 0, s>>>(n, nslices, rp, ci, va, ptr, sci, sva);
    AMG_HIP(hipGetLastError());
}

}  // namespace amg

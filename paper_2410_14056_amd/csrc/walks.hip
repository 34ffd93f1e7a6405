// Random-walk generation: Alg. 2 (one lane per walk) and Alg. 3 (bouquets: the
// walks of one start vertex advance side by side in a wavefront), with the
// neighbour choice of Eq. (5) and the keyed seed arrangement of Sec. 3.3.
//
// Counting.  Per-step global atomics on the visit histogram serialise on hub
// vertices.  The bouquet path therefore counts without global atomics in the
// hot loop: the walk kernel writes each visited vertex to a step-major visit log
// (coalesced) and counts per block how many visits fall in each bucket of
// 2^bsh consecutive vertex ids (LDS); a scatter pass groups the log by bucket,
// and a histogram pass counts each bucket slice in LDS and adds the bins to the
// int64 outputs.  All counts are integers, so the result does not depend on the
// order of any of these steps.
#include <hip/hip_runtime.h>

#include <hipcub/device/device_radix_sort.hpp>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "saba_internal.hpp"

namespace saba {

constexpr int kWalkBlock = 256;
constexpr int kMaxBucketShift = 14;      // LDS histogram of up to 16384 bins (64 KiB)
constexpr int kMaxBuckets = 2048;        // LDS bucket counters in the walk and scatter kernels
constexpr int64_t kLogCap = 1ll << 29;   // visit-log entries per chunk of walks
// log entries per histogram block: enough blocks for the GPU (kHistBlocks), but no fewer
// entries than LDS bins flushed (a block flushes up to 4096 bins per bucket it meets)
constexpr int64_t kHistSliceMin = 1 << 14, kHistSliceMax = 1 << 18;
constexpr int64_t kHistBlocks = 2048;
constexpr int kPersistBlocks = 8192;
constexpr int64_t kPipeChunks = 4, kPipeMinWalks = (int64_t)1 << 19;

// Counts of equal keys held by adjacent active lanes are merged, so one wavefront
// issues one atomic per run of equal vertices instead of one per lane.
__device__ __forceinline__ void wave_merged_add(unsigned long long *__restrict__ counts,
                                                int32_t key, bool active) {
    const int lane = __lane_id();
    int32_t prev = __shfl_up(key, 1);
    int prev_active = __shfl_up((int)active, 1);
    bool head = active && (lane == 0 || !prev_active || prev != key);
    unsigned long long heads = __ballot(head);
    unsigned long long ends = heads | __ballot(!active);
    if (head) {
        unsigned long long after = lane == 63 ? 0ull : (ends >> (lane + 1));
        int len = after ? (__builtin_ctzll(after) + 1) : (64 - lane);
        atomicAdd(counts + key, (unsigned long long)len);
    }
}

// Sources: count the walks of every start vertex and flag invalid starts.
__global__ __launch_bounds__(kWalkBlock) void source_count_kernel(
    const int32_t *__restrict__ src, int64_t W, const int2 *__restrict__ vrec, int32_t n,
    unsigned long long *__restrict__ counts, int32_t *__restrict__ err) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < W;
         j += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = src[j];
        if (s < 0 || s >= n || vrec[s].y == 0) {
            atomicOr(err, 1);
            continue;
        }
        atomicAdd(counts + s, 1ull);
    }
}

// Sources, bucketed.  The start list is read as a log of `rows` rows of wc entries (entry r,
// i is src[r * wc + i], up to W): block k counts the starts of columns 256 (k + m * gridDim.x)
// .. + 255 (m = 0, 1, ...) per vertex bucket in LDS and writes cnt[b * gridDim.x + k], the
// column order the scatter uses.  A start outside 0 .. n - 1 sets the error flag and is not
// counted; a start without neighbours is caught by start_check_kernel once the counts are per
// vertex, so this pass reads no vertex records.
constexpr int kStartLoads = 8;

__global__ __launch_bounds__(kWalkBlock) void source_bucket_count_kernel(
    const int32_t *__restrict__ src, int64_t W, int32_t rows, int64_t wc, int32_t n, int bsh,
    int32_t nbk, long long *__restrict__ cnt, int32_t *__restrict__ err) {
    extern __shared__ uint32_t lds_sc[];
    for (int b = threadIdx.x; b < nbk; b += kWalkBlock) lds_sc[b] = 0;
    __syncthreads();
    bool bad = false;
    for (int64_t tile = blockIdx.x; tile * kWalkBlock < wc; tile += gridDim.x) {
        const int64_t i = tile * kWalkBlock + threadIdx.x;
        if (i >= wc) continue;
        for (int32_t r0 = 0; r0 < rows; r0 += kStartLoads) {
            int32_t v[kStartLoads];
            bool has[kStartLoads];
#pragma unroll
            for (int u = 0; u < kStartLoads; ++u) {
                const int64_t e = (int64_t)(r0 + u) * wc + i;
                has[u] = r0 + u < rows && e < W;
                v[u] = has[u] ? src[e] : 0;
            }
#pragma unroll
            for (int u = 0; u < kStartLoads; ++u)
                if (has[u]) {
                    if (v[u] < 0 || v[u] >= n)
                        bad = true;
                    else
                        atomicAdd(lds_sc + (v[u] >> bsh), 1u);
                }
        }
    }
    if (bad) atomicOr(err, 1);
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += kWalkBlock)
        cnt[(int64_t)b * gridDim.x + blockIdx.x] = lds_sc[b];
}

// Walks per start vertex, counted: a vertex without neighbours is not a valid start.  Its
// count is cleared (no walk is laid out for it) and the error flag set.
__global__ __launch_bounds__(kWalkBlock) void start_check_kernel(
    const int2 *__restrict__ vrec, int32_t n, unsigned long long *__restrict__ counts,
    int32_t *__restrict__ err) {
    bool bad = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        if (counts[v] != 0 && vrec[v].y == 0) {
            counts[v] = 0;
            bad = true;
        }
    if (bad) atomicOr(err, 1);
}

// Bucket order: bsrc[w] = s for offs[s] <= w < offs[s + 1].  A thread fills kFillRun
// consecutive walks; it finds the start vertex of the first by binary search and of each later
// one by a step to the next vertex or, past vertices without walks, another search.
constexpr int kFillRun = 16;

__device__ __forceinline__ int32_t last_at_or_below(const int64_t *__restrict__ offs, int32_t lo,
                                                    int32_t hi, int64_t w) {
    // largest s in [lo, hi) with offs[s] <= w, given offs[lo] <= w
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (offs[mid] <= w)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kWalkBlock) void source_fill_kernel(const int64_t *__restrict__ offs,
                                                                 int32_t n,
                                                                 int32_t *__restrict__ bsrc) {
    // a block fills 4096 consecutive walks: thread t the run 16 t .. 16 t + 15, staged in LDS
    // (17 words per run, so the 64 lanes of a wavefront hit distinct banks) and stored
    // coalesced
    constexpr int kSpan = kWalkBlock * kFillRun;
    __shared__ int32_t stage[kWalkBlock * (kFillRun + 1)];
    const int64_t W = offs[n];
    for (int64_t b0 = (int64_t)blockIdx.x * kSpan; b0 < W; b0 += (int64_t)gridDim.x * kSpan) {
        const int64_t w0 = b0 + (int64_t)threadIdx.x * kFillRun;
        if (w0 < W) {
            int32_t v = last_at_or_below(offs, 0, n, w0);
            int64_t next = offs[v + 1];
            const int64_t w1 = min(W, w0 + kFillRun);
            for (int64_t w = w0; w < w1; ++w) {
                if (w >= next) {
                    v = offs[v + 2] > w ? v + 1 : last_at_or_below(offs, v + 1, n, w);
                    next = offs[v + 1];
                }
                stage[threadIdx.x * (kFillRun + 1) + (int)(w - w0)] = v;
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < kSpan; q += kWalkBlock)
            if (b0 + q < W) bsrc[b0 + q] = stage[q + q / kFillRun];
        __syncthreads();
    }
}

// Branching statistics: the distinct vertices among each aligned group of 8 lanes, whose
// walks have consecutive indices in the order the mode runs them.  Every lane of the wavefront
// calls it; the first lane of a full group adds one to the block's LDS bin of its count.
__device__ __forceinline__ void distinct8_count(int32_t cur, bool full, uint32_t *lhist) {
    const int lane = __lane_id();
    const int base = lane & ~7, p = lane & 7;
    bool first = true;
    for (int q = 0; q < 7; ++q) {
        const int32_t v = __shfl(cur, base + q);
        if (q < p && v == cur) first = false;
    }
    const unsigned long long fm = __ballot(first);
    if (p == 0 && full) atomicAdd(lhist + __popcll((fm >> base) & 0xffull), 1u);
}

__device__ __forceinline__ void distinct8_flush(const uint32_t *lhist,
                                                unsigned long long *__restrict__ out) {
    __syncthreads();
    if (threadIdx.x < 9 && lhist[threadIdx.x])
        atomicAdd(out + threadIdx.x, (unsigned long long)lhist[threadIdx.x]);
}

// Rank of every walk among the walks of its start vertex, in list order: the walks sorted by
// start vertex (a stable sort keeps list order inside a start vertex) give position p, and
// rank = p - offs[s].
__global__ __launch_bounds__(kWalkBlock) void list_rank_kernel(
    const int32_t *__restrict__ sorted_src, const uint32_t *__restrict__ sorted_j, int64_t W,
    const int64_t *__restrict__ offs, const int2 *__restrict__ vrec, int32_t n,
    uint32_t *__restrict__ rank) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < W;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = sorted_src[p];
        if (s < 0 || s >= n || vrec[s].y == 0) continue;  // flagged by the count kernel
        rank[sorted_j[p]] = (uint32_t)(p - offs[s]);
    }
}

__global__ __launch_bounds__(kWalkBlock) void iota_kernel(uint32_t *__restrict__ v, int64_t W) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < W;
         j += (int64_t)gridDim.x * blockDim.x)
        v[j] = (uint32_t)j;
}

// Alg. 2: one lane per walk, walks in the order the sources are given, one global atomic
// per visit.  Walk j is the rank[j]-th walk of its start vertex in list order.
template <int SM, bool CNT>
__global__ __launch_bounds__(kWalkBlock) void walk_naive_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col, const int32_t *__restrict__ src,
    const uint32_t *__restrict__ rank, int64_t W, int32_t L, uint32_t seed, uint32_t G, uint32_t S,
    int32_t n, unsigned long long *__restrict__ endpoint, unsigned long long *__restrict__ visits,
    int32_t *__restrict__ err, unsigned long long *__restrict__ distinct) {
    __shared__ uint32_t lhist[9];
    if (CNT) {
        if (threadIdx.x < 9) lhist[threadIdx.x] = 0;
        __syncthreads();
    }
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = j < W;
    int32_t s = 0;
    if (act) {
        s = src[j];
        if (s < 0 || s >= n || vrec[s].y == 0) {
            atomicOr(err, 1);
            act = false;
        }
    }
    if (!CNT && !act) return;
    Walker w{};
    if (act) w = walker_init<SM>(walk_key(seed, (uint32_t)s, 0u, 0u, rank[j], G, S));
    const bool full = (j & ~7ll) + 8 <= W;
    int32_t cur = s;
    for (int32_t l = 1; l <= L; ++l) {
        if (act) {
            cur = walker_step<SM>(vrec, col, cur, (uint32_t)l, w);
            atomicAdd(visits + cur, 1ull);
        }
        if (CNT) distinct8_count(cur, full, lhist);
    }
    if (act) atomicAdd(endpoint + cur, 1ull);
    if (CNT) distinct8_flush(lhist, distinct);
}

// Alg. 3 for graphs too large for the bucketed count: bouquet order with equal visits
// of adjacent lanes merged before the global atomics.
template <int SM, bool CNT>
__global__ __launch_bounds__(kWalkBlock) void walk_bouquet_atomic_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
    const int32_t *__restrict__ bsrc, const int64_t *__restrict__ offs, int32_t n, int32_t L,
    uint32_t seed, uint32_t G, uint32_t S, unsigned long long *__restrict__ endpoint,
    unsigned long long *__restrict__ visits, unsigned long long *__restrict__ distinct) {
    __shared__ uint32_t lhist[9];
    if (CNT) {
        if (threadIdx.x < 9) lhist[threadIdx.x] = 0;
        __syncthreads();
    }
    // offs[n] counts only the walks whose start is a valid, non-isolated vertex
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t valid = offs[n];
    const bool active = w < valid;
    const bool full = (w & ~7ll) + 8 <= valid;
    int32_t cur = 0;
    Walker wk{};
    if (active) {
        const int32_t s = bsrc[w];
        const uint64_t r = (uint64_t)(w - offs[s]);
        wk = walker_init<SM>(walk_key(seed, (uint32_t)s, 0u, 0u, r, G, S));
        cur = s;
    }
    for (int32_t l = 1; l <= L; ++l) {
        if (active) cur = walker_step<SM>(vrec, col, cur, (uint32_t)l, wk);
        wave_merged_add(visits, cur, active);
        if (CNT) distinct8_count(cur, full, lhist);
    }
    wave_merged_add(endpoint, cur, active);
    if (CNT) distinct8_flush(lhist, distinct);
}

// Alg. 3 with the bucketed count: walks w0 .. w0 + wc of the bucket order, stepping on the
// 16-byte walk entries (one random read per step).  Walk w0 + i writes its position l to
// vlog[(l - 1) * wc + i] and its end vertex to elog[i]; the block counts its visits and ends
// per vertex bucket and writes the counts bucket-major: cnt[b * gridDim.x + blockIdx.x].
//
// kList (the walk-order ablation): the walks are taken in list order instead, walk w starting
// at lsrc[w] with rank lrank[w] among the walks of its start; a walk whose start is out of
// range or isolated (the call then fails) writes -1 everywhere, which the counting drops.
template <bool kList>
__device__ __forceinline__ bool log_walk_start(const int2 *__restrict__ vrec,
                                               const int32_t *__restrict__ bsrc,
                                               const int64_t *__restrict__ offs,
                                               const int32_t *__restrict__ lsrc,
                                               const uint32_t *__restrict__ lrank, int32_t n,
                                               int64_t w, int32_t *s, uint64_t *r) {
    if (kList) {
        const int32_t v = lsrc[w];
        if (v < 0 || v >= n || vrec[v].y == 0) return false;
        *s = v;
        *r = lrank[w];
        return true;
    }
    *s = bsrc[w];
    *r = (uint64_t)(w - offs[*s]);
    return true;
}

template <int SM, bool CNT, int WPL, bool kList>
__global__ __launch_bounds__(kWalkBlock) void walk_bouquet_log_kernel(
    const int2 *__restrict__ vrec, const int4 *__restrict__ nbr,
    const int32_t *__restrict__ bsrc, const int64_t *__restrict__ offs,
    const int32_t *__restrict__ lsrc, const uint32_t *__restrict__ lrank, int64_t nlist,
    int32_t n, int64_t w0,
    int64_t wc, int32_t L, uint32_t seed, uint32_t G, uint32_t S, int bsh, int32_t nbk,
    int32_t *__restrict__ vlog, int32_t *__restrict__ elog, long long *__restrict__ cnt_v,
    long long *__restrict__ cnt_e, unsigned long long *__restrict__ distinct) {
    extern __shared__ uint32_t lds_cnt[];
    __shared__ uint32_t lhist[9];
    uint32_t *cv = lds_cnt, *ce = lds_cnt + nbk;
    for (int i = threadIdx.x; i < 2 * nbk; i += kWalkBlock) lds_cnt[i] = 0;
    if (CNT && threadIdx.x < 9) lhist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t valid = min(wc, (kList ? nlist : offs[n]) - w0);
    // The block runs the 256-walk tiles blockIdx.x, blockIdx.x + gridDim.x, ... (the tiles the
    // scatter pass assigns to it); with WPL walks per lane it takes WPL of its tiles at a time
    // and steps their walks side by side, so WPL independent reads are in flight per lane.
    for (int64_t tile = blockIdx.x; tile * kWalkBlock < valid;
         tile += (int64_t)(CNT ? 1 : WPL) * gridDim.x) {
        const int64_t i = tile * kWalkBlock + threadIdx.x;
        if (!CNT) {
            int64_t ii[WPL];
            bool act[WPL], bad[WPL];
            Walker wk[WPL];
            WalkPos p[WPL];
#pragma unroll
            for (int k = 0; k < WPL; ++k) {
                ii[k] = (tile + (int64_t)k * gridDim.x) * kWalkBlock + threadIdx.x;
                act[k] = ii[k] < valid;
                bad[k] = false;
                p[k] = WalkPos{0, 0, 0};
                if (act[k]) {
                    int32_t s = 0;
                    uint64_t r = 0;
                    if (log_walk_start<kList>(vrec, bsrc, offs, lsrc, lrank, n, w0 + ii[k], &s,
                                              &r)) {
                        wk[k] = walker_init<SM>(walk_key(seed, (uint32_t)s, 0u, 0u, r, G, S));
                        p[k] = walk_pos(vrec, s);
                    } else {
                        act[k] = false;
                        bad[k] = true;
                    }
                }
            }
            for (int32_t l = 1; l <= L; ++l) {
#pragma unroll
                for (int k = 0; k < WPL; ++k)
                    if (act[k]) p[k] = walker_step_nbr<SM>(nbr, p[k], (uint32_t)p[k].v, (uint32_t)l,
                                                           wk[k]);
#pragma unroll
                for (int k = 0; k < WPL; ++k)
                    if (act[k]) {
                        __builtin_nontemporal_store(p[k].v, vlog + (int64_t)(l - 1) * wc + ii[k]);
                        atomicAdd(cv + (p[k].v >> bsh), 1u);
                    } else if (kList && bad[k]) {
                        vlog[(int64_t)(l - 1) * wc + ii[k]] = -1;
                    }
            }
#pragma unroll
            for (int k = 0; k < WPL; ++k)
                if (act[k]) {
                    __builtin_nontemporal_store(p[k].v, elog + ii[k]);
                    atomicAdd(ce + (p[k].v >> bsh), 1u);
                } else if (kList && bad[k]) {
                    elog[ii[k]] = -1;
                }
        } else {
            // every lane steps (idle ones in place) so the 8-lane groups stay converged
            bool act = i < valid;
            const bool in = act;
            const bool full = (i & ~7ll) + 8 <= valid;
            Walker wk{};
            WalkPos p{0, 0, 0};
            if (act) {
                int32_t s = 0;
                uint64_t r = 0;
                act = log_walk_start<kList>(vrec, bsrc, offs, lsrc, lrank, n, w0 + i, &s, &r);
                if (act) {
                    wk = walker_init<SM>(walk_key(seed, (uint32_t)s, 0u, 0u, r, G, S));
                    p = walk_pos(vrec, s);
                }
            }
            for (int32_t l = 1; l <= L; ++l) {
                if (act) {
                    p = walker_step_nbr<SM>(nbr, p, (uint32_t)p.v, (uint32_t)l, wk);
                    vlog[(int64_t)(l - 1) * wc + i] = p.v;
                    atomicAdd(cv + (p.v >> bsh), 1u);
                } else if (kList && in) {
                    vlog[(int64_t)(l - 1) * wc + i] = -1;
                }
                distinct8_count(p.v, full, lhist);
            }
            if (act) {
                elog[i] = p.v;
                atomicAdd(ce + (p.v >> bsh), 1u);
            } else if (kList && in) {
                elog[i] = -1;
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += kWalkBlock) {
        cnt_v[(int64_t)b * gridDim.x + blockIdx.x] = cv[b];
        cnt_e[(int64_t)b * gridDim.x + blockIdx.x] = ce[b];
    }
    if (CNT) distinct8_flush(lhist, distinct);
}

// Block-wide exclusive scan of one value per thread (blockDim.x == kWalkBlock).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *wave_tot) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wave_tot[w];
    __syncthreads();
    return before + inc - v;
}

// Log rows per local sort: groups of 32 rows x 256 walks for the visit log (longer runs per
// bucket) while its LDS fits 64 KiB, else 16; 16 for a single row (the end row), where the
// larger group only costs LDS.
constexpr int kSortRowsLog = 32, kSortRowsRow = 16;

// Scatter the log entries of the same blocks/tiles as the walk kernel into bucket order.
// Block k's entries of bucket b go to part[pos[b * gridDim.x + k] + 0, 1, ...], each stored
// as its 16-bit offset within the bucket (x & (2^bsh - 1); bsh <= 14), since the bucket of a
// position is known from pos: half the bytes of the vertex id for the scatter's stores and
// the histogram's loads.  Each
// group of kSortRows rows x 256 walks is first sorted by bucket in LDS, so every bucket
// leaves the block as one contiguous run.  The walks with a valid start are
// w0 .. min(w0 + wc, offs[n]) - 1, as in the walk kernel; other entries are not read.  With
// offs null all wc columns are read, and entries at r * wc + i >= limit are not.  With CHECK
// (the list of start vertices) an entry outside 0 .. n - 1 is dropped, as the count of
// source_bucket_count_kernel drops it.
template <int kSortRows, bool CHECK>
__global__ __launch_bounds__(kWalkBlock) void bucket_scatter_kernel(
    const int32_t *__restrict__ vlog, int32_t rows, int64_t wc, const int64_t *__restrict__ offs,
    int32_t n, int64_t w0, int bsh, int32_t nbk, const int64_t *__restrict__ pos,
    uint16_t *__restrict__ part, int64_t limit) {
    extern __shared__ unsigned char lds_raw[];
    int64_t *gpos = reinterpret_cast<int64_t *>(lds_raw);           // [nbk] global cursor
    uint32_t *lcnt = reinterpret_cast<uint32_t *>(gpos + nbk);       // [nbk] counts / cursors
    uint32_t *loff = lcnt + nbk;                                     // [nbk + 1] local offsets
    int32_t *keys = reinterpret_cast<int32_t *>(loff + nbk + 1);     // [kSortRows * kWalkBlock]
    uint32_t *wave_tot = reinterpret_cast<uint32_t *>(keys + kSortRows * kWalkBlock);  // [4]
    const int per = (nbk + kWalkBlock - 1) / kWalkBlock;  // buckets per thread in the scan
    for (int b = threadIdx.x; b < nbk; b += kWalkBlock) gpos[b] = pos[(int64_t)b * gridDim.x + blockIdx.x];
    const int64_t valid = rows <= 0 ? 0 : offs ? min(wc, offs[n] - w0) : wc;
    // The block's groups in order: tile blockIdx.x, blockIdx.x + gridDim.x, ..., and within a
    // tile kSortRows rows at a time.  The entries of the next group are loaded before the current
    // one is sorted, so their memory round trip overlaps the LDS passes (the barriers wait for
    // LDS operations only).
    int64_t tile = blockIdx.x;
    int32_t r0 = 0;
    int32_t v[kSortRows], nxt[kSortRows];
    const auto load_group = [&](int64_t t, int32_t r, int32_t(&dst)[kSortRows]) {
        const int64_t i = t * kWalkBlock + threadIdx.x;
        const int nr = min(kSortRows, rows - r);
#pragma unroll
        for (int k = 0; k < kSortRows; ++k) {
            const int64_t e = (int64_t)(r + k) * wc + i;
            dst[k] = (i < valid && k < nr && e < limit) ? __builtin_nontemporal_load(vlog + e) : -1;
        }
    };
    if (tile * kWalkBlock < valid) load_group(tile, r0, v);
    while (tile * kWalkBlock < valid) {
        int64_t tile2 = tile;
        int32_t r2 = r0 + kSortRows;
        if (r2 >= rows) {
            r2 = 0;
            tile2 += gridDim.x;
        }
        const bool more = tile2 * kWalkBlock < valid;
        if (more) load_group(tile2, r2, nxt);
        if (CHECK) {
#pragma unroll
            for (int k = 0; k < kSortRows; ++k)
                if (v[k] >= n) v[k] = -1;
        }
        {
            for (int b = threadIdx.x; b < nbk; b += kWalkBlock) lcnt[b] = 0;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kSortRows; ++k)
                if (v[k] >= 0) atomicAdd(lcnt + (v[k] >> bsh), 1u);
            __syncthreads();
            // local offsets: exclusive scan of lcnt, `per` buckets per thread
            uint32_t mine = 0;
            for (int q = 0; q < per; ++q) {
                const int b = threadIdx.x * per + q;
                if (b < nbk) mine += lcnt[b];
            }
            uint32_t run = block_exclusive_scan(mine, wave_tot);
            for (int q = 0; q < per; ++q) {
                const int b = threadIdx.x * per + q;
                if (b < nbk) {
                    loff[b] = run;
                    run += lcnt[b];
                }
            }
            if (threadIdx.x == kWalkBlock - 1) loff[nbk] = run;
            __syncthreads();
            for (int b = threadIdx.x; b < nbk; b += kWalkBlock) lcnt[b] = 0;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kSortRows; ++k) {
                if (v[k] >= 0) {
                    const int32_t b = v[k] >> bsh;
                    keys[loff[b] + atomicAdd(lcnt + b, 1u)] = v[k];
                }
            }
            __syncthreads();
            const uint32_t total = loff[nbk];
            const int32_t lmask = (1 << bsh) - 1;
            for (uint32_t j = threadIdx.x; j < total; j += kWalkBlock) {
                const int32_t x = keys[j];
                const int32_t b = x >> bsh;
                part[gpos[b] + (j - loff[b])] = (uint16_t)(x & lmask);
            }
            __syncthreads();
            for (int b = threadIdx.x; b < nbk; b += kWalkBlock) gpos[b] += loff[b + 1] - loff[b];
            __syncthreads();
        }
        if (!more) break;
#pragma unroll
        for (int k = 0; k < kSortRows; ++k) v[k] = nxt[k];
        tile = tile2;
        r0 = r2;
    }
}

static size_t scatter_lds_bytes(int32_t nbk, int sort_rows) {
    return sizeof(int64_t) * nbk + sizeof(uint32_t) * (2 * (size_t)nbk + 1) +
           sizeof(int32_t) * sort_rows * kWalkBlock + sizeof(uint32_t) * 4 + 16;
}

// Histogram of the bucket-ordered entries (16-bit offsets within their bucket): block j counts
// part[j*slice, (j+1)*slice) bucket by bucket in LDS and adds the nonzero bins to out.  Bucket
// b starts at pos[b * nblk].  The entries are read 16 bytes (8 entries) at a time, kHistUnroll
// reads in flight per thread, so the stream is not bound by the latency of one read per LDS
// update.
constexpr int kHistUnroll = 4;

__device__ __forceinline__ void hist_add(uint32_t *lds_h, uint32_t x) { atomicAdd(lds_h + x, 1u); }

__device__ __forceinline__ void hist_add2(uint32_t *lds_h, uint32_t two) {
    hist_add(lds_h, two & 0xFFFFu);
    hist_add(lds_h, two >> 16);
}

__global__ __launch_bounds__(kWalkBlock) void bucket_hist_kernel(
    const uint16_t *__restrict__ part, const int64_t *__restrict__ pos, int nblk, int bsh,
    int32_t nbk, int64_t slice, int32_t n, unsigned long long *__restrict__ out) {
    extern __shared__ uint32_t lds_h[];
    const int32_t bins = 1 << bsh;
    const int64_t total = pos[(int64_t)nbk * nblk];
    const int64_t s0 = (int64_t)blockIdx.x * slice;
    const int64_t s1 = min(total, s0 + slice);
    if (s0 >= s1) return;
    int32_t lo = 0, hi = nbk;  // largest bucket b with start(b) <= s0
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (pos[(int64_t)mid * nblk] <= s0)
            lo = mid;
        else
            hi = mid;
    }
    const nbr_vec4 *part8 = reinterpret_cast<const nbr_vec4 *>(part);  // 8 entries per 16 bytes
    for (int32_t b = lo; b < nbk; ++b) {
        const int64_t bs = pos[(int64_t)b * nblk];
        const int64_t be = pos[(int64_t)(b + 1) * nblk];
        if (bs >= s1) break;
        const int64_t a = max(s0, bs), z = min(s1, be);
        if (a >= z) continue;
        for (int i = threadIdx.x; i < bins; i += kWalkBlock) lds_h[i] = 0;
        __syncthreads();
        // entries a .. z: an unaligned head and tail one by one, whole 16-byte words between
        const int64_t q0 = (a + 7) >> 3, q1 = z >> 3;
        if (q0 >= q1) {
            for (int64_t i = a + threadIdx.x; i < z; i += kWalkBlock) hist_add(lds_h, part[i]);
        } else {
            if (a + threadIdx.x < 8 * q0) hist_add(lds_h, part[a + threadIdx.x]);
            if (8 * q1 + threadIdx.x < z) hist_add(lds_h, part[8 * q1 + threadIdx.x]);
            for (int64_t q = q0 + threadIdx.x; q < q1; q += kHistUnroll * kWalkBlock) {
                nbr_vec4 x[kHistUnroll];
#pragma unroll
                for (int u = 0; u < kHistUnroll; ++u)
                    if (q + u * kWalkBlock < q1)
                        x[u] = __builtin_nontemporal_load(part8 + q + u * kWalkBlock);
#pragma unroll
                for (int u = 0; u < kHistUnroll; ++u)
                    if (q + u * kWalkBlock < q1) {
                        hist_add2(lds_h, (uint32_t)x[u].x);
                        hist_add2(lds_h, (uint32_t)x[u].y);
                        hist_add2(lds_h, (uint32_t)x[u].z);
                        hist_add2(lds_h, (uint32_t)x[u].w);
                    }
            }
        }
        __syncthreads();
        const int64_t base = (int64_t)b << bsh;
        for (int i = threadIdx.x; i < bins; i += kWalkBlock) {
            const uint32_t c = lds_h[i];
            if (c && base + i < n) atomicAdd(out + base + i, (unsigned long long)c);
        }
        __syncthreads();
    }
}

struct EventSet {
    hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~EventSet() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Histogram slice for a log of at most `bound` entries.
static int64_t hist_slice(int64_t bound) {
    return std::min(kHistSliceMax, std::max(kHistSliceMin, (bound + kHistBlocks - 1) / kHistBlocks));
}

// Bucketed count of one log (rows x wc entries, `valid` walks per row) into out.
static int bucket_count(const int32_t *vlog, int32_t rows, int64_t wc, const int64_t *offs,
                        int64_t w0, int nblk, int bsh, int32_t nbk, int64_t *cnt, int64_t *pos,
                        void *scan_tmp, uint16_t *part, int32_t n, unsigned long long *out,
                        hipStream_t s, int64_t limit, bool check = false) {
    const int64_t ncnt = (int64_t)nbk * nblk;
    SABA_TRY(scan_i64(cnt, pos, ncnt, scan_tmp, s));
    const size_t lds_log = scatter_lds_bytes(nbk, kSortRowsLog);
    const size_t lds_row = scatter_lds_bytes(nbk, kSortRowsRow);
    const bool tall = rows >= kSortRowsLog && lds_log <= 65536;
    if (check && tall)
        bucket_scatter_kernel<kSortRowsLog, true><<<nblk, kWalkBlock, lds_log, s>>>(
            vlog, rows, wc, offs, n, w0, bsh, nbk, pos, part, limit);
    else if (check)
        bucket_scatter_kernel<kSortRowsRow, true><<<nblk, kWalkBlock, lds_row, s>>>(
            vlog, rows, wc, offs, n, w0, bsh, nbk, pos, part, limit);
    else if (tall)
        bucket_scatter_kernel<kSortRowsLog, false><<<nblk, kWalkBlock, lds_log, s>>>(
            vlog, rows, wc, offs, n, w0, bsh, nbk, pos, part, limit);
    else
        bucket_scatter_kernel<kSortRowsRow, false><<<nblk, kWalkBlock, lds_row, s>>>(
            vlog, rows, wc, offs, n, w0, bsh, nbk, pos, part, limit);
    SABA_HIP_TRY(hipGetLastError());
    const int64_t bound = (int64_t)rows * wc;  // at least the number of entries counted
    const int64_t slice = hist_slice(bound);
    const unsigned hblocks = (unsigned)std::max<int64_t>(1, (bound + slice - 1) / slice);
    bucket_hist_kernel<<<hblocks, kWalkBlock, sizeof(uint32_t) << bsh, s>>>(
        part, pos, nblk, bsh, nbk, slice, n, out);
    SABA_HIP_TRY(hipGetLastError());
    return SABA_OK;
}

// Launches of the kernel instantiations for sampler sm and branching statistics on/off.
template <int SM>
static void launch_naive_sm(bool cnt, unsigned blocks, hipStream_t s, const Graph *g,
                            const saba_walk_params *p, const uint32_t *rank,
                            unsigned long long *ep, unsigned long long *vi, int32_t *err,
                            unsigned long long *dist) {
    if (cnt)
        walk_naive_kernel<SM, true><<<blocks, kWalkBlock, 0, s>>>(
            g->vrec, g->col_idx, p->d_sources, rank, p->n_walks, p->length, p->seed, p->group,
            p->spread, g->n, ep, vi, err, dist);
    else
        walk_naive_kernel<SM, false><<<blocks, kWalkBlock, 0, s>>>(
            g->vrec, g->col_idx, p->d_sources, rank, p->n_walks, p->length, p->seed, p->group,
            p->spread, g->n, ep, vi, err, dist);
}

template <int SM>
static void launch_atomic_sm(bool cnt, unsigned blocks, hipStream_t s, const Graph *g,
                             const saba_walk_params *p, const int32_t *bsrc, const int64_t *offs,
                             unsigned long long *ep, unsigned long long *vi,
                             unsigned long long *dist) {
    if (cnt)
        walk_bouquet_atomic_kernel<SM, true><<<blocks, kWalkBlock, 0, s>>>(
            g->vrec, g->col_idx, bsrc, offs, g->n, p->length, p->seed, p->group, p->spread, ep,
            vi, dist);
    else
        walk_bouquet_atomic_kernel<SM, false><<<blocks, kWalkBlock, 0, s>>>(
            g->vrec, g->col_idx, bsrc, offs, g->n, p->length, p->seed, p->group, p->spread, ep,
            vi, dist);
}

template <int SM, bool LIST>
static void launch_log_sm2(bool cnt, int wpl, int nblk, size_t lds, hipStream_t s,
                           const Graph *g, const saba_walk_params *p, const int32_t *bsrc,
                           const int64_t *offs, const uint32_t *lrank, int64_t w0, int64_t wc,
                           int bsh, int32_t nbk, int32_t *vlog, int32_t *elog, long long *cnt_v,
                           long long *cnt_e, unsigned long long *dist) {
#define SABA_LOG_LAUNCH(C, W)                                                                   \
    walk_bouquet_log_kernel<SM, C, W, LIST><<<nblk, kWalkBlock, lds, s>>>(                       \
        g->vrec, g->nbr, bsrc, offs, p->d_sources, lrank, p->n_walks, g->n, w0, wc, p->length,  \
        p->seed, p->group, p->spread, bsh, nbk, vlog, elog, cnt_v, cnt_e, dist)
    if (cnt)
        SABA_LOG_LAUNCH(true, 1);
    else if (wpl >= 4)
        SABA_LOG_LAUNCH(false, 4);
    else if (wpl == 2)
        SABA_LOG_LAUNCH(false, 2);
    else
        SABA_LOG_LAUNCH(false, 1);
#undef SABA_LOG_LAUNCH
}

// lrank != null: the walks in list order (the naive-log ablation)
template <int SM>
static void launch_log_sm(bool cnt, int wpl, int nblk, size_t lds, hipStream_t s,
                          const Graph *g, const saba_walk_params *p, const int32_t *bsrc,
                          const int64_t *offs, const uint32_t *lrank, int64_t w0, int64_t wc,
                          int bsh, int32_t nbk, int32_t *vlog, int32_t *elog, long long *cnt_v,
                          long long *cnt_e, unsigned long long *dist) {
    if (lrank)
        launch_log_sm2<SM, true>(cnt, wpl, nblk, lds, s, g, p, bsrc, offs, lrank, w0, wc, bsh, nbk,
                                 vlog, elog, cnt_v, cnt_e, dist);
    else
        launch_log_sm2<SM, false>(cnt, wpl, nblk, lds, s, g, p, bsrc, offs, lrank, w0, wc, bsh,
                                  nbk, vlog, elog, cnt_v, cnt_e, dist);
}

// Uniform sources: walk j starts at pool[floor(h_j npool / 2^32)] with
// h_j = Murmur2(LE32(j mod 2^32) | LE32(j / 2^32), seed).
__global__ void uniform_sources_kernel(const int32_t *__restrict__ pool, int64_t npool,
                                       uint32_t seed, int64_t W, int32_t *__restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < W;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = hash_w2((uint32_t)j, (uint32_t)((uint64_t)j >> 32), seed);
        out[j] = pool[(int64_t)(((uint64_t)h * (uint64_t)npool) >> 32)];
    }
}

// The pool of the uniform source mode, built once per handle from the host copy of the CSR.
static int ensure_pool(Graph *g, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g->pool_mu);
    if (g->npool >= 0) return SABA_OK;
    std::vector<int32_t> pool;
    const int32_t *rp = g->h_row_ptr.data();
    for (int32_t v = 0; v < g->n; ++v)
        if (rp[v + 1] > rp[v]) pool.push_back(v);
    if (!pool.empty()) {
        SABA_HIP_TRY(hipMalloc(&g->pool, sizeof(int32_t) * pool.size()));
        SABA_HIP_TRY(hipMemcpyAsync(g->pool, pool.data(), sizeof(int32_t) * pool.size(),
                                    hipMemcpyHostToDevice, s));
        SABA_HIP_TRY(hipStreamSynchronize(s));
    }
    g->npool = (int64_t)pool.size();
    return SABA_OK;
}

// Events of one call's per-chunk timing, destroyed with the call.
struct EventList {
    std::vector<hipEvent_t> e;
    int create(int64_t k) {
        e.assign((size_t)k, nullptr);
        for (auto &x : e) SABA_HIP_TRY(hipEventCreate(&x));
        return SABA_OK;
    }
    ~EventList() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// The walk call's second stream (default priority) and the events that hand the visit-log
// buffers between the walks and the counting passes, created once per handle.
static int ensure_walk_pipeline(Graph *g) {
    if (g->walk_aux) return SABA_OK;
    hipStream_t st = nullptr;
    SABA_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    for (auto &e : g->walk_ev) {
        if (e) continue;
        const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) {
            (void)hipStreamDestroy(st);
            set_error(std::string("hipEventCreateWithFlags: ") + hipGetErrorString(r));
            return SABA_E_HIP;
        }
    }
    g->walk_aux = st;
    return SABA_OK;
}

// The fixed scratch of saba_walks_noalloc: one region per device, held until the process ends.
// Host code uses only the address hipGetSymbolAddress returns for the current device (the
// array's name is a host-side stand-in, not a device address).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int noalloc_scratch(void **out) {
    int dev = 0;
    SABA_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the fixed-scratch table");
        return SABA_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        SABA_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_error("hipGetSymbolAddress returned no address for the fixed scratch");
            return SABA_E_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SABA_OK;
}

// Scratch of one walk call: the handle's grow-only buffers, or a fixed device region carved
// front to back (the entry point that allocates nothing).  Each slot is taken once per call.
struct WalkArena {
    Graph *g = nullptr;
    char *base = nullptr;  // fixed region, or null for the handle's buffers
    size_t cap = 0, used = 0;
    static size_t up(size_t x) { return (x + 255) & ~(size_t)255; }
    size_t left() const { return up(used) >= cap ? 0 : cap - up(used); }
    template <class T>
    int get(int slot, size_t bytes, T **out) {
        if (!base) {
            SABA_TRY(g->walk_scratch[slot].ensure(bytes));
            *out = g->walk_scratch[slot].as<T>();
            return SABA_OK;
        }
        if (bytes > left()) {
            set_error("the walk call needs more scratch than the fixed region holds");
            return SABA_E_INVALID;
        }
        *out = reinterpret_cast<T *>(base + up(used));
        used = up(used) + bytes;
        return SABA_OK;
    }
};

static int walks_impl(Graph *g, const saba_walk_params *p, int64_t *d_endpoint,
                      int64_t *d_visits, saba_stats *st, hipStream_t s, WalkArena &ar) {
    const int64_t W = p->n_walks;
    const int32_t n = g->n;
    const int32_t L = p->length;
    if (W < 0 || L < 0 || p->group < 1 || p->spread > 31 ||
        (p->group > 1 && ((uint64_t)(p->group - 1) << p->spread) > 0xFFFFFFFFull) ||
        (p->source_mode != SABA_SOURCES_EXPLICIT && p->source_mode != SABA_SOURCES_UNIFORM) ||
        (W > 0 && p->source_mode == SABA_SOURCES_EXPLICIT && !p->d_sources) || !d_endpoint ||
        !d_visits ||
        (p->mode != SABA_WALK_NAIVE && p->mode != SABA_WALK_BOUQUET &&
         p->mode != SABA_WALK_NAIVE_LOG) || p->sampler < 0 ||
        p->sampler > SABA_SAMPLER_LITERAL ||
        (p->mode != SABA_WALK_BOUQUET && W >= ((int64_t)1 << 31))) {
        set_error("invalid walk parameters");
        return SABA_E_INVALID;
    }
    if ((__int128)W * (L > 0 ? L : 1) >= ((__int128)1 << 62)) {
        set_error("walk count too large");
        return SABA_E_OVERFLOW;
    }
    if (W > (int64_t)0xFFFFFFFFll) {  // walk keys carry a 32-bit walk index
        set_error("more than 2^32 - 1 walks: walks of one start would repeat");
        return SABA_E_OVERFLOW;
    }
    EventSet ev;
    const bool timing = st && p->time_kernels;
    if (timing)
        for (auto &e : ev.e) SABA_HIP_TRY(hipEventCreate(&e));
    if (timing) SABA_HIP_TRY(hipEventRecord(ev.e[0], s));

    saba_walk_params drawn;
    if (W > 0 && p->source_mode == SABA_SOURCES_UNIFORM) {
        SABA_TRY(ensure_pool(g, s));
        if (g->npool == 0) {
            set_error("uniform sources need a vertex with an edge");
            return SABA_E_INVALID;
        }
        int32_t *src = nullptr;
        SABA_TRY(ar.get(7, sizeof(int32_t) * (size_t)W, &src));
        uniform_sources_kernel<<<(unsigned)std::min<int64_t>((W + 255) / 256, 1 << 16), 256, 0, s>>>(
            g->pool, g->npool, p->seed, W, src);
        SABA_HIP_TRY(hipGetLastError());
        drawn = *p;
        drawn.d_sources = src;
        drawn.source_mode = SABA_SOURCES_EXPLICIT;
        p = &drawn;
    }

    int32_t *err = nullptr;
    SABA_TRY(ar.get(3, sizeof(int32_t), &err));
    SABA_HIP_TRY(hipMemsetAsync(err, 0, sizeof(int32_t), s));
    SABA_HIP_TRY(hipMemsetAsync(d_endpoint, 0, sizeof(int64_t) * (size_t)n, s));
    SABA_HIP_TRY(hipMemsetAsync(d_visits, 0, sizeof(int64_t) * (size_t)n, s));
    auto *ep = reinterpret_cast<unsigned long long *>(d_endpoint);
    auto *vi = reinterpret_cast<unsigned long long *>(d_visits);
    const bool cnt = p->d_distinct != nullptr;
    auto *dist = reinterpret_cast<unsigned long long *>(p->d_distinct);
    if (cnt) SABA_HIP_TRY(hipMemsetAsync(p->d_distinct, 0, sizeof(int64_t) * 9, s));
    const int sm = p->sampler;
    bool counted_separately = false;
    int64_t launches = W > 0 ? 1 : 0;  // walk-kernel launches (visit-log chunks)

    if (W > 0 && p->mode == SABA_WALK_NAIVE) {
        // rank of each walk among the walks of its start vertex, in list order
        unsigned long long *counts = nullptr;
        int64_t *offs = nullptr;
        int32_t *sorted_src = nullptr;
        uint32_t *iota = nullptr, *rank = nullptr;
        void *sort_tmp = nullptr;
        SABA_TRY(ar.get(0, sizeof(int64_t) * (size_t)n, &counts));
        SABA_TRY(ar.get(1, sizeof(int64_t) * ((size_t)n + 1) + scan_tmp_bytes(n), &offs));
        SABA_TRY(ar.get(2, sizeof(int32_t) * (size_t)W, &sorted_src));
        SABA_TRY(ar.get(4, sizeof(uint32_t) * 2 * (size_t)W, &iota));
        SABA_TRY(ar.get(5, sizeof(uint32_t) * (size_t)W, &rank));
        void *scan_tmp = offs + n + 1;
        uint32_t *sorted_j = iota + W;
        size_t sort_bytes = 0;
        SABA_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, p->d_sources,
                                                        sorted_src, iota, sorted_j, (int)W, 0,
                                                        32, s));
        SABA_TRY(ar.get(6, std::max<size_t>(sort_bytes, 1), &sort_tmp));
        SABA_HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int64_t) * (size_t)n, s));
        const unsigned cblocks =
            (unsigned)std::min<int64_t>((W + kWalkBlock - 1) / kWalkBlock, 1 << 16);
        source_count_kernel<<<cblocks, kWalkBlock, 0, s>>>(p->d_sources, W, g->vrec, n, counts,
                                                            err);
        SABA_HIP_TRY(hipGetLastError());
        SABA_TRY(scan_i64(reinterpret_cast<int64_t *>(counts), offs, n, scan_tmp, s));
        iota_kernel<<<cblocks, kWalkBlock, 0, s>>>(iota, W);
        SABA_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(sort_tmp, sort_bytes,
                                                        p->d_sources, sorted_src, iota, sorted_j,
                                                        (int)W, 0, 32, s));
        list_rank_kernel<<<cblocks, kWalkBlock, 0, s>>>(sorted_src, sorted_j, W, offs, g->vrec, n,
                                                         rank);
        SABA_HIP_TRY(hipGetLastError());
        if (timing) SABA_HIP_TRY(hipEventRecord(ev.e[1], s));
        const unsigned blocks = (unsigned)((W + kWalkBlock - 1) / kWalkBlock);
        switch (sm) {
            case SABA_SAMPLER_KEYED:
                launch_naive_sm<SABA_SAMPLER_KEYED>(cnt, blocks, s, g, p, rank, ep, vi, err, dist);
                break;
            case SABA_SAMPLER_KEYED_MOD:
                launch_naive_sm<SABA_SAMPLER_KEYED_MOD>(cnt, blocks, s, g, p, rank, ep, vi, err,
                                                        dist);
                break;
            case SABA_SAMPLER_STREAM_MOD:
                launch_naive_sm<SABA_SAMPLER_STREAM_MOD>(cnt, blocks, s, g, p, rank, ep, vi, err,
                                                         dist);
                break;
            default:
                launch_naive_sm<SABA_SAMPLER_LITERAL>(cnt, blocks, s, g, p, rank, ep, vi, err,
                                                      dist);
        }
        SABA_HIP_TRY(hipGetLastError());
        if (timing) SABA_HIP_TRY(hipEventRecord(ev.e[2], s));
    } else if (W > 0) {
        // bucket order of the walks
        unsigned long long *counts = nullptr;
        int64_t *offs = nullptr;
        int32_t *bsrc = nullptr;
        SABA_TRY(ar.get(0, sizeof(int64_t) * (size_t)n, &counts));
        SABA_TRY(ar.get(1, sizeof(int64_t) * ((size_t)n + 1) + scan_tmp_bytes(n), &offs));
        SABA_TRY(ar.get(2, sizeof(int32_t) * (size_t)W, &bsrc));
        void *scan_tmp = offs + n + 1;
        SABA_HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int64_t) * (size_t)n, s));
        const unsigned cblocks =
            (unsigned)std::min<int64_t>((W + kWalkBlock - 1) / kWalkBlock, 1 << 16);
        // walks per start vertex counted into `counts`: offsets and the bucket order follow
        const auto order_walks = [&]() -> int {
            SABA_TRY(scan_i64(reinterpret_cast<int64_t *>(counts), offs, n, scan_tmp, s));
            const unsigned fblocks = (unsigned)std::min<int64_t>(
                (W + (int64_t)kWalkBlock * kFillRun - 1) / ((int64_t)kWalkBlock * kFillRun), 1 << 16);
            source_fill_kernel<<<fblocks, kWalkBlock, 0, s>>>(offs, n, bsrc);
            SABA_HIP_TRY(hipGetLastError());
            return SABA_OK;
        };

        int bsh = 12;
        while (bsh < kMaxBucketShift && (((int64_t)n + (1 << bsh) - 1) >> bsh) > kMaxBuckets) ++bsh;
        const int32_t nbk = (int32_t)(((int64_t)n + (1 << bsh) - 1) >> bsh);
        const bool list = p->mode == SABA_WALK_NAIVE_LOG;
        if (list && nbk > kMaxBuckets) {
            set_error("the naive-log order needs at most 2^25 vertices (the bucketed count)");
            return SABA_E_INVALID;
        }
        if (nbk > kMaxBuckets) {
            source_count_kernel<<<cblocks, kWalkBlock, 0, s>>>(p->d_sources, W, g->vrec, n, counts,
                                                                err);
            SABA_HIP_TRY(hipGetLastError());
            SABA_TRY(order_walks());
            if (timing) SABA_HIP_TRY(hipEventRecord(ev.e[1], s));
            unsigned blocks = (unsigned)((W + kWalkBlock - 1) / kWalkBlock);
            switch (sm) {
                case SABA_SAMPLER_KEYED:
                    launch_atomic_sm<SABA_SAMPLER_KEYED>(cnt, blocks, s, g, p, bsrc, offs, ep, vi,
                                                         dist);
                    break;
                case SABA_SAMPLER_KEYED_MOD:
                    launch_atomic_sm<SABA_SAMPLER_KEYED_MOD>(cnt, blocks, s, g, p, bsrc, offs, ep,
                                                             vi, dist);
                    break;
                case SABA_SAMPLER_STREAM_MOD:
                    launch_atomic_sm<SABA_SAMPLER_STREAM_MOD>(cnt, blocks, s, g, p, bsrc, offs,
                                                              ep, vi, dist);
                    break;
                default:
                    launch_atomic_sm<SABA_SAMPLER_LITERAL>(cnt, blocks, s, g, p, bsrc, offs, ep,
                                                           vi, dist);
            }
            SABA_HIP_TRY(hipGetLastError());
            if (timing) SABA_HIP_TRY(hipEventRecord(ev.e[2], s));
        } else {
            counted_separately = true;
            // chunks of walks whose visit log fits kLogCap entries, and with the handle's buffers
            // the requested number of chunks (by default kPipeChunks while a chunk keeps
            // kPipeMinWalks walks, one full round of the persistent grid)
            int64_t wc = std::max<int64_t>(kWalkBlock, kLogCap / std::max<int32_t>(L, 1));
            wc = std::min<int64_t>(W, wc / kWalkBlock * kWalkBlock);
            const int want_blocks = g->cfg.walk_blocks > 0 ? g->cfg.walk_blocks : kPersistBlocks;
            const int wpl = g->cfg.walks_per_lane > 0 ? g->cfg.walks_per_lane : 1;
            if (!ar.base) {
                const int64_t want_ch =
                    g->cfg.walk_chunks > 0 ? g->cfg.walk_chunks
                                           : std::max<int64_t>(1, std::min<int64_t>(kPipeChunks, W / kPipeMinWalks));
                const int64_t per = ((W + want_ch - 1) / want_ch + kWalkBlock - 1) / kWalkBlock * kWalkBlock;
                wc = std::min<int64_t>(wc, std::max<int64_t>(kWalkBlock, per));
            }
            // With the handle's buffers and more than one chunk, the counting of chunk k runs on
            // a second stream while chunk k + 1 walks: the logs and the per-block bucket counts
            // are double-buffered (the walks are bound by the rate of random line fetches, the
            // counting passes stream, so they share the memory system well).  A fixed region
            // keeps one buffer set and runs everything in order on the caller's stream.
            const bool overlap = !ar.base && W > wc;
            const int nbuf = overlap ? 2 : 1;
            // scratch of the chunk loop for chunks of c walks: the visit and endpoint logs, the
            // bucket-ordered entries of the largest log (the visit log, or the start list) and
            // the per-bucket counters (nbuf sets of per-block counts, one scan) with their scan
            const auto chunk_bytes = [&](int64_t c, size_t *lg, size_t *pt, size_t *cn) {
                const int nb = (int)std::min<int64_t>(want_blocks, (c + kWalkBlock - 1) / kWalkBlock);
                const int64_t nc = (int64_t)nbk * nb;
                *lg = sizeof(int32_t) * (size_t)(std::max<int64_t>((int64_t)L * c, 1) + c);
                *pt = sizeof(uint16_t) * (size_t)std::max<int64_t>((int64_t)std::max<int32_t>(L, 1) * c, W);
                *cn = sizeof(int64_t) * (size_t)(2 * nbuf * nc + nc + 2) + scan_tmp_bytes(nc);
                return nbuf * WalkArena::up(*lg) + WalkArena::up(*pt) + WalkArena::up(*cn);
            };
            size_t lg_b = 0, pt_b = 0, cn_b = 0;
            if (ar.base)  // a fixed region: shorter chunks until the chunk scratch fits
                while (wc > kWalkBlock && chunk_bytes(wc, &lg_b, &pt_b, &cn_b) > ar.left())
                    wc = std::max<int64_t>(kWalkBlock, (wc / 2) / kWalkBlock * kWalkBlock);
            chunk_bytes(wc, &lg_b, &pt_b, &cn_b);
            const int nblk = (int)std::min<int64_t>(want_blocks, (wc + kWalkBlock - 1) / kWalkBlock);
            const int64_t ncnt = (int64_t)nbk * nblk;
            const int64_t logn = std::max<int64_t>((int64_t)L * wc, 1);
            const size_t lg_stride = WalkArena::up(lg_b) / sizeof(int32_t);
            int32_t *vlog_all = nullptr;
            uint16_t *part = nullptr;
            int64_t *cnt_all = nullptr;
            SABA_TRY(ar.get(4, (size_t)(nbuf - 1) * WalkArena::up(lg_b) + lg_b, &vlog_all));
            SABA_TRY(ar.get(5, pt_b, &part));
            SABA_TRY(ar.get(6, cn_b, &cnt_all));
            int64_t *pos = cnt_all + 2 * nbuf * ncnt;  // ncnt + 1 entries
            void *ctmp = pos + ncnt + 2;
            // the start-count phase uses the first counter set
            int64_t *cnt_v = cnt_all;
            // walks per start vertex, counted like the visits: the start list read as a log of
            // up to 32 rows (per bucket and block in LDS, then bucket order, then a histogram
            // per bucket), then starts without neighbours cleared and flagged
            const int32_t srows = (int32_t)std::min<int64_t>(
                kSortRowsLog, std::max<int64_t>(1, W / kWalkBlock));
            const int64_t wcs = ((W + srows - 1) / srows + kWalkBlock - 1) / kWalkBlock * kWalkBlock;
            const int sblk = (int)std::min<int64_t>(nblk, wcs / kWalkBlock);
            source_bucket_count_kernel<<<sblk, kWalkBlock, sizeof(uint32_t) * nbk, s>>>(
                p->d_sources, W, srows, wcs, n, bsh, nbk, reinterpret_cast<long long *>(cnt_v), err);
            SABA_HIP_TRY(hipGetLastError());
            SABA_TRY(bucket_count(p->d_sources, srows, wcs, nullptr, 0, sblk, bsh, nbk, cnt_v, pos,
                                  ctmp, part, n, counts, s, W, true));
            start_check_kernel<<<(unsigned)std::min<int64_t>((n + kWalkBlock - 1) / kWalkBlock, 1 << 16),
                                 kWalkBlock, 0, s>>>(g->vrec, n, counts, err);
            SABA_HIP_TRY(hipGetLastError());
            SABA_TRY(order_walks());
            // naive-log order: the rank of each walk among the walks of its start, in list
            // order (a stable sort of the list by start, then the position within the start)
            uint32_t *lrank = nullptr;
            if (list) {
                int32_t *sorted_src = nullptr;
                uint32_t *iota = nullptr;
                void *sort_tmp = nullptr;
                SABA_TRY(ar.get(8, sizeof(int32_t) * (size_t)W, &sorted_src));
                SABA_TRY(ar.get(9, sizeof(uint32_t) * 2 * (size_t)W, &iota));
                SABA_TRY(ar.get(10, sizeof(uint32_t) * (size_t)W, &lrank));
                size_t sort_bytes = 0;
                SABA_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, p->d_sources,
                                                                sorted_src, iota, iota + W, (int)W,
                                                                0, 32, s));
                SABA_TRY(ar.get(11, std::max<size_t>(sort_bytes, 1), &sort_tmp));
                iota_kernel<<<cblocks, kWalkBlock, 0, s>>>(iota, W);
                SABA_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(sort_tmp, sort_bytes, p->d_sources,
                                                                sorted_src, iota, iota + W, (int)W,
                                                                0, 32, s));
                list_rank_kernel<<<cblocks, kWalkBlock, 0, s>>>(sorted_src, iota + W, W, offs,
                                                                 g->vrec, n, lrank);
                SABA_HIP_TRY(hipGetLastError());
            }
            hipStream_t sc = s;  // the counting stream
            if (overlap) {
                SABA_TRY(ensure_walk_pipeline(g));
                sc = g->walk_aux;
            }
            const int64_t nchunks = (W + wc - 1) / wc;
            launches = nchunks;
            EventList tev;  // per chunk: walk start / end on s, count start / end on sc
            if (timing) SABA_TRY(tev.create(4 * nchunks));
            for (int64_t k = 0; k < nchunks; ++k) {
                const int64_t w0 = k * wc;
                const int64_t this_wc = std::min<int64_t>(wc, W - w0);
                const int bi = (int)(k % nbuf);
                int32_t *vl = vlog_all + (size_t)bi * lg_stride;
                int32_t *el = vl + logn;
                auto *cv = reinterpret_cast<long long *>(cnt_all + (int64_t)bi * 2 * ncnt);
                auto *ce = cv + ncnt;
                // buffer bi is free once the counting of chunk k - 2 has read it
                if (overlap && k >= 2) SABA_HIP_TRY(hipStreamWaitEvent(s, g->walk_ev[2 + bi], 0));
                if (timing) SABA_HIP_TRY(hipEventRecord(tev.e[4 * k], s));
                const size_t lds = sizeof(uint32_t) * 2 * nbk;
                switch (sm) {
                    case SABA_SAMPLER_KEYED:
                        launch_log_sm<SABA_SAMPLER_KEYED>(cnt, wpl, nblk, lds, s, g, p, bsrc, offs, lrank, w0,
                                                          this_wc, bsh, nbk, vl, el, cv, ce, dist);
                        break;
                    case SABA_SAMPLER_KEYED_MOD:
                        launch_log_sm<SABA_SAMPLER_KEYED_MOD>(cnt, wpl, nblk, lds, s, g, p, bsrc, offs, lrank,
                                                              w0, this_wc, bsh, nbk, vl, el, cv, ce,
                                                              dist);
                        break;
                    case SABA_SAMPLER_STREAM_MOD:
                        launch_log_sm<SABA_SAMPLER_STREAM_MOD>(cnt, wpl, nblk, lds, s, g, p, bsrc,
                                                               offs, lrank, w0, this_wc, bsh, nbk, vl, el,
                                                               cv, ce, dist);
                        break;
                    default:
                        launch_log_sm<SABA_SAMPLER_LITERAL>(cnt, wpl, nblk, lds, s, g, p, bsrc, offs, lrank,
                                                            w0, this_wc, bsh, nbk, vl, el, cv, ce,
                                                            dist);
                }
                SABA_HIP_TRY(hipGetLastError());
                if (timing) SABA_HIP_TRY(hipEventRecord(tev.e[4 * k + 1], s));
                if (overlap) {
                    SABA_HIP_TRY(hipEventRecord(g->walk_ev[bi], s));
                    SABA_HIP_TRY(hipStreamWaitEvent(sc, g->walk_ev[bi], 0));
                }
                if (timing) SABA_HIP_TRY(hipEventRecord(tev.e[4 * k + 2], sc));
                if (L > 0)
                    SABA_TRY(bucket_count(vl, L, this_wc, offs, w0, nblk, bsh, nbk,
                                          reinterpret_cast<int64_t *>(cv), pos, ctmp, part, n, vi,
                                          sc, (int64_t)L * this_wc));
                SABA_TRY(bucket_count(el, 1, this_wc, offs, w0, nblk, bsh, nbk,
                                      reinterpret_cast<int64_t *>(ce), pos, ctmp, part, n, ep, sc,
                                      this_wc));
                if (timing) SABA_HIP_TRY(hipEventRecord(tev.e[4 * k + 3], sc));
                if (overlap) SABA_HIP_TRY(hipEventRecord(g->walk_ev[2 + bi], sc));
            }
            // the caller's stream sees the last counting pass (and with it every earlier one)
            if (overlap)
                SABA_HIP_TRY(hipStreamWaitEvent(s, g->walk_ev[2 + (int)((nchunks - 1) % nbuf)], 0));
            float walk_ms = 0.f, count_ms = 0.f;
            if (timing) {
                SABA_HIP_TRY(hipEventSynchronize(tev.e[4 * (nchunks - 1) + 3]));
                for (int64_t k = 0; k < nchunks; ++k) {
                    float a = 0.f, b = 0.f;
                    SABA_HIP_TRY(hipEventElapsedTime(&a, tev.e[4 * k], tev.e[4 * k + 1]));
                    SABA_HIP_TRY(hipEventElapsedTime(&b, tev.e[4 * k + 2], tev.e[4 * k + 3]));
                    walk_ms += a;
                    count_ms += b;
                }
            }
            if (st && timing) {
                st->kernel_ms = walk_ms;
                st->count_ms = count_ms;
            }
        }
    }
    if (timing) SABA_HIP_TRY(hipEventRecord(ev.e[4], s));
    int32_t h_err = 0;
    SABA_HIP_TRY(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipStreamSynchronize(s));
    if (h_err) {
        set_error("a walk source is out of range or an isolated vertex");
        return SABA_E_INVALID;
    }
    if (st) {
        const double kms = st->kernel_ms, cms = st->count_ms;
        *st = saba_stats{};
        st->walks = W;
        st->walk_steps = W * (int64_t)L;
        st->batches = launches;
        if (timing) {
            float a = 0.f, b = 0.f;
            if (W > 0 && !counted_separately) SABA_HIP_TRY(hipEventElapsedTime(&a, ev.e[1], ev.e[2]));
            SABA_HIP_TRY(hipEventElapsedTime(&b, ev.e[0], ev.e[4]));
            st->kernel_ms = counted_separately ? kms : a;
            st->count_ms = counted_separately ? cms : 0.0;
            st->total_ms = b;
        }
    }
    return SABA_OK;
}

}  // namespace saba

using namespace saba;

extern "C" int saba_walks_noalloc(saba_graph *gh, const saba_walk_params *p,
                                  int64_t *d_endpoint, int64_t *d_visits, saba_stats *st,
                                  void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p) {
        set_error("params is NULL");
        return SABA_E_INVALID;
    }
    if (p->mode != SABA_WALK_BOUQUET || p->source_mode != SABA_SOURCES_EXPLICIT) {
        set_error("saba_walks_noalloc runs bouquet walks from explicit sources only");
        return SABA_E_INVALID;
    }
    void *base = nullptr;
    SABA_TRY(noalloc_scratch(&base));
    saba_walk_params q = *p;
    q.time_kernels = 0;  // no event objects either
    WalkArena ar;
    ar.g = G(gh);
    ar.base = static_cast<char *>(base);
    ar.cap = kNoAllocScratchBytes;
    return walks_impl(G(gh), &q, d_endpoint, d_visits, st, static_cast<hipStream_t>(stream), ar);
}

extern "C" int saba_walks(saba_graph *gh, const saba_walk_params *p, int64_t *d_endpoint,
                          int64_t *d_visits, saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p) {
        set_error("params is NULL");
        return SABA_E_INVALID;
    }
    WalkArena ar;
    ar.g = G(gh);
    return walks_impl(G(gh), p, d_endpoint, d_visits, st, static_cast<hipStream_t>(stream), ar);
}

extern "C" int saba_autotune_walks(saba_graph *gh, const saba_walk_params *sample,
                                   saba_exec_config *best, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!sample) {
        set_error("sample is NULL");
        return SABA_E_INVALID;
    }
    Graph *g = G(gh);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf out;
    SABA_TRY(out.ensure(sizeof(int64_t) * 2 * (size_t)std::max<int32_t>(g->n, 1)));
    struct Guard {
        DevBuf *b;
        ~Guard() { b->release(); }
    } guard{&out};
    int64_t *ep = out.as<int64_t>(), *vi = ep + std::max<int32_t>(g->n, 1);
    saba_walk_params p = *sample;
    p.mode = SABA_WALK_BOUQUET;
    p.time_kernels = 1;
    p.d_distinct = nullptr;
    const saba_exec_config saved = g->cfg;
    saba_exec_config pick = saved;
    double best_ms = 1e300;
    const int wpls[] = {1, 2, 4};
    const int blocks[] = {1024, 2048, 4096, 8192};
    const int chunks[] = {1, 4, 8};
    for (int wpl : wpls)
        for (int nb : blocks)
            for (int ch : chunks) {
                g->cfg = saved;
                g->cfg.walks_per_lane = wpl;
                g->cfg.walk_blocks = nb;
                g->cfg.walk_chunks = ch;
                double ms = 0.0;
                for (int rep = 0; rep < 3; ++rep) {  // one warm-up, two timed
                    saba_stats st{};
                    WalkArena ar;
                    ar.g = g;
                    const int rc = walks_impl(g, &p, ep, vi, &st, s, ar);
                    if (rc != SABA_OK) {
                        g->cfg = saved;
                        return rc;
                    }
                    if (rep > 0) ms += st.total_ms;  // the whole call: walks and counting passes
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    pick = g->cfg;
                }
            }
    g->cfg = pick;
    if (best) *best = pick;
    return SABA_OK;
}

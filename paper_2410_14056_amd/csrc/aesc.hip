// TGT+ all-edges spanning centrality (Alg. 1) on the GPU.
//
// Per source s the estimator needs, for every neighbour t:
//   tau_st   truncation length from the spectral tail bound
//            (1/d_s + 1/d_t) lambda^(tau+1) <= (eps/2)(1 - lambda);
//   h_l      h_l(x) = probability that a walk from x is at s after l steps, built level by
//            level with the pull recursion h_{l+1}(x) = (sum_{y in Gamma(x)} h_l(y)) / d(x);
//   ttau_s   the level at which the push stops: while the support volume of h_l is below
//            the number of walk pairs still needed, push one more level (Alg. 1 while-loop);
//   D_st     sum_{l <= min(ttau, tau)} (h_l(s) - h_l(t));
//   n_st     walk pairs, NWalks = max(1, ceil(c q^2)), q = L hmax / d_s, c = 32 ln(4m/delta)/eps^2;
//   MC_st    sum over pairs k of X_k = sum_b h_ttau(W^s_k[b]) - sum_b h_ttau(W^t_k[b]), b = 1..L;
// and g(s,t) = (D_st + MC_st / n_st) / d_s, SC(u,v) = g(u,v) + g(v,u).
//
// Work items.  A call evaluates a set of requests; each request names a graph of the handle
// and a parameter set (eps, delta, lambda, seed, grouping).  An *instance* is a (source vertex,
// parameter set) pair that some request needs, and an *instance edge* is a directed edge out
// of an instance's vertex.  Everything an instance computes depends only on its graph, its
// parameters and the vertex, and keys and hashes use the graph's own vertex ids, so a result
// is the same whether its request runs alone or batched with others, on a handle holding one
// graph or many.
//
// Work layout.  Instances are processed in batches that fit a memory budget.  Each instance of
// a batch owns a slot: dense FP64 h vectors (two levels), frontier lists and support bitmaps
// (two levels) sized to its graph, and a bitmap over its graph's CSR positions for hub rows.
// All of these are cleared sparsely through the frontier lists, so they are zeroed only once.
// The deterministic levels run level-synchronously over the whole batch.  A wavefront walks
// the concatenated rows of 64 frontier vertices in chunks of 64 entries, so long rows are split
// across lanes; the pull folds only the terms whose vertex is in the support bitmap (a zero
// term leaves a sum of non-negative numbers unchanged), in row order, so every h value is
// bit-identical to the sequential left fold over the whole row.  The walk pairs of all instance
// edges of the batch are cut into chunks of 64 walks; one persistent launch covers all of them
// (a fixed wavefront stride, per-XCD work queues, or tiles of one source's chunks per block with
// the source's support bitmap staged in LDS), a wavefront reduces a chunk in a fixed butterfly
// order, and each edge sums its chunks in chunk order, so results do not depend on the schedule
// or the launch shape.  The synchronous calls may run the levels of the next batch on a second
// stream, with a second pool set, while the walk pairs of the current batch run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "estimator.hpp"

namespace saba {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kChunk = 64;  // walks per wavefront chunk
constexpr int kWalkGrid = 1024;

struct BatchState {  // one per slot; [2] entries are indexed by level parity
    int32_t active;
    int32_t finalbuf;
    int32_t fsz[2];                 // frontier (support) sizes
    unsigned long long vol[2];      // support volume sum of d(x)
    unsigned long long hmaxbits[2]; // max of h over the support, as IEEE bits (h > 0)
    double hmax;                    // max of h_ttau once the source has stopped
    int32_t maxtau;
    int32_t ttau;
};

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ long long wave_sum_ll(long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// CalculateTau(e, eps/2): smallest tau >= 0 with w * lambda^(tau+1) <= (eps/2)(1 - lambda),
// w = 1/d_s + 1/d_t, the power formed by repeated multiplication; capped at tau_cap.
__device__ __forceinline__ int32_t tau_of(int32_t ds, int32_t dt, double lambda, double eps,
                                          int32_t cap) {
    const double w = 1.0 / (double)ds + 1.0 / (double)dt;
    const double rhs = (eps / 2.0) * (1.0 - lambda);
    double p = lambda;
    int32_t tau = 0;
    while (w * p > rhs && tau < cap) {
        p = p * lambda;
        tau += 1;
    }
    return tau;
}

constexpr long long kMaxPairs = 0xFFFFFFFFll;  // walk pairs of one directed edge

// NWalks (Hoeffding): max(1, ceil(c * q * q)), q = L * hmax / d_s; -1 on overflow.
__device__ __forceinline__ long long nwalks(int32_t L, double hmax, int32_t ds, double c) {
    const double q = ((double)L * hmax) / (double)ds;
    const double x = c * q * q;
    if (!(x < 4.0e18)) return -1;
    long long r = (long long)ceil(x);
    return r < 1 ? 1 : r;
}

// ------------------------------------------------------------ kernels
// Level 0 of every instance of the batch: h_0 = e_s, support {s}; tau of its edges, per-edge
// accumulators reset.
__global__ __launch_bounds__(kBlock) void batch_init_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col, const Slot *__restrict__ slots,
    const PSet *__restrict__ psets, int32_t nb, BatchState *__restrict__ bs,
    double *__restrict__ hA, int32_t *__restrict__ FA, uint32_t *__restrict__ bmA,
    int32_t *__restrict__ tau, double *__restrict__ D, long long *__restrict__ nreq,
    double *__restrict__ MC, unsigned long long *__restrict__ vis0,
    unsigned long long *__restrict__ vis1, int2 *__restrict__ hubs0, Flags *__restrict__ fl) {
    const int lane = __lane_id();
    const int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (b >= nb) return;
    const Slot sl = slots[b];
    const PSet ps = psets[sl.p];
    const int2 r = vrec[sl.v];
    int mx = 0, capped = 0;
    for (int32_t i = lane; i < r.y; i += 64) {
        const int64_t ie = sl.ie + i;
        const int32_t tv = tau_of(r.y, vrec[col[r.x + i]].y, ps.lambda, ps.eps, ps.tau_cap);
        tau[ie] = tv;
        mx = max(mx, tv);
        capped |= tv >= ps.tau_cap ? 1 : 0;
        D[ie] = 0.0;
        nreq[ie] = 0;
        MC[ie] = 0.0;
        vis0[ie] = 0;
        vis1[ie] = 0;
    }
    mx = wave_max_i(mx);
    capped = wave_max_i(capped);
    if (lane == 0) {
        const int32_t sl_local = sl.v - sl.goff;
        BatchState st;
        st.active = 1;
        st.finalbuf = 0;
        st.fsz[0] = 1;
        st.fsz[1] = 0;
        st.vol[0] = (unsigned long long)r.y;
        st.vol[1] = 0;
        st.hmaxbits[0] = (unsigned long long)__double_as_longlong(1.0);
        st.hmaxbits[1] = 0;
        st.hmax = 0.0;
        st.maxtau = mx;
        st.ttau = 0;
        bs[b] = st;
        hA[sl.hoff + sl_local] = 1.0;
        FA[sl.hoff] = sl.v;
        bmA[sl.bmoff + (sl_local >> 5)] = 1u << (sl_local & 31);
        if (r.y > kHubRow) hubs0[atomicAdd(&fl->nhub[0], 1)] = make_int2((int32_t)b, sl.v);
        atomicMax(&fl->max_tau, mx);
        if (capped) atomicOr(&fl->warnings, 1);
    }
}

// Alg. 1 loop test at level l for each active instance: with the support volume and maximum
// of h_l (accumulated when h_l was built), add the deterministic terms of level l and compare
// the volume with the walk pairs that would still be needed.
__global__ __launch_bounds__(kBlock) void level_decide_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col, const Slot *__restrict__ slots,
    const PSet *__restrict__ psets, BatchState *__restrict__ bs, int32_t nb, int32_t level,
    const double *__restrict__ hcur_all, const int32_t *__restrict__ tau, double *__restrict__ D,
    int32_t *__restrict__ ttau_inst, Flags *__restrict__ fl) {
    const int lane = __lane_id();
    const int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cur = level & 1, nxt = cur ^ 1;
    // the hub-row list of level l + 1 is filled by this level's compaction (its previous
    // contents, level l - 1's hub rows, were last used by the previous level's expansion)
    if (blockIdx.x == 0 && threadIdx.x == 0) fl->nhub[nxt] = 0;
    if (b >= nb || !bs[b].active) return;
    const Slot sl = slots[b];
    const PSet ps = psets[sl.p];
    const double *h = hcur_all + sl.hoff;  // indexed by graph-local vertex ids
    const long long vol = (long long)bs[b].vol[cur];
    const double hmax = __longlong_as_double((long long)bs[b].hmaxbits[cur]);
    const int2 r = vrec[sl.v];
    const double hs = h[sl.v - sl.goff];
    long long need = 0;
    int ovf = 0;
    for (int32_t i = lane; i < r.y; i += 64) {
        const int64_t ie = sl.ie + i;
        const int32_t te = tau[ie];
        if (level <= te) D[ie] += hs - h[col[r.x + i] - sl.goff];
        if (te > level) {
            const long long w = nwalks(te - level, hmax, r.y, ps.c);
            if (w < 0)
                ovf = 1;
            else
                need += w;
        }
    }
    need = wave_sum_ll(need);
    ovf = wave_max_i(ovf);
    if (lane == 0) {
        if (ovf) atomicOr(&fl->err, kErrOverflow);
        bool stop = ps.push_all ? (level >= bs[b].maxtau) : !(vol < need);
        if (ps.tilde_tau_max >= 0 && level >= ps.tilde_tau_max) stop = true;
        if (ovf) stop = true;
        if (stop) {
            bs[b].active = 0;
            bs[b].finalbuf = cur;
            bs[b].hmax = hmax;
            bs[b].ttau = level;
            ttau_inst[sl.inst] = level;
            atomicMax(&fl->max_ttau, level);
        } else {
            // level l + 1 is built into the buffers of parity nxt (cleared after level l - 1)
            bs[b].fsz[nxt] = 0;
            bs[b].vol[nxt] = 0;
            bs[b].hmaxbits[nxt] = 0;
            fl->any_active = 1;
        }
    }
}

// Rows of the 64 frontier entries [base, base + 64) of one instance, as seen by each lane:
// its own row and the exclusive prefix of the row lengths over the wavefront.  Hub rows
// count as empty when `skip_hubs` is set (they are handled separately).
struct WaveRows {
    int32_t x, start, deg, len, pre, total;  // len = deg, or 0 for a skipped hub row
};

__device__ __forceinline__ WaveRows wave_rows(const int2 *__restrict__ vrec,
                                              const int32_t *__restrict__ F, int64_t base,
                                              int32_t fsz, bool skip_hubs) {
    const int lane = __lane_id();
    WaveRows w;
    w.x = -1;
    w.start = 0;
    w.deg = 0;
    w.len = 0;
    if (base + lane < fsz) {
        w.x = F[base + lane];
        const int2 r = vrec[w.x];
        w.start = r.x;
        w.deg = r.y;
        w.len = (skip_hubs && r.y > kHubRow) ? 0 : r.y;
    }
    int32_t inc = w.len;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    // readfirstlane makes the loop bounds derived from the total provably wave-uniform, so the
    // compiler keeps the wavefront converged around the cross-lane operations in those loops
    w.total = __builtin_amdgcn_readfirstlane(__shfl(inc, 63));
    w.pre = inc - w.len;
    return w;
}

// Owner lane of flattened entry j (0 <= j < total): the largest lane whose prefix is <= j,
// which is always a lane whose row contains entry j.
__device__ __forceinline__ int wave_owner(int32_t pre, int32_t j) {
    int lo = 0, hi = 64;
    for (int it = 0; it < 6; ++it) {  // 64 -> 1 candidates: a fixed, uniform trip count
        const int mid = (lo + hi) >> 1;
        if (__shfl(pre, mid) <= j)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const int32_t lo = __builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(uint64_t)x);
    const int32_t hi = __builtin_amdgcn_readfirstlane((int32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// XCD-aware block order.  The dispatcher deals the blocks of a launch round-robin over the
// 8 XCDs, so blocks with equal blockIdx.x mod 8 share one L2.  Numbering those blocks
// consecutively (a permutation of the block ids when the grid is a multiple of 8) makes the
// waves of one XCD take consecutive work items, which belong to the same source.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t i = blockIdx.x, nb = gridDim.x;
    if (nb % kXcds) return i;
    return (i % kXcds) * (nb / kXcds) + i / kXcds;
}

__device__ __forceinline__ int64_t upper_index(const int64_t *__restrict__ a, int64_t len,
                                               int64_t key) {
    // largest i in [0, len) with a[i] <= key (a non-decreasing, a[0] <= key)
    int64_t lo = 0, hi = len;
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= key)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Frontier groups.  A level's frontier lists are cut into groups of 64 vertices per slot and
// gofs[b] (b < nb) is the first group of slot b (inactive slots have none; gofs[nb] = total).
// Wavefront w of the push kernels takes groups w, w + W, w + 2W, ... of the whole batch (W
// wavefronts in the grid), so a slot with a huge frontier is spread over the whole grid and the
// heavy first groups of the slots (frontiers are in ascending vertex order) land on different
// wavefronts.  Hub rows are not part of the groups' work: they go to the hub-row lists.
constexpr int kPushGrid = 2048;
constexpr int kHubGrid = 1024;  // blocks of the hub-row kernels
constexpr int kPullWin = 16;    // 64-entry chunks per pass of the ordinary-row push kernels

__global__ __launch_bounds__(1024) void group_scan_kernel(const BatchState *__restrict__ bs,
                                                          int32_t nb, int parity,
                                                          int64_t *__restrict__ gofs) {
    // tiles of kTile slots: their group counts are staged in LDS (consecutive threads read
    // consecutive slot records), then each thread scans kTile / 1024 consecutive counts
    constexpr int kTile = 8192, kPer = kTile / 1024;
    __shared__ uint32_t cnt[kTile];
    __shared__ long long wtot[16];
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    long long carry = 0;
    for (int32_t t0 = 0; t0 < nb; t0 += kTile) {
        const int32_t tn = min(kTile, nb - t0);
        for (int32_t i = tid; i < tn; i += 1024) {
            const BatchState &x = bs[t0 + i];
            cnt[i] = x.active ? (uint32_t)(((long long)x.fsz[parity] + 63) / 64) : 0u;
        }
        __syncthreads();
        const int32_t i0 = tid * kPer;
        long long loc = 0;
        for (int k = 0; k < kPer; ++k)
            if (i0 + k < tn) loc += cnt[i0 + k];
        long long inc = loc;
        for (int o = 1; o < 64; o <<= 1) {
            const long long t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        if (lane == 63) wtot[wave] = inc;
        __syncthreads();
        long long run = carry + inc - loc, tile_total = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < wave) run += wtot[k];
            tile_total += wtot[k];
        }
        for (int k = 0; k < kPer; ++k)
            if (i0 + k < tn) {
                gofs[t0 + i0 + k] = run;
                run += cnt[i0 + k];
            }
        carry += tile_total;
        __syncthreads();  // cnt and wtot are rewritten by the next tile
    }
    if (tid == 0) gofs[nb] = carry;
}

struct GroupCursor {  // the slot of the current group of a wavefront (all fields wave-uniform)
    int64_t b = -1, gbase = 0, gnext = 0;
};

// Moves the cursor to the slot holding group gi (called when gi >= cursor.gnext).
__device__ __forceinline__ void group_seek(GroupCursor &c, const int64_t *__restrict__ gofs,
                                           int32_t nb, int64_t gi) {
    c.b = uniform64(upper_index(gofs, nb + 1, gi));
    c.gbase = uniform64(gofs[c.b]);
    c.gnext = uniform64(gofs[c.b + 1]);
}

// First group, stride and total of this wavefront's groups (all wave-uniform).
__device__ __forceinline__ void wave_groups(const int64_t *__restrict__ gofs, int32_t nb,
                                            int64_t &first, int64_t &stride, int64_t &total) {
    total = uniform64(gofs[nb]);
    stride = (int64_t)gridDim.x * kWavesPerBlock;
    first = uniform64(xcd_block() * kWavesPerBlock + (threadIdx.x >> 6));
}

// Push the current support one hop: set the bit of every neighbour in the next level's
// support bitmap and, for neighbours with hub rows, the bit of the reverse CSR position in
// the slot's CSR-position bitmap.  Fire-and-forget atomics; the next frontier list is built
// from the bitmap afterwards, in ascending vertex order.  Ordinary rows go by frontier groups
// here; hub rows of the frontier are expanded by expand_hub_kernel.
__device__ __forceinline__ void expand_entry(const int32_t *__restrict__ col,
                                             const int32_t *__restrict__ slotv, const Slot &sl,
                                             uint32_t *__restrict__ bm, uint32_t *__restrict__ sbm,
                                             int32_t e) {
    // Bits only go from 0 to 1 while the support is built, so a read that already sees the bit
    // set makes the atomic OR redundant; a read that misses a bit set meanwhile (by another
    // compute unit, or an older cached copy) only costs the OR.  The read is a relaxed atomic
    // at workgroup scope: it may be served by this compute unit's cache.  Most bits are
    // reached from several frontier vertices.
    const auto set_bit = [](uint32_t *words, int32_t i) {
        uint32_t *w = words + (i >> 5);
        const uint32_t bit = 1u << (i & 31);
        if (!(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) & bit))
            atomicOr(w, bit);
    };
    set_bit(bm, col[e] - sl.goff);
    const int32_t slot = slotv[e];
    if (slot >= 0) set_bit(sbm, slot - sl.gpos);
}

// expand_entry for kPullWin entries per lane (e[u], valid positions; in[u]: the entry is
// wanted), with the entry, hub-slot and support-word loads of all of them in flight together
// before the atomic ORs.
__device__ __forceinline__ void expand_entries(const int32_t *__restrict__ col,
                                               const int32_t *__restrict__ slotv, const Slot &sl,
                                               uint32_t *__restrict__ bm,
                                               uint32_t *__restrict__ sbm,
                                               const int32_t (&e)[kPullWin],
                                               const bool (&in)[kPullWin]) {
    int32_t x[kPullWin], sv[kPullWin];
    uint32_t wx[kPullWin], ws[kPullWin];
#pragma unroll
    for (int u = 0; u < kPullWin; ++u) x[u] = col[e[u]] - sl.goff;
#pragma unroll
    for (int u = 0; u < kPullWin; ++u) sv[u] = slotv[e[u]];
#pragma unroll
    for (int u = 0; u < kPullWin; ++u)
        wx[u] = __hip_atomic_load(bm + (x[u] >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int u = 0; u < kPullWin; ++u) {
        ws[u] = ~0u;
        if (sv[u] >= 0)
            ws[u] = __hip_atomic_load(sbm + ((sv[u] - sl.gpos) >> 5), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
    }
#pragma unroll
    for (int u = 0; u < kPullWin; ++u) {
        const uint32_t bit = 1u << (x[u] & 31);
        if (in[u] && !(wx[u] & bit)) atomicOr(bm + (x[u] >> 5), bit);
    }
#pragma unroll
    for (int u = 0; u < kPullWin; ++u) {
        if (!in[u] || sv[u] < 0) continue;
        const int32_t i = sv[u] - sl.gpos;
        const uint32_t bit = 1u << (i & 31);
        if (!(ws[u] & bit)) atomicOr(sbm + (i >> 5), bit);
    }
}

__global__ __launch_bounds__(kBlock) void expand_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
    const int32_t *__restrict__ slotv, const Slot *__restrict__ slots,
    const BatchState *__restrict__ bs, int32_t nb, int32_t level, const int64_t *__restrict__ gofs,
    const int32_t *__restrict__ Fcur_all, uint32_t *__restrict__ bmnext_all,
    uint32_t *__restrict__ slotbm_all, Flags *__restrict__ fl) {
    const int cur = level & 1;
    const int lane = __lane_id();
    int64_t first, stride, total;
    wave_groups(gofs, nb, first, stride, total);
    GroupCursor gc;
    Slot sl{};
    int32_t fsz = 0;
    unsigned long long visits = 0;
    for (int64_t gi = first; gi < total; gi += stride) {
        if (gi >= gc.gnext) {
            group_seek(gc, gofs, nb, gi);
            sl = slots[gc.b];
            fsz = bs[gc.b].fsz[cur];
        }
        const int32_t *F = Fcur_all + sl.hoff;
        uint32_t *bm = bmnext_all + sl.bmoff;
        uint32_t *sbm = slotbm_all + sl.sboff;
        const WaveRows w = wave_rows(vrec, F, (gi - gc.gbase) * 64, fsz, true);
        if (lane == 0) visits += w.total;
        for (int32_t j0 = 0; j0 < w.total; j0 += 64 * kPullWin) {
            // cross-lane reads happen with every lane active; only memory accesses are masked
            int32_t e[kPullWin];
            bool in[kPullWin];
#pragma unroll
            for (int u = 0; u < kPullWin; ++u) {
                const int32_t j = j0 + 64 * u + lane;
                in[u] = j < w.total;
                if (j0 + 64 * u >= w.total) {  // wave-uniform: a chunk past the group's end
                    e[u] = e[0];                 // (a valid position; nothing is taken from it)
                    continue;
                }
                const int32_t jc = in[u] ? j : w.total - 1;
                const int o = wave_owner(w.pre, jc);
                const int32_t ost = __shfl(w.start, o), opre = __shfl(w.pre, o);
                e[u] = ost + (jc - opre);
            }
            expand_entries(col, slotv, sl, bm, sbm, e, in);
        }
    }
    visits = wave_sum_ll((long long)visits);
    if (lane == 0 && visits) atomicAdd(&fl->push_visits, visits);
}

// Hub rows of the current frontier (the list of this level's parity): one block per row.
__global__ __launch_bounds__(kBlock) void expand_hub_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
    const int32_t *__restrict__ slotv, const Slot *__restrict__ slots,
    const BatchState *__restrict__ bs, int32_t level, const int2 *__restrict__ hubs_all,
    int64_t hubcap, uint32_t *__restrict__ bmnext_all, uint32_t *__restrict__ slotbm_all,
    Flags *__restrict__ fl) {
    const int cur = level & 1;
    const int2 *hubs = hubs_all + cur * hubcap;
    const int32_t nh = fl->nhub[cur];
    unsigned long long visits = 0;
    for (int32_t k = (int32_t)xcd_block(); k < nh; k += gridDim.x) {
        const int2 hb = hubs[k];
        if (!bs[hb.x].active) continue;  // the list was made before this level's stop test
        const Slot sl = slots[hb.x];
        const int2 r = vrec[hb.y];
        uint32_t *bm = bmnext_all + sl.bmoff;
        uint32_t *sbm = slotbm_all + sl.sboff;
        for (int32_t i = threadIdx.x; i < r.y; i += kBlock)
            expand_entry(col, slotv, sl, bm, sbm, r.x + i);
        if (threadIdx.x == 0) visits += (unsigned long long)r.y;
    }
    if (threadIdx.x == 0 && visits) atomicAdd(&fl->push_visits, visits);
}

// Next frontier list of each active instance: the set bits of its next-level support bitmap,
// in ascending vertex order (one block per instance).  Its hub rows are also appended, in any
// order, to the hub-row list of the next level's parity.
// Hub bits of the 32 vertices v0 .. v0 + 31 (handle ids) from the handle's hub bitmap.
constexpr int kCompactWords = 8;  // bitmap words per thread and round of the compaction

__device__ __forceinline__ uint32_t hub_word(const uint32_t *__restrict__ hubbm, int32_t v0) {
    const int32_t w = v0 >> 5, sh = v0 & 31;
    return sh == 0 ? hubbm[w] : (hubbm[w] >> sh) | (hubbm[w + 1] << (32 - sh));
}

__global__ __launch_bounds__(kBlock) void compact_frontier_kernel(
    const uint32_t *__restrict__ hubbm, const Slot *__restrict__ slots, BatchState *__restrict__ bs,
    int32_t level, const uint32_t *__restrict__ bmnext_all, int32_t *__restrict__ Fnext_all,
    int2 *__restrict__ hubs_all, int64_t hubcap, Flags *__restrict__ fl) {
    __shared__ uint32_t wave_tot[kCompactWords][kWavesPerBlock];
    __shared__ int32_t carry;
    const int64_t b = blockIdx.x;
    if (!bs[b].active) return;
    const int nxt = (level & 1) ^ 1;
    const Slot sl = slots[b];
    const uint32_t *bm = bmnext_all + sl.bmoff;
    int32_t *Fn = Fnext_all + sl.hoff;
    const int64_t nw = ((int64_t)sl.gn + 31) / 32;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    // A round covers kCompactWords stripes of kBlock consecutive words; thread t takes word t
    // of every stripe (all loads in flight together), and the stripes are written one after
    // the other, each by consecutive threads at consecutive positions.
    for (int64_t w0 = 0; w0 < nw; w0 += (int64_t)kBlock * kCompactWords) {
        uint32_t words[kCompactWords], cnt[kCompactWords], inc[kCompactWords];
#pragma unroll
        for (int k = 0; k < kCompactWords; ++k) {
            const int64_t wi = w0 + (int64_t)k * kBlock + threadIdx.x;
            words[k] = wi < nw ? bm[wi] : 0u;
            cnt[k] = __popc(words[k]);
            inc[k] = cnt[k];
        }
#pragma unroll
        for (int k = 0; k < kCompactWords; ++k)
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc[k], o);
                if (lane >= o) inc[k] += t;
            }
        if (lane == 63)
#pragma unroll
            for (int k = 0; k < kCompactWords; ++k) wave_tot[k][wave] = inc[k];
        __syncthreads();
        int32_t base = carry;
#pragma unroll
        for (int k = 0; k < kCompactWords; ++k) {
            uint32_t before = 0, all = 0;
            for (int w = 0; w < kWavesPerBlock; ++w) {
                if (w < wave) before += wave_tot[k][w];
                all += wave_tot[k][w];
            }
            int32_t pos = base + (int32_t)(before + inc[k] - cnt[k]);
            base += (int32_t)all;
            uint32_t rest = words[k];
            if (!rest) continue;
            const int64_t wi = w0 + (int64_t)k * kBlock + threadIdx.x;
            const uint32_t hw = hub_word(hubbm, sl.goff + (int32_t)(wi * 32));
            while (rest) {
                const int bit = __builtin_ctz(rest);
                rest &= rest - 1;
                const int32_t x = sl.goff + (int32_t)(wi * 32 + bit);
                Fn[pos++] = x;
                if ((hw >> bit) & 1u)
                    hubs_all[nxt * hubcap + atomicAdd(&fl->nhub[nxt], 1)] =
                        make_int2((int32_t)b, x);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) carry = base;
        __syncthreads();
    }
    if (threadIdx.x == 0) bs[b].fsz[nxt] = carry;
}

// h_{l+1}(x) = (left fold over Gamma(x) in CSR order of h_l) / d(x) for x in the next support.
// Only terms in the support of h_l are nonzero, and adding +0.0 leaves a sum of non-negative
// numbers bit-identical, so both kernels below produce the sequential fold exactly.
//  - pull_kernel, ordinary rows: the wavefront walks the concatenated rows of its 64 vertices,
//    fetches one entry per lane (h_l where the support bitmap has the neighbour, else 0),
//    stages the 64 values in LDS and each lane folds its own row's part in row order;
//  - pull_hub_kernel, hub rows: the set bits of the CSR-position bitmap over the row mark
//    exactly the in-support positions; they are listed in row order, their values staged in
//    LDS and folded by one lane.  The row's bits are cleared on the way.
// Both accumulate the support volume and maximum of h_{l+1} per slot.
__global__ __launch_bounds__(kBlock) void pull_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col, const Slot *__restrict__ slots,
    BatchState *__restrict__ bs, int32_t nb, int32_t level, const int64_t *__restrict__ gofs,
    const double *__restrict__ hcur_all, const uint32_t *__restrict__ bmcur_all,
    double *__restrict__ hnext_all, const int32_t *__restrict__ Fnext_all,
    Flags *__restrict__ fl) {
    __shared__ double stage[kWavesPerBlock][64 * kPullWin];
    const int nxt = (level & 1) ^ 1;
    const int lane = __lane_id();
    double *lds = stage[threadIdx.x >> 6];
    int64_t first, stride, total;
    wave_groups(gofs, nb, first, stride, total);
    GroupCursor gc;
    Slot sl{};
    int32_t fsz = 0;
    unsigned long long visits = 0, vol = 0;
    double hmax = 0.0;
    // support volume and maximum of h_{l+1} are flushed to their slot when the wavefront
    // moves on to another slot, and at the end
    auto flush = [&]() {
        const unsigned long long v = (unsigned long long)wave_sum_ll((long long)vol);
        const double hm = wave_max_d(hmax);
        if (lane == 0 && gc.b >= 0 && v) {
            atomicAdd(&bs[gc.b].vol[nxt], v);
            atomicMax(&bs[gc.b].hmaxbits[nxt], (unsigned long long)__double_as_longlong(hm));
        }
        vol = 0;
        hmax = 0.0;
    };
    for (int64_t gi = first; gi < total; gi += stride) {
        if (gi >= gc.gnext) {
            flush();
            group_seek(gc, gofs, nb, gi);
            sl = slots[gc.b];
            fsz = bs[gc.b].fsz[nxt];
        }
        const double *h = hcur_all + sl.hoff;  // indexed by graph-local vertex ids
        const uint32_t *bm = bmcur_all + sl.bmoff;
        double *hn = hnext_all + sl.hoff;
        const int32_t *F = Fnext_all + sl.hoff;
        const WaveRows w = wave_rows(vrec, F, (gi - gc.gbase) * 64, fsz, true);
        if (lane == 0) visits += w.total;
        double acc = 0.0;  // the fold of this lane's own row
        // kPullWin chunks of 64 entries per pass: their dependent loads (entry, support word,
        // value) are issued together so that more of them are in flight per wavefront
        for (int32_t j0 = 0; j0 < w.total; j0 += 64 * kPullWin) {
            int32_t e[kPullWin], y[kPullWin];
            uint32_t wd[kPullWin];
            bool in[kPullWin];
#pragma unroll
            for (int u = 0; u < kPullWin; ++u) {
                const int32_t j = j0 + 64 * u + lane;
                in[u] = j < w.total;
                if (j0 + 64 * u >= w.total) {  // wave-uniform: a chunk past the group's end
                    e[u] = e[0];                 // (a valid position; nothing is taken from it)
                    continue;
                }
                const int32_t jc = in[u] ? j : w.total - 1;
                const int o = wave_owner(w.pre, jc);
                const int32_t ost = __shfl(w.start, o), opre = __shfl(w.pre, o);
                e[u] = ost + (jc - opre);
            }
            // every e[u] is a position in one of the group's rows (j is clamped to the last
            // entry), so the entry and support-word loads need no guard and go out together;
            // the value loads are all issued before the first LDS store waits on them
#pragma unroll
            for (int u = 0; u < kPullWin; ++u) y[u] = col[e[u]] - sl.goff;
#pragma unroll
            for (int u = 0; u < kPullWin; ++u) wd[u] = bm[y[u] >> 5];
            // the support bit as plain arithmetic, so no load is moved under a branch
            uint32_t bit[kPullWin];
#pragma unroll
            for (int u = 0; u < kPullWin; ++u) bit[u] = (wd[u] >> (y[u] & 31)) & (uint32_t)in[u];
            double v[kPullWin];
#pragma unroll
            for (int u = 0; u < kPullWin; ++u) {
                v[u] = 0.0;
                if (bit[u] & 1u) v[u] = h[y[u]];
            }
#pragma unroll
            for (int u = 0; u < kPullWin; ++u) lds[64 * u + lane] = v[u];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int32_t k0 = max(w.pre, j0) - j0;
            const int32_t k1 = min(w.pre + w.len, j0 + 64 * kPullWin) - j0;
            for (int32_t k = k0; k < k1; ++k) acc += lds[k];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (w.x >= 0 && w.deg <= kHubRow) {
            const double hv = acc / (double)w.deg;
            hn[w.x - sl.goff] = hv;
            vol += (unsigned long long)w.deg;
            hmax = fmax(hmax, hv);
        }
    }
    flush();
    visits = wave_sum_ll((long long)visits);
    if (lane == 0 && visits) atomicAdd(&fl->push_visits, visits);
}

constexpr int kHubSpan = 2048;  // row positions per pass (64 bitmap words, one per lane)
constexpr int kHubVals = 256;   // values staged per fold step

__global__ __launch_bounds__(kBlock) void pull_hub_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col, const Slot *__restrict__ slots,
    BatchState *__restrict__ bs, int32_t level, const int2 *__restrict__ hubs_all,
    int64_t hubcap, const double *__restrict__ hcur_all, uint32_t *__restrict__ slotbm_all,
    double *__restrict__ hnext_all, Flags *__restrict__ fl) {
    __shared__ int32_t spos[kWavesPerBlock][kHubSpan];
    __shared__ double sval[kWavesPerBlock][kHubVals];
    const int nxt = (level & 1) ^ 1;
    const int lane = __lane_id();
    int32_t *lpos = spos[threadIdx.x >> 6];
    double *lval = sval[threadIdx.x >> 6];
    const int2 *hubs = hubs_all + nxt * hubcap;
    const int32_t nh = __builtin_amdgcn_readfirstlane(fl->nhub[nxt]);
    const int32_t nwaves = (int32_t)gridDim.x * kWavesPerBlock;
    unsigned long long visits = 0;
    for (int32_t k = __builtin_amdgcn_readfirstlane((int32_t)(xcd_block() * kWavesPerBlock +
                                                              (threadIdx.x >> 6)));
         k < nh; k += nwaves) {
        const int2 hb = hubs[k];
        const Slot sl = slots[hb.x];
        const double *h = hcur_all + sl.hoff;
        uint32_t *sbm = slotbm_all + sl.sboff;
        const int2 r = vrec[hb.y];
        const int32_t a = r.x - sl.gpos, e1 = a + r.y;  // local row positions [a, e1)
        const int64_t wfirst = a >> 5, wlast = (e1 - 1) >> 5;
        double hacc = 0.0;  // lane 0's fold of the row
        for (int64_t wc = wfirst; wc <= wlast; wc += 64) {
            const int64_t wi = wc + lane;
            uint32_t word = 0;
            if (wi <= wlast) {
                word = sbm[wi];
                if (wi == wfirst) word &= ~0u << (a & 31);
                if (wi == wlast && (e1 & 31)) word &= (1u << (e1 & 31)) - 1u;
            }
            const int32_t cnt = __popc(word);
            int32_t inc = cnt;
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t t = __shfl_up(inc, o);
                if (lane >= o) inc += t;
            }
            const int32_t T = __builtin_amdgcn_readfirstlane(__shfl(inc, 63));
            // in-support positions of this pass, in row order
            {
                uint32_t rest = word;
                int32_t p = inc - cnt;
                while (rest) {
                    const int bit = __builtin_ctz(rest);
                    rest &= rest - 1;
                    lpos[p++] = (int32_t)(wi * 32 + bit);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int32_t r0 = 0; r0 < T; r0 += kHubVals) {
                for (int32_t q = 0; q < kHubVals; q += 64) {
                    const int32_t i = r0 + q + lane;
                    if (i < T) lval[q + lane] = h[col[sl.gpos + lpos[i]] - sl.goff];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane == 0) {
                    const int32_t n = min(kHubVals, T - r0);
                    for (int32_t i = 0; i < n; ++i) hacc += lval[i];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            // this row's bits are consumed: clear them (boundary words are shared)
            if (wi <= wlast) {
                const bool edge = (wi == wfirst && (a & 31)) || (wi == wlast && (e1 & 31));
                if (edge) {
                    uint32_t mask = ~0u;
                    if (wi == wfirst) mask &= ~0u << (a & 31);
                    if (wi == wlast && (e1 & 31)) mask &= (1u << (e1 & 31)) - 1u;
                    atomicAnd(sbm + wi, ~mask);
                } else {
                    sbm[wi] = 0u;
                }
            }
            if (lane == 0) visits += (unsigned long long)T;
        }
        if (lane == 0) {
            const double hv = hacc / (double)r.y;
            hnext_all[sl.hoff + (hb.y - sl.goff)] = hv;
            atomicAdd(&bs[hb.x].vol[nxt], (unsigned long long)r.y);
            atomicMax(&bs[hb.x].hmaxbits[nxt], (unsigned long long)__double_as_longlong(hv));
        }
    }
    if (lane == 0 && visits) atomicAdd(&fl->push_visits, visits);
}

// The end of a batch: zero h_ttau and its support bitmap over the final support of every
// slot (the buffers of the slot's last level), so the scratch is clean for the next batch.
// Every set bit of a touched bitmap word belongs to the support, so the whole word is cleared.
__global__ __launch_bounds__(kBlock) void clear_final_kernel(
    const Slot *__restrict__ slots, const BatchState *__restrict__ bs, double *__restrict__ hA,
    double *__restrict__ hB, uint32_t *__restrict__ bmA, uint32_t *__restrict__ bmB,
    const int32_t *__restrict__ FA, const int32_t *__restrict__ FB) {
    const int64_t b = blockIdx.y;
    const Slot sl = slots[b];
    const int pb = bs[b].finalbuf;
    double *h = (pb ? hB : hA) + sl.hoff;
    uint32_t *bm = (pb ? bmB : bmA) + sl.bmoff;
    const int32_t *F = (pb ? FB : FA) + sl.hoff;
    const int32_t fsz = bs[b].fsz[pb];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < fsz;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = F[i] - sl.goff;
        h[x] = 0.0;
        bm[x >> 5] = 0u;
    }
}

// The end of a level: h_l and its support bitmap (parity `parity`) cleared over the frontier of
// every active slot, so both are clean when the buffers are reused for level l + 2.  The work
// goes by the frontier groups numbered in gofs (the level's expansion groups), so it follows
// the frontiers rather than the number of slots.
__global__ __launch_bounds__(kBlock) void clear_groups_kernel(
    const Slot *__restrict__ slots, const BatchState *__restrict__ bs, int32_t nb, int parity,
    const int64_t *__restrict__ gofs, double *__restrict__ h_all, uint32_t *__restrict__ bm_all,
    const int32_t *__restrict__ F_all) {
    const int lane = __lane_id();
    int64_t first, stride, total;
    wave_groups(gofs, nb, first, stride, total);
    GroupCursor gc;
    Slot sl{};
    int32_t fsz = 0;
    for (int64_t gi = first; gi < total; gi += stride) {
        if (gi >= gc.gnext) {
            group_seek(gc, gofs, nb, gi);
            sl = slots[gc.b];
            fsz = bs[gc.b].fsz[parity];
        }
        const int64_t i = (gi - gc.gbase) * 64 + lane;
        if (i < fsz) {
            const int32_t x = F_all[sl.hoff + i] - sl.goff;
            h_all[sl.hoff + x] = 0.0;
            bm_all[sl.bmoff + (x >> 5)] = 0u;
        }
    }
}

// Walk pairs per wanted instance edge and the number of 64-walk chunks they need.
__global__ __launch_bounds__(kBlock) void nreq_kernel(
    const int2 *__restrict__ vrec, const Slot *__restrict__ slots, const PSet *__restrict__ psets,
    const BatchState *__restrict__ bs, int32_t nb, int64_t ie0, const int32_t *__restrict__ tau,
    const uint8_t *__restrict__ want, long long *__restrict__ nreq, long long *__restrict__ chunks,
    Flags *__restrict__ fl) {
    const int lane = __lane_id();
    const int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (b >= nb) return;
    const Slot sl = slots[b];
    const double c = psets[sl.p].c;
    const int2 r = vrec[sl.v];
    const int32_t tt = bs[b].ttau;
    const double hmax = bs[b].hmax;
    long long steps = 0, walks = 0;
    int ovf = 0;
    for (int32_t i = lane; i < r.y; i += 64) {
        const int64_t ie = sl.ie + i;
        long long nr = 0;
        const int32_t L = tau[ie] - tt;
        if (want[ie] && L > 0) {
            nr = nwalks(L, hmax, r.y, c);
            // walk keys carry a 32-bit walk index: 2^32 pairs or more would repeat walks
            if (nr < 0 || nr > kMaxPairs) {
                ovf = 1;
                nr = 0;
            }
        }
        nreq[ie] = nr;
        chunks[ie - ie0] = (2 * nr + kChunk - 1) / kChunk;
        steps += 2 * nr * (long long)(L > 0 ? L : 0);
        walks += 2 * nr;
    }
    steps = wave_sum_ll(steps);
    walks = wave_sum_ll(walks);
    ovf = wave_max_i(ovf);
    if (lane == 0) {
        if (steps) atomicAdd(&fl->walk_steps, (unsigned long long)steps);
        if (walks) atomicAdd(&fl->walks, (unsigned long long)walks);
        if (ovf) atomicOr(&fl->err, kErrOverflow);
    }
}

// The walk pairs (Alg. 1 inner loop).  Chunk c of local edge le holds walks
// j = 64 (c - coff[le]) + lane; j < n walk from s (side 0, index j), n <= j < 2n walk from t
// (side 1, index j - n).  Each walk sums h_ttau over its positions 1..L.  The persistent grid
// covers the flat chunk space of the whole batch (every instance edge of every request) in a
// fixed wavefront-strided order; the loop control depends only on the wavefront index, so the
// wavefront stays converged around its reductions.
//
// kCount (the counts export): every visit to the support of h_ttau also adds one to the
// integer histogram entry of (edge, side, support rank of the vertex), the rank found by
// binary search in the slot's final frontier list (the support in ascending order).  The
// walks, the sums and the totals are those of the plain instantiation.
struct CountArgs {
    const int32_t *FA = nullptr, *FB = nullptr;  // frontier lists of the two level parities
    const int64_t *hoff = nullptr;  // per instance: first histogram entry, -1 if not exported
    const int64_t *expect = nullptr;  // per instance: the support size of the caller's layout
    unsigned long long *hist = nullptr;
};

__device__ __forceinline__ int32_t support_rank(const int32_t *__restrict__ F, int32_t fsz,
                                                int32_t v) {
    int32_t lo = 0, hi = fsz;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (F[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Work queue of the walk-pair launch (kQueue): the flat chunk space is cut into kXcds
// contiguous ranges, one counter each.  A wavefront takes chunks from the range of its own
// XCD first (consecutive chunks belong to one source, whose support bitmap and h values then
// stay in that XCD's L2), then from the other ranges in turn.  The dequeue is wave-uniform by
// construction: the lowest active lane takes the ticket and readfirstlane, which reads that
// same lane, puts it in a scalar register, so every loop bound and cross-lane operation that
// follows sees one value.  Each counter only grows, so every wavefront leaves every range.
__device__ __forceinline__ int64_t wave_dequeue(unsigned long long *ctr) {
    const unsigned long long act = __ballot(1);
    const int leader = __builtin_ctzll(act);
    unsigned long long v = 0;
    if ((int)__lane_id() == leader) v = atomicAdd(ctr, 1ull);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Arguments of the walk-pair kernels.
struct McArgs {
    const int2 *vrec;
    const int32_t *col;
    const int4 *nbr;
    const Slot *slots;
    const PSet *psets;
    const BatchState *bs;
    int32_t nb;
    const int64_t *eb;
    int64_t ie0;
    const int64_t *coff;
    int64_t nle;
    const int32_t *tau;
    const long long *nreq;
    const double *hA, *hB;
    const uint32_t *bmA, *bmB;
    double *partial;
    unsigned long long *vis0, *vis1;
    CountArgs ca;
};

// The support bitmap of the slot a block has staged in LDS (mc_walk_staged_kernel).
extern __shared__ uint32_t mc_stage[];

// Chunk c of the walk pairs: 64 walks of one instance edge, reduced over the wavefront in a
// fixed order.  kLds: the support test reads the bitmap staged in LDS (the caller has staged
// the chunk's slot), else the slot's bitmap in global memory.
template <bool kCount, bool kLds>
__device__ __forceinline__ void mc_chunk(const McArgs &a, int64_t c) {
    const int lane = __lane_id();
    const int64_t le = upper_index(a.coff, a.nle + 1, c);
    const int64_t b = upper_index(a.eb, a.nb + 1, le);
    const Slot sl = a.slots[b];
    const PSet ps = a.psets[sl.p];
    const int2 rs = a.vrec[sl.v];
    const int32_t i = (int32_t)(le - a.eb[b]);
    const int64_t ie = a.ie0 + le;
    const int32_t t = a.col[rs.x + i];
    const long long nr = a.nreq[ie];
    const int32_t L = a.tau[ie] - a.bs[b].ttau;
    const int fb = a.bs[b].finalbuf;
    const double *h = (fb ? a.hB : a.hA) + sl.hoff;
    const uint32_t *bm = (fb ? a.bmB : a.bmA) + sl.bmoff;
    const long long j = (c - a.coff[le]) * kChunk + lane;
    const bool active = j < 2 * nr;
    const int side = j >= nr ? 1 : 0;
    const long long k = j - side * nr;
    double acc = 0.0;
    long long hits = 0;
    const int32_t *F = nullptr;
    int32_t fsz = 0;
    int64_t hrow = -1;
    if (kCount) {
        F = (fb ? a.ca.FB : a.ca.FA) + sl.hoff;
        fsz = a.bs[b].fsz[fb];
        // a support that differs from the layout's is not counted (the export flags it)
        const int64_t h0 = a.ca.hoff[sl.inst];
        if (h0 >= 0 && a.ca.expect[sl.inst] == fsz) hrow = h0 + ((int64_t)i * 2 + side) * fsz;
    }
    if (active) {
        const int32_t sloc = sl.v - sl.goff, tloc = t - sl.goff;
        Walker wk = walker_init<SABA_SAMPLER_KEYED>(walk_key(
            ps.seed, (uint32_t)sloc, (uint32_t)tloc, (uint32_t)side, (uint64_t)k, ps.G, ps.S));
        WalkPos p = walk_pos(a.vrec, side ? t : sl.v);
        for (int32_t l = 1; l <= L; ++l) {
            // the hash sees the graph's own vertex ids; the entry read is non-temporal where the
            // support bitmap is read from global memory (so that the random entry stream does
            // not push it out of L2) and cached where the bitmap sits in LDS
            if constexpr (kLds)
                p = walker_step_nbr<SABA_SAMPLER_KEYED>(a.nbr, p, (uint32_t)(p.v - sl.goff),
                                                        (uint32_t)l, wk);
            else
                p = walker_step_nbr_nt<SABA_SAMPLER_KEYED>(a.nbr, p, (uint32_t)(p.v - sl.goff),
                                                           (uint32_t)l, wk);
            const int32_t xl = p.v - sl.goff;
            uint32_t word;
            if constexpr (kLds)
                word = mc_stage[xl >> 5];
            else
                word = bm[xl >> 5];
            if (word & (1u << (xl & 31))) {  // h_ttau is zero off its support
                acc += h[xl];  // cached: the hubs' values are read again and again
                hits += 1;
                if (kCount && hrow >= 0)
                    atomicAdd(a.ca.hist + hrow + support_rank(F, fsz, p.v), 1ull);
            }
        }
    }
    const double sum = wave_sum_d(active ? (side ? -acc : acc) : 0.0);
    const long long h0 = wave_sum_ll(active && !side ? hits : 0);
    const long long h1 = wave_sum_ll(active && side ? hits : 0);
    if (lane == 0) {
        a.partial[c] = sum;
        if (h0) atomicAdd(a.vis0 + ie, (unsigned long long)h0);
        if (h1) atomicAdd(a.vis1 + ie, (unsigned long long)h1);
    }
}

template <bool kCount, bool kQueue>
__global__ __launch_bounds__(kBlock) void mc_walk_kernel(McArgs a, unsigned long long *__restrict__ wq) {
    const int64_t T = a.coff[a.nle];
    if (kQueue) {
        const int xcd = (int)(blockIdx.x % kXcds);  // the dispatcher deals blocks round-robin
        for (int r = 0; r < kXcds; ++r) {
            const int q = (xcd + r) % kXcds;
            const int64_t q0 = T * q / kXcds, q1 = T * (q + 1) / kXcds;
            for (;;) {
                const int64_t c = q0 + wave_dequeue(wq + q);
                if (c >= q1) break;
                mc_chunk<kCount, false>(a, c);
            }
        }
    } else {
        const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
        for (int64_t c = xcd_block() * kWavesPerBlock + (threadIdx.x >> 6); c < T; c += nwaves)
            mc_chunk<kCount, false>(a, c);
    }
}

// Tiles of the staged walk-pair launch: the chunks of slot b, [coff[eb[b]], coff[eb[b + 1]]),
// cut into tiles of up to kStageTile chunks; ntile[b] tiles.
constexpr int kStageBlock = 1024;  // threads of a staged block (16 wavefronts)
constexpr size_t kStageStatic = 256;  // room for the staged kernel's own LDS variables
constexpr int kMaxThreadsPerCu = 2048;
constexpr int kStageTile = 32;     // chunks per tile (two per wavefront)
constexpr int kStageMin = 16;      // a tile of fewer chunks is not worth staging the bitmap
constexpr int kStageLoads = 8;     // bitmap words per thread in flight while staging
__global__ __launch_bounds__(kBlock) void stage_tiles_kernel(const int64_t *__restrict__ eb,
                                                             int32_t nb,
                                                             const int64_t *__restrict__ coff,
                                                             int64_t *__restrict__ ntile) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int64_t nch = coff[eb[b + 1]] - coff[eb[b]];
    ntile[b] = (nch + kStageTile - 1) / kStageTile;
}

// The walk pairs with each slot's support bitmap staged in LDS.  A block takes a tile (chunks of
// one slot) from the work queue of its XCD's range of tiles, then from the other ranges; when
// the tile's slot differs from the staged one and the tile holds at least kStageMin chunks, the
// block copies the slot's bitmap into LDS; its wavefronts then take the tile's chunks one at a
// time from an LDS counter.  The support test of a step then reads LDS, so it no longer waits
// in line with the walk-entry and h loads.  A chunk's walks, sums and counts are those of the
// other walk-pair schedules.
__global__ __launch_bounds__(kStageBlock) void mc_walk_staged_kernel(
    McArgs a, const int64_t *__restrict__ toff, unsigned long long *__restrict__ tq) {
    __shared__ int64_t s_tile;
    __shared__ unsigned int s_next;
    const int32_t nb = a.nb;
    const int64_t TT = toff[nb];
    int64_t staged = -1;  // slot whose bitmap the LDS holds (block-uniform)
    const int xcd = (int)(blockIdx.x % kXcds);
    for (int r = 0; r < kXcds; ++r) {
        const int q = (xcd + r) % kXcds;
        const int64_t q0 = TT * q / kXcds, q1 = TT * (q + 1) / kXcds;
        for (;;) {
            if (threadIdx.x == 0) {
                s_tile = q0 + (int64_t)atomicAdd(tq + q, 1ull);
                s_next = 0;
            }
            __syncthreads();
            const int64_t u = s_tile;
            if (u >= q1) {
                __syncthreads();  // s_tile is read by every thread before it is rewritten
                break;
            }
            const int64_t b = upper_index(toff, nb + 1, u);
            const int64_t cb0 = a.coff[a.eb[b]], cb1 = a.coff[a.eb[b + 1]];
            const int64_t c0 = cb0 + (u - toff[b]) * kStageTile;
            const int64_t c1 = min(cb1, c0 + kStageTile);
            const bool stage = c1 - c0 >= kStageMin;
            if (stage && b != staged) {
                const Slot sl = a.slots[b];
                const uint32_t *bm = (a.bs[b].finalbuf ? a.bmB : a.bmA) + sl.bmoff;
                const int32_t words = (sl.gn + 31) >> 5;
                // kStageLoads coalesced loads in flight per thread before their LDS stores
                for (int32_t w0 = threadIdx.x; w0 < words; w0 += kStageLoads * kStageBlock) {
                    uint32_t v[kStageLoads];
#pragma unroll
                    for (int u = 0; u < kStageLoads; ++u) {
                        const int32_t w = w0 + u * kStageBlock;
                        v[u] = w < words ? bm[w] : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < kStageLoads; ++u) {
                        const int32_t w = w0 + u * kStageBlock;
                        if (w < words) mc_stage[w] = v[u];
                    }
                }
                staged = b;
                __syncthreads();
            }
            for (;;) {
                unsigned int v = 0;
                const unsigned long long act = __ballot(1);
                if ((int)__lane_id() == __builtin_ctzll(act)) v = atomicAdd(&s_next, 1u);
                const int64_t c = c0 + (int64_t)__builtin_amdgcn_readfirstlane(v);
                if (c >= c1) break;
                if (stage)
                    mc_chunk<false, true>(a, c);
                else
                    mc_chunk<false, false>(a, c);
            }
            __syncthreads();  // the tile is done before s_tile, s_next and the LDS are rewritten
        }
    }
}

// Counts export, per slot: the size of the final support and, where the instance is exported
// (soff >= 0), the support in ascending order (graph-local ids) with h_ttau there.  A support
// whose size differs from the one the caller laid its arrays out for sets kErrLayout and is
// not written.
struct CountExport {
    int64_t *supp_sz = nullptr;      // per instance, out
    const int64_t *soff = nullptr;   // per instance: first support entry, -1 if not exported
    const int64_t *expect = nullptr; // per instance: the support size of the layout
    int32_t *supp = nullptr;
    double *h = nullptr;
    CountArgs ca;
};

__global__ __launch_bounds__(kBlock) void count_support_kernel(
    const Slot *__restrict__ slots, const BatchState *__restrict__ bs, const double *__restrict__ hA,
    const double *__restrict__ hB, const int32_t *__restrict__ FA, const int32_t *__restrict__ FB,
    CountExport cx, Flags *__restrict__ fl) {
    const int64_t b = blockIdx.y;
    const Slot sl = slots[b];
    const int pb = bs[b].finalbuf;
    const int32_t fsz = bs[b].fsz[pb];
    if (blockIdx.x == 0 && threadIdx.x == 0) cx.supp_sz[sl.inst] = fsz;
    if (!cx.supp) return;
    const int64_t so = cx.soff[sl.inst];
    if (so < 0) return;
    if (cx.expect[sl.inst] != fsz) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&fl->err, kErrLayout);
        return;
    }
    const double *h = (pb ? hB : hA) + sl.hoff;
    const int32_t *F = (pb ? FB : FA) + sl.hoff;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < fsz;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = F[i] - sl.goff;
        cx.supp[so + i] = x;
        cx.h[so + i] = h[x];
    }
}

// Per instance edge: MC = the sum of its chunk sums; g(s,t) = (D + MC / n) / d_s.  The order of
// that sum depends only on the edge's chunk count: up to kSerialChunks chunks are added left to
// right by one lane; more are split over the 64 lanes of a wavefront (lane l adds chunks
// l, l + 64, ... left to right) and the lane sums are combined in the butterfly order of lane 0.
// Neither depends on where the edge sits in its batch.
constexpr int64_t kSerialChunks = 64;

__device__ __forceinline__ void edge_finish(const int2 *__restrict__ vrec,
                                            const Slot *__restrict__ slots, int32_t nb,
                                            const int64_t *__restrict__ eb, int64_t le,
                                            int64_t ie, const long long *__restrict__ nreq,
                                            const double *__restrict__ D, double mc,
                                            double *__restrict__ MC, double *__restrict__ g) {
    const int64_t b = upper_index(eb, nb + 1, le);
    const int32_t ds = vrec[slots[b].v].y;
    const long long nr = nreq[ie];
    MC[ie] = mc;
    g[ie] = nr > 0 ? (D[ie] + mc / (double)nr) / (double)ds : D[ie] / (double)ds;
}

__global__ __launch_bounds__(kBlock) void edge_reduce_kernel(
    const int2 *__restrict__ vrec, const Slot *__restrict__ slots, int32_t nb,
    const int64_t *__restrict__ eb, int64_t ie0, const int64_t *__restrict__ coff, int64_t nle,
    const uint8_t *__restrict__ want, const long long *__restrict__ nreq,
    const double *__restrict__ D, const double *__restrict__ partial, double *__restrict__ MC,
    double *__restrict__ g) {
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    // each wavefront owns 64 consecutive edges per round; the round count is wave-uniform
    for (int64_t base = ((int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)) * 64;
         base < nle; base += nwaves * 64) {
        const int64_t le = base + lane;
        const bool mine = le < nle && want[ie0 + le];
        const int64_t c0 = mine ? coff[le] : 0, c1 = mine ? coff[le + 1] : 0;
        const bool big = mine && (c1 - c0) > kSerialChunks;
        if (mine && !big) {
            double mc = 0.0;
            for (int64_t c = c0; c < c1; ++c) mc += partial[c];
            edge_finish(vrec, slots, nb, eb, le, ie0 + le, nreq, D, mc, MC, g);
        }
        unsigned long long bigs = __ballot(big);
        while (bigs) {  // wave-uniform: the ballot is the same in every lane
            const int src = __builtin_ctzll(bigs);
            bigs &= bigs - 1;
            const int64_t b0 = __shfl(c0, src), b1 = __shfl(c1, src);
            double part = 0.0;
            for (int64_t c = b0 + lane; c < b1; c += 64) part += partial[c];
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
            // lanes may round the butterfly differently: lane 0's order is the defined one
            const double tot = __shfl(part, 0);
            if (lane == src) edge_finish(vrec, slots, nb, eb, le, ie0 + le, nreq, D, tot, MC, g);
        }
    }
}

// SC of the i-th canonical edge of a graph whose instances are all its vertices, in order:
// the instance edge of a CSR position e is base + (e - gpos).
__global__ void finalize_all_kernel(const int32_t *__restrict__ canon,
                                    const int32_t *__restrict__ rev, int64_t cb, int64_t m,
                                    int64_t base, int32_t gpos, const double *__restrict__ g,
                                    double *__restrict__ sc) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = canon[cb + i];
        sc[i] = g[base + (e - gpos)] + g[base + (rev[e] - gpos)];
    }
}

__global__ void finalize_pairs_kernel(const int64_t *__restrict__ pairs, int64_t q,
                                      const double *__restrict__ g, double *__restrict__ sc) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q;
         j += (int64_t)gridDim.x * blockDim.x)
        sc[j] = g[pairs[2 * j]] + g[pairs[2 * j + 1]];
}

// All edges of one graph in canonical order: the edge (row_of[e], col[e]) with its tau.
__global__ void tail_all_kernel(const int32_t *__restrict__ canon, const int32_t *__restrict__ row_of,
                                const int32_t *__restrict__ col, int64_t cb, int64_t m,
                                int64_t base, int32_t gpos, int32_t goff,
                                const int32_t *__restrict__ tau, const double *__restrict__ theta,
                                const double *__restrict__ y, int64_t gn, int32_t pairs,
                                double *__restrict__ sc) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = canon[cb + i];
        sc[i] += eigen_tail(theta, y, gn, pairs, row_of[e] - goff, col[e] - goff,
                            tau[base + (e - gpos)]);
    }
}

// Query pairs (graph-local ids) with the tau of their first instance edge.
__global__ void tail_pairs_kernel(const int32_t *__restrict__ edges,
                                  const int64_t *__restrict__ pairs_ie, int64_t q,
                                  const int32_t *__restrict__ tau, const double *__restrict__ theta,
                                  const double *__restrict__ y, int64_t gn, int32_t pairs,
                                  double *__restrict__ sc) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q;
         j += (int64_t)gridDim.x * blockDim.x)
        sc[j] += eigen_tail(theta, y, gn, pairs, edges[2 * j], edges[2 * j + 1],
                            tau[pairs_ie[2 * j]]);
}

__global__ void export_ttau_kernel(const int32_t *__restrict__ row_of, int64_t nnz,
                                   const int32_t *__restrict__ ttau_inst,
                                   int32_t *__restrict__ ttau) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        ttau[e] = ttau_inst[row_of[e]];
}

// ------------------------------------------------------------ batch executor
unsigned grid_for(int64_t items, int per_block, unsigned cap) {
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

int check_request(const Graph *g, int32_t graph, const saba_aesc_params &pr, int64_t q,
                  const void *edges) {
    const saba_aesc_params *p = &pr;
    if (graph < 0 || graph >= g->ngraphs) {
        set_error("request names a graph the handle does not hold");
        return SABA_E_INVALID;
    }
    if (!(p->eps > 0.0) || !(p->delta > 0.0 && p->delta < 1.0) || !(p->lambda > 0.0) ||
        p->group < 1 || p->spread > 31 ||
        (p->group > 1 && ((uint64_t)(p->group - 1) << p->spread) > 0xFFFFFFFFull) || q < -1 ||
        (q > 0 && !edges)) {
        set_error("invalid estimator parameters");
        return SABA_E_INVALID;
    }
    const int32_t a = g->goff[graph], z = g->goff[graph + 1];
    if (p->omega < 0 || p->omega > kMaxOmega || (p->omega > 0 && p->omega >= z - a)) {
        set_error("omega must lie in [0, 64] and below the vertex count of the graph");
        return SABA_E_INVALID;
    }
    if (!g->gconnected[graph] || z - a < 2) {
        set_error("the estimator needs a connected graph with at least one edge");
        return SABA_E_DISCONNECTED;
    }
    if (g->gbipartite[graph] || !(p->lambda < 1.0)) {
        set_error("the estimator needs a non-bipartite graph (lambda < 1)");
        return SABA_E_BIPARTITE;
    }
    return SABA_OK;
}

PSet make_pset(const Graph *g, int32_t graph, const saba_aesc_params &p) {
    const int32_t *rp = g->h_row_ptr.data();
    const int64_t m = ((int64_t)rp[g->goff[graph + 1]] - rp[g->goff[graph]]) / 2;
    PSet ps;
    ps.lambda = p.lambda;
    ps.eps = p.eps;
    ps.c = 32.0 * std::log(4.0 * (double)m / p.delta) / (p.eps * p.eps);
    ps.seed = p.seed;
    ps.G = p.group;
    ps.S = p.spread;
    ps.tau_cap = p.tau_cap > 0 ? p.tau_cap : 4096;
    ps.tilde_tau_max = p.tilde_tau_max;
    ps.push_all = p.push_all ? 1 : 0;
    return ps;
}

bool same_pset(const PSet &a, const PSet &b) {
    return a.lambda == b.lambda && a.eps == b.eps && a.c == b.c && a.seed == b.seed &&
           a.G == b.G && a.S == b.S && a.tau_cap == b.tau_cap &&
           a.tilde_tau_max == b.tilde_tau_max && a.push_all == b.push_all;
}

SlotSize slot_size(const Graph *g, int32_t graph) {
    const int32_t *rp = g->h_row_ptr.data();
    const int32_t ga = g->goff[graph], gz = g->goff[graph + 1];
    const int64_t gn = gz - ga, gnnz = (int64_t)rp[gz] - rp[ga];
    SlotSize z;
    z.h = gn;
    z.bm = (gn + 31) / 32;
    z.sb = (gnnz + 31) / 32;
    z.hubs = g->ghubs[graph];
    z.bytes = gn * (2 * 8 + 2 * 4) + 2 * 4 * z.bm + 4 * z.sb + 2 * 8 * z.hubs;
    return z;
}

int ensure_edge_arrays(Workspace &ws, int64_t ne, int64_t ninst, int32_t np, EdgeArrays *out) {
    auto &E = ws.b;
    const int64_t n1 = std::max<int64_t>(ne, 1);
    SABA_TRY(E[B_PSET].ensure(sizeof(PSet) * std::max(np, 1)));
    SABA_TRY(E[B_WANT].ensure(n1));
    SABA_TRY(E[B_TAU].ensure(sizeof(int32_t) * n1));
    SABA_TRY(E[B_D].ensure(sizeof(double) * n1));
    SABA_TRY(E[B_NREQ].ensure(sizeof(long long) * n1));
    SABA_TRY(E[B_MC].ensure(sizeof(double) * n1));
    SABA_TRY(E[B_VIS0].ensure(sizeof(long long) * n1));
    SABA_TRY(E[B_VIS1].ensure(sizeof(long long) * n1));
    SABA_TRY(E[B_G].ensure(sizeof(double) * n1));
    SABA_TRY(E[B_TTAU].ensure(sizeof(int32_t) * std::max<int64_t>(ninst, 1)));
    SABA_TRY(E[B_FLAGS].ensure(sizeof(Flags)));
    out->psets = E[B_PSET].as<PSet>();
    out->want = E[B_WANT].as<uint8_t>();
    out->tau = E[B_TAU].as<int32_t>();
    out->D = E[B_D].as<double>();
    out->nreq = E[B_NREQ].as<long long>();
    out->MC = E[B_MC].as<double>();
    out->vis0 = E[B_VIS0].as<unsigned long long>();
    out->vis1 = E[B_VIS1].as<unsigned long long>();
    out->g = E[B_G].as<double>();
    out->ttau_inst = E[B_TTAU].as<int32_t>();
    out->fl = E[B_FLAGS].as<Flags>();
    return SABA_OK;
}

int ensure_pools(Workspace &ws, int64_t h, int64_t bm, int64_t sb, int64_t hubs, int64_t nb,
                 int64_t ne, hipStream_t s) {
    auto &E = ws.b;
    h = std::max<int64_t>(h, 1);
    bm = std::max<int64_t>(bm, 1);
    sb = std::max<int64_t>(sb, 1);
    nb = std::max<int64_t>(nb, 1);
    ne = std::max<int64_t>(ne, 1);
    const bool grow = E[B_HA].bytes < sizeof(double) * (size_t)h ||
                      E[B_BMA].bytes < sizeof(uint32_t) * (size_t)bm ||
                      E[B_SLOTBM].bytes < sizeof(uint32_t) * (size_t)sb;
    if (grow) ws.clean = false;  // new pools hold garbage until zeroed below
    SABA_TRY(E[B_HA].ensure(sizeof(double) * h));
    SABA_TRY(E[B_HB].ensure(sizeof(double) * h));
    SABA_TRY(E[B_FA].ensure(sizeof(int32_t) * h));
    SABA_TRY(E[B_FB].ensure(sizeof(int32_t) * h));
    SABA_TRY(E[B_BMA].ensure(sizeof(uint32_t) * bm));
    SABA_TRY(E[B_BMB].ensure(sizeof(uint32_t) * bm));
    SABA_TRY(E[B_SLOTBM].ensure(sizeof(uint32_t) * sb));
    SABA_TRY(E[B_SLOT].ensure(sizeof(Slot) * nb));
    SABA_TRY(E[B_EB].ensure(sizeof(int64_t) * (nb + 1)));
    SABA_TRY(E[B_BSTATE].ensure(sizeof(BatchState) * nb));
    SABA_TRY(E[B_GOFS].ensure(sizeof(int64_t) * 2 * (nb + 1)));
    SABA_TRY(E[B_TILES].ensure(sizeof(int64_t) * (2 * nb + 1)));
    SABA_TRY(E[B_HUBS].ensure(sizeof(int2) * 2 * std::max<int64_t>(hubs, 1)));
    SABA_TRY(E[B_CHUNKS].ensure(sizeof(long long) * ne));
    SABA_TRY(E[B_COFF].ensure(sizeof(int64_t) * (ne + 1)));
    SABA_TRY(E[B_SCAN].ensure(scan_tmp_bytes(ne)));
    if (grow || !ws.clean) {
        // dense vectors and bitmaps start at zero and are kept clean by the sparse clears
        SABA_HIP_TRY(hipMemsetAsync(E[B_HA].ptr, 0, E[B_HA].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(E[B_HB].ptr, 0, E[B_HB].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(E[B_BMA].ptr, 0, E[B_BMA].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(E[B_BMB].ptr, 0, E[B_BMB].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(E[B_SLOTBM].ptr, 0, E[B_SLOTBM].bytes, s));
        ws.clean = true;
    }
    return SABA_OK;
}

int batch_levels(const Graph *g, Workspace &ws, const EdgeArrays &ea,
                 const std::vector<Slot> &hslots, const std::vector<int64_t> &heb, int64_t ie0,
                 int64_t nle, int64_t maxgn, int64_t hubcap, hipStream_t s, BatchPlan *plan) {
    auto &E = ws.b;
    const int32_t nb = (int32_t)hslots.size();
    *plan = BatchPlan{};
    if (nb == 0) return SABA_OK;
    if (nb > 65535) {
        set_error("a batch holds at most 65535 instances");
        return SABA_E_INVALID;
    }
    double *hA = E[B_HA].as<double>(), *hB = E[B_HB].as<double>();
    int32_t *FA = E[B_FA].as<int32_t>(), *FB = E[B_FB].as<int32_t>();
    uint32_t *bmA = E[B_BMA].as<uint32_t>(), *bmB = E[B_BMB].as<uint32_t>();
    uint32_t *slotbm = E[B_SLOTBM].as<uint32_t>();
    Slot *d_slots = E[B_SLOT].as<Slot>();
    int64_t *d_eb = E[B_EB].as<int64_t>();
    BatchState *bs = E[B_BSTATE].as<BatchState>();
    long long *chunks = E[B_CHUNKS].as<long long>();
    int64_t *coff = E[B_COFF].as<int64_t>();
    int64_t *gofs_cur = E[B_GOFS].as<int64_t>(), *gofs_nxt = gofs_cur + (nb + 1);
    int2 *hubs = E[B_HUBS].as<int2>();
    hubcap = std::max<int64_t>(hubcap, 1);
    Flags *fl = ea.fl;
    // execution knobs of the handle (none changes a result)
    const unsigned push_blocks = g->cfg.est_push_blocks > 0 ? g->cfg.est_push_blocks : kPushGrid;
    ws.clean = false;  // until the batch has cleared everything it touched

    SABA_HIP_TRY(hipMemcpyAsync(d_slots, hslots.data(), sizeof(Slot) * nb, hipMemcpyHostToDevice,
                                s));
    SABA_HIP_TRY(hipMemcpyAsync(d_eb, heb.data(), sizeof(int64_t) * (nb + 1),
                                hipMemcpyHostToDevice, s));
    SABA_HIP_TRY(hipMemsetAsync(&fl->nhub[0], 0, 2 * sizeof(int32_t), s));
    batch_init_kernel<<<grid_for(nb, kWavesPerBlock), kBlock, 0, s>>>(
        g->vrec, g->col_idx, d_slots, ea.psets, nb, bs, hA, FA, bmA, ea.tau, ea.D, ea.nreq, ea.MC,
        ea.vis0, ea.vis1, hubs, fl);
    SABA_HIP_TRY(hipGetLastError());
    const unsigned ysplit = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, maxgn / 4096));
    for (int32_t level = 0;; ++level) {
        const int cur = level & 1;
        double *hcur = cur ? hB : hA, *hnext = cur ? hA : hB;
        int32_t *Fcur = cur ? FB : FA, *Fnext = cur ? FA : FB;
        uint32_t *bmcur = cur ? bmB : bmA, *bmnext = cur ? bmA : bmB;
        SABA_HIP_TRY(hipMemsetAsync(&fl->any_active, 0, sizeof(int32_t), s));
        level_decide_kernel<<<grid_for(nb, kWavesPerBlock), kBlock, 0, s>>>(
            g->vrec, g->col_idx, d_slots, ea.psets, bs, nb, level, hcur, ea.tau, ea.D,
            ea.ttau_inst, fl);
        SABA_HIP_TRY(hipGetLastError());
        int32_t any = 0;
        SABA_HIP_TRY(
            hipMemcpyAsync(&any, &fl->any_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipStreamSynchronize(s));
        if (!any) break;
        group_scan_kernel<<<1, 1024, 0, s>>>(bs, nb, cur, gofs_cur);
        expand_kernel<<<push_blocks, kBlock, 0, s>>>(g->vrec, g->col_idx, g->slotv, d_slots, bs, nb,
                                                   level, gofs_cur, Fcur, bmnext, slotbm, fl);
        expand_hub_kernel<<<kHubGrid, kBlock, 0, s>>>(g->vrec, g->col_idx, g->slotv, d_slots, bs,
                                                      level, hubs, hubcap, bmnext, slotbm, fl);
        compact_frontier_kernel<<<(unsigned)nb, kBlock, 0, s>>>(g->hubbm, d_slots, bs, level,
                                                                bmnext, Fnext, hubs, hubcap, fl);
        group_scan_kernel<<<1, 1024, 0, s>>>(bs, nb, cur ^ 1, gofs_nxt);
        pull_kernel<<<push_blocks, kBlock, 0, s>>>(g->vrec, g->col_idx, d_slots, bs, nb, level,
                                                 gofs_nxt, hcur, bmcur, hnext, Fnext, fl);
        pull_hub_kernel<<<kHubGrid, kBlock, 0, s>>>(g->vrec, g->col_idx, d_slots, bs, level, hubs,
                                                    hubcap, hcur, slotbm, hnext, fl);
        clear_groups_kernel<<<push_blocks, kBlock, 0, s>>>(d_slots, bs, nb, cur, gofs_cur, hcur,
                                                            bmcur, Fcur);
        SABA_HIP_TRY(hipGetLastError());
    }
    // walk pairs of the batch's instance edges
    nreq_kernel<<<grid_for(nb, kWavesPerBlock), kBlock, 0, s>>>(
        g->vrec, d_slots, ea.psets, bs, nb, ie0, ea.tau, ea.want, ea.nreq, chunks, fl);
    SABA_HIP_TRY(hipGetLastError());
    SABA_TRY(scan_i64(reinterpret_cast<int64_t *>(chunks), coff, nle, E[B_SCAN].ptr, s));
    int64_t T = 0;
    int32_t err = 0;
    SABA_HIP_TRY(hipMemcpyAsync(&T, coff + nle, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipMemcpyAsync(&err, &fl->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipStreamSynchronize(s));
    if (err & kErrOverflow) {
        set_error("walk count overflows the 64-bit range (eps too small?)");
        return SABA_E_OVERFLOW;  // the pools stay marked dirty: re-zeroed before the next use
    }
    SABA_TRY(E[B_PART].ensure(sizeof(double) * std::max<int64_t>(T, 1)));
    plan->nb = nb;
    plan->ie0 = ie0;
    plan->nle = nle;
    plan->T = T;
    plan->ysplit = ysplit;
    plan->maxgn = maxgn;
    return SABA_OK;
}

int batch_walks(const Graph *g, Workspace &ws, const EdgeArrays &ea, const BatchPlan &plan,
                hipEvent_t t0, hipEvent_t t1, hipStream_t s, const CountExport *cx) {
    auto &E = ws.b;
    const int32_t nb = plan.nb;
    if (nb == 0) return SABA_OK;
    const int64_t ie0 = plan.ie0, nle = plan.nle, T = plan.T;
    double *hA = E[B_HA].as<double>(), *hB = E[B_HB].as<double>();
    int32_t *FA = E[B_FA].as<int32_t>(), *FB = E[B_FB].as<int32_t>();
    uint32_t *bmA = E[B_BMA].as<uint32_t>(), *bmB = E[B_BMB].as<uint32_t>();
    Slot *d_slots = E[B_SLOT].as<Slot>();
    int64_t *d_eb = E[B_EB].as<int64_t>();
    BatchState *bs = E[B_BSTATE].as<BatchState>();
    int64_t *coff = E[B_COFF].as<int64_t>();
    double *partial = E[B_PART].as<double>();
    Flags *fl = ea.fl;
    const unsigned walk_blocks = g->cfg.est_walk_blocks > 0 ? g->cfg.est_walk_blocks : kWalkGrid;
    const dim3 grid(plan.ysplit, (unsigned)nb);
    if (T > 0) {
        const bool timing = t0 && t1;
        const bool counts = cx && cx->supp;
        const McArgs ma{g->vrec, g->col_idx, g->nbr, d_slots, ea.psets, bs, nb, d_eb, ie0, coff,
                        nle, ea.tau, ea.nreq, hA, hB, bmA, bmB, partial, ea.vis0, ea.vis1,
                        counts ? cx->ca : CountArgs{}};
        // the staged schedule needs the largest graph's support bitmap to fit a block's LDS
        int max_lds = 0;
        SABA_HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                           g->device));
        const size_t stage_lds = sizeof(uint32_t) * (size_t)((plan.maxgn + 31) / 32);
        const bool staged = g->cfg.est_walk_queue == 2 && !counts &&
                            stage_lds + kStageStatic <= (size_t)max_lds;
        const bool queue = g->cfg.est_walk_queue >= 1 && !staged;
        int64_t *ntile = E[B_TILES].as<int64_t>(), *toff = ntile + nb;
        if (staged) {
            stage_tiles_kernel<<<grid_for(nb, kBlock), kBlock, 0, s>>>(d_eb, nb, coff, ntile);
            SABA_HIP_TRY(hipGetLastError());
            SABA_TRY(scan_i64(ntile, toff, nb, E[B_SCAN].ptr, s));
            // the limit is a property of the kernel, shared by every caller in the process: it
            // is always set to the same value (the most a block may take), so calls from several
            // host threads (the server's lanes, on graphs of different sizes) agree on it
            SABA_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&mc_walk_staged_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             max_lds - (int)kStageStatic));
        }
        if (staged || queue) SABA_HIP_TRY(hipMemsetAsync(fl->wq, 0, sizeof(fl->wq), s));
        if (timing) SABA_HIP_TRY(hipEventRecord(t0, s));
        if (staged) {
            // as many blocks as the compute units hold at once (the LDS bounds them)
            const int per_cu = (int)std::max<size_t>(
                1, std::min<size_t>(kMaxThreadsPerCu / kStageBlock,
                                    (size_t)max_lds / (stage_lds + kStageStatic)));
            int cus = 0;
            SABA_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                               g->device));
            mc_walk_staged_kernel<<<(unsigned)(std::max(cus, 1) * per_cu), kStageBlock,
                                    stage_lds, s>>>(ma, toff, fl->wq);
        } else {
            const unsigned wgrid = grid_for(T, kWavesPerBlock, walk_blocks);
            if (counts) {
                if (queue)
                    mc_walk_kernel<true, true><<<wgrid, kBlock, 0, s>>>(ma, fl->wq);
                else
                    mc_walk_kernel<true, false><<<wgrid, kBlock, 0, s>>>(ma, fl->wq);
            } else if (queue) {
                mc_walk_kernel<false, true><<<wgrid, kBlock, 0, s>>>(ma, fl->wq);
            } else {
                mc_walk_kernel<false, false><<<wgrid, kBlock, 0, s>>>(ma, fl->wq);
            }
        }
        SABA_HIP_TRY(hipGetLastError());
        if (timing) SABA_HIP_TRY(hipEventRecord(t1, s));
    }
    edge_reduce_kernel<<<grid_for(nle, kBlock, 1 << 16), kBlock, 0, s>>>(
        g->vrec, d_slots, nb, d_eb, ie0, coff, nle, ea.want, ea.nreq, ea.D, partial, ea.MC, ea.g);
    if (cx)
        count_support_kernel<<<grid, kBlock, 0, s>>>(d_slots, bs, hA, hB, FA, FB, *cx, fl);
    // leave the dense vectors and bitmaps of the batch zero: clear h_ttau over its support
    clear_final_kernel<<<grid, kBlock, 0, s>>>(d_slots, bs, hA, hB, bmA, bmB, FA, FB);
    SABA_HIP_TRY(hipGetLastError());
    ws.clean = true;
    return SABA_OK;
}

int run_batch(const Graph *g, Workspace &ws, const EdgeArrays &ea, const std::vector<Slot> &hslots,
              const std::vector<int64_t> &heb, int64_t ie0, int64_t nle, int64_t maxgn,
              int64_t hubcap, BatchTiming *tm, hipStream_t s, const CountExport *cx) {
    BatchPlan plan;
    SABA_TRY(batch_levels(g, ws, ea, hslots, heb, ie0, nle, maxgn, hubcap, s, &plan));
    const bool timing = tm && tm->on && plan.T > 0;
    SABA_TRY(batch_walks(g, ws, ea, plan, timing ? tm->a : nullptr, timing ? tm->b : nullptr, s,
                         cx));
    if (timing) {
        SABA_HIP_TRY(hipEventSynchronize(tm->b));
        float ms = 0.f;
        SABA_HIP_TRY(hipEventElapsedTime(&ms, tm->a, tm->b));
        tm->walk_ms += ms;
    }
    return SABA_OK;
}

// ------------------------------------------------------------ synchronous calls
struct Request {
    int32_t graph = 0;
    saba_aesc_params p{};
    const int32_t *edges = nullptr;  // device, graph-local ids
    int64_t q = -1;                  // -1: all edges of the graph
    double *sc = nullptr;
    int32_t pid = -1;
    const Spectrum *spec = nullptr;  // eigenpairs of the omega > 0 correction
};

struct Exports {  // per CSR position (single graph, all edges)
    int32_t *tau = nullptr, *ttau = nullptr;
    int64_t *nreq = nullptr, *vis0 = nullptr, *vis1 = nullptr;
    double *D = nullptr, *MC = nullptr, *g = nullptr;
};

// The counts export of saba_aesc_counts: one request whose instances are the listed sources,
// with all their edges wanted.
struct CountJob {
    std::vector<int32_t> src;        // graph-local source vertices, in the caller's order
    saba_count_source *layout = nullptr;
    int32_t *supp = nullptr;         // all three null: layout only
    double *h = nullptr;
    int64_t *hist = nullptr;
    Exports edges;                   // per-edge outputs, indexed by layout[k].edge_off + i
};

struct Opts {
    int64_t mem_budget = 0;
    int32_t batch_sources = 0;
    int32_t time_kernels = 0;
};

static bool same_params(const Request &a, const Request &b) {
    const saba_aesc_params &x = a.p, &y = b.p;
    return a.graph == b.graph && x.eps == y.eps && x.delta == y.delta && x.lambda == y.lambda &&
           x.seed == y.seed && x.group == y.group && x.spread == y.spread &&
           x.tau_cap == y.tau_cap && x.tilde_tau_max == y.tilde_tau_max &&
           (x.push_all != 0) == (y.push_all != 0);
}

// The estimator's second stream (default priority) and its hand-over events, created once per
// handle.
static int ensure_est_pipeline(Graph *g) {
    if (g->est_aux) return SABA_OK;
    for (auto &e : g->est_ev)
        if (!e) SABA_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipStream_t st = nullptr;
    SABA_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    g->est_aux = st;
    return SABA_OK;
}

static void merge_flags(Flags &a, const Flags &b) {
    a.err |= b.err;
    a.max_tau = std::max(a.max_tau, b.max_tau);
    a.max_ttau = std::max(a.max_ttau, b.max_ttau);
    a.warnings |= b.warnings;
    a.walk_steps += b.walk_steps;
    a.push_visits += b.push_visits;
    a.walks += b.walks;
}

static int aesc_run(Graph *g, std::vector<Request> &reqs, const Opts &opt, const Exports *ex,
                    saba_stats *st, hipStream_t s, CountJob *cj = nullptr) {
    const int32_t *rp = g->h_row_ptr.data();
    const int32_t *ci = g->h_col_idx.data();
    for (auto &r : reqs) {
        if (r.graph < 0 || r.graph >= g->ngraphs || !g->gconnected[r.graph]) continue;
        const int32_t gn = g->goff[r.graph + 1] - g->goff[r.graph];
        if (r.p.omega > 0 && r.p.omega <= kMaxOmega && r.p.omega < gn && !g->gbipartite[r.graph]) {
            // tau from the radius of the spectrum outside the kept pairs
            SABA_TRY(resolve_spectrum(g, r.graph, r.p.omega, &r.spec, s));
            if (r.p.lambda <= 0.0)
                r.p.lambda = std::min(std::max(r.spec->lambda_rest_bound, DBL_MIN), 1.0 - 1e-12);
        } else if (r.p.lambda <= 0.0 && r.p.omega == 0) {
            SABA_TRY(resolve_lambda(g, r.graph, &r.p.lambda, s));
        }
    }
    for (auto &r : reqs) SABA_TRY(check_request(g, r.graph, r.p, r.q, r.edges));

    // parameter sets: requests with equal (graph, parameters) share their instances
    std::vector<PSet> psets;
    std::vector<int32_t> pgraph;
    std::vector<int32_t> plead;  // a request of each parameter set
    for (size_t i = 0; i < reqs.size(); ++i) {
        int32_t pid = -1;
        for (size_t k = 0; k < plead.size(); ++k)
            if (same_params(reqs[plead[k]], reqs[i])) pid = (int32_t)k;
        if (pid < 0) {
            pid = (int32_t)psets.size();
            psets.push_back(make_pset(g, reqs[i].graph, reqs[i].p));
            pgraph.push_back(reqs[i].graph);
            plead.push_back((int32_t)i);
        }
        reqs[i].pid = pid;
    }
    const int32_t P = (int32_t)psets.size();

    // query pairs to the host (validated there against the resident CSR copy)
    std::vector<std::vector<int32_t>> hq(reqs.size());
    for (size_t i = 0; i < reqs.size(); ++i) {
        if (reqs[i].q <= 0) continue;
        hq[i].resize(2 * reqs[i].q);
        SABA_HIP_TRY(hipMemcpyAsync(hq[i].data(), reqs[i].edges, sizeof(int32_t) * 2 * reqs[i].q,
                                    hipMemcpyDeviceToHost, s));
    }
    SABA_HIP_TRY(hipStreamSynchronize(s));
    auto find_pos = [&](int32_t u, int32_t v) -> int32_t {
        const int32_t *a = ci + rp[u], *z = ci + rp[u + 1];
        const int32_t *f = std::lower_bound(a, z, v);
        return (f != z && *f == v) ? (int32_t)(f - ci) : -1;
    };

    // instances: per parameter set, every vertex of its graph (an all-edges request) or the
    // distinct endpoints of its query pairs; the instance list is ordered by (parameter set,
    // vertex).  Query-only sets keep their endpoints as a sorted list, so the set-up costs
    // O(q log q) per set, not a pass over the graph's vertices.
    std::vector<uint8_t> pall(P, 0);
    std::vector<std::vector<int32_t>> pverts(P);
    for (size_t i = 0; i < reqs.size(); ++i) {
        const Request &r = reqs[i];
        const int32_t ga = g->goff[r.graph], gn = g->goff[r.graph + 1] - ga;
        if (cj) {
            for (const int32_t x : cj->src) pverts[r.pid].push_back(x);
            continue;
        }
        if (r.q < 0) {
            pall[r.pid] = 1;
            continue;
        }
        for (int64_t j = 0; j < r.q; ++j) {
            const int32_t u = hq[i][2 * j], v = hq[i][2 * j + 1];
            if (u < 0 || v < 0 || u >= gn || v >= gn || find_pos(ga + u, ga + v) < 0) {
                set_error("a query pair is not an edge of the graph");
                return SABA_E_NOT_EDGE;
            }
            pverts[r.pid].push_back(u);
            pverts[r.pid].push_back(v);
        }
    }
    std::vector<int32_t> inst_v, inst_p;
    std::vector<int64_t> iebase;
    std::vector<int64_t> pbase(P, 0), pfirst(P, 0);
    int64_t NE = 0;
    for (int32_t k = 0; k < P; ++k) {
        const int32_t ga = g->goff[pgraph[k]];
        const int32_t gn = g->goff[pgraph[k] + 1] - ga;
        pbase[k] = NE;
        pfirst[k] = (int64_t)inst_v.size();
        const auto add = [&](int32_t x) {
            inst_v.push_back(ga + x);
            inst_p.push_back(k);
            iebase.push_back(NE);
            NE += rp[ga + x + 1] - rp[ga + x];
        };
        if (pall[k]) {
            pverts[k].clear();
            for (int32_t x = 0; x < gn; ++x) add(x);
        } else {
            std::vector<int32_t> &pv = pverts[k];
            std::sort(pv.begin(), pv.end());
            pv.erase(std::unique(pv.begin(), pv.end()), pv.end());
            for (const int32_t x : pv) add(x);
        }
    }
    // the instance of graph-local vertex x in parameter set k (x an instance vertex of k)
    const auto inst_of = [&](int32_t k, int32_t x) -> int64_t {
        if (pall[k]) return pfirst[k] + x;
        const std::vector<int32_t> &pv = pverts[k];
        return pfirst[k] + (std::lower_bound(pv.begin(), pv.end(), x) - pv.begin());
    };
    const int64_t ns = (int64_t)inst_v.size();
    iebase.push_back(NE);

    // wanted instance edges and the instance-edge pairs of every query
    std::vector<uint8_t> want((size_t)std::max<int64_t>(NE, 1), 0);
    std::vector<std::vector<int64_t>> qpairs(reqs.size());
    for (int32_t k = 0; k < P; ++k)
        if (pall[k]) {
            const int32_t ga = g->goff[pgraph[k]], gz = g->goff[pgraph[k] + 1];
            std::fill(want.begin() + pbase[k], want.begin() + pbase[k] + (rp[gz] - rp[ga]), 1);
        }
    if (cj)
        for (const int32_t x : cj->src) {
            const int64_t k = inst_of(0, x);
            std::fill(want.begin() + iebase[k], want.begin() + iebase[k + 1], 1);
        }
    for (size_t i = 0; i < reqs.size(); ++i) {
        const Request &r = reqs[i];
        if (r.q <= 0) continue;
        const int32_t ga = g->goff[r.graph];
        qpairs[i].resize(2 * r.q);
        for (int64_t j = 0; j < r.q; ++j) {
            const int32_t u = hq[i][2 * j], v = hq[i][2 * j + 1];
            const int32_t euv = find_pos(ga + u, ga + v), evu = find_pos(ga + v, ga + u);
            const int64_t a = iebase[inst_of(r.pid, u)] + (euv - rp[ga + u]);
            const int64_t b = iebase[inst_of(r.pid, v)] + (evu - rp[ga + v]);
            want[a] = want[b] = 1;
            qpairs[i][2 * j] = a;
            qpairs[i][2 * j + 1] = b;
        }
    }

    const bool timing = st && opt.time_kernels;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // walk-pair launch bounds of every batch (timing), read once the call has finished
    std::vector<hipEvent_t> wev;
    struct EvGuard {
        hipEvent_t *e[2];
        std::vector<hipEvent_t> *v;
        ~EvGuard() {
            for (auto *x : e)
                if (*x) (void)hipEventDestroy(*x);
            for (auto x : *v)
                if (x) (void)hipEventDestroy(x);
        }
    } evguard{{&ev0, &ev1}, &wev};
    if (timing) {
        SABA_HIP_TRY(hipEventCreate(&ev0));
        SABA_HIP_TRY(hipEventCreate(&ev1));
        SABA_HIP_TRY(hipEventRecord(ev0, s));
    }

    Workspace &ws = g->est;
    EdgeArrays ea;
    SABA_TRY(ensure_edge_arrays(ws, NE, ns, P, &ea));
    SABA_HIP_TRY(hipMemcpyAsync(const_cast<PSet *>(ea.psets), psets.data(), sizeof(PSet) * P,
                                hipMemcpyHostToDevice, s));
    SABA_HIP_TRY(hipMemcpyAsync(const_cast<uint8_t *>(ea.want), want.data(),
                                std::max<int64_t>(NE, 1), hipMemcpyHostToDevice, s));
    SABA_HIP_TRY(hipMemsetAsync(ea.fl, 0, sizeof(Flags), s));

    // batches: consecutive instances whose slots fit the memory budget
    size_t freeb = 0, totalb = 0;
    SABA_HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    const int64_t budget = opt.mem_budget > 0
                               ? opt.mem_budget
                               : std::min<int64_t>(32ll << 30, (int64_t)(0.4 * (double)freeb));
    // two pool sets (levels of the next batch beside the walk pairs of this one) share it
    const int lanes = (!cj && g->cfg.est_batch_streams == 2) ? 2 : 1;
    const int64_t lane_budget = budget / lanes;
    std::vector<SlotSize> ssz(P);
    for (int32_t k = 0; k < P; ++k) ssz[k] = slot_size(g, pgraph[k]);
    struct Batch {
        int64_t i0, i1, h, bm, sb, hubs, ne;
    };
    std::vector<Batch> batches;
    int64_t maxh = 0, maxbm = 0, maxsb = 0, maxhubs = 0, maxne = 0, maxnb = 0;
    for (int64_t i = 0; i < ns;) {
        Batch bt{i, i, 0, 0, 0, 0, 0};
        int64_t bytes = 0;
        while (bt.i1 < ns) {
            const SlotSize &z = ssz[inst_p[bt.i1]];
            if (bt.i1 > bt.i0 && (bytes + z.bytes > lane_budget || bt.i1 - bt.i0 >= 65535 ||
                                  (opt.batch_sources > 0 && bt.i1 - bt.i0 >= opt.batch_sources)))
                break;
            bytes += z.bytes;
            bt.h += z.h;
            bt.bm += z.bm;
            bt.sb += z.sb;
            bt.hubs += z.hubs;
            ++bt.i1;
        }
        bt.ne = iebase[bt.i1] - iebase[bt.i0];
        maxh = std::max(maxh, bt.h);
        maxbm = std::max(maxbm, bt.bm);
        maxsb = std::max(maxsb, bt.sb);
        maxhubs = std::max(maxhubs, bt.hubs);
        maxne = std::max(maxne, bt.ne);
        maxnb = std::max(maxnb, bt.i1 - bt.i0);
        batches.push_back(bt);
        i = bt.i1;
    }
    SABA_TRY(ensure_pools(ws, maxh, maxbm, maxsb, maxhubs, maxnb, maxne, s));
    const bool overlap = lanes == 2 && batches.size() >= 2;
    Workspace *wsl[2] = {&ws, &g->est2};
    EdgeArrays eal[2] = {ea, ea};
    hipStream_t slev = s;  // stream of the levels phases
    if (overlap) {
        SABA_TRY(ensure_est_pipeline(g));
        SABA_TRY(ensure_pools(g->est2, maxh, maxbm, maxsb, maxhubs, maxnb, maxne, s));
        SABA_TRY(g->est2.b[B_FLAGS].ensure(sizeof(Flags)));
        eal[1].fl = g->est2.b[B_FLAGS].as<Flags>();
        SABA_HIP_TRY(hipMemsetAsync(eal[1].fl, 0, sizeof(Flags), s));
        slev = g->est_aux;
        // the levels stream starts after the set-up above
        SABA_HIP_TRY(hipEventRecord(g->est_ev[0], s));
        SABA_HIP_TRY(hipStreamWaitEvent(slev, g->est_ev[0], 0));
    }

    // counts export: per-instance support offsets and histogram offsets in the caller's layout
    CountExport cx;
    struct BufGuard {
        DevBuf b;
        ~BufGuard() { b.release(); }
    } cbuf;
    std::vector<int64_t> hsz;
    if (cj) {
        const size_t K = cj->src.size();
        std::vector<int64_t> per(4 * (size_t)ns, -1);  // soff, hoff, expect, (support sizes)
        if (cj->supp)
            for (size_t k = 0; k < K; ++k) {
                const int64_t i = inst_of(0, cj->src[k]);
                per[i] = cj->layout[k].supp_off;
                per[ns + i] = cj->layout[k].hist_off;
                per[2 * ns + i] = cj->layout[k].support;
            }
        SABA_TRY(cbuf.b.ensure(sizeof(int64_t) * per.size()));
        int64_t *dp = cbuf.b.as<int64_t>();
        SABA_HIP_TRY(hipMemcpyAsync(dp, per.data(), sizeof(int64_t) * per.size(),
                                    hipMemcpyHostToDevice, s));
        cx.soff = dp;
        cx.ca.hoff = dp + ns;
        cx.expect = dp + 2 * ns;
        cx.ca.expect = cx.expect;
        cx.supp_sz = dp + 3 * ns;
        cx.supp = cj->supp;
        cx.h = cj->h;
        cx.ca.hist = reinterpret_cast<unsigned long long *>(cj->hist);
        cx.ca.FA = ws.b[B_FA].as<int32_t>();
        cx.ca.FB = ws.b[B_FB].as<int32_t>();
        if (cj->hist) {
            int64_t tot = 0;
            for (size_t k = 0; k < K; ++k)
                tot = std::max(tot, cj->layout[k].hist_off +
                                        2 * (int64_t)cj->layout[k].degree * cj->layout[k].support);
            if (tot > 0) SABA_HIP_TRY(hipMemsetAsync(cj->hist, 0, sizeof(int64_t) * tot, s));
        }
    }

    // Batch k uses pool set k mod 2 when the phases overlap: its levels run on slev once the walk
    // pairs of batch k - 2 (the same pool set) are done, and its walk pairs on s once its levels
    // are; the levels of batch k + 1 then run beside them.  Batches write disjoint instance
    // edges and instances, so the results are those of the batches in order.
    const auto drain = [&]() {
        (void)hipStreamSynchronize(s);
        if (slev != s) (void)hipStreamSynchronize(slev);
    };
    std::vector<Slot> hslots;
    std::vector<int64_t> heb;
    for (size_t bi = 0; bi < batches.size(); ++bi) {
        const Batch &bt = batches[bi];
        const int lane = overlap ? (int)(bi & 1) : 0;
        const int32_t nb = (int32_t)(bt.i1 - bt.i0);
        const int64_t ie0 = iebase[bt.i0];
        hslots.resize(nb);
        heb.resize(nb + 1);
        int64_t ho = 0, bo = 0, so = 0, maxgn = 1;
        for (int32_t b = 0; b < nb; ++b) {
            const int64_t i = bt.i0 + b;
            const int32_t k = inst_p[i], gi = pgraph[k];
            Slot &sl = hslots[b];
            sl.hoff = ho;
            sl.bmoff = bo;
            sl.sboff = so;
            sl.ie = iebase[i];
            sl.inst = i;
            sl.v = inst_v[i];
            sl.p = k;
            sl.goff = g->goff[gi];
            sl.gn = g->goff[gi + 1] - g->goff[gi];
            sl.gpos = rp[sl.goff];
            sl.pad = 0;
            ho += ssz[k].h;
            bo += ssz[k].bm;
            so += ssz[k].sb;
            maxgn = std::max<int64_t>(maxgn, sl.gn);
            heb[b] = iebase[i] - ie0;
        }
        heb[nb] = bt.ne;
        int rc = SABA_OK;
        if (overlap && bi >= 2)
            rc = SABA_HIP_STATUS(hipStreamWaitEvent(slev, g->est_ev[2 + lane], 0));
        BatchPlan plan;
        if (rc == SABA_OK)
            rc = batch_levels(g, *wsl[lane], eal[lane], hslots, heb, ie0, bt.ne, maxgn, bt.hubs,
                              slev, &plan);
        if (rc == SABA_OK && overlap) {
            rc = SABA_HIP_STATUS(hipEventRecord(g->est_ev[lane], slev));
            if (rc == SABA_OK) rc = SABA_HIP_STATUS(hipStreamWaitEvent(s, g->est_ev[lane], 0));
        }
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (rc == SABA_OK && timing && plan.T > 0) {
            wev.push_back(nullptr);
            rc = SABA_HIP_STATUS(hipEventCreate(&wev.back()));
            t0 = wev.back();
            wev.push_back(nullptr);
            if (rc == SABA_OK) rc = SABA_HIP_STATUS(hipEventCreate(&wev.back()));
            t1 = wev.back();
        }
        if (rc == SABA_OK)
            rc = batch_walks(g, *wsl[lane], eal[lane], plan, t0, t1, s, cj ? &cx : nullptr);
        if (rc == SABA_OK && overlap)
            rc = SABA_HIP_STATUS(hipEventRecord(g->est_ev[2 + lane], s));
        if (rc != SABA_OK) {
            drain();  // nothing of this call stays in flight on the handle's pools
            return rc;
        }
    }
    if (cj) {
        // layout of the caller's arrays in list order, then the per-edge outputs
        const size_t K = cj->src.size();
        std::vector<int64_t> sz((size_t)ns);
        std::vector<int32_t> tt((size_t)ns);
        SABA_HIP_TRY(hipMemcpyAsync(sz.data(), cx.supp_sz, sizeof(int64_t) * ns,
                                    hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipMemcpyAsync(tt.data(), ea.ttau_inst, sizeof(int32_t) * ns,
                                    hipMemcpyDeviceToHost, s));
        int32_t err = 0;
        SABA_HIP_TRY(hipMemcpyAsync(&err, &ea.fl->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipStreamSynchronize(s));
        if (err & kErrLayout) {
            set_error("a support size differs from the layout: pass the layout the sizing call "
                      "returned for the same parameters");
            return SABA_E_INVALID;
        }
        // a source list that is an ascending run of vertices exports its per-edge values with
        // one copy per array: its instances, and their edges, are consecutive in that order
        bool run = true;
        for (size_t k = 1; k < K && run; ++k) run = cj->src[k] == cj->src[0] + (int32_t)k;
        int64_t so = 0, eo = 0, ho = 0;
        for (size_t k = 0; k < K; ++k) {
            const int64_t i = inst_of(0, cj->src[k]);
            saba_count_source &c = cj->layout[k];
            const int32_t d = (int32_t)(iebase[i + 1] - iebase[i]);
            if (!cj->supp) {
                c.degree = d;
                c.support = sz[i];
                c.supp_off = so;
                c.edge_off = eo;
                c.hist_off = ho;
            }
            c.ttau = tt[i];
            so += sz[i];
            eo += d;
            ho += 2 * (int64_t)d * sz[i];
            const Exports &x = cj->edges;
            int64_t e0 = iebase[i], o = c.edge_off, cnt = d;
            if (run) {  // everything in one copy, at the first source
                if (k > 0) continue;
                cnt = iebase[inst_of(0, cj->src[K - 1]) + 1] - e0;
            }
            auto cp = [&](void *dst, const void *src, size_t bytes) -> int {
                if (dst && bytes)
                    SABA_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
                return SABA_OK;
            };
            SABA_TRY(cp(x.tau ? x.tau + o : nullptr, ea.tau + e0, sizeof(int32_t) * cnt));
            SABA_TRY(cp(x.nreq ? x.nreq + o : nullptr, ea.nreq + e0, sizeof(int64_t) * cnt));
            SABA_TRY(cp(x.D ? x.D + o : nullptr, ea.D + e0, sizeof(double) * cnt));
            SABA_TRY(cp(x.MC ? x.MC + o : nullptr, ea.MC + e0, sizeof(double) * cnt));
            SABA_TRY(cp(x.vis0 ? x.vis0 + o : nullptr, ea.vis0 + e0, sizeof(int64_t) * cnt));
            SABA_TRY(cp(x.vis1 ? x.vis1 + o : nullptr, ea.vis1 + e0, sizeof(int64_t) * cnt));
            SABA_TRY(cp(x.g ? x.g + o : nullptr, ea.g + e0, sizeof(double) * cnt));
        }
    }

    // results of every request
    int64_t npairs = 0;
    for (auto &qp : qpairs) npairs += (int64_t)qp.size();
    SABA_TRY(ws.b[B_PAIRS].ensure(sizeof(int64_t) * std::max<int64_t>(npairs, 1)));
    int64_t *d_pairs = ws.b[B_PAIRS].as<int64_t>();
    int64_t off = 0;
    for (size_t i = 0; i < reqs.size(); ++i) {
        const Request &r = reqs[i];
        if (!r.sc) continue;
        if (r.q < 0) {
            const int32_t ga = g->goff[r.graph];
            const int64_t cb = g->cbase[r.graph], m = g->cbase[r.graph + 1] - cb;
            if (m > 0) {
                finalize_all_kernel<<<grid_for(m, 256, 1 << 16), 256, 0, s>>>(
                    g->canon, g->rev, cb, m, pbase[r.pid], rp[ga], ea.g, r.sc);
                if (r.spec && r.spec->pairs > 0)
                    tail_all_kernel<<<grid_for(m, 256, 1 << 16), 256, 0, s>>>(
                        g->canon, g->row_of, g->col_idx, cb, m, pbase[r.pid], rp[ga], ga, ea.tau,
                        r.spec->d_theta(), r.spec->d_y(), g->goff[r.graph + 1] - ga,
                        r.spec->pairs, r.sc);
            }
        } else if (r.q > 0) {
            SABA_HIP_TRY(hipMemcpyAsync(d_pairs + off, qpairs[i].data(),
                                        sizeof(int64_t) * qpairs[i].size(), hipMemcpyHostToDevice,
                                        s));
            finalize_pairs_kernel<<<grid_for(r.q, 256, 1 << 16), 256, 0, s>>>(d_pairs + off, r.q,
                                                                             ea.g, r.sc);
            if (r.spec && r.spec->pairs > 0)
                tail_pairs_kernel<<<grid_for(r.q, 256, 1 << 16), 256, 0, s>>>(
                    r.edges, d_pairs + off, r.q, ea.tau, r.spec->d_theta(), r.spec->d_y(),
                    g->goff[r.graph + 1] - g->goff[r.graph], r.spec->pairs, r.sc);
            off += (int64_t)qpairs[i].size();
        }
        SABA_HIP_TRY(hipGetLastError());
    }
    if (ex) {  // single graph, one all-edges request: instance edges are CSR positions
        const int64_t nnz = g->nnz;
        auto cp = [&](void *dst, const void *src, size_t bytes) -> int {
            if (dst) SABA_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
            return SABA_OK;
        };
        SABA_TRY(cp(ex->tau, ea.tau, sizeof(int32_t) * nnz));
        SABA_TRY(cp(ex->nreq, ea.nreq, sizeof(int64_t) * nnz));
        SABA_TRY(cp(ex->D, ea.D, sizeof(double) * nnz));
        SABA_TRY(cp(ex->MC, ea.MC, sizeof(double) * nnz));
        SABA_TRY(cp(ex->vis0, ea.vis0, sizeof(int64_t) * nnz));
        SABA_TRY(cp(ex->vis1, ea.vis1, sizeof(int64_t) * nnz));
        SABA_TRY(cp(ex->g, ea.g, sizeof(double) * nnz));
        if (ex->ttau && nnz > 0) {
            export_ttau_kernel<<<grid_for(nnz, 256, 1 << 16), 256, 0, s>>>(g->row_of, nnz,
                                                                           ea.ttau_inst, ex->ttau);
            SABA_HIP_TRY(hipGetLastError());
        }
    }
    if (timing) SABA_HIP_TRY(hipEventRecord(ev1, s));
    Flags hf, hf1{};
    SABA_HIP_TRY(hipMemcpyAsync(&hf, ea.fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
    if (overlap)
        SABA_HIP_TRY(hipMemcpyAsync(&hf1, eal[1].fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipStreamSynchronize(s));
    if (overlap) merge_flags(hf, hf1);
    if (st) {
        *st = saba_stats{};
        st->walks = (int64_t)hf.walks;
        st->walk_steps = (int64_t)hf.walk_steps;
        st->push_edge_visits = (int64_t)hf.push_visits;
        st->sources = ns;
        st->batches = (int64_t)batches.size();
        st->max_tau = hf.max_tau;
        st->max_ttau = hf.max_ttau;
        st->warnings = hf.warnings;
        if (timing) {
            float tot = 0.f, walk_ms = 0.f;
            SABA_HIP_TRY(hipEventElapsedTime(&tot, ev0, ev1));
            for (size_t i = 0; i + 1 < wev.size(); i += 2) {
                float ms = 0.f;
                SABA_HIP_TRY(hipEventElapsedTime(&ms, wev[i], wev[i + 1]));
                walk_ms += ms;
            }
            st->kernel_ms = walk_ms;
            st->total_ms = tot;
        }
    }
    return SABA_OK;
}

static Opts opts_of(const saba_aesc_params *p) {
    Opts o;
    o.mem_budget = p->mem_budget;
    o.batch_sources = p->batch_sources;
    o.time_kernels = p->time_kernels;
    return o;
}

static int single_graph(const Graph *g) {
    if (g->ngraphs != 1) {
        set_error("this call needs a handle with one graph; use saba_aesc_batch");
        return SABA_E_INVALID;
    }
    return SABA_OK;
}

}  // namespace saba

using namespace saba;

extern "C" int saba_aesc(saba_graph *gh, const saba_aesc_params *p, double *d_sc, saba_stats *st,
                         void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p || !d_sc) {
        set_error("params or output is NULL");
        return SABA_E_INVALID;
    }
    SABA_TRY(single_graph(G(gh)));
    std::vector<Request> reqs(1);
    reqs[0].p = *p;
    reqs[0].sc = d_sc;
    return aesc_run(G(gh), reqs, opts_of(p), nullptr, st, static_cast<hipStream_t>(stream));
}

extern "C" int saba_aesc_query(saba_graph *gh, const saba_aesc_params *p, const int32_t *d_edges,
                               int64_t q, double *d_sc, saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p || q < 0 || (q > 0 && (!d_edges || !d_sc))) {
        set_error("invalid query arguments");
        return SABA_E_INVALID;
    }
    SABA_TRY(single_graph(G(gh)));
    std::vector<Request> reqs(1);
    reqs[0].p = *p;
    reqs[0].edges = d_edges;
    reqs[0].q = q;
    reqs[0].sc = d_sc;
    return aesc_run(G(gh), reqs, opts_of(p), nullptr, st, static_cast<hipStream_t>(stream));
}

extern "C" int saba_aesc_edge_stats(saba_graph *gh, const saba_aesc_params *p, double *d_sc,
                                    int32_t *d_tau, int32_t *d_ttau, int64_t *d_nreq, double *d_D,
                                    double *d_MC, int64_t *d_vis0, int64_t *d_vis1, double *d_g,
                                    saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p) {
        set_error("params is NULL");
        return SABA_E_INVALID;
    }
    SABA_TRY(single_graph(G(gh)));
    std::vector<Request> reqs(1);
    reqs[0].p = *p;
    reqs[0].sc = d_sc;  // may be NULL: then only the per-edge internals are written
    Exports ex;
    ex.tau = d_tau;
    ex.ttau = d_ttau;
    ex.nreq = d_nreq;
    ex.D = d_D;
    ex.MC = d_MC;
    ex.vis0 = d_vis0;
    ex.vis1 = d_vis1;
    ex.g = d_g;
    return aesc_run(G(gh), reqs, opts_of(p), &ex, st, static_cast<hipStream_t>(stream));
}

extern "C" int saba_aesc_counts(saba_graph *gh, const saba_aesc_params *p,
                                saba_count_source *layout, int32_t nsrc, int32_t *d_supp,
                                double *d_h, int64_t *d_hist, int32_t *d_tau, int64_t *d_nreq,
                                double *d_D, double *d_MC, int64_t *d_vis0, int64_t *d_vis1,
                                double *d_g, saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p || nsrc < 1 || !layout) {
        set_error("params or layout is NULL, or the source list is empty");
        return SABA_E_INVALID;
    }
    const bool fill = d_supp || d_h || d_hist;
    if (fill && !(d_supp && d_h && d_hist)) {
        set_error("d_supp, d_h and d_hist are given together or not at all");
        return SABA_E_INVALID;
    }
    SABA_TRY(single_graph(G(gh)));
    Graph *g = G(gh);
    CountJob cj;
    cj.src.resize((size_t)nsrc);
    std::vector<int32_t> sorted((size_t)nsrc);
    for (int32_t k = 0; k < nsrc; ++k) {
        const int32_t v = layout[k].source;
        if (v < 0 || v >= g->n || g->h_row_ptr[v + 1] == g->h_row_ptr[v]) {
            set_error("a source is out of range or an isolated vertex");
            return SABA_E_INVALID;
        }
        cj.src[k] = sorted[k] = v;
    }
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
        set_error("a source is listed twice");
        return SABA_E_INVALID;
    }
    if (fill) {  // the layout must be a dense packing, as the sizing call returns it
        int64_t so = 0, eo = 0, ho = 0;
        for (int32_t k = 0; k < nsrc; ++k) {
            const saba_count_source &c = layout[k];
            const int32_t v = c.source;
            if (c.degree != g->h_row_ptr[v + 1] - g->h_row_ptr[v] || c.support < 1 ||
                c.supp_off != so || c.edge_off != eo || c.hist_off != ho) {
                set_error("the layout is not the one the sizing call returned");
                return SABA_E_INVALID;
            }
            so += c.support;
            eo += c.degree;
            ho += 2 * (int64_t)c.degree * c.support;
        }
    }
    cj.layout = layout;
    cj.supp = d_supp;
    cj.h = d_h;
    cj.hist = d_hist;
    cj.edges.tau = d_tau;
    cj.edges.nreq = d_nreq;
    cj.edges.D = d_D;
    cj.edges.MC = d_MC;
    cj.edges.vis0 = d_vis0;
    cj.edges.vis1 = d_vis1;
    cj.edges.g = d_g;
    std::vector<Request> reqs(1);
    reqs[0].p = *p;
    reqs[0].q = 0;
    return aesc_run(g, reqs, opts_of(p), nullptr, st, static_cast<hipStream_t>(stream), &cj);
}

extern "C" int saba_aesc_sources(saba_graph *gh, const saba_aesc_params *p, int32_t src_begin,
                                 int32_t src_end, double *d_g, saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p || !d_g) {
        set_error("params or output is NULL");
        return SABA_E_INVALID;
    }
    SABA_TRY(single_graph(G(gh)));
    Graph *g = G(gh);
    if (src_begin < 0 || src_end > g->n || src_begin >= src_end) {
        set_error("the source range must satisfy 0 <= begin < end <= n");
        return SABA_E_INVALID;
    }
    if (p->omega != 0) {
        set_error("the source-range form keeps no eigenpair tail: use saba_aesc for omega > 0");
        return SABA_E_INVALID;
    }
    CountJob cj;
    std::vector<saba_count_source> layout((size_t)(src_end - src_begin));
    cj.src.resize(layout.size());
    for (int32_t v = src_begin; v < src_end; ++v) {
        cj.src[v - src_begin] = v;
        layout[v - src_begin].source = v;
    }
    cj.layout = layout.data();
    cj.edges.g = d_g + g->h_row_ptr[src_begin];
    std::vector<Request> reqs(1);
    reqs[0].p = *p;
    reqs[0].q = 0;
    return aesc_run(g, reqs, opts_of(p), nullptr, st, static_cast<hipStream_t>(stream), &cj);
}

extern "C" int saba_aesc_combine(saba_graph *gh, const double *d_g, double *d_sc, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!d_g || !d_sc) {
        set_error("input or output is NULL");
        return SABA_E_INVALID;
    }
    SABA_TRY(single_graph(G(gh)));
    Graph *g = G(gh);
    const int64_t m = g->nnz / 2;
    if (m > 0) {
        finalize_all_kernel<<<grid_for(m, 256, 1 << 16), 256, 0, static_cast<hipStream_t>(stream)>>>(
            g->canon, g->rev, 0, m, 0, 0, d_g, d_sc);
        SABA_HIP_TRY(hipGetLastError());
    }
    return SABA_OK;
}

extern "C" int saba_aesc_batch(saba_graph *gh, const saba_aesc_request *reqs, int32_t nreq,
                               const saba_batch_options *opt, saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (nreq < 0 || (nreq > 0 && !reqs)) {
        set_error("invalid request list");
        return SABA_E_INVALID;
    }
    std::vector<Request> rs((size_t)nreq);
    for (int32_t i = 0; i < nreq; ++i) {
        if (reqs[i].q != 0 && !reqs[i].d_sc) {
            set_error("a request has no output array");
            return SABA_E_INVALID;
        }
        rs[i].graph = reqs[i].graph;
        rs[i].p = reqs[i].params;
        rs[i].edges = reqs[i].d_edges;
        rs[i].q = reqs[i].q;
        rs[i].sc = reqs[i].d_sc;
    }
    Opts o;
    if (opt) {
        o.mem_budget = opt->mem_budget;
        o.batch_sources = opt->batch_sources;
        o.time_kernels = opt->time_kernels;
    }
    if (nreq == 0) {
        if (st) *st = saba_stats{};
        return SABA_OK;
    }
    return aesc_run(G(gh), rs, o, nullptr, st, static_cast<hipStream_t>(stream));
}

extern "C" int saba_autotune_aesc(saba_graph *gh, const saba_aesc_request *sample, int32_t nreq,
                                  const saba_batch_options *opt, saba_exec_config *best,
                                  void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (nreq < 1 || !sample) {
        set_error("the autotuner needs a sample of at least one request");
        return SABA_E_INVALID;
    }
    Graph *g = G(gh);
    saba_batch_options o{};
    if (opt) o = *opt;
    o.time_kernels = 1;
    const saba_exec_config saved = g->cfg;
    saba_exec_config pick = saved;
    double best_ms = 1e300;
    const int walk_blocks[] = {512, 1024, 2048, 4096};
    const int push_blocks[] = {1024, 2048, 4096, 8192};
    for (int streams = 1; streams <= 2; ++streams)
        for (int wq = 0; wq <= 2; ++wq)
            for (int wb : walk_blocks)
                for (int pb : push_blocks) {
                    if (wq == 2 && wb != walk_blocks[0]) continue;  // its grid follows the LDS
                    g->cfg = saved;
                    g->cfg.est_walk_blocks = wb;
                    g->cfg.est_push_blocks = pb;
                    g->cfg.est_walk_queue = wq;
                    g->cfg.est_batch_streams = streams;
                    double ms = 0.0;
                    for (int rep = 0; rep < 3; ++rep) {  // one warm-up, two timed
                        saba_stats st{};
                        const int rc = saba_aesc_batch(gh, sample, nreq, &o, &st, stream);
                        if (rc != SABA_OK) {
                            g->cfg = saved;
                            return rc;
                        }
                        if (rep > 0) ms += st.total_ms;
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

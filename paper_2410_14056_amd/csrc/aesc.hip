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
// Work layout: sources are processed in batches that fit a memory budget.  Each source of a
// batch owns dense FP64 h vectors (two levels), frontier lists and support bitmaps (two
// levels); they are cleared sparsely through the frontier lists, so they are zeroed only
// once.  The deterministic levels run level-synchronously over the whole batch.  A wavefront
// walks the concatenated rows of 64 frontier vertices in chunks of 64 entries, so hub rows are
// split across lanes; the pull folds only the terms whose vertex is in the support bitmap (a
// zero term leaves a sum of non-negative numbers unchanged), in row order, so every h value is
// bit-identical to the sequential left fold over the whole row.  The walk pairs of
// all directed edges of the batch are cut into chunks of 64 walks; one wavefront walks one
// chunk and reduces it in a fixed butterfly order, and each edge sums its chunks in chunk
// order, so results do not depend on the launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "saba_internal.hpp"

namespace saba {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kChunk = 64;  // walks per wavefront chunk

enum : int32_t { kErrOverflow = 1, kErrNotEdge = 2 };

// scratch slots in Graph::est
enum {
    B_TAU, B_D, B_NREQ, B_MC, B_VIS0, B_VIS1, B_G, B_TTAU_SRC, B_MAXTAU_SRC, B_WANT, B_SRCMARK,
    B_SRCPOS, B_LIST, B_HA, B_HB, B_FA, B_FB, B_BMA, B_BMB, B_SLOTBM, B_BSRC, B_BSTATE, B_EBASE, B_CHUNKS,
    B_COFF, B_PART, B_SCAN, B_FLAGS, B_QE, B_DEG64, B_COUNT
};

struct BatchState {  // one per source of a batch; [2] entries are indexed by level parity
    int32_t active;
    int32_t finalbuf;
    int32_t fsz[2];                 // frontier (support) sizes
    unsigned long long vol[2];      // support volume sum of d(x)
    unsigned long long hmaxbits[2]; // max of h over the support, as IEEE bits (h > 0)
    double hmax;                    // max of h_ttau once the source has stopped
};

struct Flags {
    int32_t err;
    int32_t any_active;
    int32_t max_tau;
    int32_t max_ttau;
    int32_t warnings;
    int32_t pad;
    unsigned long long walk_steps;
    unsigned long long push_visits;
    unsigned long long walks;
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

// NWalks (Hoeffding): max(1, ceil(c * q * q)), q = L * hmax / d_s; -1 on overflow.
__device__ __forceinline__ long long nwalks(int32_t L, double hmax, int32_t ds, double c) {
    const double q = ((double)L * hmax) / (double)ds;
    const double x = c * q * q;
    if (!(x < 4.0e18)) return -1;
    long long r = (long long)ceil(x);
    return r < 1 ? 1 : r;
}

// ------------------------------------------------------------ kernels
// tau for every directed entry of the listed sources' rows (all vertices when list == NULL),
// and the largest tau of each source.
__global__ __launch_bounds__(kBlock) void tau_kernel(const int2 *__restrict__ vrec,
                                                     const int32_t *__restrict__ col, int32_t n,
                                                     double lambda, double eps, int32_t cap,
                                                     int32_t *__restrict__ tau,
                                                     int32_t *__restrict__ maxtau,
                                                     Flags *__restrict__ fl) {
    const int lane = __lane_id();
    const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t s = wid; s < n; s += nw) {
        const int2 r = vrec[s];
        int mx = 0, capped = 0;
        for (int32_t i = lane; i < r.y; i += 64) {
            const int32_t t = col[r.x + i];
            const int32_t tv = tau_of(r.y, vrec[t].y, lambda, eps, cap);
            tau[r.x + i] = tv;
            mx = max(mx, tv);
            capped |= (tv >= cap) ? 1 : 0;
        }
        mx = wave_max_i(mx);
        capped = wave_max_i(capped);
        if (lane == 0) {
            maxtau[s] = mx;
            atomicMax(&fl->max_tau, mx);
            if (capped) atomicOr(&fl->warnings, 1);
        }
    }
}

__global__ void iota_kernel(int32_t *__restrict__ a, int32_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (int32_t)i;
}

__device__ __forceinline__ int32_t find_entry(const int2 *__restrict__ vrec,
                                              const int32_t *__restrict__ col, int32_t u,
                                              int32_t v) {
    const int2 r = vrec[u];
    int32_t lo = r.x, hi = r.x + r.y;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < r.x + r.y && col[lo] == v) ? lo : -1;
}

// Query edges: locate both directed entries, mark them wanted and their endpoints as sources.
__global__ void query_mark_kernel(const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
                                  int32_t n, const int32_t *__restrict__ edges, int64_t q,
                                  uint8_t *__restrict__ want, long long *__restrict__ srcmark,
                                  int32_t *__restrict__ qe, Flags *__restrict__ fl) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = edges[2 * j], v = edges[2 * j + 1];
        int32_t euv = -1, evu = -1;
        if (u >= 0 && u < n && v >= 0 && v < n) {
            euv = find_entry(vrec, col, u, v);
            evu = find_entry(vrec, col, v, u);
        }
        if (euv < 0 || evu < 0) {
            atomicOr(&fl->err, kErrNotEdge);
            qe[2 * j] = qe[2 * j + 1] = 0;
            continue;
        }
        want[euv] = 1;
        want[evu] = 1;
        srcmark[u] = 1;
        srcmark[v] = 1;
        qe[2 * j] = euv;
        qe[2 * j + 1] = evu;
    }
}

__global__ void compact_kernel(const long long *__restrict__ mark, const int64_t *__restrict__ pos,
                               int32_t n, int32_t *__restrict__ list) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x)
        if (mark[s]) list[pos[s]] = (int32_t)s;
}

// Level 0 of every source of the batch: h_0 = e_s, support {s}; per-edge accumulators reset.
__global__ __launch_bounds__(kBlock) void batch_init_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ list, int64_t i0, int32_t nb,
    int32_t n, int64_t nw, int32_t *__restrict__ bsrc, BatchState *__restrict__ bs,
    double *__restrict__ hA, int32_t *__restrict__ FA, uint32_t *__restrict__ bmA,
    double *__restrict__ D, long long *__restrict__ nreq, double *__restrict__ MC,
    unsigned long long *__restrict__ vis0, unsigned long long *__restrict__ vis1,
    long long *__restrict__ deg64) {
    const int lane = __lane_id();
    const int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (b >= nb) return;
    const int32_t s = list[i0 + b];
    const int2 r = vrec[s];
    if (lane == 0) {
        bsrc[b] = s;
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
        bs[b] = st;
        hA[b * n + s] = 1.0;
        FA[b * n] = s;
        bmA[b * nw + (s >> 5)] = 1u << (s & 31);
        deg64[b] = r.y;
    }
    for (int32_t i = lane; i < r.y; i += 64) {
        D[r.x + i] = 0.0;
        nreq[r.x + i] = 0;
        MC[r.x + i] = 0.0;
        vis0[r.x + i] = 0;
        vis1[r.x + i] = 0;
    }
}

// Alg. 1 loop test at level l for each active source: with the support volume and maximum of
// h_l (accumulated when h_l was built), add the deterministic terms of level l and compare the
// volume with the walk pairs that would still be needed.
__global__ __launch_bounds__(kBlock) void level_decide_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
    const int32_t *__restrict__ bsrc, BatchState *__restrict__ bs, int32_t nb, int32_t n,
    int32_t level, const double *__restrict__ hcur_all, const int32_t *__restrict__ tau,
    const int32_t *__restrict__ maxtau, double *__restrict__ D, int32_t *__restrict__ ttau_src,
    double c, int32_t push_all, int32_t tilde_tau_max, Flags *__restrict__ fl) {
    const int lane = __lane_id();
    const int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (b >= nb || !bs[b].active) return;
    const int cur = level & 1, nxt = cur ^ 1;
    const int32_t s = bsrc[b];
    const double *h = hcur_all + b * n;
    const long long vol = (long long)bs[b].vol[cur];
    const double hmax = __longlong_as_double((long long)bs[b].hmaxbits[cur]);
    const int2 r = vrec[s];
    const double hs = h[s];
    long long need = 0;
    int ovf = 0;
    for (int32_t i = lane; i < r.y; i += 64) {
        const int32_t e = r.x + i;
        const int32_t te = tau[e];
        if (level <= te) D[e] += hs - h[col[e]];
        if (te > level) {
            const long long w = nwalks(te - level, hmax, r.y, c);
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
        bool stop = push_all ? (level >= maxtau[s]) : !(vol < need);
        if (tilde_tau_max >= 0 && level >= tilde_tau_max) stop = true;
        if (ovf) stop = true;
        if (stop) {
            bs[b].active = 0;
            bs[b].finalbuf = cur;
            bs[b].hmax = hmax;
            ttau_src[s] = level;
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

// Rows of the 64 frontier entries [base, base + 64) of one source, as seen by each lane:
// its own row and the exclusive prefix of the row lengths over the wavefront.  Hub rows
// count as empty when `skip_hubs` is set (they are handled separately).
struct WaveRows {
    int32_t x, start, len, pre, total;
};

__device__ __forceinline__ WaveRows wave_rows(const int2 *__restrict__ vrec,
                                              const int32_t *__restrict__ F, int64_t base,
                                              int32_t fsz, bool skip_hubs) {
    const int lane = __lane_id();
    WaveRows w;
    w.x = -1;
    w.start = 0;
    w.len = 0;
    if (base + lane < fsz) {
        w.x = F[base + lane];
        const int2 r = vrec[w.x];
        w.start = r.x;
        w.len = (skip_hubs && r.y > kHubRow) ? 0 : r.y;
    }
    int32_t inc = w.len;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    w.total = __shfl(inc, 63);
    w.pre = inc - w.len;
    return w;
}

// Owner lane of flattened entry j (0 <= j < total): the largest lane whose prefix is <= j,
// which is always a lane whose row contains entry j.
__device__ __forceinline__ int wave_owner(int32_t pre, int32_t j) {
    int lo = 0, hi = 64;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (__shfl(pre, mid) <= j)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Push the current support one hop: set the bit of every neighbour in the next level's
// support bitmap and, for neighbours with hub rows, the bit of the reverse CSR position in
// the hub-slot bitmap.  Fire-and-forget atomics; the next frontier list is built from the
// bitmap afterwards, in ascending vertex order.
__global__ __launch_bounds__(kBlock) void expand_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
    const int32_t *__restrict__ slotv, BatchState *__restrict__ bs, int32_t n, int64_t nw,
    int64_t nsw, int32_t level, const int32_t *__restrict__ Fcur_all,
    uint32_t *__restrict__ bmnext_all, uint32_t *__restrict__ slotbm_all, Flags *__restrict__ fl) {
    const int64_t b = blockIdx.y;
    if (!bs[b].active) return;
    const int cur = level & 1;
    const int32_t *F = Fcur_all + b * n;
    uint32_t *bm = bmnext_all + b * nw;
    uint32_t *sbm = slotbm_all + b * nsw;
    const int32_t fsz = bs[b].fsz[cur];
    const int lane = __lane_id();
    const int64_t wstride = (int64_t)gridDim.x * kBlock;
    unsigned long long visits = 0;
    for (int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); base < fsz;
         base += wstride) {
        const WaveRows w = wave_rows(vrec, F, base, fsz, false);
        if (lane == 0) visits += w.total;
        for (int32_t j0 = 0; j0 < w.total; j0 += 64) {
            // cross-lane reads happen with every lane active; only memory accesses are masked
            const int32_t j = j0 + lane;
            const bool inr = j < w.total;
            const int32_t jc = inr ? j : w.total - 1;
            const int o = wave_owner(w.pre, jc);
            const int32_t ost = __shfl(w.start, o), opre = __shfl(w.pre, o);
            if (inr) {
                const int32_t e = ost + (jc - opre);
                const int32_t x = col[e];
                atomicOr(bm + (x >> 5), 1u << (x & 31));
                const int32_t slot = slotv[e];
                if (slot >= 0) atomicOr(sbm + (slot >> 5), 1u << (slot & 31));
            }
        }
    }
    visits = wave_sum_ll((long long)visits);
    if (lane == 0 && visits) atomicAdd(&fl->push_visits, visits);
}

// Next frontier list of each active source: the set bits of its next-level support bitmap,
// in ascending vertex order (one block per source).
__global__ __launch_bounds__(kBlock) void compact_frontier_kernel(
    BatchState *__restrict__ bs, int32_t n, int64_t nw, int32_t level,
    const uint32_t *__restrict__ bmnext_all, int32_t *__restrict__ Fnext_all) {
    __shared__ uint32_t wave_tot[kWavesPerBlock];
    __shared__ int32_t carry;
    const int64_t b = blockIdx.x;
    if (!bs[b].active) return;
    const int nxt = (level & 1) ^ 1;
    const uint32_t *bm = bmnext_all + b * nw;
    int32_t *Fn = Fnext_all + b * n;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t w0 = 0; w0 < nw; w0 += kBlock) {
        const int64_t wi = w0 + threadIdx.x;
        const uint32_t word = wi < nw ? bm[wi] : 0u;
        const uint32_t cnt = __popc(word);
        uint32_t inc = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        if (lane == 63) wave_tot[wave] = inc;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) {
            if (k < wave) before += wave_tot[k];
            all += wave_tot[k];
        }
        int32_t pos = carry + (int32_t)(before + inc - cnt);
        uint32_t rest = word;
        while (rest) {
            const int bit = __builtin_ctz(rest);
            rest &= rest - 1;
            Fn[pos++] = (int32_t)(wi * 32 + bit);
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += (int32_t)all;
        __syncthreads();
    }
    if (threadIdx.x == 0) bs[b].fsz[nxt] = carry;
}

constexpr int kFoldWindow = 256;  // LDS values per wavefront in the hub-row fold

// h_{l+1}(x) = (left fold over Gamma(x) in CSR order of h_l) / d(x) for x in the next support.
// Only terms in the support of h_l are folded (the others are zero), in row order:
//  - ordinary rows: the wavefront walks the concatenated rows of its 64 vertices and checks
//    each neighbour in the current support bitmap;
//  - hub rows: the set bits of the hub-slot bitmap over the row mark exactly the occupied
//    positions; their values are staged in LDS in row order and folded by one lane.
// Also accumulates the support volume and maximum of h_{l+1}, and clears the hub-slot bits.
__global__ __launch_bounds__(kBlock) void pull_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col, BatchState *__restrict__ bs,
    int32_t n, int64_t nw, int64_t nsw, int32_t level, const double *__restrict__ hcur_all,
    const uint32_t *__restrict__ bmcur_all, uint32_t *__restrict__ slotbm_all,
    double *__restrict__ hnext_all, const int32_t *__restrict__ Fnext_all,
    Flags *__restrict__ fl) {
    __shared__ double stage[kWavesPerBlock][kFoldWindow];
    const int64_t b = blockIdx.y;
    if (!bs[b].active) return;
    const int nxt = (level & 1) ^ 1;
    const double *h = hcur_all + b * n;
    const uint32_t *bm = bmcur_all + b * nw;
    uint32_t *sbm = slotbm_all + b * nsw;
    double *hn = hnext_all + b * n;
    const int32_t *F = Fnext_all + b * n;
    const int32_t fsz = bs[b].fsz[nxt];
    const int lane = __lane_id();
    double *lds = stage[threadIdx.x >> 6];
    const int64_t wstride = (int64_t)gridDim.x * kBlock;
    unsigned long long visits = 0, vol = 0;
    double hmax = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); base < fsz;
         base += wstride) {
        const WaveRows w = wave_rows(vrec, F, base, fsz, true);
        if (lane == 0) visits += w.total;
        double acc = 0.0;  // the fold of this lane's own (ordinary) row
        for (int32_t j0 = 0; j0 < w.total; j0 += 64) {
            const int32_t j = j0 + lane;
            const bool inr = j < w.total;
            const int32_t jc = inr ? j : w.total - 1;
            const int o = wave_owner(w.pre, jc);
            const int32_t ost = __shfl(w.start, o), opre = __shfl(w.pre, o);
            double v = 0.0;
            bool nz = false;
            if (inr) {
                const int32_t y = col[ost + (jc - opre)];
                if (bm[y >> 5] & (1u << (y & 31))) {
                    v = h[y];
                    nz = true;
                }
            }
            unsigned long long m = __ballot(nz);
            while (m) {  // ascending lanes = ascending row positions
                const int src = __builtin_ctzll(m);
                m &= m - 1;
                const double t = __shfl(v, src);
                const int owner = __shfl(o, src);
                if (lane == owner) acc += t;
            }
        }
        // hub rows of this group, one at a time
        const int2 rr = (w.x >= 0) ? vrec[w.x] : make_int2(0, 0);
        unsigned long long hubs = __ballot(rr.y > kHubRow);
        while (hubs) {
            const int hl = __builtin_ctzll(hubs);
            hubs &= hubs - 1;
            const int32_t a = __shfl(rr.x, hl), d = __shfl(rr.y, hl);
            const int32_t e1 = a + d;  // row positions [a, e1)
            const int64_t wfirst = a >> 5, wlast = (e1 - 1) >> 5;
            double hacc = 0.0;
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
                const int32_t T = __shfl(inc, 63);
                const int32_t pos0 = inc - cnt;
                for (int32_t r0 = 0; r0 < T; r0 += kFoldWindow) {
                    uint32_t rest = word;
                    int32_t p = pos0;
                    while (rest) {
                        const int bit = __builtin_ctz(rest);
                        rest &= rest - 1;
                        if (p >= r0 && p < r0 + kFoldWindow) {
                            const int32_t y = col[wi * 32 + bit];
                            lds[p - r0] = h[y];
                        }
                        ++p;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (lane == 0) {
                        const int32_t cntw = min(kFoldWindow, T - r0);
                        for (int32_t i = 0; i < cntw; ++i) hacc += lds[i];
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
            }
            hacc = __shfl(hacc, 0);
            if (lane == hl) acc = hacc;
        }
        if (w.x >= 0) {
            const double hv = acc / (double)rr.y;
            hn[w.x] = hv;
            vol += (unsigned long long)rr.y;
            hmax = fmax(hmax, hv);
        }
    }
    visits = wave_sum_ll((long long)visits);
    vol = wave_sum_ll((long long)vol);
    hmax = wave_max_d(hmax);
    if (lane == 0) {
        if (visits) atomicAdd(&fl->push_visits, visits);
        if (vol) {
            atomicAdd(&bs[b].vol[nxt], vol);
            atomicMax(&bs[b].hmaxbits[nxt], (unsigned long long)__double_as_longlong(hmax));
        }
    }
}

// After a level: zero h_l and its support bitmap over the support, so both are clean when the
// buffers are reused for level l + 2.  (Every set bit of a touched bitmap word belongs to the
// support, so the whole word is cleared.)
__global__ __launch_bounds__(kBlock) void clear_level_kernel(const BatchState *__restrict__ bs,
                                                             int32_t n, int64_t nw, int parity,
                                                             bool only_active,
                                                             double *__restrict__ hA,
                                                             double *__restrict__ hB,
                                                             uint32_t *__restrict__ bmA,
                                                             uint32_t *__restrict__ bmB,
                                                             const int32_t *__restrict__ FA,
                                                             const int32_t *__restrict__ FB) {
    const int64_t b = blockIdx.y;
    if (only_active && !bs[b].active) return;
    const int pb = parity < 0 ? bs[b].finalbuf : parity;
    double *h = (pb ? hB : hA) + b * (int64_t)n;
    uint32_t *bm = (pb ? bmB : bmA) + b * nw;
    const int32_t *F = (pb ? FB : FA) + b * (int64_t)n;
    const int32_t fsz = bs[b].fsz[pb];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < fsz;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = F[i];
        h[x] = 0.0;
        bm[x >> 5] = 0u;
    }
}

// Walk pairs per wanted directed edge and the number of 64-walk chunks they need.
__global__ __launch_bounds__(kBlock) void nreq_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ bsrc,
    const BatchState *__restrict__ bs, int32_t nb, const int64_t *__restrict__ ebase,
    const int32_t *__restrict__ tau, const int32_t *__restrict__ ttau_src,
    const uint8_t *__restrict__ want, double c, long long *__restrict__ nreq,
    long long *__restrict__ chunks, Flags *__restrict__ fl) {
    const int lane = __lane_id();
    const int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (b >= nb) return;
    const int32_t s = bsrc[b];
    const int2 r = vrec[s];
    const int32_t tt = ttau_src[s];
    const double hmax = bs[b].hmax;
    long long steps = 0, walks = 0;
    int ovf = 0;
    for (int32_t i = lane; i < r.y; i += 64) {
        const int32_t e = r.x + i;
        long long nr = 0;
        const int32_t L = tau[e] - tt;
        if (want[e] && L > 0) {
            nr = nwalks(L, hmax, r.y, c);
            if (nr < 0) {
                ovf = 1;
                nr = 0;
            }
        }
        nreq[e] = nr;
        chunks[ebase[b] + i] = (2 * nr + kChunk - 1) / kChunk;
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

// The walk pairs (Alg. 1 inner loop): chunk c of local edge le holds walks
// j = 64 (c - coff[le]) + lane; j < n walk from s (side 0, index j), n <= j < 2n walk from t
// (side 1, index j - n).  Each walk sums h_ttau over its positions 1..L.
__global__ __launch_bounds__(kBlock) void mc_walk_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
    const int32_t *__restrict__ bsrc, const BatchState *__restrict__ bs, int32_t nb, int32_t n,
    const int64_t *__restrict__ ebase, const int64_t *__restrict__ coff, int64_t nle,
    const int32_t *__restrict__ tau, const int32_t *__restrict__ ttau_src,
    const long long *__restrict__ nreq, const double *__restrict__ hA,
    const double *__restrict__ hB, const uint32_t *__restrict__ bmA,
    const uint32_t *__restrict__ bmB, int64_t nw, uint32_t seed, uint32_t G, uint32_t S,
    double *__restrict__ partial, unsigned long long *__restrict__ vis0,
    unsigned long long *__restrict__ vis1) {
    const int lane = __lane_id();
    const int64_t T = coff[nle];
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); c < T;
         c += nwaves) {
        const int64_t le = upper_index(coff, nle + 1, c);
        const int64_t b = upper_index(ebase, nb + 1, le);
        const int32_t s = bsrc[b];
        const int2 rs = vrec[s];
        const int32_t e = rs.x + (int32_t)(le - ebase[b]);
        const int32_t t = col[e];
        const long long nr = nreq[e];
        const int32_t L = tau[e] - ttau_src[s];
        const int fb = bs[b].finalbuf;
        const double *h = (fb ? hB : hA) + b * (int64_t)n;
        const uint32_t *bm = (fb ? bmB : bmA) + b * nw;
        const long long j = (c - coff[le]) * kChunk + lane;
        const bool active = j < 2 * nr;
        const int side = j >= nr ? 1 : 0;
        const long long k = j - side * nr;
        double acc = 0.0;
        long long hits = 0;
        if (active) {
            const WalkKey key = walk_key(seed, (uint32_t)s, (uint32_t)t, (uint32_t)side,
                                         (uint64_t)k, G, S);
            int32_t cur = side ? t : s;
            for (int32_t l = 1; l <= L; ++l) {
                cur = walk_step(vrec, col, cur, (uint32_t)l, key);
                if (bm[cur >> 5] & (1u << (cur & 31))) {  // h_ttau is zero off its support
                    acc += h[cur];
                    hits += 1;
                }
            }
        }
        const double sum = wave_sum_d(active ? (side ? -acc : acc) : 0.0);
        const long long h0 = wave_sum_ll(active && !side ? hits : 0);
        const long long h1 = wave_sum_ll(active && side ? hits : 0);
        if (lane == 0) {
            partial[c] = sum;
            if (h0) atomicAdd(vis0 + e, (unsigned long long)h0);
            if (h1) atomicAdd(vis1 + e, (unsigned long long)h1);
        }
    }
}

// Per directed edge: MC = its chunk sums in chunk order; g(s,t) = (D + MC / n) / d_s.
__global__ void edge_reduce_kernel(const int2 *__restrict__ vrec, const int32_t *__restrict__ bsrc,
                                   int32_t nb, const int64_t *__restrict__ ebase,
                                   const int64_t *__restrict__ coff, int64_t nle,
                                   const uint8_t *__restrict__ want,
                                   const long long *__restrict__ nreq,
                                   const double *__restrict__ D, const double *__restrict__ partial,
                                   double *__restrict__ MC, double *__restrict__ g) {
    for (int64_t le = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; le < nle;
         le += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = upper_index(ebase, nb + 1, le);
        const int32_t s = bsrc[b];
        const int2 rs = vrec[s];
        const int32_t e = rs.x + (int32_t)(le - ebase[b]);
        if (!want[e]) continue;
        double mc = 0.0;
        for (int64_t c = coff[le]; c < coff[le + 1]; ++c) mc += partial[c];
        const long long nr = nreq[e];
        MC[e] = mc;
        g[e] = nr > 0 ? (D[e] + mc / (double)nr) / (double)rs.y : D[e] / (double)rs.y;
    }
}

__global__ void finalize_all_kernel(const int32_t *__restrict__ canon,
                                    const int32_t *__restrict__ rev, int64_t m,
                                    const double *__restrict__ g, double *__restrict__ sc) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = canon[i];
        sc[i] = g[e] + g[rev[e]];
    }
}

__global__ void finalize_query_kernel(const int32_t *__restrict__ qe, int64_t q,
                                      const double *__restrict__ g, double *__restrict__ sc) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q;
         j += (int64_t)gridDim.x * blockDim.x)
        sc[j] = g[qe[2 * j]] + g[qe[2 * j + 1]];
}

__global__ void export_kernel(const int32_t *__restrict__ row_of, int64_t nnz,
                              const int32_t *__restrict__ ttau_src, int32_t *__restrict__ ttau) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        ttau[e] = ttau_src[row_of[e]];
}

// ------------------------------------------------------------ host driver
static unsigned grid_for(int64_t items, int per_block, unsigned cap = 1u << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

struct Outputs {
    double *sc = nullptr;       // [m] (all) or [q] (query)
    const int32_t *edges = nullptr;
    int64_t q = -1;             // -1: all edges
    int32_t *tau = nullptr, *ttau = nullptr;
    int64_t *nreq = nullptr, *vis0 = nullptr, *vis1 = nullptr;
    double *D = nullptr, *MC = nullptr, *g = nullptr;
};

static int aesc_impl(Graph *g, const saba_aesc_params *p, const Outputs &o, saba_stats *st,
                     hipStream_t s) {
    const int32_t n = g->n;
    const int64_t nnz = g->nnz, m = nnz / 2;
    if (!(p->eps > 0.0) || !(p->delta > 0.0 && p->delta < 1.0) || !(p->lambda >= 0.0) ||
        p->group < 1 || p->spread > 31 ||
        (p->group > 1 && ((uint64_t)(p->group - 1) << p->spread) > 0xFFFFFFFFull)) {
        set_error("invalid estimator parameters");
        return SABA_E_INVALID;
    }
    if (!g->connected || n < 2) {
        set_error("the estimator needs a connected graph with at least one edge");
        return SABA_E_DISCONNECTED;
    }
    if (g->bipartite || !(p->lambda < 1.0)) {
        set_error("the estimator needs a non-bipartite graph (lambda < 1)");
        return SABA_E_BIPARTITE;
    }
    const int32_t cap = p->tau_cap > 0 ? p->tau_cap : 4096;
    const double c = 32.0 * std::log(4.0 * (double)m / p->delta) / (p->eps * p->eps);
    const bool timing = st && p->time_kernels;
    hipEvent_t ev[4] = {};
    if (timing)
        for (auto &e : ev) SABA_HIP_TRY(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *ev;
        ~EvGuard() {
            for (int i = 0; i < 4; ++i)
                if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    } evguard{ev};
    float walk_ms = 0.f;
    if (timing) SABA_HIP_TRY(hipEventRecord(ev[0], s));

    auto &E = g->est;
    SABA_TRY(E[B_TAU].ensure(sizeof(int32_t) * nnz));
    SABA_TRY(E[B_D].ensure(sizeof(double) * nnz));
    SABA_TRY(E[B_NREQ].ensure(sizeof(long long) * nnz));
    SABA_TRY(E[B_MC].ensure(sizeof(double) * nnz));
    SABA_TRY(E[B_VIS0].ensure(sizeof(long long) * nnz));
    SABA_TRY(E[B_VIS1].ensure(sizeof(long long) * nnz));
    SABA_TRY(E[B_G].ensure(sizeof(double) * nnz));
    SABA_TRY(E[B_TTAU_SRC].ensure(sizeof(int32_t) * n));
    SABA_TRY(E[B_MAXTAU_SRC].ensure(sizeof(int32_t) * n));
    SABA_TRY(E[B_WANT].ensure(nnz));
    SABA_TRY(E[B_LIST].ensure(sizeof(int32_t) * n));
    SABA_TRY(E[B_FLAGS].ensure(sizeof(Flags)));
    int32_t *tau = E[B_TAU].as<int32_t>();
    double *D = E[B_D].as<double>();
    long long *nreq = E[B_NREQ].as<long long>();
    double *MC = E[B_MC].as<double>();
    auto *vis0 = E[B_VIS0].as<unsigned long long>();
    auto *vis1 = E[B_VIS1].as<unsigned long long>();
    double *gd = E[B_G].as<double>();
    int32_t *ttau_src = E[B_TTAU_SRC].as<int32_t>();
    int32_t *maxtau = E[B_MAXTAU_SRC].as<int32_t>();
    uint8_t *want = E[B_WANT].as<uint8_t>();
    int32_t *list = E[B_LIST].as<int32_t>();
    Flags *fl = E[B_FLAGS].as<Flags>();
    SABA_HIP_TRY(hipMemsetAsync(fl, 0, sizeof(Flags), s));

    tau_kernel<<<grid_for(n, kWavesPerBlock, 1 << 16), kBlock, 0, s>>>(
        g->vrec, g->col_idx, n, p->lambda, p->eps, cap, tau, maxtau, fl);
    SABA_HIP_TRY(hipGetLastError());

    // sources and wanted directed edges
    int64_t ns = n;
    int32_t *qe = nullptr;
    if (o.q < 0) {
        SABA_HIP_TRY(hipMemsetAsync(want, 1, nnz, s));
        iota_kernel<<<grid_for(n, 256, 1 << 16), 256, 0, s>>>(list, n);
        SABA_HIP_TRY(hipGetLastError());
    } else {
        SABA_TRY(E[B_SRCMARK].ensure(sizeof(long long) * n));
        SABA_TRY(E[B_SRCPOS].ensure(sizeof(int64_t) * (n + 1)));
        SABA_TRY(E[B_SCAN].ensure(scan_tmp_bytes(n)));
        SABA_TRY(E[B_QE].ensure(sizeof(int32_t) * 2 * std::max<int64_t>(o.q, 1)));
        qe = E[B_QE].as<int32_t>();
        long long *srcmark = E[B_SRCMARK].as<long long>();
        int64_t *srcpos = E[B_SRCPOS].as<int64_t>();
        SABA_HIP_TRY(hipMemsetAsync(want, 0, nnz, s));
        SABA_HIP_TRY(hipMemsetAsync(srcmark, 0, sizeof(long long) * n, s));
        if (o.q > 0) {
            query_mark_kernel<<<grid_for(o.q, 256, 1 << 16), 256, 0, s>>>(
                g->vrec, g->col_idx, n, o.edges, o.q, want, srcmark, qe, fl);
            SABA_HIP_TRY(hipGetLastError());
        }
        SABA_TRY(scan_i64(reinterpret_cast<int64_t *>(srcmark), srcpos, n, E[B_SCAN].ptr, s));
        compact_kernel<<<grid_for(n, 256, 1 << 16), 256, 0, s>>>(srcmark, srcpos, n, list);
        SABA_HIP_TRY(hipGetLastError());
        Flags hf;
        SABA_HIP_TRY(hipMemcpyAsync(&ns, srcpos + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipMemcpyAsync(&hf, fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipStreamSynchronize(s));
        if (hf.err & kErrNotEdge) {
            set_error("a query pair is not an edge of the graph");
            return SABA_E_NOT_EDGE;
        }
    }

    // batch size from the memory budget: two dense FP64 levels, two frontiers, two bitmaps
    size_t freeb = 0, totalb = 0;
    SABA_HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    int64_t budget = p->mem_budget > 0 ? p->mem_budget
                                       : std::min<int64_t>(8ll << 30, (int64_t)(0.4 * (double)freeb));
    const int64_t nw = ((int64_t)n + 31) / 32;
    const int64_t nsw = (nnz + 31) / 32;
    const int64_t per_src = (int64_t)n * (2 * 8 + 2 * 4) + 2 * 4 * nw + 4 * nsw;
    int64_t B = p->batch_sources > 0 ? p->batch_sources : std::max<int64_t>(1, budget / per_src);
    B = std::min<int64_t>({B, std::max<int64_t>(ns, 1), 65535});

    const bool grow = E[B_HA].bytes < sizeof(double) * (size_t)(B * n) ||
                      E[B_BMA].bytes < sizeof(uint32_t) * (size_t)(B * nw) ||
                      E[B_SLOTBM].bytes < sizeof(uint32_t) * (size_t)(B * nsw);
    SABA_TRY(E[B_HA].ensure(sizeof(double) * B * n));
    SABA_TRY(E[B_HB].ensure(sizeof(double) * B * n));
    SABA_TRY(E[B_FA].ensure(sizeof(int32_t) * B * n));
    SABA_TRY(E[B_FB].ensure(sizeof(int32_t) * B * n));
    SABA_TRY(E[B_BMA].ensure(sizeof(uint32_t) * B * nw));
    SABA_TRY(E[B_BMB].ensure(sizeof(uint32_t) * B * nw));
    SABA_TRY(E[B_SLOTBM].ensure(sizeof(uint32_t) * B * nsw));
    SABA_TRY(E[B_BSRC].ensure(sizeof(int32_t) * B));
    SABA_TRY(E[B_BSTATE].ensure(sizeof(BatchState) * B));
    SABA_TRY(E[B_EBASE].ensure(sizeof(int64_t) * (B + 1)));
    SABA_TRY(E[B_DEG64].ensure(sizeof(long long) * B));
    SABA_TRY(E[B_SCAN].ensure(std::max(scan_tmp_bytes(B), scan_tmp_bytes(nnz))));
    double *hA = E[B_HA].as<double>(), *hB = E[B_HB].as<double>();
    int32_t *FA = E[B_FA].as<int32_t>(), *FB = E[B_FB].as<int32_t>();
    uint32_t *bmA = E[B_BMA].as<uint32_t>(), *bmB = E[B_BMB].as<uint32_t>();
    uint32_t *slotbm = E[B_SLOTBM].as<uint32_t>();
    int32_t *bsrc = E[B_BSRC].as<int32_t>();
    BatchState *bs = E[B_BSTATE].as<BatchState>();
    int64_t *ebase = E[B_EBASE].as<int64_t>();
    long long *deg64 = E[B_DEG64].as<long long>();
    if (grow || !g->est_clean) {
        // dense vectors and bitmaps start at zero and are kept clean by the sparse clears
        SABA_HIP_TRY(hipMemsetAsync(hA, 0, E[B_HA].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(hB, 0, E[B_HB].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(bmA, 0, E[B_BMA].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(bmB, 0, E[B_BMB].bytes, s));
        SABA_HIP_TRY(hipMemsetAsync(slotbm, 0, E[B_SLOTBM].bytes, s));
    }
    g->est_clean = false;  // until this call has cleared everything it touched

    const unsigned ysplit = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, n / 4096));
    int64_t batches = 0;
    for (int64_t i0 = 0; i0 < ns; i0 += B) {
        const int32_t nb = (int32_t)std::min<int64_t>(B, ns - i0);
        ++batches;
        batch_init_kernel<<<grid_for(nb, kWavesPerBlock), kBlock, 0, s>>>(
            g->vrec, list, i0, nb, n, nw, bsrc, bs, hA, FA, bmA, D, nreq, MC, vis0, vis1, deg64);
        SABA_HIP_TRY(hipGetLastError());
        const dim3 grid(ysplit, (unsigned)nb);
        for (int32_t level = 0;; ++level) {
            const int cur = level & 1;
            double *hcur = cur ? hB : hA, *hnext = cur ? hA : hB;
            int32_t *Fcur = cur ? FB : FA, *Fnext = cur ? FA : FB;
            uint32_t *bmcur = cur ? bmB : bmA, *bmnext = cur ? bmA : bmB;
            SABA_HIP_TRY(hipMemsetAsync(&fl->any_active, 0, sizeof(int32_t), s));
            level_decide_kernel<<<grid_for(nb, kWavesPerBlock), kBlock, 0, s>>>(
                g->vrec, g->col_idx, bsrc, bs, nb, n, level, hcur, tau, maxtau, D, ttau_src, c,
                p->push_all, p->tilde_tau_max, fl);
            SABA_HIP_TRY(hipGetLastError());
            int32_t any = 0;
            SABA_HIP_TRY(hipMemcpyAsync(&any, &fl->any_active, sizeof(int32_t),
                                        hipMemcpyDeviceToHost, s));
            SABA_HIP_TRY(hipStreamSynchronize(s));
            if (!any) break;
            expand_kernel<<<grid, kBlock, 0, s>>>(g->vrec, g->col_idx, g->slotv, bs, n, nw, nsw,
                                                  level, Fcur, bmnext, slotbm, fl);
            compact_frontier_kernel<<<(unsigned)nb, kBlock, 0, s>>>(bs, n, nw, level, bmnext,
                                                                    Fnext);
            pull_kernel<<<grid, kBlock, 0, s>>>(g->vrec, g->col_idx, bs, n, nw, nsw, level, hcur,
                                                bmcur, slotbm, hnext, Fnext, fl);
            clear_level_kernel<<<grid, kBlock, 0, s>>>(bs, n, nw, cur, true, hA, hB, bmA, bmB, FA,
                                                       FB);
            SABA_HIP_TRY(hipGetLastError());
        }
        // walk pairs of the batch's edges
        SABA_TRY(scan_i64(reinterpret_cast<int64_t *>(deg64), ebase, nb, E[B_SCAN].ptr, s));
        int64_t nle = 0;
        SABA_HIP_TRY(hipMemcpyAsync(&nle, ebase + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipStreamSynchronize(s));
        SABA_TRY(E[B_CHUNKS].ensure(sizeof(long long) * std::max<int64_t>(nle, 1)));
        SABA_TRY(E[B_COFF].ensure(sizeof(int64_t) * (nle + 1)));
        long long *chunks = E[B_CHUNKS].as<long long>();
        int64_t *coff = E[B_COFF].as<int64_t>();
        nreq_kernel<<<grid_for(nb, kWavesPerBlock), kBlock, 0, s>>>(
            g->vrec, bsrc, bs, nb, ebase, tau, ttau_src, want, c, nreq, chunks, fl);
        SABA_HIP_TRY(hipGetLastError());
        SABA_TRY(scan_i64(reinterpret_cast<int64_t *>(chunks), coff, nle, E[B_SCAN].ptr, s));
        int64_t T = 0;
        Flags hf;
        SABA_HIP_TRY(hipMemcpyAsync(&T, coff + nle, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipMemcpyAsync(&hf, fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipStreamSynchronize(s));
        if (hf.err & kErrOverflow) {
            set_error("walk count overflows the 64-bit range (eps too small?)");
            return SABA_E_OVERFLOW;  // scratch stays marked dirty: re-zeroed on the next call
        }
        SABA_TRY(E[B_PART].ensure(sizeof(double) * std::max<int64_t>(T, 1)));
        double *partial = E[B_PART].as<double>();
        if (T > 0) {
            if (timing) SABA_HIP_TRY(hipEventRecord(ev[1], s));
            mc_walk_kernel<<<grid_for(T, kWavesPerBlock, 2048), kBlock, 0, s>>>(
                g->vrec, g->col_idx, bsrc, bs, nb, n, ebase, coff, nle, tau, ttau_src, nreq, hA,
                hB, bmA, bmB, nw, p->seed, p->group, p->spread, partial, vis0, vis1);
            SABA_HIP_TRY(hipGetLastError());
            if (timing) {
                SABA_HIP_TRY(hipEventRecord(ev[2], s));
                SABA_HIP_TRY(hipEventSynchronize(ev[2]));
                float ms = 0.f;
                SABA_HIP_TRY(hipEventElapsedTime(&ms, ev[1], ev[2]));
                walk_ms += ms;
            }
        }
        edge_reduce_kernel<<<grid_for(nle, 256, 1 << 16), 256, 0, s>>>(
            g->vrec, bsrc, nb, ebase, coff, nle, want, nreq, D, partial, MC, gd);
        // leave the dense vectors and bitmaps of the batch zero: clear h_ttau over its support
        clear_level_kernel<<<grid, kBlock, 0, s>>>(bs, n, nw, -1, false, hA, hB, bmA, bmB, FA, FB);
        SABA_HIP_TRY(hipGetLastError());
    }
    g->est_clean = true;

    if (o.sc) {
        if (o.q < 0) {
            finalize_all_kernel<<<grid_for(m, 256, 1 << 16), 256, 0, s>>>(g->canon, g->rev, m, gd,
                                                                         o.sc);
        } else if (o.q > 0) {
            finalize_query_kernel<<<grid_for(o.q, 256, 1 << 16), 256, 0, s>>>(qe, o.q, gd, o.sc);
        }
        SABA_HIP_TRY(hipGetLastError());
    }
    auto cp = [&](void *dst, const void *src, size_t bytes) -> int {
        if (dst) SABA_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
        return SABA_OK;
    };
    SABA_TRY(cp(o.tau, tau, sizeof(int32_t) * nnz));
    SABA_TRY(cp(o.nreq, nreq, sizeof(int64_t) * nnz));
    SABA_TRY(cp(o.D, D, sizeof(double) * nnz));
    SABA_TRY(cp(o.MC, MC, sizeof(double) * nnz));
    SABA_TRY(cp(o.vis0, vis0, sizeof(int64_t) * nnz));
    SABA_TRY(cp(o.vis1, vis1, sizeof(int64_t) * nnz));
    SABA_TRY(cp(o.g, gd, sizeof(double) * nnz));
    if (o.ttau) {
        export_kernel<<<grid_for(nnz, 256, 1 << 16), 256, 0, s>>>(g->row_of, nnz, ttau_src, o.ttau);
        SABA_HIP_TRY(hipGetLastError());
    }
    if (timing) SABA_HIP_TRY(hipEventRecord(ev[3], s));
    Flags hf;
    SABA_HIP_TRY(hipMemcpyAsync(&hf, fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipStreamSynchronize(s));
    if (st) {
        *st = saba_stats{};
        st->walks = (int64_t)hf.walks;
        st->walk_steps = (int64_t)hf.walk_steps;
        st->push_edge_visits = (int64_t)hf.push_visits;
        st->sources = ns;
        st->batches = batches;
        st->max_tau = hf.max_tau;
        st->max_ttau = hf.max_ttau;
        st->warnings = hf.warnings;
        if (timing) {
            float tot = 0.f;
            SABA_HIP_TRY(hipEventElapsedTime(&tot, ev[0], ev[3]));
            st->kernel_ms = walk_ms;
            st->total_ms = tot;
        }
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
    Outputs o;
    o.sc = d_sc;
    return aesc_impl(G(gh), p, o, st, static_cast<hipStream_t>(stream));
}

extern "C" int saba_aesc_query(saba_graph *gh, const saba_aesc_params *p, const int32_t *d_edges,
                               int64_t q, double *d_sc, saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p || q < 0 || (q > 0 && (!d_edges || !d_sc))) {
        set_error("invalid query arguments");
        return SABA_E_INVALID;
    }
    Outputs o;
    o.sc = d_sc;
    o.edges = d_edges;
    o.q = q;
    return aesc_impl(G(gh), p, o, st, static_cast<hipStream_t>(stream));
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
    Outputs o;
    o.sc = d_sc;
    o.tau = d_tau;
    o.ttau = d_ttau;
    o.nreq = d_nreq;
    o.D = d_D;
    o.MC = d_MC;
    o.vis0 = d_vis0;
    o.vis1 = d_vis1;
    o.g = d_g;
    return aesc_impl(G(gh), p, o, st, static_cast<hipStream_t>(stream));
}

// Random-walk generation: Alg. 2 (one lane per walk) and Alg. 3 (bouquets: the
// walks of one start vertex advance side by side in a wavefront), with the
// neighbour choice of Eq. (5) and the keyed seed arrangement of Sec. 3.3.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "saba_internal.hpp"

namespace saba {

constexpr int kWalkBlock = 256;

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

// Bucket order: bsrc[w] = s for offs[s] <= w < offs[s + 1].
__global__ __launch_bounds__(kWalkBlock) void source_fill_kernel(const int64_t *__restrict__ offs,
                                                                 int32_t n,
                                                                 int32_t *__restrict__ bsrc) {
    const int64_t W = offs[n];
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < W;
         w += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = n;  // largest s with offs[s] <= w
        while (hi - lo > 1) {
            int32_t mid = lo + ((hi - lo) >> 1);
            if (offs[mid] <= w)
                lo = mid;
            else
                hi = mid;
        }
        bsrc[w] = lo;
    }
}

// Alg. 2: one lane per walk, walks in the order the sources are given.  The rank of
// a walk among the walks of its source is taken from a per-source counter; the set
// of (source, rank) pairs, and so the histograms, does not depend on which walk
// receives which rank.
__global__ __launch_bounds__(kWalkBlock) void walk_naive_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col, const int32_t *__restrict__ src,
    int64_t W, int32_t L, uint32_t seed, uint32_t G, uint32_t S, int32_t n,
    uint32_t *__restrict__ cursor, unsigned long long *__restrict__ endpoint,
    unsigned long long *__restrict__ visits, int32_t *__restrict__ err) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    const int32_t s = src[j];
    if (s < 0 || s >= n || vrec[s].y == 0) {
        atomicOr(err, 1);
        return;
    }
    const uint32_t r = atomicAdd(cursor + s, 1u);
    const WalkKey key = walk_key(seed, (uint32_t)s, 0u, 0u, r, G, S);
    int32_t cur = s;
    for (int32_t l = 1; l <= L; ++l) {
        cur = walk_step(vrec, col, cur, (uint32_t)l, key);
        atomicAdd(visits + cur, 1ull);
    }
    atomicAdd(endpoint + cur, 1ull);
}

// Alg. 3: bouquets.  Walks are taken in bucket order, so the lanes of a wavefront
// hold consecutive walks of the same start vertex: their first gathers hit the
// same row, lanes standing on the same vertex share one request, and equal visits
// of adjacent lanes are merged before the atomics.
__global__ __launch_bounds__(kWalkBlock) void walk_bouquet_kernel(
    const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
    const int32_t *__restrict__ bsrc, const int64_t *__restrict__ offs, int32_t n, int32_t L,
    uint32_t seed, uint32_t G, uint32_t S, unsigned long long *__restrict__ endpoint,
    unsigned long long *__restrict__ visits) {
    // offs[n] counts only the walks whose start is a valid, non-isolated vertex
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = w < offs[n];
    int32_t cur = 0;
    WalkKey key{0u, 0u};
    if (active) {
        const int32_t s = bsrc[w];
        const uint64_t r = (uint64_t)(w - offs[s]);
        key = walk_key(seed, (uint32_t)s, 0u, 0u, r, G, S);
        cur = s;
    }
    for (int32_t l = 1; l <= L; ++l) {
        if (active) cur = walk_step(vrec, col, cur, (uint32_t)l, key);
        wave_merged_add(visits, cur, active);
    }
    wave_merged_add(endpoint, cur, active);
}

static int walks_impl(Graph *g, const saba_walk_params *p, int64_t *d_endpoint,
                      int64_t *d_visits, saba_stats *st, hipStream_t s) {
    const int64_t W = p->n_walks;
    const int32_t n = g->n;
    if (W < 0 || p->length < 0 || p->group < 1 || p->spread > 31 ||
        (p->group > 1 && ((uint64_t)(p->group - 1) << p->spread) > 0xFFFFFFFFull) ||
        (W > 0 && !p->d_sources) || !d_endpoint || !d_visits ||
        (p->mode != SABA_WALK_NAIVE && p->mode != SABA_WALK_BOUQUET)) {
        set_error("invalid walk parameters");
        return SABA_E_INVALID;
    }
    if ((__int128)W * (p->length > 0 ? p->length : 1) >= ((__int128)1 << 62)) {
        set_error("walk count too large");
        return SABA_E_OVERFLOW;
    }
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const bool timing = st && p->time_kernels;
    if (timing)
        for (auto &e : ev) SABA_HIP_TRY(hipEventCreate(&e));
    auto cleanup = [&]() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    if (timing) SABA_HIP_TRY(hipEventRecord(ev[0], s));

    SABA_TRY(g->walk_scratch[3].ensure(sizeof(int32_t)));
    int32_t *err = g->walk_scratch[3].as<int32_t>();
    SABA_HIP_TRY(hipMemsetAsync(err, 0, sizeof(int32_t), s));
    SABA_HIP_TRY(hipMemsetAsync(d_endpoint, 0, sizeof(int64_t) * (size_t)n, s));
    SABA_HIP_TRY(hipMemsetAsync(d_visits, 0, sizeof(int64_t) * (size_t)n, s));
    auto *ep = reinterpret_cast<unsigned long long *>(d_endpoint);
    auto *vi = reinterpret_cast<unsigned long long *>(d_visits);

    if (W > 0 && p->mode == SABA_WALK_NAIVE) {
        SABA_TRY(g->walk_scratch[0].ensure(sizeof(uint32_t) * (size_t)n));
        uint32_t *cursor = g->walk_scratch[0].as<uint32_t>();
        SABA_HIP_TRY(hipMemsetAsync(cursor, 0, sizeof(uint32_t) * (size_t)n, s));
        if (timing) SABA_HIP_TRY(hipEventRecord(ev[1], s));
        unsigned blocks = (unsigned)((W + kWalkBlock - 1) / kWalkBlock);
        walk_naive_kernel<<<blocks, kWalkBlock, 0, s>>>(g->vrec, g->col_idx, p->d_sources, W,
                                                        p->length, p->seed, p->group, p->spread,
                                                        n, cursor, ep, vi, err);
        SABA_HIP_TRY(hipGetLastError());
        if (timing) SABA_HIP_TRY(hipEventRecord(ev[2], s));
    } else if (W > 0) {
        SABA_TRY(g->walk_scratch[0].ensure(sizeof(int64_t) * (size_t)n));
        SABA_TRY(g->walk_scratch[1].ensure(sizeof(int64_t) * ((size_t)n + 1) + scan_tmp_bytes(n)));
        SABA_TRY(g->walk_scratch[2].ensure(sizeof(int32_t) * (size_t)W));
        auto *counts = g->walk_scratch[0].as<unsigned long long>();
        int64_t *offs = g->walk_scratch[1].as<int64_t>();
        void *scan_tmp = offs + n + 1;
        int32_t *bsrc = g->walk_scratch[2].as<int32_t>();
        SABA_HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int64_t) * (size_t)n, s));
        unsigned cblocks = (unsigned)std::min<int64_t>((W + kWalkBlock - 1) / kWalkBlock, 1 << 16);
        source_count_kernel<<<cblocks, kWalkBlock, 0, s>>>(p->d_sources, W, g->vrec, n, counts, err);
        SABA_HIP_TRY(hipGetLastError());
        SABA_TRY(scan_i64(reinterpret_cast<int64_t *>(counts), offs, n, scan_tmp, s));
        source_fill_kernel<<<cblocks, kWalkBlock, 0, s>>>(offs, n, bsrc);
        SABA_HIP_TRY(hipGetLastError());
        if (timing) SABA_HIP_TRY(hipEventRecord(ev[1], s));
        unsigned blocks = (unsigned)((W + kWalkBlock - 1) / kWalkBlock);
        walk_bouquet_kernel<<<blocks, kWalkBlock, 0, s>>>(g->vrec, g->col_idx, bsrc, offs, n,
                                                          p->length, p->seed, p->group, p->spread,
                                                          ep, vi);
        SABA_HIP_TRY(hipGetLastError());
        if (timing) SABA_HIP_TRY(hipEventRecord(ev[2], s));
    }
    if (timing) SABA_HIP_TRY(hipEventRecord(ev[3], s));
    int32_t h_err = 0;
    SABA_HIP_TRY(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipStreamSynchronize(s));
    if (h_err) {
        cleanup();
        set_error("a walk source is out of range or an isolated vertex");
        return SABA_E_INVALID;
    }
    if (st) {
        *st = saba_stats{};
        st->walks = W;
        st->walk_steps = W * (int64_t)p->length;
        if (timing) {
            float a = 0.f, b = 0.f;
            if (W > 0) SABA_HIP_TRY(hipEventElapsedTime(&a, ev[1], ev[2]));
            SABA_HIP_TRY(hipEventElapsedTime(&b, ev[0], ev[3]));
            st->kernel_ms = a;
            st->total_ms = b;
        }
    }
    cleanup();
    return SABA_OK;
}

}  // namespace saba

using namespace saba;

extern "C" int saba_walks(saba_graph *gh, const saba_walk_params *p, int64_t *d_endpoint,
                          int64_t *d_visits, saba_stats *st, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!p) {
        set_error("params is NULL");
        return SABA_E_INVALID;
    }
    return walks_impl(G(gh), p, d_endpoint, d_visits, st, static_cast<hipStream_t>(stream));
}

// The grouped-bouquet autotuner: the fastest key schedule (G, S) of the walk call whose walks
// stay within a correlation budget, measured with the branching statistic of the walks
// themselves (Sec. 3.3; the distinct vertices per vector of 8 consecutive walks, the Table 5
// experiment).  G > 1 changes which walks are drawn, so the schedule is returned, never kept.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "saba_internal.hpp"

using namespace saba;

extern "C" int saba_autotune_bouquet(saba_graph *gh, const saba_walk_params *sample,
                                     double min_distinct, saba_bouquet_choice *best,
                                     void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!sample || !best || !(min_distinct >= 1.0 && min_distinct <= 8.0)) {
        set_error("sample or best is NULL, or the budget lies outside [1, 8]");
        return SABA_E_INVALID;
    }
    Graph *g = G(gh);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t n1 = g->n > 0 ? g->n : 1;
    DevBuf out;
    SABA_TRY(out.ensure(sizeof(int64_t) * (2 * (size_t)n1 + 9)));
    struct Guard {
        DevBuf *b;
        ~Guard() { b->release(); }
    } guard{&out};
    int64_t *ep = out.as<int64_t>(), *vi = ep + n1, *dist = vi + n1;
    saba_walk_params p = *sample;
    p.mode = SABA_WALK_BOUQUET;
    struct Cand {
        uint32_t G, S;
    };
    std::vector<Cand> cands{{1u, 0u}};
    for (uint32_t Gc : {8u, 64u, 256u})
        for (uint32_t Sc = 4; Sc <= 28; Sc += 4)
            if (((uint64_t)(Gc - 1) << Sc) <= 0xFFFFFFFFull) cands.push_back({Gc, Sc});
    saba_bouquet_choice pick{};
    pick.ms = 1e300;
    int64_t h[9];
    for (const Cand &c : cands) {
        p.group = c.G;
        p.spread = c.S;
        // the branching statistic of this schedule (the counting kernels), then its speed
        p.d_distinct = dist;
        p.time_kernels = 0;
        SABA_TRY(saba_walks(gh, &p, ep, vi, nullptr, stream));
        SABA_HIP_TRY(hipMemcpyAsync(h, dist, sizeof(h), hipMemcpyDeviceToHost, s));
        SABA_HIP_TRY(hipStreamSynchronize(s));
        double tot = 0.0, wsum = 0.0;
        for (int k = 1; k <= 8; ++k) {
            tot += (double)h[k];
            wsum += (double)k * (double)h[k];
        }
        const double mean = tot > 0.0 ? wsum / tot : 8.0;
        if (!(mean >= min_distinct)) continue;
        p.d_distinct = nullptr;
        p.time_kernels = 1;
        double ms = 0.0;
        for (int rep = 0; rep < 3; ++rep) {  // one warm-up, two timed
            saba_stats st{};
            SABA_TRY(saba_walks(gh, &p, ep, vi, &st, stream));
            if (rep > 0) ms += 0.5 * st.total_ms;
        }
        if (ms < pick.ms) {
            pick.group = c.G;
            pick.spread = c.S;
            pick.distinct_mean = mean;
            pick.ms = ms;
        }
    }
    *best = pick;
    return SABA_OK;
}

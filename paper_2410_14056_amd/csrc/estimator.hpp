// Internal interface of the TGT+ estimator engine (Alg. 1): the batch executor that the
// synchronous calls and the request server share.
//
// A batch is a set of instances, each a (source vertex, parameter set) pair with a slot of
// dense scratch sized to its graph.  The executor runs the deterministic levels of every slot
// level-synchronously, then the walk pairs of every wanted instance edge in one launch, then
// the per-edge reduction g(s,t) = (D + MC / n) / d_s.  Instance-edge arrays are indexed by
// ie0 + (instance edge within the batch), so a caller may keep one array over many batches
// (the synchronous calls) or give each batch its own (the server).
#pragma once

#include <vector>

#include "saba_internal.hpp"

namespace saba {

// buffers of a Workspace
enum {
    B_PSET, B_SLOT, B_EB, B_BSTATE, B_WANT, B_TAU, B_D, B_NREQ, B_MC, B_VIS0, B_VIS1, B_G,
    B_TTAU, B_HA, B_HB, B_FA, B_FB, B_BMA, B_BMB, B_SLOTBM, B_CHUNKS, B_COFF, B_PART, B_SCAN,
    B_FLAGS, B_PAIRS, B_MAP, B_GOFS, B_HUBS, B_TILES, B_COUNT
};
static_assert(B_COUNT <= 32, "Workspace holds 32 buffers");

enum : int32_t { kErrOverflow = 1, kErrLayout = 2 };

struct PSet {  // one parameter set; c = 32 ln(4m / delta) / eps^2 uses its graph's m
    double lambda, eps, c;
    uint32_t seed, G, S;
    int32_t tau_cap, tilde_tau_max, push_all;
};

struct Slot {  // one instance of a batch
    int64_t hoff;   // first element of its dense vectors and frontier lists
    int64_t bmoff;  // first word of its vertex bitmaps
    int64_t sboff;  // first word of its CSR-position bitmap
    int64_t ie;     // first instance edge (index into the instance-edge arrays)
    int64_t inst;   // index into the per-instance ttau array
    int32_t v;      // source vertex (handle ids)
    int32_t p;      // parameter set
    int32_t goff;   // first vertex of its graph
    int32_t gn;     // vertices of its graph
    int32_t gpos;   // first CSR position of its graph
    int32_t pad;
};

struct Flags {
    int32_t err;
    int32_t any_active;
    int32_t nhub[2];  // entries of the hub-row lists of the two level parities
    int32_t max_tau;
    int32_t max_ttau;
    int32_t warnings;
    int32_t pad;
    unsigned long long walk_steps;
    unsigned long long push_visits;
    unsigned long long walks;
    unsigned long long wq[8];  // work-queue counters of the walk-pair launch, one per XCD range
};

// Device arrays a batch reads and writes, per instance edge unless noted.
struct EdgeArrays {
    const PSet *psets = nullptr;  // per parameter set
    const uint8_t *want = nullptr;
    int32_t *tau = nullptr;
    double *D = nullptr;
    long long *nreq = nullptr;
    double *MC = nullptr;
    unsigned long long *vis0 = nullptr, *vis1 = nullptr;
    double *g = nullptr;
    int32_t *ttau_inst = nullptr;  // per instance
    Flags *fl = nullptr;           // accumulated over batches until the caller resets it
};

// Dense scratch of one slot of a graph: two FP64 levels and two frontier lists of gn entries,
// two vertex bitmaps, one bitmap over the graph's CSR positions, and room for the graph's hub
// rows in the two hub-row lists.
struct SlotSize {
    int64_t h, bm, sb, hubs, bytes;
};

struct BatchTiming {
    bool on = false;
    hipEvent_t a = nullptr, b = nullptr;
    float walk_ms = 0.f;
};

// The omega > 0 form of CalculateTau: the kept eigenpairs' exact contribution beyond the
// truncation, sum_k (y_k(a) - y_k(b))^2 theta_k^(tau+1) / (1 - theta_k) with y_k = u_k / sqrt(d)
// (the geometric tail of the spectral series of the resistance).  The power by squaring.
__device__ __forceinline__ double eigen_tail(const double *__restrict__ theta,
                                             const double *__restrict__ y, int64_t gn,
                                             int32_t pairs, int32_t a, int32_t b, int32_t tau) {
    double acc = 0.0;
    for (int32_t k = 0; k < pairs; ++k) {
        const double t = theta[k];
        const double c = y[(int64_t)k * gn + a] - y[(int64_t)k * gn + b];
        double p = 1.0, base = t;
        for (uint32_t e = (uint32_t)tau + 1u; e; e >>= 1) {
            if (e & 1u) p *= base;
            base *= base;
        }
        acc += c * c * p / (1.0 - t);
    }
    return acc;
}

unsigned grid_for(int64_t items, int per_block, unsigned cap = 1u << 20);

// Validates one request against the handle (graph index, parameters, connectivity, lambda).
int check_request(const Graph *g, int32_t graph, const saba_aesc_params &p, int64_t q,
                  const void *edges);
PSet make_pset(const Graph *g, int32_t graph, const saba_aesc_params &p);
bool same_pset(const PSet &a, const PSet &b);
SlotSize slot_size(const Graph *g, int32_t graph);

// Instance-edge arrays for ne instance edges, ninst instances and np parameter sets.
int ensure_edge_arrays(Workspace &ws, int64_t ne, int64_t ninst, int32_t np, EdgeArrays *out);
// Pools for batches of up to nb slots holding h / bm / sb / hubs pool entries and ne instance
// edges.  Newly allocated pools are zeroed on stream s.
int ensure_pools(Workspace &ws, int64_t h, int64_t bm, int64_t sb, int64_t hubs, int64_t nb,
                 int64_t ne, hipStream_t s);
// Runs one batch on stream s.  hslots carry pool offsets (laid out by the caller within the
// sizes given to ensure_pools) and instance edges ie relative to the arrays; eb[b] is the first
// instance edge of slot b relative to ie0 (eb[nb] = nle).  Leaves every pool entry it touched
// zero again.  Returns after the walk launch has been queued; g is final once the stream has
// reached the end of the batch.
// cx (the counts export, may be null) also writes each slot's support and integer visit
// histograms before the batch's scratch is cleared.
struct CountExport;
int run_batch(const Graph *g, Workspace &ws, const EdgeArrays &ea, const std::vector<Slot> &hslots,
              const std::vector<int64_t> &eb, int64_t ie0, int64_t nle, int64_t maxgn,
              int64_t hubs, BatchTiming *tm, hipStream_t s, const CountExport *cx = nullptr);

// The two phases of run_batch, for callers that overlap the phases of consecutive batches on
// two streams with two workspaces.  batch_levels uploads the slots and runs the deterministic
// levels and the walk-pair counts on stream s; it returns with s drained (it reads the chunk
// total back).  batch_walks queues the walk pairs, the per-edge reduction and the clears of the
// same workspace on its stream, which must first wait for the levels phase; until they have
// run, the workspace may not be handed to another batch.  t0/t1 (may be null) are recorded
// around the walk-pair launch.
struct BatchPlan {
    int32_t nb = 0;
    int64_t ie0 = 0, nle = 0, T = 0;  // T: 64-walk chunks of the walk-pair launch
    int64_t maxgn = 1;                // vertices of the batch's largest graph
    unsigned ysplit = 1;
};
int batch_levels(const Graph *g, Workspace &ws, const EdgeArrays &ea,
                 const std::vector<Slot> &hslots, const std::vector<int64_t> &eb, int64_t ie0,
                 int64_t nle, int64_t maxgn, int64_t hubs, hipStream_t s, BatchPlan *plan);
int batch_walks(const Graph *g, Workspace &ws, const EdgeArrays &ea, const BatchPlan &plan,
                hipEvent_t t0, hipEvent_t t1, hipStream_t s, const CountExport *cx = nullptr);

}  // namespace saba

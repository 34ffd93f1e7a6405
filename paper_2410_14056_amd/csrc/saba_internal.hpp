// Internal declarations of libsaba: the graph handle, device scratch buffers,
// error reporting and the device functions of the walk sampler.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "saba.h"

namespace saba {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
void clear_error();

#define SABA_HIP_TRY(expr)                                                                   \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess) {                                                              \
            ::saba::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));            \
            return SABA_E_HIP;                                                               \
        }                                                                                    \
    } while (0)

// The library status of a HIP call's result (the message is set on failure), for code that has
// to clean up before it returns.
#define SABA_HIP_STATUS(expr)                                                                \
    ([&]() -> int {                                                                          \
        hipError_t _e = (expr);                                                              \
        if (_e == hipSuccess) return SABA_OK;                                                \
        ::saba::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));                \
        return SABA_E_HIP;                                                                   \
    }())

#define SABA_TRY(expr)                 \
    do {                               \
        int _rc = (expr);              \
        if (_rc != SABA_OK) return _rc; \
    } while (0)

// Grow-only device buffer.  A buffer that has to grow is reallocated with a quarter of
// headroom, so a sequence of slowly growing requests reallocates only a few times.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want);
    void release();
    template <class T>
    T *as() const { return static_cast<T *>(ptr); }
};

// Scratch of one estimator stream: per-batch pools and per-instance-edge arrays.  `clean`
// records that the dense vectors and bitmaps of the pools are all zero (the estimator keeps
// them so by clearing exactly what it touched).
struct Workspace {
    DevBuf b[32];
    bool clean = false;
    void release() {
        for (auto &x : b) x.release();
        clean = false;
    }
};

// Device-resident graph.  vrec[v] = (row start, degree) so one 8-byte gather gives
// both; rev[e] is the CSR position of the reverse entry of e; canon[i] is the CSR
// position of the i-th undirected edge in canonical (u < v, lexicographic) order.
struct Graph {
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t d_max = 0;
    int32_t n_isolated = 0;
    int32_t connected = 0;
    int32_t bipartite = 0;
    // A handle may hold several graphs side by side (block-diagonal CSR).  Graph k owns the
    // vertices [goff[k], goff[k+1]); its canonical edges are canon[cbase[k] .. cbase[k+1]).
    int32_t ngraphs = 1;
    std::vector<int32_t> goff;
    std::vector<int64_t> cbase;
    std::vector<int8_t> gconnected, gbipartite;
    std::vector<int64_t> ghubs;  // vertices of each graph whose rows are hub rows
    std::vector<int32_t> h_row_ptr, h_col_idx;
    int32_t *row_ptr = nullptr;
    int32_t *col_idx = nullptr;
    int2 *vrec = nullptr;
    int32_t *rev = nullptr;
    int32_t *canon = nullptr;
    int32_t *row_of = nullptr;  // source vertex of each CSR entry
    int32_t *slotv = nullptr;   // rev[e] if the row of col[e] is longer than kHubRow, else -1
    uint32_t *hubbm = nullptr;  // bit v set if the row of v is longer than kHubRow (n/32 + 2 words)
    // Walk entries, one aligned 16-byte record per CSR position e: (col[e], row start of
    // col[e], degree of col[e], 0).  A walk step reads one record at a random position and
    // gets its next vertex together with what the following step needs, so a step costs one
    // random sector instead of two (the vertex record, then the adjacency entry).
    int4 *nbr = nullptr;
    // reusable scratch of the synchronous calls
    DevBuf walk_scratch[12];
    // the walk call's second stream and its buffer hand-over events (walks done x2, counting
    // done x2), created on first use
    hipStream_t walk_aux = nullptr;
    hipEvent_t walk_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    Workspace est;
    // the synchronous estimator's second pool set and stream: the deterministic levels of one
    // batch run there while the walk pairs of the previous batch run on the caller's stream;
    // events: levels done x2, walk pairs done x2 (one per pool set), created on first use
    Workspace est2;
    hipStream_t est_aux = nullptr;
    hipEvent_t est_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    saba_exec_config cfg{};  // execution knobs (0 = default)
    // lambda of each graph computed on the device for requests that leave it to the library
    std::mutex lam_mu;
    std::vector<double> glambda;
    // the non-isolated vertices in ascending order (device), built on first use by the uniform
    // source mode of the walks
    std::mutex pool_mu;
    int32_t *pool = nullptr;
    int64_t npool = -1;
    // leading eigenpairs of graphs the estimator was asked to correct with (omega > 0)
    std::mutex spec_mu;
    std::vector<std::unique_ptr<struct Spectrum>> spectra;
};

// The omega nontrivial eigenpairs (theta_k, u_k) of N = D^-1/2 A D^-1/2 of largest |theta|
// that a Lanczos run found for one graph, and the radius of the rest of the spectrum.
struct Spectrum {
    int32_t graph = -1, omega = 0;  // request
    int32_t pairs = 0;              // pairs kept (omega, or fewer on an exhausted Krylov space)
    int32_t iterations = 0, converged = 0;
    double lambda_rest = 0.0, lambda_rest_bound = 0.0, max_residual = 0.0;
    std::vector<double> theta;      // host copy of the kept eigenvalues
    // device: theta[pairs], then y[pairs][gn] with y_k = u_k / sqrt(d) (the estimator's
    // correction reads y_k at both ends of an edge), then u[pairs][gn]
    DevBuf dev;
    const double *d_theta() const { return dev.as<double>(); }
    const double *d_y() const { return dev.as<double>() + pairs; }
    const double *d_u(int64_t gn) const { return dev.as<double>() + pairs + pairs * gn; }
};

// Rows longer than this are "hub rows": the estimator finds their terms through a bitmap
// over CSR positions instead of scanning them.
constexpr int32_t kHubRow = 256;

int check_graph(const saba_graph *g);

// Lanczos estimate of lambda for graph `graph` of the handle, and the cached upper estimate
// (lambda_bound, below 1) the estimator uses when a request passes lambda <= 0.
int graph_lambda(Graph *g, int32_t graph, int32_t max_iters, double tol, uint32_t seed,
                 saba_lambda_result *out, hipStream_t s);
int resolve_lambda(Graph *g, int32_t graph, double *lam, hipStream_t s);
// Leading eigenpairs of graph `graph` (Lanczos with full reorthogonalisation), and the cached
// set with the library's defaults that the estimator's correction uses for omega > 0.
constexpr int32_t kMaxOmega = 64;
int graph_spectrum(Graph *g, int32_t graph, int32_t omega, int32_t max_iters, double tol,
                   uint32_t seed, Spectrum *out, hipStream_t s);
int resolve_spectrum(Graph *g, int32_t graph, int32_t omega, const Spectrum **out, hipStream_t s);
inline Graph *G(saba_graph *g) { return reinterpret_cast<Graph *>(g); }
inline const Graph *G(const saba_graph *g) { return reinterpret_cast<const Graph *>(g); }

// Exclusive prefix sum of int64 values on the device: out[0] = 0, out[i] = sum in[0..i).
// out has n + 1 entries (out[n] = total).  tmp must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
int scan_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, hipStream_t s);

// ----------------------------------------------------------- device sampler
// MurmurHash2 (32-bit) over little-endian 32-bit words: multiplier 0x5bd1e995,
// rotation-free mixing with shift 24, seed XOR byte length, final avalanche
// (>>13, *m, >>15).  Only whole 32-bit words occur here.
constexpr uint32_t kMurmurM = 0x5bd1e995u;

__device__ __forceinline__ uint32_t mm2_block(uint32_t h, uint32_t k) {
    k *= kMurmurM;
    k ^= k >> 24;
    k *= kMurmurM;
    h *= kMurmurM;
    return h ^ k;
}

__device__ __forceinline__ uint32_t mm2_final(uint32_t h) {
    h ^= h >> 13;
    h *= kMurmurM;
    h ^= h >> 15;
    return h;
}

__device__ __forceinline__ uint32_t hash_w2(uint32_t a, uint32_t b, uint32_t seed) {
    uint32_t h = seed ^ 8u;
    h = mm2_block(h, a);
    h = mm2_block(h, b);
    return mm2_final(h);
}

__device__ __forceinline__ uint32_t hash_w4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                            uint32_t seed) {
    uint32_t h = seed ^ 16u;
    h = mm2_block(h, a);
    h = mm2_block(h, b);
    h = mm2_block(h, c);
    h = mm2_block(h, d);
    return mm2_final(h);
}

// Key of walk index k of address (a0, a1, a2) under grouping (G, S): the walks of a
// group share key_hi, and lane r = k mod G is written at bit S of key_lo.
struct WalkKey {
    uint32_t hi, lo;
};

__device__ __forceinline__ WalkKey walk_key(uint32_t seed, uint32_t a0, uint32_t a1, uint32_t a2,
                                            uint64_t k, uint32_t G, uint32_t S) {
    WalkKey key;
    if (G == 1) {
        key.hi = hash_w4(a0, a1, a2, (uint32_t)k, seed);
        key.lo = 0u;
    } else {
        uint64_t grp = k / G;
        uint32_t r = (uint32_t)(k - grp * G);
        key.hi = hash_w4(a0, a1, a2, (uint32_t)grp, seed);
        key.lo = r << S;
    }
    return key;
}

// One step (Eq. (5)): choose entry floor(u * d / 2^32) of the row of `cur`, where
// u = Murmur2(cur | l, key_hi) XOR key_lo and l is the position being filled.
__device__ __forceinline__ int32_t walk_step(const int2 *__restrict__ vrec,
                                             const int32_t *__restrict__ col, int32_t cur,
                                             uint32_t l, WalkKey key) {
    int2 r = vrec[cur];
    uint32_t u = hash_w2((uint32_t)cur, l, key.hi) ^ key.lo;
    uint32_t k = (uint32_t)(((uint64_t)u * (uint32_t)r.y) >> 32);
    return col[r.x + (int32_t)k];
}

// The same step for a graph stored at vertex offset goff of a multi-graph handle: the hash
// sees the graph's own vertex id, so the walk equals the one in the graph alone.
__device__ __forceinline__ int32_t walk_step_local(const int2 *__restrict__ vrec,
                                                   const int32_t *__restrict__ col, int32_t cur,
                                                   uint32_t l, WalkKey key, int32_t goff) {
    int2 r = vrec[cur];
    uint32_t u = hash_w2((uint32_t)(cur - goff), l, key.hi) ^ key.lo;
    uint32_t k = (uint32_t)(((uint64_t)u * (uint32_t)r.y) >> 32);
    return col[r.x + (int32_t)k];
}

// Samplers of the walk benchmark (SABA_SAMPLER_*).  A walker carries its key and, for the
// per-walk stream of Eq. (3), the generator state.
struct Walker {
    WalkKey key;
    uint32_t x;
};

template <int SM>
__device__ __forceinline__ Walker walker_init(WalkKey key) {
    Walker w;
    w.key = key;
    w.x = key.hi ^ key.lo;
    if (SM == SABA_SAMPLER_STREAM_MOD && w.x == 0u) w.x = 0x9E3779B9u;
    return w;
}

// One step with sampler SM: keyed Eq. (5) (multiply-high), keyed Eq. (4) (modulo), the
// Eq. (3) stream (Marsaglia's xorshift32, shifts 13 / 17 / 5, then modulo) or Eq. (5) read
// literally (unkeyed step hash XOR the walk's fixed seed, multiply-high).
template <int SM>
__device__ __forceinline__ uint32_t walker_choice(uint32_t cur, uint32_t d, uint32_t l,
                                                  Walker &w) {
    if (SM == SABA_SAMPLER_KEYED_MOD) return (hash_w2(cur, l, w.key.hi) ^ w.key.lo) % d;
    if (SM == SABA_SAMPLER_STREAM_MOD) {
        uint32_t x = w.x;
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        w.x = x;
        return x % d;
    }
    const uint32_t u = SM == SABA_SAMPLER_LITERAL
                           ? (w.key.hi ^ w.key.lo) ^ hash_w2(cur, l, 0u)
                           : hash_w2(cur, l, w.key.hi) ^ w.key.lo;
    return (uint32_t)(((uint64_t)u * d) >> 32);
}

template <int SM>
__device__ __forceinline__ int32_t walker_step(const int2 *__restrict__ vrec,
                                               const int32_t *__restrict__ col, int32_t cur,
                                               uint32_t l, Walker &w) {
    const int2 r = vrec[cur];
    return col[r.x + (int32_t)walker_choice<SM>((uint32_t)cur, (uint32_t)r.y, l, w)];
}

// A walk's position for the walk-entry layout: vertex, its row start and degree.
struct WalkPos {
    int32_t v, rs, d;
};

__device__ __forceinline__ WalkPos walk_pos(const int2 *__restrict__ vrec, int32_t v) {
    const int2 r = vrec[v];
    return WalkPos{v, r.x, r.y};
}

// One step on the walk entries (the same choice as walker_step); `hv` is the vertex id the
// hash sees (the graph-local id on a multi-graph handle).
template <int SM>
__device__ __forceinline__ WalkPos walker_step_nbr(const int4 *__restrict__ nbr, WalkPos p,
                                                   uint32_t hv, uint32_t l, Walker &w) {
    const int4 f = nbr[p.rs + (int32_t)walker_choice<SM>(hv, (uint32_t)p.d, l, w)];
    return WalkPos{f.x, f.y, f.z};
}

// The same step with the entry read marked non-temporal, so that the random entry stream does
// not push data with reuse (a source's support bitmap) out of the caches.
typedef int32_t nbr_vec4 __attribute__((ext_vector_type(4)));
template <int SM>
__device__ __forceinline__ WalkPos walker_step_nbr_nt(const int4 *__restrict__ nbr, WalkPos p,
                                                      uint32_t hv, uint32_t l, Walker &w) {
    const nbr_vec4 f = __builtin_nontemporal_load(
        reinterpret_cast<const nbr_vec4 *>(nbr) + p.rs +
        (int32_t)walker_choice<SM>(hv, (uint32_t)p.d, l, w));
    return WalkPos{f.x, f.y, f.z};
}

}  // namespace saba

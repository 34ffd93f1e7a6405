// Graph handle, validation, error reporting and the device prefix sum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "saba_internal.hpp"

namespace saba {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// Failure injection for tests of the error paths: when positive, the allocation that brings
// the count down to zero fails as an out-of-memory would.
static std::atomic<int64_t> g_fail_alloc{0};

int DevBuf::ensure(size_t want) {
    if (want <= bytes && ptr) return SABA_OK;
    const size_t grown = bytes + bytes / 4;
    release();
    int64_t c = g_fail_alloc.load(std::memory_order_relaxed);
    while (c > 0 && !g_fail_alloc.compare_exchange_weak(c, c - 1, std::memory_order_relaxed)) {
    }
    if (c == 1) {
        set_error("injected allocation failure");
        return SABA_E_NOMEM;
    }
    size_t sz = std::max<size_t>(std::max(want, grown), 256);
    hipError_t e = hipMalloc(&ptr, sz);
    if (e != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        set_error("device allocation of " + std::to_string(sz) + " bytes failed");
        return SABA_E_NOMEM;
    }
    bytes = sz;
    return SABA_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

int check_graph(const saba_graph *g) {
    if (!g) {
        set_error("graph handle is NULL");
        return SABA_E_INVALID;
    }
    return SABA_OK;
}

// ------------------------------------------------------------------ scan
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;

__global__ __launch_bounds__(kScanBlock) void scan_tile_kernel(const int64_t *__restrict__ in,
                                                               int64_t *__restrict__ out, int64_t n,
                                                               int64_t *__restrict__ tile_sums) {
    __shared__ int64_t sh[kScanBlock];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    int64_t v[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        sum += v[i];
    }
    sh[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int64_t t = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    int64_t run = sh[tid] - sum;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (tid == kScanBlock - 1) tile_sums[blockIdx.x] = sh[tid];
}

__global__ __launch_bounds__(kScanBlock) void scan_add_kernel(int64_t *__restrict__ out, int64_t n,
                                                              const int64_t *__restrict__ offs,
                                                              int64_t ntiles) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int64_t add = offs[blockIdx.x];
    for (int64_t i = base + threadIdx.x; i < base + kScanTile && i < n; i += kScanBlock) out[i] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = offs[ntiles];
}

size_t scan_tmp_bytes(int64_t n) {
    int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt <= 1) return 0;
    return (size_t)(2 * nt + 1) * sizeof(int64_t) + scan_tmp_bytes(nt);
}

int scan_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, hipStream_t s) {
    if (n <= 0) {
        SABA_HIP_TRY(hipMemsetAsync(out, 0, sizeof(int64_t), s));
        return SABA_OK;
    }
    int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 1) {
        scan_tile_kernel<<<1, kScanBlock, 0, s>>>(in, out, n, out + n);
        SABA_HIP_TRY(hipGetLastError());
        return SABA_OK;
    }
    int64_t *sums = static_cast<int64_t *>(tmp);
    int64_t *offs = sums + nt;
    void *rest = offs + nt + 1;
    scan_tile_kernel<<<(unsigned)nt, kScanBlock, 0, s>>>(in, out, n, sums);
    SABA_HIP_TRY(hipGetLastError());
    SABA_TRY(scan_i64(sums, offs, nt, rest, s));
    scan_add_kernel<<<(unsigned)nt, kScanBlock, 0, s>>>(out, n, offs, nt);
    SABA_HIP_TRY(hipGetLastError());
    return SABA_OK;
}

// ---------------------------------------------------------- graph kernels
__global__ void build_vrec_kernel(const int32_t *__restrict__ row_ptr, int32_t n,
                                  int2 *__restrict__ vrec, int32_t *__restrict__ row_of) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = row_ptr[v], b = row_ptr[v + 1];
        vrec[v] = make_int2(a, b - a);
        for (int32_t e = a; e < b; ++e) row_of[e] = (int32_t)v;
    }
}

// rev[e]: position of (t, s) in row t for the entry e = (s, t); rows are sorted.
__global__ void build_rev_kernel(const int32_t *__restrict__ row_ptr,
                                 const int32_t *__restrict__ col, const int32_t *__restrict__ row_of,
                                 int64_t nnz, int32_t *__restrict__ rev) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = row_of[e], t = col[e];
        int32_t lo = row_ptr[t], hi = row_ptr[t + 1];
        while (lo < hi) {
            int32_t mid = lo + ((hi - lo) >> 1);
            if (col[mid] < s)
                lo = mid + 1;
            else
                hi = mid;
        }
        rev[e] = lo;
    }
}

__global__ void build_slotv_kernel(const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
                                   const int32_t *__restrict__ rev, int64_t nnz,
                                   int32_t *__restrict__ slotv) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        slotv[e] = vrec[col[e]].y > kHubRow ? rev[e] : -1;
}

// Walk entries: nbr[e] = (col[e], row start of col[e], degree of col[e], 0).
__global__ void build_nbr_kernel(const int2 *__restrict__ vrec, const int32_t *__restrict__ col,
                                 int64_t nnz, int4 *__restrict__ nbr) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t y = col[e];
        const int2 r = vrec[y];
        nbr[e] = make_int4(y, r.x, r.y, 0);
    }
}

static int validate_host(const int32_t *rp, const int32_t *ci, int32_t n, int64_t nnz,
                         const std::vector<int32_t> &goff) {
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) {
        set_error("row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
        return SABA_E_GRAPH;
    }
    size_t gi = 0;
    for (int32_t v = 0; v < n; ++v) {
        while (v >= goff[gi + 1]) ++gi;
        if (rp[v + 1] < rp[v]) {
            set_error("row_ptr is not non-decreasing at vertex " + std::to_string(v));
            return SABA_E_GRAPH;
        }
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t t = ci[e];
            if (t < 0 || t >= n) {
                set_error("col_idx out of range at entry " + std::to_string(e));
                return SABA_E_GRAPH;
            }
            if (t == v) {
                set_error("self-loop at vertex " + std::to_string(v));
                return SABA_E_GRAPH;
            }
            if (t < goff[gi] || t >= goff[gi + 1]) {
                set_error("edge of vertex " + std::to_string(v) + " leaves its graph");
                return SABA_E_GRAPH;
            }
            if (e > rp[v] && ci[e - 1] >= t) {
                set_error("row " + std::to_string(v) + " is not strictly ascending");
                return SABA_E_GRAPH;
            }
            if (!std::binary_search(ci + rp[t], ci + rp[t + 1], v)) {
                set_error("graph is not symmetric: missing reverse of entry " + std::to_string(e));
                return SABA_E_GRAPH;
            }
        }
    }
    return SABA_OK;
}

static void graph_properties(Graph *g) {
    const int32_t n = g->n;
    const int32_t *rp = g->h_row_ptr.data();
    const int32_t *ci = g->h_col_idx.data();
    g->d_max = 0;
    g->n_isolated = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t d = rp[v + 1] - rp[v];
        g->d_max = std::max(g->d_max, d);
        g->n_isolated += d == 0;
    }
    // breadth-first search from the first vertex of each graph: connectivity, two-colouring
    std::vector<int8_t> color(n, -1);
    std::vector<int32_t> queue;
    queue.reserve(n);
    g->gconnected.assign(g->ngraphs, 0);
    g->gbipartite.assign(g->ngraphs, 0);
    for (int32_t k = 0; k < g->ngraphs; ++k) {
        const int32_t a = g->goff[k], z = g->goff[k + 1];
        if (a >= z) continue;
        queue.clear();
        color[a] = 0;
        queue.push_back(a);
        bool bip = true;
        for (size_t h = 0; h < queue.size(); ++h) {
            int32_t x = queue[h];
            for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
                int32_t y = ci[e];
                if (color[y] < 0) {
                    color[y] = (int8_t)(1 - color[x]);
                    queue.push_back(y);
                } else if (color[y] == color[x]) {
                    bip = false;
                }
            }
        }
        g->gconnected[k] = (int64_t)queue.size() == (int64_t)(z - a) ? 1 : 0;
        g->gbipartite[k] = (g->gconnected[k] && bip) ? 1 : 0;
    }
    g->connected = (g->ngraphs == 1 && n > 0) ? g->gconnected[0] : 0;
    g->bipartite = (g->ngraphs == 1 && n > 0) ? g->gbipartite[0] : 0;
    g->ghubs.assign(g->ngraphs, 0);
    for (int32_t k = 0; k < g->ngraphs; ++k)
        for (int32_t v = g->goff[k]; v < g->goff[k + 1]; ++v) g->ghubs[k] += rp[v + 1] - rp[v] > kHubRow;
}

static void destroy_graph(Graph *g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    if (g->row_ptr) (void)hipFree(g->row_ptr);
    if (g->col_idx) (void)hipFree(g->col_idx);
    if (g->vrec) (void)hipFree(g->vrec);
    if (g->rev) (void)hipFree(g->rev);
    if (g->canon) (void)hipFree(g->canon);
    if (g->row_of) (void)hipFree(g->row_of);
    if (g->slotv) (void)hipFree(g->slotv);
    if (g->hubbm) (void)hipFree(g->hubbm);
    if (g->nbr) (void)hipFree(g->nbr);
    if (g->pool) (void)hipFree(g->pool);
    for (auto &b : g->walk_scratch) b.release();
    for (auto &e : g->walk_ev)
        if (e) (void)hipEventDestroy(e);
    if (g->walk_aux) (void)hipStreamDestroy(g->walk_aux);
    g->est.release();
    g->est2.release();
    for (auto &e : g->est_ev)
        if (e) (void)hipEventDestroy(e);
    if (g->est_aux) (void)hipStreamDestroy(g->est_aux);
    for (auto &sp : g->spectra) sp->dev.release();
    delete g;
}

}  // namespace saba

using namespace saba;

extern "C" int saba_version(void) { return SABA_ABI_VERSION; }

extern "C" int saba_debug_fail_allocation(int32_t n) {
    clear_error();
    if (n < 0) {
        set_error("n must be >= 0");
        return SABA_E_INVALID;
    }
    g_fail_alloc.store(n, std::memory_order_relaxed);
    return SABA_OK;
}

extern "C" const char *saba_last_error(void) { return g_last_error.c_str(); }

static int create_impl(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int64_t nnz,
                       int32_t ngraphs, const int32_t *offsets, uint32_t flags, void *stream,
                       saba_graph **out) {
    if (!out) {
        set_error("out is NULL");
        return SABA_E_INVALID;
    }
    *out = nullptr;
    if (!row_ptr || (nnz > 0 && !col_idx) || n < 0 || nnz < 0 || nnz >= (1ll << 31)) {
        set_error("invalid CSR arguments");
        return SABA_E_INVALID;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        set_error("no HIP device");
        return SABA_E_NODEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error(std::string("library is built for gfx950, device is ") + prop.gcnArchName);
        return SABA_E_NODEVICE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Graph *g = new (std::nothrow) Graph();
    if (!g) {
        set_error("host allocation failed");
        return SABA_E_NOMEM;
    }
    g->device = dev;
    g->n = n;
    g->nnz = nnz;
    g->ngraphs = ngraphs;
    g->goff.assign(offsets, offsets + ngraphs + 1);
    try {
        g->h_row_ptr.resize((size_t)n + 1);
        g->h_col_idx.resize((size_t)nnz);
    } catch (...) {
        delete g;
        set_error("host allocation failed");
        return SABA_E_NOMEM;
    }
    int rc = SABA_OK;
    auto fail = [&](int code) {
        destroy_graph(g);
        return code;
    };
    if (flags & SABA_DEVICE_PTRS) {
        if (hipMemcpyAsync(g->h_row_ptr.data(), row_ptr, sizeof(int32_t) * ((size_t)n + 1),
                           hipMemcpyDeviceToHost, s) != hipSuccess ||
            (nnz > 0 && hipMemcpyAsync(g->h_col_idx.data(), col_idx, sizeof(int32_t) * (size_t)nnz,
                                       hipMemcpyDeviceToHost, s) != hipSuccess) ||
            hipStreamSynchronize(s) != hipSuccess) {
            (void)hipGetLastError();
            set_error("copy of device CSR to host failed");
            return fail(SABA_E_HIP);
        }
    } else {
        std::memcpy(g->h_row_ptr.data(), row_ptr, sizeof(int32_t) * ((size_t)n + 1));
        if (nnz > 0) std::memcpy(g->h_col_idx.data(), col_idx, sizeof(int32_t) * (size_t)nnz);
    }
    if (!(flags & SABA_TRUSTED)) {
        rc = validate_host(g->h_row_ptr.data(), g->h_col_idx.data(), n, nnz, g->goff);
        if (rc != SABA_OK) return fail(rc);
    }
    graph_properties(g);

    // canonical edge order: the entries (u, v) with u < v in CSR order
    std::vector<int32_t> canon;
    canon.reserve((size_t)(nnz / 2));
    g->cbase.assign(ngraphs + 1, 0);
    for (int32_t k = 0, u = 0; k < ngraphs; ++k) {
        g->cbase[k] = (int64_t)canon.size();
        for (; u < g->goff[k + 1]; ++u)
            for (int32_t e = g->h_row_ptr[u]; e < g->h_row_ptr[u + 1]; ++e)
                if (g->h_col_idx[e] > u) canon.push_back(e);
    }
    g->cbase[ngraphs] = (int64_t)canon.size();

    size_t nb = sizeof(int32_t) * std::max<int64_t>(nnz, 1);
    std::vector<uint32_t> hubbm((size_t)n / 32 + 2, 0u);
    for (int32_t v = 0; v < n; ++v)
        if (g->h_row_ptr[v + 1] - g->h_row_ptr[v] > kHubRow) hubbm[v >> 5] |= 1u << (v & 31);
    if (hipMalloc(&g->row_ptr, sizeof(int32_t) * ((size_t)n + 1)) != hipSuccess ||
        hipMalloc(&g->hubbm, sizeof(uint32_t) * hubbm.size()) != hipSuccess ||
        hipMalloc(&g->col_idx, nb) != hipSuccess ||
        hipMalloc(&g->vrec, sizeof(int2) * std::max<int32_t>(n, 1)) != hipSuccess ||
        hipMalloc(&g->rev, nb) != hipSuccess || hipMalloc(&g->row_of, nb) != hipSuccess ||
        hipMalloc(&g->slotv, nb) != hipSuccess ||
        hipMalloc(&g->nbr, sizeof(int4) * std::max<int64_t>(nnz, 1)) != hipSuccess ||
        hipMalloc(&g->canon, sizeof(int32_t) * std::max<size_t>(canon.size(), 1)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation for the graph failed");
        return fail(SABA_E_NOMEM);
    }
    if (hipMemcpyAsync(g->row_ptr, g->h_row_ptr.data(), sizeof(int32_t) * ((size_t)n + 1),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        (nnz > 0 && hipMemcpyAsync(g->col_idx, g->h_col_idx.data(), sizeof(int32_t) * (size_t)nnz,
                                   hipMemcpyHostToDevice, s) != hipSuccess) ||
        (!canon.empty() && hipMemcpyAsync(g->canon, canon.data(), sizeof(int32_t) * canon.size(),
                                          hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(g->hubbm, hubbm.data(), sizeof(uint32_t) * hubbm.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess) {
        (void)hipGetLastError();
        set_error("upload of the graph failed");
        return fail(SABA_E_HIP);
    }
    if (n > 0) {
        unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65535);
        build_vrec_kernel<<<blocks, 256, 0, s>>>(g->row_ptr, n, g->vrec, g->row_of);
    }
    if (nnz > 0) {
        unsigned blocks = (unsigned)std::min<int64_t>((nnz + 255) / 256, 1 << 20);
        build_rev_kernel<<<blocks, 256, 0, s>>>(g->row_ptr, g->col_idx, g->row_of, nnz, g->rev);
        build_slotv_kernel<<<blocks, 256, 0, s>>>(g->vrec, g->col_idx, g->rev, nnz, g->slotv);
        build_nbr_kernel<<<blocks, 256, 0, s>>>(g->vrec, g->col_idx, nnz, g->nbr);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("graph set-up kernels failed");
        return fail(SABA_E_HIP);
    }
    *out = reinterpret_cast<saba_graph *>(g);
    return SABA_OK;
}

extern "C" int saba_graph_create(const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                                 int64_t nnz, uint32_t flags, void *stream, saba_graph **out) {
    clear_error();
    const int32_t offsets[2] = {0, n};
    return create_impl(row_ptr, col_idx, n, nnz, 1, offsets, flags, stream, out);
}

extern "C" int saba_graph_create_multi(const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                                       int64_t nnz, int32_t ngraphs,
                                       const int32_t *vertex_offsets, uint32_t flags,
                                       void *stream, saba_graph **out) {
    clear_error();
    if (out) *out = nullptr;
    if (ngraphs < 1 || !vertex_offsets || vertex_offsets[0] != 0 || vertex_offsets[ngraphs] != n) {
        set_error("vertex_offsets must hold ngraphs + 1 entries from 0 to n");
        return SABA_E_INVALID;
    }
    for (int32_t k = 0; k < ngraphs; ++k)
        if (vertex_offsets[k + 1] < vertex_offsets[k]) {
            set_error("vertex_offsets must be non-decreasing");
            return SABA_E_INVALID;
        }
    return create_impl(row_ptr, col_idx, n, nnz, ngraphs, vertex_offsets, flags, stream, out);
}

extern "C" int saba_graph_destroy(saba_graph *g) {
    clear_error();
    destroy_graph(G(g));
    return SABA_OK;
}

extern "C" int saba_graph_info(const saba_graph *gh, saba_graph_info_t *out) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!out) {
        set_error("out is NULL");
        return SABA_E_INVALID;
    }
    const Graph *g = G(gh);
    out->n = g->n;
    out->nnz = g->nnz;
    out->m = g->nnz / 2;
    out->d_max = g->d_max;
    out->n_isolated = g->n_isolated;
    out->connected = g->connected;
    out->bipartite = g->bipartite;
    out->ngraphs = g->ngraphs;
    return SABA_OK;
}

extern "C" int saba_graph_get_config(const saba_graph *gh, saba_exec_config *out) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!out) {
        set_error("out is NULL");
        return SABA_E_INVALID;
    }
    *out = G(gh)->cfg;
    return SABA_OK;
}

extern "C" int saba_graph_set_config(saba_graph *gh, const saba_exec_config *cfg) {
    clear_error();
    SABA_TRY(check_graph(gh));
    if (!cfg || !(cfg->walks_per_lane == 0 || cfg->walks_per_lane == 1 ||
                  cfg->walks_per_lane == 2 || cfg->walks_per_lane == 4) ||
        cfg->walk_blocks < 0 || cfg->walk_blocks > (1 << 16) || cfg->est_walk_blocks < 0 ||
        cfg->est_walk_blocks > (1 << 16) || cfg->est_push_blocks < 0 ||
        cfg->est_push_blocks > (1 << 16) || cfg->walk_chunks < 0 || cfg->walk_chunks > 64 ||
        cfg->est_walk_queue < 0 || cfg->est_walk_queue > 2 || cfg->est_batch_streams < 0 ||
        cfg->est_batch_streams > 2) {
        set_error("invalid execution configuration");
        return SABA_E_INVALID;
    }
    G(gh)->cfg = *cfg;
    return SABA_OK;
}

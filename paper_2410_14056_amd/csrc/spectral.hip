// The estimator's spectral input on the device: lambda = max(|lambda_2|, |lambda_n|) of
// N = D^-1/2 A D^-1/2 (Sec. 2.2; the truncation length of Alg. 1's CalculateTau depends on it).
//
// N is symmetric with top eigenvalue 1 and eigenvector u1 = sqrt(d) / sqrt(2m) on a connected
// graph, so lambda is the spectral radius of N' = N - u1 u1^T.  A Lanczos iteration on N'
// (FP64, started from a hashed vector, u1 projected out after every product) builds the
// tridiagonal T_k; its extreme eigenvalues (Sturm bisection on the host) approach lambda_2 and
// lambda_n from inside the spectrum, and the residual of the extreme Ritz pairs
// (beta_{k+1} |last component of the Ritz vector|) bounds their distance to an eigenvalue.
// Every sum on the device runs in a fixed order, so the result depends only on the graph, the
// seed and the iteration count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "saba_internal.hpp"

namespace saba {
namespace {

constexpr int kBlk = 256;
constexpr int kDotBlocks = 512;  // fixed partition of every dot product

// s_i = 1 / sqrt(d_i), u1_i = sqrt(d_i) / sqrt(vol) over the graph's vertices.
__global__ void spec_init_kernel(const int2 *__restrict__ vrec, int32_t goff, int32_t gn,
                                 double vol, double *__restrict__ sc, double *__restrict__ u1) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x) {
        const double d = (double)vrec[goff + i].y;
        sc[i] = 1.0 / sqrt(d);
        u1[i] = sqrt(d) / sqrt(vol);
    }
}

// Start vector: MurmurHash2-style finaliser of (i, seed) mapped to [-1, 1).
__global__ void spec_start_kernel(int32_t gn, uint32_t seed, double *__restrict__ v) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x) {
        uint32_t h = seed ^ 8u;
        h = mm2_block(h, (uint32_t)i);
        h = mm2_block(h, 0x2545F491u);
        h = mm2_final(h);
        v[i] = (double)h * (2.0 / 4294967296.0) - 1.0;
    }
}

// z = s o x
__global__ void spec_scale_kernel(int32_t gn, const double *__restrict__ sc,
                                  const double *__restrict__ x, double *__restrict__ z) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x)
        z[i] = sc[i] * x[i];
}

// y_i = s_i * sum_{j in Gamma(i)} z_j for ordinary rows (one lane per row, CSR order).
__global__ void spec_spmv_rows_kernel(const int2 *__restrict__ vrec,
                                      const int32_t *__restrict__ col, int32_t goff, int32_t gn,
                                      const double *__restrict__ sc, const double *__restrict__ z,
                                      double *__restrict__ y) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x) {
        const int2 r = vrec[goff + i];
        if (r.y > kHubRow) continue;
        double acc = 0.0;
        for (int32_t e = r.x; e < r.x + r.y; ++e) acc += z[col[e] - goff];
        y[i] = sc[i] * acc;
    }
}

// Hub rows: one wavefront per row; lane l adds entries l, l + 64, ... in order, then lane 0's
// butterfly combines the lanes.
__global__ void spec_spmv_hubs_kernel(const int2 *__restrict__ vrec,
                                      const int32_t *__restrict__ col, int32_t goff,
                                      const int32_t *__restrict__ hubs, int32_t nh,
                                      const double *__restrict__ sc, const double *__restrict__ z,
                                      double *__restrict__ y) {
    const int lane = __lane_id();
    const int32_t nw = gridDim.x * (blockDim.x / 64);
    for (int32_t k = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * (blockDim.x / 64) +
                                                              (threadIdx.x >> 6)));
         k < nh; k += nw) {
        const int32_t i = hubs[k];
        const int2 r = vrec[goff + i];
        double acc = 0.0;
        for (int32_t e = r.x + lane; e < r.x + r.y; e += 64) acc += z[col[e] - goff];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        acc = __shfl(acc, 0);
        if (lane == 0) y[i] = sc[i] * acc;
    }
}

// Fixed-partition dot product: block b sums its contiguous range (thread-strided, then a tree
// over the block), the final kernel adds the block sums in order.
__global__ __launch_bounds__(kBlk) void spec_dot_kernel(int32_t gn, const double *__restrict__ a,
                                                        const double *__restrict__ b,
                                                        double *__restrict__ part) {
    __shared__ double red[kBlk];
    const int32_t chunk = (gn + kDotBlocks - 1) / kDotBlocks;
    const int32_t lo = blockIdx.x * chunk, hi = min(gn, lo + chunk);
    double acc = 0.0;
    for (int32_t i = lo + threadIdx.x; i < hi; i += kBlk) acc += a[i] * b[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kBlk / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void spec_dot_final_kernel(const double *__restrict__ part, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double acc = 0.0;
        for (int k = 0; k < kDotBlocks; ++k) acc += part[k];
        *out = acc;
    }
}

// x = x - (*c) * u  (c read on the device)
__global__ void spec_axpy_dev_kernel(int32_t gn, const double *__restrict__ c,
                                     const double *__restrict__ u, double *__restrict__ x) {
    const double cv = *c;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x)
        x[i] -= cv * u[i];
}

// Lanczos update: w = w - alpha v - beta vprev (alpha, beta read on the device).
__global__ void spec_lanczos_update_kernel(int32_t gn, const double *__restrict__ alpha,
                                           const double *__restrict__ beta,
                                           const double *__restrict__ v,
                                           const double *__restrict__ vprev,
                                           double *__restrict__ w) {
    const double a = *alpha, b = *beta;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x)
        w[i] = w[i] - a * v[i] - b * vprev[i];
}

// beta_next = sqrt(ww); v_next = w / beta_next.  A beta_next below 1e-12 (the Lanczos vectors
// have unit norm and |N'| <= 1) means the Krylov space is exhausted: beta_next and v_next are
// set to 0, so every later step adds a decoupled zero row to T.
__global__ void spec_normalize_kernel(int32_t gn, const double *__restrict__ ww,
                                      double *__restrict__ beta_next, const double *__restrict__ w,
                                      double *__restrict__ vnext) {
    const double raw = sqrt(fmax(*ww, 0.0));
    const double nb = raw > 1e-12 ? raw : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *beta_next = nb;
    const double inv = nb > 0.0 ? 1.0 / nb : 0.0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x)
        vnext[i] = w[i] * inv;
}

// ---------------------------------------------------------------- host: tridiagonal
// Number of eigenvalues of T (diagonal a[0..k), off-diagonal b[1..k)) below x (Sturm count).
int sturm_below(const std::vector<double> &a, const std::vector<double> &b, int k, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        const double off = i > 0 ? b[i] * b[i] : 0.0;
        q = a[i] - x - (i > 0 ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// The j-th smallest eigenvalue of T (0-based) by bisection on the Gershgorin interval.
double tri_eig(const std::vector<double> &a, const std::vector<double> &b, int k, int j) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < k ? std::fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_below(a, b, k, mid) > j)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for eigenvalue theta (inverse iteration).
double tri_last_component(const std::vector<double> &a, const std::vector<double> &b, int k,
                          double theta) {
    std::vector<double> x(k, 1.0), c(k), d(k), y(k);
    const double shift = theta + 1e-13 * std::max(1.0, std::fabs(theta));
    for (int rep = 0; rep < 3; ++rep) {
        // solve (T - shift I) y = x with the Thomas algorithm (no pivoting; shift off the
        // spectrum keeps it stable enough for an eigenvector estimate)
        for (int i = 0; i < k; ++i) {
            const double diag = a[i] - shift - (i > 0 ? b[i] * c[i - 1] : 0.0);
            const double dg = diag == 0.0 ? 1e-300 : diag;
            c[i] = (i + 1 < k) ? b[i + 1] / dg : 0.0;
            d[i] = (x[i] - (i > 0 ? b[i] * d[i - 1] : 0.0)) / dg;
        }
        for (int i = k - 1; i >= 0; --i) y[i] = d[i] - (i + 1 < k ? c[i] * y[i + 1] : 0.0);
        double nrm = 0.0;
        for (double v : y) nrm += v * v;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return 1.0;
        for (int i = 0; i < k; ++i) x[i] = y[i] / nrm;
    }
    return std::fabs(x[k - 1]);
}

}  // namespace

int graph_lambda(Graph *g, int32_t graph, int32_t max_iters, double tol, uint32_t seed,
                 saba_lambda_result *out, hipStream_t s) {
    const int32_t *rp = g->h_row_ptr.data();
    const int32_t goff = g->goff[graph], gn = g->goff[graph + 1] - goff;
    const double vol = (double)((int64_t)rp[goff + gn] - rp[goff]);
    if (!g->gconnected[graph] || gn < 2) {
        set_error("lambda needs a connected graph with at least one edge");
        return SABA_E_DISCONNECTED;
    }
    const int K = std::max(4, std::min(max_iters, gn - 1));
    std::vector<int32_t> hubs;
    for (int32_t i = 0; i < gn; ++i)
        if (rp[goff + i + 1] - rp[goff + i] > kHubRow) hubs.push_back(i);
    // device scratch: sc, u1, three Lanczos vectors, z, y, dot partials, scalars
    DevBuf buf;
    const size_t nvec = 6;
    const size_t bytes = sizeof(double) * ((size_t)gn * nvec + kDotBlocks + 8 + 2 * (size_t)K + 4) +
                         sizeof(int32_t) * std::max<size_t>(hubs.size(), 1);
    SABA_TRY(buf.ensure(bytes));
    struct Guard {
        DevBuf *b;
        ~Guard() { b->release(); }
    } guard{&buf};
    double *sc = buf.as<double>(), *u1 = sc + gn, *vprev = u1 + gn, *v = vprev + gn,
           *w = v + gn, *z = w + gn;
    double *part = z + gn, *scal = part + kDotBlocks;  // scal[0]: the last dot product
    double *alpha = scal + 8, *beta = alpha + K + 2;   // beta[j]: off-diagonal before v_j
    int32_t *d_hubs = reinterpret_cast<int32_t *>(beta + K + 2);
    const unsigned grid = (unsigned)std::min<int64_t>((gn + kBlk - 1) / kBlk, 4096);
    SABA_HIP_TRY(hipMemsetAsync(scal, 0, sizeof(double) * (8 + 2 * (size_t)K + 4), s));
    if (!hubs.empty())
        SABA_HIP_TRY(hipMemcpyAsync(d_hubs, hubs.data(), sizeof(int32_t) * hubs.size(),
                                    hipMemcpyHostToDevice, s));
    SABA_HIP_TRY(hipMemsetAsync(vprev, 0, sizeof(double) * gn, s));
    spec_init_kernel<<<grid, kBlk, 0, s>>>(g->vrec, goff, gn, vol, sc, u1);
    spec_start_kernel<<<grid, kBlk, 0, s>>>(gn, seed, w);
    auto dot = [&](const double *a, const double *b, double *dst) {
        spec_dot_kernel<<<kDotBlocks, kBlk, 0, s>>>(gn, a, b, part);
        spec_dot_final_kernel<<<1, 64, 0, s>>>(part, dst);
    };
    // w = start - u1 (u1 . start); v = w / |w|
    dot(u1, w, scal);
    spec_axpy_dev_kernel<<<grid, kBlk, 0, s>>>(gn, scal, u1, w);
    dot(w, w, scal);
    spec_normalize_kernel<<<grid, kBlk, 0, s>>>(gn, scal, beta + 0, w, v);
    SABA_HIP_TRY(hipGetLastError());

    std::vector<double> ha(K + 2), hb(K + 2);
    double th_max = 0.0, th_min = 0.0, prev_max = 2.0, prev_min = 2.0;
    int k = 0;
    bool converged = false, exhausted = false;
    const int check = 10;
    for (int j = 0; j < K; ++j) {
        // w = N' v = N v - u1 (u1 . N v)
        spec_scale_kernel<<<grid, kBlk, 0, s>>>(gn, sc, v, z);
        spec_spmv_rows_kernel<<<grid, kBlk, 0, s>>>(g->vrec, g->col_idx, goff, gn, sc, z, w);
        if (!hubs.empty())
            spec_spmv_hubs_kernel<<<std::min<int>(1024, ((int)hubs.size() + 3) / 4), kBlk, 0, s>>>(
                g->vrec, g->col_idx, goff, d_hubs, (int32_t)hubs.size(), sc, z, w);
        dot(u1, w, scal);
        spec_axpy_dev_kernel<<<grid, kBlk, 0, s>>>(gn, scal, u1, w);
        // alpha_j = w . v ; w = w - alpha_j v - beta_j vprev
        dot(w, v, alpha + j);
        spec_lanczos_update_kernel<<<grid, kBlk, 0, s>>>(gn, alpha + j, beta + j, v, vprev, w);
        dot(w, w, scal);
        // rotate: vprev <- v, v <- w / beta_{j+1}
        std::swap(vprev, v);
        spec_normalize_kernel<<<grid, kBlk, 0, s>>>(gn, scal, beta + j + 1, w, v);
        SABA_HIP_TRY(hipGetLastError());
        k = j + 1;
        if (k % check == 0 || k == K) {
            SABA_HIP_TRY(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * k, hipMemcpyDeviceToHost, s));
            SABA_HIP_TRY(hipMemcpyAsync(hb.data(), beta, sizeof(double) * (k + 1),
                                        hipMemcpyDeviceToHost, s));
            SABA_HIP_TRY(hipStreamSynchronize(s));
            int kb = k;  // leading block of T before the first vanished off-diagonal
            for (int i = 1; i <= k; ++i)
                if (hb[i] == 0.0) {
                    kb = i;
                    break;
                }
            th_max = tri_eig(ha, hb, kb, kb - 1);
            th_min = tri_eig(ha, hb, kb, 0);
            if (kb < k || hb[k] == 0.0) {  // an invariant subspace: the block is exact
                exhausted = true;
                k = kb;
                break;
            }
            if (std::fabs(th_max - prev_max) <= tol && std::fabs(th_min - prev_min) <= tol) {
                converged = true;
                break;
            }
            prev_max = th_max;
            prev_min = th_min;
        }
    }
    const double bk = hb[k];
    const double rmax = exhausted ? 0.0 : bk * tri_last_component(ha, hb, k, th_max);
    const double rmin = exhausted ? 0.0 : bk * tri_last_component(ha, hb, k, th_min);
    saba_lambda_result r{};
    r.lambda2 = th_max;
    r.lambdan = th_min;
    r.lambda = std::max(std::fabs(th_max), std::fabs(th_min));
    r.residual = std::max(rmax, rmin);
    r.lambda_bound = std::max(std::fabs(th_max) + rmax, std::fabs(th_min) + rmin);
    r.iterations = k;
    r.converged = (converged || exhausted) ? 1 : 0;
    *out = r;
    return SABA_OK;
}

int resolve_lambda(Graph *g, int32_t graph, double *lam, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(g->lam_mu);
        if (g->glambda.size() == (size_t)g->ngraphs && g->glambda[graph] > 0.0) {
            *lam = g->glambda[graph];
            return SABA_OK;
        }
    }
    if (graph < 0 || graph >= g->ngraphs) {
        set_error("request names a graph the handle does not hold");
        return SABA_E_INVALID;
    }
    if (g->gbipartite[graph]) {
        set_error("the estimator needs a non-bipartite graph (lambda < 1)");
        return SABA_E_BIPARTITE;
    }
    saba_lambda_result r{};
    SABA_TRY(graph_lambda(g, graph, 300, 1e-12, 1u, &r, s));
    const double v = std::min(r.lambda_bound, 1.0 - 1e-12);
    std::lock_guard<std::mutex> lk(g->lam_mu);
    if (g->glambda.size() != (size_t)g->ngraphs) g->glambda.assign(g->ngraphs, 0.0);
    g->glambda[graph] = v;
    *lam = v;
    return SABA_OK;
}

}  // namespace saba

using namespace saba;

extern "C" int saba_graph_lambda(saba_graph *gh, const saba_lambda_params *p,
                                 saba_lambda_result *out, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    Graph *g = G(gh);
    saba_lambda_params q{};
    if (p) q = *p;
    if (!out || q.graph < 0 || q.graph >= g->ngraphs || q.max_iters < 0 || q.tol < 0.0) {
        set_error("invalid lambda arguments");
        return SABA_E_INVALID;
    }
    const int32_t iters = q.max_iters > 0 ? q.max_iters : 300;
    const double tol = q.tol > 0.0 ? q.tol : 1e-12;
    return graph_lambda(g, q.graph, iters, tol, q.seed, out, static_cast<hipStream_t>(stream));
}

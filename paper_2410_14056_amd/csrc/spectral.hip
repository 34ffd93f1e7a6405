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


// Partial sums of h = V[0..nk)^T w over the fixed partition: block (b, k) sums block b's range
// of V[k] o w (thread-strided, then a tree over the block).
__global__ __launch_bounds__(kBlk) void spec_mdot_kernel(int32_t gn, const double *__restrict__ V,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ part) {
    __shared__ double red[kBlk];
    const double *a = V + (int64_t)blockIdx.y * gn;
    const int32_t chunk = (gn + kDotBlocks - 1) / kDotBlocks;
    const int32_t lo = blockIdx.x * chunk, hi = min(gn, lo + chunk);
    double acc = 0.0;
    for (int32_t i = lo + threadIdx.x; i < hi; i += kBlk) acc += a[i] * w[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kBlk / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * kDotBlocks + blockIdx.x] = red[0];
}

// h[k] = sum of block k's partials in order (one block per k).
__global__ void spec_mdot_final_kernel(const double *__restrict__ part, double *__restrict__ h) {
    if (threadIdx.x == 0) {
        const double *p = part + (int64_t)blockIdx.x * kDotBlocks;
        double acc = 0.0;
        for (int b = 0; b < kDotBlocks; ++b) acc += p[b];
        h[blockIdx.x] = acc;
    }
}

// w = w - sum_{k < nk} h[k] V[k], the terms taken in order of k.
__global__ void spec_mupdate_kernel(int32_t gn, const double *__restrict__ V, int32_t nk,
                                    const double *__restrict__ h, double *__restrict__ w) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x) {
        double acc = w[i];
        for (int32_t k = 0; k < nk; ++k) acc -= h[k] * V[(int64_t)k * gn + i];
        w[i] = acc;
    }
}

// Ritz vectors: U[p] = sum_{j < k} S[p][j] V[j] (terms in order of j).
__global__ void spec_ritz_kernel(int32_t gn, const double *__restrict__ V, int32_t k,
                                 const double *__restrict__ S, double *__restrict__ U) {
    const double *sp = S + (int64_t)blockIdx.y * k;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int32_t j = 0; j < k; ++j) acc += sp[j] * V[(int64_t)j * gn + i];
        U[(int64_t)blockIdx.y * gn + i] = acc;
    }
}

// x = x / sqrt(*nn)
__global__ void spec_unit_kernel(int32_t gn, const double *__restrict__ nn, double *__restrict__ x) {
    const double inv = 1.0 / sqrt(*nn);
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x)
        x[i] *= inv;
}

// x = x - c u  (c from the host)
__global__ void spec_axpy_kernel(int32_t gn, double c, const double *__restrict__ u,
                                 double *__restrict__ x) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < gn; i += gridDim.x * blockDim.x)
        x[i] -= c * u[i];
}

// Unit eigenvector of T (diagonal a[0..k), off-diagonal b[1..k)) for the eigenvalue theta:
// inverse iteration with T - shift I factored by Gaussian elimination with partial pivoting
// (rows keep at most two entries right of the diagonal).  Empty on failure.
std::vector<double> tri_eigvec(const std::vector<double> &a, const std::vector<double> &b, int k,
                               double theta) {
    const double shift = theta + 1e-14 * std::max(1.0, std::fabs(theta));
    std::vector<double> D(k), U1(k, 0.0), U2(k, 0.0), L(k, 0.0);
    std::vector<uint8_t> swp(k, 0);
    double cd = a[0] - shift, cu1 = k > 1 ? b[1] : 0.0, cu2 = 0.0;
    for (int i = 0; i < k; ++i) {
        if (i == k - 1) {
            D[i] = cd;
            break;
        }
        const double nl = b[i + 1], nd = a[i + 1] - shift, nu = i + 2 < k ? b[i + 2] : 0.0;
        if (std::fabs(cd) >= std::fabs(nl)) {
            const double m = cd != 0.0 ? nl / cd : 0.0;
            D[i] = cd;
            U1[i] = cu1;
            U2[i] = cu2;
            L[i] = m;
            cd = nd - m * cu1;
            cu1 = nu - m * cu2;
        } else {
            const double m = cd / nl;
            swp[i] = 1;
            D[i] = nl;
            U1[i] = nd;
            U2[i] = nu;
            L[i] = m;
            cd = cu1 - m * nd;
            cu1 = cu2 - m * nu;
        }
        cu2 = 0.0;
    }
    double tiny = 0.0;
    for (int i = 0; i < k; ++i) tiny = std::max(tiny, std::fabs(a[i]) + std::fabs(b[i]));
    tiny = std::max(tiny, 1.0) * 1e-300;
    for (int i = 0; i < k; ++i)
        if (D[i] == 0.0) D[i] = tiny;
    std::vector<double> x(k), r(k);
    for (int i = 0; i < k; ++i) x[i] = 1.0 + 0.125 * (double)((i * 7) % 11);
    for (int rep = 0; rep < 4; ++rep) {
        r = x;
        for (int i = 0; i + 1 < k; ++i) {
            if (swp[i]) std::swap(r[i], r[i + 1]);
            r[i + 1] -= L[i] * r[i];
        }
        for (int i = k - 1; i >= 0; --i) {
            double v = r[i];
            if (i + 1 < k) v -= U1[i] * x[i + 1];
            if (i + 2 < k) v -= U2[i] * x[i + 2];
            x[i] = v / D[i];
        }
        double nrm = 0.0, big = 0.0;
        for (double v : x) big = std::max(big, std::fabs(v));
        if (!(big > 0.0) || !std::isfinite(big)) return {};
        for (double &v : x) v /= big;  // rescale before squaring
        for (double v : x) nrm += v * v;
        nrm = std::sqrt(nrm);
        for (double &v : x) v /= nrm;
    }
    return x;
}

// The m Ritz values of T (order k) of largest |theta|, by decreasing |theta| (ties: the
// positive one first): the candidates are the m smallest and the m largest eigenvalues.
std::vector<double> top_ritz(const std::vector<double> &a, const std::vector<double> &b, int k,
                             int m) {
    m = std::min(m, k);
    std::vector<int> idx;
    for (int i = 0; i < m; ++i) {
        idx.push_back(i);
        idx.push_back(k - 1 - i);
    }
    std::sort(idx.begin(), idx.end());
    idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
    std::vector<double> th;
    for (int j : idx) th.push_back(tri_eig(a, b, k, j));
    std::sort(th.begin(), th.end(), [](double x, double y) {
        return std::fabs(x) != std::fabs(y) ? std::fabs(x) > std::fabs(y) : x > y;
    });
    th.resize(m);
    return th;
}

// The operator N' = N - u1 u1^T of one graph of the handle and the scratch of its products:
// s = 1/sqrt(d), u1, a product vector z, dot-product partials and a few device scalars.
struct SpecOp {
    Graph *g = nullptr;
    int32_t goff = 0, gn = 0;
    double vol = 0.0;
    hipStream_t s = nullptr;
    unsigned grid = 1;
    DevBuf buf;
    double *sc = nullptr, *u1 = nullptr, *z = nullptr, *part = nullptr, *scal = nullptr;
    int32_t *d_hubs = nullptr;
    int32_t nh = 0;
    ~SpecOp() { buf.release(); }

    int init(Graph *gr, int32_t graph, hipStream_t st) {
        g = gr;
        s = st;
        const int32_t *rp = g->h_row_ptr.data();
        goff = g->goff[graph];
        gn = g->goff[graph + 1] - goff;
        vol = (double)((int64_t)rp[goff + gn] - rp[goff]);
        if (!g->gconnected[graph] || gn < 2) {
            set_error("the spectrum needs a connected graph with at least one edge");
            return SABA_E_DISCONNECTED;
        }
        std::vector<int32_t> hubs;
        for (int32_t i = 0; i < gn; ++i)
            if (rp[goff + i + 1] - rp[goff + i] > kHubRow) hubs.push_back(i);
        nh = (int32_t)hubs.size();
        const size_t bytes = sizeof(double) * ((size_t)gn * 3 + kDotBlocks + 8) +
                             sizeof(int32_t) * std::max<size_t>(hubs.size(), 1);
        SABA_TRY(buf.ensure(bytes));
        sc = buf.as<double>();
        u1 = sc + gn;
        z = u1 + gn;
        part = z + gn;
        scal = part + kDotBlocks;
        d_hubs = reinterpret_cast<int32_t *>(scal + 8);
        grid = (unsigned)std::min<int64_t>((gn + kBlk - 1) / kBlk, 4096);
        SABA_HIP_TRY(hipMemsetAsync(scal, 0, sizeof(double) * 8, s));
        if (nh)
            SABA_HIP_TRY(hipMemcpyAsync(d_hubs, hubs.data(), sizeof(int32_t) * hubs.size(),
                                        hipMemcpyHostToDevice, s));
        spec_init_kernel<<<grid, kBlk, 0, s>>>(g->vrec, goff, gn, vol, sc, u1);
        SABA_HIP_TRY(hipGetLastError());
        return SABA_OK;
    }
    void dot(const double *a, const double *b, double *dst) const {
        spec_dot_kernel<<<kDotBlocks, kBlk, 0, s>>>(gn, a, b, part);
        spec_dot_final_kernel<<<1, 64, 0, s>>>(part, dst);
    }
    // w = w - u (u . w)
    void project(const double *u, double *w) const {
        dot(u, w, scal);
        spec_axpy_dev_kernel<<<grid, kBlk, 0, s>>>(gn, scal, u, w);
    }
    // w = N v - u1 (u1 . N v)
    void apply(const double *v, double *w) const {
        spec_scale_kernel<<<grid, kBlk, 0, s>>>(gn, sc, v, z);
        spec_spmv_rows_kernel<<<grid, kBlk, 0, s>>>(g->vrec, g->col_idx, goff, gn, sc, z, w);
        if (nh)
            spec_spmv_hubs_kernel<<<std::min<int>(1024, (nh + 3) / 4), kBlk, 0, s>>>(
                g->vrec, g->col_idx, goff, d_hubs, nh, sc, z, w);
        project(u1, w);
    }
};

// Lanczos without reorthogonalisation on N' restricted to the complement of `nx` further unit
// vectors x[nx][gn] (projected out of the start vector and of every product after u1): the
// extreme Ritz values, their residuals and the bound max(|theta| + residual).
int lanczos_extremes(const SpecOp &op, const double *x, int32_t nx, int32_t max_iters,
                     double tol, uint32_t seed, saba_lambda_result *out) {
    const int32_t gn = op.gn;
    const hipStream_t s = op.s;
    const int K = std::max(4, std::min(max_iters, gn - 1));
    DevBuf buf;
    // vectors, the tridiagonal coefficients, and the partial and final dots of the projection
    // against x
    const size_t nxd = nx > 0 ? (size_t)nx * (kDotBlocks + 1) : 0;
    SABA_TRY(buf.ensure(sizeof(double) * ((size_t)gn * 3 + 2 * (size_t)K + 4 + nxd)));
    struct Guard {
        DevBuf *b;
        ~Guard() { b->release(); }
    } guard{&buf};
    double *vprev = buf.as<double>(), *v = vprev + gn, *w = v + gn;
    double *alpha = w + gn, *beta = alpha + K + 2;  // beta[j]: off-diagonal before v_j
    double *xpart = beta + K + 2, *xh = xpart + (size_t)nx * kDotBlocks;
    SABA_HIP_TRY(hipMemsetAsync(alpha, 0, sizeof(double) * (2 * (size_t)K + 4), s));
    SABA_HIP_TRY(hipMemsetAsync(vprev, 0, sizeof(double) * gn, s));
    const unsigned grid = op.grid;
    // y = y - X (X^T y), twice (classical Gram-Schmidt with one reorthogonalisation pass):
    // the nx dots in one launch, the update in another, instead of nx sequential projections
    auto project_x = [&](double *y) {
        if (nx <= 0) return;
        for (int rep = 0; rep < 2; ++rep) {
            spec_mdot_kernel<<<dim3(kDotBlocks, nx), kBlk, 0, s>>>(gn, x, y, xpart);
            spec_mdot_final_kernel<<<nx, 64, 0, s>>>(xpart, xh);
            spec_mupdate_kernel<<<grid, kBlk, 0, s>>>(gn, x, nx, xh, y);
        }
    };
    auto deflate = [&](double *y) {
        op.project(op.u1, y);
        project_x(y);
    };
    // w = start with u1 (and x) projected out; v = w / |w|
    spec_start_kernel<<<grid, kBlk, 0, s>>>(gn, seed, w);
    deflate(w);
    op.dot(w, w, op.scal);
    spec_normalize_kernel<<<grid, kBlk, 0, s>>>(gn, op.scal, beta + 0, w, v);
    SABA_HIP_TRY(hipGetLastError());

    std::vector<double> ha(K + 2), hb(K + 2);
    double th_max = 0.0, th_min = 0.0, prev_max = 2.0, prev_min = 2.0;
    int k = 0;
    bool converged = false, exhausted = false;
    const int check = 10;
    for (int j = 0; j < K; ++j) {
        // w = N' v with x projected out
        op.apply(v, w);
        project_x(w);
        // alpha_j = w . v ; w = w - alpha_j v - beta_j vprev
        op.dot(w, v, alpha + j);
        spec_lanczos_update_kernel<<<grid, kBlk, 0, s>>>(gn, alpha + j, beta + j, v, vprev, w);
        op.dot(w, w, op.scal);
        // rotate: vprev <- v, v <- w / beta_{j+1}
        std::swap(vprev, v);
        spec_normalize_kernel<<<grid, kBlk, 0, s>>>(gn, op.scal, beta + j + 1, w, v);
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

}  // namespace

int graph_lambda(Graph *g, int32_t graph, int32_t max_iters, double tol, uint32_t seed,
                 saba_lambda_result *out, hipStream_t s) {
    SpecOp op;
    SABA_TRY(op.init(g, graph, s));
    return lanczos_extremes(op, nullptr, 0, max_iters, tol, seed, out);
}

int graph_spectrum(Graph *g, int32_t graph, int32_t omega, int32_t max_iters, double tol,
                   uint32_t seed, Spectrum *out, hipStream_t s) {
    SpecOp op;
    SABA_TRY(op.init(g, graph, s));
    const int32_t gn = op.gn;
    if (omega < 1 || omega > kMaxOmega || omega >= gn) {
        set_error("omega must lie in [1, 64] and below the vertex count of the graph");
        return SABA_E_INVALID;
    }
    // the basis V[0..K] takes (K + 1) gn doubles: at most 32 GiB and half of free memory
    size_t freeb = 0, totalb = 0;
    SABA_HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    const int64_t room = std::min<int64_t>(32ll << 30, (int64_t)(freeb / 2));
    const int64_t kfit = room / (int64_t)(sizeof(double) * (size_t)gn) - 1;
    const int32_t K = (int32_t)std::min<int64_t>(std::min({max_iters, gn - 1, 16384}), kfit);
    if (K < std::min(gn - 1, 2 * omega + 2)) {
        set_error("not enough device memory for the Lanczos basis");
        return SABA_E_NOMEM;
    }
    DevBuf buf;
    const size_t nV = (size_t)(K + 1) * gn;
    SABA_TRY(buf.ensure(sizeof(double) * (nV + 2 * (size_t)gn + 3 * ((size_t)K + 2) +
                                          (size_t)(K + 1) * kDotBlocks)));
    struct Guard {
        DevBuf *b;
        ~Guard() { b->release(); }
    } guard{&buf};
    double *V = buf.as<double>(), *w = V + nV, *zero = w + gn;
    double *alpha = zero + gn, *beta = alpha + K + 2, *h = beta + K + 2, *mpart = h + K + 2;
    const unsigned grid = op.grid;
    SABA_HIP_TRY(hipMemsetAsync(zero, 0, sizeof(double) * (gn + 3 * ((size_t)K + 2)), s));
    // V[0] = start with u1 projected out, normalised
    spec_start_kernel<<<grid, kBlk, 0, s>>>(gn, seed, w);
    op.project(op.u1, w);
    op.dot(w, w, op.scal);
    spec_normalize_kernel<<<grid, kBlk, 0, s>>>(gn, op.scal, beta + 0, w, V);
    SABA_HIP_TRY(hipGetLastError());

    std::vector<double> ha(K + 2), hb(K + 2);
    int k = 0, kb = 0;
    const int check = 5;
    for (int j = 0; j < K; ++j) {
        double *vj = V + (size_t)j * gn;
        const double *vp = j > 0 ? vj - gn : zero;
        op.apply(vj, w);
        op.dot(w, vj, alpha + j);
        spec_lanczos_update_kernel<<<grid, kBlk, 0, s>>>(gn, alpha + j, beta + j, vj, vp, w);
        // full reorthogonalisation against V[0..j], twice
        for (int rep = 0; rep < 2; ++rep) {
            spec_mdot_kernel<<<dim3(kDotBlocks, j + 1), kBlk, 0, s>>>(gn, V, w, mpart);
            spec_mdot_final_kernel<<<j + 1, 64, 0, s>>>(mpart, h);
            spec_mupdate_kernel<<<grid, kBlk, 0, s>>>(gn, V, j + 1, h, w);
        }
        op.dot(w, w, op.scal);
        spec_normalize_kernel<<<grid, kBlk, 0, s>>>(gn, op.scal, beta + j + 1, w, vj + gn);
        SABA_HIP_TRY(hipGetLastError());
        k = j + 1;
        if (k % check == 0 || k == K) {
            SABA_HIP_TRY(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * k, hipMemcpyDeviceToHost, s));
            SABA_HIP_TRY(hipMemcpyAsync(hb.data(), beta, sizeof(double) * (k + 1),
                                        hipMemcpyDeviceToHost, s));
            SABA_HIP_TRY(hipStreamSynchronize(s));
            kb = k;
            for (int i = 1; i <= k; ++i)
                if (hb[i] == 0.0) {
                    kb = i;
                    break;
                }
            if (kb < k || hb[k] == 0.0) break;  // the Krylov space is exhausted: T_kb is exact
            // residual of each wanted Ritz pair: beta_{k} |last component of its vector|
            bool ok = k >= omega;
            for (double th : ok ? top_ritz(ha, hb, k, omega) : std::vector<double>()) {
                const std::vector<double> y = tri_eigvec(ha, hb, k, th);
                if (y.empty() || hb[k] * std::fabs(y[k - 1]) > 0.5 * tol) {
                    ok = false;
                    break;
                }
            }
            if (ok) break;
        }
    }
    // Ritz pairs of the leading block
    const int32_t pairs = std::min(omega, kb);
    const std::vector<double> th = top_ritz(ha, hb, kb, pairs);
    std::vector<double> S((size_t)pairs * kb);
    for (int32_t p = 0; p < pairs; ++p) {
        std::vector<double> y = tri_eigvec(ha, hb, kb, th[p]);
        if (y.empty()) {
            set_error("inverse iteration on the Lanczos matrix failed");
            return SABA_E_INVALID;
        }
        for (int32_t q = 0; q < p; ++q) {  // keep the pairs' vectors orthonormal
            const double *yq = S.data() + (size_t)q * kb;
            double c = 0.0;
            for (int i = 0; i < kb; ++i) c += y[i] * yq[i];
            for (int i = 0; i < kb; ++i) y[i] -= c * yq[i];
        }
        double nrm = 0.0;
        for (double v : y) nrm += v * v;
        nrm = std::sqrt(nrm);
        for (int i = 0; i < kb; ++i) S[(size_t)p * kb + i] = y[i] / nrm;
    }
    Spectrum sp;
    struct SpGuard {  // frees the pairs' device copy unless they are handed out
        Spectrum *sp;
        ~SpGuard() {
            if (sp) sp->dev.release();
        }
    } spguard{&sp};
    sp.graph = graph;
    sp.omega = omega;
    sp.pairs = pairs;
    sp.iterations = k;
    sp.theta = th;
    SABA_TRY(sp.dev.ensure(sizeof(double) * ((size_t)pairs + 2 * (size_t)pairs * gn + 1)));
    double *d_theta = sp.dev.as<double>(), *Y = d_theta + pairs, *U = Y + (size_t)pairs * gn;
    // S goes through the reorthogonalisation scratch (h, mpart: (K + 1)(kDotBlocks + 1) doubles)
    double *d_S = mpart;
    SABA_HIP_TRY(hipMemcpyAsync(d_S, S.data(), sizeof(double) * S.size(), hipMemcpyHostToDevice, s));
    SABA_HIP_TRY(hipMemcpyAsync(d_theta, th.data(), sizeof(double) * pairs, hipMemcpyHostToDevice, s));
    spec_ritz_kernel<<<dim3(grid, pairs), kBlk, 0, s>>>(gn, V, kb, d_S, U);
    SABA_HIP_TRY(hipGetLastError());
    // unit length, residual norms ||N' u - theta u||, and y = u / sqrt(d)
    for (int32_t p = 0; p < pairs; ++p) {
        double *u = U + (size_t)p * gn;
        op.dot(u, u, op.scal);
        spec_unit_kernel<<<grid, kBlk, 0, s>>>(gn, op.scal, u);
        op.apply(u, w);
        spec_axpy_kernel<<<grid, kBlk, 0, s>>>(gn, th[p], u, w);
        op.dot(w, w, h + p);
        spec_scale_kernel<<<grid, kBlk, 0, s>>>(gn, op.sc, u, Y + (size_t)p * gn);
    }
    SABA_HIP_TRY(hipGetLastError());
    std::vector<double> res2(std::max(pairs, 1));
    SABA_HIP_TRY(hipMemcpyAsync(res2.data(), h, sizeof(double) * pairs, hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipStreamSynchronize(s));
    sp.converged = 1;
    for (int32_t p = 0; p < pairs; ++p) {
        const double r = std::sqrt(std::max(res2[p], 0.0));
        sp.max_residual = std::max(sp.max_residual, r);
        if (!(r <= tol)) sp.converged = 0;
    }
    // the rest of the spectrum: deflated Lanczos on the complement of u1 and the kept vectors,
    // from a second start vector (the first one's part in each eigenspace is exactly the kept
    // vector, so it would leave nothing in eigenspaces of repeated eigenvalues)
    saba_lambda_result lr{};
    SABA_TRY(lanczos_extremes(op, U, pairs, 300, 1e-12, seed + 0x9E3779B9u, &lr));
    sp.lambda_rest = lr.lambda;
    sp.lambda_rest_bound = lr.lambda_bound;
    *out = std::move(sp);
    spguard.sp = nullptr;
    return SABA_OK;
}

int resolve_spectrum(Graph *g, int32_t graph, int32_t omega, const Spectrum **out,
                     hipStream_t s) {
    std::lock_guard<std::mutex> lk(g->spec_mu);
    for (auto &sp : g->spectra)
        if (sp->graph == graph && sp->omega == omega) {
            *out = sp.get();
            return SABA_OK;
        }
    auto sp = std::make_unique<Spectrum>();
    const int rc = graph_spectrum(g, graph, omega, 1000, 1e-10, 1u, sp.get(), s);
    if (rc != SABA_OK) {
        sp->dev.release();
        return rc;
    }
    *out = sp.get();
    g->spectra.push_back(std::move(sp));
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

extern "C" int saba_graph_spectrum(saba_graph *gh, const saba_spectrum_params *p, double *values,
                                   double *d_vectors, saba_spectrum_result *out, void *stream) {
    clear_error();
    SABA_TRY(check_graph(gh));
    Graph *g = G(gh);
    if (!p || !values || !out || p->graph < 0 || p->graph >= g->ngraphs || p->max_iters < 0 ||
        p->tol < 0.0) {
        set_error("invalid spectrum arguments");
        return SABA_E_INVALID;
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    Spectrum sp;
    struct Guard {
        Spectrum *sp;
        ~Guard() { sp->dev.release(); }
    } guard{&sp};
    const int32_t gn = g->goff[p->graph + 1] - g->goff[p->graph];
    const int32_t iters = p->max_iters > 0 ? p->max_iters : 1000;
    SABA_TRY(graph_spectrum(g, p->graph, p->omega, iters, p->tol > 0.0 ? p->tol : 1e-10, p->seed,
                            &sp, s));
    for (int32_t k = 0; k < p->omega; ++k) values[k] = k < sp.pairs ? sp.theta[k] : 0.0;
    if (d_vectors) {
        const size_t row = sizeof(double) * (size_t)gn;
        if (sp.pairs > 0)
            SABA_HIP_TRY(hipMemcpyAsync(d_vectors, sp.d_u(gn), row * sp.pairs,
                                        hipMemcpyDeviceToDevice, s));
        if (sp.pairs < p->omega)
            SABA_HIP_TRY(hipMemsetAsync(d_vectors + (size_t)sp.pairs * gn, 0,
                                        row * (p->omega - sp.pairs), s));
    }
    SABA_HIP_TRY(hipStreamSynchronize(s));
    saba_spectrum_result r{};
    r.lambda_rest = sp.lambda_rest;
    r.lambda_rest_bound = sp.lambda_rest_bound;
    r.max_residual = sp.max_residual;
    r.pairs = sp.pairs;
    r.iterations = sp.iterations;
    r.converged = sp.converged;
    *out = r;
    return SABA_OK;
}

/*
 * saba_oracle.c -- CPU oracle for the random-bouquet walk generator and the
 * TGT+ all-edges spanning-centrality estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code with the GPU
 * library (no headers, helpers or tables); both are written from the paper
 * and from the published definition of MurmurHash2.
 *
 * Readings of the paper taken here (the paper is silent or garbled on them):
 *  - Hash (Sec. 3.1 and the AESC experiments, which name Murmur2): 32-bit
 *    MurmurHash2 over little-endian 32-bit words.
 *  - Neighbour choice (Eq. (5), with divisions replaced by multiplications as
 *    in Sec. 4): k = floor(u * d / 2^32) for a 32-bit u, i.e. h_max is the
 *    exclusive bound 2^32.
 *  - Per-walk seed (Eq. (4)/(5), Sec. 3.3): a keyed form.  A walk with
 *    address (a0,a1,a2) and index k in its bouquet schedule (G, S) has
 *    key_hi = Murmur2(a0|a1|a2|floor(k/G), seed) and key_lo = (k mod G) << S;
 *    step l at vertex cur draws u = Murmur2(cur|l, key_hi) XOR key_lo.
 *  - Walk semantics (Alg. 2): position 0 is the start; positions 1..L are
 *    filled by steps l = 1..L; visits are counted at positions 1..L and the
 *    endpoint is position L.
 *  - TGT+ (Alg. 1) as read: truncation tau from the spectral tail bound,
 *    deterministic pull recursion for the p-vectors, the Alg. 1 while-loop
 *    stop rule, NWalks from a Hoeffding bound, and per-pair Monte-Carlo
 *    accumulation as in the paper's inner loop.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* MurmurHash2, 32-bit (Austin Appleby's public-domain algorithm), written
 * from its published description: multiplier 0x5bd1e995, shift 24, seed
 * XOR length, 4-byte little-endian blocks, byte tail, final avalanche
 * (>>13, *m, >>15). */
uint32_t orc_murmur2(const uint8_t *data, int32_t len, uint32_t seed)
{
    const uint32_t m = 0x5bd1e995u;
    uint32_t h = seed ^ (uint32_t)len;
    int32_t i = 0;
    for (; i + 4 <= len; i += 4) {
        uint32_t k = (uint32_t)data[i] | ((uint32_t)data[i + 1] << 8) |
                     ((uint32_t)data[i + 2] << 16) | ((uint32_t)data[i + 3] << 24);
        k *= m;
        k ^= k >> 24;
        k *= m;
        h *= m;
        h ^= k;
    }
    int32_t rest = len - i;
    if (rest == 3) h ^= (uint32_t)data[i + 2] << 16;
    if (rest >= 2) h ^= (uint32_t)data[i + 1] << 8;
    if (rest >= 1) {
        h ^= (uint32_t)data[i];
        h *= m;
    }
    h ^= h >> 13;
    h *= m;
    h ^= h >> 15;
    return h;
}

static void put_le32(uint8_t *p, uint32_t v)
{
    p[0] = (uint8_t)(v & 0xffu);
    p[1] = (uint8_t)((v >> 8) & 0xffu);
    p[2] = (uint8_t)((v >> 16) & 0xffu);
    p[3] = (uint8_t)((v >> 24) & 0xffu);
}

/* Murmur2 of a sequence of 32-bit words, serialised little-endian. */
uint32_t orc_hash_words(const uint32_t *w, int32_t nw, uint32_t seed)
{
    uint8_t buf[64];
    for (int32_t i = 0; i < nw; ++i) put_le32(buf + 4 * i, w[i]);
    return orc_murmur2(buf, 4 * nw, seed);
}

/* Batch form used by the statistical tests: out[i] = Murmur2(a[i]|b[i], seed). */
void orc_hash2_batch(const uint32_t *a, const uint32_t *b, int64_t n, uint32_t seed, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w[2];
        w[0] = a[i];
        w[1] = b[i];
        out[i] = orc_hash_words(w, 2, seed);
    }
}

/* Uniform start vertices (the benchmark's "uniform random sources", drawn by the hash so that
 * both sides can reproduce them): the pool is the vertices with at least one edge, in
 * ascending order; walk j starts at pool[floor(h * |pool| / 2^32)] with h the Murmur2 of the
 * 64-bit walk number j as two little-endian words (low word first) under the walk seed.
 * Returns -1 if the pool is empty and n_walks > 0. */
int32_t orc_uniform_sources(const int32_t *row_ptr, int32_t n, int64_t n_walks, uint32_t seed,
                            int32_t *out)
{
    int64_t np = 0;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] > row_ptr[v]) ++np;
    if (np == 0) return n_walks > 0 ? -1 : 0;
    int32_t *pool = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    if (!pool) return -2;
    int64_t k = 0;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] > row_ptr[v]) pool[k++] = v;
    for (int64_t j = 0; j < n_walks; ++j) {
        uint32_t w[2];
        w[0] = (uint32_t)((uint64_t)j & 0xffffffffu);
        w[1] = (uint32_t)((uint64_t)j >> 32);
        const uint64_t h = orc_hash_words(w, 2, seed);
        /* floor(h * np / 2^32) with h < 2^32 and np < 2^31: below np, no overflow */
        out[j] = pool[(int64_t)((h * (uint64_t)np) >> 32)];
    }
    free(pool);
    return 0;
}

/* Eq. (5): scale the hashed value to [0, d) without a modulo. */
uint32_t orc_choice(uint32_t u, uint32_t d)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)d) >> 32);
}

/* Sec. 3.3 (SABA arrangement) in keyed form: walks k of one address are
 * grouped G at a time; members of a group share key_hi and differ in key_lo. */
void orc_walk_key(uint32_t seed, uint32_t a0, uint32_t a1, uint32_t a2, uint64_t k,
                  uint32_t G, uint32_t S, uint32_t *key_hi, uint32_t *key_lo)
{
    uint32_t w[4];
    uint64_t g = k / G;
    uint32_t r = (uint32_t)(k % G);
    w[0] = a0;
    w[1] = a1;
    w[2] = a2;
    w[3] = (uint32_t)g;
    *key_hi = orc_hash_words(w, 4, seed);
    *key_lo = (G > 1) ? (r << S) : 0u;
}

/* Alg. 2 step: pick the next vertex of a walk standing at `cur` while
 * filling position l. */
static int32_t orc_step(const int32_t *row_ptr, const int32_t *col_idx, int32_t cur,
                        uint32_t l, uint32_t key_hi, uint32_t key_lo)
{
    uint32_t w[2];
    w[0] = (uint32_t)cur;
    w[1] = l;
    uint32_t u = orc_hash_words(w, 2, key_hi) ^ key_lo;
    uint32_t d = (uint32_t)(row_ptr[cur + 1] - row_ptr[cur]);
    uint32_t k = orc_choice(u, d);
    return col_idx[row_ptr[cur] + (int32_t)k];
}

/* ------------------------------------------------------------------ */
/* Samplers of the walk benchmark, the neighbour-choice functions the paper compares
 * (Sec. 3.3 and the Table 4, 5 and 7 experiments).  The estimator uses sampler 0 only.
 *   0  keyed Eq. (5): u = Murmur2(cur|l, key_hi) XOR key_lo, k = floor(u d / 2^32);
 *   1  keyed Eq. (4): the same u, k = u mod d (the modulo the paper removes);
 *   2  Eq. (3): rand() mod d with a sequential generator per walk, here Marsaglia's
 *      xorshift32 (shifts 13, 17, 5; Marsaglia 2003), seeded with key_hi XOR key_lo
 *      (0x9E3779B9 if that is zero) and advanced once before every step;
 *   3  Eq. (5) read literally: u = X_W XOR Murmur2(cur|l, 0) with the unkeyed hash and the
 *      walk's seed X_W = key_hi XOR key_lo fixed for the whole walk, k = floor(u d / 2^32).
 *      Every step then reads the same top bits of X_W, so a walk is decided by a few bits
 *      of its seed; kept as the negative ablation. */
uint32_t orc_xorshift32(uint32_t x)
{
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

typedef struct {
    uint32_t key_hi, key_lo, x;
} orc_walker;

static void orc_walker_init(int32_t sampler, uint32_t key_hi, uint32_t key_lo, orc_walker *w)
{
    w->key_hi = key_hi;
    w->key_lo = key_lo;
    w->x = key_hi ^ key_lo;
    if (sampler == 2 && w->x == 0) w->x = 0x9E3779B9u;
}

static int32_t orc_step_sampler(const int32_t *row_ptr, const int32_t *col_idx, int32_t cur,
                                uint32_t l, int32_t sampler, orc_walker *w)
{
    uint32_t d = (uint32_t)(row_ptr[cur + 1] - row_ptr[cur]);
    uint32_t words[2];
    uint32_t k;
    words[0] = (uint32_t)cur;
    words[1] = l;
    if (sampler == 1) {
        k = (orc_hash_words(words, 2, w->key_hi) ^ w->key_lo) % d;
    } else if (sampler == 2) {
        w->x = orc_xorshift32(w->x);
        k = w->x % d;
    } else if (sampler == 3) {
        k = orc_choice((w->key_hi ^ w->key_lo) ^ orc_hash_words(words, 2, 0u), d);
    } else {
        return orc_step(row_ptr, col_idx, cur, l, w->key_hi, w->key_lo);
    }
    return col_idx[row_ptr[cur] + (int32_t)k];
}

/* Alg. 2: the whole path of one walk, positions 0..L (path has L+1 slots). */
int32_t orc_walk_path(const int32_t *row_ptr, const int32_t *col_idx, int32_t start,
                      int32_t L, uint32_t key_hi, uint32_t key_lo, int32_t *path)
{
    int32_t cur = start;
    path[0] = cur;
    for (int32_t l = 1; l <= L; ++l) {
        if (row_ptr[cur + 1] == row_ptr[cur]) return -1; /* isolated vertex */
        cur = orc_step(row_ptr, col_idx, cur, (uint32_t)l, key_hi, key_lo);
        path[l] = cur;
    }
    return 0;
}

/* Synthetic random-walk benchmark (Sec. 5.4): walks from the given start
 * vertices, counting vertex visits at positions 1..L and endpoints at
 * position L (the start itself when L = 0).
 * Walk j starting at s is the r-th walk of s in list order (r counts the
 * earlier list entries with the same start); its key is that of address
 * (s, 0, 0) and index r. */
int32_t orc_walks_histogram(const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                            const int32_t *sources, int64_t n_walks, int32_t L,
                            uint32_t seed, uint32_t G, uint32_t S, int32_t sampler,
                            int64_t *endpoint, int64_t *visits, int32_t nthreads)
{
    if (sampler < 0 || sampler > 3) return -3;
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_walks > 0 ? n_walks : 1));
    int64_t *seen = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!rank || !seen) {
        free(rank);
        free(seen);
        return -2;
    }
    for (int64_t j = 0; j < n_walks; ++j) {
        int32_t s = sources[j];
        if (s < 0 || s >= n || row_ptr[s + 1] == row_ptr[s]) {
            free(rank);
            free(seen);
            return -1;
        }
        rank[j] = seen[s]++;
    }
    memset(endpoint, 0, sizeof(int64_t) * (size_t)n);
    memset(visits, 0, sizeof(int64_t) * (size_t)n);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4096)
#endif
    for (int64_t j = 0; j < n_walks; ++j) {
        uint32_t khi, klo;
        orc_walker w;
        orc_walk_key(seed, (uint32_t)sources[j], 0u, 0u, (uint64_t)rank[j], G, S, &khi, &klo);
        orc_walker_init(sampler, khi, klo, &w);
        int32_t cur = sources[j];
        for (int32_t l = 1; l <= L; ++l) {
            cur = orc_step_sampler(row_ptr, col_idx, cur, (uint32_t)l, sampler, &w);
#ifdef _OPENMP
#pragma omp atomic
#endif
            visits[cur] += 1;
        }
#ifdef _OPENMP
#pragma omp atomic
#endif
        endpoint[cur] += 1;
    }
    free(rank);
    free(seen);
    return 0;
}

/* Branching statistics (the Table 5 experiment): the walks are taken in an order, cut
 * into consecutive vectors of 8 walks (a last, partial vector is left out), and for
 * every vector and every position l = 1..L the number of distinct vertices among its
 * 8 walks is counted: hist[k] = number of (vector, position) pairs with k distinct
 * vertices (k = 1..8; hist[0] stays 0).  order 0: the order the sources are given;
 * order 1: by start vertex, then by rank (the bouquet order). */
static const int32_t *orc_sort_src;
static const int64_t *orc_sort_rank;
static int orc_cmp_bouquet(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    if (orc_sort_src[x] != orc_sort_src[y]) return orc_sort_src[x] < orc_sort_src[y] ? -1 : 1;
    if (orc_sort_rank[x] != orc_sort_rank[y]) return orc_sort_rank[x] < orc_sort_rank[y] ? -1 : 1;
    return 0;
}

int32_t orc_distinct8(const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                      const int32_t *sources, int64_t n_walks, int32_t L, uint32_t seed,
                      uint32_t G, uint32_t S, int32_t sampler, int32_t order, int64_t *hist)
{
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_walks > 0 ? n_walks : 1));
    int64_t *seen = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_walks > 0 ? n_walks : 1));
    int32_t *path = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_walks > 0 ? n_walks : 1) *
                                      (size_t)(L + 1));
    int32_t rc = 0;
    memset(hist, 0, sizeof(int64_t) * 9);
    if (!rank || !seen || !ord || !path || sampler < 0 || sampler > 3) {
        rc = -2;
        goto done;
    }
    for (int64_t j = 0; j < n_walks; ++j) {
        int32_t s = sources[j];
        if (s < 0 || s >= n || row_ptr[s + 1] == row_ptr[s]) {
            rc = -1;
            goto done;
        }
        rank[j] = seen[s]++;
        ord[j] = j;
    }
    if (order == 1) {
        orc_sort_src = sources;
        orc_sort_rank = rank;
        qsort(ord, (size_t)n_walks, sizeof(int64_t), orc_cmp_bouquet);
    }
    for (int64_t j = 0; j < n_walks; ++j) {
        uint32_t khi, klo;
        orc_walker w;
        orc_walk_key(seed, (uint32_t)sources[j], 0u, 0u, (uint64_t)rank[j], G, S, &khi, &klo);
        orc_walker_init(sampler, khi, klo, &w);
        int32_t *p = path + (size_t)j * (size_t)(L + 1);
        p[0] = sources[j];
        for (int32_t l = 1; l <= L; ++l)
            p[l] = orc_step_sampler(row_ptr, col_idx, p[l - 1], (uint32_t)l, sampler, &w);
    }
    for (int64_t v = 0; v + 8 <= n_walks; v += 8) {
        for (int32_t l = 1; l <= L; ++l) {
            int32_t k = 0;
            for (int32_t a = 0; a < 8; ++a) {
                int32_t x = path[(size_t)ord[v + a] * (size_t)(L + 1) + (size_t)l];
                int32_t first = 1;
                for (int32_t b = 0; b < a; ++b)
                    if (path[(size_t)ord[v + b] * (size_t)(L + 1) + (size_t)l] == x) first = 0;
                k += first;
            }
            hist[k] += 1;
        }
    }
done:
    free(rank);
    free(seen);
    free(ord);
    free(path);
    return rc;
}

/* ------------------------------------------------------------------ */
/* TGT+ as read (Alg. 1). */

/* CalculateTau(e, eps/2): smallest tau >= 0 with
 * (1/d_s + 1/d_t) * lambda^(tau+1) <= (eps/2) * (1 - lambda),
 * the spectral tail bound of the truncated resistance series; powers by
 * repeated multiplication. Capped at tau_cap. */
int32_t orc_tau(int32_t ds, int32_t dt, double lambda, double eps, int32_t tau_cap)
{
    double w = 1.0 / (double)ds + 1.0 / (double)dt;
    double rhs = (eps / 2.0) * (1.0 - lambda);
    double p = lambda;
    int32_t tau = 0;
    while (w * p > rhs && tau < tau_cap) {
        p = p * lambda;
        tau += 1;
    }
    return tau;
}

/* NWalks: number of walk pairs so that the Monte-Carlo part of one directed
 * estimate is within eps/4 with probability 1 - delta/(2m) (Hoeffding: each
 * pair's statistic lies in a range of width 2*L*hmax/d_s). c is
 * 32*ln(4m/delta)/eps^2. */
int64_t orc_nwalks(int32_t L, double hmax, int32_t ds, double c)
{
    double q = ((double)L * hmax) / (double)ds;
    double x = c * q * q;
    if (!(x < 4.0e18)) return -1;
    int64_t r = (int64_t)ceil(x);
    return r < 1 ? 1 : r;
}

double orc_cconst(double eps, double delta, int64_t m)
{
    return 32.0 * log(4.0 * (double)m / delta) / (eps * eps);
}

typedef struct {
    int64_t ebase;   /* the arrays below hold directed edges ebase, ebase + 1, ... */
    int32_t *tau;    /* [nnz] per directed edge (CSR position) */
    int32_t *ttau;   /* [nnz] tilde-tau of the edge's source */
    int64_t *nreq;   /* [nnz] walk pairs */
    double *D;       /* [nnz] deterministic part sum_{l<=min(ttau,tau)} (h_l(s)-h_l(t)) */
    double *MC;      /* [nnz] sum over pairs of X_k */
    int64_t *vis0;   /* [nnz] walk positions from s landing in supp(h_ttau) */
    int64_t *vis1;   /* [nnz] walk positions from t landing in supp(h_ttau) */
    double *g;       /* [nnz] directed estimate g(s,t) */
} orc_edge_out;

/* Integer form of the Monte-Carlo statistic of one source (the per-pair X of
 * Alg. 1's inner loop, split by side and by support vertex):
 *   supp[p]  the p-th vertex of supp(h_ttau) in ascending order (ns of them);
 *   h[p]     h_ttau(supp[p]);
 *   hist[(i*2 + side)*ns + p]  positions 1..L of the side-`side` walks of the
 *            i-th edge of the source (CSR order) that are at supp[p];
 *   MCh[i]   sum over p ascending of h[p] * (c0[p] - c1[p]), the Monte-Carlo
 *            sum of that edge formed from the counts.
 * With supp == NULL only ns is produced (the walks are not run). */
typedef struct {
    int32_t *pos;   /* [n] scratch: support rank of each support vertex */
    int64_t ns;     /* out: support size */
    int32_t *supp;
    double *h;
    int64_t *hist;
    double *MCh;
} orc_count_out;

/* Walk keys carry a 32-bit walk index (the group number hashed into key_hi), so
 * an edge needing 2^32 pairs or more would repeat walks; the estimate would no
 * longer rest on independent walks and the call fails instead. */
#define ORC_MAX_PAIRS 0xFFFFFFFFll

/* Per-source part of Alg. 1 (its outer loop body) for source s: push levels
 * while the support volume is below the walks still needed, then the walk
 * pairs for the directed edges s->t that are wanted (want[e] != 0). */
static int32_t orc_source(const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                          int32_t s, double lambda, double eps, double c, int32_t tau_cap,
                          int32_t tilde_tau_max, int32_t push_all, uint32_t seed,
                          uint32_t G, uint32_t S, const uint8_t *want, orc_edge_out *o,
                          double *hcur, double *hnext, orc_count_out *co)
{
    int32_t e0 = row_ptr[s], e1 = row_ptr[s + 1];
    int32_t ds = e1 - e0;
    int32_t maxtau = 0;
    for (int32_t e = e0; e < e1; ++e) {
        int32_t t = col_idx[e];
        int32_t dt = row_ptr[t + 1] - row_ptr[t];
        o->tau[e - o->ebase] = orc_tau(ds, dt, lambda, eps, tau_cap);
        if (o->tau[e - o->ebase] > maxtau) maxtau = o->tau[e - o->ebase];
        o->D[e - o->ebase] = 0.0;
    }
    for (int32_t x = 0; x < n; ++x) hcur[x] = 0.0;
    hcur[s] = 1.0; /* p_0(., v_i) = e_{v_i} */
    int32_t l = 0;
    double hmax = 0.0;
    for (;;) {
        /* support volume and maximum of p_l */
        int64_t vol = 0;
        hmax = 0.0;
        for (int32_t x = 0; x < n; ++x) {
            if (hcur[x] != 0.0) {
                vol += row_ptr[x + 1] - row_ptr[x];
                if (hcur[x] > hmax) hmax = hcur[x];
            }
        }
        /* deterministic terms of level l */
        for (int32_t e = e0; e < e1; ++e) {
            if (l <= o->tau[e - o->ebase]) o->D[e - o->ebase] += hcur[s] - hcur[col_idx[e]];
        }
        /* walks still needed if the push stopped here */
        int64_t need = 0;
        for (int32_t e = e0; e < e1; ++e) {
            if (o->tau[e - o->ebase] > l) {
                int64_t nw = orc_nwalks(o->tau[e - o->ebase] - l, hmax, ds, c);
                if (nw < 0) return -3;
                need += nw;
            }
        }
        int stop;
        if (push_all)
            stop = (l >= maxtau);
        else
            stop = !(vol < need);
        if (tilde_tau_max >= 0 && l >= tilde_tau_max) stop = 1;
        if (stop) break;
        /* one more level: p_{l+1}(x) = (sum_{y in Gamma(x)} p_l(y)) / d(x) */
        for (int32_t x = 0; x < n; ++x) {
            double acc = 0.0;
            for (int32_t i = row_ptr[x]; i < row_ptr[x + 1]; ++i) acc += hcur[col_idx[i]];
            int32_t dx = row_ptr[x + 1] - row_ptr[x];
            hnext[x] = dx > 0 ? acc / (double)dx : 0.0;
        }
        double *tmp = hcur;
        hcur = hnext;
        hnext = tmp;
        l += 1;
    }
    int32_t ttau = l;
    int64_t ns = 0;
    if (co) {
        /* the support of h_ttau in ascending vertex order */
        for (int32_t x = 0; x < n; ++x) {
            if (hcur[x] != 0.0) {
                if (co->supp) {
                    co->supp[ns] = x;
                    co->h[ns] = hcur[x];
                    co->pos[x] = (int32_t)ns;
                }
                ns += 1;
            }
        }
        co->ns = ns;
        if (!co->supp) return 0;
        memset(co->hist, 0, sizeof(int64_t) * (size_t)(2 * ds) * (size_t)ns);
    }
    for (int32_t e = e0; e < e1; ++e) {
        o->ttau[e - o->ebase] = ttau;
        o->nreq[e - o->ebase] = 0;
        o->MC[e - o->ebase] = 0.0;
        o->vis0[e - o->ebase] = 0;
        o->vis1[e - o->ebase] = 0;
        if (!want[e]) continue;
        int32_t t = col_idx[e];
        double g = o->D[e - o->ebase] / (double)ds;
        int32_t L = o->tau[e - o->ebase] - ttau;
        if (L > 0) {
            int64_t nr = orc_nwalks(L, hmax, ds, c);
            if (nr < 0 || nr > ORC_MAX_PAIRS) return -3;
            o->nreq[e - o->ebase] = nr;
            double mc = 0.0;
            for (int64_t k = 0; k < nr; ++k) {
                /* one walk from s (side 0) and one from t (side 1), as in the
                 * inner loop of Alg. 1 */
                double sum[2];
                for (int side = 0; side < 2; ++side) {
                    uint32_t khi, klo;
                    orc_walk_key(seed, (uint32_t)s, (uint32_t)t, (uint32_t)side, (uint64_t)k, G, S,
                                 &khi, &klo);
                    int32_t cur = side == 0 ? s : t;
                    double acc = 0.0;
                    int64_t hits = 0;
                    for (int32_t b = 1; b <= L; ++b) {
                        cur = orc_step(row_ptr, col_idx, cur, (uint32_t)b, khi, klo);
                        acc += hcur[cur];
                        hits += hcur[cur] != 0.0;
                        if (co && hcur[cur] != 0.0)
                            co->hist[((int64_t)(e - e0) * 2 + side) * ns + co->pos[cur]] += 1;
                    }
                    sum[side] = acc;
                    if (side == 0)
                        o->vis0[e - o->ebase] += hits;
                    else
                        o->vis1[e - o->ebase] += hits;
                }
                double X = sum[0] - sum[1];
                mc += X;
                g += X / ((double)nr * (double)ds);
            }
            o->MC[e - o->ebase] = mc;
        }
        if (co) {
            const int64_t *c0 = co->hist + (int64_t)(e - e0) * 2 * ns, *c1 = c0 + ns;
            double mch = 0.0;
            for (int64_t p = 0; p < ns; ++p) mch += co->h[p] * (double)(c0[p] - c1[p]);
            co->MCh[e - e0] = mch;
        }
        o->g[e - o->ebase] = g;
    }
    return 0;
}

/* Alg. 1 driver.  If query == NULL all edges are estimated and sc_out[i] is
 * the estimate of the i-th canonical edge (u < v, lexicographic); otherwise
 * sc_out[j] is the estimate of query edge j = (query[2j], query[2j+1]).
 * Per-directed-edge diagnostics go to the arrays of `o` (may be NULL). */
int32_t orc_aesc(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, double eps,
                 double delta, double lambda, uint32_t seed, uint32_t G, uint32_t S,
                 int32_t tau_cap, int32_t tilde_tau_max, int32_t push_all,
                 const int32_t *query, int64_t q, double *sc_out,
                 int32_t *tau, int32_t *ttau, int64_t *nreq, double *D, double *MC,
                 int64_t *vis0, int64_t *vis1, double *gout, int32_t nthreads)
{
    int64_t nnz = row_ptr[n];
    int64_t m = nnz / 2;
    double c = orc_cconst(eps, delta, m);
    orc_edge_out o;
    int own = 0;
    if (!tau) {
        own = 1;
        tau = (int32_t *)malloc(sizeof(int32_t) * nnz);
        ttau = (int32_t *)malloc(sizeof(int32_t) * nnz);
        nreq = (int64_t *)malloc(sizeof(int64_t) * nnz);
        D = (double *)malloc(sizeof(double) * nnz);
        MC = (double *)malloc(sizeof(double) * nnz);
        vis0 = (int64_t *)malloc(sizeof(int64_t) * nnz);
        vis1 = (int64_t *)malloc(sizeof(int64_t) * nnz);
        gout = (double *)malloc(sizeof(double) * nnz);
    }
    o.ebase = 0;
    o.tau = tau; o.ttau = ttau; o.nreq = nreq; o.D = D; o.MC = MC;
    o.vis0 = vis0; o.vis1 = vis1; o.g = gout;
    uint8_t *want = (uint8_t *)calloc((size_t)nnz, 1);
    uint8_t *srcw = (uint8_t *)calloc((size_t)n, 1);
    int32_t rc = 0;
    if (query == NULL) {
        memset(want, 1, (size_t)nnz);
        memset(srcw, 1, (size_t)n);
    } else {
        for (int64_t j = 0; j < q && rc == 0; ++j) {
            int32_t u = query[2 * j], v = query[2 * j + 1];
            int32_t euv = -1, evu = -1;
            if (u < 0 || v < 0 || u >= n || v >= n) { rc = -1; break; }
            for (int32_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) if (col_idx[i] == v) euv = i;
            for (int32_t i = row_ptr[v]; i < row_ptr[v + 1]; ++i) if (col_idx[i] == u) evu = i;
            if (euv < 0 || evu < 0) { rc = -1; break; }
            want[euv] = want[evu] = 1;
            srcw[u] = srcw[v] = 1;
        }
    }
    if (rc == 0) {
#ifdef _OPENMP
        if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
        {
            double *ha = (double *)malloc(sizeof(double) * (size_t)n);
            double *hb = (double *)malloc(sizeof(double) * (size_t)n);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int32_t s = 0; s < n; ++s) {
                if (!srcw[s]) continue;
                int32_t r = orc_source(row_ptr, col_idx, n, s, lambda, eps, c, tau_cap,
                                       tilde_tau_max, push_all, seed, G, S, want, &o, ha, hb,
                                       NULL);
                if (r != 0) {
#ifdef _OPENMP
#pragma omp critical
#endif
                    rc = r;
                }
            }
            free(ha);
            free(hb);
        }
    }
    if (rc == 0) {
        /* final combine: s(e_ij) = g(v_i, v_j) + g(v_j, v_i) */
        if (query == NULL) {
            int64_t i = 0;
            for (int32_t u = 0; u < n; ++u) {
                for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                    int32_t v = col_idx[e];
                    if (v <= u) continue;
                    int32_t evu = -1;
                    for (int32_t f = row_ptr[v]; f < row_ptr[v + 1]; ++f) if (col_idx[f] == u) evu = f;
                    sc_out[i++] = o.g[e] + o.g[evu];
                }
            }
        } else {
            for (int64_t j = 0; j < q; ++j) {
                int32_t u = query[2 * j], v = query[2 * j + 1];
                int32_t euv = -1, evu = -1;
                for (int32_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) if (col_idx[i] == v) euv = i;
                for (int32_t i = row_ptr[v]; i < row_ptr[v + 1]; ++i) if (col_idx[i] == u) evu = i;
                sc_out[j] = o.g[euv] + o.g[evu];
            }
        }
    }
    free(want);
    free(srcw);
    if (own) {
        free(tau); free(ttau); free(nreq); free(D); free(MC); free(vis0); free(vis1); free(gout);
    }
    return rc;
}

/* Exported for the tests: the c constant and the NWalks count as the oracle
 * evaluates them. */
double orc_cconst_export(double eps, double delta, int64_t m) { return orc_cconst(eps, delta, m); }
int64_t orc_nwalks_export(int32_t L, double hmax, int32_t ds, double c) { return orc_nwalks(L, hmax, ds, c); }
int32_t orc_tau_export(int32_t ds, int32_t dt, double lambda, double eps, int32_t tau_cap)
{
    return orc_tau(ds, dt, lambda, eps, tau_cap);
}

/* The counts of one source s (see orc_count_out): the push and the walk pairs
 * of all edges of s exactly as orc_aesc runs them, with the visits to the
 * support of h_ttau tallied per edge, side and support vertex.  The per-edge
 * outputs tau .. g (required, d_s entries each) are indexed by the edge's
 * position i in the row of s.  supp == NULL: only the support size is
 * computed (and tau, D of the push).  Returns the support size,
 * or a negative code (-1 bad source, -2 memory, -3 walk-count overflow). */
int64_t orc_source_counts(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t s,
                          double eps, double delta, double lambda, uint32_t seed, uint32_t G,
                          uint32_t S, int32_t tau_cap, int32_t tilde_tau_max, int32_t push_all,
                          int32_t *supp, double *h, int64_t *hist, double *MCh, int32_t *tau,
                          int32_t *ttau, int64_t *nreq, double *D, double *MC, int64_t *vis0,
                          int64_t *vis1, double *g)
{
    if (s < 0 || s >= n || row_ptr[s + 1] == row_ptr[s]) return -1;
    int64_t m = (int64_t)row_ptr[n] / 2;
    double c = orc_cconst(eps, delta, m);
    int32_t ds = row_ptr[s + 1] - row_ptr[s];
    orc_edge_out o;
    o.ebase = row_ptr[s];
    o.tau = tau; o.ttau = ttau; o.nreq = nreq; o.D = D; o.MC = MC;
    o.vis0 = vis0; o.vis1 = vis1; o.g = g;
    uint8_t *want = (uint8_t *)calloc((size_t)row_ptr[n] + 1, 1);
    double *ha = (double *)malloc(sizeof(double) * (size_t)n);
    double *hb = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t rc = -2;
    if (want && ha && hb && pos) {
        memset(want + row_ptr[s], 1, (size_t)ds);
        orc_count_out co;
        co.pos = pos;
        co.ns = 0;
        co.supp = supp;
        co.h = h;
        co.hist = hist;
        co.MCh = MCh;
        int32_t r = orc_source(row_ptr, col_idx, n, s, lambda, eps, c, tau_cap, tilde_tau_max,
                               push_all, seed, G, S, want, &o, ha, hb, &co);
        rc = r != 0 ? (int64_t)r : co.ns;
    }
    free(want);
    free(ha);
    free(hb);
    free(pos);
    return rc;
}

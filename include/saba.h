/*
 * saba.h -- C-ABI of the MI355X random-bouquet walk and spanning-centrality
 * library (libsaba.so, HIP for gfx950).
 *
 * The library implements, on one GPU:
 *   - random-walk generation on an undirected int32 CSR graph with the
 *     hash-based neighbour choice of Eq. (5) and the grouping of walks into
 *     bouquets (Sec. 3.2-3.3, Alg. 2 and Alg. 3);
 *   - the TGT+ all-edges spanning-centrality estimator (Alg. 1) fed by those
 *     walks, for all edges or for a query edge set.
 *
 * Conventions shared by every call:
 *   - Return value: SABA_OK (0) or a negative SABA_E_* code.  No exception or
 *     abort crosses the ABI.  saba_last_error() then holds a message for the
 *     calling thread.
 *   - Pointers named d_* are device pointers (HIP device memory of the current
 *     device) owned by the caller.  Every other pointer is a host pointer.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it.  Calls that must read device results on the host
 *     (the estimator's level loop, statistics) synchronise that stream.
 *   - A graph handle may be used by one stream at a time.
 *   - A graph handle belongs to the device that was current when it was created: make that
 *     device current before every call on it (the library does not switch devices; a
 *     server's own lane threads do so themselves).
 *   - Results depend only on (graph, parameters): bouquet width, launch shape
 *     and batching never change them.
 */
#ifndef SABA_H
#define SABA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SABA_ABI_VERSION 5

/* status codes */
#define SABA_OK 0
#define SABA_E_INVALID (-1)      /* an argument is out of range or NULL where required */
#define SABA_E_NOMEM (-2)        /* host or device allocation failed */
#define SABA_E_HIP (-3)          /* a HIP runtime call failed */
#define SABA_E_GRAPH (-4)        /* the CSR arrays are not a canonical undirected graph */
#define SABA_E_DISCONNECTED (-5) /* the estimator needs a connected graph */
#define SABA_E_BIPARTITE (-6)    /* the estimator needs a non-bipartite graph (lambda < 1) */
#define SABA_E_NOT_EDGE (-7)     /* a query pair is not an edge of the graph */
#define SABA_E_OVERFLOW (-8)     /* a walk count exceeds its range (2^32 - 1 pairs per edge, 2^32 - 1 walks) */
#define SABA_E_NODEVICE (-9)     /* no usable gfx950 device */
#define SABA_E_BUSY (-10)        /* the server's admission queue is full (backpressure) */
#define SABA_E_TIMEOUT (-11)     /* a server request has not finished within the wait */
#define SABA_E_CANCELLED (-12)   /* the server was destroyed before the request finished */

/* saba_graph_create flags */
#define SABA_DEVICE_PTRS 1u /* row_ptr / col_idx are device pointers */
#define SABA_TRUSTED 2u     /* skip CSR validation */

/* walk execution modes (results are identical in both) */
#define SABA_WALK_NAIVE 0   /* one lane per walk, walks in the order the sources are given */
#define SABA_WALK_BOUQUET 1 /* walks of one start vertex run side by side in a wavefront */
#define SABA_WALK_NAIVE_LOG 2 /* the order of SABA_WALK_NAIVE on the bouquet kernel's data path
                                 (16-byte walk entries, counting through the visit log): the
                                 walk-order ablation */

/* neighbour-choice functions of the walk benchmark (the paper's comparison, Sec. 3.3).  The
 * estimator always uses SABA_SAMPLER_KEYED. */
#define SABA_SAMPLER_KEYED 0      /* Eq. (5), keyed: u = Murmur2(cur|l, key_hi) ^ key_lo,
                                     k = floor(u d / 2^32) */
#define SABA_SAMPLER_KEYED_MOD 1  /* Eq. (4), keyed: the same u, k = u mod d */
#define SABA_SAMPLER_STREAM_MOD 2 /* Eq. (3): per-walk xorshift32 stream (shifts 13, 17, 5)
                                     seeded with key_hi ^ key_lo (0x9E3779B9 if zero),
                                     advanced once per step, k = x mod d */
#define SABA_SAMPLER_LITERAL 3    /* Eq. (5) read literally: u = (key_hi ^ key_lo) ^
                                     Murmur2(cur|l, 0), k = floor(u d / 2^32); each walk is
                                     decided by a few top bits of its seed (negative ablation) */

/* Where saba_walks takes the start vertices from. */
#define SABA_SOURCES_EXPLICIT 0 /* walk j starts at d_sources[j] */
#define SABA_SOURCES_UNIFORM 1  /* walk j starts at pool[floor(h_j * |pool| / 2^32)], pool = the
                                   non-isolated vertices in ascending order and
                                   h_j = Murmur2(LE32(j mod 2^32) | LE32(j / 2^32), seed):
                                   uniform sources drawn on the device */

typedef struct saba_graph saba_graph;

typedef struct {
    int32_t n;          /* vertices */
    int64_t nnz;        /* directed entries = 2m */
    int64_t m;          /* undirected edges */
    int32_t d_max;      /* maximum degree */
    int32_t n_isolated; /* vertices of degree 0 */
    int32_t connected;  /* 1 / 0 (0 when the handle holds several graphs) */
    int32_t bipartite;  /* 1 / 0 */
    int32_t ngraphs;    /* graphs held side by side (saba_graph_create_multi) */
} saba_graph_info_t;

typedef struct {
    int64_t walks;            /* walks generated */
    int64_t walk_steps;       /* steps taken by those walks */
    int64_t push_edge_visits; /* adjacency entries read by the estimator's deterministic levels */
    int64_t sources;          /* sources processed by the estimator */
    int64_t batches;          /* source batches (estimator); walk-kernel launches, one per
                                 visit-log chunk (walk calls) */
    int32_t max_tau;          /* largest truncation length */
    int32_t max_ttau;         /* largest deterministic level count */
    int32_t warnings;         /* bit 0: some tau was capped at tau_cap */
    int32_t reserved;
    double kernel_ms;         /* time of the dominant kernel (walk kernel), when timing was asked */
    double total_ms;          /* time of the whole call on its stream, when timing was asked */
    double count_ms;          /* time of the histogram passes after the walk kernel, if timed */
} saba_stats;

typedef struct {
    int64_t n_walks;         /* number of walks */
    int32_t length;          /* steps per walk L >= 0 (positions 1..L are counted) */
    uint32_t seed;           /* walk seed */
    uint32_t group;          /* G >= 1: walks per key group (1 = independent walks) */
    uint32_t spread;         /* S: bit offset of the lane index inside key_lo; G << S <= 2^32 */
    int32_t mode;            /* SABA_WALK_NAIVE, SABA_WALK_BOUQUET or SABA_WALK_NAIVE_LOG */
    int32_t time_kernels;    /* nonzero: fill saba_stats kernel_ms / total_ms (synchronises) */
    const int32_t *d_sources; /* [n_walks] start vertex of each walk (device); read only with
                                SABA_SOURCES_EXPLICIT */
    int32_t sampler;         /* SABA_SAMPLER_* (0: keyed Eq. (5)) */
    int32_t source_mode;     /* SABA_SOURCES_EXPLICIT (0) or SABA_SOURCES_UNIFORM */
    int64_t *d_distinct;     /* NULL, or [9] int64 (device): branching statistics (the Table 5
                                experiment).  The walks are cut into consecutive vectors of 8
                                in the order the mode runs them (naive and naive-log: the order
                                of d_sources; bouquet: by start vertex, then rank), a last partial
                                vector left out; d_distinct[k] receives the number of (vector,
                                position l = 1..L) pairs with k distinct vertices.  Slower
                                kernels are used while it is set; results are unchanged. */
} saba_walk_params;

typedef struct {
    double eps;            /* absolute error target (0 < eps) */
    double delta;          /* failure probability (0 < delta < 1) */
    double lambda;         /* max(|lambda_2|, |lambda_n|) of D^-1/2 A D^-1/2, 0 < lambda < 1;
                              <= 0: computed on the device (saba_graph_lambda's lambda_bound,
                              cached in the handle per graph) */
    uint32_t seed;         /* walk seed */
    uint32_t group;        /* G >= 1 walk key grouping (1 = independent walks) */
    uint32_t spread;       /* S, as in saba_walk_params */
    int32_t tau_cap;       /* upper bound on tau (<= 0: 4096) */
    int32_t tilde_tau_max; /* upper bound on deterministic levels (-1: none; 0: walks only) */
    int32_t push_all;      /* nonzero: deterministic levels up to tau, no walks */
    int32_t batch_sources; /* sources per batch (0: chosen from mem_budget); no effect on results */
    int32_t time_kernels;  /* nonzero: fill kernel_ms / total_ms in saba_stats */
    int64_t mem_budget;    /* bytes of batch scratch (0: the smaller of 32 GiB and 40% of free memory);
                              with two batch streams each pool set holds half of it */
    int32_t omega;         /* eigenpairs used (Alg. 1's omega), 0 <= omega <= 64.  0: the plain
                              truncated series with tau from lambda.  omega > 0: the library
                              finds the omega nontrivial eigenpairs of N of largest |theta|
                              (saba_graph_spectrum with its defaults, cached per graph and
                              omega), adds their exact contribution beyond each edge's tau to
                              the estimate, and takes tau from the radius of the rest of the
                              spectrum: lambda > 0 is then that radius, given by the caller,
                              and lambda <= 0 leaves it to the library (lambda_rest_bound).
                              The pairs stay cached in the handle until it is destroyed
                              (16 omega n bytes per graph and omega; the first request of
                              a (graph, omega) also needs the Lanczos basis for the
                              duration of the call, as saba_graph_spectrum). */
    int32_t reserved;      /* 0 */
} saba_aesc_params;

/* One estimator request of saba_aesc_batch. */
typedef struct {
    int32_t graph;            /* index of the graph in the handle (0 for a single graph) */
    int32_t reserved;
    saba_aesc_params params;  /* eps, delta, lambda, seed, group, spread, tau_cap, tilde_tau_max,
                                 push_all (the execution fields are taken from the options) */
    const int32_t *d_edges;   /* [2q] query pairs in the graph's own vertex ids (device) */
    int64_t q;                /* number of pairs, or -1 for all edges of the graph */
    double *d_sc;             /* [q] results, or [m of the graph] in canonical order when q = -1 */
} saba_aesc_request;

/* Execution options of saba_aesc_batch; none of them changes a result. */
typedef struct {
    int64_t mem_budget;    /* bytes of batch scratch (0: the smaller of 32 GiB and 40% of free memory);
                              with two batch streams each pool set holds half of it */
    int32_t batch_sources; /* cap on instances per batch (0: from mem_budget) */
    int32_t time_kernels;  /* nonzero: fill kernel_ms / total_ms in saba_stats */
} saba_batch_options;

/* saba_graph_lambda arguments. */
typedef struct {
    int32_t graph;      /* graph of the handle */
    int32_t max_iters;  /* Lanczos steps at most (0: 300) */
    double tol;         /* stop when both extreme Ritz values move less than this over 10 steps
                           (0: 1e-12) */
    uint32_t seed;      /* start vector */
    int32_t reserved;
} saba_lambda_params;

/* saba_graph_lambda result. */
typedef struct {
    double lambda;       /* max(|lambda2|, |lambdan|) */
    double lambda_bound; /* max over the two extreme Ritz values of |theta| + its residual */
    double lambda2;      /* largest Ritz value of N restricted to the complement of sqrt(d) */
    double lambdan;      /* smallest Ritz value, the estimate of lambda_n */
    double residual;     /* largest residual norm of the two extreme Ritz pairs */
    int32_t iterations;  /* Lanczos steps taken */
    int32_t converged;   /* 1 if the tolerance was met or an invariant subspace was found */
} saba_lambda_result;

/* saba_graph_spectrum arguments. */
typedef struct {
    int32_t graph;      /* graph of the handle */
    int32_t omega;      /* eigenpairs wanted, 1 <= omega <= 64 and omega < n of the graph */
    int32_t max_iters;  /* Lanczos steps at most (0: the smaller of n - 1 and 1000) */
    uint32_t seed;      /* start vector (the estimator uses 1) */
    double tol;         /* residual norm each kept pair must reach (0: 1e-10) */
} saba_spectrum_params;

/* saba_graph_spectrum result. */
typedef struct {
    double lambda_rest;       /* largest |Ritz value| of N on the complement of sqrt(d) and
                                 of the kept eigenvectors */
    double lambda_rest_bound; /* lambda_rest plus the residual norm of its Ritz pair */
    double max_residual;      /* largest ||N u_k - theta_k u_k|| over the kept pairs */
    int32_t pairs;            /* pairs kept: omega, or fewer when the Krylov space of the start
                                 vector is exhausted first (repeated eigenvalues) */
    int32_t iterations;       /* Lanczos steps of the eigenpair run */
    int32_t converged;        /* 1 if every kept pair met tol */
    int32_t reserved;
} saba_spectrum_result;

/* Execution knobs of a handle.  None of them changes a result: walks, counts and estimates are
 * the same under every setting (the tests compare them bit for bit). */
typedef struct {
    int32_t walks_per_lane;  /* walks stepped side by side per lane in the bouquet walk kernel:
                                1, 2 or 4 (0: 1) */
    int32_t walk_blocks;     /* blocks of the persistent bouquet walk kernel (0: 8192) */
    int32_t est_walk_blocks; /* blocks of the estimator's walk-pair kernel (0: 1024) */
    int32_t est_push_blocks; /* blocks of the estimator's frontier kernels (0: 2048) */
    int32_t walk_chunks;     /* chunks a bouquet walk call's visit log is cut into; the counting
                                passes of a chunk run on a second stream while the next chunk
                                walks (0: 4 when each chunk still holds 2^19 walks, else as few
                                as the 2^29-entry log allows; at most 64) */
    int32_t est_walk_queue;  /* the estimator's walk-pair schedule.  0: a fixed wavefront stride
                                over the chunks; 1: device work queues, one per XCD range of
                                the chunk space; 2: staged tiles, blocks of 1024 threads take
                                up to 32 chunks of one source at a time from per-XCD queues
                                and test support membership against the source's bitmap
                                copied into LDS (falls back to 1 when the largest graph's
                                bitmap exceeds a block's LDS, and for saba_aesc_counts) */
    int32_t est_batch_streams; /* streams of the synchronous estimator calls: 1 (and 0) = every
                                  batch in order on the caller's stream; 2 = two pool sets of
                                  half the memory budget each, the deterministic levels of
                                  batch k + 1 on the handle's second stream while the walk
                                  pairs of batch k run on the caller's stream.  The counts
                                  export (saba_aesc_counts) always runs in order */
} saba_exec_config;

/* Options of saba_server_create; none of them changes a result. */
typedef struct {
    int64_t mem_budget;        /* bytes of source scratch over all lanes (0: the smaller of 32 GiB and 40% of free
                                  memory); each lane batches sources up to its equal share */
    int64_t max_queued_edges;  /* admission bound: query edges submitted and not finished; a
                                  request beyond it is refused with SABA_E_BUSY (0: 2^20) */
    int64_t arena_edges;       /* query edges whose directed estimates can be held at once; a
                                  request is admitted to the batches when its 2q entries fit
                                  (0: 2^22); a request with q > arena_edges is invalid */
    int32_t lanes;             /* batches in flight, each on its own stream (0: 2; at most 8) */
    int32_t max_batch_sources; /* sources per batch (0: 4096; at most 65535) */
} saba_server_options;

/* One query of the server. */
typedef struct {
    int32_t graph;            /* index of the graph in the handle */
    int32_t reserved;
    saba_aesc_params params;  /* eps, delta, lambda, seed, group, spread, tau_cap, tilde_tau_max,
                                 push_all (the execution fields are ignored) */
    const int32_t *edges;     /* [2q] query pairs (host) in the graph's own vertex ids; copied by
                                 saba_server_submit, so the caller may free them on return */
    int64_t q;                /* number of pairs, q >= 0 */
    double *d_sc;             /* [q] results (device), written before the request is reported
                                 finished; must stay valid until then */
} saba_server_request;

/* Outcome of one server request. */
typedef struct {
    int32_t status;     /* SABA_OK or the error the request failed with */
    int32_t batches;    /* batches that carried its sources */
    int64_t instances;  /* sources (distinct endpoints) it needed */
    double queue_ms;    /* submit -> admission to the batches */
    double latency_ms;  /* submit -> results written */
} saba_server_result;

/* Counters of a server since its creation. */
typedef struct {
    int64_t submitted;         /* requests accepted by saba_server_submit */
    int64_t rejected;          /* requests refused with SABA_E_BUSY */
    int64_t completed;         /* requests finished with SABA_OK */
    int64_t failed;            /* requests finished with an error */
    int64_t batches;           /* batches run */
    int64_t instances;         /* sources run */
    int64_t walk_steps;        /* walk steps taken */
    int64_t queued_edges;      /* query edges submitted and not yet finished, now */
    int64_t queued_requests;   /* requests submitted and not yet finished, now */
    int64_t peak_queued_edges; /* largest value queued_edges has had */
    double busy_ms;            /* wall time the lanes spent running batches, summed over lanes */
} saba_server_stats_t;

typedef struct saba_server saba_server;

/* ABI version (SABA_ABI_VERSION). */
int saba_version(void);

/* Message of the last failing call on this thread ("" if none). Valid until the next call. */
const char *saba_last_error(void);

/*
 * Upload a graph (Sec. 2 notation: Gamma(v) is row v of the CSR, d(v) its length).
 *   row_ptr[n+1], col_idx[nnz]: int32 CSR, host arrays unless SABA_DEVICE_PTRS.
 *   The graph must be canonical: row_ptr[0] = 0, row_ptr[n] = nnz, rows strictly
 *   ascending (no duplicates), no self-loops, symmetric.  Checked unless
 *   SABA_TRUSTED (SABA_E_GRAPH on failure).
 * The library copies the arrays into device memory it owns; the caller may free its
 * arrays when the call returns.  *out receives the handle (NULL on failure).
 */
int saba_graph_create(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int64_t nnz,
                      uint32_t flags, void *stream, saba_graph **out);

/*
 * Upload several graphs at once, side by side (a block-diagonal CSR): graph k owns the
 * vertices vertex_offsets[k] .. vertex_offsets[k+1]-1 (host array of ngraphs + 1 entries,
 * from 0 to n) and no edge may leave its graph (SABA_E_GRAPH).  Otherwise as
 * saba_graph_create.  Estimator requests name a graph by k and use its own vertex ids, and
 * each result equals the one computed on a handle holding that graph alone.
 */
int saba_graph_create_multi(const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                            int64_t nnz, int32_t ngraphs, const int32_t *vertex_offsets,
                            uint32_t flags, void *stream, saba_graph **out);

/*
 * The estimator's spectral input on the device (the lambda of CalculateTau, Alg. 1):
 * max(|lambda_2|, |lambda_n|) of N = D^-1/2 A D^-1/2 for one connected graph of the handle,
 * by a Lanczos iteration in FP64 on N with its top eigenvector sqrt(d) projected out.  Ritz
 * values lie inside the spectrum, so lambda approaches the true value from below;
 * lambda_bound adds each extreme pair's residual norm.  Deterministic for given arguments.
 * Synchronises `stream`.  Errors: SABA_E_DISCONNECTED, SABA_E_INVALID.
 */
int saba_graph_lambda(saba_graph *g, const saba_lambda_params *p, saba_lambda_result *out,
                      void *stream);

/*
 * Leading eigenpairs of N = D^-1/2 A D^-1/2 for one connected graph of the handle: the
 * `pairs` nontrivial eigenpairs of largest |theta| (omega of them unless the Krylov space of
 * the start vector runs out first), the spectral input of the omega > 0 form of
 * CalculateTau (Alg. 1).  Lanczos in FP64 on N with sqrt(d) projected out and every new
 * vector reorthogonalised against all earlier ones (twice); Ritz values from Sturm
 * bisection of the tridiagonal matrix and Ritz vectors from inverse iteration, mapped back
 * through the stored basis.  A second, deflated Lanczos run on the complement of sqrt(d) and
 * the kept vectors, from another start vector, gives lambda_rest, so that eigenvalues the
 * first run could not separate (copies of a repeated eigenvalue) still bound the truncation.
 *   values[omega] (host): theta_k by decreasing |theta| (equal |theta|: positive first);
 *   entries past `pairs` are set to 0.
 *   d_vectors (device, may be NULL): [omega][n of the graph] unit eigenvectors u_k, row k
 *   for theta_k (the sign is deterministic, not specified); rows past `pairs` are set to 0.
 * Needs (min(max_iters, n - 1) + 1) * n * 8 bytes of device scratch, released on return.
 * Deterministic for given arguments.  Synchronises `stream`.  Errors: SABA_E_DISCONNECTED,
 * SABA_E_INVALID, SABA_E_NOMEM.
 */
int saba_graph_spectrum(saba_graph *g, const saba_spectrum_params *p, double *values,
                        double *d_vectors, saba_spectrum_result *out, void *stream);

/* Read or replace the execution knobs of a handle (SABA_E_INVALID for values out of range).
 * The knobs are read without a lock by every call on the handle and by the lanes of a server
 * over it: replace them (here or through an autotuner, which sets them while it times) only
 * while no other call on g and no server over g runs. */
int saba_graph_get_config(const saba_graph *g, saba_exec_config *out);
int saba_graph_set_config(saba_graph *g, const saba_exec_config *cfg);

/*
 * Autotuner of the bouquet walk kernel: runs the walk workload `sample` (bouquet mode) under
 * each candidate (walks per lane 1, 2, 4; 1024, 2048, 4096 or 8192 persistent blocks; 1, 4 or
 * 8 visit-log chunks), times
 * the whole call (walks and counting passes) with HIP events, keeps the fastest in the handle
 * and returns it in *best
 * (may be NULL).  The sample's outputs are written to scratch the call allocates.
 */
int saba_autotune_walks(saba_graph *g, const saba_walk_params *sample, saba_exec_config *best,
                        void *stream);

/*
 * Grouped-bouquet autotuner (Sec. 3.3): among the key schedules (G, S) whose walks stay within
 * a stated correlation budget, the fastest on the caller's walk sample (bouquet mode, its
 * sources, length and seed).  G > 1 changes which walks are drawn (walks of a group share
 * their path until their choices split), so, unlike the execution knobs, the schedule is
 * returned to the caller and not kept in the handle.  The budget min_distinct is the least
 * mean number of distinct vertices per vector of 8 consecutive walks, at every position,
 * measured on the sample (the branching statistic of saba_walks): about 7.7 for independent
 * walks (G = 1, which is always a candidate), 1 for walks that move together.  Candidates:
 * G = 1, and G in {8, 64, 256} with S = 4, 8, ..., 28 and (G - 1) << S < 2^32.  Each is timed
 * as a whole call (one warm-up, two timed).  *best: the schedule, its distinct mean and its
 * time per call.  Errors: SABA_E_INVALID (NULL sample or best, budget outside [1, 8]), and
 * those of saba_walks.  Only G = 1 carries the estimator's eps guarantee.
 */
typedef struct {
    uint32_t group;
    uint32_t spread;
    double distinct_mean;
    double ms;
} saba_bouquet_choice;

int saba_autotune_bouquet(saba_graph *g, const saba_walk_params *sample, double min_distinct,
                          saba_bouquet_choice *best, void *stream);

/*
 * Autotuner of the estimator: runs the requests `sample` (as saba_aesc_batch, with `opt`,
 * which may be NULL) under each candidate grid (512, 1024, 2048 or 4096 blocks for the
 * walk-pair kernel x 1024, 2048, 4096 or 8192 blocks for the frontier-group kernels x the
 * static, the work-queue or the staged walk-pair schedule (whose grid follows from its LDS, so
 * it is tried at one walk-pair grid) x one or two batch streams), times whole
 * calls with HIP events, keeps the fastest in the handle and returns it in *best (may be
 * NULL).  The knobs do not change results; the sample's outputs hold its results on return.
 * Errors: those of saba_aesc_batch, SABA_E_INVALID for an empty sample.
 */
int saba_autotune_aesc(saba_graph *g, const saba_aesc_request *sample, int32_t nreq,
                       const saba_batch_options *opt, saba_exec_config *best, void *stream);

/*
 * Diagnostic: dependent random 16-byte reads per second on this GPU, the access pattern of a
 * walk step (every lane of 8192 x 256 follows its own chain of `steps` reads at hashed positions
 * of a buffer of 2^log2_records aligned 16-byte records, 10 <= log2_records <= 30).  It gives
 * the measured random-access ceiling the walk kernels are compared with.  *ms (may be NULL)
 * receives the timed launch.  Allocates and frees its buffer; synchronises `stream`.
 */
int saba_probe_random_reads(int32_t log2_records, int32_t steps, double *reads_per_s, double *ms,
                            void *stream);

/*
 * Failure injection, for callers that test their own error handling: with n > 0, the n-th
 * scratch allocation the library makes from now on fails with SABA_E_NOMEM, as a real
 * out-of-memory would (n = 0 disarms it).  Process-wide.  A call that fails this way leaves
 * every handle usable: the next call on it computes the same results as if nothing had failed.
 */
int saba_debug_fail_allocation(int32_t n);

/* Free every resource of a handle.  NULL is accepted.  Synchronises the device. */
int saba_graph_destroy(saba_graph *g);

/* Fill *out with the graph's sizes and properties. */
int saba_graph_info(const saba_graph *g, saba_graph_info_t *out);

/*
 * Random-walk generation (Alg. 2 / Alg. 3, neighbour choice of Eq. (5), bouquet
 * arrangement of Sec. 3.3), the synthetic benchmark of Sec. 5.4.
 *   Walk j starts at d_sources[j] (which must not be isolated), or, with
 *   SABA_SOURCES_UNIFORM, at the j-th hashed draw from the non-isolated vertices
 *   (SABA_E_INVALID if the graph has none).  The walks that start at a vertex s are
 *   numbered r = 0, 1, ... in the order of j and walk r of s draws its choices from
 *   the key of address (s, 0, 0) and index r under (seed, G, S) with the chosen
 *   sampler, so the histograms depend only on the multiset of sources.
 *   d_endpoint[n] (int64): walks ending at each vertex after L steps.
 *   d_visits[n] (int64): visits at positions 1..L.
 *   Both outputs are overwritten (the library clears them on `stream`).
 *   stats may be NULL.
 *   Errors (SABA_E_INVALID; the outputs are then unspecified and the handle stays usable):
 *   a start outside 0 .. n-1 or on an isolated vertex, anywhere in the list; n_walks < 0,
 *   L < 0, G = 0, S > 31 or (G - 1) << S beyond 32 bits; an unknown mode, sampler or source
 *   mode; a null output or source array; n_walks >= 2^31 in either naive order.  SABA_E_OVERFLOW:
 *   n_walks * max(L, 1) >= 2^62, or n_walks >= 2^32 (a walk key holds a 32-bit index, so
 *   more walks from one start would repeat earlier ones).
 */
int saba_walks(saba_graph *g, const saba_walk_params *p, int64_t *d_endpoint, int64_t *d_visits,
               saba_stats *stats, void *stream);

/*
 * saba_walks for callers that cannot allocate device memory (tight serving loops, harnesses
 * that forbid hipMalloc): the same walks and the same histograms, bit for bit, with every
 * scratch buffer taken from a fixed 256 MiB region of
 * device memory that the library holds on each device until the process ends.  The call
 * makes no hipMalloc, hipFree or other allocating call; the caller passes d_endpoint and
 * d_visits (device, n int64 each) and the sources.  Only mode SABA_WALK_BOUQUET with
 * SABA_SOURCES_EXPLICIT is accepted; time_kernels is ignored (no events are created).
 * Scratch use: 8 n + 8 (n + 1) bytes for the start offsets, 4 W for the walk order, and the
 * visit log of a chunk of walks (chunks shrink to fit, down to 256 walks).  A call that does
 * not fit returns SABA_E_INVALID ("more scratch than the fixed region holds") before any walk
 * runs.  All calls on one device share the region: calls that overlap in time on one device
 * (other streams or threads) race and must not be issued.  Like saba_walks, the call clears
 * its outputs and counters with hipMemsetAsync and synchronises `stream` before it returns
 * (it reads the kernels' error flag), so it is not meant to be recorded into a HIP graph.
 * Errors: those of saba_walks, and SABA_E_INVALID for another mode or source mode.
 */
int saba_walks_noalloc(saba_graph *g, const saba_walk_params *p, int64_t *d_endpoint,
                       int64_t *d_visits, saba_stats *stats, void *stream);

/*
 * All-edges spanning centrality (Alg. 1, TGT+), SC(e) as defined in Sec. 2.1,
 * estimated to within eps with probability 1 - delta when group == 1.
 *   d_sc[m] (double): estimate of the i-th undirected edge in canonical order
 *   (u < v, lexicographic).  Errors: SABA_E_DISCONNECTED, SABA_E_BIPARTITE,
 *   SABA_E_INVALID (parameters), SABA_E_OVERFLOW (a directed edge needing 2^32 or more
 *   walk pairs: walk keys carry a 32-bit index).
 */
int saba_aesc(saba_graph *g, const saba_aesc_params *p, double *d_sc, saba_stats *stats,
              void *stream);

/*
 * Spanning centrality of a query edge set (Alg. 1 restricted to the sources
 * and directed edges the queries need).
 *   d_edges[2q] (int32, device): pairs (u, v) in either orientation; each must be
 *   an edge (SABA_E_NOT_EDGE).  d_sc[q] (double): the estimate of each pair,
 *   identical to saba_aesc's entry for the same edge and parameters.
 */
int saba_aesc_query(saba_graph *g, const saba_aesc_params *p, const int32_t *d_edges, int64_t q,
                    double *d_sc, saba_stats *stats, void *stream);

/*
 * Per-directed-edge internals of saba_aesc (for parity checks), indexed by CSR
 * position e (the edge s -> col_idx[e] of row s).  Any output may be NULL.
 *   d_tau[nnz] int32: truncation length; d_ttau[nnz] int32: deterministic levels of s;
 *   d_nreq[nnz] int64: walk pairs; d_D[nnz] double: deterministic part
 *   sum_{l <= min(ttau, tau)} (h_l(s) - h_l(t)); d_MC[nnz] double: sum over pairs of the
 *   walk statistic; d_vis0 / d_vis1[nnz] int64: walk positions of the walks from s / t
 *   that land where h_ttau is nonzero; d_g[nnz] double: directed estimate g(s, t) of the
 *   truncated series (without the eigenpair tail of omega > 0).
 *   d_sc[m] as in saba_aesc (may be NULL); it includes the tail when omega > 0.
 */
int saba_aesc_edge_stats(saba_graph *g, const saba_aesc_params *p, double *d_sc, int32_t *d_tau,
                         int32_t *d_ttau, int64_t *d_nreq, double *d_D, double *d_MC,
                         int64_t *d_vis0, int64_t *d_vis1, double *d_g, saba_stats *stats,
                         void *stream);

/*
 * The directed estimates of the edges out of a range of sources (Alg. 1's outer loop over the
 * sources src_begin .. src_end - 1): d_g[e] = g(s, col_idx[e]) for every CSR position e of
 * those rows (d_g is the caller's device array over all nnz positions; other entries are not
 * touched), exactly the entry saba_aesc_edge_stats writes.  A caller covers the sources in
 * pieces (for memory or progress) and forms SC with saba_aesc_combine; each source's
 * deterministic levels run once.  Errors: SABA_E_INVALID (range outside 0 .. n, an empty
 * range, omega > 0: the eigenpair tail belongs to the undirected edge, use saba_aesc), and
 * saba_aesc's errors.
 */
int saba_aesc_sources(saba_graph *g, const saba_aesc_params *p, int32_t src_begin,
                      int32_t src_end, double *d_g, saba_stats *stats, void *stream);

/*
 * Spanning centrality of all edges from directed estimates (Alg. 1's final combine):
 * d_sc[i] = d_g[e] + d_g[rev(e)] for the i-th canonical edge (u < v, lexicographic), e its CSR
 * position u -> v.  d_g[nnz] and d_sc[m] are device arrays; with d_g from saba_aesc_sources
 * over all sources, d_sc equals saba_aesc's output bit for bit (omega = 0).
 */
int saba_aesc_combine(saba_graph *g, const double *d_g, double *d_sc, void *stream);

/*
 * Integer visit counts of the walk pairs of Alg. 1 (its inner loop) for a list of sources,
 * for parity checks: the statistic X of a pair is sum_b h(W^s[b]) - sum_b h(W^t[b]) over
 * positions b = 1..L, so the Monte-Carlo sum of a directed edge (s, t) is
 * MC = sum over x in supp(h_ttau) of h_ttau(x) (c0(x) - c1(x)), where c0(x) and c1(x) count
 * the positions of the walks from s and from t that are at x.  These counts, the support and
 * h_ttau are exported exactly; the estimator itself sums h_ttau per walk.
 * layout[nsrc] (host): per source, `source` (vertex id, in) and, filled by the library:
 *   degree d_s, ttau, support |supp(h_ttau)|, and the offsets of a dense packing in list
 *   order: supp_off (into d_supp / d_h), edge_off (into the per-edge arrays) and hist_off.
 * Two calls.  Sizing: d_supp = d_h = d_hist = NULL; the library fills layout (the per-edge
 *   arrays may be given already).  Totals: supp_off + support, edge_off + degree and
 *   hist_off + 2 degree support of the last entry.
 * Filling: all three given (device), with the layout of the sizing call for the same graph
 *   and parameters:
 *   d_supp[] int32: the support of each source, ascending vertex ids;
 *   d_h[] double: h_ttau at those vertices;
 *   d_hist[] int64: entry hist_off + (2 i + side) support + p counts the positions of the
 *   side-`side` walks (0: from s, 1: from t = the i-th neighbour of s in row order) of edge i
 *   that are at the p-th support vertex.
 * Per-edge outputs (device, entry edge_off + i; any may be NULL in either call): d_tau int32,
 * d_nreq int64, d_D double, d_MC double (the estimator's own per-walk sum), d_vis0 / d_vis1
 * int64 (the totals of the two histograms), d_g double, as saba_aesc_edge_stats defines them.
 * Every value equals what saba_aesc computes for that source and edge.
 * Errors: SABA_E_INVALID (empty or repeated source list, an isolated or out-of-range source,
 * partial outputs, a layout that is not the sizing call's), and saba_aesc's errors.
 */
typedef struct saba_count_source {
    int32_t source;
    int32_t degree;
    int32_t ttau;
    int32_t reserved;
    int64_t support;
    int64_t supp_off;
    int64_t edge_off;
    int64_t hist_off;
} saba_count_source;

int saba_aesc_counts(saba_graph *g, const saba_aesc_params *p, saba_count_source *layout,
                     int32_t nsrc, int32_t *d_supp, double *d_h, int64_t *d_hist, int32_t *d_tau,
                     int64_t *d_nreq, double *d_D, double *d_MC, int64_t *d_vis0,
                     int64_t *d_vis1, double *d_g, saba_stats *stats, void *stream);

/*
 * Several estimator requests evaluated together (Alg. 1 for each): batched multi-graph
 * estimation and the shared launches of the query server.  Requests with equal graph and
 * parameters share their source instances; every instance of every request runs in the same
 * batches and walk launches.  Each request's d_sc receives exactly what saba_aesc (q = -1) or
 * saba_aesc_query (q >= 0) returns for that graph and parameters alone.  opt may be NULL.
 * Errors as saba_aesc / saba_aesc_query; no output is written when a request is invalid.
 */
int saba_aesc_batch(saba_graph *g, const saba_aesc_request *reqs, int32_t nreq,
                    const saba_batch_options *opt, saba_stats *stats, void *stream);

/*
 * Query server over a resident handle: spanning-centrality requests (edge sets of one graph
 * at given parameters; per-edge estimates are independent, Sec. 2.1) are admitted as they
 * arrive and their sources are batched together into shared launches (Alg. 1 per source).
 * The server owns host threads (one per lane), one HIP stream per lane, and device scratch
 * within opt->mem_budget plus the result arena.  g must outlive the server.  Other calls on
 * g may run meanwhile from one other thread (they use the handle's own scratch).
 * opt may be NULL.  *out receives the server (NULL on failure).
 */
int saba_server_create(saba_graph *g, const saba_server_options *opt, saba_server **out);

/*
 * Submit one request; never blocks on the GPU.  The pairs are validated here (SABA_E_NOT_EDGE,
 * SABA_E_INVALID, SABA_E_DISCONNECTED, SABA_E_BIPARTITE, SABA_E_OVERFLOW when eps is too small
 * for tau_cap, SABA_E_NOMEM when one source of the graph exceeds a lane's budget) and
 * SABA_E_BUSY is returned while the admission queue is full.  On SABA_OK *ticket names the
 * request until saba_server_wait reports it finished.  Its d_sc receives exactly what
 * saba_aesc_query returns for the same graph and parameters alone.
 */
int saba_server_submit(saba_server *srv, const saba_server_request *req, uint64_t *ticket);

/*
 * Wait up to timeout_ms (< 0: without limit; 0: poll) for a request to finish.  Returns
 * SABA_OK when it finished and its d_sc is written (visible to every stream), the request's
 * error when it failed, SABA_E_TIMEOUT when it has not finished (the ticket stays valid), or
 * SABA_E_INVALID for an unknown ticket.  Once a finished request is reported its ticket is
 * released.  res may be NULL.
 */
int saba_server_wait(saba_server *srv, uint64_t ticket, int32_t timeout_ms,
                     saba_server_result *res);

/* Fill *out with the server's counters. */
int saba_server_stats(saba_server *srv, saba_server_stats_t *out);

/*
 * Stop the server: requests not yet in a batch finish with SABA_E_CANCELLED, running batches
 * complete, the lanes are joined and every resource is freed.  No other call on srv may be in
 * progress or follow.  NULL is accepted.
 */
int saba_server_destroy(saba_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SABA_H */

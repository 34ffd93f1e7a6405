// Query server: continuous batching of spanning-centrality requests over a resident handle.
//
// Per-edge estimates are independent of each other (Sec. 2.1: SC of an edge is a property of
// that edge alone), and everything the estimator computes for a source depends only on
// (graph, parameters, source), so the work of many requests can be cut into source instances
// and regrouped freely.  The server does exactly that:
//
//   submit   validates a request on the calling thread (parameters, every pair an edge of its
//            graph), splits it into instances (one per distinct endpoint, listing the directed
//            edges it must estimate) and appends it to the arrival queue.  The queue is
//            bounded in query edges: beyond the bound submit fails with SABA_E_BUSY.
//   admit    moves arrivals, in order, into the instance queue as soon as the result arena
//            has room for their 2q directed estimates.
//   lanes    each lane is a host thread with its own HIP stream and scratch.  A lane takes
//            instances from the front of the queue until its share of the memory budget is
//            used (each instance costs the dense scratch of its graph), runs them as one batch
//            (shared deterministic levels and one walk launch for all of them), and scatters
//            the directed estimates into the arena.  Lanes run concurrently, so the batches of
//            different lanes overlap on the device, and a request that arrives while batches
//            run joins the next batch any lane forms.
//   finish   when the last instance of a request is done, its results SC = g(u,v) + g(v,u) are
//            written to the caller's output and waiters are woken.
//
// A request's result is bit-identical to saba_aesc_query for the same graph and parameters:
// instance results do not depend on the batch they ran in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "estimator.hpp"

namespace saba {
namespace {

using Clock = std::chrono::steady_clock;

__global__ void scatter_kernel(const int64_t *__restrict__ map, int64_t n,
                               const double *__restrict__ g, double *__restrict__ arena) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        arena[map[2 * i + 1]] = g[map[2 * i]];
}

// SC of pair j from its two directed estimates, plus (omega > 0) the eigenpair tail the
// batches left at a[2q + j]; the same additions in the same order as the synchronous calls.
__global__ void finalize_arena_kernel(const double *__restrict__ a, int64_t q, int has_tail,
                                      double *__restrict__ sc) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q;
         j += (int64_t)gridDim.x * blockDim.x) {
        double v = a[2 * j] + a[2 * j + 1];
        if (has_tail) v += a[2 * q + j];
        sc[j] = v;
    }
}

// Eigenpair tails (omega > 0) of the pairs whose first directed edge ran in this batch:
// entry i = (instance edge, arena position, u | v graph-local, theta, y, n of the graph,
// kept pairs); tau is the batch's tau of that instance edge (symmetric in the pair).
__global__ void tail_scatter_kernel(const int64_t *__restrict__ tm, int64_t n,
                                    const int32_t *__restrict__ tau, double *__restrict__ arena) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t *m = tm + 7 * i;
        const int32_t u = (int32_t)(m[2] >> 32), v = (int32_t)(m[2] & 0xffffffffll);
        arena[m[1]] = eigen_tail(reinterpret_cast<const double *>(m[3]),
                                 reinterpret_cast<const double *>(m[4]), m[5], (int32_t)m[6], u,
                                 v, tau[m[0]]);
    }
}

struct Req;

struct Inst {                      // one source instance of a request
    std::shared_ptr<Req> req;
    int32_t v = 0;                 // handle vertex id
    std::vector<int64_t> want;     // (row position, arena entry within the request) pairs
};

struct Req {
    uint64_t ticket = 0;
    int32_t graph = 0;
    PSet ps{};
    SlotSize sz{};
    int64_t q = 0;
    double *d_sc = nullptr;
    std::vector<Inst> insts;       // until admitted
    int64_t ninst = 0;
    int64_t remaining = 0;
    int64_t arena_off = -1;
    int64_t arena_len = 0;             // 2q, or 3q with the eigenpair tails (omega > 0)
    const Spectrum *spec = nullptr;    // kept eigenpairs of the omega > 0 correction
    int32_t status = SABA_OK;
    std::string err;
    int32_t batches = 0;
    int64_t last_batch = -1;
    bool done = false;
    Clock::time_point t_submit, t_admit, t_done;
};

// First-fit allocator over the result arena (entries of 8 bytes).
struct Arena {
    std::map<int64_t, int64_t> free;  // offset -> length
    void init(int64_t n) {
        free.clear();
        if (n > 0) free[0] = n;
    }
    int64_t alloc(int64_t n) {
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < n) continue;
            const int64_t off = it->first, len = it->second;
            free.erase(it);
            if (len > n) free[off + n] = len - n;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t n) {
        if (n <= 0) return;
        auto it = free.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

struct Lane {
    hipStream_t s = nullptr;
    Workspace ws;
    DevBuf map;
    DevBuf tmap;  // tail entries of a batch (omega > 0 requests)
    std::thread th;
};

}  // namespace

struct Server {
    Graph *g = nullptr;
    int64_t lane_budget = 0, max_queued_edges = 0, arena_edges = 0;
    int32_t nlanes = 0, max_batch = 0;
    DevBuf arena_buf;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Req>> arrivals;
    std::deque<Inst> pending;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> live;
    uint64_t next_ticket = 1;
    int64_t next_batch = 0;
    bool stopping = false;
    saba_server_stats_t st{};
    std::vector<std::unique_ptr<Lane>> lanes;

    void admit_locked();
    void take_batch_locked(std::vector<Inst> &batch, int64_t *id);
    int exec_batch(Lane &ln, std::vector<Inst> &batch, int64_t *steps);
    void complete(Lane &ln, std::vector<Inst> &batch, int64_t id, int rc, const std::string &msg);
    void lane_main(Lane *ln);
};

void Server::admit_locked() {
    while (!arrivals.empty()) {
        const std::shared_ptr<Req> &r = arrivals.front();
        const int64_t off = arena.alloc(r->arena_len);
        if (off < 0) break;  // in order: later arrivals wait for the arena too
        r->arena_off = off;
        r->t_admit = Clock::now();
        for (auto &x : r->insts) pending.push_back(std::move(x));
        r->insts.clear();
        r->insts.shrink_to_fit();
        arrivals.pop_front();
    }
}

void Server::take_batch_locked(std::vector<Inst> &batch, int64_t *id) {
    batch.clear();
    int64_t bytes = 0;
    while (!pending.empty() && (int64_t)batch.size() < max_batch) {
        const int64_t b = pending.front().req->sz.bytes;
        if (!batch.empty() && bytes + b > lane_budget) break;
        bytes += b;
        batch.push_back(std::move(pending.front()));
        pending.pop_front();
    }
    *id = next_batch++;
}

int Server::exec_batch(Lane &ln, std::vector<Inst> &batch, int64_t *steps) {
    const int32_t *rp = g->h_row_ptr.data();
    hipStream_t s = ln.s;
    const int32_t nb = (int32_t)batch.size();
    std::vector<PSet> ps;
    std::vector<Slot> slots(nb);
    std::vector<int64_t> eb(nb + 1);
    std::vector<int64_t> map, tmap;
    int64_t ne = 0, ho = 0, bo = 0, so = 0, hubs = 0, maxgn = 1;
    for (int32_t b = 0; b < nb; ++b) {
        const Inst &x = batch[b];
        const Req &r = *x.req;
        int32_t pid = -1;
        if (!ps.empty() && same_pset(ps.back(), r.ps)) pid = (int32_t)ps.size() - 1;
        for (int32_t k = 0; pid < 0 && k < (int32_t)ps.size(); ++k)
            if (same_pset(ps[k], r.ps)) pid = k;
        if (pid < 0) {
            pid = (int32_t)ps.size();
            ps.push_back(r.ps);
        }
        Slot &sl = slots[b];
        sl.hoff = ho;
        sl.bmoff = bo;
        sl.sboff = so;
        sl.ie = ne;
        sl.inst = b;
        sl.v = x.v;
        sl.p = pid;
        sl.goff = g->goff[r.graph];
        sl.gn = g->goff[r.graph + 1] - sl.goff;
        sl.gpos = rp[sl.goff];
        sl.pad = 0;
        ho += r.sz.h;
        bo += r.sz.bm;
        so += r.sz.sb;
        hubs += r.sz.hubs;
        maxgn = std::max<int64_t>(maxgn, sl.gn);
        eb[b] = ne;
        for (size_t k = 0; k < x.want.size(); k += 2) {
            map.push_back(ne + x.want[k]);
            map.push_back(r.arena_off + x.want[k + 1]);
            if (r.spec && r.spec->pairs > 0 && (x.want[k + 1] & 1) == 0) {
                // the pair's first directed edge carries its tail
                const int64_t j = x.want[k + 1] >> 1;
                const int32_t u = x.v - sl.goff;
                const int32_t v = g->h_col_idx[rp[x.v] + x.want[k]] - sl.goff;
                tmap.push_back(ne + x.want[k]);
                tmap.push_back(r.arena_off + 2 * r.q + j);
                tmap.push_back(((int64_t)u << 32) | (int64_t)(uint32_t)v);
                tmap.push_back((int64_t)reinterpret_cast<uintptr_t>(r.spec->d_theta()));
                tmap.push_back((int64_t)reinterpret_cast<uintptr_t>(r.spec->d_y()));
                tmap.push_back(sl.gn);
                tmap.push_back(r.spec->pairs);
            }
        }
        ne += rp[x.v + 1] - rp[x.v];
    }
    eb[nb] = ne;
    std::vector<uint8_t> want((size_t)std::max<int64_t>(ne, 1), 0);
    for (size_t k = 0; k < map.size(); k += 2) want[map[k]] = 1;
    const int64_t nmap = (int64_t)map.size() / 2;

    EdgeArrays ea;
    SABA_TRY(ensure_edge_arrays(ln.ws, ne, nb, (int32_t)ps.size(), &ea));
    SABA_TRY(ln.map.ensure(sizeof(int64_t) * std::max<size_t>(map.size(), 2)));
    SABA_HIP_TRY(hipMemcpyAsync(const_cast<PSet *>(ea.psets), ps.data(), sizeof(PSet) * ps.size(),
                                hipMemcpyHostToDevice, s));
    SABA_HIP_TRY(hipMemcpyAsync(const_cast<uint8_t *>(ea.want), want.data(), want.size(),
                                hipMemcpyHostToDevice, s));
    if (nmap > 0)
        SABA_HIP_TRY(hipMemcpyAsync(ln.map.ptr, map.data(), sizeof(int64_t) * map.size(),
                                    hipMemcpyHostToDevice, s));
    SABA_HIP_TRY(hipMemsetAsync(ea.fl, 0, sizeof(Flags), s));
    SABA_TRY(ensure_pools(ln.ws, ho, bo, so, hubs, nb, ne, s));
    SABA_TRY(run_batch(g, ln.ws, ea, slots, eb, 0, ne, maxgn, hubs, nullptr, s));
    if (nmap > 0) {
        scatter_kernel<<<grid_for(nmap, 256, 1 << 14), 256, 0, s>>>(
            ln.map.as<int64_t>(), nmap, ea.g, arena_buf.as<double>());
        SABA_HIP_TRY(hipGetLastError());
    }
    const int64_t ntail = (int64_t)tmap.size() / 7;
    if (ntail > 0) {
        SABA_TRY(ln.tmap.ensure(sizeof(int64_t) * tmap.size()));
        SABA_HIP_TRY(hipMemcpyAsync(ln.tmap.ptr, tmap.data(), sizeof(int64_t) * tmap.size(),
                                    hipMemcpyHostToDevice, s));
        tail_scatter_kernel<<<grid_for(ntail, 256, 1 << 14), 256, 0, s>>>(
            ln.tmap.as<int64_t>(), ntail, ea.tau, arena_buf.as<double>());
        SABA_HIP_TRY(hipGetLastError());
    }
    Flags hf;
    SABA_HIP_TRY(hipMemcpyAsync(&hf, ea.fl, sizeof(Flags), hipMemcpyDeviceToHost, s));
    SABA_HIP_TRY(hipStreamSynchronize(s));
    *steps = (int64_t)hf.walk_steps;
    return SABA_OK;
}

void Server::complete(Lane &ln, std::vector<Inst> &batch, int64_t id, int rc,
                      const std::string &msg) {
    std::vector<std::shared_ptr<Req>> fin;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (Inst &x : batch) {
            Req &r = *x.req;
            if (rc != SABA_OK && r.status == SABA_OK) {
                r.status = rc;
                r.err = msg;
            }
            if (r.last_batch != id) {
                r.last_batch = id;
                r.batches += 1;
            }
            if (--r.remaining == 0) fin.push_back(x.req);
        }
    }
    batch.clear();
    if (fin.empty()) return;
    int frc = SABA_OK;
    std::string fmsg;
    for (auto &r : fin) {
        if (r->status != SABA_OK || r->q == 0) continue;
        finalize_arena_kernel<<<grid_for(r->q, 256, 1 << 14), 256, 0, ln.s>>>(
            arena_buf.as<double>() + r->arena_off, r->q, r->arena_len > 2 * r->q ? 1 : 0,
            r->d_sc);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ln.s);
    if (e != hipSuccess) {
        frc = SABA_E_HIP;
        fmsg = std::string("finishing a request: ") + hipGetErrorString(e);
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto now = Clock::now();
        for (auto &r : fin) {
            if (frc != SABA_OK && r->status == SABA_OK) {
                r->status = frc;
                r->err = fmsg;
            }
            r->done = true;
            r->t_done = now;
            arena.release(r->arena_off, r->arena_len);
            st.queued_edges -= r->q;
            st.queued_requests -= 1;
            if (r->status == SABA_OK)
                st.completed += 1;
            else
                st.failed += 1;
        }
    }
    cv_done.notify_all();
    cv_work.notify_all();  // arena room may admit waiting arrivals
}

void Server::lane_main(Lane *ln) {
    (void)hipSetDevice(g->device);
    std::vector<Inst> batch;
    for (;;) {
        int64_t id = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stopping) return;
                admit_locked();
                if (!pending.empty()) break;
                cv_work.wait(lk);
            }
            take_batch_locked(batch, &id);
            if (!pending.empty()) cv_work.notify_one();
        }
        const auto t0 = Clock::now();
        int64_t steps = 0;
        clear_error();
        const int rc = exec_batch(*ln, batch, &steps);
        const std::string msg = rc == SABA_OK ? std::string() : std::string(saba_last_error());
        if (rc != SABA_OK) {
            // a failed batch may leave work queued on the stream: drain it before the
            // arena entries of its requests are reused
            (void)hipStreamSynchronize(ln->s);
            (void)hipGetLastError();
        }
        const double ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        {
            std::lock_guard<std::mutex> lk(mu);
            st.batches += 1;
            st.instances += (int64_t)batch.size();
            st.walk_steps += steps;
            st.busy_ms += ms;
        }
        complete(*ln, batch, id, rc, msg);
    }
}

}  // namespace saba

using namespace saba;

namespace {

int find_pos(const Graph *g, int32_t u, int32_t v) {
    const int32_t *rp = g->h_row_ptr.data(), *ci = g->h_col_idx.data();
    const int32_t *a = ci + rp[u], *z = ci + rp[u + 1];
    const int32_t *f = std::lower_bound(a, z, v);
    return (f != z && *f == v) ? (int32_t)(f - a) : -1;  // position within the row
}

void shutdown(Server *sv) {
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
        const auto now = Clock::now();
        auto cancel = [&](Req &r) {
            if (r.status == SABA_OK) {
                r.status = SABA_E_CANCELLED;
                r.err = "the server was destroyed before the request finished";
            }
        };
        for (auto &r : sv->arrivals) {
            cancel(*r);
            r->insts.clear();  // its instances hold the request: break the cycle
            r->remaining = 0;
            r->done = true;
            r->t_done = now;
        }
        sv->arrivals.clear();
        for (Inst &x : sv->pending) {
            cancel(*x.req);
            if (--x.req->remaining == 0) {
                x.req->done = true;
                x.req->t_done = now;
            }
        }
        sv->pending.clear();
    }
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
    for (auto &ln : sv->lanes)
        if (ln->th.joinable()) ln->th.join();
    for (auto &ln : sv->lanes) {
        if (ln->s) (void)hipStreamSynchronize(ln->s);
        ln->ws.release();
        ln->map.release();
        ln->tmap.release();
        if (ln->s) (void)hipStreamDestroy(ln->s);
        ln->s = nullptr;
    }
    sv->arena_buf.release();
}

}  // namespace

extern "C" int saba_server_create(saba_graph *gh, const saba_server_options *opt,
                                  saba_server **out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return SABA_E_INVALID;
    }
    *out = nullptr;
    SABA_TRY(check_graph(gh));
    saba_server_options o{};
    if (opt) o = *opt;
    if (o.lanes < 0 || o.lanes > 8 || o.max_batch_sources < 0 || o.max_batch_sources > 65535 ||
        o.mem_budget < 0 || o.max_queued_edges < 0 || o.arena_edges < 0) {
        set_error("invalid server options");
        return SABA_E_INVALID;
    }
    Graph *g = G(gh);
    SABA_HIP_TRY(hipSetDevice(g->device));
    size_t freeb = 0, totalb = 0;
    SABA_HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    std::unique_ptr<Server> sv(new Server);
    sv->g = g;
    sv->nlanes = o.lanes > 0 ? o.lanes : 2;
    const int64_t budget = o.mem_budget > 0
                               ? o.mem_budget
                               : std::min<int64_t>(32ll << 30, (int64_t)(0.4 * (double)freeb));
    sv->lane_budget = budget / sv->nlanes;
    sv->max_queued_edges = o.max_queued_edges > 0 ? o.max_queued_edges : (1ll << 20);
    sv->arena_edges = o.arena_edges > 0 ? o.arena_edges : (1ll << 22);
    sv->max_batch = o.max_batch_sources > 0 ? o.max_batch_sources : 4096;
    SABA_TRY(sv->arena_buf.ensure(sizeof(double) * 2 * (size_t)sv->arena_edges));
    sv->arena.init(2 * sv->arena_edges);
    for (int32_t i = 0; i < sv->nlanes; ++i) {
        std::unique_ptr<Lane> ln(new Lane);
        hipError_t e = hipStreamCreateWithFlags(&ln->s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ln->s = nullptr;
            shutdown(sv.get());
            set_error(std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
            return SABA_E_HIP;
        }
        sv->lanes.push_back(std::move(ln));
    }
    // Pools at their largest under a lane's budget, allocated and zeroed once here so that no
    // batch reallocates them (a reallocation would also stall the other lanes).  A pool entry
    // count over any batch is bounded by the budget times the best entries-per-byte ratio of a
    // graph, plus one slot, and by max_batch slots of the largest graph.
    {
        double rh = 0.0, rbm = 0.0, rsb = 0.0, rhub = 0.0;
        int64_t mh = 0, mbm = 0, msb = 0, mhub = 0;
        for (int32_t k = 0; k < g->ngraphs; ++k) {
            const SlotSize z = slot_size(g, k);
            if (z.bytes <= 0) continue;
            rh = std::max(rh, (double)z.h / (double)z.bytes);
            rbm = std::max(rbm, (double)z.bm / (double)z.bytes);
            rsb = std::max(rsb, (double)z.sb / (double)z.bytes);
            rhub = std::max(rhub, (double)z.hubs / (double)z.bytes);
            mh = std::max(mh, z.h);
            mbm = std::max(mbm, z.bm);
            msb = std::max(msb, z.sb);
            mhub = std::max(mhub, z.hubs);
        }
        auto cap = [&](double ratio, int64_t mx) {
            const double by_budget = ratio * (double)sv->lane_budget + (double)mx;
            const double by_count = (double)sv->max_batch * (double)mx;
            return (int64_t)std::min(by_budget, by_count);
        };
        const int64_t ph = cap(rh, mh), pbm = cap(rbm, mbm), psb = cap(rsb, msb);
        const int64_t phub = cap(rhub, mhub);
        for (auto &ln : sv->lanes) {
            int rc = ensure_pools(ln->ws, ph, pbm, psb, phub, sv->max_batch,
                                  (int64_t)sv->max_batch * 64, ln->s);
            if (rc == SABA_OK && hipStreamSynchronize(ln->s) != hipSuccess) {
                set_error("zeroing the server's pools failed");
                rc = SABA_E_HIP;
            }
            if (rc != SABA_OK) {
                const std::string msg = saba_last_error();
                shutdown(sv.get());
                set_error(msg);
                return rc;
            }
        }
    }
    try {
        for (auto &ln : sv->lanes) ln->th = std::thread(&Server::lane_main, sv.get(), ln.get());
    } catch (...) {
        shutdown(sv.get());
        set_error("could not start the server's lane threads");
        return SABA_E_NOMEM;
    }
    *out = reinterpret_cast<saba_server *>(sv.release());
    return SABA_OK;
}

extern "C" int saba_server_submit(saba_server *sh, const saba_server_request *rq,
                                  uint64_t *ticket) {
    clear_error();
    Server *sv = reinterpret_cast<Server *>(sh);
    if (!sv || !rq || !ticket || rq->q < 0 || (rq->q > 0 && (!rq->edges || !rq->d_sc))) {
        set_error("invalid request (the server takes q >= 0 query pairs and an output)");
        return SABA_E_INVALID;
    }
    const auto t_entry = Clock::now();
    Graph *g = sv->g;
    {
        // refuse cheaply while the queue is full, before the pairs are validated
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->st.queued_edges > 0 && sv->st.queued_edges + rq->q > sv->max_queued_edges) {
            sv->st.rejected += 1;
            set_error("the admission queue is full");
            return SABA_E_BUSY;
        }
    }
    saba_aesc_params prm = rq->params;
    const Spectrum *spec = nullptr;
    if (rq->graph >= 0 && rq->graph < g->ngraphs && g->gconnected[rq->graph]) {
        const int32_t gn = g->goff[rq->graph + 1] - g->goff[rq->graph];
        const bool eig = prm.omega > 0 && prm.omega <= kMaxOmega && prm.omega < gn &&
                         !g->gbipartite[rq->graph];
        if (eig || (prm.omega == 0 && prm.lambda <= 0.0)) {
            // the spectral input, computed once per graph (and omega) on a private stream and
            // cached: the kept eigenpairs and the radius of the rest, or lambda
            hipStream_t ls = nullptr;
            SABA_HIP_TRY(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));
            const int rc = eig ? resolve_spectrum(g, rq->graph, prm.omega, &spec, ls)
                               : resolve_lambda(g, rq->graph, &prm.lambda, ls);
            (void)hipStreamDestroy(ls);
            SABA_TRY(rc);
            if (eig && prm.lambda <= 0.0)
                prm.lambda = std::min(std::max(spec->lambda_rest_bound, DBL_MIN), 1.0 - 1e-12);
        }
    }
    SABA_TRY(check_request(g, rq->graph, prm, rq->q, rq->edges));
    const int64_t arena_len = (spec && spec->pairs > 0 ? 3 : 2) * rq->q;
    if (arena_len > 2 * sv->arena_edges) {
        set_error("the request has more pairs than the server's result arena holds");
        return SABA_E_INVALID;
    }
    auto r = std::make_shared<Req>();
    r->graph = rq->graph;
    r->ps = make_pset(g, rq->graph, prm);
    r->sz = slot_size(g, rq->graph);
    r->q = rq->q;
    r->d_sc = rq->d_sc;
    r->spec = spec;
    r->arena_len = arena_len;
    // NWalks <= c * tau_cap^2 (q = L hmax / d_s <= L <= tau_cap): rule out an overflow of the
    // walk counts here, so that no batch can fail on behalf of another request
    if (!(r->ps.c * (double)r->ps.tau_cap * (double)r->ps.tau_cap < 4.0e18)) {
        set_error("walk counts may overflow the 64-bit range (eps too small for tau_cap)");
        return SABA_E_OVERFLOW;
    }
    if (r->sz.bytes > sv->lane_budget) {
        set_error("one source of this graph needs more scratch than a lane's memory budget");
        return SABA_E_NOMEM;
    }
    // instances: one per distinct endpoint, listing (row position, arena entry) pairs
    const int32_t ga = g->goff[rq->graph], gn = g->goff[rq->graph + 1] - ga;
    struct E {
        int32_t v, pos;
        int64_t slot;
    };
    std::vector<E> ent((size_t)(2 * rq->q));
    for (int64_t j = 0; j < rq->q; ++j) {
        const int32_t u = rq->edges[2 * j], v = rq->edges[2 * j + 1];
        const int32_t puv = (u >= 0 && v >= 0 && u < gn && v < gn) ? find_pos(g, ga + u, ga + v)
                                                                    : -1;
        if (puv < 0) {
            set_error("a query pair is not an edge of the graph");
            return SABA_E_NOT_EDGE;
        }
        ent[2 * j] = E{ga + u, puv, 2 * j};
        ent[2 * j + 1] = E{ga + v, find_pos(g, ga + v, ga + u), 2 * j + 1};
    }
    std::sort(ent.begin(), ent.end(), [](const E &a, const E &b) {
        return a.v != b.v ? a.v < b.v : a.slot < b.slot;
    });
    for (size_t k = 0; k < ent.size();) {
        Inst x;
        x.req = r;
        x.v = ent[k].v;
        for (; k < ent.size() && ent[k].v == x.v; ++k) {
            x.want.push_back(ent[k].pos);
            x.want.push_back(ent[k].slot);
        }
        r->insts.push_back(std::move(x));
    }
    r->ninst = (int64_t)r->insts.size();
    r->remaining = r->ninst;
    r->t_submit = t_entry;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stopping) {
            set_error("the server is shutting down");
            return SABA_E_CANCELLED;
        }
        if (sv->st.queued_edges > 0 && sv->st.queued_edges + r->q > sv->max_queued_edges) {
            sv->st.rejected += 1;
            set_error("the admission queue is full");
            return SABA_E_BUSY;
        }
        r->ticket = sv->next_ticket++;
        *ticket = r->ticket;
        sv->live[r->ticket] = r;
        sv->st.submitted += 1;
        if (r->q == 0) {
            r->done = true;
            r->t_admit = r->t_done = r->t_submit;
            sv->st.completed += 1;
            return SABA_OK;
        }
        sv->arrivals.push_back(r);
        sv->st.queued_edges += r->q;
        sv->st.queued_requests += 1;
        sv->st.peak_queued_edges = std::max(sv->st.peak_queued_edges, sv->st.queued_edges);
    }
    sv->cv_work.notify_one();
    return SABA_OK;
}

extern "C" int saba_server_wait(saba_server *sh, uint64_t ticket, int32_t timeout_ms,
                                saba_server_result *res) {
    clear_error();
    Server *sv = reinterpret_cast<Server *>(sh);
    if (!sv) {
        set_error("server is NULL");
        return SABA_E_INVALID;
    }
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) {
        set_error("unknown ticket");
        return SABA_E_INVALID;
    }
    std::shared_ptr<Req> r = it->second;
    auto pred = [&] { return r->done; };
    if (timeout_ms < 0)
        sv->cv_done.wait(lk, pred);
    else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
        set_error("the request has not finished yet");
        return SABA_E_TIMEOUT;
    }
    if (res) {
        res->status = r->status;
        res->batches = r->batches;
        res->instances = r->ninst;
        const auto ta = r->arena_off >= 0 ? r->t_admit : r->t_done;
        res->queue_ms = std::chrono::duration<double, std::milli>(ta - r->t_submit).count();
        res->latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    }
    sv->live.erase(it);
    if (r->status != SABA_OK) set_error(r->err);
    return r->status;
}

extern "C" int saba_server_stats(saba_server *sh, saba_server_stats_t *out) {
    clear_error();
    Server *sv = reinterpret_cast<Server *>(sh);
    if (!sv || !out) {
        set_error("server or out is NULL");
        return SABA_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    return SABA_OK;
}

extern "C" int saba_server_destroy(saba_server *sh) {
    clear_error();
    Server *sv = reinterpret_cast<Server *>(sh);
    if (!sv) return SABA_OK;
    shutdown(sv);
    delete sv;
    return SABA_OK;
}

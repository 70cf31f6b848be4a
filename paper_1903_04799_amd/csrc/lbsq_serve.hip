// lbsq_serve.hip -- many resident simulations advanced together: the
// lb_step_batch call and the continuous-batching server (lb_server_*) of
// include/lbsq.h.
//
// Both run the step kernels over a table of simulation descriptors: each
// step is one fluid launch and one geometry launch whose blocks are divided
// among the simulations (contiguous ranges per simulation), so a batch costs
// two launches per step however many simulations it holds.  A simulation's
// descriptor fixes its time levels (t = t0 + k for step k of a launch
// sequence), so a chunk of steps can be captured once as a HIP graph and
// replayed for as long as the set of resident simulations stays the same.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "lbsq_sim.h"

using namespace lbsq;

namespace {

// Block ranges of a batch and the largest body count (LDS size).
struct Batch {
    BatchMap map;
    int nbody_max;
};

Batch make_batch(lb_sim *const *sims, int n)
{
    Batch b;
    std::memset(&b, 0, sizeof(b));
    b.map.nsim = n;
    for (int j = 0; j < n; ++j) {
        uint32_t f = 0, g = 0;
        lbsq_sim_blocks(sims[j], &f, &g);
        b.map.fluid0[j + 1] = b.map.fluid0[j] + f;
        b.map.geo0[j + 1] = b.map.geo0[j] + g;
        b.nbody_max = std::max(b.nbody_max, int(sims[j]->bodies.size()));
    }
    return b;
}

// Steps k = 0 .. K-1 of a batch whose descriptors are on the device.
hipError_t enqueue_steps(int storage, const SimDesc *d_desc, const Batch &b, int K, hipStream_t st)
{
    BatchLaunch L;
    std::memset(&L, 0, sizeof(L));
    L.desc = d_desc;
    L.map = b.map;
    L.nbody_max = b.nbody_max;
    L.stream = st;
    for (int k = 0; k < K; ++k) {
        L.k = k;
        const hipError_t e = launch_batch_step(storage, L);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Can this handle share a batched launch with others of the same storage?
bool batchable(const lb_sim *s)
{
    const bool force = s->args.g[0] != 0.0f || s->args.g[1] != 0.0f || s->args.g[2] != 0.0f;
    return !force && s->p.audit_every == 0 && !s->timing && int(s->bodies.size()) <= FUSE_MAX;
}

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// the serving loop

namespace {

// First-fit allocator over one device allocation (256-byte granules);
// neighbouring free ranges are merged.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_, used_;  // offset -> bytes

    void reset(char *b, size_t n)
    {
        base = b;
        size = n;
        free_.clear();
        used_.clear();
        free_[0] = n;
    }
    void *alloc(size_t bytes)
    {
        bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > bytes) free_[off + bytes] = sz - bytes;
            used_[off] = bytes;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p)
    {
        if (!p) return;
        const size_t off = size_t(static_cast<char *>(p) - base);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t sz = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + sz) {
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += sz;
                return;
            }
        }
        free_[off] = sz;
    }
    size_t in_use() const
    {
        size_t t = 0;
        for (const auto &u : used_) t += u.second;
        return t;
    }
};

struct Job {
    uint64_t ticket = 0;
    lb_request rq{};
    double t_submit = 0.0, t_admit = 0.0;
    lb_sim *sim = nullptr;
    uint64_t fluid = 0;
    bool cancelled = false;  // left the batch early; ends as LB_ECANCELED
};

struct Chunk {
    hipEvent_t ev = nullptr;
    hipGraphExec_t exec = nullptr;  // the graph this chunk replayed, if any
    std::vector<Job *> done;        // requests whose last step is in this chunk
};

constexpr int RING = 3;      // pinned descriptor tables (two chunks queued at most)
constexpr int MAX_QUEUED = 2;

}  // namespace

struct lb_server {
    lb_server_params p{};
    int device = 0;
    hipStream_t stream = nullptr, setup = nullptr, capture = nullptr;
    bool own_stream = false;
    Arena arena;
    void *arena_mem = nullptr;
    uint64_t next_ticket = 1;
    std::deque<Job *> queue;
    std::vector<Job *> active;
    std::deque<Chunk> inflight;
    std::deque<lb_result> results;
    SimDesc *d_desc = nullptr;  // descriptors read by the chunk kernels
    SimDesc *h_desc = nullptr;  // RING pinned tables of MAXSIM descriptors
    int ring = 0;
    hipEvent_t setup_ev = nullptr;
    hipGraphExec_t exec = nullptr;  // graph of the current set of requests
    std::vector<uint32_t> exec_key;
    lb_server_stats stats{};
    std::chrono::steady_clock::time_point t0;
};

namespace {

void *arena_alloc(size_t bytes, void *ctx) { return static_cast<lb_server *>(ctx)->arena.alloc(bytes); }
void arena_free(void *p, void *ctx) { static_cast<lb_server *>(ctx)->arena.release(p); }

// Device bytes a request needs (each allocation of the handle rounded to
// the arena granule), for rejecting requests that can never fit.
size_t request_bytes(const lb_request *rq, int storage)
{
    auto g = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); };
    const uint64_t n = uint64_t(rq->nx) * rq->ny * rq->nz;
    const uint64_t stride = ((n + 255) / 256) * 256 + 256;
    const size_t es = storage == LB_STORAGE_F32 ? 4 : 2;
    const uint64_t nblk = (n + BLOCK - 1) / BLOCK;
    size_t t = g(size_t(Q) * stride * es) + 2 * g(n * sizeof(float)) + 2 * g(n) + 2 * g(MAXB * sizeof(DevBody));
    t += g(4 * (MAXB + 1) * sizeof(int)) + g(sizeof(SimDesc)) + g(NACCSET * ACCSET_SIZE * sizeof(unsigned long long));
    t += g(nblk * 5 * sizeof(double)) + g(8 * sizeof(double)) + g(4 * sizeof(int));
    return t;
}

void finish(lb_server *sv, Job *j, int status)
{
    lb_result r;
    std::memset(&r, 0, sizeof(r));
    r.ticket = j->ticket;
    r.tag = j->rq.tag;
    r.nbody = j->rq.nbody;
    r.t_submit = j->t_submit;
    r.t_admit = j->t_admit;
    r.fluid_cells = j->fluid;
    if (j->sim) {
        lb_sim *s = j->sim;
        r.steps = s->steps;
        for (int b = 0; b < int(s->bodies.size()) && status == LB_OK; ++b) {
            status = lb_body_state(s, b, r.pos[b], r.e[b], r.v[b], r.w[b], nullptr);
            if (status == LB_OK) status = lb_force_torque(s, b, r.F[b], r.T[b]);
        }
        if (status == LB_OK) {
            double P[3];
            status = lb_audit(s, &r.mass, P);
        }
        lb_destroy(s);
        j->sim = nullptr;
    }
    r.status = status;
    r.t_done = seconds_since(sv->t0);
    sv->results.push_back(r);
    sv->stats.completed++;
    delete j;
}

// Retire the oldest queued chunk if it is done (or wait for it).
int retire_front(lb_server *sv, bool block, bool *retired)
{
    *retired = false;
    if (sv->inflight.empty()) return LB_OK;
    Chunk &c = sv->inflight.front();
    if (block) {
        const TraceRange tr("lb_server wait");
        if (hipEventSynchronize(c.ev) != hipSuccess) return LB_EDEVICE;
    } else {
        const hipError_t q = hipEventQuery(c.ev);
        if (q == hipErrorNotReady) return LB_OK;
        if (q != hipSuccess) return LB_EDEVICE;
    }
    for (Job *j : c.done) finish(sv, j, j->cancelled ? LB_ECANCELED : LB_OK);
    (void)hipEventDestroy(c.ev);
    const hipGraphExec_t used = c.exec;
    sv->inflight.pop_front();
    if (used && used != sv->exec) {
        bool still = false;
        for (const Chunk &o : sv->inflight) still |= o.exec == used;
        if (!still) (void)hipGraphExecDestroy(used);
    }
    *retired = true;
    return LB_OK;
}

// Admit queued requests while slots and arena memory allow (first come,
// first served).  Set-up work runs on the set-up stream; the batch stream
// waits for it before the next chunk.
int admit(lb_server *sv)
{
    if (sv->queue.empty() || int(sv->active.size()) >= sv->p.max_active) return LB_OK;
    const TraceRange tr("lb_server admit");
    bool any = false;
    while (!sv->queue.empty() && int(sv->active.size()) < sv->p.max_active) {
        Job *j = sv->queue.front();
        const lb_request &rq = j->rq;
        lb_params p;
        std::memset(&p, 0, sizeof(p));
        p.nx = rq.nx;
        p.ny = rq.ny;
        p.nz = rq.nz;
        p.nu = rq.nu;
        p.magic = 3.0 / 16.0;
        p.rho0 = 1.0;
        p.storage = sv->p.storage;
        p.scale_log2 = sv->p.scale_log2;
        p.wca_sigma = sv->p.wca_sigma;
        p.wca_eps = sv->p.wca_eps;
        p.stream = sv->setup;
        p.alloc = arena_alloc;
        p.free = arena_free;
        p.alloc_ctx = sv;
        lb_sim *s = nullptr;
        int rc = lb_create(&p, &s);
        for (int b = 0; rc == LB_OK && b < rq.nbody; ++b) {
            int id = 0;
            rc = lb_add_squirmer(s, &rq.body[b], &id);
        }
        if (rc == LB_OK) rc = lbsq_prepare(s);
        if (rc == LB_OK) rc = lb_info(s, &j->fluid, nullptr);
        if (rc == LB_ENOMEM) {
            if (s) lb_destroy(s);
            // nothing else holds memory: it will never fit
            if (!sv->active.empty() || !sv->inflight.empty()) break;
            sv->queue.pop_front();
            finish(sv, j, LB_EBUDGET);
            continue;
        }
        sv->queue.pop_front();
        j->t_admit = seconds_since(sv->t0);
        if (rc != LB_OK) {
            if (s) lb_destroy(s);
            finish(sv, j, rc);
            continue;
        }
        j->sim = s;
        if (rq.nsteps == 0) {
            finish(sv, j, LB_OK);
            continue;
        }
        sv->active.push_back(j);
        any = true;
    }
    if (any) {
        if (hipEventRecord(sv->setup_ev, sv->setup) != hipSuccess ||
            hipStreamWaitEvent(sv->stream, sv->setup_ev, 0) != hipSuccess)
            return LB_EDEVICE;
    }
    return LB_OK;
}

// Enqueue one chunk of the resident requests.
int launch_chunk(lb_server *sv)
{
    const TraceRange tr("lb_server chunk");
    const int n = int(sv->active.size());
    std::vector<lb_sim *> sims(n);
    int64_t kmax = 0;
    for (int j = 0; j < n; ++j) {
        sims[j] = sv->active[j]->sim;
        kmax = std::max(kmax, sv->active[j]->rq.nsteps - sims[j]->steps);
    }
    const Batch b = make_batch(sims.data(), n);
    SimDesc *h = sv->h_desc + size_t(sv->ring) * MAXSIM;
    sv->ring = (sv->ring + 1) % RING;
    for (int j = 0; j < n; ++j) lbsq_fill_desc(sims[j], sims[j]->steps, sv->active[j]->rq.nsteps, h[j]);
    if (hipMemcpyAsync(sv->d_desc, h, size_t(n) * sizeof(SimDesc), hipMemcpyHostToDevice, sv->stream) != hipSuccess)
        return LB_EDEVICE;
    Chunk c;
    const int K = sv->p.chunk_steps;
    if (sv->p.use_graph) {
        // one graph per set of resident requests (their block ranges)
        std::vector<uint32_t> key;
        key.push_back(uint32_t(K));
        key.push_back(uint32_t(b.nbody_max));
        for (int j = 0; j <= n; ++j) {
            key.push_back(b.map.fluid0[j]);
            key.push_back(b.map.geo0[j]);
        }
        if (!sv->exec || key != sv->exec_key) {
            hipGraph_t g = nullptr;
            hipGraphExec_t e = nullptr;
            if (hipStreamBeginCapture(sv->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return LB_EDEVICE;
            const hipError_t le = enqueue_steps(sv->p.storage, sv->d_desc, b, K, sv->capture);
            const hipError_t ce = hipStreamEndCapture(sv->capture, &g);
            if (le != hipSuccess || ce != hipSuccess) return LB_EDEVICE;
            const hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) return LB_EDEVICE;
            // the previous graph goes when no queued chunk uses it any more
            bool still = false;
            for (const Chunk &o : sv->inflight) still |= o.exec == sv->exec;
            if (sv->exec && !still) (void)hipGraphExecDestroy(sv->exec);
            sv->exec = e;
            sv->exec_key = key;
            sv->stats.graphs++;
        }
        if (hipGraphLaunch(sv->exec, sv->stream) != hipSuccess) return LB_EDEVICE;
        c.exec = sv->exec;
    } else {
        const int kk = int(std::min<int64_t>(K, kmax));
        if (enqueue_steps(sv->p.storage, sv->d_desc, b, kk, sv->stream) != hipSuccess) return LB_EDEVICE;
    }
    if (hipEventCreateWithFlags(&c.ev, hipEventDisableTiming) != hipSuccess) return LB_EDEVICE;
    if (hipEventRecord(c.ev, sv->stream) != hipSuccess) {
        (void)hipEventDestroy(c.ev);
        return LB_EDEVICE;
    }
    std::vector<Job *> keep;
    for (Job *j : sv->active) {
        lb_sim *s = j->sim;
        const int64_t adv = std::min<int64_t>(K, j->rq.nsteps - s->steps);
        s->steps += adv;
        s->cur = int(s->steps & 1);
        sv->stats.cell_updates += j->fluid * uint64_t(adv);
        if (s->steps == j->rq.nsteps) c.done.push_back(j);
        else keep.push_back(j);
    }
    sv->active.swap(keep);
    sv->inflight.push_back(c);
    sv->stats.chunks++;
    return LB_OK;
}

int pump(lb_server *sv)
{
    bool r = true;
    while (r) {
        const int st = retire_front(sv, false, &r);
        if (st != LB_OK) return st;
    }
    int st = admit(sv);
    if (st != LB_OK) return st;
    if (!sv->active.empty() && int(sv->inflight.size()) < MAX_QUEUED) return launch_chunk(sv);
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_step_batch(lb_sim *const *sims, int n, int nsteps)
{
    if ((!sims && n > 0) || n < 0 || nsteps < 0) return LB_EINVAL;
    for (int k = 0; k < n; ++k) {
        if (!sims[k]) return LB_EINVAL;
        for (int j = 0; j < k; ++j)
            if (sims[j] == sims[k]) return LB_EINVAL;
    }
    if (n == 0 || nsteps == 0) return LB_OK;
    const TraceRange tr("lb_step_batch");
    bool together = n <= MAXSIM;
    for (int k = 0; k < n && together; ++k)
        together = batchable(sims[k]) && sims[k]->p.storage == sims[0]->p.storage &&
                   sims[k]->device == sims[0]->device;
    if (!together) {
        for (int k = 0; k < n; ++k) {
            const int rc = lb_step(sims[k], nsteps);
            if (rc != LB_OK) return rc;
        }
        return LB_OK;
    }
    lb_sim *h = sims[0];
    (void)hipSetDevice(h->device);
    for (int k = 0; k < n; ++k) {
        const int rc = lbsq_prepare(sims[k]);
        if (rc != LB_OK) return rc;
    }
    if (!h->d_batch_desc) {
        h->d_batch_desc = static_cast<SimDesc *>(lbsq_dev_alloc(h, MAXSIM * sizeof(SimDesc)));
        if (!h->d_batch_desc) return LB_ENOMEM;
    }
    // the previous batch led by h may still read the table
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LB_EDEVICE;
    std::vector<SimDesc> d(n);
    for (int k = 0; k < n; ++k) lbsq_fill_desc(sims[k], sims[k]->steps, sims[k]->steps + nsteps, d[k]);
    if (hipMemcpy(h->d_batch_desc, d.data(), size_t(n) * sizeof(SimDesc), hipMemcpyHostToDevice) != hipSuccess)
        return LB_EDEVICE;
    // the batch runs on h's stream after the work queued on every stream
    std::vector<hipEvent_t> evs;
    hipError_t e = hipSuccess;
    for (int k = 1; k < n && e == hipSuccess; ++k) {
        if (sims[k]->stream == h->stream) continue;
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) break;
        evs.push_back(ev);
        e = hipEventRecord(ev, sims[k]->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, ev, 0);
    }
    const Batch b = make_batch(sims, n);
    if (e == hipSuccess) e = enqueue_steps(h->p.storage, h->d_batch_desc, b, nsteps, h->stream);
    if (e == hipSuccess) {
        hipEvent_t done;
        e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e == hipSuccess) {
            evs.push_back(done);
            e = hipEventRecord(done, h->stream);
            for (int k = 1; k < n && e == hipSuccess; ++k)
                if (sims[k]->stream != h->stream) e = hipStreamWaitEvent(sims[k]->stream, done, 0);
        }
    }
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    if (e != hipSuccess) return LB_EDEVICE;
    for (int k = 0; k < n; ++k) {
        sims[k]->steps += nsteps;
        sims[k]->cur = int(sims[k]->steps & 1);
    }
    return LB_OK;
}

int lb_server_create(const lb_server_params *p, lb_server **out)
{
    if (!p || !out) return LB_EINVAL;
    *out = nullptr;
    if (p->budget_bytes < (size_t(1) << 20) || p->max_active < 1 || p->max_active > LB_SERVER_MAXACTIVE ||
        p->chunk_steps < 1 || p->chunk_steps > 100000 || p->storage < 0 || p->storage > 2 || p->scale_log2 < 0 ||
        p->scale_log2 > 20 || !(p->wca_sigma > 0.0) || p->wca_eps < 0.0)
        return LB_EINVAL;
    static_assert(LB_SERVER_MAXACTIVE <= MAXSIM, "batch table too small");
    lb_server *sv = new (std::nothrow) lb_server();
    if (!sv) return LB_ENOMEM;
    sv->p = *p;
    sv->t0 = std::chrono::steady_clock::now();
    (void)hipGetDevice(&sv->device);
    int rc = LB_OK;
    if (p->stream) {
        sv->stream = static_cast<hipStream_t>(p->stream);
    } else {
        if (hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) rc = LB_EDEVICE;
        sv->own_stream = rc == LB_OK;
    }
    if (rc == LB_OK && (hipStreamCreateWithFlags(&sv->setup, hipStreamNonBlocking) != hipSuccess ||
                        hipStreamCreateWithFlags(&sv->capture, hipStreamNonBlocking) != hipSuccess ||
                        hipEventCreateWithFlags(&sv->setup_ev, hipEventDisableTiming) != hipSuccess))
        rc = LB_EDEVICE;
    if (rc == LB_OK && (hipMalloc(&sv->arena_mem, p->budget_bytes) != hipSuccess ||
                        hipMalloc(&sv->d_desc, MAXSIM * sizeof(SimDesc)) != hipSuccess ||
                        hipHostMalloc(&sv->h_desc, RING * MAXSIM * sizeof(SimDesc), hipHostMallocDefault) !=
                            hipSuccess))
        rc = LB_ENOMEM;
    if (rc != LB_OK) {
        lb_server_destroy(sv);
        return rc;
    }
    sv->arena.reset(static_cast<char *>(sv->arena_mem), p->budget_bytes);
    *out = sv;
    return LB_OK;
}

int lb_server_submit(lb_server *sv, const lb_request *rq, uint64_t *ticket)
{
    if (!sv || !rq) return LB_EINVAL;
    if (rq->nx < 4 || rq->ny < 4 || rq->nz < 4 || !(rq->nu > 0.0) || rq->nbody < 0 ||
        rq->nbody > LB_REQ_MAXBODY || rq->nsteps < 0)
        return LB_EINVAL;
    if (uint64_t(rq->nx) * rq->ny * rq->nz >= (uint64_t(1) << 32)) return LB_EINVAL;
    if (request_bytes(rq, sv->p.storage) > sv->p.budget_bytes) return LB_EBUDGET;
    Job *j = new (std::nothrow) Job();
    if (!j) return LB_ENOMEM;
    j->ticket = sv->next_ticket++;
    j->rq = *rq;
    j->t_submit = seconds_since(sv->t0);
    sv->queue.push_back(j);
    if (ticket) *ticket = j->ticket;
    return LB_OK;
}

int lb_server_progress(lb_server *sv, int wait, int *active, int *queued)
{
    if (!sv) return LB_EINVAL;
    (void)hipSetDevice(sv->device);
    int st = LB_OK;
    if (wait && !sv->inflight.empty()) {
        bool r = false;
        st = retire_front(sv, true, &r);
    }
    if (st == LB_OK) st = pump(sv);
    // keep the device fed: a second chunk behind the running one
    if (st == LB_OK && !sv->active.empty() && int(sv->inflight.size()) < MAX_QUEUED) st = pump(sv);
    if (active) *active = int(sv->active.size() + [&] {
        size_t t = 0;
        for (const Chunk &c : sv->inflight) t += c.done.size();
        return t;
    }());
    if (queued) *queued = int(sv->queue.size());
    return st;
}

int lb_server_cancel(lb_server *sv, uint64_t ticket)
{
    if (!sv) return LB_EINVAL;
    if (ticket == 0 || ticket >= sv->next_ticket) return LB_EINVAL;
    (void)hipSetDevice(sv->device);
    for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it) {
        if ((*it)->ticket != ticket) continue;
        Job *j = *it;
        sv->queue.erase(it);
        finish(sv, j, LB_ECANCELED);
        return LB_OK;
    }
    for (auto it = sv->active.begin(); it != sv->active.end(); ++it) {
        if ((*it)->ticket != ticket) continue;
        Job *j = *it;
        sv->active.erase(it);
        j->cancelled = true;
        // queued chunks may still step it: it ends with the newest of them
        if (sv->inflight.empty()) finish(sv, j, LB_ECANCELED);
        else sv->inflight.back().done.push_back(j);
        return LB_OK;
    }
    return LB_ESTATE;
}

int lb_server_results(lb_server *sv, lb_result *out, int cap, int *n)
{
    if (!sv || !n || cap < 0 || (!out && cap > 0)) return LB_EINVAL;
    int k = 0;
    while (k < cap && !sv->results.empty()) {
        out[k++] = sv->results.front();
        sv->results.pop_front();
    }
    *n = k;
    return LB_OK;
}

int lb_server_stats_get(lb_server *sv, lb_server_stats *st)
{
    if (!sv || !st) return LB_EINVAL;
    *st = sv->stats;
    st->arena_in_use = sv->arena.in_use();
    return LB_OK;
}

int lb_server_clock(lb_server *sv, double *t)
{
    if (!sv || !t) return LB_EINVAL;
    *t = seconds_since(sv->t0);
    return LB_OK;
}

int lb_server_destroy(lb_server *sv)
{
    if (!sv) return LB_EINVAL;
    (void)hipSetDevice(sv->device);
    if (sv->stream) (void)hipStreamSynchronize(sv->stream);
    while (!sv->inflight.empty()) {
        bool r = false;
        if (retire_front(sv, true, &r) != LB_OK || !r) break;
    }
    for (Job *j : sv->active) {
        if (j->sim) lb_destroy(j->sim);
        delete j;
    }
    for (Job *j : sv->queue) delete j;
    for (Chunk &c : sv->inflight) {
        for (Job *j : c.done) {
            if (j->sim) lb_destroy(j->sim);
            delete j;
        }
        (void)hipEventDestroy(c.ev);
    }
    if (sv->exec) (void)hipGraphExecDestroy(sv->exec);
    if (sv->setup) (void)hipStreamSynchronize(sv->setup);
    if (sv->arena_mem) (void)hipFree(sv->arena_mem);
    if (sv->d_desc) (void)hipFree(sv->d_desc);
    if (sv->h_desc) (void)hipHostFree(sv->h_desc);
    if (sv->setup_ev) (void)hipEventDestroy(sv->setup_ev);
    if (sv->capture) (void)hipStreamDestroy(sv->capture);
    if (sv->setup) (void)hipStreamDestroy(sv->setup);
    if (sv->own_stream && sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
    return LB_OK;
}

}  // extern "C"

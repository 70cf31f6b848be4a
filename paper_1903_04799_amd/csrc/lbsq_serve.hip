// lbsq_serve.hip -- many resident simulations advanced together: the
// lb_step_batch call and the continuous-batching server (lb_server_*) of
// include/lbsq.h.
//
// The server's policy (queue, admission, chunks, retirement, cancellation)
// is lbsq_sched.h; this file gives it the HIP backend.
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

#include "lbsq_sched.h"
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
// the serving loop: the policy of lbsq_sched.h over the HIP backend below

namespace {

constexpr int RING = 3;  // pinned descriptor tables (two chunks queued at most)
static_assert(RING > SERVE_MAX_QUEUED, "a queued chunk's descriptor table must not be overwritten");

struct GpuBackend;

}  // namespace

struct lb_server {
    lb_server_params p{};
    int device = 0;
    hipStream_t stream = nullptr, setup = nullptr, capture = nullptr;
    bool own_stream = false;
    Arena arena;
    void *arena_mem = nullptr;
    SimDesc *d_desc = nullptr;  // descriptors read by the chunk kernels
    SimDesc *h_desc = nullptr;  // RING pinned tables of MAXSIM descriptors
    int ring = 0;
    hipEvent_t setup_ev = nullptr;
    hipGraphExec_t exec = nullptr;  // graph of the current set of requests
    std::vector<uint32_t> exec_key;
    std::map<hipGraphExec_t, int> graph_refs;  // queued chunks replaying each graph
    uint64_t graphs = 0;
    std::chrono::steady_clock::time_point t0;
    GpuBackend *be = nullptr;
    ServeCore<GpuBackend> *core = nullptr;
};

namespace {

void *arena_alloc(size_t bytes, void *ctx) { return static_cast<lb_server *>(ctx)->arena.alloc(bytes); }
void arena_free(void *p, void *ctx) { static_cast<lb_server *>(ctx)->arena.release(p); }

// Device bytes a request needs (each allocation of the handle rounded to
// the arena granule), for rejecting requests that can never fit.
size_t request_bytes(const lb_request *rq, int storage, int layout)
{
    auto g = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); };
    const uint64_t n = uint64_t(rq->nx) * rq->ny * rq->nz;
    const uint64_t stride = ((n + 255) / 256) * 256 + 256;
    const size_t es = storage == LB_STORAGE_F32 ? 4 : 2;
    const uint64_t nblk = (n + BLOCK - 1) / BLOCK;
    const size_t npop = layout == LB_LAYOUT_AB ? 2 : 1;
    size_t t = npop * g(size_t(Q) * stride * es) + 2 * g(n * sizeof(float)) + 2 * g(n) + 2 * g(MAXB * sizeof(DevBody));
    t += g(4 * (MAXB + 1) * sizeof(int)) + g(sizeof(SimDesc)) + g(NACCSET * ACCSET_SIZE * sizeof(unsigned long long));
    t += g(nblk * 5 * sizeof(double)) + g(8 * sizeof(double)) + g(4 * sizeof(int));
    return t;
}

// Simulations are lb_sim handles allocated in the server's arena; a chunk is
// one descriptor upload plus K batched steps (a graph replay, or launches
// one by one) and the event recorded after them.
struct GpuBackend {
    lb_server *sv;
    using Sim = lb_sim *;
    struct Token {
        hipEvent_t ev = nullptr;
        hipGraphExec_t exec = nullptr;  // the graph this chunk replayed, if any
    };

    double now() const { return seconds_since(sv->t0); }
    int64_t steps(Sim s) const { return s->steps; }
    void advance(Sim s, int64_t n)
    {
        s->steps += n;
        s->cur = int(s->steps & 1);
    }
    void destroy(Sim s) { lb_destroy(s); }

    // Set-up work runs on the set-up stream while chunks run.
    int create(const lb_request &rq, Sim *out, uint64_t *fluid)
    {
        const TraceRange tr("lb_server admit");
        *out = nullptr;
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
        p.layout = sv->p.layout;
        lb_sim *s = nullptr;
        int rc = lb_create(&p, &s);
        for (int b = 0; rc == LB_OK && b < rq.nbody; ++b) {
            int id = 0;
            rc = lb_add_squirmer(s, &rq.body[b], &id);
        }
        if (rc == LB_OK) rc = lbsq_prepare(s);
        if (rc == LB_OK) rc = lb_info(s, fluid, nullptr);
        if (rc != LB_OK) {
            if (s) lb_destroy(s);
            return rc;
        }
        *out = s;
        return LB_OK;
    }

    // The batch stream waits for the set-up work before the next chunk.
    int admitted()
    {
        if (hipEventRecord(sv->setup_ev, sv->setup) != hipSuccess ||
            hipStreamWaitEvent(sv->stream, sv->setup_ev, 0) != hipSuccess)
            return LB_EDEVICE;
        return LB_OK;
    }

    int launch(const std::vector<Sim> &sims, const std::vector<int64_t> &ends, int K, Token *tok)
    {
        const TraceRange tr("lb_server chunk");
        const int n = int(sims.size());
        int64_t kmax = 0;
        for (int j = 0; j < n; ++j) kmax = std::max(kmax, ends[j] - sims[j]->steps);
        const Batch b = make_batch(sims.data(), n);
        SimDesc *h = sv->h_desc + size_t(sv->ring) * MAXSIM;
        sv->ring = (sv->ring + 1) % RING;
        for (int j = 0; j < n; ++j) lbsq_fill_desc(sims[j], sims[j]->steps, ends[j], h[j]);
        if (hipMemcpyAsync(sv->d_desc, h, size_t(n) * sizeof(SimDesc), hipMemcpyHostToDevice, sv->stream) !=
            hipSuccess)
            return LB_EDEVICE;
        Token t;
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
                if (hipStreamBeginCapture(sv->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return LB_EDEVICE;
                const hipError_t le = enqueue_steps(sv->p.storage, sv->d_desc, b, K, sv->capture);
                const hipError_t ce = hipStreamEndCapture(sv->capture, &g);
                if (le != hipSuccess || ce != hipSuccess) return LB_EDEVICE;
                const hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) return LB_EDEVICE;
                // the previous graph goes when no queued chunk replays it
                if (sv->exec && sv->graph_refs.find(sv->exec) == sv->graph_refs.end())
                    (void)hipGraphExecDestroy(sv->exec);
                sv->exec = e;
                sv->exec_key = key;
                sv->graphs++;
            }
            if (hipGraphLaunch(sv->exec, sv->stream) != hipSuccess) return LB_EDEVICE;
            t.exec = sv->exec;
            sv->graph_refs[sv->exec]++;
        } else {
            const int kk = int(std::min<int64_t>(K, kmax));
            if (enqueue_steps(sv->p.storage, sv->d_desc, b, kk, sv->stream) != hipSuccess) return LB_EDEVICE;
        }
        if (hipEventCreateWithFlags(&t.ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(t.ev, sv->stream) != hipSuccess) {
            // the chunk is queued but cannot be tracked: let it finish first
            (void)hipStreamSynchronize(sv->stream);
            release(t);
            return LB_EDEVICE;
        }
        *tok = t;
        return LB_OK;
    }

    int poll(Token &t, bool block, bool *done)
    {
        *done = false;
        if (block) {
            const TraceRange tr("lb_server wait");
            if (hipEventSynchronize(t.ev) != hipSuccess) return LB_EDEVICE;
        } else {
            const hipError_t q = hipEventQuery(t.ev);
            if (q == hipErrorNotReady) return LB_OK;
            if (q != hipSuccess) return LB_EDEVICE;
        }
        *done = true;
        return LB_OK;
    }

    void release(Token &t)
    {
        if (t.ev) (void)hipEventDestroy(t.ev);
        if (t.exec) {
            auto it = sv->graph_refs.find(t.exec);
            if (it != sv->graph_refs.end() && --it->second == 0) {
                if (t.exec != sv->exec) (void)hipGraphExecDestroy(t.exec);
                sv->graph_refs.erase(it);
            }
        }
        t = Token{};
    }

    int read_result(Sim s, lb_result *r)
    {
        int status = LB_OK;
        for (int b = 0; b < int(s->bodies.size()) && status == LB_OK; ++b) {
            status = lb_body_state(s, b, r->pos[b], r->e[b], r->v[b], r->w[b], nullptr);
            if (status == LB_OK) status = lb_force_torque(s, b, r->F[b], r->T[b]);
        }
        if (status == LB_OK) {
            double P[3];
            status = lb_audit(s, &r->mass, P);
        }
        return status;
    }
};

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
        p->scale_log2 > 20 || !(p->wca_sigma > 0.0) || p->wca_eps < 0.0 ||
        (p->layout != LB_LAYOUT_INPLACE && p->layout != LB_LAYOUT_AB && p->layout != LB_LAYOUT_AUTO))
        return LB_EINVAL;
    static_assert(LB_SERVER_MAXACTIVE <= MAXSIM, "batch table too small");
    lb_server *sv = new (std::nothrow) lb_server();
    if (!sv) return LB_ENOMEM;
    sv->p = *p;
    // a batch of resident requests streams from HBM, where the pull layout
    // is the faster one
    if (sv->p.layout == LB_LAYOUT_AUTO) sv->p.layout = LB_LAYOUT_AB;
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
    if (rc == LB_OK) {
        sv->arena.reset(static_cast<char *>(sv->arena_mem), p->budget_bytes);
        sv->be = new (std::nothrow) GpuBackend{sv};
        if (sv->be) sv->core = new (std::nothrow) ServeCore<GpuBackend>(*sv->be, p->max_active, p->chunk_steps);
        if (!sv->core) rc = LB_ENOMEM;
    }
    if (rc != LB_OK) {
        lb_server_destroy(sv);
        return rc;
    }
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
    if (request_bytes(rq, sv->p.storage, sv->p.layout) > sv->p.budget_bytes) return LB_EBUDGET;
    return sv->core->submit(*rq, ticket);
}

int lb_server_cancel(lb_server *sv, uint64_t ticket)
{
    if (!sv) return LB_EINVAL;
    (void)hipSetDevice(sv->device);
    return sv->core->cancel(ticket);
}

int lb_server_progress(lb_server *sv, int wait, int *active, int *queued)
{
    if (!sv) return LB_EINVAL;
    (void)hipSetDevice(sv->device);
    return sv->core->progress(wait != 0, active, queued);
}

int lb_server_results(lb_server *sv, lb_result *out, int cap, int *n)
{
    if (!sv || !n || cap < 0 || (!out && cap > 0)) return LB_EINVAL;
    return sv->core->results(out, cap, n);
}

int lb_server_stats_get(lb_server *sv, lb_server_stats *st)
{
    if (!sv || !st) return LB_EINVAL;
    std::memset(st, 0, sizeof(*st));
    st->cell_updates = sv->core->cell_updates;
    st->chunks = sv->core->chunks;
    st->graphs = sv->graphs;
    st->completed = sv->core->completed;
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
    delete sv->core;  // waits for the queued chunks and drops the rest
    delete sv->be;
    for (auto &g : sv->graph_refs)
        if (g.first != sv->exec) (void)hipGraphExecDestroy(g.first);
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

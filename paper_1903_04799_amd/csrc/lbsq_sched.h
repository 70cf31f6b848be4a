// lbsq_sched.h -- the serving policy behind the lb_server_* calls, apart from
// the device: a first-come-first-served queue admitted by free slots and
// memory, chunks of steps for every resident request, in-order retirement of
// finished chunks, and cancellation.
//
// The device side is the Backend template argument: it creates a simulation
// for a request (in memory it owns, failing with LB_ENOMEM when that memory
// is full), queues a chunk of steps for a set of simulations, reports when a
// chunk has run, and reads a finished simulation's result.  lbsq_serve.hip
// gives the HIP backend; the scheduler's unit test gives a host-side fake.
// Host code only: nothing here touches the device.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/lbsq.h"

namespace lbsq {

// First-fit allocator over one block of memory (256-byte granules);
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

// Most chunks queued on the device at once: one running, one behind it.
constexpr int SERVE_MAX_QUEUED = 2;

// Backend requirements (B::Sim is a pointer-like handle, B::Token one queued
// chunk):
//   int create(const lb_request &, Sim *out, uint64_t *fluid_cells)
//       LB_OK, LB_ENOMEM when its memory is full, or the request's error;
//       on failure nothing is left allocated and *out is null;
//   void destroy(Sim);
//   int64_t steps(Sim);  void advance(Sim, int64_t n);
//   int launch(const std::vector<Sim> &, const std::vector<int64_t> &ends,
//              int K, Token *)   queue up to K steps of every simulation
//              (each stops at its end), from its current step count;
//   int poll(Token &, bool block, bool *done);  void release(Token &);
//   int read_result(Sim, lb_result *)   body states, forces and mass;
//   int admitted()   called once after a round that admitted requests;
//   double now()     seconds since the server started.
template <class B>
class ServeCore {
  public:
    using Sim = typename B::Sim;
    using Token = typename B::Token;

    ServeCore(B &backend, int max_active, int chunk_steps)
        : be_(backend), max_active_(max_active), K_(chunk_steps)
    {
    }
    ServeCore(const ServeCore &) = delete;
    ServeCore &operator=(const ServeCore &) = delete;
    ~ServeCore() { shutdown(); }

    uint64_t cell_updates = 0, chunks = 0, completed = 0;

    int submit(const lb_request &rq, uint64_t *ticket)
    {
        Job *j = new (std::nothrow) Job();
        if (!j) return LB_ENOMEM;
        j->ticket = next_ticket_++;
        j->rq = rq;
        j->t_submit = be_.now();
        queue_.push_back(j);
        if (ticket) *ticket = j->ticket;
        return LB_OK;
    }

    // A queued request ends at once.  A resident one leaves the batch and
    // ends with the newest chunk already queued with it, so its simulation
    // is destroyed only after every chunk that steps it has run.
    int cancel(uint64_t ticket)
    {
        if (ticket == 0 || ticket >= next_ticket_) return LB_EINVAL;
        for (auto it = queue_.begin(); it != queue_.end(); ++it) {
            if ((*it)->ticket != ticket) continue;
            Job *j = *it;
            queue_.erase(it);
            finish(j, LB_ECANCELED);
            return LB_OK;
        }
        for (auto it = active_.begin(); it != active_.end(); ++it) {
            if ((*it)->ticket != ticket) continue;
            Job *j = *it;
            active_.erase(it);
            j->cancelled = true;
            if (inflight_.empty()) finish(j, LB_ECANCELED);
            else inflight_.back().done.push_back(j);
            return LB_OK;
        }
        return LB_ESTATE;
    }

    int progress(bool wait, int *active, int *queued)
    {
        int st = LB_OK;
        if (wait && !inflight_.empty()) {
            bool r = false;
            st = retire_front(true, &r);
        }
        if (st == LB_OK) st = pump();
        // keep the device fed: a second chunk behind the running one
        if (st == LB_OK && !active_.empty() && int(inflight_.size()) < SERVE_MAX_QUEUED) st = pump();
        if (active) {
            size_t t = active_.size();
            for (const Chunk &c : inflight_) t += c.done.size();
            *active = int(t);
        }
        if (queued) *queued = int(queue_.size());
        return st;
    }

    int results(lb_result *out, int cap, int *n)
    {
        int k = 0;
        while (k < cap && !results_.empty()) {
            out[k++] = results_.front();
            results_.pop_front();
        }
        *n = k;
        return LB_OK;
    }

    // Wait for the queued chunks, then drop every request still resident or
    // queued.
    void shutdown()
    {
        while (!inflight_.empty()) {
            bool r = false;
            if (retire_front(true, &r) != LB_OK || !r) break;
        }
        for (Job *j : active_) {
            if (j->sim) be_.destroy(j->sim);
            delete j;
        }
        active_.clear();
        for (Job *j : queue_) delete j;
        queue_.clear();
        for (Chunk &c : inflight_) {
            for (Job *j : c.done) {
                if (j->sim) be_.destroy(j->sim);
                delete j;
            }
            be_.release(c.tok);
        }
        inflight_.clear();
    }

  private:
    struct Job {
        uint64_t ticket = 0;
        lb_request rq{};
        double t_submit = 0.0, t_admit = 0.0;
        Sim sim{};
        uint64_t fluid = 0;
        bool cancelled = false;  // left the batch early; ends as LB_ECANCELED
    };
    struct Chunk {
        Token tok{};
        std::vector<Job *> done;  // requests that end when this chunk has run
    };

    B &be_;
    int max_active_, K_;
    uint64_t next_ticket_ = 1;
    std::deque<Job *> queue_;
    std::vector<Job *> active_;
    std::deque<Chunk> inflight_;
    std::deque<lb_result> results_;

    void finish(Job *j, int status)
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
            r.steps = be_.steps(j->sim);
            if (status == LB_OK) status = be_.read_result(j->sim, &r);
            be_.destroy(j->sim);
            j->sim = Sim{};
        }
        r.status = status;
        r.t_done = be_.now();
        results_.push_back(r);
        completed++;
        delete j;
    }

    // Retire the oldest queued chunk if it has run (or wait for it).
    int retire_front(bool block, bool *retired)
    {
        *retired = false;
        if (inflight_.empty()) return LB_OK;
        Chunk &c = inflight_.front();
        bool done = false;
        const int st = be_.poll(c.tok, block, &done);
        if (st != LB_OK) return st;
        if (!done) return LB_OK;
        for (Job *j : c.done) finish(j, j->cancelled ? LB_ECANCELED : LB_OK);
        be_.release(c.tok);
        inflight_.pop_front();
        *retired = true;
        return LB_OK;
    }

    // Admit queued requests in order while slots and memory allow.
    int admit()
    {
        bool any = false;
        while (!queue_.empty() && int(active_.size()) < max_active_) {
            Job *j = queue_.front();
            Sim s{};
            const int rc = be_.create(j->rq, &s, &j->fluid);
            if (rc == LB_ENOMEM) {
                // nothing else holds memory: it will never fit
                if (!active_.empty() || !inflight_.empty()) break;
                queue_.pop_front();
                finish(j, LB_EBUDGET);
                continue;
            }
            queue_.pop_front();
            j->t_admit = be_.now();
            if (rc != LB_OK) {
                finish(j, rc);
                continue;
            }
            j->sim = s;
            if (j->rq.nsteps == 0) {
                finish(j, LB_OK);
                continue;
            }
            active_.push_back(j);
            any = true;
        }
        return any ? be_.admitted() : LB_OK;
    }

    // Queue one chunk of the resident requests.
    int launch_chunk()
    {
        std::vector<Sim> sims;
        std::vector<int64_t> ends;
        for (Job *j : active_) {
            sims.push_back(j->sim);
            ends.push_back(j->rq.nsteps);
        }
        Chunk c;
        const int st = be_.launch(sims, ends, K_, &c.tok);
        if (st != LB_OK) return st;
        std::vector<Job *> keep;
        for (Job *j : active_) {
            const int64_t adv = std::min<int64_t>(K_, j->rq.nsteps - be_.steps(j->sim));
            be_.advance(j->sim, adv);
            cell_updates += j->fluid * uint64_t(adv);
            if (be_.steps(j->sim) == j->rq.nsteps) c.done.push_back(j);
            else keep.push_back(j);
        }
        active_.swap(keep);
        inflight_.push_back(c);
        chunks++;
        return LB_OK;
    }

    int pump()
    {
        bool r = true;
        while (r) {
            const int st = retire_front(false, &r);
            if (st != LB_OK) return st;
        }
        const int st = admit();
        if (st != LB_OK) return st;
        if (!active_.empty() && int(inflight_.size()) < SERVE_MAX_QUEUED) return launch_chunk();
        return LB_OK;
    }
};

}  // namespace lbsq

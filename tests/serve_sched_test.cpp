// Unit test of the serving policy (paper_1903_04799_amd/csrc/lbsq_sched.h)
// with a host-side fake backend: a simulation is a block of a host arena, a
// queued chunk has run once it has been polled a few times (or waited for).
// The fake checks what the policy promises:
//   - first come, first served;
//   - at most max_active requests per chunk, at most two chunks queued;
//   - every request runs exactly its steps, in chunks of K;
//   - a request that can never fit ends with LB_EBUDGET, a bad one with its
//     own error, without stopping the others;
//   - a cancelled request ends with LB_ECANCELED, and no simulation is
//     destroyed while a queued chunk that steps it has not yet run;
//   - shutdown leaves nothing allocated.
// Host code only; the test that builds it runs it under ASan and UBSan.
#include <cstdio>
#include <map>
#include <vector>

#include "../paper_1903_04799_amd/csrc/lbsq_sched.h"

static int failures = 0;
#define EXPECT(c)                                                        \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);     \
            ++failures;                                                  \
        }                                                                \
    } while (0)

struct FakeSim {
    int64_t steps = 0;
    void *mem = nullptr;
    int pending = 0;  // queued chunks that step it and have not run yet
};

struct Fake {
    using Sim = FakeSim *;
    struct Token {
        int id = -1;
        bool ran = false;
        std::vector<FakeSim *> sims;
    };
    lbsq::Arena arena;
    std::vector<char> buf;
    double clock = 0.0;
    int next_id = 0, queued = 0, max_queued = 0, live = 0, max_live = 0;
    size_t max_batch = 0;
    std::vector<uint64_t> admitted_tags;
    std::map<int, int> polls;

    explicit Fake(size_t bytes) : buf(bytes) { arena.reset(buf.data(), bytes); }

    double now() { return clock += 1.0; }
    int64_t steps(Sim s) { return s->steps; }
    void advance(Sim s, int64_t n) { s->steps += n; }
    int create(const lb_request &rq, Sim *out, uint64_t *fluid)
    {
        *out = nullptr;
        if (rq.nbody > 0 && rq.body[0].R <= 0.0) return LB_EGEOM;  // a bad request
        void *m = arena.alloc(size_t(rq.nx) * rq.ny * rq.nz);
        if (!m) return LB_ENOMEM;
        FakeSim *s = new FakeSim();
        s->mem = m;
        *out = s;
        *fluid = uint64_t(rq.nx) * rq.ny * rq.nz;
        admitted_tags.push_back(rq.tag);
        max_live = std::max(max_live, ++live);
        return LB_OK;
    }
    void destroy(Sim s)
    {
        EXPECT(s->pending == 0);
        arena.release(s->mem);
        --live;
        delete s;
    }
    int admitted() { return LB_OK; }
    int launch(const std::vector<Sim> &sims, const std::vector<int64_t> &ends, int K, Token *t)
    {
        EXPECT(!sims.empty() && K > 0);
        for (size_t j = 0; j < sims.size(); ++j) {
            EXPECT(sims[j]->steps < ends[j]);
            ++sims[j]->pending;
        }
        max_batch = std::max(max_batch, sims.size());
        max_queued = std::max(max_queued, ++queued);
        t->id = next_id++;
        t->sims = sims;
        polls[t->id] = 0;
        return LB_OK;
    }
    int poll(Token &t, bool block, bool *done)
    {
        *done = block || ++polls[t.id] > 2;
        if (*done && !t.ran) {
            t.ran = true;
            for (FakeSim *s : t.sims) --s->pending;
        }
        return LB_OK;
    }
    void release(Token &t)
    {
        if (!t.ran)
            for (FakeSim *s : t.sims) --s->pending;
        --queued;
        t = Token{};
    }
    int read_result(Sim s, lb_result *r)
    {
        r->mass = double(s->steps);
        return LB_OK;
    }
};

using Core = lbsq::ServeCore<Fake>;

static lb_request request(int n, int64_t nsteps, uint64_t tag, bool bad = false)
{
    lb_request rq{};
    rq.nx = rq.ny = rq.nz = n;
    rq.nu = 1.0 / 6.0;
    rq.nsteps = nsteps;
    rq.tag = tag;
    if (bad) {
        rq.nbody = 1;
        rq.body[0].R = 0.0;
    }
    return rq;
}

// Run until n results have come back; alternate polling and waiting.
static std::map<uint64_t, lb_result> drain(Core &core, size_t n)
{
    std::map<uint64_t, lb_result> out;
    for (int spin = 0; out.size() < n && spin < 100000; ++spin) {
        EXPECT(core.progress(spin % 3 == 2, nullptr, nullptr) == LB_OK);
        lb_result r[8];
        int got = 0;
        core.results(r, 8, &got);
        for (int k = 0; k < got; ++k) out[r[k].tag] = r[k];
    }
    EXPECT(out.size() == n);
    return out;
}

static void test_order_slots_and_steps()
{
    Fake fk(1 << 20);
    {
        Core core(fk, 2, 8);
        const int64_t nsteps[5] = {20, 8, 0, 13, 30};
        for (int k = 0; k < 5; ++k) EXPECT(core.submit(request(8, nsteps[k], k), nullptr) == LB_OK);
        auto res = drain(core, 5);
        uint64_t cells = 0;
        for (int k = 0; k < 5; ++k) {
            EXPECT(res[k].status == LB_OK);
            EXPECT(res[k].steps == nsteps[k]);
            EXPECT(res[k].mass == double(nsteps[k]));
            EXPECT(res[k].t_submit <= res[k].t_admit && res[k].t_admit <= res[k].t_done);
            cells += 512 * uint64_t(nsteps[k]);
        }
        EXPECT(core.cell_updates == cells);
        EXPECT(core.completed == 5);
    }
    EXPECT((fk.admitted_tags == std::vector<uint64_t>{0, 1, 2, 3, 4}));
    EXPECT(fk.max_batch <= 2 && fk.max_queued <= 2);
    EXPECT(fk.live == 0 && fk.arena.in_use() == 0);
}

static void test_budget_and_errors()
{
    Fake fk(4096);  // one 16^3 request at a time
    {
        Core core(fk, 4, 5);
        EXPECT(core.submit(request(32, 10, 0), nullptr) == LB_OK);        // never fits
        EXPECT(core.submit(request(16, 12, 1), nullptr) == LB_OK);
        EXPECT(core.submit(request(16, 7, 2, true), nullptr) == LB_OK);   // bad request
        EXPECT(core.submit(request(16, 9, 3), nullptr) == LB_OK);
        auto res = drain(core, 4);
        EXPECT(res[0].status == LB_EBUDGET && res[0].steps == 0);
        EXPECT(res[1].status == LB_OK && res[1].steps == 12);
        EXPECT(res[2].status == LB_EGEOM);
        EXPECT(res[3].status == LB_OK && res[3].steps == 9);
        EXPECT(res[3].t_admit >= res[1].t_done);  // admitted once the memory was free
    }
    EXPECT(fk.max_live == 1 && fk.live == 0 && fk.arena.in_use() == 0);
}

static void test_cancel()
{
    Fake fk(1 << 20);
    {
        Core core(fk, 2, 8);
        uint64_t ta = 0, tb = 0, tc = 0;
        EXPECT(core.submit(request(8, 100, 0), &ta) == LB_OK);
        EXPECT(core.submit(request(8, 100, 1), &tb) == LB_OK);
        EXPECT(core.submit(request(8, 20, 2), &tc) == LB_OK);  // waits for a slot
        EXPECT(core.cancel(tc) == LB_OK);
        EXPECT(core.cancel(tc) == LB_ESTATE);
        EXPECT(core.cancel(0) == LB_EINVAL && core.cancel(999) == LB_EINVAL);
        EXPECT(core.progress(false, nullptr, nullptr) == LB_OK);
        EXPECT(core.progress(false, nullptr, nullptr) == LB_OK);
        EXPECT(core.cancel(tb) == LB_OK);  // resident, with chunks queued
        auto res = drain(core, 3);
        EXPECT(res[2].status == LB_ECANCELED && res[2].steps == 0);
        EXPECT(res[1].status == LB_ECANCELED);
        EXPECT(res[1].steps > 0 && res[1].steps < 100 && res[1].steps % 8 == 0);
        EXPECT(res[0].status == LB_OK && res[0].steps == 100);
        EXPECT(core.cancel(ta) == LB_ESTATE);
    }
    EXPECT(fk.live == 0 && fk.arena.in_use() == 0);
}

static void test_shutdown_with_work_left()
{
    Fake fk(1 << 20);
    {
        Core core(fk, 2, 4);
        for (int k = 0; k < 5; ++k) EXPECT(core.submit(request(8, 50, k), nullptr) == LB_OK);
        EXPECT(core.progress(false, nullptr, nullptr) == LB_OK);
        int active = -1, queued = -1;
        EXPECT(core.progress(false, &active, &queued) == LB_OK);
        EXPECT(active == 2 && queued == 3);
    }
    EXPECT(fk.live == 0 && fk.arena.in_use() == 0 && fk.queued == 0);
}

int main()
{
    test_order_slots_and_steps();
    test_budget_and_errors();
    test_cancel();
    test_shutdown_with_work_left();
    if (failures) {
        std::printf("%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("serving policy: all checks passed\n");
    return 0;
}

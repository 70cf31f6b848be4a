"""Batched stepping and the continuous-batching server, through the C ABI.

A simulation advanced inside a batch (``lb_step_batch``) or as a served
request (``lb_server_*``) runs the same kernels on the same data as one
stepped alone by ``lb_step``: its results must agree bit for bit, whatever
else shares the launches, whether the chunks are replayed as HIP graphs or
launched one by one, and however the requests are admitted over time.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_04799_amd import lbsq
    return lbsq


def note(msg):
    print("[gpu-serving] " + msg, flush=True)
    sys.stdout.flush()


# Requests: box, bodies, steps.  Swimmers fast enough (B1 = 0.02) that cells
# change owner within the run, pairs close enough to interact, step counts
# that are not multiples of the chunk length.
REQUESTS = [
    ((24, 24, 24), [dict(pos=(10.3, 12.1, 11.7), e=(1, 0.2, 0), R=3.5, B1=0.02, beta=2.0)], 41),
    ((28, 26, 30), [dict(pos=(8.2, 13.0, 15.5), e=(1, 0, 0), R=3.0, B1=0.02, beta=-3.0),
                    dict(pos=(18.9, 12.4, 15.1), e=(-1, 0.3, 0.1), R=4.0, B1=0.02, beta=5.0)], 53),
    ((20, 22, 24), [dict(pos=(9.5, 11.0, 12.0), e=(0, 0, 1), R=3.0, B1=0.0, mode="fixed")], 17),
    ((32, 24, 28), [dict(pos=(15.2, 11.9, 14.3), e=(0.3, -1, 0.2), R=4.5, B1=0.02, beta=0.0)], 64),
    ((24, 24, 24), [], 9),
    ((26, 26, 26), [dict(pos=(12.9, 13.1, 12.2), e=(0, 1, 0), R=3.2, B1=0.015, beta=-5.0)], 30),
]


def alone(lbsq, shape, bodies, nsteps, storage="f32", layout="inplace"):
    s = lbsq.Sim(shape, storage=storage, layout=layout)
    for b in bodies:
        s.add_squirmer(**b)
    fluid0 = s.info()["n_fluid"]
    s.step(nsteps)
    out = {k: [] for k in ("pos", "e", "v", "w", "F", "T")}
    for i in range(len(bodies)):
        st = s.body(i)
        F, T = s.force_torque(i)
        for k in ("pos", "e", "v", "w"):
            out[k].append(st[k])
        out["F"].append(F)
        out["T"].append(T)
    out = {k: np.array(v).reshape(len(bodies), 3) for k, v in out.items()}
    out["mass"] = s.audit()[0]
    out["fluid"] = fluid0
    out["pops"] = s.populations()
    s.close()
    return out


def assert_same(res, ref, what):
    for k in ("pos", "e", "v", "w", "F", "T"):
        assert np.array_equal(res[k], ref[k]), "%s: %s differs: %s vs %s" % (what, k, res[k], ref[k])
    assert res["mass"] == ref["mass"], "%s: mass %r vs %r" % (what, res["mass"], ref["mass"])


def test_step_batch_matches_alone():
    note("lb_step_batch vs lb_step")
    lbsq = gpu()
    sel = [REQUESTS[0], REQUESTS[1], REQUESTS[2], REQUESTS[4]]
    sims = []
    for shape, bodies, _ in sel:
        s = lbsq.Sim(shape)
        for b in bodies:
            s.add_squirmer(**b)
        sims.append(s)
    # uneven pattern: batches, single steps, batches again
    lbsq.step_batch(sims, 7)
    sims[1].step(3)
    lbsq.step_batch(sims[:2], 5)
    lbsq.step_batch(sims, 11)
    counts = [7 + 11, 7 + 3 + 5 + 11, 7 + 11, 7 + 11]
    counts[0] += 5
    for (shape, bodies, _), s, n in zip(sel, sims, counts):
        ref = alone(lbsq, shape, bodies, n)
        assert s.info()["steps"] == n
        assert np.array_equal(s.populations(), ref["pops"]), "populations differ for %s" % (shape,)
        for i in range(len(bodies)):
            st = s.body(i)
            F, T = s.force_torque(i)
            assert np.array_equal(st["pos"], ref["pos"][i]) and np.array_equal(st["v"], ref["v"][i])
            assert np.array_equal(F, ref["F"][i]) and np.array_equal(T, ref["T"][i])
        s.close()


def test_step_batch_rejects_repeated_handle():
    lbsq = gpu()
    s = lbsq.Sim((16, 16, 16))
    with pytest.raises(lbsq.LBError) as ei:
        lbsq.step_batch([s, s], 1)
    assert ei.value.code == lbsq.LB_EINVAL


def run_server(lbsq, requests, storage="f32", use_graph=True, chunk=8, max_active=3, budget=None,
               layout="inplace"):
    if budget is None:
        budget = 1 << 30
    results = {}
    with lbsq.Server(budget, max_active=max_active, chunk_steps=chunk, use_graph=use_graph,
                     storage=storage, layout=layout) as sv:
        tickets = {}
        # half the requests up front, the rest while the first ones run
        for j, (shape, bodies, n) in enumerate(requests[: len(requests) // 2]):
            tickets[sv.submit(shape, bodies, n, tag=j)] = j
        sv.progress()
        for j, (shape, bodies, n) in enumerate(requests[len(requests) // 2:], start=len(requests) // 2):
            tickets[sv.submit(shape, bodies, n, tag=j)] = j
            sv.progress()
        spins = 0
        while len(results) < len(requests):
            sv.progress(wait=True)
            for r in sv.results():
                results[r["tag"]] = r
            spins += 1
            assert spins < 10000, "server made no progress"
        stats = sv.stats()
    return results, stats


@pytest.mark.parametrize("use_graph", [True, False])
def test_server_matches_alone(use_graph):
    note("server vs lb_step, graph=%s" % use_graph)
    lbsq = gpu()
    results, stats = run_server(lbsq, REQUESTS, use_graph=use_graph)
    note("stats %s" % stats)
    assert stats["completed"] == len(REQUESTS)
    if use_graph:
        assert stats["graphs"] >= 1
    for j, (shape, bodies, n) in enumerate(REQUESTS):
        r = results[j]
        assert r["status"] == lbsq.LB_OK, lbsq.strerror(r["status"])
        assert r["steps"] == n and r["nbody"] == len(bodies)
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        ref = alone(lbsq, shape, bodies, n)
        assert r["fluid_cells"] == ref["fluid"]
        assert_same(r, ref, "request %d" % j)


def test_server_f16_matches_alone():
    note("server f16 storage vs lb_step f16")
    lbsq = gpu()
    sel = REQUESTS[:4]
    results, _ = run_server(lbsq, sel, storage="f16", chunk=16, max_active=4)
    for j, (shape, bodies, n) in enumerate(sel):
        assert results[j]["status"] == lbsq.LB_OK
        assert_same(results[j], alone(lbsq, shape, bodies, n, storage="f16"), "f16 request %d" % j)


def test_server_budget_admission():
    """An arena that holds one request at a time: requests run one after the
    other, each admitted only once the previous one has left, and every
    result is still exact."""
    note("server admission by budget")
    lbsq = gpu()
    sel = [REQUESTS[0], REQUESTS[5], REQUESTS[0]]
    # a 24^3 or 26^3 request needs 4-5 MiB (populations, owners, bodies,
    # force sums): 6 MiB holds one of them, never two
    budget = 6 << 20
    results, stats = run_server(lbsq, sel, chunk=10, max_active=3, budget=budget)
    order = sorted(results.values(), key=lambda r: r["t_admit"])
    for a, b in zip(order, order[1:]):
        assert b["t_admit"] >= a["t_done"], "admitted before the previous request left"
    assert stats["arena_in_use"] == 0
    for j, (shape, bodies, n) in enumerate(sel):
        assert results[j]["status"] == lbsq.LB_OK
        assert_same(results[j], alone(lbsq, shape, bodies, n), "budget request %d" % j)
    with lbsq.Server(budget) as sv:
        with pytest.raises(lbsq.LBError) as ei:
            sv.submit((128, 128, 128), [], 1)
        assert ei.value.code == lbsq.LB_EBUDGET


def test_server_reports_geometry_errors():
    """Overlapping bodies end the request with LB_EGEOM, not the server."""
    lbsq = gpu()
    bad = ((24, 24, 24), [dict(pos=(12, 12, 12), R=4.0), dict(pos=(14, 12, 12), R=4.0)], 5)
    results, _ = run_server(lbsq, [bad, REQUESTS[4]])
    assert results[0]["status"] == lbsq.LB_EGEOM
    assert results[1]["status"] == lbsq.LB_OK


def test_server_cancel():
    """Cancelling a queued request ends it at once, with LB_ECANCELED and no
    steps. Cancelling a resident one takes it out of the batch at a chunk
    boundary; it then reports the steps it ran. The request left in the
    batch still matches its standalone run bit for bit, and the arena is
    empty at the end."""
    note("server cancellation")
    lbsq = gpu()
    keep, other, queued = REQUESTS[0], REQUESTS[3], REQUESTS[5]
    results = {}
    with lbsq.Server(1 << 30, max_active=2, chunk_steps=8) as sv:
        tk = sv.submit(keep[0], keep[1], keep[2], tag=0)
        to = sv.submit(other[0], other[1], 200, tag=1)
        tq = sv.submit(queued[0], queued[1], queued[2], tag=2)  # waits for a slot
        assert sv.cancel(tq)
        assert not sv.cancel(tq)
        sv.progress()
        sv.progress()
        assert sv.cancel(to)
        spins = 0
        while len(results) < 3:
            sv.progress(wait=True)
            for r in sv.results():
                results[r["tag"]] = r
            spins += 1
            assert spins < 10000, "server made no progress"
        assert not sv.cancel(tk)
        with pytest.raises(lbsq.LBError) as ei:
            sv.cancel(10 ** 6)
        assert ei.value.code == lbsq.LB_EINVAL
        stats = sv.stats()
    assert results[2]["status"] == lbsq.LB_ECANCELED and results[2]["steps"] == 0
    assert results[1]["status"] == lbsq.LB_ECANCELED
    assert 0 < results[1]["steps"] < 200 and results[1]["steps"] % 8 == 0
    assert results[0]["status"] == lbsq.LB_OK and results[0]["steps"] == keep[2]
    assert_same(results[0], alone(lbsq, keep[0], keep[1], keep[2]), "request kept beside cancellations")
    assert stats["arena_in_use"] == 0


def test_server_isolates_a_diverging_request():
    """A request whose fluid diverges (a slip of 5 lattice units per step,
    far beyond the lattice speed) ends with its own error, LB_ENAN or
    LB_EGEOM. The request batched with it still matches its standalone run
    bit for bit."""
    note("server: diverging request beside a normal one")
    lbsq = gpu()
    bad = ((24, 24, 24), [dict(pos=(12.2, 11.8, 12.1), e=(1, 0, 0), R=4.0, B1=5.0, beta=0.0)], 120)
    good = REQUESTS[0]
    results, stats = run_server(lbsq, [bad, good], chunk=8, max_active=2)
    assert results[0]["status"] in (lbsq.LB_ENAN, lbsq.LB_EGEOM), lbsq.strerror(results[0]["status"])
    assert results[1]["status"] == lbsq.LB_OK
    assert_same(results[1], alone(lbsq, good[0], good[1], good[2]), "request beside a diverging one")
    assert stats["arena_in_use"] == 0


def test_step_batch_mixes_layouts():
    """lb_step_batch over simulations in the in-place and the two-buffer
    layout at once: each block takes its own simulation's layout, and every
    result equals the same simulation stepped alone."""
    note("lb_step_batch with both population layouts")
    lbsq = gpu()
    sel = [(REQUESTS[0], "ab"), (REQUESTS[1], "inplace"), (REQUESTS[5], "ab")]
    sims = []
    for (shape, bodies, _), layout in sel:
        s = lbsq.Sim(shape, layout=layout)
        for b in bodies:
            s.add_squirmer(**b)
        sims.append(s)
    lbsq.step_batch(sims, 9)
    lbsq.step_batch(sims, 14)
    for ((shape, bodies, _), layout), s in zip(sel, sims):
        ref = lbsq.Sim(shape, layout=layout)
        for b in bodies:
            ref.add_squirmer(**b)
        ref.step(23)
        assert np.array_equal(s.populations(), ref.populations()), layout
        for i in range(len(bodies)):
            for k in ("pos", "v", "w"):
                assert np.array_equal(s.body(i)[k], ref.body(i)[k])
        ref.close()
        s.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_server_two_buffer_layout_matches_alone(storage):
    """Requests served in the two-buffer pull layout equal the same
    simulations stepped alone in that layout, bit for bit."""
    note("server in the two-buffer layout, %s" % storage)
    lbsq = gpu()
    sel = REQUESTS[:4]
    results, stats = run_server(lbsq, sel, storage=storage, chunk=16, max_active=3, layout="ab")
    assert stats["arena_in_use"] == 0
    for j, (shape, bodies, n) in enumerate(sel):
        assert results[j]["status"] == lbsq.LB_OK
        assert_same(results[j], alone(lbsq, shape, bodies, n, storage=storage, layout="ab"), "ab request %d" % j)

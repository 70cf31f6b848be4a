"""Throughput of the fused D3Q19 squirmer step on one MI355X.

Workload of `value` (the plain FP32 configuration): 128^3 periodic box,
nu = 1/6, one free squirmer of radius 8 at the box centre swimming along +x,
B1 = 1e-3, beta = 0, FP32 deviation storage, the library's default
population layout.  One step is the whole path: fused stream-collide-
bounce-back with the momentum exchange, rigid-body update, geometry and cell
conversion.  Every leg develops the flow first (at least 4 max(n) steps, so
that no part of the box still streams the exact zeros of the fluid at rest)
and then times its steps with inputs resident in device memory.

Prints one JSON line:
  - value: MLUPS over fluid cells at 128^3;
  - roofline: the fluid-update kernel where its populations stream from HBM
    (256^3, R = 16; 2.55 GB in the pull layout), from HIP events on the
    stream it runs on, beside the committed rocprofv3 figures of the same
    configuration (used only while the kernel sources are the ones profiled);
  - roofline_llc: the same kernel at 128^3, whose populations fit the 256 MB
    last-level cache;
  - fp16_storage: FP16 deviation storage at 128^3 (at 256^3 under roofline);
  - tube: the confined scene, MFLUPS over its fluid cells;
  - audit: the cost of the fused FP64 mass/momentum audit;
  - served: the continuous-batching server on a seeded Poisson request
    stream (capacity, then p50/p99 latency at a fixed rate, FP32 and FP16);
  - cpu_baseline: the FP64 CPU oracle on a bounded sample of the 128^3
    workload, on all host threads and on one.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 152, "f16": 76, "bf16": 76}
PROFILES = Path(ROOT) / "profiles"
TRACE_256 = PROFILES / "k_fluid_256cube_kernel_trace.md"
TRAFFIC_256 = PROFILES / "k_fluid_256cube_traffic.md"
TRACE_TUBE = PROFILES / "k_fluid_tube_kernel_trace.md"
LEGS = ("value", "roofline", "fp16", "tube", "audit", "serve", "cpu")


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in ("lbsq_kernels.hip", "lbsq_device.h", "lbsq_launch.h"):
        h.update((Path(ROOT) / "paper_1903_04799_amd" / "csrc" / f).read_bytes())
    return h.hexdigest()[:16]


def profile_values(path):
    """key = value lines of a committed profile summary, or None unless the
    summary was taken on the kernel sources as they stand."""
    if not path.exists():
        return None
    kv = {}
    for line in path.read_text().splitlines():
        if "=" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256_16") != kernel_sources_hash():
        return None
    return kv


def profiled(path, key):
    kv = profile_values(path)
    v = kv.get(key) if kv else None
    return float(v) if v else None


def copy_calibration(mib, reps=5):
    """A plain device-to-device copy of known size (torch's copy kernel), run
    beside the step so that hardware byte counters (FETCH_SIZE, WRITE_SIZE)
    can be scaled by what they read for exactly mib MiB in and out."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def copy_rate(nbytes, reps=20):
    """GB/s of a plain device copy of nbytes (read + write counted): the
    same-footprint reference for the fluid kernel's bandwidth."""
    import torch
    n = nbytes // 4
    src = torch.randn(n, dtype=torch.float32, device="cuda") * 1e-4
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    s = a.elapsed_time(b) / 1e3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / s / 1e9


def develop_steps(shape, warmup):
    return max(int(warmup), 4 * max(shape))


def run_gpu(storage, shape, R, beta, steps, warmup, layout="auto", mask=None, pos=None, e=(1.0, 0.0, 0.0),
            audit_every=0):
    """Develop the flow, time `steps` steps, then time the fluid launches of
    as many steps again with HIP events (a second pass: per-launch events
    cost host time inside the step loop)."""
    import torch
    from paper_1903_04799_amd import Sim
    c = [s / 2.0 for s in shape] if pos is None else list(pos)
    sim = Sim(shape, storage=storage, layout=layout, audit_every=audit_every)
    if mask is not None:
        sim.set_static_mask(mask)
    sim.add_squirmer(c, e, R, B1=1e-3, beta=beta, mode="free")
    dev = develop_steps(shape, warmup)
    sim.step(dev)
    sim.sync()
    n_fluid = sim.info()["n_fluid"]
    mass0 = sim.audit()[0]  # FP64 fluid mass, outside the timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mass1 = sim.audit()[0]
    n_fluid1 = sim.info()["n_fluid"]
    sim.kernel_timing(True)
    sim.step(steps)
    ms, launches = sim.kernel_time()
    sim.kernel_timing(False)
    b = sim.body(0)
    sim.close()
    torch.cuda.empty_cache()
    avg_s = ms / 1e3 / launches
    bytes_launch = BYTES_PER_UPDATE[storage] * n_fluid
    import numpy as np
    return {
        "mlups": n_fluid * steps / dt / 1e6,
        "ms_per_step": dt * 1e3 / steps,
        "n_fluid": n_fluid,
        "develop_steps": dev,
        "kernel_us": avg_s * 1e6,
        "kernel_gbs": bytes_launch / avg_s / 1e9,
        "bytes_per_launch": bytes_launch,
        "speed_over_v0": float(np.dot(b["v"], b["e"]) / (2.0 / 3.0 * 1e-3)),
        # FP64 fluid mass over the timed steps: its relative change, the
        # change in fluid cells as the sphere moves across the lattice, and
        # the relative change of the mean density (mass per fluid cell)
        "conservation": {"mass_rel_change": (mass1 - mass0) / mass0,
                         "fluid_cells_change": int(n_fluid1) - int(n_fluid),
                         "mean_density_rel_change": (mass1 / n_fluid1) / (mass0 / n_fluid) - 1.0},
    }


def population_bytes(shape, storage, layout):
    """Bytes of the population buffers (planes padded to whole groups of 256
    cells plus one group, 19 planes; two buffers in the pull layout)."""
    n = shape[0] * shape[1] * shape[2]
    stride = ((n + 255) // 256) * 256 + 256
    return 19 * stride * (4 if storage == "f32" else 2) * (2 if layout == "ab" else 1)


def resolved_layout(shape, layout):
    n = shape[0] * shape[1] * shape[2]
    if layout != "auto":
        return layout
    return "ab" if n > 5500000 else "inplace"


def serve(storage, reqs, arrivals, chunk, max_active, budget, layout="auto"):
    """Run the request stream through a server; arrivals None = all at once.
    Latency of a request = completion time - scheduled arrival."""
    import numpy as np
    from paper_1903_04799_amd import lbsq
    n = len(reqs)
    order = list(range(n))
    if arrivals is None:
        arrivals = np.zeros(n)
    done = {}
    with lbsq.Server(budget, max_active=max_active, chunk_steps=chunk, use_graph=True, storage=storage,
                     layout=layout) as sv:
        t0 = sv.clock()
        nxt = 0
        while len(done) < n:
            now = sv.clock() - t0
            while nxt < n and arrivals[order[nxt]] <= now:
                j = order[nxt]
                shape, bodies, steps = reqs[j]
                sv.submit(shape, bodies, steps, tag=j)
                nxt += 1
            active, queued = sv.progress()
            for r in sv.results():
                done[r["tag"]] = r
            if len(done) == n:
                break
            if active == 0 and queued == 0 and nxt < n:
                time.sleep(max(0.0, min(0.05, arrivals[order[nxt]] - (sv.clock() - t0))))
            elif active or queued:
                sv.progress(wait=True)
                for r in sv.results():
                    done[r["tag"]] = r
        stats = sv.stats()
    bad = [r for r in done.values() if r["status"] != 0]
    if bad:
        raise RuntimeError("served request failed: %s" % lbsq.strerror(bad[0]["status"]))
    lat = np.array([done[j]["t_done"] - t0 - arrivals[j] for j in range(n)])
    t_end = max(r["t_done"] for r in done.values()) - t0
    span = t_end - float(np.min(arrivals))
    # swim speed along e of each single squirmer after its run, per request
    speed = {j: float(np.dot(done[j]["v"][0], done[j]["e"][0])) for j in range(n) if done[j]["nbody"] == 1}
    return {"mlups": stats["cell_updates"] / span / 1e6, "p50_ms": float(np.percentile(lat, 50)) * 1e3,
            "p99_ms": float(np.percentile(lat, 99)) * 1e3, "span_s": span, "req_per_s": n / span,
            "chunks": stats["chunks"], "graphs": stats["graphs"], "speed": speed}


def run_served(n_req, seed, chunk, max_active, budget_gb, storages, layout="auto"):
    """Capacity (all requests at once) in FP32, then each storage at a fixed
    Poisson rate of 0.6 x that capacity."""
    import numpy as np
    from paper_1903_04799_amd import workloads
    budget = int(budget_gb * (1 << 30))
    reqs = workloads.request_stream(n_req, seed=seed)
    warm = workloads.request_stream(2, seed=seed + 1, steps=50)
    serve("f32", warm, None, chunk, max_active, budget, layout)
    cap = serve("f32", reqs, None, chunk, max_active, budget, layout)
    qps = 0.6 * cap["req_per_s"]
    arrivals = workloads.poisson_arrivals(n_req, qps, seed=seed)
    out = {"workload": "Poisson stream of %d requests (seed %d): cubic boxes {48..192}^3, R {4,6,8,12}, "
                       "beta U[-5,5], B1 1e-3, 1000 steps, half single squirmers, half pairs" % (n_req, seed),
           "capacity_req_per_s": round(cap["req_per_s"], 2), "capacity_mlups": round(cap["mlups"], 1),
           "qps": round(qps, 2), "chunk_steps": chunk, "max_active": max_active,
           "layout": "ab" if layout == "auto" else layout}
    speeds = {}
    for st in storages:
        r = serve(st, reqs, arrivals, chunk, max_active, budget, layout)
        speeds[st] = r.pop("speed")
        out[st] = {"mlups": round(r["mlups"], 1), "p50_ms": round(r["p50_ms"], 1), "p99_ms": round(r["p99_ms"], 1),
                   "req_per_s": round(r["req_per_s"], 2), "chunks": r["chunks"], "graphs": r["graphs"]}
    if "f32" in speeds and "f16" in speeds:
        rel = [abs(speeds["f16"][j] - speeds["f32"][j]) / abs(speeds["f32"][j]) for j in speeds["f32"]
               if speeds["f32"][j] != 0.0]
        out["f16_swim_speed_rel_diff_max"] = float(np.max(rel)) if rel else None
    return out


def cpu_model():
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(shape, R, beta, seconds):
    """The FP64 oracle (as it stands) on a bounded sample of the workload:
    first on every thread it runs on, then on one thread."""
    from oracle import oracle as O
    O.build()
    c = [s / 2.0 for s in shape]
    o = O.OracleSim(*shape)
    o.add_body(c, (1.0, 0.0, 0.0), R, B1=1e-3, beta=beta)
    o.step(1)
    n_fluid = int((o.fields()[2] == 0).sum())
    res = []
    threads_all = O.threads()
    for nthr in (threads_all, 1):
        O.set_threads(nthr)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds:
            o.step(1)
            steps += 1
        dt = time.perf_counter() - t0
        res.append((nthr, steps, dt))
    O.set_threads(threads_all)
    o.close()
    (nall, sall, dall), (_, s1, d1) = res
    return {"value": n_fluid * sall / dall / 1e6, "unit": "MLUPS", "cores": nall, "kind": "oracle",
            "sample": "%dx%dx%d box, R=%g squirmer, %d FP64 steps (%.1f s) on %d OpenMP threads"
                      % (*shape, R, sall, dall, nall),
            "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
            "single_core": {"value": n_fluid * s1 / d1 / 1e6, "unit": "MLUPS", "cores": 1,
                            "sample": "%d FP64 steps (%.1f s) on one thread" % (s1, d1)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps before timing (at least 4 max(n) are taken, to develop the flow)")
    ap.add_argument("--n", type=int, default=128, help="cubic box edge of the value leg")
    ap.add_argument("--R", type=float, default=8.0)
    ap.add_argument("--beta", type=float, default=0.0)
    ap.add_argument("--layout", choices=["auto", "inplace", "ab"], default="auto",
                    help="population layout of the value leg (the library default is auto)")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated subset of %s" % ",".join(LEGS))
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain copy of this many MiB (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-seed", type=int, default=0)
    ap.add_argument("--serve-chunk", type=int, default=200)
    ap.add_argument("--serve-active", type=int, default=16)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-layout", choices=["auto", "inplace", "ab"], default="auto",
                    help="population layout of the served requests (auto: the pull layout)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    legs = set(x.strip() for x in args.legs.split(",") if x.strip())
    if not legs <= set(LEGS):
        print("unknown legs: %s" % sorted(legs - set(LEGS)), file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        copy_calibration(args.copy_calibration_mib)
    shape = (args.n, args.n, args.n)
    out = {"metric": "D3Q19 MLUPS FP32 vs FP16-storage; served sweep p50/p99 latency at fixed error",
           "value": None, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic"}
    lay = resolved_layout(shape, args.layout)
    if "value" in legs:
        f32 = run_gpu("f32", shape, args.R, args.beta, args.steps, args.warmup, args.layout)
        out["value"] = round(f32["mlups"], 1)
        out["ms_per_step"] = round(f32["ms_per_step"], 5)
        out["config"] = {"workload": "free squirmer R = %g in a periodic %d^3 box" % (args.R, args.n),
                         "box": list(shape), "R": args.R, "beta": args.beta, "B1": 1e-3, "nu": 1 / 6,
                         "storage": "f32 deviations", "layout": lay, "n_fluid": f32["n_fluid"],
                         "developed": True, "develop_steps": f32["develop_steps"]}
        ws = population_bytes(shape, "f32", lay)
        out["roofline_llc"] = {"bound": "llc", "achieved": round(f32["kernel_gbs"], 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(f32["kernel_gbs"] / HBM_PEAK_GBS, 4),
                               "kernel": "k_fluid", "kernel_us": round(f32["kernel_us"], 2),
                               "working_set_mb": round(ws / 1e6, 1),
                               "note": "populations fit the 256 MB last-level cache; the peak is HBM's"}
        out["conservation"] = f32["conservation"]
        # speed along e at the end of the run over 2 B1 / 3, in this periodic
        # box (its finite-size correction is not taken out here)
        out["swim_speed_over_v0"] = round(f32["speed_over_v0"], 5)
    if "roofline" in legs:
        # the same kernel where its populations stream from HBM: 256^3, the
        # library default layout there (pull, two buffers, 2.55 GB)
        n2 = (256, 256, 256)
        k2 = max(args.steps, 100)
        h = run_gpu("f32", n2, 16.0, args.beta, k2, args.warmup)
        l2 = resolved_layout(n2, "auto")
        ws = population_bytes(n2, "f32", l2)
        prof_us = profiled(TRACE_256, "k_fluid_us_f32_" + l2)
        cp = copy_rate(ws // 2)
        out["roofline"] = {"bound": "hbm", "achieved": round(h["kernel_gbs"], 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(h["kernel_gbs"] / HBM_PEAK_GBS, 4),
                           "traffic": profiled(TRAFFIC_256, "traffic_bytes_per_launch_f32_" + l2),
                           "traffic_unit": "bytes/launch", "kernel": "k_fluid",
                           "workload": "free squirmer R = 16 in a periodic 256^3 box, FP32, %s layout" % l2,
                           "kernel_us": round(h["kernel_us"], 2), "steps_timed": k2,
                           "algorithmic_bytes_per_launch": h["bytes_per_launch"], "bytes_per_update": 152,
                           "n_fluid": h["n_fluid"], "working_set_mb": round(ws / 1e6, 1),
                           "step_mlups": round(h["mlups"], 1), "ms_per_step": round(h["ms_per_step"], 5),
                           "developed": True, "develop_steps": h["develop_steps"],
                           "profile_kernel_us": prof_us,
                           "profile_frac": (round(h["bytes_per_launch"] / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                            if prof_us else None),
                           "copy_gbs_same_footprint": round(cp, 1),
                           "frac_of_copy": round(h["kernel_gbs"] / cp, 4)}
        hi = run_gpu("f32", n2, 16.0, args.beta, k2, args.warmup, "inplace")
        out["roofline"]["inplace"] = {"kernel_us": round(hi["kernel_us"], 2),
                                      "achieved": round(hi["kernel_gbs"], 1),
                                      "frac": round(hi["kernel_gbs"] / HBM_PEAK_GBS, 4),
                                      "step_mlups": round(hi["mlups"], 1),
                                      "working_set_mb": round(population_bytes(n2, "f32", "inplace") / 1e6, 1),
                                      "profile_kernel_us": profiled(TRACE_256, "k_fluid_us_f32_inplace")}
        h16 = run_gpu("f16", n2, 16.0, args.beta, k2, args.warmup)
        prof16 = profiled(TRACE_256, "k_fluid_us_f16_" + l2)
        out["roofline"]["f16"] = {
            "mlups": round(h16["mlups"], 1), "kernel_us": round(h16["kernel_us"], 2),
            "achieved": round(h16["kernel_gbs"], 1), "frac": round(h16["kernel_gbs"] / HBM_PEAK_GBS, 4),
            "bytes_per_update": 76, "traffic": profiled(TRAFFIC_256, "traffic_bytes_per_launch_f16_" + l2),
            "working_set_mb": round(population_bytes(n2, "f16", l2) / 1e6, 1), "profile_kernel_us": prof16,
            "profile_frac": (round(h16["bytes_per_launch"] / (prof16 * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                             if prof16 else None)}
    if "fp16" in legs:
        f16 = run_gpu("f16", shape, args.R, args.beta, args.steps, args.warmup, args.layout)
        out["fp16_storage"] = {"value": round(f16["mlups"], 1), "unit": "MLUPS",
                               "workload": "as the value leg, FP16 deviations (scale 2^14)",
                               "ms_per_step": round(f16["ms_per_step"], 5),
                               "kernel_us": round(f16["kernel_us"], 2),
                               "kernel_gbs": round(f16["kernel_gbs"], 1), "bytes_per_update": 76,
                               "speedup_vs_f32": (round(f16["mlups"] / out["value"], 3) if out["value"] else None),
                               "conservation": f16["conservation"],
                               "swim_speed_over_v0": round(f16["speed_over_v0"], 5)}
    if "tube" in legs:
        # the confined scene: 96 x 96 x 512, static tube wall of radius 24
        # (80% of the cells), squirmer R = 12 on the axis along +z
        import numpy as np
        from tests.scenes import tube_mask
        ts = (96, 96, 512)
        mask = tube_mask(*ts, 24.0)
        t = {}
        for st in ("f32", "f16"):
            r = run_gpu(st, ts, 12.0, args.beta, args.steps, args.warmup, "auto", mask=mask,
                        pos=(48.0, 48.0, 256.0), e=(0.0, 0.0, 1.0))
            t[st] = r
        n = ts[0] * ts[1] * ts[2]
        # what the wall costs: groups of 256 consecutive cells (x fastest)
        # that hold only walls get no streaming block; in the other groups
        # a wall cell's lane loads only its owner byte, but the fluid lanes'
        # loads bring in whole 128-byte lines, wall slots included (the
        # committed counter traffic below)
        wall = mask.reshape(-1).astype(bool)
        ng = (n + 255) // 256
        grp_wall = np.logical_and.reduceat(wall, np.arange(0, n, 256))
        walls_streamed = int(wall.reshape(ng, 256)[~grp_wall].sum()) if n % 256 == 0 else None
        fl = t["f32"]["n_fluid"]
        traffic = profiled(TRACE_TUBE, "traffic_bytes_per_launch_f32_tube")
        prof_us = profiled(TRACE_TUBE, "k_fluid_us_f32_tube")
        # the same scene rotated so that the tube runs along x, the fastest
        # axis of the cell numbering: every x-row is then all wall or all fluid
        tx = (ts[2], ts[1], ts[0])
        mask_x = tube_mask(*tx, 24.0, axis="x")
        ax = {}
        for st in ("f32", "f16"):
            ax[st] = run_gpu(st, tx, 12.0, args.beta, args.steps, args.warmup, "auto", mask=mask_x,
                             pos=(256.0, 48.0, 48.0), e=(1.0, 0.0, 0.0))
        wall_x = mask_x.reshape(-1).astype(bool)
        grp_x = np.logical_and.reduceat(wall_x, np.arange(0, n, 256))
        out["tube"] = {"workload": "squirmer R = 12 on the axis of a tube of radius 24 in 96x96x512 "
                                   "(static no-slip wall, 80% of the cells)",
                       "cells": n, "fluid_cells": fl,
                       "mflups_f32": round(t["f32"]["mlups"], 1), "mflups_f16": round(t["f16"]["mlups"], 1),
                       "kernel_us_f32": round(t["f32"]["kernel_us"], 2),
                       "kernel_us_f16": round(t["f16"]["kernel_us"], 2),
                       "fluid_gbs_f32": round(t["f32"]["kernel_gbs"], 1),
                       "fluid_gbs_f16": round(t["f16"]["kernel_gbs"], 1),
                       "frac_f32": round(t["f32"]["kernel_gbs"] / HBM_PEAK_GBS, 4),
                       "streamed_groups": int((~grp_wall).sum()), "groups": int(ng),
                       "requested_bytes_per_wall_cell": (round(walls_streamed / int(wall.sum()), 4)
                                                         if walls_streamed is not None else None),
                       "traffic": traffic, "traffic_unit": "bytes/launch (FP32, committed rocprofv3 counters)",
                       "traffic_over_fluid_algorithmic": (round(traffic / (152.0 * fl), 3) if traffic else None),
                       "profile_kernel_us_f32": prof_us,
                       "note": "GB/s count 152 / 76 B per fluid-cell update only. Groups of 256 cells that hold "
                               "only walls get no block; a wall cell elsewhere requests its owner byte "
                               "(requested_bytes_per_wall_cell averages that over all wall cells), but shares "
                               "128-byte lines with fluid cells, whose loads bring its slots in: the counter "
                               "traffic is the measured cost",
                       "along_x": {"workload": "the same scene rotated: 512x96x96, tube along x",
                                   "mflups_f32": round(ax["f32"]["mlups"], 1),
                                   "mflups_f16": round(ax["f16"]["mlups"], 1),
                                   "kernel_us_f32": round(ax["f32"]["kernel_us"], 2),
                                   "kernel_us_f16": round(ax["f16"]["kernel_us"], 2),
                                   "fluid_gbs_f32": round(ax["f32"]["kernel_gbs"], 1),
                                   "frac_f32": round(ax["f32"]["kernel_gbs"] / HBM_PEAK_GBS, 4),
                                   "streamed_groups": int((~grp_x).sum())}}
    if "audit" in legs:
        # the fused FP64 audit: a step with it against one without
        plain = run_gpu("f32", shape, args.R, args.beta, args.steps, args.warmup, args.layout)
        aud = run_gpu("f32", shape, args.R, args.beta, args.steps, args.warmup, args.layout, audit_every=1)
        extra = aud["ms_per_step"] - plain["ms_per_step"]
        out["audit"] = {"ms_per_step_plain": round(plain["ms_per_step"], 5),
                        "ms_per_step_audited": round(aud["ms_per_step"], 5),
                        "audited_step_extra_us": round(extra * 1e3, 2),
                        "overhead_at_every_100": round(extra / 100.0 / plain["ms_per_step"], 5)}
    if "serve" in legs:
        out["served"] = run_served(args.serve_requests, args.serve_seed, args.serve_chunk, args.serve_active,
                                   args.serve_budget_gb, ["f32", "f16"], args.serve_layout)
    if "cpu" in legs:
        out["cpu_baseline"] = cpu_baseline(shape, args.R, args.beta, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

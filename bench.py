"""Throughput of the fused D3Q19 squirmer step on one MI355X.

Workload (default): 128^3 periodic box, nu = 1/6, one free squirmer of
radius 8 at the box centre swimming along +x, B1 = 1e-3, beta = 0, FP32
deviation storage.  One step is the whole path: geometry, conversion, force
and torque, fused stream-collide-bounce-back, rigid-body update.

Prints one JSON line: MLUPS over fluid cells (inputs resident in HBM), the
roofline of the fluid-update kernel measured with HIP events on the stream it
runs on, the same figures for FP16 deviation storage, the served form (a
seeded Poisson stream of independent requests through the continuous-batching
server: capacity, then p50/p99 latency at a fixed rate, FP32 and FP16), and
the FP64 CPU oracle timed on a bounded sample of the same workload.
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


TRAFFIC_FILE = Path(ROOT) / "profiles" / "k_fluid_128cube_traffic.md"


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in ("lbsq_kernels.hip", "lbsq_device.h", "lbsq_launch.h"):
        h.update((Path(ROOT) / "paper_1903_04799_amd" / "csrc" / f).read_bytes())
    return h.hexdigest()[:16]


def measured_traffic(storage, shape, R):
    """HBM bytes per launch of the fluid kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size); None
    unless the kernels are the ones the counters were taken on and the
    workload is the one they were taken for."""
    if tuple(shape) != (128, 128, 128) or R != 8.0 or not TRAFFIC_FILE.exists():
        return None
    kv = {}
    for line in TRAFFIC_FILE.read_text().splitlines():
        if "=" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("traffic_sources_sha256_16") != kernel_sources_hash():
        return None
    v = kv.get("traffic_bytes_per_launch_" + storage)
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


def run_gpu(storage, shape, R, beta, steps, warmup, layout="inplace"):
    import torch
    from paper_1903_04799_amd import Sim
    c = [s / 2.0 for s in shape]
    sim = Sim(shape, storage=storage, layout=layout)
    sim.add_squirmer(c, (1.0, 0.0, 0.0), R, B1=1e-3, beta=beta, mode="free")
    sim.step(warmup)
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
    # kernel-level timing of the fused stream-collide launches (HIP events
    # recorded on the simulation's own stream)
    sim.kernel_timing(True)
    sim.step(steps)
    ms, launches = sim.kernel_time()
    sim.kernel_timing(False)
    v = sim.body(0)["v"]
    sim.close()
    avg_s = ms / 1e3 / launches
    bytes_launch = BYTES_PER_UPDATE[storage] * n_fluid
    return {
        "mlups": n_fluid * steps / dt / 1e6,
        "ms_per_step": dt * 1e3 / steps,
        "n_fluid": n_fluid,
        "kernel_us": avg_s * 1e6,
        "kernel_gbs": bytes_launch / avg_s / 1e9,
        "bytes_per_launch": bytes_launch,
        "v_over_v0": float(v[0] / (2.0 / 3.0 * 1e-3)),
        # FP64 fluid mass over the timed steps: its relative change, the
        # change in fluid cells as the sphere moves across the lattice, and
        # the relative change of the mean density (mass per fluid cell)
        "conservation": {"mass_rel_change": (mass1 - mass0) / mass0,
                         "fluid_cells_change": int(n_fluid1) - int(n_fluid),
                         "mean_density_rel_change": (mass1 / n_fluid1) / (mass0 / n_fluid) - 1.0},
    }


def serve(storage, reqs, arrivals, chunk, max_active, budget, layout="inplace"):
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


def run_served(n_req, seed, chunk, max_active, budget_gb, storages, layout="inplace"):
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
           "qps": round(qps, 2), "chunk_steps": chunk, "max_active": max_active, "layout": layout}
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


def cpu_baseline(shape, R, beta, seconds):
    from oracle import oracle as O
    O.build()
    c = [s / 2.0 for s in shape]
    o = O.OracleSim(*shape)
    o.add_body(c, (1.0, 0.0, 0.0), R, B1=1e-3, beta=beta)
    o.step(1)
    n_fluid = int((o.fields()[2] == 0).sum())
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_fluid * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%dx%dx%d box, R=%g squirmer, %d FP64 steps (%.1f s)" % (*shape, R, steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=128, help="cubic box edge")
    ap.add_argument("--R", type=float, default=8.0)
    ap.add_argument("--beta", type=float, default=0.0)
    ap.add_argument("--layout", choices=["inplace", "ab"], default="inplace",
                    help="population layout of the main run: one buffer in place, or two buffers (pull)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-hbm", action="store_true",
                    help="skip the 256^3 run whose working set exceeds the last-level cache")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain copy of this many MiB (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-seed", type=int, default=0)
    ap.add_argument("--serve-chunk", type=int, default=200)
    ap.add_argument("--serve-active", type=int, default=16)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-layout", choices=["inplace", "ab"], default="ab",
                    help="population layout of the served requests (the batch streams from HBM, where the "
                         "two-buffer layout is faster)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    shape = (args.n, args.n, args.n)
    if args.copy_calibration_mib > 0:
        copy_calibration(args.copy_calibration_mib)
    f32 = run_gpu("f32", shape, args.R, args.beta, args.steps, args.warmup, args.layout)
    out = {
        "metric": "D3Q19 MLUPS FP32 vs FP16-storage; served sweep p50/p99 latency at fixed error",
        "value": round(f32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "free squirmer in a periodic %d^3 box" % args.n, "box": list(shape),
                   "R": args.R, "beta": args.beta, "B1": 1e-3, "nu": 1 / 6, "storage": "f32 deviations",
                   "layout": args.layout,
                   "n_fluid": f32["n_fluid"]},
        "roofline": {"bound": "hbm", "achieved": round(f32["kernel_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(f32["kernel_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("f32", shape, args.R), "traffic_unit": "bytes/launch",
                     "algorithmic_bytes_per_launch": f32["bytes_per_launch"],
                     "kernel": "k_fluid", "kernel_us": round(f32["kernel_us"], 2),
                     "bytes_per_update": BYTES_PER_UPDATE["f32"]},
        "conservation": f32["conservation"],
        # swim speed along x at the end of the run over 2 B1 / 3, in this
        # periodic box (its finite-size correction is not taken out here)
        "swim_speed_over_v0": round(f32["v_over_v0"], 5),
    }
    if not args.no_fp16:
        f16 = run_gpu("f16", shape, args.R, args.beta, args.steps, args.warmup, args.layout)
        out["fp16_storage"] = {"value": round(f16["mlups"], 1), "unit": "MLUPS",
                               "ms_per_step": round(f16["ms_per_step"], 5),
                               "kernel_us": round(f16["kernel_us"], 2),
                               "kernel_gbs": round(f16["kernel_gbs"], 1), "bytes_per_update": 76,
                               "traffic": measured_traffic("f16", shape, args.R),
                               "speedup_vs_f32": round(f16["mlups"] / f32["mlups"], 3),
                               "conservation": f16["conservation"],
                               "swim_speed_over_v0": round(f16["v_over_v0"], 5)}
    if not args.no_hbm:
        # the same kernel where the in-place working set (1.28 GB) cannot
        # stay in the 256 MB last-level cache: the HBM-bound figure
        n2 = (256, 256, 256)
        h = run_gpu("f32", n2, 16.0, args.beta, 200, 50)
        ws = 19 * (((256 ** 3 + 255) // 256) * 256 + 256) * 4
        out["hbm_bound"] = {"workload": "free squirmer R = 16 in a periodic 256^3 box", "mlups": round(h["mlups"], 1),
                            "ms_per_step": round(h["ms_per_step"], 5), "kernel_us": round(h["kernel_us"], 2),
                            "achieved_gbs": round(h["kernel_gbs"], 1),
                            "frac": round(h["kernel_gbs"] / HBM_PEAK_GBS, 4),
                            "working_set_mb": round(ws / 1e6, 1), "layout": "inplace"}
        # the same with two population buffers (pull streaming), the layout
        # for boxes that stream from HBM
        h2 = run_gpu("f32", n2, 16.0, args.beta, 200, 50, "ab")
        out["hbm_bound"]["ab"] = {"mlups": round(h2["mlups"], 1), "ms_per_step": round(h2["ms_per_step"], 5),
                                  "kernel_us": round(h2["kernel_us"], 2), "achieved_gbs": round(h2["kernel_gbs"], 1),
                                  "frac": round(h2["kernel_gbs"] / HBM_PEAK_GBS, 4),
                                  "working_set_mb": round(2 * ws / 1e6, 1)}
    if not args.no_serve:
        out["served"] = run_served(args.serve_requests, args.serve_seed, args.serve_chunk, args.serve_active,
                                   args.serve_budget_gb, ["f32"] if args.no_fp16 else ["f32", "f16"],
                                   args.serve_layout)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(shape, args.R, args.beta, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

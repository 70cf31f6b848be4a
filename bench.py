"""Throughput of the fused D3Q19 squirmer step on one MI355X.

Workload (default): 128^3 periodic box, nu = 1/6, one free squirmer of
radius 8 at the box centre swimming along +x, B1 = 1e-3, beta = 0, FP32
deviation storage.  One step is the whole path: geometry, conversion, force
and torque, fused stream-collide-bounce-back, rigid-body update.

Prints one JSON line: MLUPS over fluid cells (inputs resident in HBM), the
roofline of the fused stream-collide kernel measured with HIP events on the
stream it runs on, the same figures for FP16 deviation storage, and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 152, "f16": 76, "bf16": 76}


def run_gpu(storage, shape, R, beta, steps, warmup):
    import torch
    from paper_1903_04799_amd import Sim
    c = [s / 2.0 for s in shape]
    sim = Sim(shape, storage=storage)
    sim.add_squirmer(c, (1.0, 0.0, 0.0), R, B1=1e-3, beta=beta, mode="free")
    sim.step(warmup)
    sim.sync()
    n_fluid = sim.info()["n_fluid"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
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
    }


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
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    shape = (args.n, args.n, args.n)
    f32 = run_gpu("f32", shape, args.R, args.beta, args.steps, args.warmup)
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
                   "n_fluid": f32["n_fluid"]},
        "roofline": {"bound": "hbm", "achieved": round(f32["kernel_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(f32["kernel_gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_fluid", "kernel_us": round(f32["kernel_us"], 2),
                     "bytes_per_update": BYTES_PER_UPDATE["f32"]},
    }
    if not args.no_fp16:
        f16 = run_gpu("f16", shape, args.R, args.beta, args.steps, args.warmup)
        out["fp16_storage"] = {"value": round(f16["mlups"], 1), "unit": "MLUPS",
                               "ms_per_step": round(f16["ms_per_step"], 5),
                               "kernel_us": round(f16["kernel_us"], 2),
                               "kernel_gbs": round(f16["kernel_gbs"], 1), "bytes_per_update": 76,
                               "speedup_vs_f32": round(f16["mlups"] / f32["mlups"], 3)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(shape, args.R, args.beta, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

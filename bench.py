#!/usr/bin/env python3
"""Throughput benchmark of the HO-DMAS beamformer on one MI355X.

Workload (default): 128-element array, 2048 samples per channel, 512 x 512
grid, float32 RF, orders k = 1..6.  A step beamforms a batch of B resident
frames (distinct seeds, already in HBM) at every order: B x 6 launches.  The
metric is beamformed pixel-channel pairs per second (Gpixel*ch/s), summed
over the orders, with the per-order rates beside it.

Prints ONE JSON line.  Also reports:
  roofline      the dominant kernel (the order with the most device time) against
                the VALU issue peak, from HIP events on the launch stream;
  cpu_baseline  the FP64 oracle timed on this host on the same batch.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU slots per pixel-channel for order k: the delay (4 FP32 ops +
# sqrt + reciprocal), interpolation (6), the signed root, k-2 products and k
# power-sum adds; every transcendental (sqrt, rcp, log2, exp2) weighs 4 slots,
# being quarter-rate against the FP32 FMA issue rate.
SLOTS = {1: 19, 2: 25, 3: 32, 4: 32, 5: 36, 6: 38}
# 157.3 TFLOP/s FP32 vector (published) = 78.6e12 FMA lane-slots/s
# (256 CUs x 128 FP32 lanes/clock x 2.4 GHz).
VALU_PEAK_TSLOT = 78.64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8, help="frames per step")
    ap.add_argument("--orders", default="1,2,3,4,5,6")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (for HBM counter scaling)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not part of it "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2203_14906_amd import hodmas, phantom as ph

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    orders = [int(k) for k in args.orders.split(",")]
    p = ph.CONFIGS[2]
    frames = [ph.make_frame(p["n_elements"], p["n_samples"], p["nx"], p["nz"], n_points=p["n_points"],
                            n_lines=p["n_lines"], snr_db=p["snr_db"], seed=2000 + b)
              for b in range(args.batch)]
    geom, grid = frames[0].geometry, frames[0].grid
    n_el, S = p["n_elements"], p["n_samples"]
    plan = hodmas.Plan(geom, grid, S, "f32", max_order=max(orders))
    info = plan.info()
    rf_host = [ph.to_fp32(f.rf) for f in frames]
    rf_dev = [torch.from_numpy(a).to(dev) for a in rf_host]
    out = [torch.empty((grid.nz, grid.nx), dtype=torch.float32, device=dev) for _ in frames]
    stream = torch.cuda.current_stream()
    pixch = grid.nx * grid.nz * n_el

    if args.calibrate_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(events=None):
        for k in orders:
            if events is not None:
                events[k][0].record(stream)
            for b in range(args.batch):
                plan.beamform(rf_dev[b], k, out[b], stream=stream)
            if events is not None:
                events[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for k in orders} for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    per_order_ms = {k: sum(e[k][0].elapsed_time(e[k][1]) for e in ev) / (args.steps * args.batch)
                    for k in orders}
    per_order = {str(k): round(pixch / (per_order_ms[k] * 1e-3) / 1e9, 2) for k in orders}
    total_pixch = pixch * args.batch * len(orders) * args.steps
    value = total_pixch / elapsed / 1e9
    dom = max(orders, key=lambda k: per_order_ms[k])
    achieved = SLOTS[dom] * pixch / (per_order_ms[dom] * 1e-3) / 1e12

    # relative L2 of the last images against the oracle is checked by the tests;
    # here only the CPU oracle's throughput on the same batch is measured.
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle
        t_cpu = time.perf_counter()
        n_pix = 0
        for b, f in enumerate(frames):
            for k in orders:
                oracle.beamform(rf_host[b], geom, grid, k)
                n_pix += pixch
            if time.perf_counter() - t_cpu > 30.0:
                break
        dt = time.perf_counter() - t_cpu
        cpu = {"value": round(n_pix / dt / 1e9, 4), "unit": "Gpixel*ch/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": "%d frame(s) x orders %s of the same batch, FP64, %.1f s" %
                         (n_pix // (pixch * len(orders)), ",".join(map(str, orders)), dt)}

    res = {
        "metric": "beamformed Gpixel*ch/s (sum over orders k=%s)" % ",".join(map(str, orders)),
        "value": round(value, 2),
        "unit": "Gpixel*ch/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain HO-DMAS, 128-element array, 2048 samples/channel, 512x512 grid, "
                               "FP32 RF, orders 1-6, %d resident frames per step" % args.batch,
                   "n_elements": n_el, "n_samples": S, "grid": [grid.nx, grid.nz],
                   "batch_frames": args.batch, "orders": orders,
                   "tiling": [info.tiling.tile_x, info.tiling.tile_z, info.tiling.split, info.tiling.chunk]},
        "per_order_gpixch_s": per_order,
        "per_order_kernel_us": {str(k): round(per_order_ms[k] * 1e3, 2) for k in orders},
        "roofline": {"bound": "alu", "kernel": "hodmas_frame_kernel<%d, f32>" % dom,
                     "achieved": round(achieved, 2), "peak": VALU_PEAK_TSLOT, "unit": "Tslot/s",
                     "frac": round(achieved / VALU_PEAK_TSLOT, 4),
                     "slots_per_pixch": SLOTS[dom], "traffic": None},
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(res))
    plan.close()


if __name__ == "__main__":
    main()

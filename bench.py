#!/usr/bin/env python3
"""Throughput benchmark of the HO-DMAS beamformer on one MI355X.

Workload (default): 128-element array, 2048 samples per channel, 512 x 512
grid, float32 RF, orders k = 1..6.  A step beamforms a batch of B resident
frames (distinct seeds, already in HBM) at every order: one persistent batched
launch per order over the B frames (--per-frame-step: B x 6 per-frame
launches), with mirror pairs -- the array and the grid are symmetric about
x = 0, so one workgroup forms a tile and its mirror image from one set of
delays (--no-mirror: unpaired).  The unpaired forms are timed beside it.  The metric is beamformed
pixel-channel pairs per second (Gpixel*ch/s), summed over the orders, with
the per-order rates beside it.

Prints ONE JSON line.  Also reports:
  roofline      the dominant kernel (the order with the most device time) against
                the published FP32 vector peak, from HIP events on the launch
                stream, and every order against the ceiling set by this
                device's measured unpacked-FP32 and transcendental issue rates;
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

# Algorithmic work per pixel-channel for order k, in FP32 issue slots: 12 for
# the delay, the sample index and fraction, the record test and the
# interpolation; 2k for the powers and the power-sum adds (k-2 products and k
# adds; one add at k = 1); 4 per transcendental (quarter rate), of which the
# delay takes one and the signed root one (k = 2) or two (k >= 3).  The
# roofline's `achieved` is ALGO_SLOTS[k] x pixel-channels / kernel time.
ALGO_SLOTS = {1: 18, 2: 24, 3: 30, 4: 32, 5: 34, 6: 36}
# 157.3 TFLOP/s FP32 vector (published) = 78.6e12 FMA lane-slots/s
# (256 CUs x 128 FP32 lanes/clock x 2.4 GHz).
VALU_PEAK_TSLOT = 78.64
# The same work as this library's kernels spell it out per pixel-channel (the
# delay as 4 FP32 ops + sqrt + reciprocal; interpolation 6; the signed root;
# k-2 products; k adds), transcendentals weighted 4: reported beside the
# roofline, not used for it.
METHOD_SLOTS = {1: 19, 2: 25, 3: 32, 4: 32, 5: 36, 6: 38}
# METHOD_SLOTS split into plain FP32 operations and transcendentals (METHOD_SLOTS
# = NONTRANS + 4 TRANS): the ceiling against the device's measured issue rates
# is 1 / (NONTRANS / R_fp32 + TRANS / R_trans) pixel-channels per second.
NONTRANS = {1: 11, 2: 13, 3: 16, 4: 16, 5: 20, 6: 22}
TRANS = {1: 2, 2: 3, 3: 4, 4: 4, 5: 4, 6: 4}
# The all-orders kernel computes the delay and interpolation once (18 slots),
# the roots of every order from shared transcendentals, and one add per
# distinct power sum (1, 3, 5, 8, 12, 15 sums for orders up to 1..6).
FUSED_SLOTS = {1: 19, 2: 26, 3: 38, 4: 47, 5: 59, 6: 68}


def frac_of_peak(k, pixch, seconds):
    """Fraction of the FP32 issue peak: ALGO_SLOTS[k] x pixel-channels / time."""
    return ALGO_SLOTS[k] * pixch / seconds / 1e12 / VALU_PEAK_TSLOT


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="plain", choices=["plain", "small", "reduced", "batch", "serve", "display"],
                    help="plain: 128 el / 512^2 / FP32 (default); small: 64 el / 128^2 / FP32 latency and "
                         "back-to-back throughput; reduced: 256 el / 1024^2 / int16+FP16; "
                         "batch: 256 mixed FP16 frames in one persistent launch vs 256 FP32 launches; "
                         "serve: Poisson arrivals, continuous batching vs plain FP32 per request; "
                         "display: band-pass + Hilbert envelope + log compression of beamformed images")
    ap.add_argument("--rates", default="500,1000,2000", help="serve: arrival rates (frames/s)")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds per rate")
    ap.add_argument("--budget-gb", type=float, default=32.0, help="serve: HBM admission budget")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8, help="frames per step")
    ap.add_argument("--orders", default="1,2,3,4,5,6")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-frame-step", action="store_true",
                    help="plain: time one launch per frame and order instead of one batched launch per order")
    ap.add_argument("--no-compare", action="store_true", help="plain: skip timing the other launch forms")
    ap.add_argument("--no-mirror", action="store_true",
                    help="plain and batch: no mirror pairs (plain: also skip the per-frame paired comparison)")
    ap.add_argument("--no-peaks", action="store_true",
                    help="plain: skip measuring the device's issue and copy rates (the measured ceilings)")
    ap.add_argument("--no-tune", action="store_true", help="batch: default tilings instead of the autotuner's")
    ap.add_argument("--tune-cache", default=os.path.join("/tmp", "hodmas_tune_cache.jsonl"),
                    help="batch and plain mirror pairs: autotuner cache file (JSON lines)")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain: skip the short mixed-batch and serving runs embedded in its line")
    ap.add_argument("--extra-rates", default="500,2000,16000,24000",
                    help="plain: arrival rates of the embedded serving run (frames/s)")
    ap.add_argument("--extra-duration", type=float, default=3.0,
                    help="plain: seconds per rate of the embedded serving run")
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
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        _copy_256mib(torch)
    {"plain": bench_plain, "small": bench_small, "reduced": bench_reduced, "batch": bench_batch,
     "serve": bench_serve, "display": bench_display}[args.workload](args, torch)


def _profiled_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's readings), or
    None when no summary covers it or the kernel source changed since."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2203_14906_amd", "csrc", "hodmas_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        text = open(path).read()
        if "kernel_source_sha256: " + sha not in text:
            continue
        for line in text.splitlines():
            line = line.strip()
            if line.startswith("traffic_bytes_per_launch " + kernel + ":"):
                return int(line.rsplit(":", 1)[1])
    return None


def _issued_slots(kernel, pixch, seconds):
    """The slots the kernel actually issues per pixel-channel -- plain VALU
    instructions plus 4 per transcendental, from the committed rocprofv3
    counter summary of the current kernel source -- and the fraction of the
    peak they make at the measured time; None when no summary covers it.
    Mirror pairs issue fewer slots than the algorithmic count (one delay
    serves two pixels), so this fraction is the lower one for them."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2203_14906_amd", "csrc", "hodmas_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.md"))):
        text = open(path).read()
        if "kernel_source_sha256: " + sha not in text:
            continue
        for line in text.splitlines():
            line = line.strip()
            if line.startswith("issued_slots_per_pixch " + kernel + ":"):
                slots = float(line.rsplit(":", 1)[1])
                return {"slots_per_pixch": slots,
                        "frac": round(slots * pixch / seconds / 1e12 / VALU_PEAK_TSLOT, 4),
                        "source": os.path.basename(path)}
    return None


def _copy_256mib(torch):
    """A plain 256 MiB device-to-device copy, three times: the known byte
    count that HBM counter readings are scaled by."""
    src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _events(torch, n):
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]


def bench_plain(args, torch):
    from paper_2203_14906_amd import hodmas, phantom as ph
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

    # A step beamforms the B resident frames at every order.  By default each
    # order is one persistent batched launch over the B frames (their work
    # lists are built here, outside the timed region; workgroups drift out of
    # step, so one tile's staging overlaps another's arithmetic and the
    # frames' tails overlap); --per-frame-step runs B per-frame launches per
    # order instead.  The step's plan pairs mirror tiles when the geometry
    # allows it (HODMAS_FLAG_MIRROR: each delay serves a pixel and its mirror
    # image; the images are the unpaired kernel's up to rounding).  The other
    # forms are timed beside it for comparison.
    mplan = None
    if not args.no_mirror:
        try:
            mplan = hodmas.Plan(geom, grid, S, "f32", max_order=max(orders), flags=hodmas.FLAG_MIRROR)
        except hodmas.HodmasError:
            mplan = None
    splan = mplan if mplan is not None else plan
    sinfo = splan.info()
    can_batch = all(q.tiling.tile_x * q.tiling.tile_z * q.tiling.split == 256 for q in (info, sinfo))
    batched_step = can_batch and not args.per_frame_step

    def make_batches(q):
        qi = q.info()
        res = {}
        for k in orders:
            bt = hodmas.Batch(max_frames=args.batch, max_units=qi.n_tiles * args.batch, max_lds_bytes=qi.lds_bytes)
            bt.set([q] * args.batch, rf_dev, [k] * args.batch, out, stream=stream)
            res[k] = bt
        return res

    bts = make_batches(splan) if can_batch and (batched_step or not args.no_compare) else {}
    bts_u = (make_batches(plan) if mplan is not None and can_batch and not args.no_compare else bts)

    def run_batched(k):
        bts[k].launch(stream=stream)

    def run_batched_unpaired(k):
        bts_u[k].launch(stream=stream)

    def run_per_frame(k):
        for b in range(args.batch):
            splan.beamform(rf_dev[b], k, out[b], stream=stream)

    def run_per_frame_unpaired(k):
        for b in range(args.batch):
            plan.beamform(rf_dev[b], k, out[b], stream=stream)

    run_order = run_batched if batched_step else run_per_frame

    def step(events=None):
        for k in orders:
            if events is not None:
                events[k][0].record(stream)
            run_order(k)
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
    achieved = ALGO_SLOTS[dom] * pixch / (per_order_ms[dom] * 1e-3) / 1e12
    dom_kernel = "%s<%d, f32, comp%s>" % ("hodmas_batch_kernel" if batched_step else "hodmas_frame_kernel", dom,
                                          ", mirror pairs" if mplan is not None else "")

    def time_form(run):
        """Per-frame milliseconds of each order when its B frames run through `run`."""
        ms = {}
        for k in orders:
            for _ in range(max(1, args.warmup)):
                run(k)
            fev = _events(torch, args.steps)
            torch.cuda.synchronize()
            for s_ in range(args.steps):
                fev[s_][0].record(stream)
                run(k)
                fev[s_][1].record(stream)
            torch.cuda.synchronize()
            ms[k] = sum(a.elapsed_time(z) for a, z in fev) / (args.steps * args.batch)
        return ms

    # the other launch forms of the same step
    others = {}
    pf_ms = per_order_ms if not batched_step and mplan is None else None
    if not args.no_compare:
        cand = []
        if batched_step and mplan is not None:
            cand.append(("batched_unpaired", "one batched launch per order, unpaired", run_batched_unpaired))
        if not batched_step and can_batch:
            cand.append(("batched", "one batched launch per order" + (", mirror pairs" if mplan else ""),
                         run_batched))
        if batched_step or mplan is not None:
            cand.append(("per_frame_unpaired", "per-frame launches, unpaired", run_per_frame_unpaired))
        for key, desc, run in cand:
            alt_ms = time_form(run)
            if key == "per_frame_unpaired":
                pf_ms = alt_ms
            others[key] = {"form": desc,
                           "kernel_us_per_frame": {str(k): round(v * 1e3, 3) for k, v in alt_ms.items()},
                           "frac_of_peak": {str(k): round(frac_of_peak(k, pixch, v * 1e-3), 4)
                                            for k, v in alt_ms.items()},
                           "gpixch_s_sum_orders": round(pixch * len(orders) / (sum(alt_ms.values()) * 1e-3) / 1e9,
                                                        2),
                           "headline_speedup": round(sum(alt_ms.values()) / sum(per_order_ms.values()), 3)}
    for bt in set(bts.values()) | set(bts_u.values()):
        bt.close()

    # every order 1..kmax from one launch per frame
    fused = None
    kmax = max(orders)
    if sorted(orders) == list(range(1, kmax + 1)):
        outs_all = [[torch.empty((grid.nz, grid.nx), dtype=torch.float32, device=dev) for _ in orders]
                    for _ in frames]
        for _ in range(args.warmup):
            for b in range(args.batch):
                plan.beamform_orders(rf_dev[b], kmax, outs_all[b], stream=stream)
        fev = _events(torch, args.steps)
        torch.cuda.synchronize()
        for s in range(args.steps):
            fev[s][0].record(stream)
            for b in range(args.batch):
                plan.beamform_orders(rf_dev[b], kmax, outs_all[b], stream=stream)
            fev[s][1].record(stream)
        torch.cuda.synchronize()
        f_ms = sum(a.elapsed_time(z) for a, z in fev) / (args.steps * args.batch)
        f_ach = FUSED_SLOTS[kmax] * pixch / (f_ms * 1e-3) / 1e12
        fused = {"kernel": "hodmas_orders_kernel<%d, f32, comp>" % kmax, "kernel_us_per_frame": round(f_ms * 1e3, 2),
                 "gpixch_s_sum_orders": round(pixch * len(orders) / (f_ms * 1e-3) / 1e9, 2),
                 "speedup_vs_per_order_launches": (round(sum(pf_ms.values()) / f_ms, 3) if pf_ms else None),
                 "slots_per_pixch": FUSED_SLOTS[kmax], "achieved_tslot_s": round(f_ach, 2),
                 "frac": round(f_ach / VALU_PEAK_TSLOT, 4),
                 "traffic": _profiled_traffic("hodmas_orders_kernel<%d, f32, comp>" % kmax)}

    # mirror pairs as per-frame launches, tiling per order from the autotuner
    mirrored = None
    if mplan is not None:
        m_us, m_tiling = {}, {}
        for k in orders:
            t = hodmas.autotune(geom, grid, S, "f32", k, flags=hodmas.FLAG_MIRROR, cache_path=args.tune_cache)
            mp = hodmas.Plan(geom, grid, S, "f32", max_order=k, tiling=t, flags=hodmas.FLAG_MIRROR)
            for _ in range(max(1, args.warmup)):
                for b in range(args.batch):
                    mp.beamform(rf_dev[b], k, out[b], stream=stream)
            mev = _events(torch, args.steps)
            torch.cuda.synchronize()
            for s_ in range(args.steps):
                mev[s_][0].record(stream)
                for b in range(args.batch):
                    mp.beamform(rf_dev[b], k, out[b], stream=stream)
                mev[s_][1].record(stream)
            torch.cuda.synchronize()
            m_us[k] = sum(a.elapsed_time(z) for a, z in mev) / (args.steps * args.batch) * 1e3
            mt = mp.info().tiling
            m_tiling[str(k)] = [mt.tile_x, mt.tile_z, mt.split, mt.chunk]
            mp.close()
        mirrored = {"form": "per-frame launches, mirror pairs, autotuned tiling per order",
                    "kernel": "hodmas_frame_kernel<k, f32, comp, mirror pairs>",
                    "kernel_us_per_frame": {str(k): round(v, 2) for k, v in m_us.items()},
                    "tilings": m_tiling,
                    "speedup_vs_unpaired_per_frame": ({str(k): round(pf_ms[k] * 1e3 / m_us[k], 3) for k in orders}
                                                      if pf_ms else None)}

    # ceilings from the measured issue rates of this device (unpacked FP32 add,
    # the mean of the four transcendentals) and its HBM copy rate
    measured = None
    if not args.no_peaks:
        pk = hodmas.measure_peaks(stream=stream)
        r_v = pk["fp32_add"]
        r_t = (pk["exp2"] + pk["log2"] + pk["sqrt"] + pk["rcp"]) / 4.0
        ceil = {k: 1e3 / (NONTRANS[k] / r_v + TRANS[k] / r_t) for k in orders}   # Gpixel*ch/s
        got = {k: pixch / (per_order_ms[k] * 1e-3) / 1e9 for k in orders}
        measured = {"fp32_add_tlane_s": round(r_v, 2), "fp32_fma_tlane_s": round(pk["fp32_fma"], 2),
                    "fp32_fma_sgpr_tlane_s": round(pk["fp32_fma_sgpr"], 2),
                    "trans_tlane_s": {n: round(pk[n], 2) for n in ("exp2", "log2", "sqrt", "rcp")},
                    "bitwise_bfi_tlane_s": round(pk["int_bfi"], 2), "fract_tlane_s": round(pk["fract"], 2),
                    "inner_loop_cycles_per_wave_element": {"constants_in_sgprs": round(pk["loop_cycles_sgpr"], 1),
                                                           "constants_in_vgprs": round(pk["loop_cycles_vgpr"], 1)},
                    "hbm_copy_tb_s": round(pk["hbm_copy_tb_s"], 3),
                    "ceiling_gpixch_s": {str(k): round(v, 1) for k, v in ceil.items()},
                    "frac_of_ceiling": {str(k): round(got[k] / ceil[k], 4) for k in orders},
                    "frac_dominant": round(got[dom] / ceil[dom], 4)}

    # relative L2 of the last images against the oracle is checked by the tests;
    # here only the CPU oracle's throughput on the same batch is measured.
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(rf_host, geom, grid, orders, pixch)
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
                               "FP32 RF, orders 1-6, %d resident frames per step, %s%s" % (
                                   args.batch, "each order one persistent batched launch over the frames"
                                   if batched_step else "one launch per frame and order",
                                   ", mirror pairs" if mplan is not None else ""),
                   "n_elements": n_el, "n_samples": S, "grid": [grid.nx, grid.nz],
                   "batch_frames": args.batch, "orders": orders, "mirror_pairs": mplan is not None,
                   "tiling": [sinfo.tiling.tile_x, sinfo.tiling.tile_z, sinfo.tiling.split, sinfo.tiling.chunk]},
        "per_order_gpixch_s": per_order,
        "per_order_kernel_us": {str(k): round(per_order_ms[k] * 1e3, 2) for k in orders},
        "fused_all_orders": fused,
        "other_forms": others,
        "mirror_paired_per_frame": mirrored,
        "roofline": {"bound": "alu", "kernel": dom_kernel,
                     "achieved": round(achieved, 2), "peak": VALU_PEAK_TSLOT, "unit": "Tslot/s",
                     "frac": round(achieved / VALU_PEAK_TSLOT, 4),
                     "slots_per_pixch": ALGO_SLOTS[dom],
                     "slots_model": "algorithmic FP32 issue slots per pixel-channel: 12 + 2k + 4 per "
                                    "transcendental (18/24/30/32/34/36 for k=1..6)",
                     "frac_method_slots": round(METHOD_SLOTS[dom] * pixch / (per_order_ms[dom] * 1e-3) / 1e12
                                                / VALU_PEAK_TSLOT, 4),
                     "issued": _issued_slots(dom_kernel, pixch, per_order_ms[dom] * 1e-3),
                     "traffic": _profiled_traffic(dom_kernel),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "measured": measured},
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_extras:
        # the metric's second half: frames/s and latency, batched vs plain, on
        # the mixed 256-frame batch and under Poisson arrivals (short runs)
        res["config4_batched_vs_plain"] = batch_workload(args, torch)
        res["config5_serving"] = serve_workload(args, torch, [float(r) for r in args.extra_rates.split(",")],
                                                args.extra_duration)
    print(json.dumps(res))
    plan.close()
    if mplan is not None:
        mplan.close()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _cpu_baseline(rf_host, geom, grid, orders, pixch):
    """The FP64 oracle on this host's cores: whole frames of the batch at every
    order, cycling, for at least 8 s on all threads (never past ~25 s), then
    one frame's orders on one thread (at least 3 s)."""
    from oracle import oracle

    def timed(min_s, max_s):
        t0 = time.perf_counter()
        n_pix = n_frames = 0
        while True:
            b = n_frames % len(rf_host)
            for k in orders:
                oracle.beamform(rf_host[b], geom, grid, k)
                n_pix += pixch
            n_frames += 1
            el = time.perf_counter() - t0
            if el >= min_s or el * (n_frames + 1) / n_frames > max_s:
                return n_pix, n_frames, time.perf_counter() - t0

    threads = oracle.max_threads()
    n_pix, n_frames, dt = timed(8.0, 25.0)
    oracle.set_threads(1)
    try:
        n1, f1, dt1 = timed(3.0, 12.0)
    finally:
        oracle.set_threads(threads)
    return {"value": round(n_pix / dt / 1e9, 4), "unit": "Gpixel*ch/s", "cores": threads, "kind": "oracle",
            "sample": "%d frame(s) (cycling over the %d of the batch) x orders %s, FP64, %.1f s"
                      % (n_frames, len(rf_host), ",".join(map(str, orders)), dt),
            "one_thread": {"value": round(n1 / dt1 / 1e9, 4), "cores": 1,
                           "sample": "%d frame(s) x orders %s, %.1f s" % (f1, ",".join(map(str, orders)), dt1)},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def bench_small(args, torch):
    """Config 1: 64 elements, 1024 samples, 128x128 grid, FP32 RF, orders 1..4.
    A frame is about a microsecond of GPU work, so one launch is bound by launch
    overhead: report single-launch latency (host wall clock of launch plus
    synchronize, and the kernel's own time from HIP events) and throughput over
    1024 back-to-back frames, as per-frame launches and as one persistent batch
    launch (unpaired and with mirror pairs; the batch plans take the tiling the
    autotuner picks for batches, and the graph replay is timed beside the
    direct launch)."""
    from paper_2203_14906_amd import hodmas, phantom as ph
    dev = torch.device("cuda:0")
    p = ph.CONFIGS[1]
    orders = list(p["orders"])
    n_res, n_frames = 16, 1024                    # resident records, frames per throughput run
    frames = [ph.config_frame(1, b) for b in range(n_res)]
    geom, grid = frames[0].geometry, frames[0].grid
    S = p["n_samples"]
    pixch = grid.nx * grid.nz * p["n_elements"]
    plan = hodmas.Plan(geom, grid, S, "f32", max_order=max(orders))
    info = plan.info()
    rf = [torch.from_numpy(ph.to_fp32(fr.rf)).to(dev) for fr in frames]
    outs = [torch.empty((grid.nz, grid.nx), dtype=torch.float32, device=dev) for _ in range(n_frames)]
    stream = torch.cuda.current_stream()
    res = {"metric": "config-1 single-launch latency and back-to-back throughput", "unit": "us / Gpixel*ch/s",
           "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "64 elements, 1024 samples/channel, 128x128 grid, FP32 RF, orders 1-4",
                      "tiling": [info.tiling.tile_x, info.tiling.tile_z, info.tiling.split, info.tiling.chunk],
                      "n_tiles": info.n_tiles, "frames_back_to_back": n_frames},
           "per_order": {}}
    batch_rf = [rf[i % n_res] for i in range(n_frames)]

    def time_batch(q, k):
        """(direct launch ms, graph replay ms) for the n_frames frames under plan q."""
        qi = q.info()
        b = hodmas.Batch(max_frames=n_frames, max_units=qi.n_tiles * n_frames, max_lds_bytes=qi.lds_bytes)
        b.set([q] * n_frames, batch_rf, [k] * n_frames, outs)
        out = []
        for replay in (False, True):
            if replay:
                b.capture()
            run = (lambda: b.replay(stream=stream)) if replay else (lambda: b.launch(stream=stream))
            for _ in range(2):
                run()
            torch.cuda.synchronize()
            bev = _events(torch, max(3, args.steps))
            for e in bev:
                e[0].record(stream)
                run()
                e[1].record(stream)
            torch.cuda.synchronize()
            out.append(sorted(a.elapsed_time(z) for a, z in bev)[len(bev) // 2])
        b.close()
        return out

    for k in orders:
        for _ in range(max(3, args.warmup)):
            plan.beamform(rf[0], k, outs[0], stream=stream)
        torch.cuda.synchronize()
        wall = []
        for r in range(200):
            t0 = time.perf_counter()
            plan.beamform(rf[r % n_res], k, outs[0], stream=stream)
            torch.cuda.synchronize()
            wall.append((time.perf_counter() - t0) * 1e6)
        ev = _events(torch, 200)
        for r in range(200):
            ev[r][0].record(stream)
            plan.beamform(rf[r % n_res], k, outs[0], stream=stream)
            ev[r][1].record(stream)
        torch.cuda.synchronize()
        kern = sorted(a.elapsed_time(z) * 1e3 for a, z in ev)
        # back-to-back: n_frames launches, one event pair around them
        e0, e1 = _events(torch, 1)[0]
        e0.record(stream)
        for i in range(n_frames):
            plan.beamform(rf[i % n_res], k, outs[i], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        b2b_ms = e0.elapsed_time(e1)
        wall.sort()
        row = {"latency_wall_us_p50": round(wall[len(wall) // 2], 2),
               "latency_wall_us_p99": round(wall[int(0.99 * (len(wall) - 1))], 2),
               "kernel_us_p50": round(kern[len(kern) // 2], 2),
               "back_to_back_us_per_frame": round(b2b_ms * 1e3 / n_frames, 3),
               "back_to_back_gpixch_s": round(pixch * n_frames / (b2b_ms * 1e-3) / 1e9, 2)}
        # the same frames as one persistent launch, with the tiling the
        # autotuner picks for batches (timed as a batch runs them), and with
        # the plan's default tiling (made for a single frame) for comparison
        for name, flags in (("batched", 0), ("batched_mirror_pairs", hodmas.FLAG_MIRROR),
                            ("batched_default_tiling", 0)):
            if flags and args.no_mirror:
                continue
            if name == "batched_default_tiling":
                t = None
            else:
                t = hodmas.autotune(geom, grid, S, "f32", k, flags=hodmas.FLAG_TUNE_BATCH | flags,
                                    cache_path=args.tune_cache)
            q = hodmas.Plan(geom, grid, S, "f32", max_order=k, tiling=t, flags=flags)
            direct_ms, replay_ms = time_batch(q, k)
            qt = q.info().tiling
            row[name + "_us_per_frame"] = round(direct_ms * 1e3 / n_frames, 3)
            row[name + "_gpixch_s"] = round(pixch * n_frames / (direct_ms * 1e-3) / 1e9, 2)
            row[name + "_frac_of_peak"] = round(frac_of_peak(k, pixch * n_frames, direct_ms * 1e-3), 4)
            row[name + "_graph_replay_us_per_frame"] = round(replay_ms * 1e3 / n_frames, 3)
            row[name + "_tiling"] = [qt.tile_x, qt.tile_z, qt.split, qt.chunk]
            q.close()
        res["per_order"][str(k)] = row
    plan.close()
    print(json.dumps(res))


def bench_reduced(args, torch):
    """256 elements, 1024^2, int16 and FP16 storage, k = 1..6: throughput per
    order and relative L2 per order against the FP64 oracle on the same stored
    values (gated in the tests) and on the float64 RF before quantisation."""
    import numpy as np
    from oracle import oracle
    from paper_2203_14906_amd import hodmas, phantom as ph
    f = ph.config_frame(3)
    geom, grid = f.geometry, f.grid
    pixch = grid.nx * grid.nz * f.rf.shape[0]
    rng = np.random.default_rng(1)
    ix = rng.integers(0, grid.nx, 4096).astype(np.int32)
    iz = rng.integers(0, grid.nz, 4096).astype(np.int32)
    res = {"metric": "beamformed Gpixel*ch/s per order, reduced-precision storage", "unit": "Gpixel*ch/s",
           "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "256 elements, 2048 samples/channel, 1024x1024 grid, int16 and FP16 RF"},
           "forms": {}}
    for dt in ("i16", "f16"):
        if dt == "i16":
            arr, scale = ph.to_int16(f.rf, 3000)
            scale = float(scale)
        else:
            arr, scale = ph.to_fp16(f.rf), 1.0
        rf_dev = torch.from_numpy(arr).cuda()
        out = torch.empty((grid.nz, grid.nx), dtype=torch.float32, device="cuda")
        # one launch per frame and order, unpaired and -- the array and grid
        # being symmetric about x = 0 -- with mirror pairs
        variants = [("", 0)] + ([] if args.no_mirror else [("_mirror_pairs", hodmas.FLAG_MIRROR)])
        for suffix, flags in variants:
            plan = hodmas.Plan(geom, grid, arr.shape[1], dt, max_order=6, dequant_scale=scale, flags=flags)
            form = {}
            for k in range(1, 7):
                for _ in range(args.warmup):
                    plan.beamform(rf_dev, k, out)
                ev = _events(torch, 1)[0]
                ev[0].record()
                for _ in range(args.steps):
                    plan.beamform(rf_dev, k, out)
                ev[1].record()
                torch.cuda.synchronize()
                us = ev[0].elapsed_time(ev[1]) / args.steps * 1e3
                g = out.cpu().numpy().astype(np.float64)[iz, ix]
                same = oracle.beamform(arr, geom, grid, k, dequant_scale=scale if dt == "i16" else None,
                                       pixels=(ix, iz))
                pre = oracle.beamform(f.rf, geom, grid, k, pixels=(ix, iz))
                form[str(k)] = {"kernel_us": round(us, 2), "gpixch_s": round(pixch / (us * 1e-6) / 1e9, 2),
                                "rel_l2_same_values": float("%.3e" % (np.linalg.norm(g - same) /
                                                                      np.linalg.norm(same))),
                                "rel_l2_vs_fp64_rf": float("%.3e" % (np.linalg.norm(g - pre) / np.linalg.norm(pre)))}
            res["forms"][dt + suffix] = form
            plan.close()
    res["sample"] = "relative L2 over 4096 seeded pixels"
    print(json.dumps(res))


def _mixed_frames(torch, specs, with_fp32, tune_cache=None, mirror=False):
    """Device-resident frames of the mixed workload; the RF of each (N, S)
    shape comes from one seeded phantom shared by the frames of that shape.
    With ``tune_cache`` the FP16 plans take the autotuner's tiling (tuned at
    order 6 among the tilings a batch accepts, cached in that file).  With
    ``mirror`` the FP16 plans pair mirror tiles (the arrays are centred and the
    grids symmetric about x = 0); the FP32 plans stay unpaired."""
    from paper_2203_14906_amd import hodmas, phantom as ph
    rf_cache, plans, frames = {}, {}, []
    for sp in specs:
        n, S, side = sp["n_elements"], sp["n_samples"], sp["side"]
        if (n, S) not in rf_cache:
            fr = ph.make_frame(n, S, 8, 8, n_points=50, n_lines=3, snr_db=10.0, seed=4000 + n + S)
            rf_cache[(n, S)] = (torch.from_numpy(ph.to_fp16(fr.rf)).cuda(),
                                torch.from_numpy(ph.to_fp32(fr.rf)).cuda() if with_fp32 else None)
        if (n, S, side) not in plans:
            w, d = ph.field_of_view(n, S)
            grid = ph.make_grid(side, side, w, d)
            geom = ph.Geometry(n)
            tiling = None
            pflags = hodmas.FLAG_MIRROR if mirror else 0
            if tune_cache is not None:
                tiling = hodmas.autotune(geom, grid, S, "f16", 6, flags=hodmas.FLAG_TUNE_BATCH | pflags,
                                         cache_path=tune_cache)
            plans[(n, S, side)] = (hodmas.Plan(geom, grid, S, "f16", max_order=6, tiling=tiling, flags=pflags),
                                   hodmas.Plan(geom, grid, S, "f32", max_order=6) if with_fp32 else None)
        frames.append(dict(spec=sp, rf16=rf_cache[(n, S)][0], rf32=rf_cache[(n, S)][1],
                           plan16=plans[(n, S, side)][0], plan32=plans[(n, S, side)][1],
                           pixch=side * side * n))
    return frames, plans


def bench_batch(args, torch):
    print(json.dumps(batch_workload(args, torch)))


def batch_workload(args, torch):
    """256 mixed frames (N, S, grid side, order drawn per frame; FP16 RF) in one
    persistent launch replayed from a HIP graph, with mirror pairs (--no-mirror:
    unpaired), against 256 plain per-frame FP32 launches on one stream.  All frames are submitted at t = 0; latency is
    each frame's completion time."""
    import numpy as np
    from paper_2203_14906_amd import hodmas, phantom as ph
    specs = ph.mixed_batch_specs(256, seed=4000)
    t_tune = time.perf_counter()
    frames, plans = _mixed_frames(torch, specs, with_fp32=True,
                                  tune_cache=None if args.no_tune else args.tune_cache, mirror=not args.no_mirror)
    t_tune = time.perf_counter() - t_tune
    outs_b = [torch.empty((f["spec"]["side"],) * 2, dtype=torch.float32, device="cuda") for f in frames]
    outs_p = [torch.empty_like(o) for o in outs_b]
    orders = [f["spec"]["order"] for f in frames]
    lds = max(p[0].info().lds_bytes for p in plans.values())
    batch = hodmas.Batch(max_frames=256, max_units=1 << 22, max_lds_bytes=lds)
    batch.set([f["plan16"] for f in frames], [f["rf16"] for f in frames], orders, outs_b)
    batch.capture()
    for _ in range(args.warmup):
        batch.replay()
        for f, o, k in zip(frames, outs_p, orders):
            f["plan32"].beamform(f["rf32"], k, o)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    tb = []
    for _ in range(reps):
        ev = _events(torch, 1)[0]
        ev[0].record()
        batch.replay()
        ev[1].record()
        torch.cuda.synchronize()
        tb.append(ev[0].elapsed_time(ev[1]))
    tp, lat_p = [], []
    for _ in range(reps):
        start = torch.cuda.Event(enable_timing=True)
        ends = [torch.cuda.Event(enable_timing=True) for _ in frames]
        start.record()
        for f, o, k, e in zip(frames, outs_p, orders, ends):
            f["plan32"].beamform(f["rf32"], k, o)
            e.record()
        torch.cuda.synchronize()
        tp.append(start.elapsed_time(ends[-1]))
        lat_p.append([start.elapsed_time(e) for e in ends])
    tb_ms, tp_ms = float(np.median(tb)), float(np.median(tp))
    lat_p = np.array(lat_p[int(np.argsort(tp)[len(tp) // 2])])
    pixch = sum(f["pixch"] for f in frames)
    worst = 0.0
    for f, ob, op in zip(frames[:16], outs_b[:16], outs_p[:16]):
        a, b = ob.double(), op.double()
        worst = max(worst, float(torch.linalg.norm(a - b) / torch.linalg.norm(b).clamp_min(1e-300)))
    inf = batch.info()
    res = {"metric": "frames/s and p99 latency, batched (one persistent launch) vs plain per-frame FP32",
           "unit": "frames/s", "n_gpus": 1, "data": "synthetic", "dtype": "f16 storage / f32 compute",
           "config": {"workload": "256 mixed frames: N in {64,128,256}, S in {1024,2048,4096}, "
                                  "grid side in {256,512,768,1024}, order 1..6, seed 4000",
                      "units": inf.n_units, "grid": inf.grid, "lds_bytes": inf.lds_bytes,
                      "tilings": "autotuned" if not args.no_tune else "default",
                      "mirror_pairs": not args.no_mirror,
                      "setup_s_incl_tuning": round(t_tune, 1)},
           "batched": {"frames_per_s": round(256 / (tb_ms * 1e-3), 1), "batch_ms": round(tb_ms, 3),
                       "p50_ms": round(tb_ms, 3), "p99_ms": round(tb_ms, 3),
                       "gpixch_s": round(pixch / (tb_ms * 1e-3) / 1e9, 1)},
           "plain_fp32": {"frames_per_s": round(256 / (tp_ms * 1e-3), 1), "total_ms": round(tp_ms, 3),
                          "p50_ms": round(float(np.percentile(lat_p, 50)), 3),
                          "p99_ms": round(float(np.percentile(lat_p, 99)), 3),
                          "gpixch_s": round(pixch / (tp_ms * 1e-3) / 1e9, 1)},
           "speedup": round(tp_ms / tb_ms, 3),
           "rel_l2_batched_fp16_vs_plain_fp32_first16": float("%.3e" % worst),
           "pixel_channels": pixch}
    batch.close()
    for p16, p32 in plans.values():
        p16.close()
        p32.close()
    return res


def bench_serve(args, torch):
    print(json.dumps(serve_workload(args, torch, [float(r) for r in args.rates.split(",")], args.duration)))


def serve_workload(args, torch, rates, duration):
    """Poisson arrivals at each rate for `duration` s; continuous batching of
    FP16 frames (mirror pairs unless --no-mirror) vs a plain synchronous FP32
    launch per request."""
    from paper_2203_14906_amd import serve
    pool = serve.FramePool(torch, "cuda", seed=5000, mirror=not args.no_mirror)
    out = {"metric": "p50/p99 latency and sustained frames/s, continuous batching vs plain FP32",
           "unit": "frames/s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "Poisson arrivals, mixed N/S/grid/order frames from a pool of %d "
                                  "resident frames (%d resident plans)" % (len(pool.frames), len(pool._plans)),
                      "duration_s": duration, "budget_gb": args.budget_gb,
                      "fp16_mirror_pairs": not args.no_mirror},
           "rates": {}}
    warm = serve.poisson_requests(500.0, 0.5, len(pool.frames), seed=1)
    srv = serve.Server(torch, pool, slots=3, budget_bytes=int(args.budget_gb * (1 << 30)))
    srv.run(warm)
    serve.run_plain(torch, pool, warm[:50])
    for rate in rates:
        reqs = serve.poisson_requests(rate, duration, len(pool.frames), seed=int(rate))
        b = srv.run(reqs).summary()
        reqs = serve.poisson_requests(rate, duration, len(pool.frames), seed=int(rate))
        p = serve.run_plain(torch, pool, reqs).summary()
        out["rates"][str(int(rate))] = {"batched": b, "plain_fp32": p}
        print("rate %g: batched %s | plain %s" % (rate, b, p), file=sys.stderr, flush=True)
    srv.close()
    pool.close()
    return out




def bench_display(args, torch):
    """Display chain (band-pass 2-8 MHz, 63 taps, Hilbert envelope, 60 dB log
    compression) of B beamformed 512x512 images (128 elements, order 3): image
    throughput, the envelope kernel's HBM rate, and the FP64 oracle beside it."""
    import numpy as np
    from paper_2203_14906_amd import hodmas, phantom as ph
    p = ph.CONFIGS[2]
    frames = [ph.make_frame(p["n_elements"], p["n_samples"], p["nx"], p["nz"], n_points=p["n_points"],
                            n_lines=p["n_lines"], snr_db=p["snr_db"], seed=2000 + b) for b in range(args.batch)]
    grid = frames[0].grid
    plan = hodmas.Plan(frames[0].geometry, grid, p["n_samples"], "f32", max_order=3)
    images = [plan.beamform(torch.from_numpy(ph.to_fp32(f.rf)).cuda(), 3) for f in frames]
    disp = hodmas.Display(grid.nx, grid.nz, grid.dz_m, 1540.0, 2e6, 8e6, 63, 60.0)
    envs = [torch.empty_like(im) for im in images]
    dbs = [torch.empty_like(im) for im in images]
    stream = torch.cuda.current_stream()

    def step():
        for im, e, d in zip(images, envs, dbs):
            disp.run(im, e, d, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = _events(torch, args.steps)
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        step()
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = sum(a.elapsed_time(b) for a, b in ev) / (args.steps * args.batch)
    npx = grid.nx * grid.nz
    # algorithmic bytes per image: read the image, write envelope and dB image
    algo_bytes = 3 * 4 * npx
    # the same images through hodmas_display_run_batch (up to 16 per launch pair)
    for _ in range(args.warmup):
        disp.run_batch(images, envs, dbs, stream=stream)
    torch.cuda.synchronize()
    evb = _events(torch, args.steps)
    for s in range(args.steps):
        evb[s][0].record(stream)
        disp.run_batch(images, envs, dbs, stream=stream)
        evb[s][1].record(stream)
    torch.cuda.synchronize()
    ms_b = sum(a.elapsed_time(b) for a, b in evb) / (args.steps * args.batch)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import display as D
        t_cpu, n = time.perf_counter(), 0
        for im in images:
            D.display(im.cpu().numpy().astype(np.float64), grid.dz_m, 1540.0, 2e6, 8e6, 63, 60.0)
            n += 1
            if time.perf_counter() - t_cpu > 20.0:
                break
        dt = time.perf_counter() - t_cpu
        cpu = {"value": round(n * npx / dt / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
               "sample": "%d image(s) of the same batch, numpy FP64, %.1f s" % (n, dt)}
    res = {"metric": "display chain Mpixel/s (band-pass, Hilbert envelope, log compression)",
           "value": round(npx / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
           "data": "synthetic", "dtype": "f32",
           "config": {"workload": "display chain of %d beamformed 512x512 images (128 elements, order 3), "
                                  "2-8 MHz band-pass with 63 taps, 60 dB" % args.batch},
           "us_per_image": round(ms * 1e3, 2),
           "batched": {"form": "hodmas_display_run_batch, %d images per call (16 per launch pair)" % args.batch,
                       "us_per_image": round(ms_b * 1e3, 2),
                       "mpixel_s": round(npx / (ms_b * 1e-3) / 1e6, 1),
                       "hbm_gb_s": round(algo_bytes / (ms_b * 1e-3) / 1e9, 1),
                       "hbm_frac": round(algo_bytes / (ms_b * 1e-3) / 1e9 / 8000.0, 4)},
           "roofline": {"bound": "hbm", "achieved": round(algo_bytes / (ms * 1e-3) / 1e9, 1), "peak": 8000.0,
                        "unit": "GB/s", "frac": round(algo_bytes / (ms * 1e-3) / 1e9 / 8000.0, 4),
                        "traffic": None},
           "cpu_baseline": cpu}
    print(json.dumps(res))
    disp.close()
    plan.close()


if __name__ == "__main__":
    main()

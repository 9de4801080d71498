"""Continuous-batching frame server on one GPU.

Requests (a frame to beamform at some order) arrive over time.  Array geometry
and the plans' delay tables stay resident on the device.  A request is admitted
while the in-flight footprint (its RF and image bytes) fits an HBM budget; the
admitted requests that are waiting when a launch slot frees up go out together
on that slot's stream -- as one batched submission, or as the frame's own
kernel when only one is waiting -- while earlier slots may still be running,
so work from different arrivals overlaps on the GPU.
Completion is observed through HIP events; latency = completion - arrival.

The plain comparison runs one synchronous float32 hodmas_beamform per request
in arrival order on one stream.

Only scheduling lives here: every image value comes from the HIP library.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import hodmas, phantom as ph


@dataclass
class Request:
    rid: int
    arrival: float            # seconds from the start of the run
    frame: int                # index into the frame pool
    order: int
    done: float = -1.0        # completion time, seconds from the start
    image: object = None      # device tensor
    nbytes: int = 0
    waited: bool = False      # held back at least once by the HBM budget


@dataclass
class PoolFrame:
    n_elements: int
    n_samples: int
    side: int
    rf16: object               # device float16 [N][S]
    rf32: object               # device float32 [N][S]
    plan16: object = None
    plan32: object = None


@dataclass
class ServeStats:
    mode: str
    n_requests: int
    wall_s: float
    latencies_ms: np.ndarray = field(default_factory=lambda: np.zeros(0))
    launches: int = 0
    max_inflight: int = 0
    admission_waits: int = 0     # requests held back at least once by the budget

    def summary(self) -> dict:
        lat = self.latencies_ms
        return {"mode": self.mode, "requests": self.n_requests,
                "frames_per_s": round(self.n_requests / self.wall_s, 2) if self.wall_s > 0 else None,
                "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
                "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
                "mean_ms": round(float(lat.mean()), 3) if lat.size else None,
                "launches": self.launches, "max_inflight_requests": self.max_inflight,
                "admission_waits": self.admission_waits}


class FramePool:
    """Pre-generated, device-resident frames and their resident plans.

    Shapes follow the mixed workload: N in {64,128,256}, S in {1024,2048,4096},
    square grids of side {256,512,768,1024}; ``per_shape`` distinct phantoms
    per (N, S) are shared by the grid sides."""

    def __init__(self, torch, device, n_elements=(64, 128, 256), n_samples=(1024, 2048, 4096),
                 sides=(256, 512, 768, 1024), per_shape=1, seed=5000, plain=True):
        self.torch = torch
        self.frames: list[PoolFrame] = []
        self._plans = {}
        k = 0
        for n in n_elements:
            for S in n_samples:
                for rep in range(per_shape):
                    f = ph.make_frame(n, S, 8, 8, n_points=50, n_lines=3, snr_db=10.0,
                                      seed=seed + k)
                    k += 1
                    rf16 = torch.from_numpy(ph.to_fp16(f.rf)).to(device)
                    rf32 = torch.from_numpy(ph.to_fp32(f.rf)).to(device) if plain else None
                    for side in sides:
                        self.frames.append(PoolFrame(n, S, side, rf16, rf32))
        for fr in self.frames:
            key = (fr.n_elements, fr.n_samples, fr.side)
            if key not in self._plans:
                w, d = ph.field_of_view(fr.n_elements, fr.n_samples)
                grid = ph.make_grid(fr.side, fr.side, w, d)
                geom = ph.Geometry(fr.n_elements)
                p16 = hodmas.Plan(geom, grid, fr.n_samples, "f16", max_order=6)
                p32 = hodmas.Plan(geom, grid, fr.n_samples, "f32", max_order=6) if plain else None
                self._plans[key] = (p16, p32)
            fr.plan16, fr.plan32 = self._plans[key]

    @property
    def max_lds_bytes(self):
        return max(p.info().lds_bytes for p, _ in self._plans.values())

    def close(self):
        for p16, p32 in self._plans.values():
            p16.close()
            if p32 is not None:
                p32.close()
        self._plans = {}


def poisson_requests(rate_hz, duration_s, n_frames, seed=0, orders=(1, 2, 3, 4, 5, 6)):
    """Seeded Poisson arrivals; each request draws a pool frame and an order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append(Request(rid=len(out), arrival=t, frame=int(rng.integers(n_frames)),
                           order=int(rng.choice(orders))))
    return out


class Server:
    """Slots x streams continuous batching with HBM-budget admission."""

    def __init__(self, torch, pool: FramePool, slots=3, budget_bytes=32 << 30, max_batch=64,
                 max_units=1 << 20):
        self.torch = torch
        self.pool = pool
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        lds = pool.max_lds_bytes
        self.slots = []
        for _ in range(slots):
            b = hodmas.Batch(max_frames=max_batch, max_units=max_units, max_lds_bytes=lds)
            self.slots.append({"batch": b, "stream": torch.cuda.Stream(), "event": None,
                               "reqs": []})

    def close(self):
        for s in self.slots:
            s["batch"].close()
        self.slots = []

    def _footprint(self, r: Request) -> int:
        fr = self.pool.frames[r.frame]
        return fr.side * fr.side * 4 + fr.n_elements * fr.n_samples * 2

    def run(self, requests: list[Request], keep_images=False) -> ServeStats:
        torch = self.torch
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        admitted: deque = deque()
        inflight_bytes = 0
        inflight_reqs = 0
        stats = ServeStats("batched", len(requests), 0.0)
        total = len(requests)
        finished = 0
        t0 = time.perf_counter()
        while finished < total:
            now = time.perf_counter() - t0
            # completions
            for s in self.slots:
                if s["event"] is not None and s["event"].query():
                    for r in s["reqs"]:
                        r.done = now
                        inflight_bytes -= r.nbytes
                        if not keep_images:
                            r.image = None
                    finished += len(s["reqs"])
                    inflight_reqs -= len(s["reqs"])
                    s["event"], s["reqs"] = None, []
            # arrivals -> admission by HBM budget (in arrival order)
            while pending and pending[0].arrival <= now:
                r = pending[0]
                nb = self._footprint(r)
                if inflight_bytes + nb > self.budget and (inflight_bytes > 0 or admitted):
                    if not r.waited:
                        r.waited = True
                        stats.admission_waits += 1
                    break
                pending.popleft()
                r.nbytes = nb
                inflight_bytes += nb
                fr = self.pool.frames[r.frame]
                r.image = torch.empty((fr.side, fr.side), dtype=torch.float32, device="cuda")
                admitted.append(r)
            # a free slot takes everything admitted so far
            if admitted:
                for s in self.slots:
                    if s["event"] is None:
                        take = [admitted.popleft() for _ in range(min(self.max_batch, len(admitted)))]
                        frs = [self.pool.frames[r.frame] for r in take]
                        if len(take) == 1:
                            # a lone request runs its frame's own kernel: no work list to build
                            frs[0].plan16.beamform(frs[0].rf16, take[0].order, take[0].image,
                                                   stream=s["stream"])
                        else:
                            b = s["batch"]
                            b.set([f.plan16 for f in frs], [f.rf16 for f in frs], [r.order for r in take],
                                  [r.image for r in take], stream=s["stream"])
                            b.launch(stream=s["stream"])
                        ev = torch.cuda.Event()
                        ev.record(s["stream"])
                        s["event"], s["reqs"] = ev, take
                        inflight_reqs += len(take)
                        stats.launches += 1
                        stats.max_inflight = max(stats.max_inflight, inflight_reqs)
                        break
            if finished < total:
                # idle: sleep until shortly before the next arrival; with work in
                # flight keep polling the completion events
                nxt = pending[0].arrival if pending else None
                busy = any(s["event"] is not None for s in self.slots)
                if not busy and not admitted and nxt is not None:
                    delay = nxt - (time.perf_counter() - t0)
                    if delay > 2e-4:
                        time.sleep(delay - 1e-4)
        stats.wall_s = max(r.done for r in requests) if requests else 0.0
        stats.latencies_ms = np.array([(r.done - r.arrival) * 1e3 for r in requests])
        return stats


def run_plain(torch, pool: FramePool, requests: list[Request], keep_images=False) -> ServeStats:
    """One synchronous float32 launch per request, in arrival order, one stream."""
    stats = ServeStats("plain_fp32", len(requests), 0.0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda x: x.arrival):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        fr = pool.frames[r.frame]
        r.image = torch.empty((fr.side, fr.side), dtype=torch.float32, device="cuda")
        fr.plan32.beamform(fr.rf32, r.order, r.image, stream=stream)
        stream.synchronize()
        r.done = time.perf_counter() - t0
        stats.launches += 1
        if not keep_images:
            r.image = None
    stats.wall_s = max(r.done for r in requests) if requests else 0.0
    stats.latencies_ms = np.array([(r.done - r.arrival) * 1e3 for r in requests])
    return stats

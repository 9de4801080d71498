"""Continuous-batching frame server on one GPU.

Requests (a frame to beamform at some order) arrive over time.  Array geometry
and the plans' delay tables stay resident on the device.  A request is admitted
while the in-flight footprint (its RF and image bytes) fits an HBM budget; the
admitted requests that are waiting when a launch slot frees up go out together
on that slot's stream -- as one batched submission, or as the frame's own
kernel when only one is waiting -- while earlier slots may still be running,
so work from different arrivals overlaps on the GPU.
Completion is observed through HIP events; latency = completion - arrival.
A failure stays with its request: unknown frames and orders outside 1..6 are
rejected on arrival, requests whose deadline passes before launch are
dropped, and a refused batched launch is retried one request at a time.

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
    deadline: float | None = None   # seconds after arrival by which it must have launched
    done: float = -1.0        # completion (or rejection / drop / failure) time, from the start
    status: str = "pending"   # done | rejected | dropped | failed
    image: object = None      # device tensor
    nbytes: int = 0
    waited: bool = False      # held back at least once by the HBM budget
    solo: bool = False        # to be launched alone (its batch failed to launch)


@dataclass
class ServeStats:
    mode: str
    n_requests: int
    wall_s: float
    latencies_ms: np.ndarray = field(default_factory=lambda: np.zeros(0))
    launches: int = 0
    max_inflight: int = 0
    admission_waits: int = 0     # requests held back at least once by the budget
    rejected: int = 0            # refused on arrival (unknown frame, order outside 1..6)
    dropped: int = 0             # deadline passed before launch
    failed: int = 0              # the library refused the launch of this request
    batch_sizes: list = field(default_factory=list)   # requests per launch, in launch order

    def launch_histogram(self) -> dict:
        """Launches by the number of requests they carried (1, 2-3, 4-7, ...)."""
        hist = {}
        for n in self.batch_sizes:
            lo = 1 << (int(n).bit_length() - 1)
            key = "1" if lo == 1 else "%d-%d" % (lo, 2 * lo - 1)
            hist[key] = hist.get(key, 0) + 1
        return dict(sorted(hist.items(), key=lambda kv: int(kv[0].split("-")[0])))

    def summary(self) -> dict:
        lat = self.latencies_ms
        served = self.n_requests - self.rejected - self.dropped - self.failed
        sizes = np.asarray(self.batch_sizes, dtype=np.float64)
        return {"mode": self.mode, "requests": self.n_requests,
                "frames_per_s": round(served / self.wall_s, 2) if self.wall_s > 0 else None,
                "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
                "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
                "mean_ms": round(float(lat.mean()), 3) if lat.size else None,
                "launches": self.launches, "max_inflight_requests": self.max_inflight,
                "admission_waits": self.admission_waits, "rejected": self.rejected,
                "dropped": self.dropped, "failed": self.failed,
                "requests_per_launch": {"mean": round(float(sizes.mean()), 2) if sizes.size else None,
                                        "max": int(sizes.max()) if sizes.size else None,
                                        "histogram": self.launch_histogram()}}


@dataclass
class PoolFrame:
    n_elements: int
    n_samples: int
    side: int
    rf16: object               # device float16 [N][S]
    rf32: object               # device float32 [N][S]
    plan16: object = None
    plan32: object = None


class FramePool:
    """Pre-generated, device-resident frames and their resident plans.

    Shapes follow the mixed workload: N in {64,128,256}, S in {1024,2048,4096},
    square grids of side {256,512,768,1024}; ``per_shape`` distinct phantoms
    per (N, S) are shared by the grid sides.  With ``mirror`` the FP16 plans
    pair mirror tiles wherever the tiling allows it (the arrays are centred
    and the grids symmetric about x = 0); the FP32 plans stay unpaired."""

    def __init__(self, torch, device, n_elements=(64, 128, 256), n_samples=(1024, 2048, 4096),
                 sides=(256, 512, 768, 1024), per_shape=1, seed=5000, plain=True, mirror=False):
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
                p16 = None
                if mirror:
                    try:
                        p16 = hodmas.Plan(geom, grid, fr.n_samples, "f16", max_order=6, flags=hodmas.FLAG_MIRROR)
                    except hodmas.HodmasError:
                        p16 = None   # no even split of the grid's tile columns: unpaired
                if p16 is None:
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


class LaunchError(RuntimeError):
    """An executor could not enqueue a launch (nothing of it was enqueued)."""


class TorchExecutor:
    """Launch slots on the GPU: each slot owns a stream and a batch object;
    a launch of one request runs its frame's own kernel, of several one
    batched submission.  Completion is a HIP event on the slot's stream."""

    def __init__(self, torch, pool, slots=3, max_batch=64, max_units=1 << 20):
        self.torch = torch
        self.pool = pool
        lds = pool.max_lds_bytes
        self.slots = [{"batch": hodmas.Batch(max_frames=max_batch, max_units=max_units, max_lds_bytes=lds),
                       "stream": torch.cuda.Stream()} for _ in range(slots)]

    @property
    def n_slots(self):
        return len(self.slots)

    def launch(self, slot, reqs):
        torch, s = self.torch, self.slots[slot]
        frs = [self.pool.frames[r.frame] for r in reqs]
        for r, fr in zip(reqs, frs):
            if r.image is None:
                r.image = torch.empty((fr.side, fr.side), dtype=torch.float32, device="cuda")
        try:
            if len(reqs) == 1:
                frs[0].plan16.beamform(frs[0].rf16, reqs[0].order, reqs[0].image, stream=s["stream"])
            else:
                b = s["batch"]
                b.set([f.plan16 for f in frs], [f.rf16 for f in frs], [r.order for r in reqs],
                      [r.image for r in reqs], stream=s["stream"])
                b.launch(stream=s["stream"])
        except (hodmas.HodmasError, ValueError) as e:
            raise LaunchError(str(e)) from e
        ev = torch.cuda.Event()
        ev.record(s["stream"])
        return ev

    @staticmethod
    def done(handle):
        return handle.query()

    def close(self):
        for s in self.slots:
            s["batch"].close()
        self.slots = []


class Server:
    """Slots x streams continuous batching with HBM-budget admission.

    Requests are admitted in arrival order while their footprint fits the
    budget; whenever a launch slot is free, everything admitted goes out on it.
    Failures stay with their own request: an unknown frame or an order outside
    1..6 is rejected on arrival, a request whose deadline passes before launch
    is dropped, and when a batched launch is refused its requests are launched
    one by one, so only the request the library refuses fails.  The scheduling
    here is host logic over an executor (by default the GPU one above)."""

    def __init__(self, torch, pool, slots=3, budget_bytes=32 << 30, max_batch=64, max_units=1 << 20,
                 executor=None, clock=time.perf_counter, sleep=time.sleep):
        self.pool = pool
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.executor = executor if executor is not None else TorchExecutor(torch, pool, slots, max_batch,
                                                                             max_units)
        self.clock, self.sleep = clock, sleep

    def close(self):
        if isinstance(self.executor, TorchExecutor):
            self.executor.close()

    def _footprint(self, r: Request) -> int:
        fr = self.pool.frames[r.frame]
        return fr.side * fr.side * 4 + fr.n_elements * fr.n_samples * 2

    def _valid(self, r: Request) -> bool:
        return 0 <= r.frame < len(self.pool.frames) and 1 <= r.order <= hodmas.MAX_ORDER

    @staticmethod
    def _expired(r: Request, now: float) -> bool:
        return r.deadline is not None and now - r.arrival > r.deadline

    def run(self, requests: list[Request], keep_images=False) -> ServeStats:
        ex = self.executor
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        admitted: deque = deque()
        inflight = [None] * ex.n_slots          # (completion handle, requests) per slot
        state = {"bytes": 0, "reqs": 0, "finished": 0}
        stats = ServeStats("batched", len(requests), 0.0)
        total = len(requests)
        t0 = self.clock()

        def finish(r, status, now):
            r.status, r.done = status, now
            state["bytes"] -= r.nbytes
            r.nbytes = 0
            state["finished"] += 1
            if status != "done" or not keep_images:
                r.image = None

        while state["finished"] < total:
            now = self.clock() - t0
            # completions
            for i, slot in enumerate(inflight):
                if slot is not None and ex.done(slot[0]):
                    for r in slot[1]:
                        finish(r, "done", now)
                    state["reqs"] -= len(slot[1])
                    inflight[i] = None
            # arrivals -> validation, deadlines, admission by HBM budget (in arrival order)
            while pending and pending[0].arrival <= now:
                r = pending[0]
                if not self._valid(r):
                    pending.popleft()
                    finish(r, "rejected", now)
                    stats.rejected += 1
                    continue
                if self._expired(r, now):
                    pending.popleft()
                    finish(r, "dropped", now)
                    stats.dropped += 1
                    continue
                nb = self._footprint(r)
                if state["bytes"] + nb > self.budget and (state["bytes"] > 0 or admitted):
                    if not r.waited:
                        r.waited = True
                        stats.admission_waits += 1
                    break
                pending.popleft()
                r.nbytes = nb
                state["bytes"] += nb
                admitted.append(r)
            # admitted requests whose deadline passed before a slot freed up
            if admitted and any(r.deadline is not None for r in admitted):
                keep = deque()
                for r in admitted:
                    if self._expired(r, now):
                        finish(r, "dropped", now)
                        stats.dropped += 1
                    else:
                        keep.append(r)
                admitted = keep
            # a free slot takes everything admitted so far (or one request marked solo)
            if admitted:
                for i in range(len(inflight)):
                    if inflight[i] is not None:
                        continue
                    if admitted[0].solo:
                        take = [admitted.popleft()]
                    else:
                        take = []
                        while admitted and not admitted[0].solo and len(take) < self.max_batch:
                            take.append(admitted.popleft())
                    try:
                        handle = ex.launch(i, take)
                    except LaunchError:
                        if len(take) == 1:
                            finish(take[0], "failed", now)
                            stats.failed += 1
                        else:
                            for r in reversed(take):
                                r.solo = True
                                admitted.appendleft(r)
                        break
                    inflight[i] = (handle, take)
                    state["reqs"] += len(take)
                    stats.launches += 1
                    stats.batch_sizes.append(len(take))
                    stats.max_inflight = max(stats.max_inflight, state["reqs"])
                    break
            if state["finished"] < total:
                # idle: sleep until shortly before the next arrival; with work in
                # flight keep polling the completion events
                nxt = pending[0].arrival if pending else None
                busy = any(s is not None for s in inflight)
                if not busy and not admitted and nxt is not None:
                    delay = nxt - (self.clock() - t0)
                    if delay > 2e-4:
                        self.sleep(delay - 1e-4)
        served = [r for r in requests if r.status == "done"]
        stats.wall_s = max((r.done for r in served), default=0.0)
        stats.latencies_ms = np.array([(r.done - r.arrival) * 1e3 for r in served])
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
        r.status = "done"
        stats.launches += 1
        stats.batch_sizes.append(1)
        if not keep_images:
            r.image = None
    stats.wall_s = max(r.done for r in requests) if requests else 0.0
    stats.latencies_ms = np.array([(r.done - r.arrival) * 1e3 for r in requests])
    return stats

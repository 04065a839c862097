"""Continuous-batching server for population magnitude requests.

Each request is a galaxy population (parametric SFH, metallicity, dust and
redshift per galaxy) asking for six-band magnitudes, optionally with the
gradient of sum (m - target)^2 w.r.t. every per-galaxy parameter.  The SSP
block and the filter set stay resident; forward requests run on the BF16 table
and gradient requests on the FP32 table (both resident).

Scheduling (continuous batching):
  * Requests wait in one FIFO queue per kind (forward / gradient).
  * At most `max_inflight_per_kind` batches of a kind run at once (two by
    default, each on its own stream, so a new batch never waits behind a
    running one).  While the limit is reached, arrivals accumulate in the
    queue; when a batch completes, the next takes the queued requests in order
    while their galaxies fit the largest slot, so load is absorbed by larger
    batches rather than by a queue of launches on a stream.
  * A batch runs in the smallest slot bucket that holds it, padded with inert
    galaxies (z = 1000: no filter ever sees them, so they skip the
    contraction).  Slot choice, in order: an idle slot of that bucket; a new
    one if it fits the HBM byte budget; an idle larger slot; a new one after
    evicting idle slots.
  * Slots (device buffers + pinned staging + a captured hipGraph of the
    batch's whole launch sequence) are allocated under the budget, ahead of
    traffic by `warm()` or on first use.  Each slot has its own stream, so
    batches in flight (of either kind) run concurrently; a batch's inputs go
    over the copy stream and its graph replays on the slot's stream.

"""

from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api

PAD_Z = 1000.0
KIND_FWD = "fwd"      # magnitudes only, BF16 table
KIND_GRAD = "grad"    # magnitudes + adjoint, FP32 table


@dataclass
class Request:
    """One population request.

    sfh_params [5, n] float64; z, lgmet, sigma_z, av, delta, bump [n] float32;
    targets [n, n_band] float32 (gradient requests only).
    """

    rid: int
    sfh_params: np.ndarray
    z: np.ndarray
    lgmet: np.ndarray
    sigma_z: np.ndarray
    av: np.ndarray
    delta: np.ndarray
    bump: np.ndarray
    grad: bool = False
    targets: np.ndarray | None = None
    precision: str | None = None
    t_submit: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    mags: np.ndarray | None = None
    grads: dict | None = None
    error: str | None = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def n(self):
        return int(self.z.shape[0])

    @property
    def kind(self):
        return KIND_GRAD if self.grad else KIND_FWD

    @property
    def latency(self):
        return self.t_done - self.t_submit


# ---------------------------------------------------------------- planning
class AdmissionPlanner:
    """Pure scheduling policy (no GPU): FIFO batching into bucketed slots
    under an HBM byte budget."""

    def __init__(self, buckets, bytes_per_galaxy: dict, budget_bytes: int, slots_per_bucket=1,
                 max_inflight_per_kind=1):
        self.buckets = sorted(int(b) for b in buckets)
        self.bpg = dict(bytes_per_galaxy)
        self.budget = int(budget_bytes)
        self.slots_per_bucket = slots_per_bucket
        self.max_inflight = max_inflight_per_kind
        self.queues = {KIND_FWD: deque(), KIND_GRAD: deque()}
        self.allocated = {}          # (kind, bucket) -> number of slots allocated
        self.busy = {}               # (kind, bucket) -> number of slots in flight
        self.inflight = {KIND_FWD: 0, KIND_GRAD: 0}
        self.reserved = 0
        self.evicted = []            # idle slots the engine must free

    def slot_bytes(self, kind, bucket):
        return self.bpg[kind] * bucket

    def enqueue(self, req) -> bool:
        if req.n > self.buckets[-1] or self.slot_bytes(req.kind, self.bucket_for(req.n)) > self.budget:
            req.error = (f"request of {req.n} galaxies exceeds the largest slot "
                         f"({self.buckets[-1]}) or the HBM budget")
            return False
        self.queues[req.kind].append(req)
        return True

    def bucket_for(self, n):
        for b in self.buckets:
            if n <= b:
                return b
        return None

    def next_batch(self, kind):
        """Requests for the next batch of `kind` and its bucket, or None."""
        q = self.queues[kind]
        if not q or self.inflight[kind] >= self.max_inflight:
            return None
        take, total = [], 0
        for r in q:
            if total + r.n > self.buckets[-1]:
                break
            take.append(r)
            total += r.n
        need = self.bucket_for(total)
        key = (kind, need)
        nbytes = self.slot_bytes(kind, need)
        can_add = self.allocated.get(key, 0) < self.slots_per_bucket
        bucket = None
        if self._idle(key) > 0:                                   # 1. idle exact slot
            bucket = need
        elif can_add and self.reserved + nbytes <= self.budget:  # 2. new exact slot
            self._allocate(key)
            bucket = need
        else:
            for b in self.buckets:                                # 3. idle larger slot
                if b > need and self._idle((kind, b)) > 0:
                    bucket = b
                    break
        if bucket is None:
            if not can_add:
                return None
            # 4. evict idle slots (least useful first: other kind, then larger)
            victims = sorted((k for k in self.allocated if self._idle(k) > 0),
                             key=lambda k: (k[0] == kind, -k[1]))
            for vk in victims:
                while self._idle(vk) > 0 and self.reserved + nbytes > self.budget:
                    self.allocated[vk] -= 1
                    self.reserved -= self.slot_bytes(*vk)
                    self.evicted.append(vk)
            if self.reserved + nbytes > self.budget:
                return None
            self._allocate(key)
            bucket = need
        key = (kind, bucket)
        self.busy[key] = self.busy.get(key, 0) + 1
        self.inflight[kind] += 1
        for _ in take:
            q.popleft()
        return take, bucket

    def _allocate(self, key):
        self.allocated[key] = self.allocated.get(key, 0) + 1
        self.reserved += self.slot_bytes(*key)

    def _idle(self, key):
        return self.allocated.get(key, 0) - self.busy.get(key, 0)

    def release(self, kind, bucket):
        self.busy[(kind, bucket)] -= 1
        self.inflight[kind] -= 1


# ---------------------------------------------------------------- GPU slots
class _Slot:
    """Device buffers, pinned staging and the captured graph for one batch
    capacity of one kind."""

    def __init__(self, eng, kind, cap):
        self.kind, self.cap = kind, cap
        d = eng.device
        f32, f64 = torch.float32, torch.float64
        nb = eng.n_band
        self.h_in64 = torch.empty((5, cap), dtype=f64, pin_memory=True)
        self.h_in32 = torch.empty((6 + (nb if kind == KIND_GRAD else 0) + 1, cap), dtype=f32, pin_memory=True)
        self.d_par = torch.empty((5, cap), dtype=f64, device=d)
        self.d_in32 = torch.empty_like(self.h_in32, device=d)
        self.pop = api.DevicePopulation(eng.t_table, None, self.d_par, self.d_in32[0], self.d_in32[1],
                                        self.d_in32[2], self.d_in32[3], self.d_in32[4], self.d_in32[5])
        self.mags = torch.empty((cap, nb), dtype=f32, device=d)
        prec = "bf16" if kind == KIND_FWD else "fp32"
        self.ws = api.Workspace(api.workspace_size(2, eng.ssp_h, eng.flt_h, cap, eng.n_t, prec), d)
        outs = [self.mags]
        if kind == KIND_GRAD:
            self.targets = self.d_in32[6:6 + nb].t()          # [cap, nb] view
            self.valid = self.d_in32[6 + nb]
            self.bands = torch.empty((cap, 2, nb), dtype=f32, device=d)
            self.moments = torch.empty((cap, 3, nb), dtype=f32, device=d)
            self.bar = torch.empty((cap, nb), dtype=f32, device=d)
            self.ws_b = api.Workspace(api.workspace_size(3, eng.ssp_h, eng.flt_h, cap, eng.n_t, "fp32"), d)
            self.g64 = torch.empty((5, cap), dtype=f64, device=d)
            self.g32 = torch.empty((5, cap), dtype=f32, device=d)
            self.outs = {"sfh_params": self.g64, "lgmet": self.g32[0], "sigma_z": self.g32[1],
                         "av": self.g32[2], "delta": self.g32[3], "bump": self.g32[4]}
            outs += [self.g64, self.g32]
        self.h_mags = torch.empty((cap, nb), dtype=f32, pin_memory=True)
        if kind == KIND_GRAD:
            self.h_g64 = torch.empty((5, cap), dtype=f64, pin_memory=True)
            self.h_g32 = torch.empty((5, cap), dtype=f32, pin_memory=True)
        self.eng = eng
        self.stream = torch.cuda.Stream(device=d)
        self.graph = None
        self.done = torch.cuda.Event()
        self.batch = None

    def run_body(self):
        """The batch's launch sequence (captured once, replayed per batch)."""
        e = self.eng
        if self.kind == KIND_FWD:
            api.mags(e.ssp_h, e.flt_h, e.cosmo, self.pop, precision="bf16", workspace=self.ws, out=self.mags)
        else:
            api.mags(e.ssp_h, e.flt_h, e.cosmo, self.pop, precision="fp32", with_moments=True,
                     workspace=self.ws, out=self.mags, bands_out=self.bands, moments_out=self.moments)
            torch.sub(self.mags, self.targets, out=self.bar)
            self.bar.mul_(self.valid[:, None] * 2.0)
            api.mags_vjp(e.ssp_h, e.flt_h, e.cosmo, self.pop, self.bar, bands=self.bands,
                         moments=self.moments, workspace=self.ws_b, outs=self.outs)

    def capture(self):
        stream = self.stream
        self.h_in32[0].fill_(PAD_Z)     # inert galaxies for the eager warm-up
        self.h_in64[0].fill_(1.0)
        self.h_in64[1].fill_(1.0)
        self.d_in32.copy_(self.h_in32)
        self.d_par.copy_(self.h_in64)
        with torch.cuda.stream(stream):
            self.run_body()
        stream.synchronize()
        if self.eng.use_graphs:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph, stream=stream):
                self.run_body()
            stream.synchronize()


class ServeEngine:
    """Continuous-batching server on one GPU (see the module docstring)."""

    def __init__(self, ssp, filters, cosmo=None, n_t=100,
                 buckets=(8192, 12288, 16384, 24576, 32768, 49152, 65536, 98304, 131072),
                 hbm_budget_bytes=48 << 30, slots_per_bucket=2, max_inflight_per_kind=2,
                 use_graphs=True, device="cuda"):
        import synth
        self.device = torch.device(device)
        self.n_t = n_t
        self.cosmo = cosmo or api.Cosmology()
        self.ssp_h = api.SspBlock.from_synth(ssp, precisions=("fp32", "bf16"))
        self.flt_h = api.FilterBank.from_synth(filters)
        self.n_band = self.flt_h.n_band
        self.t_table = torch.tensor(synth.population.make_time_grid(n_t), dtype=torch.float64,
                                    device=self.device)
        self.use_graphs = use_graphs
        ref = 65536
        bpg = {}
        for kind, prec in ((KIND_FWD, "bf16"), (KIND_GRAD, "fp32")):
            ws = api.workspace_size(2, self.ssp_h, self.flt_h, ref, n_t, prec)
            if kind == KIND_GRAD:
                ws += api.workspace_size(3, self.ssp_h, self.flt_h, ref, n_t, "fp32")
            io = 5 * 8 + 7 * 4 + self.n_band * 4 * (1 if kind == KIND_FWD else 8) + (60 if kind == KIND_GRAD else 0)
            bpg[kind] = int(math.ceil(ws / ref)) + io
        self.planner = AdmissionPlanner(buckets, bpg, hbm_budget_bytes, slots_per_bucket,
                                        max_inflight_per_kind)
        self.free_slots = {}
        self.inflight = []
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.lock = threading.Lock()
        self.incoming = deque()
        self.completed = []
        self._stop = False
        self._thread = None
        self.galaxies_done = 0
        self.batches_run = 0

    # -------------------------------------------------------------- client
    def submit(self, req: Request):
        req.t_submit = time.perf_counter()
        with self.lock:
            self.incoming.append(req)
        return req

    def start(self):
        self._thread = threading.Thread(target=self._loop, name="dsps-serve", daemon=True)
        self._thread.start()

    def stop(self, drain=True):
        if drain:
            while True:
                with self.lock:
                    idle = not self.incoming
                if idle and not self.inflight and not any(self.planner.queues.values()):
                    break
                time.sleep(0.001)
        self._stop = True
        if self._thread:
            self._thread.join()

    def warm(self, kinds=(KIND_FWD, KIND_GRAD), buckets=None):
        """Allocate and capture slots ahead of traffic."""
        for kind in kinds:
            for b in buckets or self.planner.buckets:
                key = (kind, b)
                while (self.planner.allocated.get(key, 0) < self.planner.slots_per_bucket and
                       self.planner.reserved + self.planner.slot_bytes(kind, b) <= self.planner.budget):
                    self.planner._allocate(key)
                    slot = _Slot(self, kind, b)
                    slot.capture()
                    self.free_slots.setdefault(key, []).append(slot)

    # -------------------------------------------------------------- engine
    def _get_slot(self, kind, bucket):
        key = (kind, bucket)
        lst = self.free_slots.setdefault(key, [])
        if lst:
            return lst.pop()
        slot = _Slot(self, kind, bucket)
        slot.capture()
        return slot

    def _launch(self, kind, reqs, bucket):
        slot = self._get_slot(kind, bucket)
        nb = self.n_band
        h64, h32 = slot.h_in64.numpy(), slot.h_in32.numpy()
        o = 0
        for r in reqs:
            n = r.n
            h64[:, o:o + n] = r.sfh_params
            h32[0, o:o + n] = r.z
            h32[1, o:o + n] = r.lgmet
            h32[2, o:o + n] = r.sigma_z
            h32[3, o:o + n] = r.av
            h32[4, o:o + n] = r.delta
            h32[5, o:o + n] = r.bump
            if kind == KIND_GRAD:
                h32[6:6 + nb, o:o + n] = r.targets.T
                h32[6 + nb, o:o + n] = 1.0
            r.t_start = time.perf_counter()
            o += n
        # inert padding
        h32[0, o:] = PAD_Z
        h32[1:6, o:] = 0.1
        h64[:, o:] = 1.0
        if kind == KIND_GRAD:
            h32[6:, o:] = 0.0
        stream = slot.stream
        ev = torch.cuda.Event()
        with torch.cuda.stream(self.copy_stream):
            slot.d_par.copy_(slot.h_in64, non_blocking=True)
            slot.d_in32.copy_(slot.h_in32, non_blocking=True)
            ev.record(self.copy_stream)
        stream.wait_event(ev)
        with torch.cuda.stream(stream):
            if slot.graph is not None:
                slot.graph.replay()
            else:
                slot.run_body()
            slot.h_mags.copy_(slot.mags, non_blocking=True)
            if kind == KIND_GRAD:
                slot.h_g64.copy_(slot.g64, non_blocking=True)
                slot.h_g32.copy_(slot.g32, non_blocking=True)
            slot.done.record(stream)
        slot.batch = reqs
        self.inflight.append(slot)

    def _finish(self, slot):
        mags = slot.h_mags.numpy()
        names = ("lgmet", "sigma_z", "av", "delta", "bump")
        o = 0
        now = time.perf_counter()
        for r in slot.batch:
            n = r.n
            r.mags = mags[o:o + n].copy()
            if slot.kind == KIND_GRAD:
                g = {"sfh_params": slot.h_g64.numpy()[:, o:o + n].copy()}
                g32 = slot.h_g32.numpy()
                for i, k in enumerate(names):
                    g[k] = g32[i, o:o + n].copy()
                r.grads = g
            r.t_done = now
            r.done.set()
            o += n
            self.galaxies_done += n
        self.completed.extend(slot.batch)
        self.batches_run += 1
        self.planner.release(slot.kind, slot.cap)
        slot.batch = None
        self.free_slots.setdefault((slot.kind, slot.cap), []).append(slot)

    def _loop(self):
        while not self._stop:
            with self.lock:
                while self.incoming:
                    r = self.incoming.popleft()
                    if not self.planner.enqueue(r):
                        r.t_done = time.perf_counter()
                        r.done.set()
            progressed = False
            for kind in (KIND_GRAD, KIND_FWD):
                nxt = self.planner.next_batch(kind)
                for vk in self.planner.evicted:
                    self.free_slots[vk].pop()        # drop an idle slot's buffers and graph
                self.planner.evicted.clear()
                if nxt is not None:
                    self._launch(kind, *nxt)
                    progressed = True
            still = []
            for slot in self.inflight:
                if slot.done.query():
                    self._finish(slot)
                    progressed = True
                else:
                    still.append(slot)
            self.inflight = still
            if not progressed:
                time.sleep(0.0002)


def make_trace(n_requests, rate_hz=200.0, seed=6, grad_fraction=0.3, n_band=6,
               n_range=(1e3, 1e5)):
    """Poisson arrivals; N ~ logU[n_range]; per-request z range
    z_lo ~ U[0.1, 2.5], z_hi = min(3, z_lo + U[0.05, 0.5]); a fraction of the
    requests ask for gradients.  Returns (arrival offsets [s], requests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n_requests):
        n = int(round(10.0 ** rng.uniform(math.log10(n_range[0]), math.log10(n_range[1]))))
        z_lo = rng.uniform(0.1, 2.5)
        z_hi = min(3.0, z_lo + rng.uniform(0.05, 0.5))
        grad = bool(rng.uniform() < grad_fraction)
        f32 = lambda a: np.asarray(a, dtype=np.float32)
        par = np.stack([10.0 ** rng.uniform(0, 2, n), rng.uniform(1, 5, n), rng.uniform(0.5, 3, n),
                        rng.uniform(0, 1, n), rng.uniform(2, 13, n)])
        reqs.append(Request(
            rid=i, sfh_params=np.ascontiguousarray(par), z=f32(rng.uniform(z_lo, z_hi, n)),
            lgmet=f32(rng.uniform(-3, -1.7, n)), sigma_z=f32(rng.uniform(0.1, 0.5, n)),
            av=f32(rng.uniform(0, 2, n)), delta=f32(rng.uniform(-0.7, 0.3, n)),
            bump=f32(rng.uniform(0, 3, n)), grad=grad,
            targets=f32(rng.normal(22.0, 1.0, (n, n_band))) if grad else None))
    return t, reqs


def replay_trace(engine: ServeEngine, arrivals, reqs, timeout_s=600.0):
    """Submit requests at their arrival offsets (open loop) and wait for all."""
    t0 = time.perf_counter()
    for t_arr, r in zip(arrivals, reqs):
        while time.perf_counter() - t0 < t_arr:
            time.sleep(min(0.0005, max(0.0, t_arr - (time.perf_counter() - t0))))
        engine.submit(r)
    deadline = time.perf_counter() + timeout_s
    for r in reqs:
        if not r.done.wait(max(0.0, deadline - time.perf_counter())):
            raise TimeoutError(f"request {r.rid} not served")
    return time.perf_counter() - t0


def latency_summary(reqs, wall_s):
    lat = np.array([r.latency for r in reqs if r.error is None]) * 1e3
    gal = sum(r.n for r in reqs if r.error is None)
    return {"requests": len(reqs), "galaxies": int(gal), "wall_s": wall_s,
            "throughput_galaxies_per_s": gal / wall_s,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "rejected": sum(r.error is not None for r in reqs)}


def serial_baseline(ssp_h, flt_h, cosmo, t_table, arrivals, reqs):
    """The same trace served one request at a time on the plain FP32 path
    (no batching, no graphs): latency includes queueing behind earlier
    requests."""
    t0 = time.perf_counter()
    lat = []
    for t_arr, r in zip(arrivals, reqs):
        now = time.perf_counter() - t0
        if now < t_arr:
            time.sleep(t_arr - now)
        d = torch.device("cuda")
        pop = api.DevicePopulation(t_table, None, torch.tensor(r.sfh_params, device=d),
                                   *(torch.tensor(getattr(r, k), device=d) for k in
                                     ("z", "lgmet", "sigma_z", "av", "delta", "bump")))
        if r.grad:
            m, bands, mom = api.mags(ssp_h, flt_h, cosmo, pop, precision="fp32", with_moments=True)
            bar = 2.0 * (m - torch.tensor(r.targets, device=d))
            api.mags_vjp(ssp_h, flt_h, cosmo, pop, bar, bands=bands, moments=mom)
        else:
            api.mags(ssp_h, flt_h, cosmo, pop, precision="fp32")
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) - t_arr)
    wall = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    gal = sum(r.n for r in reqs)
    return {"requests": len(reqs), "galaxies": int(gal), "wall_s": wall,
            "throughput_galaxies_per_s": gal / wall, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max())}

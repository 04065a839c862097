"""Continuous-batching server for population magnitude requests.

Each request is a galaxy population (parametric SFH, metallicity, dust and
redshift per galaxy) asking for six-band magnitudes, optionally with the
gradient of sum (m - target)^2 w.r.t. every per-galaxy parameter.  The SSP
block, the filter set and the SFH time grid stay resident; forward requests
run on the BF16 table (dsps_mags) and gradient requests on the FP32 table in
one fused call (dsps_mags_residual_vjp: one ordering sort, one weights pass,
the forward contraction and the reverse pass).

Scheduling:
  * Requests wait in one FIFO queue per kind (forward / gradient).  A request
    may carry a timeout: if it has not started by then, or if it is cancelled
    before it starts, it leaves the queue with `error` set.  A request that
    has started always completes (its GPU work is not recalled).
  * Each kind has its own lanes (`max_inflight_per_kind` streams, two by
    default), so a forward batch never queues behind a gradient batch on a
    stream; with the default four lanes each stream has a hardware queue of
    its own.  Forward batches are formed first on every pass of the loop.
  * While a kind's lanes are busy, its arrivals accumulate; when a lane frees,
    the next batch takes the queued requests in order while their galaxies fit
    the kind's batch limit (at most the largest slot; for gradients also
    `batch_galaxies["grad"]` unless the first request alone is larger, so a
    large gradient request is not made to wait for others).
  * All slots are allocated and their graphs captured ahead of traffic by
    `warm()`, within the HBM byte budget: first the largest bucket of each
    kind (so every admissible request fits), then the other buckets, smallest
    first, up to `slots_per_bucket` each.  The loop never allocates, captures
    or frees: a batch runs in the smallest idle slot that holds it, or waits.
  * A slot is sized for its bucket; the batch's real size goes to the device
    as the population's live count (dsps_pop.n_live), so the kernels stop at
    the last real galaxy and padding costs nothing.  Inputs, the graph replay
    and the results' copy back all run in order on the batch's lane.
  * Every answer equals the same request run alone through the plain calls,
    bit for bit (tests/test_gpu_serve.py).
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

KIND_FWD = "fwd"      # magnitudes only, BF16 table
KIND_GRAD = "grad"    # magnitudes + gradient of the squared residual, FP32 table
KINDS = (KIND_FWD, KIND_GRAD)
GRAD_NAMES = ("lgmet", "sigma_z", "av", "delta", "bump")


@dataclass(eq=False)      # identity: a request is found in a queue by itself
class Request:
    """One population request.

    sfh_params [5, n] float64; z, lgmet, sigma_z, av, delta, bump [n] float32;
    targets [n, n_band] float32 (gradient requests only).  timeout_s: seconds
    after submission by which the request must have started, or None.
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
    timeout_s: float | None = None
    cancelled: bool = False
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
    """Pure scheduling policy (no GPU): the slot plan under an HBM byte
    budget, per-kind FIFO queues with timeouts and cancellation, and batch
    formation into the allocated slots."""

    def __init__(self, buckets, bytes_per_galaxy: dict, budget_bytes: int, slots_per_bucket=1,
                 max_inflight_per_kind=1, batch_galaxies: dict | None = None):
        self.buckets = sorted(int(b) for b in buckets)
        self.bpg = dict(bytes_per_galaxy)
        self.budget = int(budget_bytes)
        self.slots_per_bucket = slots_per_bucket
        self.max_inflight = max_inflight_per_kind
        self.batch_galaxies = dict(batch_galaxies or {})
        self.queues = {k: deque() for k in KINDS}
        self.allocated = {}          # (kind, bucket) -> slots allocated
        self.busy = {}               # (kind, bucket) -> slots in flight
        self.inflight = {k: 0 for k in KINDS}
        self.reserved = 0
        self.dropped = []            # requests that timed out or were cancelled in the queue

    def slot_bytes(self, kind, bucket):
        return self.bpg[kind] * bucket

    def plan_slots(self, kinds=KINDS):
        """Allocate the slot plan within the budget; returns the new
        (kind, bucket) slots in allocation order."""
        new = []

        def take(key):
            if (self.allocated.get(key, 0) < self.slots_per_bucket and
                    self.reserved + self.slot_bytes(*key) <= self.budget):
                self.allocated[key] = self.allocated.get(key, 0) + 1
                self.reserved += self.slot_bytes(*key)
                new.append(key)
                return True
            return False

        for kind in kinds:                       # every admissible size has a slot
            take((kind, self.buckets[-1]))
        for _ in range(self.slots_per_bucket):   # then the rest, smallest first
            for b in self.buckets:
                for kind in kinds:
                    take((kind, b))
        return new

    def largest_slot(self, kind):
        sizes = [b for (k, b), c in self.allocated.items() if k == kind and c > 0]
        return max(sizes) if sizes else 0

    def enqueue(self, req) -> bool:
        cap = self.largest_slot(req.kind)
        if req.n > cap:
            req.error = (f"request of {req.n} galaxies exceeds the largest {req.kind} slot "
                         f"({cap}) the HBM budget allows")
            return False
        self.queues[req.kind].append(req)
        return True

    def cancel(self, req) -> bool:
        """Mark a queued request cancelled (it leaves at the next batch
        formation); False if it is not queued (started, finished or unknown)."""
        if req in self.queues[req.kind]:
            req.cancelled = True
            return True
        return False

    def _purge(self, kind, now):
        q = self.queues[kind]
        if not any(r.cancelled or (r.timeout_s is not None and now - r.t_submit > r.timeout_s)
                   for r in q):
            return
        keep = deque()
        for r in q:
            if r.cancelled:
                r.error = "cancelled"
                self.dropped.append(r)
            elif r.timeout_s is not None and now - r.t_submit > r.timeout_s:
                r.error = f"timed out after {r.timeout_s:g} s in the queue"
                self.dropped.append(r)
            else:
                keep.append(r)
        self.queues[kind] = keep

    def _idle(self, key):
        return self.allocated.get(key, 0) - self.busy.get(key, 0)

    def next_batch(self, kind, now=0.0):
        """Requests for the next batch of `kind` and its slot bucket, or None
        (nothing queued, no free lane, or no idle slot holds the first
        request).  Expired and cancelled requests go to `dropped` first."""
        self._purge(kind, now)
        q = self.queues[kind]
        if not q or self.inflight[kind] >= self.max_inflight:
            return None
        idle = [b for b in self.buckets if self._idle((kind, b)) > 0]
        if not idle or idle[-1] < q[0].n:
            return None
        limit = idle[-1]
        cap = self.batch_galaxies.get(kind)
        if cap:
            limit = min(limit, max(cap, q[0].n))
        take, total = [], 0
        for r in q:
            if total + r.n > limit:
                break
            take.append(r)
            total += r.n
        bucket = next(b for b in idle if b >= total)
        key = (kind, bucket)
        self.busy[key] = self.busy.get(key, 0) + 1
        self.inflight[kind] += 1
        for _ in take:
            q.popleft()
        return take, bucket

    def release(self, kind, bucket):
        self.busy[(kind, bucket)] -= 1
        self.inflight[kind] -= 1


# ---------------------------------------------------------------- GPU slots
class _Slot:
    """Device buffers, pinned staging and the captured graph for one batch
    capacity of one kind.  The population's live count lives on the device
    (d_live), so the graph serves any batch up to the capacity."""

    def __init__(self, eng, kind, cap):
        self.kind, self.cap = kind, cap
        d = eng.device
        f32, f64 = torch.float32, torch.float64
        nb = eng.n_band
        self.h_par = torch.empty((5, cap), dtype=f64, pin_memory=True)
        self.h_in32 = torch.empty((6, cap), dtype=f32, pin_memory=True)
        self.h_live = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self.d_par = torch.empty((5, cap), dtype=f64, device=d)
        self.d_in32 = torch.empty((6, cap), dtype=f32, device=d)
        self.d_live = torch.zeros(1, dtype=torch.int32, device=d)
        self.pop = api.DevicePopulation(eng.t_table, None, self.d_par, *self.d_in32.unbind(0),
                                        n_live=self.d_live)
        self.mags = torch.empty((cap, nb), dtype=f32, device=d)
        self.h_mags = torch.empty((cap, nb), dtype=f32, pin_memory=True)
        if kind == KIND_FWD:
            self.ws = api.Workspace(api.workspace_size(api.N.OP_MAGS, eng.ssp, eng.flt, cap,
                                                       eng.n_t, "bf16"), d)
        else:
            self.ws = api.Workspace(api.workspace_size(api.N.OP_MAGS_VJP, eng.ssp, eng.flt, cap,
                                                       eng.n_t, "fp32"), d)
            self.h_tgt = torch.empty((cap, nb), dtype=f32, pin_memory=True)
            self.d_tgt = torch.empty((cap, nb), dtype=f32, device=d)
            self.g64 = torch.empty((5, cap), dtype=f64, device=d)
            self.g32 = torch.empty((5, cap), dtype=f32, device=d)
            self.h_g64 = torch.empty((5, cap), dtype=f64, pin_memory=True)
            self.h_g32 = torch.empty((5, cap), dtype=f32, pin_memory=True)
            self.outs = {"sfh_params": self.g64}
            self.outs.update({k: self.g32[i] for i, k in enumerate(GRAD_NAMES)})
        self.eng = eng
        self.graph = None
        self.batch = None
        self.lane = None
        self.done = torch.cuda.Event()

    def run_body(self):
        """The batch's launch sequence (captured once, replayed per batch)."""
        e = self.eng
        if self.kind == KIND_FWD:
            api.mags(e.ssp, e.flt, e.cosmo, self.pop, precision="bf16", workspace=self.ws,
                     out=self.mags)
        else:
            api.mags_residual_vjp(e.ssp, e.flt, e.cosmo, self.pop, self.d_tgt, None,
                                  workspace=self.ws, out=self.mags, outs=self.outs)

    def capture(self, stream):
        # valid inputs for the eager warm-up run over the whole capacity
        self.h_par.copy_(torch.tensor([[3.0], [2.0], [1.0], [0.3], [8.0]], dtype=torch.float64))
        self.h_in32.copy_(torch.tensor([[0.5], [-2.3], [0.3], [0.5], [-0.2], [1.0]]))
        self.h_live[0] = self.cap
        with torch.cuda.stream(stream):
            self.d_par.copy_(self.h_par, non_blocking=True)
            self.d_in32.copy_(self.h_in32, non_blocking=True)
            self.d_live.copy_(self.h_live, non_blocking=True)
            if self.kind == KIND_GRAD:
                self.d_tgt.fill_(22.0)
            self.run_body()
        stream.synchronize()
        if self.eng.use_graphs:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph, stream=stream):
                self.run_body()
            stream.synchronize()


class ServeEngine:
    """Continuous-batching server on one GPU (see the module docstring).

    ssp: an api.SspBlock holding both the float32 and the bfloat16 tables;
    filters: an api.FilterBank; t_table: the SFH time grid [n_t] in Gyr shared
    by every request (tensor or array, float64)."""

    def __init__(self, ssp: api.SspBlock, filters: api.FilterBank, t_table, cosmo=None,
                 buckets=(8192, 12288, 16384, 24576, 32768, 49152, 65536, 98304, 131072),
                 hbm_budget_bytes=48 << 30, slots_per_bucket=2, max_inflight_per_kind=2,
                 batch_galaxies=None, use_graphs=True, device="cuda"):
        self.device = torch.device(device)
        self.ssp, self.flt = ssp, filters
        self.cosmo = cosmo or api.Cosmology()
        self.n_band = filters.n_band
        self.t_table = torch.as_tensor(np.asarray(t_table, dtype=np.float64)
                                       if not isinstance(t_table, torch.Tensor) else t_table,
                                       dtype=torch.float64).to(self.device).contiguous()
        self.n_t = int(self.t_table.shape[0])
        self.use_graphs = use_graphs
        ref = 65536
        bpg = {}
        for kind, op, prec in ((KIND_FWD, api.N.OP_MAGS, "bf16"),
                               (KIND_GRAD, api.N.OP_MAGS_VJP, "fp32")):
            ws = api.workspace_size(op, ssp, filters, ref, self.n_t, prec)
            io = 5 * 8 + 6 * 4 + self.n_band * 4 * (1 if kind == KIND_FWD else 2)
            if kind == KIND_GRAD:
                io += 5 * 8 + 5 * 4
            bpg[kind] = int(math.ceil(ws / ref)) + io
        if batch_galaxies is None:
            batch_galaxies = {KIND_GRAD: 32768}
        self.planner = AdmissionPlanner(buckets, bpg, hbm_budget_bytes, slots_per_bucket,
                                        max_inflight_per_kind, batch_galaxies)
        self.lanes = {k: [torch.cuda.Stream(device=self.device)
                          for _ in range(max_inflight_per_kind)] for k in KINDS}
        self.free_lanes = {k: list(v) for k, v in self.lanes.items()}
        self.free_slots = {}
        self.inflight = []
        self.lock = threading.Lock()
        self.incoming = deque()
        self.completed = []
        self._stop = False
        self._thread = None
        self.warmed = False
        self.stats = {"captures_in_warm": 0, "captures_in_loop": 0, "evictions": 0,
                      "warm_s": 0.0, "batches": {k: 0 for k in KINDS},
                      "galaxies": {k: 0 for k in KINDS}, "slot_galaxies": {k: 0 for k in KINDS},
                      "dropped": 0}

    # -------------------------------------------------------------- client
    def submit(self, req: Request):
        req.t_submit = time.perf_counter()
        with self.lock:
            self.incoming.append(req)
        return req

    def cancel(self, req: Request) -> bool:
        """Cancel a request that has not started: True if it will not run
        (it completes with error "cancelled"), False if it has started or
        finished."""
        with self.lock:
            if req in self.incoming:
                req.cancelled = True
                return True
            return self.planner.cancel(req)

    def start(self):
        if not self.warmed:
            self.warm()
        self._thread = threading.Thread(target=self._loop, name="dsps-serve", daemon=True)
        self._thread.start()

    def stop(self, drain=True):
        if drain:
            while True:
                with self.lock:
                    idle = not self.incoming and not any(self.planner.queues.values())
                if idle and not self.inflight:
                    break
                time.sleep(0.001)
        self._stop = True
        if self._thread:
            self._thread.join()

    def warm(self):
        """Allocate every slot the budget allows and capture its graph."""
        t0 = time.perf_counter()
        for kind, b in self.planner.plan_slots():
            slot = _Slot(self, kind, b)
            slot.capture(self.lanes[kind][0])
            self.free_slots.setdefault((kind, b), []).append(slot)
            self.stats["captures_in_warm"] += 1
        torch.cuda.synchronize(self.device)
        self.stats["warm_s"] = time.perf_counter() - t0
        self.warmed = True

    # -------------------------------------------------------------- engine
    def _launch(self, kind, reqs, bucket):
        slot = self.free_slots[(kind, bucket)].pop()
        lane = self.free_lanes[kind].pop()
        nb = self.n_band
        par, in32 = slot.h_par.numpy(), slot.h_in32.numpy()
        o = 0
        now = time.perf_counter()
        for r in reqs:
            n = r.n
            par[:, o:o + n] = r.sfh_params
            for i, k in enumerate(("z", "lgmet", "sigma_z", "av", "delta", "bump")):
                in32[i, o:o + n] = getattr(r, k)
            if kind == KIND_GRAD:
                slot.h_tgt.numpy()[o:o + n] = r.targets
            r.t_start = now
            o += n
        slot.h_live[0] = o
        # the batch's columns only, row by row (each row slice is contiguous,
        # so every copy is one asynchronous transfer from pinned memory)
        with torch.cuda.stream(lane):
            for i in range(5):
                slot.d_par[i, :o].copy_(slot.h_par[i, :o], non_blocking=True)
            for i in range(6):
                slot.d_in32[i, :o].copy_(slot.h_in32[i, :o], non_blocking=True)
            slot.d_live.copy_(slot.h_live, non_blocking=True)
            if kind == KIND_GRAD:
                slot.d_tgt[:o].copy_(slot.h_tgt[:o], non_blocking=True)
            if slot.graph is not None:
                slot.graph.replay()
            else:
                slot.run_body()
            slot.h_mags[:o].copy_(slot.mags[:o], non_blocking=True)
            if kind == KIND_GRAD:
                for i in range(5):
                    slot.h_g64[i, :o].copy_(slot.g64[i, :o], non_blocking=True)
                    slot.h_g32[i, :o].copy_(slot.g32[i, :o], non_blocking=True)
            slot.done.record(lane)
        slot.batch, slot.lane = reqs, lane
        self.inflight.append(slot)
        self.stats["batches"][kind] += 1
        self.stats["galaxies"][kind] += o
        self.stats["slot_galaxies"][kind] += bucket

    def _finish(self, slot):
        mags = slot.h_mags.numpy()
        o = 0
        now = time.perf_counter()
        for r in slot.batch:
            n = r.n
            r.mags = mags[o:o + n].copy()
            if slot.kind == KIND_GRAD:
                g = {"sfh_params": slot.h_g64.numpy()[:, o:o + n].copy()}
                g32 = slot.h_g32.numpy()
                for i, k in enumerate(GRAD_NAMES):
                    g[k] = g32[i, o:o + n].copy()
                r.grads = g
            r.t_done = now
            r.done.set()
            o += n
        self.completed.extend(slot.batch)
        self.planner.release(slot.kind, slot.cap)
        self.free_lanes[slot.kind].append(slot.lane)
        slot.batch, slot.lane = None, None
        self.free_slots[(slot.kind, slot.cap)].append(slot)

    def _drop(self, reqs):
        now = time.perf_counter()
        for r in reqs:
            r.t_done = now
            r.done.set()
        self.stats["dropped"] += len(reqs)

    def _loop(self):
        while not self._stop:
            progressed = False
            batches = []
            with self.lock:
                while self.incoming:
                    r = self.incoming.popleft()
                    if r.cancelled:
                        r.error = "cancelled"
                        self.planner.dropped.append(r)
                    elif not self.planner.enqueue(r):
                        self.planner.dropped.append(r)
                now = time.perf_counter()
                for kind in KINDS:            # forward batches first
                    nxt = self.planner.next_batch(kind, now)
                    if nxt is not None:
                        batches.append((kind, nxt))
                dropped, self.planner.dropped = self.planner.dropped, []
            if dropped:
                self._drop(dropped)
                progressed = True
            for kind, (reqs, bucket) in batches:
                self._launch(kind, reqs, bucket)
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


# ---------------------------------------------------------------- workload
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


def _pct(lat):
    if not len(lat):
        return {"requests": 0}
    return {"requests": int(len(lat)), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(np.max(lat))}


def latency_summary(reqs, wall_s, latencies_ms=None):
    """Whole-trace throughput and latency percentiles, overall and per kind;
    latencies_ms overrides the requests' own (t_done - t_submit)."""
    ok = [i for i, r in enumerate(reqs) if r.error is None]
    lat = (np.asarray(latencies_ms, dtype=np.float64) if latencies_ms is not None
           else np.array([r.latency for r in reqs]) * 1e3)
    gal = sum(reqs[i].n for i in ok)
    out = {"requests": len(reqs), "galaxies": int(gal), "wall_s": wall_s,
           "throughput_galaxies_per_s": gal / wall_s, "rejected": len(reqs) - len(ok)}
    out.update({k: v for k, v in _pct(lat[ok]).items() if k != "requests"})
    for kind in KINDS:
        sel = [i for i in ok if reqs[i].kind == kind]
        out[kind] = _pct(lat[sel])
    return out


def serial_baseline(ssp, flt, cosmo, t_table, arrivals, reqs):
    """The same trace served one request at a time through the plain calls,
    with the server's arithmetic (forward on the BF16 table, gradients by the
    fused FP32 residual call) but no batching, graphs or lanes: a request
    waits for every earlier one."""
    d = torch.device("cuda")
    t_table = torch.as_tensor(t_table, dtype=torch.float64).to(d)
    t0 = time.perf_counter()
    lat = []
    for t_arr, r in zip(arrivals, reqs):
        now = time.perf_counter() - t0
        if now < t_arr:
            time.sleep(t_arr - now)
        pop = api.DevicePopulation(t_table, None, torch.tensor(r.sfh_params, device=d),
                                   *(torch.tensor(getattr(r, k), device=d) for k in
                                     ("z", "lgmet", "sigma_z", "av", "delta", "bump")))
        if r.grad:
            m, g = api.mags_residual_vjp(ssp, flt, cosmo, pop, torch.tensor(r.targets, device=d),
                                         want=("sfh_params",) + GRAD_NAMES)
            r.grads = {k: v.cpu().numpy() for k, v in g.items()}
        else:
            m = api.mags(ssp, flt, cosmo, pop, precision="bf16")
        r.mags = m.cpu().numpy()
        lat.append((time.perf_counter() - t0) - t_arr)
    wall = time.perf_counter() - t0
    return latency_summary(reqs, wall, np.array(lat) * 1e3)

"""Serving halo-finding requests on one GPU: continuous batching and the plain loop.

A request is one periodic subvolume (grid n, side L, particles resident in HBM)
and one wavelet scale.  Two ways of serving a stream of requests that arrive
over time are provided:

* ``plain_loop``: first come, first served; one request at a time through the
  single-call native driver, waiting for each to finish.
* ``Server.run``: continuous batching.  Arrived requests wait in a queue; they
  are admitted while everything the server holds on the device (in-flight
  buffer sets, idle pooled sets, per-stream transform workspaces) stays within
  the HBM budget and a slot is free (idle sets of other shapes are evicted,
  least recently used first, to make room); the oldest waiting request's grid size picks the
  next group, which takes every waiting request of that size (up to
  ``max_batch``); each group is enqueued on the next of ``n_streams`` streams
  as one native call (per-box deposits, one batched transform for the group,
  per-box maxima, segmentation and labels), so groups overlap on the device;
  finished groups release their buffers to a per-shape pool and admission
  continues with whatever has arrived meanwhile.

Both modes produce, for every request, exactly the results of the stand-alone
path: the kernels are deterministic and a batched transform computes each job
as it would alone.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import torch

from . import hf


def job_footprint(n: int, np_: int) -> int:
    """Device bytes a request holds while in flight: outputs, its stage
    workspace and its share of the group's batched-transform workspace."""
    cells = n ** 3
    outputs = cells * (8 + 4 + 4) + ((n + 1) // 2) ** 3 * 4 + 8 + max(np_, 1) * 4
    stage_ws = hf.workspace_size(n, 1.0, np_, hf.STAGE_DEPOSIT | hf.STAGE_MAXIMA | hf.STAGE_SEGMENT)
    return outputs + stage_ws + hf.cwt_batch_ws_bytes(n, 1)


@dataclass
class Request:
    job_id: int
    n: int
    box_len: float
    kw: float
    pos: torch.Tensor  # resident [np, 3] positions
    arrival: float     # seconds after the start of the run


@dataclass
class Completion:
    job_id: int
    n: int
    n_particles: int
    arrival: float
    done: float
    outputs: dict | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def set_bytes(bufs: dict) -> int:
    """Device bytes held by one buffer set."""
    return sum(t.numel() * t.element_size() for t in bufs.values())


class BufferPool:
    """Reusable per-request buffers, keyed by (n, number of particles).

    Idle sets are kept for reuse and counted (``idle_bytes``) so that the
    server can charge them against its budget; ``evict`` frees the least
    recently returned ones first."""

    def __init__(self, device):
        self.device = device
        self.free = collections.OrderedDict()  # (n, np) -> list of idle sets, least recently used first
        self.idle_bytes = 0

    def has(self, n: int, np_: int) -> bool:
        return bool(self.free.get((n, np_)))

    def take(self, n: int, np_: int) -> dict:
        lst = self.free.get((n, np_))
        if lst:
            bufs = lst.pop()
            self.idle_bytes -= set_bytes(bufs)
            if not lst:
                del self.free[(n, np_)]
            return bufs
        return hf.job_buffers(n, np_, self.device, with_cwt_ws=False)

    def give(self, n: int, np_: int, bufs: dict):
        key = (n, np_)
        self.free.setdefault(key, []).append(bufs)
        self.free.move_to_end(key)
        self.idle_bytes += set_bytes(bufs)

    def evict(self, need: int, keep: dict) -> int:
        """Free idle sets, least recently used shape first, until ``need``
        bytes are released or none is left, sparing keep[shape] sets of each
        shape in ``keep``; returns the bytes freed."""
        freed = 0
        for key in list(self.free):
            if freed >= need:
                break
            lst = self.free[key]
            spare = keep.get(key, 0)
            while len(lst) > spare and freed < need:
                b = set_bytes(lst.pop(0))
                freed += b
                self.idle_bytes -= b
            if not lst:
                del self.free[key]
        return freed


def _outputs(bufs: dict, np_: int) -> dict:
    cnt = int(bufs["count"].item())
    return {"maxima": bufs["maxima"][:cnt].clone(), "cell_label": bufs["cell_label"].clone(),
            "particle_label": bufs["particle_label"][:np_].clone()}


def _wait_until(t0: float, t: float):
    while True:
        d = t - (time.perf_counter() - t0)
        if d <= 0:
            return
        time.sleep(min(d, 5e-4))


def plain_loop(requests, kernel: str = "sampled", tau: float = 0.0, keep_outputs=frozenset(),
               device: int = 0) -> list:
    """One request at a time, in arrival order, each run to completion."""
    dev = torch.device("cuda", device)
    stream = torch.cuda.current_stream(dev)
    ctx = hf.context(device, stream)
    pool = BufferPool(dev)
    cwt_ws = {}
    done = []
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        _wait_until(t0, r.arrival)
        np_ = r.pos.shape[0]
        bufs = pool.take(r.n, np_)
        ws = cwt_ws.get(r.n)
        if ws is None:
            ws = cwt_ws[r.n] = torch.empty(hf.cwt_batch_ws_bytes(r.n, 1), dtype=torch.uint8, device=dev)
        hf.find_halos_group_async(r.n, [(r.pos, r.box_len, r.kw, bufs)], ws, tau=tau, kernel=kernel, ctx=ctx)
        ctx.sync()
        t = time.perf_counter() - t0
        out = _outputs(bufs, np_) if r.job_id in keep_outputs else None
        done.append(Completion(r.job_id, r.n, np_, r.arrival, t, out))
        pool.give(r.n, np_, bufs)
    return done


@dataclass
class _Group:
    stream_index: int
    n: int
    event: torch.cuda.Event
    members: list = field(default_factory=list)  # (request, bufs)
    cwt_ws: torch.Tensor | None = None
    footprint: int = 0


class Server:
    """Continuous-batching server (see the module docstring)."""

    def __init__(self, device: int = 0, budget_bytes: int = 64 << 30, n_streams: int = 4, max_slots: int = 64,
                 max_batch: int = 16, kernel: str = "sampled", tau: float = 0.0):
        if not 1 <= max_batch <= hf.CWT_BATCH_MAX:
            raise ValueError(f"max_batch must be 1..{hf.CWT_BATCH_MAX}")
        self.dev = torch.device("cuda", device)
        self.device = device
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.max_batch = int(max_batch)
        self.kernel = kernel
        self.tau = tau
        # streams keep the default priority
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(n_streams)]
        self.ctxs = [hf.context(device, s) for s in self.streams]
        self.pool = BufferPool(self.dev)
        self.cwt_ws = {}  # (stream, n, count) -> workspace
        self.stats = {}

    def _cwt_workspace(self, si: int, n: int, count: int) -> torch.Tensor:
        key = (si, n)
        ws = self.cwt_ws.get(key)
        need = hf.cwt_batch_ws_bytes(n, count)
        if ws is None or ws.numel() < need:
            with torch.cuda.stream(self.streams[si]):
                ws = torch.empty(hf.cwt_batch_ws_bytes(n, self.max_batch), dtype=torch.uint8, device=self.dev)
            self.cwt_ws[key] = ws
        return ws

    def _ws_bytes(self) -> int:
        return sum(t.numel() for t in self.cwt_ws.values())

    def _make_room(self, short: int, spare: dict, ws_keep, in_use) -> bool:
        """Release at least ``short`` bytes: idle pooled sets first (sparing
        spare[shape] of each shape), then transform workspaces that no group in
        flight uses (never ``ws_keep``)."""
        freed = self.pool.evict(short, spare)
        for key in list(self.cwt_ws):
            if freed >= short:
                break
            if key == ws_keep or key in in_use:
                continue
            freed += self.cwt_ws.pop(key).numel()
        return freed >= short

    def _resident(self, inflight_sets: int) -> int:
        """Device bytes the server holds: in-flight buffer sets, idle pooled
        sets and the per-stream transform workspaces."""
        return inflight_sets + self.pool.idle_bytes + self._ws_bytes()

    def run(self, requests, keep_outputs=frozenset()) -> list:
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            alone = job_footprint(r.n, r.pos.shape[0]) - hf.cwt_batch_ws_bytes(r.n, 1)
            if alone + hf.cwt_batch_ws_bytes(r.n, self.max_batch) > self.budget:
                raise ValueError(f"request {r.job_id} needs more than the whole budget")
        waiting = collections.deque()
        inflight = []
        busy = [0] * len(self.streams)
        used = 0  # bytes of the in-flight groups' buffer sets
        slots = 0
        nxt = 0
        si_next = 0
        done = []
        groups = 0
        peak = 0
        t0 = time.perf_counter()
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            # retire finished groups
            still = []
            for g in inflight:
                if g.event.query():
                    t = time.perf_counter() - t0
                    for r, bufs in g.members:
                        np_ = r.pos.shape[0]
                        out = _outputs(bufs, np_) if r.job_id in keep_outputs else None
                        done.append(Completion(r.job_id, r.n, np_, r.arrival, t, out))
                        self.pool.give(r.n, np_, bufs)
                    used -= g.footprint
                    slots -= len(g.members)
                    busy[g.stream_index] -= 1
                else:
                    still.append(g)
            inflight = still
            # admit and launch groups while memory and slots allow: everything
            # the server holds (in-flight sets, idle pooled sets, transform
            # workspaces) stays within the budget; idle sets of other shapes are
            # evicted when a new set or workspace needs their room
            launched = False
            while waiting and slots < self.max_slots:
                n = waiting[0].n
                si = min(range(len(self.streams)), key=lambda k: (busy[k], (k - si_next) % len(self.streams)))
                ws_new = 0 if (si, n) in self.cwt_ws else hf.cwt_batch_ws_bytes(n, self.max_batch)
                members, fp, fresh = [], 0, 0
                reuse = collections.Counter()
                for r in waiting:
                    if r.n != n:
                        continue
                    np_ = r.pos.shape[0]
                    f = job_footprint(n, np_) - hf.cwt_batch_ws_bytes(n, 1)  # the buffer set alone
                    pooled = len(self.pool.free.get((n, np_), [])) > reuse[np_]
                    grow = 0 if pooled else f
                    if slots + len(members) >= self.max_slots:
                        break
                    over = self._resident(used) + fresh + grow + ws_new - self.budget
                    if over > 0:
                        spare = {(n, k): c for k, c in reuse.items()}
                        if pooled:
                            spare[(n, np_)] = spare.get((n, np_), 0) + 1
                        if not self._make_room(over, spare, (si, n), {(g.stream_index, g.n) for g in inflight}):
                            break
                    members.append(r)
                    fp += f
                    if pooled:
                        reuse[np_] += 1
                    else:
                        fresh += f
                    if len(members) == self.max_batch:
                        break
                if not members:
                    break
                si_next = (si + 1) % len(self.streams)
                ids = {r.job_id for r in members}
                waiting = collections.deque(r for r in waiting if r.job_id not in ids)
                g = _Group(si, n, torch.cuda.Event())  # footprint: its buffer sets; workspaces are counted apart
                stream = self.streams[si]
                with torch.cuda.stream(stream):
                    entries = []
                    for r in members:
                        bufs = self.pool.take(n, r.pos.shape[0])
                        g.members.append((r, bufs))
                        entries.append((r.pos, r.box_len, r.kw, bufs))
                    fp = sum(set_bytes(b) for _, b in g.members)  # what the sets really hold
                    g.footprint = fp
                    g.cwt_ws = self._cwt_workspace(si, n, len(members))
                    hf.find_halos_group_async(n, entries, g.cwt_ws, tau=self.tau, kernel=self.kernel,
                                              ctx=self.ctxs[si])
                    g.event.record(stream)
                inflight.append(g)
                busy[si] += 1
                used += fp
                peak = max(peak, self._resident(used))
                slots += len(members)
                groups += 1
                launched = True
            if not launched:
                if waiting and not inflight and self._resident(0) == 0:
                    raise RuntimeError("the budget cannot hold the next request")  # unreachable after the check above
                # nothing to start: wait a little for a completion or an arrival
                time.sleep(5e-5)
        for c in self.ctxs:
            c.sync()
        self.stats = {"groups": groups, "mean_group": len(reqs) / max(groups, 1), "peak_resident": peak}
        return done


def summarize(done: list) -> dict:
    """Throughput and latency percentiles of a completed run."""
    if not done:
        return {}
    lat = torch.tensor(sorted(c.latency for c in done), dtype=torch.float64)
    first = min(c.arrival for c in done)
    last = max(c.done for c in done)
    span = max(last - first, 1e-9)
    particles = sum(c.n_particles for c in done)

    def pct(q):
        return float(torch.quantile(lat, q).item())

    return {"jobs": len(done), "makespan_s": span, "jobs_per_s": len(done) / span,
            "particles_per_s": particles / span, "p50_ms": 1e3 * pct(0.5), "p99_ms": 1e3 * pct(0.99),
            "mean_ms": 1e3 * float(lat.mean().item())}

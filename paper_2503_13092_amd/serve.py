"""Continuous-batching request loop for event processing.

Events arrive as an open-loop process (arrival times fixed in advance, so a
slow server cannot slow the arrivals down).  The loop admits arrived events in
arrival order into the next free *slot* — a set of device buffers of fixed
capacity with its own stream — as soon as one is free, so events that arrive
while earlier batches are still on the GPU are batched together and their
work overlaps with those batches.  An event is admitted into a batch only if
the batch still has room for its seeds and hits (memory admission).  Latency
is completion time minus *scheduled* arrival time.

Results of an event do not depend on the batch it ran in: every step of the
path is per event, and the kernels are deterministic.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import ds


@dataclasses.dataclass
class BatchResult:
    """Host copies of one batch's outputs; seed and hit indices are per event."""
    e0: int
    n_events: int
    seed_off: np.ndarray       # [n+1], rebased to 0
    nhits: np.ndarray
    hits: np.ndarray           # [S, 4]
    score: np.ndarray
    state: np.ndarray          # [S, 6]: x, y, tx, ty, qop, chi2
    vcount: np.ndarray         # [n]
    vertices: np.ndarray       # [n, cap, 6]: i, j, x, y, z, doca (i, j as float)

    def event(self, k: int) -> Dict:
        a, b = int(self.seed_off[k]), int(self.seed_off[k + 1])
        c = int(self.vcount[k])
        return dict(nhits=self.nhits[a:b], hits=self.hits[a:b], score=self.score[a:b], state=self.state[a:b],
                    vertices=self.vertices[k, :c])


class EventPool:
    """A fixed set of events served in a cycle (arrival k is event k % size)."""

    def __init__(self, batch):
        self.batch = batch
        self.size = batch.n_events
        self.seeds_per_event = np.diff(batch.seed_off).astype(np.int64)
        self.hits_per_event = (batch.hit_off[4::4] - batch.hit_off[0:-1:4]).astype(np.int64)


class GpuBackend:
    """Slots of device buffers on their own streams; the whole pool is kept in
    pinned host memory, so a batch is one asynchronous copy per array."""

    def __init__(self, pool: EventPool, geometry: Dict, weights, n_slots: int = 3, max_events: int = 512,
                 mode: int = ds.DS_MODE_PERSISTENT, vertex_cap: int = 64, device: int = 0):
        import torch
        self.torch = torch
        self.pool = pool
        self.n_slots = n_slots
        self.max_events = max_events
        self.mode = mode
        self.cap = vertex_cap
        b = pool.batch
        self.max_seeds_per_event = int(pool.seeds_per_event.max())
        self.max_hits_per_event = int(pool.hits_per_event.max())
        # capacity per slot: max_events events of the largest kind would be wasteful;
        # size for max_events events at twice the mean occupancy, admit by actual size
        self.max_seeds = int(max(2 * pool.seeds_per_event.mean() * max_events, self.max_seeds_per_event))
        self.max_hits = int(max(2 * pool.hits_per_event.mean() * max_events, self.max_hits_per_event))
        self.ctx = ds.Context(device, geometry, weights)
        # the autotuner's launch settings for this pool's workload, when it has some
        from . import autotune
        self.tuned = autotune.apply_cached(self.ctx.handle, pool.batch, int(geometry.get("algorithm", 0)))
        pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
        self.h_seed = [pin(getattr(b, k)) for k in ("sx", "sy", "stx", "sty", "sqop")]
        self.h_hu = pin(b.hu)
        self.seed_off = b.seed_off.astype(np.int64)
        self.hit_off = b.hit_off.astype(np.int64)
        dev = torch.device("cuda", device)
        self.slots = []
        for _ in range(n_slots):
            s = dict(stream=torch.cuda.Stream(device=dev))
            s["off_h"] = torch.zeros(max_events + 1 + 4 * max_events + 1, dtype=torch.int32).pin_memory()
            s["seed_off"] = torch.zeros(max_events + 1, dtype=torch.int32, device=dev)
            s["hit_off"] = torch.zeros(4 * max_events + 1, dtype=torch.int32, device=dev)
            s["seed"] = [torch.zeros(self.max_seeds, dtype=torch.float32, device=dev) for _ in range(5)]
            s["hu"] = torch.zeros(self.max_hits, dtype=torch.float32, device=dev)
            s["tracks"] = ds.DeviceTracks(self.max_seeds, device=dev, with_cand=False)
            s["vtx"] = ds.DeviceVertices(max_events, vertex_cap, device=dev)
            s["out_i"] = torch.zeros((6, self.max_seeds), dtype=torch.int32).pin_memory()     # nhits, h0..h3, pad
            s["out_f"] = torch.zeros((7, self.max_seeds), dtype=torch.float32).pin_memory()   # score, x..chi2
            s["out_vc"] = torch.zeros(max_events, dtype=torch.int32).pin_memory()
            s["out_vi"] = torch.zeros((2, max_events * vertex_cap), dtype=torch.int32).pin_memory()
            s["out_vf"] = torch.zeros((4, max_events * vertex_cap), dtype=torch.float32).pin_memory()
            s["done"] = torch.cuda.Event()
            s["busy"] = None
            self.slots.append(s)

    def fits(self, n_events: int, n_seeds: int, n_hits: int) -> bool:
        return n_events <= self.max_events and n_seeds <= self.max_seeds and n_hits <= self.max_hits

    def submit(self, slot: int, e0: int, e1: int) -> None:
        torch = self.torch
        s = self.slots[slot]
        n = e1 - e0
        sa, sb = int(self.seed_off[e0]), int(self.seed_off[e1])
        ha, hb = int(self.hit_off[4 * e0]), int(self.hit_off[4 * e1])
        offs = s["off_h"].numpy()
        offs[:n + 1] = self.seed_off[e0:e1 + 1] - sa
        offs[n + 1:n + 1 + 4 * n + 1] = self.hit_off[4 * e0:4 * e1 + 1] - ha
        with torch.cuda.stream(s["stream"]):
            s["seed_off"][:n + 1].copy_(s["off_h"][:n + 1], non_blocking=True)
            s["hit_off"][:4 * n + 1].copy_(s["off_h"][n + 1:n + 1 + 4 * n + 1], non_blocking=True)
            for k in range(5):
                s["seed"][k][:sb - sa].copy_(self.h_seed[k][sa:sb], non_blocking=True)
            s["hu"][:hb - ha].copy_(self.h_hu[ha:hb], non_blocking=True)
            ev = ds.DsEvents()
            ev.n_events, ev.n_seeds, ev.n_hits = n, sb - sa, hb - ha
            ev.max_seeds_per_event, ev.max_hits_per_event = self.max_seeds_per_event, self.max_hits_per_event
            ev.seed_off, ev.hit_off = s["seed_off"].data_ptr(), s["hit_off"].data_ptr()
            ev.sx, ev.sy, ev.stx, ev.sty, ev.sqop = (t.data_ptr() for t in s["seed"])
            ev.hu = s["hu"].data_ptr()
            holder = type("E", (), {})()
            holder.struct = ev
            tr, vt = s["tracks"], s["vtx"]
            ds.ds_process(self.ctx.handle, holder, tr, vt, self.mode, stream=s["stream"])
            S = sb - sa
            s["out_i"][0, :S].copy_(tr.nhits[:S], non_blocking=True)
            for L in range(4):
                s["out_i"][1 + L, :S].copy_(tr.hits[L, :S], non_blocking=True)
            for k, name in enumerate(("score", "x", "y", "tx", "ty", "qop", "chi2")):
                s["out_f"][k, :S].copy_(getattr(tr, name)[:S], non_blocking=True)
            s["out_vc"][:n].copy_(vt.count[:n], non_blocking=True)
            m = n * self.cap
            s["out_vi"][0, :m].copy_(vt.i[:m], non_blocking=True)
            s["out_vi"][1, :m].copy_(vt.j[:m], non_blocking=True)
            for k, name in enumerate(("x", "y", "z", "doca")):
                s["out_vf"][k, :m].copy_(getattr(vt, name)[:m], non_blocking=True)
            s["done"].record(s["stream"])
        s["busy"] = (e0, e1, sa, sb)

    def done(self, slot: int) -> bool:
        return self.slots[slot]["done"].query()

    def fetch(self, slot: int) -> BatchResult:
        s = self.slots[slot]
        e0, e1, sa, sb = s["busy"]
        n, S = e1 - e0, sb - sa
        oi, of = s["out_i"].numpy(), s["out_f"].numpy()
        vi, vf = s["out_vi"].numpy(), s["out_vf"].numpy()
        cap = self.cap
        verts = np.concatenate([vi[:, :n * cap].T.astype(np.float64), vf[:, :n * cap].T.astype(np.float64)],
                               axis=1).reshape(n, cap, 6)
        res = BatchResult(e0, n, self.seed_off[e0:e1 + 1] - sa, oi[0, :S].copy(), oi[1:5, :S].T.copy(),
                          of[0, :S].copy(), of[1:7, :S].T.copy(), s["out_vc"].numpy()[:n].copy(), verts)
        s["busy"] = None
        return res

    def close(self):
        self.torch.cuda.synchronize()
        self.ctx.close()


@dataclasses.dataclass
class ServeStats:
    rate: float
    n: int
    duration_s: float
    sustained: float
    p50_ms: float
    p99_ms: float
    p999_ms: float
    mean_batch: float
    max_in_flight: int
    rejected: int = 0
    offered: int = 0       # arrivals scheduled before the loop ended
    completed: int = 0     # events whose results came back (rejected ones excluded)
    censored: int = 0      # offered, admitted or queued, not finished when the loop ended
    saturated: bool = False  # censored > 0: the percentiles are lower bounds

    def as_dict(self):
        return dataclasses.asdict(self)


def poisson_arrivals(rate: float, n: int, seed: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


class Server:
    """Continuous batching over a backend's slots (single host thread)."""

    def __init__(self, backend, pool: EventPool, max_batch: Optional[int] = None):
        self.be = backend
        self.pool = pool
        self.max_batch = max_batch or backend.max_events

    def _take(self, head: int, tail: int) -> int:
        """Largest e1 <= tail such that events [head, e1) fit one slot and do
        not wrap the pool; head itself if the first event can never fit."""
        P = self.pool.size
        e0 = head % P
        n = min(tail - head, self.max_batch, P - e0)
        seeds = np.cumsum(self.pool.seeds_per_event[e0:e0 + n])
        hits = np.cumsum(self.pool.hits_per_event[e0:e0 + n])
        ok = (seeds <= self.be.max_seeds) & (hits <= self.be.max_hits)
        k = int(np.argmin(ok)) if not ok.all() else n
        return head + k

    def run(self, arrivals: np.ndarray, on_result=None, warmup_frac: float = 0.1, time_limit_s: float = 60.0):
        """Serve arrivals (seconds from start).  Returns (latencies_s, stats)."""
        N = len(arrivals)
        lat = np.full(N, np.nan)
        is_rej = np.zeros(N, bool)
        free = list(range(self.be.n_slots))
        busy = {}
        head = 0           # first event not yet submitted
        arrived = 0
        done_n = 0         # finished or rejected: the loop ends when every arrival is one of them
        completed = 0
        batches = []
        max_if = 0
        rejected = 0
        t0 = time.perf_counter()
        while done_n < N:
            now = time.perf_counter() - t0
            if now > time_limit_s:
                break
            while arrived < N and arrivals[arrived] <= now:
                arrived += 1
            for slot in list(busy):
                if self.be.done(slot):
                    t = time.perf_counter() - t0
                    a0, a1 = busy.pop(slot)
                    res = self.be.fetch(slot)
                    lat[a0:a1] = t - arrivals[a0:a1]
                    done_n += a1 - a0
                    completed += a1 - a0
                    free.append(slot)
                    if on_result is not None:
                        on_result(a0, a1, res)
            while free and head < arrived:
                e1 = self._take(head, arrived)
                if e1 == head:
                    # larger than a slot: rejected at admission
                    rejected += 1
                    is_rej[head] = True
                    done_n += 1
                    head += 1
                    continue
                slot = free.pop(0)
                P = self.pool.size
                self.be.submit(slot, head % P, head % P + (e1 - head))
                busy[slot] = (head, e1)
                batches.append(e1 - head)
                head = e1
            max_if = max(max_if, len(busy))
            if not busy and head >= arrived and arrived < N:
                # idle until the next arrival
                dt = arrivals[arrived] - (time.perf_counter() - t0)
                if dt > 2e-4:
                    time.sleep(dt - 1e-4)
        dur = time.perf_counter() - t0
        # events offered before the end but not finished: their latency is at
        # least (end - arrival); counted that way, so a saturated server's
        # percentiles are lower bounds rather than taken over the survivors
        offered = arrivals <= dur
        unfinished = offered & ~np.isfinite(lat) & ~is_rej
        L_all = np.where(unfinished, dur - arrivals, lat)
        k0 = int(warmup_frac * N)
        sel = offered[k0:] & ~is_rej[k0:]
        L = L_all[k0:][sel]
        rate = N / arrivals[-1] if N else 0.0
        stats = ServeStats(rate=rate, n=len(L), duration_s=dur, sustained=completed / dur if dur > 0 else 0.0,
                           p50_ms=float(np.percentile(L, 50) * 1e3) if len(L) else math.nan,
                           p99_ms=float(np.percentile(L, 99) * 1e3) if len(L) else math.nan,
                           p999_ms=float(np.percentile(L, 99.9) * 1e3) if len(L) else math.nan,
                           mean_batch=float(np.mean(batches)) if batches else 0.0, max_in_flight=max_if,
                           rejected=rejected, offered=int(offered.sum()), completed=completed,
                           censored=int(unfinished.sum()), saturated=bool(unfinished.any()))
        return lat, stats

"""Continuous-batching serving loop for the FFP on one GPU.

Requests are whole graphs (an edge list with N, tau, K, d, seed and storage
type) arriving over time, as in the paper's streaming setting (Sec. II,
Algorithm 2) generalised to a stream of independent graphs.  The loop

  * admits waiting requests in arrival order while a slot is free and the
    request's HBM footprint fits the memory budget: while its graph is being
    built, the resident footprint plus the build's transient buffers; once
    built, the resident footprint alone (a request that does not fit waits;
    nothing is rejected for lack of room unless it could never fit);
  * builds admitted graphs on a side stream from a worker thread, so graph
    construction overlaps the hops of graphs already running;
  * starts a graph's job at the next hop boundary once its build is done;
  * advances every running job by one hop per iteration, all graphs of one
    (storage, width, gather depth) class in one kernel launch (ifgp_job_step);
  * retires a job when its output is complete on the device, frees its slot
    and memory, and records its latency (completion - arrival);
  * a request whose build or job start fails (IfgpError, e.g. out of device
    memory or an id out of range) is recorded as failed with its message, its
    slot and memory are released, and the loop goes on with the others.

`sequential()` is the plain one-at-a-time path the batched loop is compared
with: build, embed, synchronise, next.

All device work runs in libifgp's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time
from typing import Callable, Optional

import numpy as np

from . import _lib as ifgp


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    src: np.ndarray
    dst: np.ndarray
    N: int
    tau: float = -1.0
    K: int = 8
    d: int = 64
    seed: int = 0
    storage: str = "bf16"
    # filled in by the server
    out: object = None             # torch tensor N x d on the GPU
    t_admit: float = float("nan")
    t_start: float = float("nan")
    t_done: float = float("nan")
    cancelled: bool = False
    error: Optional[str] = None     # set if the request failed

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival

    def footprint(self) -> int:
        """Resident device bytes while the request is served: graph, scales,
        features, statistics (ifgp_footprint_bytes with nnz <= 2E) and the
        FP32 output."""
        nnz = 2 * int(self.src.shape[0])
        return ifgp.footprint_bytes(self.N, max(nnz, 0), self.d, self.storage) + 4 * self.N * self.d

    def build_transient(self) -> int:
        """Device bytes a graph build holds on top of the resident graph until
        it returns, bounded from above: host edges staged on the device (16 per
        pair), two 64-bit keys per pair and as many for the sort's second
        buffer (32), a column index per key (8), per-tile digit counts and
        bucket bounds (under 8), and per-node sort keys and counters (32 N)."""
        return 64 * int(self.src.shape[0]) + 32 * self.N


class Admission:
    """FIFO admission by free slots and memory budget (host logic only)."""

    def __init__(self, max_slots: int, budget_bytes: int):
        if max_slots < 1 or budget_bytes <= 0:
            raise ValueError("need at least one slot and a positive budget")
        self.max_slots = max_slots
        self.budget = budget_bytes
        self.used = 0
        self.slots = 0
        self.queue: collections.deque = collections.deque()
        self.rejected: list = []

    def offer(self, req, cost: int):
        if cost > self.budget:
            self.rejected.append(req)     # can never fit
        else:
            self.queue.append((req, cost))

    def cancel(self, rid: int) -> bool:
        for i, (r, _) in enumerate(self.queue):
            if r.rid == rid:
                del self.queue[i]
                r.cancelled = True
                return True
        return False

    def admit(self):
        """Pop requests from the head while they fit; strict FIFO (a large
        request at the head is not overtaken)."""
        out = []
        while self.queue and self.slots < self.max_slots:
            r, cost = self.queue[0]
            if self.used + cost > self.budget:
                break
            self.queue.popleft()
            self.used += cost
            self.slots += 1
            out.append((r, cost))
        return out

    def shrink(self, nbytes: int):
        """Part of an admitted request's memory is no longer needed (its slot
        stays taken)."""
        self.used -= nbytes

    def release(self, cost: int):
        self.used -= cost
        self.slots -= 1


class Server:
    def __init__(self, max_slots: int = 64, budget_bytes: Optional[int] = None,
                 build_workers: int = 4, clock: Callable[[], float] = time.perf_counter):
        import threading
        import torch
        self.torch = torch
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.5)
        self.adm = Admission(max_slots, budget_bytes)
        self.clock = clock
        self.main = torch.cuda.current_stream()
        self._tls = threading.local()            # one side stream per build worker
        self.pool = cf.ThreadPoolExecutor(max_workers=max(1, build_workers))
        self.failed: list = []                   # requests whose build or job start failed
        # Library buffers come from the library's own caching allocator: build
        # worker threads then never call back into Python for memory.
        ifgp.use_hip_allocator()

    def _side(self):
        s = getattr(self._tls, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream()        # default priority
            self._tls.stream = s
        return s

    def _build(self, req: Request):
        side = self._side()
        G = ifgp.Graph(req.src, req.dst, req.N, stream=side)
        ev = self.torch.cuda.Event()
        ev.record(side)
        return G, ev

    def run(self, requests, on_done: Optional[Callable[[Request], None]] = None,
            keep_outputs: bool = True, max_seconds: float = 600.0,
            progress: Optional[Callable[[str], None]] = None):
        """Serve `requests` (arrival times relative to the call) to completion;
        returns the completed requests in completion order.  With
        keep_outputs=False each output is released once complete.  Raises
        TimeoutError after max_seconds; `progress` receives a status line
        about once a second."""
        import sys
        total = len(requests)
        next_report = 1.0
        # Build workers need the GIL around each library call; a short switch
        # interval keeps them from waiting on the scheduling loop.
        old_interval = sys.getswitchinterval()
        sys.setswitchinterval(1e-4)
        try:
            return self._run(requests, on_done, keep_outputs, max_seconds, progress, total,
                             next_report)
        finally:
            sys.setswitchinterval(old_interval)

    def _run(self, requests, on_done, keep_outputs, max_seconds, progress, total, next_report):
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        building = []     # (req, cost, future)
        active = []       # (req, cost, graph)
        finishing = []    # (req, cost, graph, event)
        done = []
        t0 = self.clock()
        while pending or self.adm.queue or building or active or finishing:
            moved = False
            now = self.clock() - t0
            if now > max_seconds:
                raise TimeoutError(f"serving did not finish in {max_seconds} s "
                                   f"({len(done)}/{total} done)")
            if progress and now >= next_report:
                progress(f"serve t={now:.1f}s done={len(done)}/{total} active={len(active)} "
                         f"building={len(building)} queued={len(self.adm.queue)}")
                next_report = now + 1.0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                self.adm.offer(r, r.footprint() + r.build_transient())
            for r, cost in self.adm.admit():
                r.t_admit = self.clock() - t0
                building.append((r, cost, self.pool.submit(self._build, r)))
                moved = True
            still = []
            for r, cost, fut in building:
                if fut.done():
                    moved = True
                    transient = r.build_transient()
                    G = None
                    try:
                        G, ev = fut.result()
                        self.adm.shrink(transient)
                        cost -= transient
                        self.main.wait_event(ev)
                        r.out = G.job_begin(r.tau, r.K, r.d, r.seed, stream=self.main,
                                            storage=r.storage)
                    except ifgp.IfgpError as e:
                        self._fail(r, cost, G, e, t0)
                        continue
                    r.t_start = self.clock() - t0
                    active.append((r, cost, G))
                else:
                    still.append((r, cost, fut))
            building = still
            if active:
                moved = True
                flags = ifgp.job_step([G for _, _, G in active], stream=self.main)
                keep = []
                for (r, cost, G), f in zip(active, flags):
                    if f:
                        ev = torch.cuda.Event()
                        ev.record(self.main)
                        finishing.append((r, cost, G, ev))
                    else:
                        keep.append((r, cost, G))
                active = keep
            still = []
            for r, cost, G, ev in finishing:
                if ev.query():
                    moved = True
                    r.t_done = self.clock() - t0
                    G.destroy()
                    self.adm.release(cost)
                    done.append(r)
                    if on_done:
                        on_done(r)
                    if not keep_outputs:
                        r.out = None
                else:
                    still.append((r, cost, G, ev))
            finishing = still
            if not moved:
                time.sleep(5e-5)     # nothing to launch: let the build workers run
            if not active and not finishing and not self.adm.queue:
                # idle: wait for a build or the next arrival
                if building:
                    cf.wait([f for _, _, f in building], timeout=0.001,
                            return_when=cf.FIRST_COMPLETED)
                elif pending:
                    dt = pending[0].arrival - (self.clock() - t0)
                    if dt > 0:
                        time.sleep(min(dt, 0.001))
        return done

    def _fail(self, r, cost, G, err, t0):
        """Record a failed request and give back its slot and memory."""
        if G is not None:
            G.destroy()
        self.adm.release(cost)
        r.error = str(err)
        r.out = None
        r.t_done = self.clock() - t0
        self.failed.append(r)

    def close(self):
        self.pool.shutdown(wait=True)


def sequential(requests, storage: str = "f32", clock: Callable[[], float] = time.perf_counter,
               keep_outputs: bool = True):
    """Plain one-at-a-time path: each request is built, embedded with
    `storage` features and synchronised before the next one starts."""
    import torch
    t0 = clock()
    done = []
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        now = clock() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.t_admit = r.t_start = clock() - t0
        G = ifgp.Graph(r.src, r.dst, r.N)
        r.out = G.embed(r.tau, r.K, r.d, r.seed, storage=storage)
        torch.cuda.synchronize()
        r.t_done = clock() - t0
        G.destroy()
        if not keep_outputs:
            r.out = None
        done.append(r)
    return done


def summarize(done):
    """graphs/s over the run and latency percentiles (ms)."""
    if not done:
        return {"graphs": 0}
    lat = np.array([r.latency for r in done]) * 1e3
    t_end = max(r.t_done for r in done)
    t_beg = min(r.arrival for r in done)
    return {"graphs": len(done), "graphs_per_s": len(done) / max(t_end - t_beg, 1e-9),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "makespan_s": float(t_end - t_beg)}

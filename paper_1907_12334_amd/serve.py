"""Request loop for MSG sample requests: HBM-budget admission and continuous
batching over several HIP streams.

A request is one Monte Carlo sample of the multi-index method (Section 3):
a seeded coefficient field and a finest index (P, Q); its answer is the
quantity of interest Q and the mixed difference Delta Q on every grid of its
rectangle, computed by the library's batched full-MSG solve.

Scheduling:
  * requests wait in one of two FIFO lanes by size (estimated W-cycle
    cell-visits), so that a few very large requests do not hold back the
    stream of small ones;
  * each lane has its own worker threads; a worker owns a library handle and
    a HIP stream (default priority) and, whenever it is free, takes the
    waiting requests of its lane in arrival order into one ragged batch, up to
    a request count, a work cap and the free HBM budget;
  * the budget (a fraction of the free device memory at start) is split into
    one device arena per worker, allocated once when the engine starts; a
    batch's buffers (fields, solutions, outputs, solver workspace) are views
    into its worker's arena, so serving allocates no device memory per
    batch.  Each request reserves its exact footprint from the budget until
    its batch completes, and a worker takes requests while their footprints
    fit its arena, so a request that arrives while other batches are on the
    device is admitted as soon as a worker is free, and its batch runs
    concurrently with theirs on another stream;
  * the standard normals of a request's field are drawn on the device from
    its stream (engine seed, sample id); fields, iterates and solutions stay
    on the device during a solve; only Q, Delta Q, status and cycle counts
    (and u on request) come back.

The library calls release the interpreter lock, so workers overlap on the
device.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import inputs as I
from . import msg


@dataclasses.dataclass
class Request:
    rid: int
    sample_id: int
    P: int
    Q: int
    t_arrival: float = 0.0           # seconds on the engine clock
    want_u: bool = False
    t_admit: float = float("nan")
    t_done: float = float("nan")
    batch_size: int = 0
    lane: str = ""
    q: Optional[np.ndarray] = None
    dq: Optional[np.ndarray] = None
    u: Optional[np.ndarray] = None
    status: int = -1
    cycles: Optional[np.ndarray] = None
    error: Optional[str] = None
    done: threading.Event = dataclasses.field(default_factory=threading.Event, repr=False)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


BIG_TAIL_LDS = 150 * 1024     # LDS bytes per problem of the large-request lane's tails
SMALL_TAIL_LDS = 100 * 1024   # ... and of the small-request lane's (unless the options set one)


def work_estimate(c: int, P: int, Q: int) -> float:
    """Cell-visits of one W-cycle over the rectangle (P, Q): every level of
    the cycle costs about one finest grid, and there are (P+1)(Q+1) grids."""
    return float((P + 1) * (Q + 1)) * (c << P) * (c << Q)


class Footprints:
    """Device bytes of one request, cached per (P, Q)."""

    def __init__(self, c: int, opts: msg.SolveOpts, mixed_fields: bool):
        self.c, self.opts, self.mixed = c, opts, mixed_fields
        self._cache: Dict[tuple, int] = {}

    def __call__(self, P: int, Q: int) -> int:
        key = (P, Q)
        if key not in self._cache:
            b = msg.Batch(self.c, [P], [Q])
            lay = b.layout()
            cells, xf, yf, grids = (int(lay[k][-1]) for k in ("cell", "xface", "yface", "grid"))
            field = (8 + (4 if self.mixed else 0)) * (xf + yf)
            outs = 8 * cells + grids * (8 + 8 + 4) + 4
            # the larger of the two lanes' plans (the large-request lane's
            # wider tails need larger tail images)
            ws = max(msg.workspace_size(b, self.opts),
                     msg.workspace_size(b, dataclasses.replace(self.opts, tail_budget=BIG_TAIL_LDS)))
            self._cache[key] = field + outs + ws + 4096
        return self._cache[key]


class Admission:
    """Lanes, FIFO order and the HBM budget (no device work; thread-safe).

    footprint(P, Q) -> bytes and work(P, Q) -> W-cycle cell-visits are
    supplied by the caller."""

    def __init__(self, budget: int, footprint, work, max_batch: int = 4096, max_batch_work: float = 6e9,
                 big_work: float = 1e6):
        self.budget = int(budget)
        self.footprint, self.work = footprint, work
        self.max_batch, self.max_batch_work, self.big_work = max_batch, max_batch_work, big_work
        self.reserved = 0
        self.lanes = {"small": collections.deque(), "big": collections.deque()}
        self.cv = threading.Condition()
        self.stopping = False

    def lane_of(self, P: int, Q: int) -> str:
        return "big" if self.work(P, Q) >= self.big_work else "small"

    def submit(self, req: Request) -> Request:
        if self.footprint(req.P, req.Q) > self.budget:
            raise ValueError(f"request ({req.P},{req.Q}) needs more than the whole HBM budget")
        with self.cv:
            if self.stopping:
                raise RuntimeError("engine is stopping")
            self.lanes[self.lane_of(req.P, req.Q)].append(req)
            self.cv.notify_all()
        return req

    def take(self, lane: str, cap: Optional[int] = None):
        """Pop the next batch of `lane` without waiting: arrival order, up to
        max_batch requests and the work cap, while the budget (and the
        worker's capacity `cap`, if given) allows.  Returns (requests, reserved
        bytes); ([], 0) if the head does not fit yet."""
        with self.cv:
            q = self.lanes[lane]
            batch, work, need = [], 0.0, 0
            while q and len(batch) < self.max_batch:
                r = q[0]
                b = self.footprint(r.P, r.Q)
                w = self.work(r.P, r.Q)
                if batch and work + w > self.max_batch_work:
                    break
                if self.reserved + need + b > self.budget or (cap is not None and need + b > cap):
                    break
                q.popleft()
                batch.append(r)
                work += w
                need += b
            self.reserved += need
            return batch, need

    def wait_batch(self, lane: str, cap: Optional[int] = None):
        """Block until a batch of `lane` can start; None once stopping and empty."""
        with self.cv:
            while True:
                if self.stopping and not self.lanes[lane]:
                    return None
                if self.lanes[lane]:
                    batch, need = self.take(lane, cap)
                    if batch:
                        return batch, need
                self.cv.wait(timeout=0.05)

    def release(self, need: int):
        with self.cv:
            self.reserved -= need
            self.cv.notify_all()

    def stop(self):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()


class Engine:
    """Continuous-batching request loop on one GPU (see the module notes)."""

    def __init__(self, field: I.FieldSpec, c: int, opts: msg.SolveOpts, device: int = 0,
                 budget_bytes: Optional[int] = None, budget_fraction: float = 0.8,
                 workers: int = 3, big_workers: int = 1, max_batch: int = 4096,
                 max_batch_work: float = 6e9, big_work: float = 1e6, seed: int = I.BASE_SEED + 5):
        import torch
        self.torch = torch
        # the workers are the concurrency: each batch stays on its worker's
        # stream (more streams than hardware queues serialise the batches)
        opts = dataclasses.replace(opts, overlap=0)
        # batches of small requests hold few problems per class: deep on-chip
        # tails save host level visits there too
        if not opts.tail_budget:
            opts = dataclasses.replace(opts, tail_budget=SMALL_TAIL_LDS)
        self.field, self.c, self.opts, self.device, self.seed = field, c, opts, device, seed
        self.dev = torch.device(f"cuda:{device}")
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            budget_bytes = int(free * budget_fraction)
        self.foot = Footprints(c, opts, opts.precision == msg.MIXED)
        self.adm = Admission(budget_bytes, self.foot, lambda P, Q: work_estimate(c, P, Q), max_batch,
                             max_batch_work, big_work)
        # one arena per worker, carved once: a share of the budget each
        n_workers = workers + big_workers
        self.arena_bytes = budget_bytes // n_workers // 256 * 256
        self.arenas = [torch.empty(self.arena_bytes, dtype=torch.uint8, device=self.dev) for _ in range(n_workers)]
        self.t0 = time.perf_counter()
        self.batches: List[dict] = []
        self.lock = threading.Lock()
        self.inflight = 0
        self.max_inflight = 0
        lanes = ["small"] * workers + ["big"] * big_workers
        self.threads = [threading.Thread(target=self._worker, args=(lane, self.arenas[k]), daemon=True)
                        for k, lane in enumerate(lanes)]
        for t in self.threads:
            t.start()

    # ---------------------------------------------------------------- client side
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> Request:
        if self.foot(req.P, req.Q) > self.arena_bytes - self.arena_bytes // 16:
            raise ValueError(f"request ({req.P},{req.Q}) needs more than a worker's arena")
        return self.adm.submit(req)

    def close(self):
        self.adm.stop()
        for t in self.threads:
            t.join()
        self.arenas = []

    def _worker(self, lane: str, arena):
        torch = self.torch
        # large requests come in batches of a few samples: their tails take a
        # CU's worth of LDS each (deeper on-chip tails, fewer launches)
        opts = dataclasses.replace(self.opts, tail_budget=BIG_TAIL_LDS) if lane == "big" else self.opts
        torch.cuda.set_device(self.dev)
        handle = msg.Handle(self.device)
        stream = torch.cuda.Stream(device=self.dev)      # default priority
        # footprints are estimates from single requests: keep 1/16 of the
        # arena for what a batch needs beyond their sum
        cap = self.arena_bytes - self.arena_bytes // 16
        try:
            while True:
                got = self.adm.wait_batch(lane, cap)
                if got is None:
                    return
                batch, need = got
                with self.lock:
                    self.inflight += 1
                    self.max_inflight = max(self.max_inflight, self.inflight)
                t_admit = self.now()
                for r in batch:
                    r.t_admit = t_admit
                try:
                    self._run(handle, stream, batch, arena, opts)
                except Exception as e:                  # report per request, keep serving
                    for r in batch:
                        r.error = f"{type(e).__name__}: {e}"
                t_done = self.now()
                self.adm.release(need)
                with self.lock:
                    self.inflight -= 1
                    self.batches.append({"lane": lane, "size": len(batch), "t_admit": t_admit, "t_done": t_done,
                                         "work": float(sum(work_estimate(self.c, r.P, r.Q) for r in batch))})
                for r in batch:
                    r.t_done = t_done
                    r.batch_size = len(batch)
                    r.lane = lane
                    r.done.set()
        finally:
            handle.close()

    def _run(self, handle: msg.Handle, stream, reqs: Sequence[Request], arena, opts: msg.SolveOpts):
        torch = self.torch
        P = [r.P for r in reqs]
        Q = [r.Q for r in reqs]
        batch = msg.Batch(self.c, P, Q)
        ids = np.array([r.sample_id for r in reqs], dtype=np.int64)
        with torch.cuda.stream(stream):
            bufs = msg.Buffers(batch, opts, arena=arena)
            msg.run(handle, self.field, batch, opts, None, bufs, stream=stream, seed=self.seed, sample_id=ids)
            q = bufs.q.cpu().numpy()
            dq = bufs.dq.cpu().numpy()
            st = bufs.status.cpu().numpy()
            cyc = bufs.cycles.cpu().numpy()
            want_u = any(r.want_u for r in reqs)
            u = bufs.u.cpu().numpy() if want_u else None
        lay = bufs.layout
        for k, r in enumerate(reqs):
            g0, g1 = int(lay["grid"][k]), int(lay["grid"][k + 1])
            r.q, r.dq, r.cycles, r.status = q[g0:g1].copy(), dq[g0:g1].copy(), cyc[g0:g1].copy(), int(st[k])
            if r.want_u:
                r.u = u[int(lay["cell"][k]):int(lay["cell"][k + 1])].copy()


def replay(engine: Engine, t_arrival: Sequence[float], P: Sequence[int], Q: Sequence[int],
           sample_ids: Sequence[int], want_u: bool = False, timeout: float = 600.0) -> List[Request]:
    """Submit requests at their arrival times (seconds from now) and wait for
    all of them."""
    start = engine.now()
    reqs = []
    for k in range(len(P)):
        due = start + float(t_arrival[k])
        while True:
            dt = due - engine.now()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.01))
        r = Request(rid=k, sample_id=int(sample_ids[k]), P=int(P[k]), Q=int(Q[k]), t_arrival=engine.now(),
                    want_u=want_u)
        reqs.append(engine.submit(r))
    deadline = time.perf_counter() + timeout
    for r in reqs:
        if not r.done.wait(max(0.0, deadline - time.perf_counter())):
            raise TimeoutError(f"request {r.rid} ({r.P},{r.Q}) not served within {timeout} s")
    return reqs


def summarize(reqs: Sequence[Request], offered_rate: Optional[float] = None) -> dict:
    """Throughput over first arrival .. last completion, latency percentiles,
    and whether the loop kept up: `drain_s` is how long the last answers came
    after the last arrival; the load saturates the loop when that backlog is
    more than a quarter of the arrival window."""
    lat = np.array([r.latency for r in reqs])
    t_first = min(r.t_arrival for r in reqs)
    t_last = max(r.t_done for r in reqs)
    t_arr = max(r.t_arrival for r in reqs)
    span = t_last - t_first
    out = {
        "requests": len(reqs),
        "samples_per_s": round(len(reqs) / span, 2) if span > 0 else None,
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
        "mean_batch": round(float(np.mean([r.batch_size for r in reqs])), 1),
        "converged": int(sum(r.status == 0 for r in reqs)),
        "errors": int(sum(r.error is not None for r in reqs)),
        "span_s": round(span, 3),
    }
    for lane in ("small", "big"):
        lt = np.array([r.latency for r in reqs if r.lane == lane])
        if len(lt):
            out[f"{lane}_lane"] = {"requests": int(len(lt)), "p50_ms": round(float(np.percentile(lt, 50)) * 1e3, 2),
                                   "p99_ms": round(float(np.percentile(lt, 99)) * 1e3, 2)}
    out["drain_s"] = round(t_last - t_arr, 3)
    if offered_rate:
        out["offered_per_s"] = offered_rate
        out["saturated"] = bool((t_last - t_arr) > 0.25 * max(t_arr - t_first, 1e-9))
    return out

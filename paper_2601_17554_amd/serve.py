"""Continuous-batching serving loop for MLPF reconstruction on one GPU.

Requests (one event each: element features [n][F], optionally the primaries' (pT, E) [n][2] for
the Eq. 2 decode) arrive at any time and are queued in FIFO order. A single scheduler thread admits
them into batches as soon as an execution slot is free: a batch takes queued events while it stays
within the slot's row and event capacity and while the HBM footprint of every batch in flight
(activations: the library's workspace for the batch's rows and events, plus its inputs and
outputs) stays within the activation budget; when the queue head does not fit, admission waits for
a batch to finish. Every slot owns its own stream and buffers, so batches of different slots
overlap on the device; a request that arrives while others run joins the next batch that a freed
slot forms ("continuous batching"). The scheduler also resolves finished batches: each request's
future gets its own rows of the outputs and its latency (arrival to result on the host) is
recorded, with the batch sizes, queue waits and batch service times.

The scheduler is independent of the device: ``GpuExecutor`` runs batches through libmlpf
(pinned host staging, asynchronous copies, captured HIP graphs per capacity bucket), and tests
drive the same scheduler with a CPU executor.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import threading
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

MAX_SEQLEN = 8192


class CapacityError(ValueError):
    """An event that can never be admitted (more elements than the per-event maximum or a slot)."""


class Request:
    __slots__ = ("x", "prim", "arrival", "future", "done_at", "attempts", "admitted_at")

    def __init__(self, x: np.ndarray, prim: Optional[np.ndarray], arrival: float):
        self.x, self.prim, self.arrival = x, prim, arrival
        self.future: cf.Future = cf.Future()
        self.done_at = 0.0
        self.admitted_at = 0.0
        self.attempts = 0

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


class Executor:
    """Interface of a batch executor with a fixed number of slots."""

    max_rows: int
    max_events: int

    def slots(self) -> int:
        raise NotImplementedError

    def launch(self, slot: int, reqs: Sequence[Request]) -> None:
        """Starts a batch on a free slot (asynchronous)."""
        raise NotImplementedError

    def done(self, slot: int) -> bool:
        """Non-blocking: has the slot's batch finished?"""
        raise NotImplementedError

    def results(self, slot: int, reqs: Sequence[Request]) -> List[Dict[str, np.ndarray]]:
        """Per-request outputs of a finished batch (host arrays owned by the caller)."""
        raise NotImplementedError

    def reset(self, slot: int) -> None:
        """Recovers a slot after a failed batch."""

    def footprint(self, rows: int, events: int) -> int:
        """HBM bytes a batch of this many rows and events occupies while in flight (0: no
        accounting)."""
        return 0


class Server:
    """FIFO continuous-batching scheduler over an Executor."""

    def __init__(self, executor: Executor, max_queue: int = 1_000_000, retries: int = 1,
                 idle_sleep: float = 50e-6, hbm_budget: Optional[int] = None):
        self.ex = executor
        self.max_queue = max_queue
        self.retries = retries
        self.idle_sleep = idle_sleep
        # Activation budget of the batches in flight (bytes; None: the executor's, if any).
        self.budget = hbm_budget if hbm_budget is not None else getattr(executor, "hbm_budget", None)
        self._q: collections.deque = collections.deque()
        self._lock = threading.Lock()
        self._busy: Dict[int, List[Request]] = {}
        self._bytes: Dict[int, int] = {}
        self._started: Dict[int, float] = {}
        self._running = True
        self.completed: List[Request] = []
        self.stats = {"batches": 0, "events": 0, "failed_batches": 0, "max_inflight_slots": 0,
                      "max_inflight_bytes": 0, "admission_blocked": 0}
        self.batch_log: List[tuple] = []  # (events, rows, bytes, service seconds) per batch
        self._blocked = False
        self._thread = threading.Thread(target=self._loop, name="mlpf-scheduler", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------------ client side
    def submit(self, x: np.ndarray, prim: Optional[np.ndarray] = None,
               arrival: Optional[float] = None) -> cf.Future:
        x = np.ascontiguousarray(x, dtype=np.float32)
        if x.ndim != 2 or x.shape[0] == 0:
            raise ValueError("an event is a non-empty [n][F] array")
        if x.shape[0] > min(MAX_SEQLEN, self.ex.max_rows):
            raise CapacityError(f"event of {x.shape[0]} elements exceeds the capacity")
        if self.budget is not None and self.ex.footprint(x.shape[0], 1) > self.budget:
            raise CapacityError(f"event of {x.shape[0]} elements needs more than the HBM budget")
        req = Request(x, prim, time.perf_counter() if arrival is None else arrival)
        with self._lock:
            if len(self._q) >= self.max_queue:
                raise RuntimeError("queue full")
            self._q.append(req)
        return req.future

    def close(self, wait: bool = True) -> None:
        if wait:
            while True:
                with self._lock:
                    if not self._q and not self._busy:
                        break
                time.sleep(1e-3)
        self._running = False
        self._thread.join()

    def latencies_ms(self) -> np.ndarray:
        return np.array([(r.done_at - r.arrival) * 1e3 for r in self.completed])

    def queue_waits_ms(self) -> np.ndarray:
        """Arrival to admission into a batch, per completed request."""
        return np.array([(r.admitted_at - r.arrival) * 1e3 for r in self.completed])

    def inflight_bytes(self) -> int:
        return sum(self._bytes.values())

    # ------------------------------------------------------------------ scheduler
    def _form_batch(self):
        """(requests, footprint bytes) of the next batch: FIFO, within the slot capacities and,
        with a budget, within what the batches in flight leave of it."""
        batch: List[Request] = []
        rows = 0
        nbytes = 0
        room = None if self.budget is None else self.budget - self.inflight_bytes()
        with self._lock:
            while self._q and len(batch) < self.ex.max_events:
                n = self._q[0].n
                if rows + n > self.ex.max_rows:
                    break
                if room is not None:
                    need = self.ex.footprint(rows + n, len(batch) + 1)
                    if need > room:
                        if not batch and not self._blocked:
                            self.stats["admission_blocked"] += 1  # a new wait for the budget
                        self._blocked = not batch
                        break
                    nbytes = need
                batch.append(self._q.popleft())
                rows += n
                self._blocked = False
        return batch, nbytes

    def _failed(self, slot: int, reqs: List[Request], exc: Exception) -> None:
        """A failed batch: its events go back to the head of the queue (the forward pass is
        idempotent) until they have failed ``retries`` + 1 times."""
        self.stats["failed_batches"] += 1
        try:
            self.ex.reset(slot)
        except Exception:
            pass
        retry = []
        for r in reqs:
            r.attempts += 1
            if r.attempts <= self.retries:
                retry.append(r)
            else:
                r.future.set_exception(exc)
        with self._lock:
            self._q.extendleft(reversed(retry))

    def _finish(self, slot: int) -> None:
        reqs = self._busy.pop(slot)
        nbytes = self._bytes.pop(slot, 0)
        started = self._started.pop(slot, 0.0)
        try:
            outs = self.ex.results(slot, reqs)
        except Exception as exc:
            self._failed(slot, reqs, exc)
            return
        now = time.perf_counter()
        for r, o in zip(reqs, outs):
            r.done_at = now
            self.completed.append(r)
            r.future.set_result(o)
        self.stats["batches"] += 1
        self.stats["events"] += len(reqs)
        self.batch_log.append((len(reqs), sum(r.n for r in reqs), nbytes, now - started))

    def _loop(self) -> None:
        while self._running:
            progressed = False
            for slot in list(self._busy):
                try:
                    finished = self.ex.done(slot)
                except Exception:
                    finished = True  # results() raises and the batch is retried
                if finished:
                    self._finish(slot)
                    progressed = True
            for slot in range(self.ex.slots()):
                if slot in self._busy:
                    continue
                batch, nbytes = self._form_batch()
                if not batch:
                    break
                progressed = True
                now = time.perf_counter()
                for r in batch:
                    r.admitted_at = now
                try:
                    self.ex.launch(slot, batch)
                except Exception as exc:
                    self._failed(slot, batch, exc)
                    continue
                self._busy[slot] = batch
                self._bytes[slot] = nbytes
                self._started[slot] = now
            self.stats["max_inflight_slots"] = max(self.stats["max_inflight_slots"], len(self._busy))
            self.stats["max_inflight_bytes"] = max(self.stats["max_inflight_bytes"], self.inflight_bytes())
            if not progressed:
                time.sleep(self.idle_sleep)


class GpuExecutor(Executor):
    """Runs batches through libmlpf. Each slot owns a stream, pinned host staging, device buffers
    sized for ``max_rows``/``max_events`` and one captured graph per capacity bucket (row
    capacities max_rows / 2^k), so a small batch replays a small graph. ``hbm_budget`` bounds the
    slots' buffers (fewer slots when they would not fit) and is the scheduler's admission budget:
    a batch's footprint is the workspace the library needs for its rows and events plus its input
    and output rows. ``decode``: requests carry the primaries and get the decoded (pT, eta, phi, E)."""

    def __init__(self, model, max_rows: int = 65536, max_events: int = 64, slots: int = 3,
                 hbm_budget: Optional[int] = None, buckets: int = 4, decode: bool = False):
        import torch
        from . import binding as B
        self.torch, self.B, self.model = torch, B, model
        self.max_rows, self.max_events = max_rows, max_events
        self.decode = decode
        f = model.cfg.n_features
        # Input features, logits, regressions, class; with the decode also primaries and decoded.
        self.row_io_bytes = (f + 6 + 5 + 1 + (2 + 4 if decode else 0)) * 4
        slot_bytes = self.footprint(max_rows, max_events)
        if hbm_budget is not None:
            slots = max(1, min(slots, hbm_budget // max(slot_bytes, 1)))
        self.hbm_budget = hbm_budget
        self.slot_bytes = slot_bytes
        self._slots = []
        caps = sorted({max(1024, max_rows >> k) for k in range(buckets)})
        for _ in range(slots):
            s = {"stream": torch.cuda.Stream()}
            with torch.cuda.stream(s["stream"]):
                s["x_pin"] = torch.zeros(max_rows, f, dtype=torch.float32).pin_memory()
                s["rs_pin"] = torch.zeros(max_events + 1, dtype=torch.int32).pin_memory()
                s["nv_pin"] = torch.zeros(max_events, dtype=torch.int32).pin_memory()
                s["x"] = torch.zeros(max_rows, f, device="cuda")
                s["rs"] = torch.zeros(max_events + 1, dtype=torch.int32, device="cuda")
                s["nv"] = torch.zeros(max_events, dtype=torch.int32, device="cuda")
                s["ws"] = model.workspace(max_rows, max_events)
                s["out"] = model.outputs(max_rows, decode=decode)
                s["prim_pin"] = torch.ones(max_rows, 2, dtype=torch.float32).pin_memory() if decode else None
                s["prim"] = torch.ones(max_rows, 2, device="cuda") if decode else None
                s["out_pin"] = {k: torch.empty(v.shape, dtype=v.dtype).pin_memory()
                                for k, v in s["out"].items()}
                s["graphs"] = {}
                for cap in caps:
                    batch = B.Batch(s["rs"], s["nv"], max_events, cap, MAX_SEQLEN)
                    s["graphs"][cap] = (B.Graph(model, s["x"], batch, s["out"], s["ws"], s["stream"],
                                                prim=s["prim"]), batch)
                s["event"] = torch.cuda.Event()
                # One replay of every graph now (empty batch: the event table above is all zeros),
                # so that no request pays a graph's first launch.
                for g, _ in s["graphs"].values():
                    g.launch(s["stream"])
            s["stream"].synchronize()
            self._slots.append(s)
        self.caps = caps

    def slots(self) -> int:
        return len(self._slots)

    def footprint(self, rows: int, events: int) -> int:
        return self.model.workspace_bytes(rows, events) + rows * self.row_io_bytes

    def launch(self, slot: int, reqs: Sequence[Request]) -> None:
        s = self._slots[slot]
        torch = self.torch
        t = 0
        rs = s["rs_pin"].numpy()
        nv = s["nv_pin"].numpy()
        xp = s["x_pin"].numpy()
        pp = s["prim_pin"].numpy() if self.decode else None
        for i, r in enumerate(reqs):
            rs[i] = t
            nv[i] = r.n
            xp[t:t + r.n] = r.x
            if pp is not None:
                pp[t:t + r.n] = r.prim if r.prim is not None else 1.0
            t += r.n
        rs[len(reqs):] = t
        nv[len(reqs):] = 0
        cap = next(c for c in self.caps if c >= t)
        s["rows"] = t
        with torch.cuda.stream(s["stream"]):
            s["x"][:t].copy_(s["x_pin"][:t], non_blocking=True)
            if self.decode:
                s["prim"][:t].copy_(s["prim_pin"][:t], non_blocking=True)
            s["rs"].copy_(s["rs_pin"], non_blocking=True)
            s["nv"].copy_(s["nv_pin"], non_blocking=True)
            s["graphs"][cap][0].launch(s["stream"])
            for k, v in s["out"].items():
                s["out_pin"][k][:t].copy_(v[:t], non_blocking=True)
            s["event"].record(s["stream"])

    def done(self, slot: int) -> bool:
        return self._slots[slot]["event"].query()

    def results(self, slot: int, reqs: Sequence[Request]) -> List[Dict[str, np.ndarray]]:
        s = self._slots[slot]
        s["event"].synchronize()
        host = {k: v.numpy() for k, v in s["out_pin"].items()}
        out, t = [], 0
        for r in reqs:
            out.append({k: v[t:t + r.n].copy() for k, v in host.items()})
            t += r.n
        return out

    def reset(self, slot: int) -> None:
        self._slots[slot]["stream"].synchronize()


def run_poisson(server: Server, events: Sequence[np.ndarray], arrivals: np.ndarray,
                prims: Optional[Sequence[np.ndarray]] = None,
                late: Optional[List[float]] = None) -> float:
    """Submits events (and their primaries, if given) at the given arrival offsets (seconds from
    now), waits for all results, and returns the wall time from the first arrival to the last
    result. A request's arrival time is its scheduled one; ``late`` (if given) receives how long
    after it each submit actually happened (seconds)."""
    t0 = time.perf_counter()
    futs = []
    for i, (x, a) in enumerate(zip(events, arrivals)):
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        if late is not None:
            late.append(time.perf_counter() - t0 - a)
        futs.append(server.submit(x, None if prims is None else prims[i], arrival=t0 + a))
    for f in futs:
        f.result()
    return time.perf_counter() - t0

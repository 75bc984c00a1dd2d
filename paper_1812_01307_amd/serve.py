"""Continuous batching of independent reconstructions (serving).

Requests are 2-D reconstructions y -> x by the epochs of Algorithm 1, each on
one of several registered geometries (a plan: the block store of A and A^T),
with its own lambda.  The server keeps the geometries resident and serves
requests through batch states: a state with S slots runs the epochs of up to
S requests of one geometry at once (the several-RHS products read each entry
of A once for all slots, and the TV prox runs per slot with per-slot theta).

Scheduling, one round of `step()`:
  1. admission: queued requests (arrival order) take a free slot of a batch
     state of their geometry; when every slot is taken, a new batch state is
     created if it fits the HBM budget (plans + states, by their workspace
     sizes), after releasing idle states if needed.  A new state has one slot
     when its request is the only one of its geometry running or waiting
     (the one-RHS pass then runs no idle columns), else as many as that
     geometry's running and waiting requests doubled, rounded up to 4, 8, ...
     and capped at the server's width; an idle state of the geometry narrower
     than that is dropped rather than reused.
     A request that does not fit waits; requests of other geometries are not
     held behind it.
  2. every batch state with an occupied slot runs `chunk` epochs on its own
     stream; the launches of all states are queued before any is waited on,
     so the work of different geometries overlaps on the device.
  3. each state's per-slot residual norms of the last two epochs are read;
     a slot stops when | ||r_{k+1}|| - ||r_k|| | / ||r_k|| < tol or after
     max_epochs epochs, is copied out and freed.

A request is admitted between rounds only, so its epochs count from a chunk
boundary and the stop rule is evaluated after the same epochs whatever else
is being served; the slots of a state do not interact (every product, norm
and prox is per slot).  A request therefore gets the same result alone and in
a mix (bitwise, for the same chunk: a one-slot state and a slot of a wider
state sum in the same order).  `cancel(rid)` drops a
queued request, or empties a running request's slot between rounds; the
other slots are untouched.

Each geometry can keep a tile-sliced store resident (the single-pass form of
the epoch products): every batch state of that geometry then reads it once
per epoch for both products of all its slots, four slots per workgroup.

The device work is done by the C entry points (through `capi`); this module
only decides what runs where.  `Server` takes a backend object so that the
policy can be exercised without a GPU.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Hashable, List, Optional


@dataclass
class Request:
    """One reconstruction: y (the backend's vector type) on `geometry`."""
    rid: int
    geometry: Hashable
    y: Any
    lam: float
    arrival: float = 0.0                 # seconds on the server's clock
    # filled in by the server
    x: Any = None
    epochs: int = 0
    admitted: Optional[float] = None
    finished: Optional[float] = None
    res_norm2: Optional[float] = None
    stop: str = ""                       # "converged", "max_epochs" or "cancelled"

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Batch:
    geometry: Hashable
    handle: Any
    nbytes: int
    slots: List[Optional[Request]]
    last_used: int = 0

    def free_slot(self) -> int:
        for k, r in enumerate(self.slots):
            if r is None:
                return k
        return -1

    @property
    def active(self) -> int:
        return sum(r is not None for r in self.slots)


class Server:
    """Continuous-batching scheduler over a backend (see `DeviceBackend`)."""

    def __init__(self, backend, slots: int = 8, chunk: int = 10, tol: float = 1e-4,
                 max_epochs: int = 300, hbm_bytes: Optional[int] = None,
                 max_states: Optional[int] = None, clock: Callable[[], float] = time.perf_counter):
        if chunk < 2 or max_epochs % chunk:
            raise ValueError("chunk must be >= 2 and divide max_epochs")
        self.backend = backend
        self.slots = slots
        self.chunk = chunk
        self.tol = tol
        self.max_epochs = max_epochs
        self.hbm_bytes = hbm_bytes
        self.max_states = max_states
        self.clock = clock
        self.t0 = clock()
        self.geometries: dict = {}
        self.batches: List[_Batch] = []
        self.queue: List[Request] = []
        self.done: List[Request] = []
        self.cancelled: List[Request] = []
        self.rounds = 0

    # -- bookkeeping ------------------------------------------------------
    def now(self) -> float:
        return self.clock() - self.t0

    def resident_bytes(self) -> int:
        return (sum(self.backend.geometry_bytes(g) for g in self.geometries.values())
                + sum(b.nbytes for b in self.batches))

    def add_geometry(self, key: Hashable, geometry) -> None:
        """Register a resident geometry (the backend's object for it)."""
        if key in self.geometries:
            raise ValueError(f"geometry {key!r} already registered")
        if self.hbm_bytes is not None:
            need = self.resident_bytes() + self.backend.geometry_bytes(geometry)
            if need > self.hbm_bytes:
                raise MemoryError(f"geometry {key!r} does not fit the HBM budget")
        self.geometries[key] = geometry

    def submit(self, req: Request) -> None:
        if req.geometry not in self.geometries:
            raise KeyError(f"unknown geometry {req.geometry!r}")
        if not (math.isfinite(req.lam) and req.lam >= 0.0):
            raise ValueError("lambda must be finite and >= 0")
        self.queue.append(req)

    def cancel(self, rid) -> bool:
        """Withdraw request `rid`: from the queue, or from its slot (which is
        emptied; the state's other slots are not touched).  Call between
        rounds.  False if the request is not queued or running."""
        for i, req in enumerate(self.queue):
            if req.rid == rid:
                del self.queue[i]
                self._cancelled(req)
                return True
        for b in self.batches:
            for k, req in enumerate(b.slots):
                if req is not None and req.rid == rid:
                    self.backend.release(b.handle, k)
                    b.slots[k] = None
                    self.backend.set_lambdas(b.handle, [r.lam if r is not None else 0.0
                                                        for r in b.slots])
                    self._cancelled(req)
                    return True
        return False

    def _cancelled(self, req: Request) -> None:
        req.stop = "cancelled"
        req.finished = self.now()
        self.cancelled.append(req)

    @property
    def busy(self) -> bool:
        return bool(self.queue) or any(b.active for b in self.batches)

    # -- admission ---------------------------------------------------------
    def _width(self, demand: int) -> int:
        """Slots of a new state for a geometry with `demand` requests running or
        waiting: one for a lone request, else the smallest power of two from 4
        that holds twice as many (room for the arrivals a loaded geometry
        keeps receiving), at most the server's width (states hold 1 or a power
        of two from 4 RHS).  A wide state's pass costs about as much as its
        slots would alone only when about half of them are occupied (at 512^2:
        0.24 ms one RHS, 0.44 ms four, 0.83 ms eight), so widths follow the
        geometry's load rather than the maximum."""
        if demand <= 1 or self.slots < 4:
            return 1
        w = 4
        while w < 2 * demand and w * 2 <= self.slots:
            w *= 2
        return w

    def _new_batch(self, key, width: Optional[int] = None) -> Optional[_Batch]:
        geom = self.geometries[key]
        width = self.slots if width is None else width
        nbytes = self.backend.state_bytes(geom, width)
        if self.max_states is not None and len(self.batches) >= self.max_states:
            if not self._release_idle(0, force_count=True):
                return None
        if self.hbm_bytes is not None:
            if not self._release_idle(self.resident_bytes() + nbytes - self.hbm_bytes):
                return None
        b = _Batch(key, self.backend.new_state(geom, width), nbytes, [None] * width)
        self.batches.append(b)
        return b

    def _release_idle(self, excess: int, force_count: bool = False) -> bool:
        """Drop idle batch states (least recently used first) until `excess`
        bytes are freed (or one state, with force_count).  False if not enough."""
        idle = sorted((b for b in self.batches if b.active == 0), key=lambda b: b.last_used)
        freed, dropped = 0, 0
        for b in idle:
            if freed >= excess and (not force_count or dropped >= 1):
                break
            self.batches.remove(b)
            self.backend.drop_state(b.handle)
            freed += b.nbytes
            dropped += 1
        return freed >= excess and (not force_count or dropped >= 1)

    def _admit(self) -> None:
        waiting = []
        changed = set()
        for i, req in enumerate(self.queue):
            # requests of this geometry running, and waiting from here on
            demand = (sum(b.active for b in self.batches if b.geometry == req.geometry)
                      + sum(r.geometry == req.geometry for r in self.queue[i:]))
            want = self._width(demand)
            target, k = None, -1
            for b in self.batches:
                # a free slot of a running state, or of an idle one wide enough
                if b.geometry == req.geometry and (b.active or len(b.slots) >= want):
                    k = b.free_slot()
                    if k >= 0:
                        target = b
                        break
            if target is None:
                # idle states of this geometry narrower than its load make room
                for b in [b for b in self.batches
                          if b.geometry == req.geometry and not b.active]:
                    self.batches.remove(b)
                    self.backend.drop_state(b.handle)
                target = self._new_batch(req.geometry, want)
                k = 0 if target is not None else -1
            if target is None:
                waiting.append(req)
                continue
            target.slots[k] = req
            req.admitted = self.now()
            req.epochs = 0
            self.backend.admit(target.handle, self.geometries[req.geometry], k, req)
            changed.add(id(target))
        self.queue = waiting
        for b in self.batches:
            if id(b) in changed:
                self.backend.set_lambdas(b.handle, [r.lam if r is not None else 0.0
                                                    for r in b.slots])

    # -- one round -----------------------------------------------------------
    def step(self) -> List[Request]:
        """Admit, run one chunk of epochs on every occupied state, retire."""
        self._admit()
        self.rounds += 1
        running = [b for b in self.batches if b.active]
        for b in running:
            b.last_used = self.rounds
            self.backend.launch(b.handle, self.geometries[b.geometry], self.chunk)
        finished = []
        for b in running:
            now, prev = self.backend.res_change(b.handle)
            for k, req in enumerate(b.slots):
                if req is None:
                    continue
                req.epochs += self.chunk
                rel = (abs(math.sqrt(now[k]) - math.sqrt(prev[k])) / math.sqrt(prev[k])
                       if prev[k] > 0.0 else math.inf)
                if rel < self.tol or req.epochs >= self.max_epochs:
                    req.stop = "converged" if rel < self.tol else "max_epochs"
                    req.res_norm2 = now[k]
                    req.x = self.backend.take_result(b.handle, k)
                    self.backend.release(b.handle, k)
                    b.slots[k] = None
                    finished.append(req)
            if any(r is None for r in b.slots) and b.active:
                self.backend.set_lambdas(b.handle, [r.lam if r is not None else 0.0
                                                    for r in b.slots])
        t = self.now()
        for req in finished:
            req.finished = t
        self.done.extend(finished)
        return finished

    def run(self, requests: List[Request], sleep: Callable[[float], None] = time.sleep
            ) -> List[Request]:
        """Serve `requests`, each submitted once the clock passes its arrival."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        i = 0
        while i < len(pending) or self.busy:
            t = self.now()
            while i < len(pending) and pending[i].arrival <= t:
                self.submit(pending[i])
                i += 1
            if not self.busy:
                sleep(max(0.0, pending[i].arrival - t))
                continue
            self.step()
        return self.done


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return v[k - 1]


@dataclass
class Geometry:
    """A resident geometry on the device: its plan, its tile-sliced store (or
    None: states then run the block store's products) and step size."""
    plan: Any
    mu: float
    prox_iters: int = 20
    vt: int = 0
    fused: Any = None


class DeviceBackend:
    """The C entry points behind `Server` (one HIP stream per batch state)."""

    def __init__(self):
        import torch
        from . import capi
        self.torch = torch
        self.capi = capi

    def geometry(self, plan, power_iters: int = 30, prox_iters: int = 20, mu=None,
                 vt: int = 0, fused: bool = True, lanczos_steps: int = 10) -> Geometry:
        """Resident geometry.  fused: build its tile-sliced store.  Step size
        mu = 0.9 / (2 u_max) (Theorem 1), u_max by Lanczos steps on the store
        (power iteration on the block store without one), unless mu is given."""
        capi = self.capi
        F = capi.bsgd_fused_create(plan, 0) if fused else None
        if mu is None:
            u = (capi.bsgd_lanczos_umax_fused(F, lanczos_steps, vt=vt) if F is not None
                 else capi.bsgd_power_umax(plan, power_iters, vt=vt))
            mu = 0.9 / (2.0 * u)
        return Geometry(plan, float(mu), prox_iters, vt, F)

    def geometry_bytes(self, g: Geometry) -> int:
        return g.plan.workspace.numel() + (g.fused.workspace.numel() if g.fused else 0)

    def state_bytes(self, g: Geometry, slots: int) -> int:
        n = self.capi.bsgd_state_workspace_size(g.plan, slots)
        if g.fused is not None:
            n += self.capi.bsgd_fused_partials_size_rhs(g.fused, slots)
        return n

    def new_state(self, g: Geometry, slots: int):
        torch, capi = self.torch, self.capi
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            st = capi.bsgd_state_create(g.plan, slots, g.vt)
            if g.fused is not None:
                capi.bsgd_state_attach_fused(st, g.fused)
            if slots > 1:
                zeros = torch.zeros(g.plan.nrows * slots, dtype=torch.float32, device="cuda")
                capi.bsgd_state_init(st, zeros, stream=stream)
        return {"state": st, "stream": stream, "slots": slots, "lam": 0.0}

    def drop_state(self, h) -> None:
        h["stream"].synchronize()
        h["state"] = None

    def admit(self, h, g: Geometry, k: int, req: Request) -> None:
        capi = self.capi
        with self.torch.cuda.stream(h["stream"]):
            if h["slots"] == 1:
                capi.bsgd_state_init(h["state"], req.y, stream=h["stream"])
                h["lam"] = req.lam
            else:
                capi.bsgd_state_set_rhs(h["state"], k, req.y, None, stream=h["stream"])

    def set_lambdas(self, h, lams) -> None:
        if h["slots"] > 1:
            self.capi.bsgd_state_set_lambda(h["state"], lams, stream=h["stream"])

    def launch(self, h, g: Geometry, epochs: int) -> None:
        lam = h["lam"] if h["slots"] == 1 else -1.0
        self.capi.bsgd_run_epochs(h["state"], g.mu, lam, epochs, g.prox_iters,
                                  stream=h["stream"])

    def res_change(self, h):
        return self.capi.bsgd_get_res_change_rhs(h["state"], stream=h["stream"])

    def take_result(self, h, k: int):
        with self.torch.cuda.stream(h["stream"]):
            if h["slots"] == 1:
                x = self.capi.bsgd_get_x(h["state"], stream=h["stream"])
            else:
                x = self.capi.bsgd_get_x_rhs(h["state"], k, stream=h["stream"])
        h["stream"].synchronize()
        return x

    def release(self, h, k: int) -> None:
        if h["slots"] > 1:
            with self.torch.cuda.stream(h["stream"]):
                self.capi.bsgd_state_set_rhs(h["state"], k, None, None, stream=h["stream"])

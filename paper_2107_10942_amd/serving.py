"""Request serving on one GPU: continuous batching of Q2X jobs.

Requests arrive with their mesh and densities in pinned host memory, tagged
with a mesh identity.  The server loop admits every request that has arrived,
in arrival order, while the device bytes it holds stay within an HBM budget
(and up to `max_batch` requests per batch):

* meshes stay resident in HBM (an LRU cache keyed by the mesh identity): a
  request whose mesh is resident is admitted without any upload; a missing
  mesh is uploaded on a copy stream, and resident meshes that no batch in
  flight uses are evicted, least recently used first, when the budget needs
  the room;
* a batch is launched as one q2x_batch_launch on one of `compute_streams`
  compute streams (round robin, all of the default priority), each with its
  own workspace that is kept and grown, never reallocated per batch; so the
  next batch's uploads and kernels overlap the batches still running;
* completions are polled, and a request's coefficients are in HBM when its
  batch's event has fired.

A request runs in FP32-mixed precision up to order `p_fp32_max` and in FP64
above it.  Latency of a request = its arrival (mesh already in pinned host
memory) to the completion of its batch, measured on the host clock.  A
request's coefficients do not depend on what it is batched with or whether
its mesh was resident (the batch path computes every job exactly as the
single call does).

Only host-side orchestration lives here; all computation is the library's.
"""
from __future__ import annotations

import time
from collections import OrderedDict
from dataclasses import dataclass, field

import numpy as np
import torch

from . import q2x


@dataclass
class Request:
    kind: int
    p: int
    verts: torch.Tensor       # pinned host, float64 [V][3]
    elems: torch.Tensor       # pinned host, int32 [N][k]
    density: torch.Tensor     # pinned host, float64 [N]
    elem_box: torch.Tensor    # pinned host, int32 [N]
    box_center: torch.Tensor  # pinned host, float64 [B][3]
    arrival: float = 0.0      # seconds after the start of serving
    mesh_id: object = None    # identity of (verts, elems, density, elem_box, box_center); None: never cached
    # filled by the server
    precision: int = -1
    done: float = -1.0
    batch: int = -1
    resident_hit: bool = False
    out: torch.Tensor | None = None

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])

    @property
    def n_boxes(self) -> int:
        return int(self.box_center.shape[0])

    def mesh_bytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in (self.verts, self.elems, self.density, self.elem_box,
                                                          self.box_center))

    def work_bytes(self) -> int:
        """HBM the request needs while in flight besides its mesh: output and workspace share."""
        outb = self.n_boxes * (self.p + 1) ** 2 * 16
        wsb = q2x.workspace_bytes(self.kind, self.n_elems, self.n_boxes, self.p, q2x.FP64)
        return outb + wsb

    def device_bytes(self) -> int:
        return self.mesh_bytes() + self.work_bytes()

    def coefficients(self) -> int:
        return self.n_elems * (self.p + 1) ** 2


def pinned(a, dtype) -> torch.Tensor:
    t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype)
    return t.pin_memory()


def pinned_mesh(job) -> dict:
    """A job's mesh, densities, box map and centres in pinned host memory (Request fields)."""
    return dict(verts=pinned(job.verts, torch.float64), elems=pinned(job.elems, torch.int32),
                density=pinned(job.density, torch.float64), elem_box=pinned(job.elem_box, torch.int32),
                box_center=pinned(job.box_center, torch.float64))


@dataclass(eq=False)
class _Resident:
    tensors: list             # device copies: verts, elems, density, elem_box, box_center
    nbytes: int
    ready: torch.cuda.Event   # the upload's completion
    users: int = 0            # batches in flight that read it


@dataclass
class _Flight:
    event: torch.cuda.Event
    reqs: list
    keep: list
    work_bytes: int
    meshes: list              # resident entries this batch reads


@dataclass
class Server:
    device: torch.device
    hbm_budget: int
    max_batch: int = 16
    p_fp32_max: int = 32
    keep_outputs: bool = False
    resident: bool = True     # keep meshes in HBM between requests
    compute_streams: int = 2
    stats: dict = field(default_factory=dict)

    def __post_init__(self):
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, self.compute_streams))]
        self.workspaces = [None] * len(self.streams)
        self.cache: OrderedDict = OrderedDict()   # mesh_id -> _Resident, least recently used first
        self.cache_bytes = 0

    # ---- resident meshes
    def _evict_for(self, need: int, budget_left) -> bool:
        """Evict unused resident meshes (LRU first) until `need` bytes fit; False if they cannot."""
        while budget_left() < need:
            victim = next((k for k, v in self.cache.items() if v.users == 0), None)
            if victim is None:
                return False
            ent = self.cache.pop(victim)
            self.cache_bytes -= ent.nbytes
        return True

    def _mesh_on_device(self, r: Request):
        """Device tensors of r's mesh: the resident copy (a hit) or a new upload on the copy stream."""
        key = r.mesh_id
        if self.resident and key is not None and key in self.cache:
            ent = self.cache[key]
            self.cache.move_to_end(key)
            r.resident_hit = True
            return ent
        with torch.cuda.stream(self.copy_stream):
            d = [t.to(self.device, non_blocking=True) for t in (r.verts, r.elems, r.density, r.elem_box,
                                                                 r.box_center)]
        ev = torch.cuda.Event()
        ev.record(self.copy_stream)
        ent = _Resident(d, r.mesh_bytes(), ev)
        if self.resident and key is not None:
            self.cache[key] = ent
            self.cache_bytes += ent.nbytes
        return ent

    def _workspace(self, i: int, nbytes: int) -> torch.Tensor:
        ws = self.workspaces[i]
        if ws is None or ws.numel() < nbytes:
            # grown, never shrunk (allocated on its compute stream, whose
            # earlier batches the allocator then waits for before reusing it)
            with torch.cuda.stream(self.streams[i]):
                buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-buf.data_ptr()) % 256
            ws = buf[off:off + nbytes]
            self.workspaces[i] = ws
        return ws

    def _is_cached(self, ent) -> bool:
        return any(v is ent for v in self.cache.values())

    def _launch(self, reqs, bid):
        si = bid % len(self.streams)
        xs = self.streams[si]
        ents = [self._mesh_on_device(r) for r in reqs]
        uniq = list({id(e): e for e in ents}.values())
        for e in uniq:
            xs.wait_event(e.ready)
            e.users += 1
            for t in e.tensors:  # uploaded on the copy stream, read on this one
                t.record_stream(xs)
        specs = []
        with torch.cuda.stream(xs):
            for r, e in zip(reqs, ents):
                d = e.tensors
                r.precision = q2x.FP32_MIXED if r.p <= self.p_fp32_max else q2x.FP64
                r.batch = bid
                specs.append(dict(kind=r.kind, verts=d[0], elems=d[1], density=d[2], elem_box=d[3],
                                  box_center=d[4], p=r.p, precision=r.precision))
            plan = q2x.BatchPlan(specs)
            ws = self._workspace(si, plan.workspace_bytes())
            plan.launch(ws, stream=xs)
            done = torch.cuda.Event()
            done.record(xs)
        for r, o in zip(reqs, plan.outs):
            r.out = o
        # meshes that are not kept resident count against the budget while the batch runs
        transient = sum(e.nbytes for e in uniq if not self._is_cached(e))
        keep = [plan] + [e.tensors for e in uniq]
        return _Flight(done, reqs, keep, sum(r.work_bytes() for r in reqs) + transient, uniq)

    def serve(self, requests: list[Request]) -> list[Request]:
        """Serve `requests` (arrival times set) to completion; returns them with done times."""
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        nxt = 0
        flights: list[_Flight] = []
        in_flight = 0  # work bytes of the batches in flight (meshes are counted in cache_bytes)
        bid = 0
        hits = misses = 0
        t0 = time.perf_counter()
        while nxt < len(order) or flights:
            now = time.perf_counter() - t0
            # completions
            still = []
            for f in flights:
                if f.event.query():
                    t = time.perf_counter() - t0
                    for r in f.reqs:
                        r.done = t
                        if not self.keep_outputs:
                            r.out = None
                    in_flight -= f.work_bytes
                    for e in f.meshes:
                        e.users -= 1
                else:
                    still.append(f)
            flights = still
            # admission: arrived requests, in order, within the budget
            batch = []
            nbytes = 0
            new_mesh = 0
            seen = set()
            held = []  # resident meshes this batch will read: not evictable meanwhile
            while nxt < len(order) and len(batch) < self.max_batch:
                r = requests[order[nxt]]
                if r.arrival > now:
                    break
                cacheable = self.resident and r.mesh_id is not None
                cached = cacheable and (r.mesh_id in self.cache or r.mesh_id in seen)
                need = r.work_bytes() + (0 if cached else r.mesh_bytes())
                if batch or flights:
                    def left():
                        return self.hbm_budget - (self.cache_bytes + in_flight + nbytes + new_mesh)
                    if left() < need and not self._evict_for(need, left):
                        break
                batch.append(r)
                nbytes += r.work_bytes()
                if cached and r.mesh_id in self.cache:
                    ent = self.cache[r.mesh_id]
                    ent.users += 1
                    held.append(ent)
                elif not cached:
                    new_mesh += r.mesh_bytes()
                    if cacheable:
                        seen.add(r.mesh_id)
                nxt += 1
            if batch:
                fl = self._launch(batch, bid)
                for ent in held:
                    ent.users -= 1
                flights.append(fl)
                hits += sum(r.resident_hit for r in batch)
                misses += sum(not r.resident_hit for r in batch)
                in_flight += fl.work_bytes
                bid += 1
                continue
            # nothing to start: wait for the next arrival or a completion
            wait = (requests[order[nxt]].arrival - now) if nxt < len(order) else 1e-4
            time.sleep(min(max(wait, 0.0), 1e-4))
        torch.cuda.synchronize(self.device)
        self.stats = {"batches": bid, "resident_hits": hits, "uploads": misses,
                      "resident_meshes": len(self.cache), "resident_bytes": self.cache_bytes}
        return requests


def latency_summary(reqs: list[Request]) -> dict:
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    coefs = sum(r.coefficients() for r in reqs)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "requests": len(reqs),
            "coefficients_per_s": coefs / span, "span_s": span,
            "fp64_fraction": float(np.mean([r.precision == q2x.FP64 for r in reqs])),
            "resident_hit_rate": float(np.mean([r.resident_hit for r in reqs]))}


def poisson_arrivals(n: int, rate: float, rng) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (per second)."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))

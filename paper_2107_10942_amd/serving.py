"""Request serving on one GPU: continuous batching of Q2X jobs.

Requests arrive with their mesh and densities in pinned host memory.  The
server loop admits every request that has arrived, in arrival order, while
the bytes of the batches in flight stay within an HBM budget (and up to
`max_batch` requests per batch); uploads the batch on a copy stream; launches
it as one batch (q2x_batch_launch) on the compute stream once the uploads are
done; and polls the batches in flight for completion, so the next batch is
uploaded while the current one computes.  A request runs in FP32-mixed
precision up to order `p_fp32_max` and in FP64 above it.

Latency of a request = its arrival (mesh already in pinned host memory) to
the completion of its batch (coefficients in HBM), measured on the host clock.
A request's coefficients do not depend on what it is batched with (the batch
path computes every job exactly as the single call does).

Only host-side orchestration lives here; all computation is the library's.
"""
from __future__ import annotations

import time
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
    # filled by the server
    precision: int = -1
    done: float = -1.0
    batch: int = -1
    out: torch.Tensor | None = None

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])

    @property
    def n_boxes(self) -> int:
        return int(self.box_center.shape[0])

    def device_bytes(self) -> int:
        """HBM the request needs while in flight: inputs, output, workspace."""
        ins = sum(t.numel() * t.element_size() for t in (self.verts, self.elems, self.density, self.elem_box,
                                                          self.box_center))
        outb = self.n_boxes * (self.p + 1) ** 2 * 16
        wsb = q2x.workspace_bytes(self.kind, self.n_elems, self.n_boxes, self.p, q2x.FP64)
        return ins + outb + wsb

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


@dataclass
class _Flight:
    event: torch.cuda.Event
    reqs: list
    keep: list
    nbytes: int


@dataclass
class Server:
    device: torch.device
    hbm_budget: int
    max_batch: int = 16
    p_fp32_max: int = 32
    keep_outputs: bool = False
    stats: dict = field(default_factory=dict)

    def __post_init__(self):
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.compute_stream = torch.cuda.Stream(device=self.device)

    def _launch(self, reqs, bid):
        cs, xs = self.copy_stream, self.compute_stream
        keep = []
        specs = []
        with torch.cuda.stream(cs):
            for r in reqs:
                d = [t.to(self.device, non_blocking=True) for t in (r.verts, r.elems, r.density, r.elem_box,
                                                                     r.box_center)]
                for t in d:
                    t.record_stream(xs)
                keep.append(d)
        up = torch.cuda.Event()
        up.record(cs)
        xs.wait_event(up)
        with torch.cuda.stream(xs):
            for r, d in zip(reqs, keep):
                r.precision = q2x.FP32_MIXED if r.p <= self.p_fp32_max else q2x.FP64
                r.batch = bid
                specs.append(dict(kind=r.kind, verts=d[0], elems=d[1], density=d[2], elem_box=d[3],
                                  box_center=d[4], p=r.p, precision=r.precision))
            plan = q2x.BatchPlan(specs)
            ws = plan.alloc_workspace(self.device)
            plan.launch(ws, stream=xs)
            done = torch.cuda.Event()
            done.record(xs)
        for r, o in zip(reqs, plan.outs):
            r.out = o
        keep.append((plan, ws))
        return _Flight(done, reqs, keep, sum(r.device_bytes() for r in reqs))

    def serve(self, requests: list[Request]) -> list[Request]:
        """Serve `requests` (arrival times set) to completion; returns them with done times."""
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        nxt = 0
        flights: list[_Flight] = []
        in_use = 0
        bid = 0
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
                    in_use -= f.nbytes
                else:
                    still.append(f)
            flights = still
            # admission: arrived requests, in order, within the budget
            batch = []
            nbytes = 0
            while nxt < len(order) and len(batch) < self.max_batch:
                r = requests[order[nxt]]
                if r.arrival > now:
                    break
                need = r.device_bytes()
                if batch or flights:
                    if in_use + nbytes + need > self.hbm_budget:
                        break
                batch.append(r)
                nbytes += need
                nxt += 1
            if batch:
                flights.append(self._launch(batch, bid))
                in_use += nbytes
                bid += 1
                continue
            # nothing to start: wait for the next arrival or a completion
            wait = (requests[order[nxt]].arrival - now) if nxt < len(order) else 1e-4
            time.sleep(min(max(wait, 0.0), 1e-4))
        torch.cuda.synchronize(self.device)
        self.stats = {"batches": bid}
        return requests


def latency_summary(reqs: list[Request]) -> dict:
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    coefs = sum(r.coefficients() for r in reqs)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "requests": len(reqs),
            "coefficients_per_s": coefs / span, "span_s": span,
            "fp64_fraction": float(np.mean([r.precision == q2x.FP64 for r in reqs]))}


def poisson_arrivals(n: int, rate: float, rng) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (per second)."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))

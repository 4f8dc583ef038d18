#!/usr/bin/env python
"""Q2X benchmark: coefficients/s at p = 16 on the 81,920-triangle perturbed
sphere (single + double layer, octree level 5), FP32-mixed vs plain FP64.

One step = q2x_tri_both over the whole mesh: one bucketing, one recursion
producing the single- and double-layer coefficients of every box, one fix-up;
inputs resident in HBM.  The same work as two separate calls
(q2x_tri_single + q2x_tri_double) is timed beside it.  Prints ONE JSON line.
Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 1.3M-triangle p=16 roofline workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-mesh batch workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving (Poisson arrivals) workload")
    ap.add_argument("--no-configs", action="store_true", help="skip the icosphere / tetrahedra / filament workloads")
    ap.add_argument("--serving-requests", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiler run) and exit")
    return ap.parse_args()


def stored_traffic(profile, src_hash):
    """HBM bytes per launch from a committed counter summary, if it measured this source."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
    except OSError:
        return None
    if f"`{src_hash}`" not in text:
        return None  # the kernel changed since the counters were taken
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return int(line.split(":")[1])
    return None


def batch_workload(dev, reps=5):
    """256 uneven meshes (perturbed spheres / ellipsoids, N log-uniform in [1k, 200k], p in {4..20},
    single/double): one replayed batch graph vs the same jobs as sequential single calls."""
    import numpy as np
    import torch

    from paper_2107_10942_amd import q2x
    from q2x_inputs import configs
    jobs = configs.batch_meshes()
    tens = [q2x.job_tensors(j, dev) for j in jobs]
    coefs = sum(j.n_elems * (j.p + 1) ** 2 for j in jobs)
    out = {"workload": f"{len(jobs)} meshes, {sum(j.n_elems for j in jobs)} triangles, "
                       f"{sum(j.n_boxes for j in jobs)} boxes, p in {{4,8,12,16,20}}, single/double",
           "element_coefficients": coefs}

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    results = {}
    for prec, name in ((q2x.FP32_MIXED, "fp32_mixed"), (q2x.FP64, "fp64")):
        specs = [dict(kind=j.kind, verts=t[0], elems=t[1], density=t[2], elem_box=t[3], box_center=t[4], p=j.p,
                      precision=prec) for j, t in zip(jobs, tens)]
        # the default schedule (serial capture, no split tiles, one group per order bucket) ...
        dplan = q2x.BatchPlan(specs)
        dplan.set_schedule(0, 0, 0)
        dplan.alloc_workspace(dev)
        ms_default = timed(dplan.run, reps)
        default_groups = dplan.groups
        dplan.close()
        # ... and the tuned one (the first run times the candidate schedules)
        plan = q2x.BatchPlan(specs)
        plan.alloc_workspace(dev)
        t0 = time.perf_counter()
        plan.run()
        torch.cuda.synchronize()
        tune_ms = (time.perf_counter() - t0) * 1e3
        ms_batch = timed(plan.run, reps)
        # the same jobs as single calls, one after the other (each with its own bucketing)
        wsz = max(q2x.workspace_bytes(j.kind, j.n_elems, j.n_boxes, j.p, prec) for j in jobs)
        ws = torch.empty(wsz + 256, dtype=torch.uint8, device=dev)
        ws = ws[(-ws.data_ptr()) % 256:][:wsz]
        seq_out = [torch.empty_like(o) for o in plan.outs]

        def sequential():
            for j, t, o in zip(jobs, tens, seq_out):
                q2x.run(j.kind, t[0], t[1], t[2], t[3], t[4], None, j.p, precision=prec, out=o, workspace=ws)
        ms_seq = timed(sequential, 2)
        same = all(torch.equal(a, b) for a, b in zip(plan.outs, seq_out))
        results[name] = {"batch_ms": ms_batch, "sequential_ms": ms_seq, "batch_coefficients_per_s": coefs / (ms_batch * 1e-3),
                         "sequential_coefficients_per_s": coefs / (ms_seq * 1e-3), "speedup": ms_seq / ms_batch,
                         "batched_equals_sequential": bool(same), "groups": plan.groups,
                         "capture": "parallel branches" if plan.mode == 1 else "serial",
                         "schedule": plan.schedule, "first_run_with_tuning_ms": tune_ms,
                         "default_schedule": {"batch_ms": ms_default, "groups": default_groups},
                         "tuned_vs_default_speedup": ms_default / ms_batch}
        plan.close()
        del seq_out
    out.update(results)
    out["speedup_batch_fp32_mixed_vs_sequential_fp64"] = results["fp64"]["sequential_ms"] / results["fp32_mixed"]["batch_ms"]
    return out


def error_stats(F, R, elem_norms, density, elem_box, boxes, p):
    """Scale-aware error max_{b,n} ||dF_{b,n}|| / A_{b,n} (A = sum over the box's elements of
    |density| * ||F^(e)_n||) and the normwise error ||dF_{b,n}|| / ||F_{b,n}|| (median, max)."""
    import numpy as np
    pos = {int(b): i for i, b in enumerate(boxes)}
    A = np.zeros((len(boxes), p + 1))
    np.add.at(A, np.array([pos[int(b)] for b in elem_box]), np.abs(density)[:, None] * elem_norms)
    def deg(X):
        return np.stack([np.linalg.norm(X[:, n * n:(n + 1) * (n + 1)], axis=1) for n in range(p + 1)], axis=1)
    dn, rn = deg(F - R), deg(R)
    with np.errstate(divide="ignore", invalid="ignore"):
        sa = np.where(A > 0, dn / A, 0.0)
        nw = np.where(rn > 0, dn / rn, 0.0)
    live = rn > 0
    # rows whose own norm is below 1e-6 of their box's scale A are cancellation-dominated: the
    # normwise error there measures the cancellation, not the method
    big = live & (rn > 1e-6 * A)
    return {"scale_aware_max": float(sa.max()), "normwise_median": float(np.median(nw[live])),
            "normwise_max": float(nw.max()),
            "normwise_rows_above_1e-5": int(np.sum(nw[live] > 1e-5)), "rows": int(np.sum(live)),
            "normwise_max_rows_not_cancelled": float(nw[big].max()) if big.any() else 0.0}


def other_workloads(dev, reps=20):
    """Single calls on the small icosphere (p = 8), the Kuhn tetrahedra and the random-walk segments
    (p = 12), FP32-mixed and FP64: coefficients/s of the call and of the recursion kernel."""
    import torch

    from paper_2107_10942_amd import flops, q2x
    from q2x_inputs import configs
    out = {}
    for name, job in (("icosphere_k3_1280_p8_single", configs.sphere_small()),
                      ("kuhn_tets_511104_p12", configs.kuhn_tet_volume()),
                      ("random_walk_segments_1000000_p12", configs.random_filaments())):
        tens = q2x.job_tensors(job, dev)
        o = torch.empty((job.n_boxes, (job.p + 1) ** 2, 2), dtype=torch.float64, device=dev)
        res = {"elements": job.n_elems, "boxes": job.n_boxes, "p": job.p}
        for prec, pn in ((q2x.FP32_MIXED, "fp32_mixed"), (q2x.FP64, "fp64")):
            ws = q2x.alloc_workspace(job.kind, job.n_elems, job.n_boxes, job.p, prec, device=dev)
            for _ in range(3):
                q2x.run(job.kind, *tens, job.p, precision=prec, out=o, workspace=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                q2x.run(job.kind, *tens, job.p, precision=prec, out=o, workspace=ws)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            q2x.profile_enable(True)  # kernel times from a second, profiled pass
            q2x.profile_reset()
            for _ in range(reps):
                q2x.run(job.kind, *tens, job.p, precision=prec, out=o, workspace=ws)
            torch.cuda.synchronize()
            rec_ms, call_ms, calls = q2x.profile_read()
            q2x.profile_enable(False)
            k = job.kind
            kern = rec_ms[k] / calls[k]
            fl = flops.scope_launch_flops(k, job.p, job.n_elems)
            # binding roof: min(VALU peak, arithmetic intensity x HBM peak)
            by = flops.launch_bytes(k, job.p, job.n_elems, job.n_boxes)
            ai = fl / by
            vpk = flops.peak_valu_tflops(prec == q2x.FP32_MIXED)
            hbm_bound = ai < vpk * 1e12 / (flops.PEAK_HBM_GBS * 1e9)
            ach_tf = fl / (kern * 1e-3) / 1e12
            ach_gbs = by / (kern * 1e-3) / 1e9
            res[pn] = {"call_ms": dt * 1e3, "kernel_ms": kern,
                       "coefficients_per_s": job.n_elems * (job.p + 1) ** 2 / dt,
                       "kernel_tflops": ach_tf, "kernel_gbs": ach_gbs, "flop_per_byte": ai,
                       "bound": "hbm" if hbm_bound else "alu",
                       "frac": (ach_gbs / flops.PEAK_HBM_GBS) if hbm_bound else (ach_tf / vpk)}
        out[name] = res
    # the random walks again with a vector density (walk tangent x strength): three outputs, one recursion
    import numpy as np
    job = configs.random_filaments()
    t = job.verts[job.elems[:, 1]] - job.verts[job.elems[:, 0]]
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    d3 = torch.as_tensor(t * np.random.default_rng(5).uniform(-1, 1, (job.n_elems, 1)), dtype=torch.float64,
                         device=dev).contiguous()
    tens = q2x.job_tensors(job, dev)
    o3 = torch.empty((3, job.n_boxes, (job.p + 1) ** 2, 2), dtype=torch.float64, device=dev)
    res = {"elements": job.n_elems, "boxes": job.n_boxes, "p": job.p, "outputs": 3}
    for prec, pn in ((q2x.FP32_MIXED, "fp32_mixed"), (q2x.FP64, "fp64")):
        ws = q2x.alloc_workspace(q2x.SEGMENT_VEC, job.n_elems, job.n_boxes, job.p, prec, device=dev)
        call = lambda: q2x.segment_vec(tens[0], tens[1], d3, tens[3], tens[4], None, job.p,  # noqa: E731
                                       precision=prec, out=o3, workspace=ws)
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[pn] = {"call_ms": dt * 1e3, "coefficients_per_s": 3 * job.n_elems * (job.p + 1) ** 2 / dt}
    out["random_walk_segments_vector_density_1000000_p12"] = res
    return out


def serving_workload(dev, n_requests, warmup=50, pool_size=24):
    """Poisson arrivals of requests (perturbed geodesic spheres, N log-uniform in [10k, 2M], p uniform in
    [8, 24], single/double), meshes in pinned host memory; latency submit -> coefficients in HBM."""
    import numpy as np
    import torch

    from paper_2107_10942_amd import q2x, serving
    from q2x_inputs import configs
    rng = np.random.default_rng(5)
    pool = [configs.serving_job(rng) for _ in range(pool_size)]
    meshes = [serving.pinned_mesh(j) for j in pool]
    free, _ = torch.cuda.mem_get_info(dev)
    # half the free HBM: the rest is headroom for the caching allocator's
    # rounding and for blocks cached by earlier phases
    budget = int(0.5 * free)

    def requests(n, rate, seed):
        r = np.random.default_rng(seed)
        arr = serving.poisson_arrivals(n, rate, r) if rate else np.zeros(n)
        out = []
        for i in range(n):
            m = int(r.integers(0, len(meshes)))
            out.append(serving.Request(kind=int(r.integers(0, 2)), p=int(r.integers(8, 25)), arrival=float(arr[i]),
                                       mesh_id=m, **meshes[m]))
        return out

    out = {"workload": f"{pool_size} perturbed geodesic spheres ({sum(j.n_elems for j in pool)} triangles in all), "
                       f"N log-uniform [10k, 2M], p uniform [8, 24], single/double; requests draw a mesh, p and kind",
           "hbm_budget_bytes": budget, "p_fp32_max": 32,
           "p_fp32_max_basis": "FP32-mixed meets the 1e-5 scale-aware bar up to p = 32 in the parity tests, "
                               "so no request falls back to FP64"}
    for resident, name in ((True, "resident_meshes"), (False, "upload_per_request")):
        srv = serving.Server(dev, hbm_budget=budget, max_batch=16, p_fp32_max=32, resident=resident,
                             compute_streams=2)
        # warm-up: a burst of the measured size (library load, the caching allocator's first
        # allocations for that many meshes in flight; fills the resident cache)
        srv.serve(requests(120, 0, 1))
        # capacity: a burst of requests all present at t = 0
        burst = srv.serve(requests(120, 0, 2))
        capacity = len(burst) / max(r.done for r in burst)
        res = {"capacity_requests_per_s": capacity, "compute_streams": 2}
        for load in (0.5, 0.7, 0.9):
            reqs = srv.serve(requests(warmup + n_requests, load * capacity, 10 + int(10 * load)))[warmup:]
            summ = serving.latency_summary(reqs)
            summ.update({k: srv.stats[k] for k in ("batches", "uploads", "resident_hits")})
            res[f"load_{load}"] = summ
        out[name] = res
        del srv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()  # the next phase starts without this one's cached blocks
    return out


def cpu_other_workloads(nthr, seconds):
    """The oracle's rate (element-coefficients/s) on the other workloads: the
    1,280-triangle icosphere (p = 8) in full; the Kuhn tetrahedra and the
    random-walk segments (p = 12) on every k-th box, k sized from a first run
    on every 400th box so that each takes about `seconds`."""
    import numpy as np

    import oracle
    from q2x_inputs import configs
    out = {}
    sm = configs.sphere_small()
    t0 = time.perf_counter()
    oracle.q2x(sm.kind, sm.p, sm.verts, sm.elems, sm.density, sm.elem_box, sm.box_center)
    dt = time.perf_counter() - t0
    out["icosphere_k3_1280_p8_single"] = {"value": sm.n_elems * (sm.p + 1) ** 2 / dt, "unit": "coefficients/s",
                                          "cores": nthr, "kind": "oracle",
                                          "sample": f"all {sm.n_boxes} boxes, {sm.n_elems} triangles, {dt:.3f} s"}
    for name, job in (("kuhn_tets_511104_p12", configs.kuhn_tet_volume()),
                      ("random_walk_segments_1000000_p12", configs.random_filaments())):
        def sample(stride):
            bx = np.arange(0, job.n_boxes, stride)
            keep = np.isin(job.elem_box, bx)
            t0 = time.perf_counter()
            oracle.q2x(job.kind, job.p, job.verts, job.elems[keep], job.density[keep], job.elem_box[keep],
                       job.box_center, boxes=bx)
            return int(keep.sum()), time.perf_counter() - t0, len(bx)
        ne, dt, nbx = sample(400)
        stride = max(1, int(math.ceil(job.n_elems / max(ne / dt * seconds, 1.0))))
        if stride < 400:
            ne, dt, nbx = sample(stride)
        out[name] = {"value": ne * (job.p + 1) ** 2 / dt, "unit": "coefficients/s", "cores": nthr, "kind": "oracle",
                     "sample": f"every {stride}th box ({nbx} boxes, {ne} elements), {dt:.1f} s"}
    return out


def coef_complex(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def receiving_side(dev, reps=20):
    """q2x_eval on the headline sphere at p = 16: the local expansion of each
    box integrated over its triangles (single and double layer), FP32-mixed and
    FP64.  Local coefficients: seeded U[-1,1]^2 times (1/h)^n, h the leaf box
    size.  Timed with HIP events on the stream the calls are enqueued on."""
    import numpy as np
    import torch

    from paper_2107_10942_amd import flops, q2x
    from q2x_inputs import configs
    single, double = configs.perturbed_sphere_pair()
    p, N, B = single.p, single.n_elems, single.n_boxes
    rng = np.random.default_rng(12)
    nidx = np.floor(np.sqrt(np.arange((p + 1) ** 2))).astype(int)
    scale = (1.0 / single.boxes.h) ** nidx
    L = np.stack([rng.uniform(-1, 1, (B, (p + 1) ** 2)) * scale, rng.uniform(-1, 1, (B, (p + 1) ** 2)) * scale], -1)
    lt = torch.as_tensor(L, dtype=torch.float64, device=dev).contiguous()
    v, e, d, eb, bc, br = q2x.job_tensors(single, dev)
    out = torch.empty((N, 2), dtype=torch.float64, device=dev)
    ws = q2x.alloc_eval_workspace(N, B, device=dev)
    occ = int(np.unique(single.elem_box).size)
    res = {"workload": f"perturbed icosphere k=6, {N} triangles, {B} boxes, p={p}", "elements": N, "p": p}
    stream = torch.cuda.current_stream()
    for kind, kname in ((q2x.TRI_SINGLE, "tri_single"), (q2x.TRI_DOUBLE, "tri_double")):
        for prec, pn in ((q2x.FP32_MIXED, "fp32_mixed"), (q2x.FP64, "fp64")):
            for _ in range(3):
                q2x.evaluate(kind, v, e, eb, bc, lt, p, precision=prec, out=out, workspace=ws, stream=stream)
            torch.cuda.synchronize()
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                q2x.evaluate(kind, v, e, eb, bc, lt, p, precision=prec, out=out, workspace=ws, stream=stream)
            z.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(z) / reps
            fl = flops.eval_element_flops(kind, p) * N
            res[f"{kname}_{pn}"] = {"call_ms": ms, "elements_per_s": N / (ms * 1e-3),
                                    "terms_per_s": N * (p + 1) ** 2 / (ms * 1e-3),
                                    "call_tflops": fl / (ms * 1e-3) / 1e12,
                                    "algorithmic_bytes": flops.eval_launch_bytes(kind, p, N, occ),
                                    "status_flags": q2x.status(ws)[0]}
    return res


def upward_pass(dev, reps=20):
    """Q2X leaves of the headline sphere (single layer, p = 16, FP32-mixed) then
    the M2M upward pass from level 5 to level 2 (q2x_m2m per level, FP64,
    children presorted in Morton order).  Timed with HIP events."""
    import torch

    from paper_2107_10942_amd import flops, q2x
    from q2x_inputs import configs, octree
    job = configs.perturbed_sphere_pair()[0]
    p = job.p
    levels, parents = octree.tree_levels(job.boxes, top=2)
    v, e, d, eb, bc, br = q2x.job_tensors(job, dev)
    leaf = q2x.run(job.kind, v, e, d, eb, bc, br, p, precision=q2x.FP32_MIXED)
    centers = [torch.as_tensor(c, dtype=torch.float64, device=dev) for _, c in levels]
    pars = [torch.as_tensor(x, dtype=torch.int32, device=dev) for x in parents]
    outs = [torch.empty((c.shape[0], (p + 1) ** 2, 2), dtype=torch.float64, device=dev) for c in centers[1:]]
    wss = [q2x.alloc_m2m_workspace(len(x), c.shape[0], device=dev) for x, c in zip(parents, centers[1:])]
    stream = torch.cuda.current_stream()

    def run_all():
        src = leaf
        for i in range(len(parents)):
            q2x.m2m(src, centers[i], pars[i], centers[i + 1], p, presorted=True, out=outs[i], workspace=wss[i],
                    stream=stream)
            src = outs[i]
    for _ in range(3):
        run_all()
    torch.cuda.synchronize()
    res = {"workload": f"perturbed icosphere k=6 leaves (level 5, {job.n_boxes} boxes) up to level 2, p={p}",
           "boxes_per_level": [int(c.shape[0]) for c in centers], "levels": []}
    for i in range(len(parents)):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        src = leaf if i == 0 else outs[i - 1]
        a.record(stream)
        for _ in range(reps):
            q2x.m2m(src, centers[i], pars[i], centers[i + 1], p, presorted=True, out=outs[i], workspace=wss[i],
                    stream=stream)
        z.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(z) / reps
        nch = len(parents[i])
        fl = flops.m2m_child_flops(p) * nch
        res["levels"].append({"children": nch, "parents": int(centers[i + 1].shape[0]), "call_ms": ms,
                              "translations_per_s": nch / (ms * 1e-3), "tflops": fl / (ms * 1e-3) / 1e12})
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        run_all()
    z.record(stream)
    torch.cuda.synchronize()
    res["upward_pass_ms"] = a.elapsed_time(z) / reps
    res["status_flags"] = [q2x.status(w)[0] for w in wss]
    return res


def near_field(dev, reps=10):
    """Near field of the headline sphere at its collocation points: targets at
    the 81,920 triangle centroids, pairs with every triangle of the 27 boxes
    around the target's box (q2x_near, closed form, FP64), single + double
    layer densities; the unit-density entries (stored near-field matrix) and
    the potentials.  Timed with HIP events."""
    import torch

    from paper_2107_10942_amd import q2x
    from q2x_inputs import configs, octree
    single, double = configs.perturbed_sphere_pair()
    cen = single.verts[single.elems].mean(axis=1)
    ps, pe = octree.near_pairs(single.boxes, single.elem_box, single.elem_box)
    t = lambda a, dt: torch.as_tensor(a, dtype=dt, device=dev).contiguous()  # noqa: E731
    v, e, c = t(single.verts, torch.float64), t(single.elems, torch.int32), t(cen, torch.float64)
    pst, pet = t(ps, torch.int64), t(pe, torch.int32)
    ds, dd = t(single.density, torch.float64), t(double.density, torch.float64)
    npair = int(pe.shape[0])
    eL = torch.empty(npair, dtype=torch.float64, device=dev)
    eM = torch.empty(npair, dtype=torch.float64, device=dev)
    pot = torch.empty(len(cen), dtype=torch.float64, device=dev)
    ws = q2x.alloc_near_workspace(dev)
    stream = torch.cuda.current_stream()
    res = {"workload": f"perturbed icosphere k=6: {len(cen)} collocation targets (centroids), pairs with the "
                       f"triangles of the 27 surrounding level-5 boxes", "pairs": npair}
    for name, kw in (("potentials", dict(entries=False, out_potential=pot)),
                     ("entries_and_potentials", dict(out_entries=(eL, eM), out_potential=pot))):
        call = lambda: q2x.near(v, e, c, pst, pet, ds, dd, workspace=ws, stream=stream, **kw)  # noqa: E731
        for _ in range(2):
            call()
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            call()
        z.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(z) / reps
        res[name] = {"call_ms": ms, "pairs_per_s": npair / (ms * 1e-3)}
    res["status"] = list(q2x.status(ws))
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(the path would shard by Morton box ranges with no communication)"}))
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_calibration:
        n = args.copy_calibration // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n, "launches": 5}))
        return

    from paper_2107_10942_amd import build as libbuild
    from paper_2107_10942_amd import flops, q2x
    from q2x_inputs import configs
    if not os.path.exists(libbuild.LIB):
        libbuild.build(force=False)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    single, double = configs.perturbed_sphere_pair()
    p = single.p
    N = single.n_elems
    B = single.n_boxes
    ts = q2x.job_tensors(single, dev)
    dens2 = torch.as_tensor(double.density, dtype=torch.float64, device=dev)
    outs = {k: torch.empty((B, (p + 1) ** 2, 2), dtype=torch.float64, device=dev) for k in (0, 1)}

    def make_step(prec, fused):
        v, e, d, eb, bc, br = ts
        if fused:
            ws = {q2x.TRI_BOTH: q2x.alloc_workspace(q2x.TRI_BOTH, N, B, p, prec, device=dev)}

            def step():
                q2x.tri_both(v, e, d, dens2, eb, bc, br, p, precision=prec, out_single=outs[0],
                             out_double=outs[1], workspace=ws[q2x.TRI_BOTH])
        else:
            ws = {k: q2x.alloc_workspace(k, N, B, p, prec, device=dev) for k in (0, 1)}

            def step():
                q2x.run(q2x.TRI_SINGLE, v, e, d, eb, bc, br, p, precision=prec, out=outs[0], workspace=ws[0])
                q2x.run(q2x.TRI_DOUBLE, v, e, dens2, eb, bc, br, p, precision=prec, out=outs[1], workspace=ws[1])
        return step, ws

    def timed(prec, fused, steps):
        step, ws = make_step(prec, fused)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # the timed steps run without the library's timing events (they add
        # stream work between the kernels); a second, profiled pass of the
        # same steps gives the per-kernel times
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        q2x.profile_enable(True)
        q2x.profile_reset()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        rec_ms, call_ms, calls = q2x.profile_read()
        q2x.profile_enable(False)
        flags = [q2x.status(w)[0] for w in ws.values()]
        ms = (t1 - t0) * 1e3 / steps
        per_kind = {}
        for k in ws:
            avg = rec_ms[k] / max(calls[k], 1)
            fl = flops.scope_launch_flops(k, p, N)
            fl_lean = flops.launch_flops(k, p, N)
            per_kind[q2x.KIND_NAMES[k]] = {"recursion_kernel_ms": avg, "call_ms": call_ms[k] / max(calls[k], 1),
                                           "algorithmic_flops": fl, "tflops": fl / (avg * 1e-3) / 1e12,
                                           "algorithmic_flops_lean": fl_lean,
                                           "tflops_lean": fl_lean / (avg * 1e-3) / 1e12}
        return {"ms_per_step": ms, "value": coefs / (ms * 1e-3), "per_kind": per_kind, "flags": flags,
                "single": coef_complex(outs[0]), "double": coef_complex(outs[1])}

    coefs = 2 * N * (p + 1) ** 2
    results, separate = {}, {}
    for prec in (q2x.FP32_MIXED, q2x.FP64):
        results[prec] = timed(prec, True, args.steps)
        separate[prec] = timed(prec, False, max(args.steps // 2, 1))
        for layer in ("single", "double"):  # the fused and separate paths give bitwise the same coefficients
            if not np.array_equal(results[prec][layer], separate[prec][layer]):
                raise SystemExit(f"fused and separate {layer}-layer results differ (precision {prec})")

    # The same step with the elements already in box order (Q2X_PRESORTED): what a caller whose
    # element -> box map is fixed across density updates (an iterative solver) pays per step after
    # sorting once.  Reported beside the metric, never as it: the metric's step includes the sort.
    presorted = {}
    v, e, d, eb, bc, br = ts
    perm = q2x.bucket(eb, B)[0].long()
    e_s, d_s, d2_s, eb_s = e[perm].contiguous(), d[perm].contiguous(), dens2[perm].contiguous(), eb[perm].contiguous()
    for prec in (q2x.FP32_MIXED, q2x.FP64):
        ws_s = q2x.alloc_workspace(q2x.TRI_BOTH, N, B, p, prec, device=dev)

        def pstep():
            q2x.tri_both(v, e_s, d_s, d2_s, eb_s, bc, br, p, precision=prec, presorted=True, out_single=outs[0],
                         out_double=outs[1], workspace=ws_s)
        for _ in range(args.warmup):
            pstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pstep()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        same = (np.array_equal(coef_complex(outs[0]), results[prec]["single"])
                and np.array_equal(coef_complex(outs[1]), results[prec]["double"]))
        presorted["fp32_mixed" if prec == q2x.FP32_MIXED else "fp64"] = {
            "ms_per_step": ms, "coefficients_per_s": coefs / (ms * 1e-3), "equals_sorting_step": bool(same)}

    mixed, plain = results[q2x.FP32_MIXED], results[q2x.FP64]
    # agreement of the two GPU precisions (scale-free check; parity vs the oracle is in tests/)
    agree = {}
    for layer in ("single", "double"):
        d = np.abs(mixed[layer] - plain[layer]).max()
        agree[layer] = float(d / max(np.abs(plain[layer]).max(), 1e-300))

    dom_name = max(mixed["per_kind"], key=lambda k: mixed["per_kind"][k]["recursion_kernel_ms"])
    dom = mixed["per_kind"][dom_name]
    peak = flops.PEAK_FP32_TFLOPS
    peak64 = flops.PEAK_FP64_TFLOPS
    traffic = stored_traffic("q2x_tile_kernel_tri_both_p16_perturbed_sphere_81920_traffic.md", libbuild.source_hash())
    roof = {"bound": "alu", "kernel": f"q2x_tile_kernel<16,{dom_name},float>", "achieved": dom["tflops"],
            "peak": peak, "unit": "TFLOP/s", "frac": dom["tflops"] / peak, "traffic": traffic,
            "launch_ms": dom["recursion_kernel_ms"], "flops_per_launch": dom["algorithmic_flops"],
            "flop_model": "recursion of Eqs. (50)-(56) as written (complex products with xi, eta at 8 FLOPs), "
                          "plus 4 FLOPs per output coefficient for the FP64 weight and box sum",
            "achieved_lean": dom["tflops_lean"], "frac_lean": dom["tflops_lean"] / peak,
            "flops_per_launch_lean": dom["algorithmic_flops_lean"],
            "flop_model_lean": "operation-by-operation count using the conjugate pair xi, eta "
                               "(paper_2107_10942_amd/flops.py element_flops)",
            "algorithmic_bytes_per_launch": flops.launch_bytes(q2x.TRI_BOTH, p, N, B)}
    fp64_dom = plain["per_kind"][dom_name]

    # the GPU's own peaks, measured (the published ones are the roofline's denominators)
    buf = torch.empty(1 << 31, dtype=torch.uint8, device=dev)
    mp = {"fp64_fma_tflops": q2x.peak_measure(q2x.PEAK_FMA64, buf)[0],
          "fp32_fma_tflops": q2x.peak_measure(q2x.PEAK_FMA32, buf)[0],
          "hbm_copy_gbs": q2x.peak_measure(q2x.PEAK_HBM_COPY, buf)[0],
          "method": "q2x_peak_measure: 8 independent FMA chains per lane on 16 waves per SIMD (FP32 non-packed); "
                    "a 1 GiB float4 copy (read + written bytes)"}
    del buf
    roof["frac_of_measured_peak"] = dom["tflops"] / mp["fp32_fma_tflops"]
    roof["peak_basis"] = ("published FP32 vector peak; plain (non-packed) FP32 FMA issues at twice the FP64 rate on "
                          "this GPU (measured_peaks.fp32_fma_tflops)")

    line = {
        "metric": "Q2X coefficients/s at p=16, FP32-mixed vs FP64 plain; serving p50/p99 latency",
        "value": mixed["value"], "unit": "coefficients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 recursion, f64 geometry+accumulation",
        "data": "synthetic",
        "config": {"workload": "perturbed icosphere k=6, 81,920 triangles, radii 1+0.1N(0,1) smoothed, "
                               "octree level 5, single+double layer, p=16",
                   "n_elements": N, "n_boxes": B, "p": p, "elements_per_step": 2 * N,
                   "coefficients_per_step": 2 * N * (p + 1) ** 2, "precision": "FP32-mixed"},
        "fp64_value": plain["value"], "fp64_ms_per_step": plain["ms_per_step"],
        "fp64_plain": {"value": plain["value"], "ms_per_step": plain["ms_per_step"], "per_kind": plain["per_kind"],
                       "kernel_peak_tflops": peak64, "kernel_frac": fp64_dom["tflops"] / peak64,
                       "kernel_frac_lean": fp64_dom["tflops_lean"] / peak64},
        "kernel_speedup_mixed_vs_fp64": fp64_dom["recursion_kernel_ms"] / dom["recursion_kernel_ms"],
        "separate_calls": {"fp32_mixed_ms_per_step": separate[q2x.FP32_MIXED]["ms_per_step"],
                           "fp64_ms_per_step": separate[q2x.FP64]["ms_per_step"],
                           "per_kind_mixed": separate[q2x.FP32_MIXED]["per_kind"]},
        "speedup_mixed_vs_fp64": plain["ms_per_step"] / mixed["ms_per_step"],
        "presorted_elements": presorted,
        # box coefficients written per second (occupied boxes x (p+1)^2, both layers)
        "box_coefficients_per_s": {"fp32_mixed": 2 * B * (p + 1) ** 2 / (mixed["ms_per_step"] * 1e-3),
                                   "fp64": 2 * B * (p + 1) ** 2 / (plain["ms_per_step"] * 1e-3)},
        "per_kind_mixed": mixed["per_kind"],
        "mixed_vs_fp64_max_rel_diff": agree,
        "status_flags": {"mixed": mixed["flags"], "fp64": plain["flags"]},
        "roofline": roof,
        "measured_peaks": mp,
    }

    if not args.no_large:
        big = configs.large_sphere()
        tb = q2x.job_tensors(big, dev)
        ob = torch.empty((big.n_boxes, (big.p + 1) ** 2, 2), dtype=torch.float64, device=dev)
        lg = {}
        for prec in (q2x.FP32_MIXED, q2x.FP64):
            wsb = q2x.alloc_workspace(big.kind, big.n_elems, big.n_boxes, big.p, prec, device=dev)
            for _ in range(2):
                q2x.run(big.kind, *tb, big.p, precision=prec, out=ob, workspace=wsb)
            torch.cuda.synchronize()
            reps = 10
            t0 = time.perf_counter()
            for _ in range(reps):
                q2x.run(big.kind, *tb, big.p, precision=prec, out=ob, workspace=wsb)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            q2x.profile_enable(True)  # kernel times from a second, profiled pass
            q2x.profile_reset()
            for _ in range(reps):
                q2x.run(big.kind, *tb, big.p, precision=prec, out=ob, workspace=wsb)
            torch.cuda.synchronize()
            rec_ms, call_ms, calls = q2x.profile_read()
            q2x.profile_enable(False)
            k = big.kind
            avg = rec_ms[k] / calls[k]
            vpk = flops.peak_valu_tflops(prec == q2x.FP32_MIXED)
            fl = flops.scope_launch_flops(k, big.p, big.n_elems)
            fl_lean = flops.launch_flops(k, big.p, big.n_elems)
            lg["fp32_mixed" if prec == q2x.FP32_MIXED else "fp64"] = {
                "recursion_kernel_ms": avg, "call_ms": call_ms[k] / calls[k],
                "coefficients_per_s": big.n_elems * (big.p + 1) ** 2 / ((t1 - t0) / reps),
                "tflops": fl / (avg * 1e-3) / 1e12, "frac_of_valu_peak": fl / (avg * 1e-3) / 1e12 / vpk,
                "frac_of_valu_peak_lean": fl_lean / (avg * 1e-3) / 1e12 / vpk}
        line["large_workload"] = {"workload": f"icosphere k=8, {big.n_elems} triangles, level 7, "
                                              f"{big.n_boxes} boxes, single layer, p=16", **lg}

    if not args.no_configs:
        line["other_workloads"] = other_workloads(dev)
        line["receiving_side"] = receiving_side(dev)
        line["upward_pass"] = upward_pass(dev)
        line["near_field"] = near_field(dev)
    if not args.no_batch:
        line["batch_workload"] = batch_workload(dev)
    if not args.no_serving:
        line["serving_workload"] = serving_workload(dev, args.serving_requests)

    if not args.no_cpu_baseline:
        import oracle
        nthr = oracle.max_threads()
        # calibrate on every 40th box, then size the sample for ~cpu_seconds
        refs = {}

        def run_sample(stride):
            bx = np.arange(0, B, stride)
            keep = np.isin(single.elem_box, bx)
            ne = int(keep.sum())
            t0 = time.perf_counter()
            for job in (single, double):
                refs[job.kind] = oracle.q2x(job.kind, p, job.verts, job.elems[keep], job.density[keep],
                                            job.elem_box[keep], job.box_center, boxes=bx)
            return ne, time.perf_counter() - t0, len(bx)
        ne, dt, nbx = run_sample(40)
        rate = 2 * ne / dt  # elements per second (both layers)
        stride = max(1, int(math.ceil(2 * N / max(rate * args.cpu_seconds, 1.0))))
        if stride < 40:
            ne, dt, nbx = run_sample(stride)
        line["cpu_baseline"] = {"value": 2 * ne * (p + 1) ** 2 / dt, "unit": "coefficients/s", "cores": nthr,
                                "kind": "oracle",
                                "sample": f"every {stride}th box ({nbx} boxes, {ne} triangles) of the same mesh, "
                                          f"single+double layer, p=16, FP64 Gauss/Duffy quadrature, {dt:.1f} s"}
        # error table of the timed GPU results against the oracle on the same boxes
        bx = np.arange(0, B, stride)
        keep = np.isin(single.elem_box, bx)
        table = {}
        for name, res in (("fp32_mixed", mixed), ("fp64", plain)):
            for job, layer in ((single, "single"), (double, "double")):
                en = oracle.element_norms(job.kind, p, job.verts, job.elems[keep], job.elem_box[keep], job.box_center)
                table[f"{name}_{layer}"] = error_stats(res[layer][bx], refs[job.kind], en, job.density[keep],
                                                       job.elem_box[keep], bx, p)
        line["cpu_baseline"]["error_vs_oracle"] = table
        line["cpu_baseline"]["other_workloads"] = cpu_other_workloads(nthr, args.cpu_seconds / 4)
        # the same oracle on one thread, on every 40th box (context for the all-core figure;
        # last, as the thread count it sets stays in force)
        bx1 = np.arange(0, B, 40)
        keep1 = np.isin(single.elem_box, bx1)
        t0 = time.perf_counter()
        for job in (single, double):
            oracle.q2x(job.kind, p, job.verts, job.elems[keep1], job.density[keep1], job.elem_box[keep1],
                       job.box_center, boxes=bx1, threads=1)
        dt1 = time.perf_counter() - t0
        line["cpu_baseline"]["one_thread"] = {"value": 2 * int(keep1.sum()) * (p + 1) ** 2 / dt1,
                                              "unit": "coefficients/s", "cores": 1,
                                              "sample": f"every 40th box ({len(bx1)} boxes, {int(keep1.sum())} "
                                                        f"triangles), {dt1:.1f} s"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

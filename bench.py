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


def coef_complex(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


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
        q2x.profile_enable(True)
        q2x.profile_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rec_ms, call_ms, calls = q2x.profile_read()
        q2x.profile_enable(False)
        flags = [q2x.status(w)[0] for w in ws.values()]
        ms = (t1 - t0) * 1e3 / steps
        per_kind = {}
        for k in ws:
            avg = rec_ms[k] / max(calls[k], 1)
            fl = flops.launch_flops(k, p, N)
            per_kind[q2x.KIND_NAMES[k]] = {"recursion_kernel_ms": avg, "call_ms": call_ms[k] / max(calls[k], 1),
                                           "algorithmic_flops": fl, "tflops": fl / (avg * 1e-3) / 1e12}
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

    mixed, plain = results[q2x.FP32_MIXED], results[q2x.FP64]
    # agreement of the two GPU precisions (scale-free check; parity vs the oracle is in tests/)
    agree = {}
    for layer in ("single", "double"):
        d = np.abs(mixed[layer] - plain[layer]).max()
        agree[layer] = float(d / max(np.abs(plain[layer]).max(), 1e-300))

    dom_name = max(mixed["per_kind"], key=lambda k: mixed["per_kind"][k]["recursion_kernel_ms"])
    dom = mixed["per_kind"][dom_name]
    peak = flops.PEAK_VALU_TFLOPS
    traffic = stored_traffic("q2x_tile_kernel_tri_both_p16_perturbed_sphere_81920_traffic.md", libbuild.source_hash())
    roof = {"bound": "alu", "kernel": f"q2x_tile_kernel<16,{dom_name},float>", "achieved": dom["tflops"],
            "peak": peak, "unit": "TFLOP/s", "frac": dom["tflops"] / peak, "traffic": traffic,
            "launch_ms": dom["recursion_kernel_ms"], "flops_per_launch": dom["algorithmic_flops"],
            "algorithmic_bytes_per_launch": flops.launch_bytes(q2x.TRI_BOTH, p, N, B)}

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
        "fp64_plain": {"value": plain["value"], "ms_per_step": plain["ms_per_step"], "per_kind": plain["per_kind"]},
        "separate_calls": {"fp32_mixed_ms_per_step": separate[q2x.FP32_MIXED]["ms_per_step"],
                           "fp64_ms_per_step": separate[q2x.FP64]["ms_per_step"],
                           "per_kind_mixed": separate[q2x.FP32_MIXED]["per_kind"]},
        "speedup_mixed_vs_fp64": plain["ms_per_step"] / mixed["ms_per_step"],
        "per_kind_mixed": mixed["per_kind"],
        "mixed_vs_fp64_max_rel_diff": agree,
        "status_flags": {"mixed": mixed["flags"], "fp64": plain["flags"]},
        "roofline": roof,
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
            q2x.profile_enable(True)
            q2x.profile_reset()
            reps = 10
            t0 = time.perf_counter()
            for _ in range(reps):
                q2x.run(big.kind, *tb, big.p, precision=prec, out=ob, workspace=wsb)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rec_ms, call_ms, calls = q2x.profile_read()
            q2x.profile_enable(False)
            k = big.kind
            avg = rec_ms[k] / calls[k]
            fl = flops.launch_flops(k, big.p, big.n_elems)
            lg["fp32_mixed" if prec == q2x.FP32_MIXED else "fp64"] = {
                "recursion_kernel_ms": avg, "call_ms": call_ms[k] / calls[k],
                "coefficients_per_s": big.n_elems * (big.p + 1) ** 2 / ((t1 - t0) / reps),
                "tflops": fl / (avg * 1e-3) / 1e12, "frac_of_valu_peak": fl / (avg * 1e-3) / 1e12 / peak}
        line["large_workload"] = {"workload": f"icosphere k=8, {big.n_elems} triangles, level 7, "
                                              f"{big.n_boxes} boxes, single layer, p=16", **lg}

    if not args.no_cpu_baseline:
        import oracle
        nthr = oracle.max_threads()
        # calibrate on every 40th box, then size the sample for ~cpu_seconds
        def run_sample(stride):
            bx = np.arange(0, B, stride)
            keep = np.isin(single.elem_box, bx)
            ne = int(keep.sum())
            t0 = time.perf_counter()
            for job in (single, double):
                oracle.q2x(job.kind, p, job.verts, job.elems[keep], job.density[keep], job.elem_box[keep],
                           job.box_center, boxes=bx)
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""GPU tests of the batch path (q2x_batch_plan / q2x_batch_run): every job's
coefficients and status equal the single call's, bitwise, on the first run
and on graph replays (with other device work and changed inputs between
them); accumulation; the uneven many-mesh workload at reduced size."""
import numpy as np
import pytest

from gpu_util import FP32_MIXED, FP64, small_job

pytestmark = pytest.mark.gpu


def _c(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def _tensors(job):
    from paper_2107_10942_amd import q2x
    v, e, d, eb, bc, br = q2x.job_tensors(job)
    return dict(kind=job.kind, verts=v, elems=e, density=d, elem_box=eb, box_center=bc, p=job.p)


def _single(spec, prec):
    import torch
    from paper_2107_10942_amd import q2x
    ws = q2x.alloc_workspace(spec["kind"], int(spec["elems"].shape[0]), int(spec["box_center"].shape[0]),
                             spec["p"], prec)
    if spec["kind"] == q2x.TRI_BOTH:
        o1, o2 = q2x.tri_both(spec["verts"], spec["elems"], spec["density"], spec["density2"], spec["elem_box"],
                              spec["box_center"], None, spec["p"], precision=prec, workspace=ws)
        out = (_c(o1), _c(o2))
    else:
        o = q2x.run(spec["kind"], spec["verts"], spec["elems"], spec["density"], spec["elem_box"],
                    spec["box_center"], None, spec["p"], precision=prec, workspace=ws)
        out = _c(o)
    st = q2x.status(ws)
    torch.cuda.synchronize()
    return out, st


def _mixed_specs():
    """Jobs of every kind, orders inside and between buckets, both precisions,
    bad box ids, empty boxes, an empty job."""
    import torch
    from paper_2107_10942_amd import q2x
    specs = []
    plan = [(0, 517, 40, 16, FP32_MIXED), (1, 300, 12, 9, FP64), (2, 777, 30, 13, FP32_MIXED),
            (3, 200, 20, 4, FP64), (0, 1500, 70, 20, FP64), (1, 640, 25, 16, FP32_MIXED),
            (3, 900, 35, 12, FP32_MIXED), (2, 64, 3, 0, FP64), (0, 129, 8, 32, FP32_MIXED),
            (0, 0, 5, 8, FP32_MIXED), (4, 420, 18, 11, FP32_MIXED), (4, 333, 9, 16, FP64)]
    for i, (kind, n, nb, p, prec) in enumerate(plan):
        job = small_job(kind if kind != 4 else 0, max(n, 1), nb, p, seed=900 + i)
        spec = _tensors(job)
        spec["kind"] = kind
        spec["precision"] = prec
        if n == 0:
            spec["elems"] = spec["elems"][:0]
            spec["density"] = spec["density"][:0]
            spec["elem_box"] = spec["elem_box"][:0]
        if kind == 4:
            spec["density2"] = torch.as_tensor(np.random.default_rng(i).uniform(-1, 1, job.n_elems),
                                               dtype=torch.float64).cuda()
        if i == 1:  # two bad box ids
            eb = spec["elem_box"].clone()
            eb[3] = -2
            eb[10] = nb + 5
            spec["elem_box"] = eb
        specs.append(spec)
    return specs


def _compare(plan, specs, outs):
    from paper_2107_10942_amd import q2x
    for j, spec in enumerate(specs):
        ref, st = _single(spec, spec["precision"])
        got = outs[j]
        if spec["kind"] == q2x.TRI_BOTH:
            assert np.array_equal(_c(got[0]), ref[0]), j
            assert np.array_equal(_c(got[1]), ref[1]), j
        else:
            assert np.array_equal(_c(got), ref), (j, spec["kind"], spec["p"])
        assert plan.status(j) == st, (j, plan.status(j), st)


def test_batch_equals_single_calls_and_replays():
    import torch
    from paper_2107_10942_amd import q2x
    specs = _mixed_specs()
    plan = q2x.BatchPlan(specs)
    assert plan.groups >= 8
    outs = plan.run()
    torch.cuda.synchronize()
    assert plan.mode in (0, 1)
    print("groups", plan.groups, "mode", plan.mode, flush=True)
    _compare(plan, specs, outs)
    # replays: other device work in between, then new densities (same buffers)
    for r in range(3):
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()
        for j, spec in enumerate(specs):
            if spec["density"].numel():
                spec["density"].copy_(torch.as_tensor(np.random.default_rng(100 * r + j).uniform(
                    -1, 1, spec["density"].numel()), dtype=torch.float64))
        plan.run()
        torch.cuda.synchronize()
        _compare(plan, specs, outs)
    plan.close()


def test_batch_accumulate_and_bad_ids_counted():
    import torch
    from paper_2107_10942_amd import q2x
    specs = _mixed_specs()[:6]
    ref = [_single(s, s["precision"])[0] for s in specs]
    for s in specs:
        s["accumulate"] = True
        s["out"] = torch.full((s["box_center"].shape[0], (s["p"] + 1) ** 2, 2), 0.5, dtype=torch.float64,
                              device="cuda")
    plan = q2x.BatchPlan(specs)
    outs = plan.run()
    torch.cuda.synchronize()
    assert plan.mode == 0  # accumulating plans are not timed
    for j, s in enumerate(specs):
        got = _c(outs[j])
        np.testing.assert_allclose(got, ref[j] + (0.5 + 0.5j), rtol=0,
                                   atol=1e-15 * max(np.max(np.abs(ref[j])), 1.0))
    f, d, k = plan.status(1)
    assert f & q2x.FLAG_BAD_BOX and k == 2
    plan.close()


def test_uneven_many_mesh_batch_reduced():
    """The many-mesh workload (perturbed spheres and ellipsoids, sizes
    log-uniform, p in {4, 8, 12, 16, 20}, single/double) at 1/20 of its
    element counts, 64 meshes: batched (FP32-mixed and FP64) == single calls."""
    import torch
    from paper_2107_10942_amd import q2x
    from q2x_inputs import configs
    jobs = configs.batch_meshes(n_meshes=64, scale=0.05)
    for prec in (FP32_MIXED, FP64):
        specs = []
        for job in jobs:
            s = _tensors(job)
            s["precision"] = prec
            specs.append(s)
        plan = q2x.BatchPlan(specs)
        outs = plan.run()
        plan.run()
        torch.cuda.synchronize()
        print("prec", prec, "groups", plan.groups, "mode", plan.mode, "elements",
              sum(j.n_elems for j in jobs), flush=True)
        _compare(plan, specs, outs)
        plan.close()


def test_batch_jobs_against_the_oracle():
    """Every job of a mixed batch (all four element kinds and the fused single
    + double layer, both precisions, orders inside and between the compiled
    buckets) against the CPU oracle on a seeded sample of its boxes, to the
    parity bar of its precision -- not only against the single calls."""
    import torch
    import metrics
    from gpu_util import TOL, oracle_ref, scale, sample_boxes, sub_job
    from paper_2107_10942_amd import q2x
    from q2x_inputs import configs
    plan_jobs = [(0, 2100, 60, 16, FP32_MIXED), (1, 900, 25, 9, FP64), (2, 1300, 30, 13, FP32_MIXED),
                 (3, 700, 40, 12, FP64), (4, 1000, 33, 16, FP32_MIXED), (3, 500, 20, 20, FP32_MIXED),
                 (1, 800, 30, 24, FP32_MIXED), (4, 600, 21, 8, FP64)]
    jobs, specs = [], []
    for i, (kind, n, nb, p, prec) in enumerate(plan_jobs):
        job = small_job(kind if kind != 4 else 0, n, nb, p, seed=700 + i)
        spec = _tensors(job)
        spec["kind"] = kind
        spec["precision"] = prec
        d2 = None
        if kind == 4:
            d2 = np.random.default_rng(70 + i).uniform(-1, 1, job.n_elems)
            spec["density2"] = torch.as_tensor(d2, dtype=torch.float64).cuda()
        jobs.append((job, d2))
        specs.append(spec)
    plan = q2x.BatchPlan(specs)
    outs = plan.run()
    torch.cuda.synchronize()
    for j, ((job, d2), spec) in enumerate(zip(jobs, specs)):
        boxes = sample_boxes(job, 10, seed=j)
        sub = sub_job(job, boxes)
        layers = [(0 if spec["kind"] == 4 else spec["kind"], sub.density, outs[j][0] if spec["kind"] == 4 else outs[j])]
        if spec["kind"] == 4:
            keep = np.isin(job.elem_box, boxes)
            layers.append((1, d2[keep], outs[j][1]))
        for kind, dens, out in layers:
            sj = configs.Job(name="s", kind=kind, p=job.p, verts=sub.verts, elems=sub.elems, density=dens,
                             boxes=sub.boxes)
            R = oracle_ref(sj, boxes=boxes)
            A = scale(sj, boxes=boxes)
            err = float(np.max(metrics.scale_aware_error(_c(out)[boxes], R, A, job.p)))
            print(f"batch job {j} kind {kind} p {job.p} prec {spec['precision']} err {err:.2e}", flush=True)
            assert err <= TOL[spec["precision"]], (j, kind, err)
        assert plan.status(j)[0] == 0
    plan.close()


@pytest.mark.parametrize("sched", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 1024), (0, 0, 2 ** 31 - 1),
                                   (1, 1, 2 ** 31 - 1)])
def test_every_schedule_equals_single_calls(sched):
    """A forced schedule (capture mode, split tiles, merged order buckets)
    changes no bit of any job's coefficients or status."""
    import torch
    from paper_2107_10942_amd import q2x
    specs = _mixed_specs()
    plan = q2x.BatchPlan(specs)
    g0 = plan.groups
    plan.set_schedule(*sched)
    sc = plan.schedule
    assert (sc["mode"], sc["split"], sc["merge"], sc["tuned"]) == (*sched, 2)
    if sched[2] == q2x.MERGE_ALL:
        # one group per (kind, precision) present
        assert plan.groups == len({(s["kind"], s["precision"]) for s in specs}) < g0
    outs = plan.run()
    torch.cuda.synchronize()
    assert plan.mode == sched[0]
    _compare(plan, specs, outs)
    plan.close()


def test_tuning_is_cached_and_persisted(tmp_path):
    """The first run times the candidate schedules and caches the winner
    (keyed by device, library build and plan shape); a second plan of the
    same shape takes it from the cache; a saved cache file reloads, and an
    entry edited in the file is the schedule a new plan then uses."""
    import torch
    from paper_2107_10942_amd import q2x
    specs = _mixed_specs()
    plan = q2x.BatchPlan(specs)
    outs = plan.run()
    torch.cuda.synchronize()
    sc = plan.schedule
    assert sc["tuned"] == 1, sc
    _compare(plan, specs, outs)
    path = tmp_path / "tune.txt"
    q2x.tune_cache_save(path)
    lines = path.read_text().splitlines()
    mine = [ln for ln in lines if ("|" + q2x.build_id() + "|") in ln]
    assert mine, lines
    plan2 = q2x.BatchPlan(specs)
    plan2.run()
    torch.cuda.synchronize()
    assert plan2.schedule == sc
    # edit the entries of this build to another schedule and reload
    want = (1 - sc["mode"], 1 - sc["split"], 0 if sc["merge"] else q2x.MERGE_ALL)
    edited = [ln.split("\t")[0] + "\t%d %d %d" % want if ("|" + q2x.build_id() + "|") in ln else ln for ln in lines]
    path.write_text("\n".join(edited) + "\n")
    q2x.tune_cache_load(path)
    plan3 = q2x.BatchPlan(specs)
    outs3 = plan3.run()
    torch.cuda.synchronize()
    s3 = plan3.schedule
    assert (s3["mode"], s3["split"], s3["merge"], s3["tuned"]) == (*want, 1), s3
    _compare(plan3, specs, outs3)
    for p in (plan, plan2, plan3):
        p.close()

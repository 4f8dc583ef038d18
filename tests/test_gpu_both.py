"""GPU parity of the fused single + double layer entry point (q2x_tri_both):
each output against the oracle of its own layer, and bitwise against the two
separate entry points on the same inputs."""
import numpy as np
import pytest

from gpu_util import FP32_MIXED, FP64, TOL, sample_boxes, scale, small_job, sub_job
import metrics
import oracle

pytestmark = pytest.mark.gpu


def _as_complex(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def _both(job, dens2, prec, p=None, norm=0, presorted=False, accumulate=False, outs=(None, None)):
    import torch
    from paper_2107_10942_amd import q2x
    p = job.p if p is None else p
    v, e, d, eb, bc, br = q2x.job_tensors(job)
    d2 = torch.as_tensor(dens2, dtype=torch.float64).cuda()
    ws = q2x.alloc_workspace(q2x.TRI_BOTH, job.n_elems, job.n_boxes, p, prec)
    o1, o2 = q2x.tri_both(v, e, d, d2, eb, bc, br, p, precision=prec, norm=norm, presorted=presorted,
                          accumulate=accumulate, out_single=outs[0], out_double=outs[1], workspace=ws)
    st = q2x.status(ws)
    torch.cuda.synchronize()
    return _as_complex(o1), _as_complex(o2), st


def _separate(job, dens2, prec, p=None):
    import torch
    from paper_2107_10942_amd import q2x
    p = job.p if p is None else p
    v, e, d, eb, bc, br = q2x.job_tensors(job)
    d2 = torch.as_tensor(dens2, dtype=torch.float64).cuda()
    o1 = q2x.tri_single(v, e, d, eb, bc, br, p, precision=prec)
    o2 = q2x.tri_double(v, e, d2, eb, bc, br, p, precision=prec)
    torch.cuda.synchronize()
    return _as_complex(o1), _as_complex(o2)


def _refs(job, dens2, p, norm=0, boxes=None):
    R1 = oracle.q2x(0, p, job.verts, job.elems, job.density, job.elem_box, job.box_center, norm=norm, boxes=boxes)
    R2 = oracle.q2x(1, p, job.verts, job.elems, dens2, job.elem_box, job.box_center, norm=norm, boxes=boxes)
    en1 = oracle.element_norms(0, p, job.verts, job.elems, job.elem_box, job.box_center)
    en2 = oracle.element_norms(1, p, job.verts, job.elems, job.elem_box, job.box_center)
    A1 = metrics.scale_denominator(en1, job.density, job.elem_box, job.n_boxes, boxes)
    A2 = metrics.scale_denominator(en2, dens2, job.elem_box, job.n_boxes, boxes)
    return R1, R2, A1, A2


def _worst(F, R, A, p, prec, label):
    err = metrics.scale_aware_error(F, R, A, p)
    worst = float(np.max(err)) if err.size else 0.0
    print(f"{label} scale-aware max {worst:.3e}", flush=True)
    assert np.all(np.isfinite(F))
    assert worst <= TOL[prec], (label, worst)


@pytest.mark.parametrize("prec", [FP64, FP32_MIXED])
@pytest.mark.parametrize("p", [0, 1, 2, 5, 8, 11, 16, 21, 24, 32])
def test_both_small_parity_and_bitwise(prec, p):
    """Ragged N, a box cut by several tile edges, empty boxes; every order
    bucket and orders between buckets (the fused chunks hold 2(n+1)
    coefficients per degree, so their boundaries differ from the one-output
    kernels)."""
    job = small_job(0, 533, 40, p, seed=500 + p)
    dens2 = np.random.default_rng(p).uniform(-1, 1, job.n_elems)
    F1, F2, st = _both(job, dens2, prec)
    assert st == (0, 0, 0)
    R1, R2, A1, A2 = _refs(job, dens2, p)
    _worst(F1, R1, A1, p, prec, f"both/single p={p} prec={prec}")
    _worst(F2, R2, A2, p, prec, f"both/double p={p} prec={prec}")
    S1, S2 = _separate(job, dens2, prec)
    assert np.array_equal(F1, S1)
    assert np.array_equal(F2, S2)
    assert np.all(F2[:, 0] == 0)
    empty = np.nonzero(job.boxes.counts == 0)[0]
    assert np.all(F1[empty] == 0) and np.all(F2[empty] == 0)


def test_both_moment_accumulate_presorted():
    import torch
    job = small_job(0, 700, 25, 9, seed=77)
    dens2 = np.random.default_rng(1).uniform(-1, 1, job.n_elems)
    F1, F2, _ = _both(job, dens2, FP64, norm=1)
    R1, R2, A1, A2 = _refs(job, dens2, 9, norm=1)
    _worst(F1, R1, 4 * np.pi * A1, 9, FP64, "both moment single")
    _worst(F2, R2, 4 * np.pi * A2, 9, FP64, "both moment double")
    # accumulate adds into both outputs
    G1, G2, _ = _both(job, dens2, FP64)
    o1 = torch.full((job.n_boxes, 100, 2), 0.25, dtype=torch.float64, device="cuda")
    o2 = torch.full((job.n_boxes, 100, 2), -0.5, dtype=torch.float64, device="cuda")
    H1, H2, _ = _both(job, dens2, FP64, accumulate=True, outs=(o1, o2))
    np.testing.assert_allclose(H1, G1 + (0.25 + 0.25j), rtol=0, atol=1e-15 * np.max(np.abs(G1)) + 1e-15)
    np.testing.assert_allclose(H2, G2 + (-0.5 - 0.5j), rtol=0, atol=1e-15 * np.max(np.abs(G2)) + 1e-15)
    # presorted input gives bitwise the same result as the internal bucketing
    from q2x_inputs import configs, octree
    order = np.argsort(job.elem_box, kind="stable")
    bx = octree.Boxes(level=0, lo=-1, half=1, h=0.25, elem_box=job.elem_box[order], center=job.box_center,
                      radius=job.box_radius, morton=job.boxes.morton, counts=job.boxes.counts)
    js = configs.Job(name="sorted", kind=0, p=9, verts=job.verts, elems=job.elems[order],
                     density=job.density[order], boxes=bx)
    P1, P2, st = _both(js, dens2[order], FP64, presorted=True)
    assert st[0] == 0
    assert np.array_equal(P1, G1) and np.array_equal(P2, G2)


def test_both_rejects_overlapping_outputs():
    import torch
    from paper_2107_10942_amd import q2x
    job = small_job(0, 100, 8, 4, seed=3)
    v, e, d, eb, bc, br = q2x.job_tensors(job)
    o = torch.empty((job.n_boxes, 25, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(q2x.Q2XError):
        q2x.tri_both(v, e, d, d, eb, bc, br, 4, out_single=o, out_double=o)


@pytest.mark.parametrize("prec", [FP64, FP32_MIXED])
def test_both_perturbed_sphere_sampled(prec):
    """81,920-triangle perturbed sphere, level 5, p = 16, both layers in the
    fused launch the benchmark times; oracle on a box sample, full output
    bitwise against the separate entry points."""
    from q2x_inputs import configs
    a, b = configs.perturbed_sphere_pair()
    F1, F2, st = _both(a, b.density, prec)
    assert st == (0, 0, 0)
    boxes = sample_boxes(a, 100, seed=5)
    sa = sub_job(a, boxes)
    keep = np.isin(a.elem_box, boxes)
    R1, R2, A1, A2 = _refs(sa, b.density[keep], a.p, boxes=boxes)
    _worst(F1[boxes], R1, A1, a.p, prec, f"perturbed both/single prec={prec}")
    _worst(F2[boxes], R2, A2, a.p, prec, f"perturbed both/double prec={prec}")
    S1, S2 = _separate(a, b.density, prec)
    assert np.array_equal(F1, S1) and np.array_equal(F2, S2)

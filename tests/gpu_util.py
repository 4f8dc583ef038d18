"""Shared helpers of the GPU tests: seeded small jobs, device runs, oracle
references and the parity bar."""
import numpy as np

import metrics
import oracle
from q2x_inputs import configs, octree

FP64, FP32_MIXED = 0, 1
# parity bar on the scale-aware per-(box, degree) error
TOL = {FP64: 1e-12, FP32_MIXED: 1e-5}
NV = {0: 3, 1: 3, 2: 2, 3: 4}


def small_job(kind, n_elems, n_boxes, p, seed=0, empty_boxes=3, big_box=150, elem_scale=0.35, level_h=0.25):
    """Random simplices grouped in boxes of very uneven size: one box larger
    than two tiles, a few empty boxes, the rest random; elements lie in and
    around their box (offsets up to ~1 box size)."""
    rng = np.random.default_rng(seed)
    side = int(np.ceil(n_boxes ** (1 / 3))) + 1
    ids = rng.choice(side ** 3, size=n_boxes, replace=False)
    ijk = np.stack(np.unravel_index(ids, (side, side, side)), 1)
    centers = -1 + (ijk + 0.5) * level_h
    radius = np.full(n_boxes, np.sqrt(3) * level_h / 2)
    occupied = np.arange(n_boxes)[empty_boxes:] if n_boxes > empty_boxes else np.arange(n_boxes)
    eb = np.empty(n_elems, dtype=np.int32)
    nbig = min(big_box, n_elems // 2) if len(occupied) > 1 else n_elems
    eb[:nbig] = occupied[0]
    if n_elems > nbig:
        w = rng.pareto(1.2, size=len(occupied)) + 0.05
        eb[nbig:] = rng.choice(occupied, size=n_elems - nbig, p=w / w.sum())
    rng.shuffle(eb)
    k = NV[kind]
    base = centers[eb] + rng.uniform(-0.5, 0.5, size=(n_elems, 3)) * level_h
    verts = (base[:, None, :] + rng.normal(size=(n_elems, k, 3)) * elem_scale * level_h / 2).reshape(-1, 3)
    elems = np.arange(n_elems * k, dtype=np.int32).reshape(n_elems, k)
    # shuffle vertex storage so that gathers are irregular
    perm = rng.permutation(verts.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    verts = verts[perm]
    elems = inv[elems].astype(np.int32)
    dens = rng.uniform(-1, 1, n_elems)
    bx = octree.Boxes(level=0, lo=-1.0, half=1.0, h=level_h, elem_box=eb, center=centers, radius=radius,
                      morton=np.arange(n_boxes), counts=np.bincount(eb, minlength=n_boxes))
    return configs.Job(name=f"small_k{kind}_{n_elems}", kind=kind, p=p, verts=verts, elems=elems, density=dens,
                       boxes=bx)


def run_gpu(job, prec, p=None, norm=0, presorted=False, accumulate=False, out=None, radius=None):
    import torch
    from paper_2107_10942_amd import q2x
    p = job.p if p is None else p
    v, e, d, eb, bc, br = q2x.job_tensors(job)
    if radius is not None:
        br = torch.as_tensor(radius, dtype=torch.float64).cuda()
    ws = q2x.alloc_workspace(job.kind, job.n_elems, job.n_boxes, p, prec)
    o = q2x.run(job.kind, v, e, d, eb, bc, br, p, precision=prec, norm=norm, presorted=presorted,
                accumulate=accumulate, out=out, workspace=ws)
    st = q2x.status(ws)
    torch.cuda.synchronize()
    a = o.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1], st


def oracle_ref(job, p=None, norm=0, boxes=None):
    p = job.p if p is None else p
    return oracle.q2x(job.kind, p, job.verts, job.elems, job.density, job.elem_box, job.box_center, norm=norm,
                      boxes=boxes)


def scale(job, p=None, boxes=None):
    p = job.p if p is None else p
    en = oracle.element_norms(job.kind, p, job.verts, job.elems, job.elem_box, job.box_center)
    return metrics.scale_denominator(en, job.density, job.elem_box, job.n_boxes, boxes)


def sample_boxes(job, n, seed=0):
    """A seeded sample of boxes that always includes the fullest box."""
    rng = np.random.default_rng(seed)
    nb = job.n_boxes
    pick = rng.choice(nb, size=min(n, nb), replace=False)
    full = int(np.argmax(job.boxes.counts))
    return np.unique(np.concatenate([pick, [full]]))


def sub_job(job, boxes):
    """The elements of the listed boxes only (box ids unchanged), for a cheap oracle."""
    keep = np.isin(job.elem_box, boxes)
    bx = octree.Boxes(level=job.boxes.level, lo=job.boxes.lo, half=job.boxes.half, h=job.boxes.h,
                      elem_box=job.elem_box[keep], center=job.box_center, radius=job.box_radius,
                      morton=job.boxes.morton, counts=np.bincount(job.elem_box[keep], minlength=job.n_boxes))
    return configs.Job(name=job.name + "_sub", kind=job.kind, p=job.p, verts=job.verts, elems=job.elems[keep],
                       density=job.density[keep], boxes=bx)

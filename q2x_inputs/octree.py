"""Uniform octree leaf assignment for synthetic inputs.

Each element goes to the finest-level box that holds its centroid (the
paper's element-to-box rule, Sec. 2 after Eq. (5), with the centroid as the
element centre).  Only occupied boxes are kept, numbered in Morton order, with
their centres and radii.  No part of the Q2X method is computed here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Boxes:
    level: int
    lo: float            # root cube is [lo, lo + 2*half]^3
    half: float          # root half-side
    h: float             # leaf box side
    elem_box: np.ndarray     # [N] int32, index into the occupied-box list
    center: np.ndarray       # [B, 3] float64
    radius: np.ndarray       # [B] float64, half-diagonal sqrt(3) h / 2
    morton: np.ndarray       # [B] int64 Morton code of each occupied box
    counts: np.ndarray       # [B] elements per box

    @property
    def n_boxes(self) -> int:
        return int(self.center.shape[0])


def _spread3(x):
    """Interleave the low 21 bits of x with two zero bits (Morton helper)."""
    x = x.astype(np.uint64) & np.uint64(0x1FFFFF)
    x = (x | (x << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    x = (x | (x << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    x = (x | (x << np.uint64(2))) & np.uint64(0x1249249249249249)
    return x


def morton3(ix, iy, iz):
    return (_spread3(ix) | (_spread3(iy) << np.uint64(1)) | (_spread3(iz) << np.uint64(2))).astype(np.int64)


def root_half_side(verts) -> float:
    """Origin-centred root cube: [-1,1]^3 when every coordinate fits, else
    the smallest origin-centred cube holding all vertices (tiny margin)."""
    m = float(np.max(np.abs(verts))) if verts.size else 1.0
    return 1.0 if m <= 1.0 else m * (1.0 + 1e-12)


def assign(verts, elems, level: int, half: float | None = None) -> Boxes:
    """Assign elements (rows of vertex indices) to occupied leaf boxes."""
    verts = np.asarray(verts, dtype=np.float64)
    elems = np.asarray(elems)
    if half is None:
        half = root_half_side(verts)
    lo = -half
    nside = 1 << level
    h = 2.0 * half / nside
    cen = verts[elems].mean(axis=1)
    idx = np.clip(np.floor((cen - lo) / h).astype(np.int64), 0, nside - 1)
    code = morton3(idx[:, 0], idx[:, 1], idx[:, 2])
    ucode, inv, counts = np.unique(code, return_inverse=True, return_counts=True)
    # decode box integer coordinates from any member element
    first = np.zeros(ucode.shape[0], dtype=np.int64)
    first[inv[::-1]] = np.arange(inv.shape[0])[::-1]
    bidx = idx[first]
    center = lo + (bidx + 0.5) * h
    radius = np.full(ucode.shape[0], np.sqrt(3.0) * h / 2.0)
    return Boxes(level=level, lo=lo, half=half, h=h, elem_box=inv.astype(np.int32), center=center,
                 radius=radius, morton=ucode, counts=counts.astype(np.int64))


def _compact3(x):
    """Inverse of _spread3: gather every third bit of x into the low 21 bits."""
    x = x.astype(np.uint64) & np.uint64(0x1249249249249249)
    x = (x | (x >> np.uint64(2))) & np.uint64(0x10C30C30C30C30C3)
    x = (x | (x >> np.uint64(4))) & np.uint64(0x100F00F00F00F00F)
    x = (x | (x >> np.uint64(8))) & np.uint64(0x1F0000FF0000FF)
    x = (x | (x >> np.uint64(16))) & np.uint64(0x1F00000000FFFF)
    x = (x | (x >> np.uint64(32))) & np.uint64(0x1FFFFF)
    return x.astype(np.int64)


def box_centers(morton, level: int, lo: float, half: float):
    """Centres of the boxes with the given Morton codes at a level."""
    m = np.asarray(morton, dtype=np.int64).astype(np.uint64)
    ijk = np.stack([_compact3(m), _compact3(m >> np.uint64(1)), _compact3(m >> np.uint64(2))], 1)
    h = 2.0 * half / (1 << level)
    return lo + (ijk + 0.5) * h


def tree_levels(boxes: Boxes, top: int = 2):
    """The occupied boxes of every level from the leaves up to `top`: a list,
    leaves first, of (morton, center) per level and, per level below the top,
    child_parent (index of each box's parent in the next list).  Parents are
    numbered in Morton order, so child_parent is non-decreasing."""
    levels = [(boxes.morton, boxes.center)]
    parents = []
    code = boxes.morton
    for lev in range(boxes.level - 1, top - 1, -1):
        pc = code >> 3
        ucode, inv = np.unique(pc, return_inverse=True)
        parents.append(inv.astype(np.int32))
        levels.append((ucode, box_centers(ucode, lev, boxes.lo, boxes.half)))
        code = ucode
    return levels, parents


def near_pairs(boxes: Boxes, elems_box, target_box):
    """Near-field pairs: every target with every element of the 27 boxes
    around (and including) its own box (same level), in compressed rows.
    elems_box [N] is the box of each element, target_box [T] the box of each
    target.  Returns (pair_start [T+1] int64, pair_elem [P] int32); within a row
    the elements are grouped by box in Morton order, increasing index inside a box."""
    nb = boxes.n_boxes
    ijk = np.rint((boxes.center - boxes.lo) / boxes.h - 0.5).astype(np.int64)
    nside = 1 << boxes.level
    code = boxes.morton
    order = np.argsort(elems_box, kind="stable")
    counts = np.bincount(elems_box, minlength=nb)
    start = np.concatenate([[0], np.cumsum(counts)])
    # neighbour lists per box (occupied neighbours only, Morton order)
    offs = np.array([(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)])
    nbr = ijk[:, None, :] + offs[None, :, :]
    valid = np.all((nbr >= 0) & (nbr < nside), axis=2)
    nbr = np.clip(nbr, 0, nside - 1)
    ncode = morton3(nbr[..., 0].ravel(), nbr[..., 1].ravel(), nbr[..., 2].ravel()).reshape(nb, 27)
    pos = np.searchsorted(code, ncode)
    pos = np.clip(pos, 0, nb - 1)
    hit = valid & (code[pos] == ncode)
    box_rows = []
    for b in range(nb):
        nbs = np.sort(pos[b][hit[b]])
        box_rows.append(np.concatenate([order[start[k]:start[k + 1]] for k in nbs]).astype(np.int32))
    row_len = np.array([len(r) for r in box_rows], dtype=np.int64)
    tl = row_len[target_box]
    pair_start = np.concatenate([[0], np.cumsum(tl)]).astype(np.int64)
    pair_elem = np.concatenate([box_rows[b] for b in target_box]).astype(np.int32) if len(target_box) else \
        np.zeros(0, np.int32)
    return pair_start, pair_elem

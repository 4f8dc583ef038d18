"""Python binding of the Q2X C ABI (``include/q2x.h``) -- argument marshalling only.

Every step of the computation runs in the HIP library ``libq2x.so``; torch is
used only to own device memory and to name the stream.  If the library has not
been built this module raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libq2x.so")

TRI_SINGLE, TRI_DOUBLE, SEGMENT, TET, TRI_BOTH, SEGMENT_VEC = 0, 1, 2, 3, 4, 5
N_KINDS = 6
KIND_NAMES = {TRI_SINGLE: "tri_single", TRI_DOUBLE: "tri_double", SEGMENT: "segment", TET: "tet",
              TRI_BOTH: "tri_both", SEGMENT_VEC: "segment_vec"}
VERTS_PER_KIND = {TRI_SINGLE: 3, TRI_DOUBLE: 3, SEGMENT: 2, TET: 4, TRI_BOTH: 3, SEGMENT_VEC: 2}
FP64, FP32_MIXED = 0, 1
NORM_FMM, NORM_MOMENT = 0, 1
ACCUMULATE, PRESORTED = 1, 2
P_MAX = 32
FLAG_BAD_BOX, FLAG_NONFINITE, FLAG_RESERVED, FLAG_BAD_VERTEX, FLAG_NOT_SORTED = 1, 2, 4, 8, 16
EXPORTS = ("q2x_workspace_bytes", "q2x_bucket_workspace_bytes", "q2x_bucket", "q2x_tri_single", "q2x_tri_double", "q2x_segment", "q2x_tet",
           "q2x_tri_both", "q2x_tri_both_noalloc", "q2x_segment_vec", "q2x_status_get", "q2x_status_string", "q2x_profile_enable", "q2x_profile_reset",
           "q2x_profile_read", "q2x_version", "q2x_batch_plan", "q2x_batch_workspace_bytes", "q2x_batch_run", "q2x_batch_launch",
           "q2x_batch_job_status", "q2x_batch_groups", "q2x_batch_mode", "q2x_batch_destroy",
           "q2x_eval_workspace_bytes", "q2x_eval", "q2x_m2m_workspace_bytes", "q2x_m2m",
           "q2x_near_workspace_bytes", "q2x_near", "q2x_peak_measure", "q2x_batch_get_schedule",
           "q2x_batch_set_schedule", "q2x_tune_cache_load", "q2x_tune_cache_save", "q2x_build_id")
MERGE_ALL = 2 ** 31 - 1  # q2x_schedule.merge: one group per kind and precision


class Q2XError(RuntimeError):
    pass


class Schedule(ctypes.Structure):
    """Mirror of `q2x_schedule` (include/q2x.h)."""
    _fields_ = [("mode", ctypes.c_int32), ("split", ctypes.c_int32), ("merge", ctypes.c_int32),
                ("tuned", ctypes.c_int32)]


class Job(ctypes.Structure):
    """Mirror of `q2x_job` (include/q2x.h)."""
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_int), ("precision", ctypes.c_int), ("norm", ctypes.c_int),
                ("flags", ctypes.c_uint), ("verts", ctypes.c_void_p), ("n_verts", ctypes.c_int64),
                ("elems", ctypes.c_void_p), ("n_elems", ctypes.c_int64), ("density", ctypes.c_void_p),
                ("density2", ctypes.c_void_p), ("elem_box", ctypes.c_void_p), ("box_center", ctypes.c_void_p),
                ("n_boxes", ctypes.c_int64), ("coeffs", ctypes.c_void_p), ("coeffs2", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libq2x.so (raises Q2XError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise Q2XError(f"{LIB_PATH} is missing: build it with paper_2107_10942_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, ci, cu, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint, ctypes.c_size_t
        L.q2x_workspace_bytes.argtypes = [ci, i64, i64, ci, ci]
        L.q2x_workspace_bytes.restype = sz
        for name in ("q2x_tri_single", "q2x_tri_double", "q2x_segment", "q2x_tet"):
            f = getattr(L, name)
            f.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, i64, ci, ci, ci, cu, vp, vp, sz, vp]
            f.restype = ci
        L.q2x_tri_both.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, vp, i64, ci, ci, ci, cu, vp, vp, vp, sz, vp]
        L.q2x_tri_both.restype = ci
        L.q2x_tri_both_noalloc.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, vp, i64, ci, ci, ci, cu, vp, vp, vp,
                                           vp]
        L.q2x_tri_both_noalloc.restype = ci
        L.q2x_segment_vec.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, i64, ci, ci, ci, cu, vp, vp, sz, vp]
        L.q2x_segment_vec.restype = ci
        L.q2x_bucket_workspace_bytes.argtypes = [i64, i64]
        L.q2x_bucket_workspace_bytes.restype = sz
        L.q2x_bucket.argtypes = [vp, i64, i64, vp, vp, vp, sz, vp]
        L.q2x_bucket.restype = ci
        L.q2x_status_get.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]
        L.q2x_status_get.restype = ci
        L.q2x_status_string.argtypes = [ci]
        L.q2x_status_string.restype = ctypes.c_char_p
        L.q2x_profile_enable.argtypes = [ci]
        L.q2x_profile_enable.restype = None
        L.q2x_profile_reset.argtypes = []
        L.q2x_profile_reset.restype = None
        L.q2x_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
        L.q2x_profile_read.restype = ci
        L.q2x_version.restype = ctypes.c_char_p
        L.q2x_batch_plan.argtypes = [ctypes.POINTER(Job), ci, ctypes.POINTER(vp)]
        L.q2x_batch_plan.restype = ci
        L.q2x_batch_workspace_bytes.argtypes = [vp]
        L.q2x_batch_workspace_bytes.restype = sz
        L.q2x_batch_run.argtypes = [vp, vp, sz, vp]
        L.q2x_batch_run.restype = ci
        L.q2x_batch_launch.argtypes = [vp, vp, sz, vp]
        L.q2x_batch_launch.restype = ci
        L.q2x_batch_job_status.argtypes = [vp, vp, ci, vp, ctypes.POINTER(ctypes.c_uint32),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.q2x_batch_job_status.restype = ci
        L.q2x_batch_groups.argtypes = [vp]
        L.q2x_batch_groups.restype = ci
        L.q2x_batch_mode.argtypes = [vp]
        L.q2x_batch_mode.restype = ci
        L.q2x_batch_destroy.argtypes = [vp]
        L.q2x_batch_destroy.restype = None
        L.q2x_batch_get_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
        L.q2x_batch_get_schedule.restype = ci
        L.q2x_batch_set_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
        L.q2x_batch_set_schedule.restype = ci
        L.q2x_tune_cache_load.argtypes = [ctypes.c_char_p]
        L.q2x_tune_cache_load.restype = ci
        L.q2x_tune_cache_save.argtypes = [ctypes.c_char_p]
        L.q2x_tune_cache_save.restype = ci
        L.q2x_build_id.argtypes = []
        L.q2x_build_id.restype = ctypes.c_char_p
        L.q2x_eval_workspace_bytes.argtypes = [i64, i64]
        L.q2x_eval_workspace_bytes.restype = sz
        L.q2x_eval.argtypes = [ci, vp, i64, vp, i64, vp, vp, i64, vp, ci, ci, cu, vp, vp, sz, vp]
        L.q2x_eval.restype = ci
        L.q2x_m2m_workspace_bytes.argtypes = [i64, i64]
        L.q2x_m2m_workspace_bytes.restype = sz
        L.q2x_m2m.argtypes = [vp, vp, vp, i64, vp, i64, ci, ci, cu, vp, vp, sz, vp]
        L.q2x_m2m.restype = ci
        L.q2x_near_workspace_bytes.argtypes = []
        L.q2x_near_workspace_bytes.restype = sz
        L.q2x_near.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, cu, vp, sz, vp]
        L.q2x_near.restype = ci
        L.q2x_peak_measure.argtypes = [ci, vp, sz, ci, vp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        L.q2x_peak_measure.restype = ci
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise Q2XError(lib().q2x_status_string(rc).decode())


def _ptr(t, dtype, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise Q2XError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise Q2XError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise Q2XError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def workspace_bytes(kind, n_elems, n_boxes, p, precision=FP32_MIXED) -> int:
    return int(lib().q2x_workspace_bytes(kind, n_elems, n_boxes, p, precision))


def alloc_workspace(kind, n_elems, n_boxes, p, precision=FP32_MIXED, device=None):
    nbytes = workspace_bytes(kind, n_elems, n_boxes, p, precision)
    if nbytes == 0:
        raise Q2XError("invalid workspace request")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def _out(out, nb, p, device, name="out"):
    if out is None:
        return torch.empty((nb, (p + 1) ** 2, 2), dtype=torch.float64, device=device)
    if tuple(out.shape) != (nb, (p + 1) ** 2, 2):
        raise Q2XError(f"{name} must have shape {(nb, (p + 1) ** 2, 2)}")
    return out


def run(kind, verts, elems, density, elem_box, box_center, box_radius, p, precision=FP32_MIXED,
        norm=NORM_FMM, accumulate=False, presorted=False, out=None, workspace=None, stream=None):
    """Q2X for one mesh of one element kind; returns out [B, (p+1)^2, 2] float64."""
    if kind in (TRI_BOTH, SEGMENT_VEC):
        raise Q2XError("use tri_both() / segment_vec() for the multi-output kinds")
    n_el = int(elems.shape[0]) if elems is not None else 0
    nb = int(box_center.shape[0])
    if elems is not None and elems.dim() == 2 and elems.shape[1] != VERTS_PER_KIND[kind]:
        raise Q2XError(f"elements of kind {KIND_NAMES[kind]} need {VERTS_PER_KIND[kind]} vertices")
    out = _out(out, nb, p, verts.device)
    if workspace is None:
        workspace = alloc_workspace(kind, n_el, nb, p, precision, device=verts.device)
    flags = (ACCUMULATE if accumulate else 0) | (PRESORTED if presorted else 0)
    fn = getattr(lib(), "q2x_" + KIND_NAMES[kind])
    rc = fn(_ptr(verts, torch.float64, "verts"), int(verts.shape[0]),
            _ptr(elems, torch.int32, "elems"), n_el,
            _ptr(density, torch.float64, "density"), _ptr(elem_box, torch.int32, "elem_box"),
            _ptr(box_center, torch.float64, "box_center"), _ptr(box_radius, torch.float64, "box_radius"),
            nb, int(p), int(precision), int(norm), flags, _ptr(out, torch.float64, "out"),
            ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream))
    _check(rc)
    return out


def tri_single(*args, **kw):
    return run(TRI_SINGLE, *args, **kw)


def tri_double(*args, **kw):
    return run(TRI_DOUBLE, *args, **kw)


def segment(*args, **kw):
    return run(SEGMENT, *args, **kw)


def tet(*args, **kw):
    return run(TET, *args, **kw)


def tri_both(verts, tris, density_single, density_double, elem_box, box_center, box_radius, p,
             precision=FP32_MIXED, norm=NORM_FMM, accumulate=False, presorted=False, out_single=None,
             out_double=None, workspace=None, stream=None):
    """Single and double layer of one triangle mesh in one call: (out_single, out_double)."""
    n_el = int(tris.shape[0]) if tris is not None else 0
    nb = int(box_center.shape[0])
    if tris is not None and tris.dim() == 2 and tris.shape[1] != 3:
        raise Q2XError("triangles need 3 vertices")
    out_single = _out(out_single, nb, p, verts.device, "out_single")
    out_double = _out(out_double, nb, p, verts.device, "out_double")
    if workspace is None:
        workspace = alloc_workspace(TRI_BOTH, n_el, nb, p, precision, device=verts.device)
    flags = (ACCUMULATE if accumulate else 0) | (PRESORTED if presorted else 0)
    rc = lib().q2x_tri_both(_ptr(verts, torch.float64, "verts"), int(verts.shape[0]),
                            _ptr(tris, torch.int32, "tris"), n_el,
                            _ptr(density_single, torch.float64, "density_single"),
                            _ptr(density_double, torch.float64, "density_double"),
                            _ptr(elem_box, torch.int32, "elem_box"),
                            _ptr(box_center, torch.float64, "box_center"),
                            _ptr(box_radius, torch.float64, "box_radius"),
                            nb, int(p), int(precision), int(norm), flags,
                            _ptr(out_single, torch.float64, "out_single"),
                            _ptr(out_double, torch.float64, "out_double"),
                            ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream))
    _check(rc)
    return out_single, out_double


NOALLOC_SCRATCH_BYTES = 64 << 20
STATUS_BYTES = 64


def tri_both_noalloc(verts, tris, density_single, density_double, elem_box, box_center, box_radius, p, status,
                     precision=FP32_MIXED, norm=NORM_FMM, accumulate=False, presorted=False, out_single=None,
                     out_double=None, stream=None):
    """tri_both without a workspace (q2x_tri_both_noalloc): the library's static
    per-GPU scratch is used; `status` is a caller-owned 64-byte device buffer
    (e.g. torch.empty(64, dtype=torch.uint8)) that receives the status block
    (read it with status(status)).  Returns (out_single, out_double)."""
    n_el = int(tris.shape[0]) if tris is not None else 0
    nb = int(box_center.shape[0])
    if tris is not None and tris.dim() == 2 and tris.shape[1] != 3:
        raise Q2XError("triangles need 3 vertices")
    if status is None or not status.is_cuda or status.numel() * status.element_size() < STATUS_BYTES:
        raise Q2XError("status must be a device buffer of at least 64 bytes")
    out_single = _out(out_single, nb, p, verts.device, "out_single")
    out_double = _out(out_double, nb, p, verts.device, "out_double")
    flags = (ACCUMULATE if accumulate else 0) | (PRESORTED if presorted else 0)
    rc = lib().q2x_tri_both_noalloc(_ptr(verts, torch.float64, "verts"), int(verts.shape[0]),
                                    _ptr(tris, torch.int32, "tris"), n_el,
                                    _ptr(density_single, torch.float64, "density_single"),
                                    _ptr(density_double, torch.float64, "density_double"),
                                    _ptr(elem_box, torch.int32, "elem_box"),
                                    _ptr(box_center, torch.float64, "box_center"),
                                    _ptr(box_radius, torch.float64, "box_radius"),
                                    nb, int(p), int(precision), int(norm), flags,
                                    _ptr(out_single, torch.float64, "out_single"),
                                    _ptr(out_double, torch.float64, "out_double"),
                                    ctypes.c_void_p(status.data_ptr()), _stream(stream))
    _check(rc)
    return out_single, out_double


class BatchPlan:
    """A batch of jobs (q2x_batch_plan / q2x_batch_run).  `jobs` is a list of
    dicts with the single-call arguments: kind, verts, elems, density,
    elem_box, box_center, p, and optionally precision, norm, accumulate,
    out (and density2 / out2 for TRI_BOTH).  Outputs are allocated when not
    given; the tensors are kept alive by the plan."""

    def __init__(self, jobs):
        self._keep = []
        arr = (Job * len(jobs))()
        self.outs = []
        for i, j in enumerate(jobs):
            kind = int(j["kind"])
            p = int(j["p"])
            nb = int(j["box_center"].shape[0])
            dev = j["verts"].device
            if kind == SEGMENT_VEC:  # density [N][3], out [3][B][(p+1)^2][2]
                out = j.get("out")
                if out is None:
                    out = torch.empty((3, nb, (p + 1) ** 2, 2), dtype=torch.float64, device=dev)
            else:
                out = _out(j.get("out"), nb, p, dev)
            out2 = _out(j.get("out2"), nb, p, dev, "out2") if kind == TRI_BOTH else None
            self.outs.append((out, out2) if kind == TRI_BOTH else out)
            flags = (ACCUMULATE if j.get("accumulate") else 0) | (PRESORTED if j.get("presorted") else 0)
            elems = j["elems"]
            if elems.dim() == 2 and elems.shape[1] != VERTS_PER_KIND[kind]:
                raise Q2XError(f"job {i}: elements of kind {KIND_NAMES[kind]} need {VERTS_PER_KIND[kind]} vertices")
            arr[i] = Job(kind, p, int(j.get("precision", FP32_MIXED)), int(j.get("norm", NORM_FMM)), flags,
                         _ptr(j["verts"], torch.float64, "verts"), int(j["verts"].shape[0]),
                         _ptr(elems, torch.int32, "elems"), int(elems.shape[0]),
                         _ptr(j["density"], torch.float64, "density"),
                         _ptr(j.get("density2"), torch.float64, "density2"),
                         _ptr(j["elem_box"], torch.int32, "elem_box"),
                         _ptr(j["box_center"], torch.float64, "box_center"), nb,
                         _ptr(out, torch.float64, "out"), _ptr(out2, torch.float64, "out2"))
            self._keep.append((j, out, out2))
        self._arr = arr
        self.n_jobs = len(jobs)
        h = ctypes.c_void_p()
        _check(lib().q2x_batch_plan(arr, len(jobs), ctypes.byref(h)))
        self._h = h
        self.workspace = None

    def workspace_bytes(self):
        return int(lib().q2x_batch_workspace_bytes(self._h))

    def alloc_workspace(self, device=None):
        nbytes = self.workspace_bytes()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-ws.data_ptr()) % 256
        self.workspace = ws[off:off + nbytes]
        return self.workspace

    def run(self, workspace=None, stream=None):
        if workspace is None:
            workspace = self.workspace if self.workspace is not None else self.alloc_workspace()
        _check(lib().q2x_batch_run(self._h, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   _stream(stream)))
        return self.outs

    def launch(self, workspace=None, stream=None):
        """Enqueue once, without a graph (q2x_batch_launch)."""
        if workspace is None:
            workspace = self.workspace if self.workspace is not None else self.alloc_workspace()
        _check(lib().q2x_batch_launch(self._h, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                      _stream(stream)))
        return self.outs

    def status(self, j, workspace=None, stream=None):
        workspace = self.workspace if workspace is None else workspace
        f = ctypes.c_uint32(0)
        d = ctypes.c_int64(0)
        s = ctypes.c_int64(0)
        _check(lib().q2x_batch_job_status(self._h, ctypes.c_void_p(workspace.data_ptr()), int(j), _stream(stream),
                                          ctypes.byref(f), ctypes.byref(d), ctypes.byref(s)))
        return int(f.value), int(d.value), int(s.value)

    @property
    def groups(self):
        return int(lib().q2x_batch_groups(self._h))

    @property
    def mode(self):
        return int(lib().q2x_batch_mode(self._h))

    @property
    def schedule(self):
        """The plan's schedule: dict(mode, split, merge, tuned) (q2x_batch_get_schedule)."""
        sc = Schedule()
        _check(lib().q2x_batch_get_schedule(self._h, ctypes.byref(sc)))
        return {"mode": sc.mode, "split": sc.split, "merge": sc.merge, "tuned": sc.tuned}

    def set_schedule(self, mode=0, split=0, merge=0):
        """Force a schedule (q2x_batch_set_schedule); the plan is then never tuned."""
        sc = Schedule(int(mode), int(split), int(merge), 0)
        _check(lib().q2x_batch_set_schedule(self._h, ctypes.byref(sc)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().q2x_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def segment_vec(verts, segs, density3, elem_box, box_center, box_radius, p, precision=FP32_MIXED, norm=NORM_FMM,
                accumulate=False, presorted=False, out=None, workspace=None, stream=None):
    """Segments with a vector density [N][3]: coefficients [3][B][(p+1)^2][2], one per component."""
    n_el = int(segs.shape[0]) if segs is not None else 0
    nb = int(box_center.shape[0])
    if segs is not None and segs.dim() == 2 and segs.shape[1] != 2:
        raise Q2XError("segments need 2 vertices")
    if density3 is not None and tuple(density3.shape) != (n_el, 3):
        raise Q2XError(f"density3 must have shape {(n_el, 3)}")
    shape = (3, nb, (p + 1) ** 2, 2)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=verts.device)
    elif tuple(out.shape) != shape:
        raise Q2XError(f"out must have shape {shape}")
    if workspace is None:
        workspace = alloc_workspace(SEGMENT_VEC, n_el, nb, p, precision, device=verts.device)
    flags = (ACCUMULATE if accumulate else 0) | (PRESORTED if presorted else 0)
    rc = lib().q2x_segment_vec(_ptr(verts, torch.float64, "verts"), int(verts.shape[0]),
                               _ptr(segs, torch.int32, "segs"), n_el, _ptr(density3, torch.float64, "density3"),
                               _ptr(elem_box, torch.int32, "elem_box"), _ptr(box_center, torch.float64, "box_center"),
                               _ptr(box_radius, torch.float64, "box_radius"), nb, int(p), int(precision), int(norm),
                               flags, _ptr(out, torch.float64, "out"), ctypes.c_void_p(workspace.data_ptr()),
                               workspace.numel(), _stream(stream))
    _check(rc)
    return out


def eval_workspace_bytes(n_elems, n_boxes) -> int:
    return int(lib().q2x_eval_workspace_bytes(int(n_elems), int(n_boxes)))


def alloc_eval_workspace(n_elems, n_boxes, device=None):
    nbytes = eval_workspace_bytes(n_elems, n_boxes)
    if nbytes == 0:
        raise Q2XError("invalid workspace request")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def evaluate(kind, verts, elems, elem_box, box_center, local, p, precision=FP32_MIXED, accumulate=False,
             presorted=False, out=None, workspace=None, stream=None):
    """Receiving side (q2x_eval): per element, sum_{n<=p,m} L_b[n,m] int_e R_n^m(y - c_b)
    (double layer: n . grad R).  local [B, (p+1)^2, 2] float64; returns out [N, 2] float64."""
    if kind not in (TRI_SINGLE, TRI_DOUBLE, SEGMENT, TET):
        raise Q2XError("evaluate takes TRI_SINGLE, TRI_DOUBLE, SEGMENT or TET")
    n_el = int(elems.shape[0]) if elems is not None else 0
    nb = int(box_center.shape[0])
    if elems is not None and elems.dim() == 2 and elems.shape[1] != VERTS_PER_KIND[kind]:
        raise Q2XError(f"elements of kind {KIND_NAMES[kind]} need {VERTS_PER_KIND[kind]} vertices")
    if local is not None and tuple(local.shape) != (nb, (p + 1) ** 2, 2):
        raise Q2XError(f"local must have shape {(nb, (p + 1) ** 2, 2)}")
    if out is None:
        out = torch.empty((n_el, 2), dtype=torch.float64, device=verts.device)
    elif tuple(out.shape) != (n_el, 2):
        raise Q2XError(f"out must have shape {(n_el, 2)}")
    if workspace is None:
        workspace = alloc_eval_workspace(n_el, nb, device=verts.device)
    flags = (ACCUMULATE if accumulate else 0) | (PRESORTED if presorted else 0)
    rc = lib().q2x_eval(int(kind), _ptr(verts, torch.float64, "verts"), int(verts.shape[0]),
                        _ptr(elems, torch.int32, "elems"), n_el, _ptr(elem_box, torch.int32, "elem_box"),
                        _ptr(box_center, torch.float64, "box_center"), nb, _ptr(local, torch.float64, "local"),
                        int(p), int(precision), flags, _ptr(out, torch.float64, "out"),
                        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream))
    _check(rc)
    return out


def alloc_m2m_workspace(n_child, n_parent, device=None):
    nbytes = int(lib().q2x_m2m_workspace_bytes(int(n_child), int(n_parent)))
    if nbytes == 0:
        raise Q2XError("invalid workspace request")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def m2m(child, child_center, child_parent, parent_center, p, norm=NORM_FMM, accumulate=False, presorted=False,
        out=None, workspace=None, stream=None):
    """Translate child expansions [C, (p+1)^2, 2] to their parents' centres and sum
    per parent (q2x_m2m); returns out [P, (p+1)^2, 2] float64."""
    nc = int(child_parent.shape[0])
    npar = int(parent_center.shape[0])
    if child is not None and tuple(child.shape) != (nc, (p + 1) ** 2, 2):
        raise Q2XError(f"child must have shape {(nc, (p + 1) ** 2, 2)}")
    out = _out(out, npar, p, parent_center.device)
    if workspace is None:
        workspace = alloc_m2m_workspace(nc, npar, device=parent_center.device)
    flags = (ACCUMULATE if accumulate else 0) | (PRESORTED if presorted else 0)
    rc = lib().q2x_m2m(_ptr(child, torch.float64, "child"), _ptr(child_center, torch.float64, "child_center"),
                       _ptr(child_parent, torch.int32, "child_parent"), nc,
                       _ptr(parent_center, torch.float64, "parent_center"), npar, int(p), int(norm), flags,
                       _ptr(out, torch.float64, "out"), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                       _stream(stream))
    _check(rc)
    return out


def upward(leaf, centers, parents, p, norm=NORM_FMM, stream=None):
    """Upward pass: `leaf` [B0, (p+1)^2, 2] about centers[0]; centers[i] [B_i, 3]
    for levels i = 0 (leaves) .. L; parents[i] [B_i] int32 (non-decreasing)
    maps level i to level i + 1.  One q2x_m2m call per level; returns the list
    of expansions, leaves first."""
    out = [leaf]
    for i, par in enumerate(parents):
        out.append(m2m(out[-1], centers[i], par, centers[i + 1], p, norm=norm, presorted=True, stream=stream))
    return out


def alloc_near_workspace(device=None):
    nbytes = int(lib().q2x_near_workspace_bytes())
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def near(verts, tris, targets, pair_start, pair_tri, density_single=None, density_double=None, entries=True,
         potential=True, accumulate=False, out_entries=None, out_potential=None, workspace=None, stream=None):
    """Near-field potentials of triangles at targets (q2x_near), pairs in CSR by
    target.  Returns (entries_L [P], entries_M [P]) or None, and potential [T] or None."""
    nt = int(targets.shape[0])
    npair = int(pair_tri.shape[0])
    if tuple(pair_start.shape) != (nt + 1,):
        raise Q2XError(f"pair_start must have shape {(nt + 1,)}")
    dev = targets.device
    eL = eM = pot = None
    if entries:
        eL, eM = out_entries if out_entries is not None else (
            torch.empty(npair, dtype=torch.float64, device=dev), torch.empty(npair, dtype=torch.float64, device=dev))
    if potential:
        pot = out_potential if out_potential is not None else torch.empty(nt, dtype=torch.float64, device=dev)
    if workspace is None:
        workspace = alloc_near_workspace(dev)
    rc = lib().q2x_near(_ptr(verts, torch.float64, "verts"), int(verts.shape[0]), _ptr(tris, torch.int32, "tris"),
                        int(tris.shape[0]), _ptr(targets, torch.float64, "targets"), nt,
                        _ptr(pair_start, torch.int64, "pair_start"), _ptr(pair_tri, torch.int32, "pair_tri"), npair,
                        _ptr(density_single, torch.float64, "density_single"),
                        _ptr(density_double, torch.float64, "density_double"),
                        _ptr(eL, torch.float64, "entries_L"), _ptr(eM, torch.float64, "entries_M"),
                        _ptr(pot, torch.float64, "potential"), ACCUMULATE if accumulate else 0,
                        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream))
    _check(rc)
    return ((eL, eM) if entries else None), pot


def bucket(elem_box, n_boxes, stream=None, workspace=None):
    """Stable grouping of elements by box: (perm [N] int32, box_start [B+1] int32, workspace)."""
    n = int(elem_box.shape[0])
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=elem_box.device)[:n]
    box_start = torch.empty(n_boxes + 1, dtype=torch.int32, device=elem_box.device)
    if workspace is None:
        nbytes = int(lib().q2x_bucket_workspace_bytes(n, n_boxes))
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=elem_box.device)
        off = (-ws.data_ptr()) % 256
        workspace = ws[off:off + nbytes]
    _check(lib().q2x_bucket(_ptr(elem_box, torch.int32, "elem_box"), n, int(n_boxes),
                            ctypes.c_void_p(perm.data_ptr()) if n else None,
                            ctypes.c_void_p(box_start.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                            workspace.numel(), _stream(stream)))
    return perm, box_start, workspace


def status(workspace, stream=None):
    """(flags, n_degenerate, n_skipped) of the last call that used `workspace`."""
    f = ctypes.c_uint32(0)
    d = ctypes.c_int64(0)
    s = ctypes.c_int64(0)
    _check(lib().q2x_status_get(ctypes.c_void_p(workspace.data_ptr()), _stream(stream), ctypes.byref(f),
                                ctypes.byref(d), ctypes.byref(s)))
    return int(f.value), int(d.value), int(s.value)


def profile_enable(on=True):
    lib().q2x_profile_enable(1 if on else 0)


def profile_reset():
    lib().q2x_profile_reset()


def profile_read():
    """Per kind (index = kind): (recursion_ms, call_ms, calls), lists of N_KINDS, since the last reset."""
    a = (ctypes.c_double * N_KINDS)()
    c = (ctypes.c_double * N_KINDS)()
    d = (ctypes.c_int64 * N_KINDS)()
    _check(lib().q2x_profile_read(a, c, d))
    return list(a), list(c), list(d)


PEAK_FMA64, PEAK_FMA32, PEAK_HBM_COPY = 0, 1, 2


def peak_measure(which, buffer, reps=20, stream=None):
    """Measured peak of the running GPU (q2x_peak_measure): (TFLOP/s or GB/s, ms per launch)."""
    v = ctypes.c_double(0.0)
    ms = ctypes.c_double(0.0)
    _check(lib().q2x_peak_measure(int(which), ctypes.c_void_p(buffer.data_ptr()), buffer.numel() * buffer.element_size(),
                                  int(reps), _stream(stream), ctypes.byref(v), ctypes.byref(ms)))
    return v.value, ms.value


def version():
    return lib().q2x_version().decode()


def job_tensors(job, device="cuda"):
    """Device tensors of a q2x_inputs Job (verts, elems, density, elem_box, box_center, box_radius)."""
    t = lambda a, dt: torch.as_tensor(a, dtype=dt).contiguous().to(device)  # noqa: E731
    return (t(job.verts, torch.float64), t(job.elems, torch.int32), t(job.density, torch.float64),
            t(job.elem_box, torch.int32), t(job.box_center, torch.float64), t(job.box_radius, torch.float64))


def tune_cache_load(path):
    """Read batch schedules from a text file (q2x_tune_cache_load)."""
    _check(lib().q2x_tune_cache_load(os.fsencode(path)))


def tune_cache_save(path):
    """Write every cached batch schedule to a text file (q2x_tune_cache_save)."""
    _check(lib().q2x_tune_cache_save(os.fsencode(path)))


def build_id():
    """Hash of the library's sources (q2x_build_id)."""
    return lib().q2x_build_id().decode()

"""The C-ABI library loads and exports every symbol include/q2x.h declares;
host-side argument validation (no GPU work is issued by these calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "q2x.h")


def _ensure_built():
    from paper_2107_10942_amd import build
    if not os.path.exists(build.LIB):
        build.build(force=False)
    return build.LIB


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(q2x_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("q2x_tri_single", "q2x_tri_double", "q2x_segment", "q2x_tet", "q2x_tri_both", "q2x_workspace_bytes",
              "q2x_status_get", "q2x_bucket"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_ensure_built())
    for n in declared_functions():
        assert hasattr(lib, n), n
    from paper_2107_10942_amd import q2x
    assert set(q2x.EXPORTS) == set(declared_functions())


def test_workspace_bytes_and_argument_errors():
    _ensure_built()
    from paper_2107_10942_amd import q2x
    L = q2x.lib()
    assert q2x.workspace_bytes(q2x.TRI_SINGLE, 1000, 100, 16) > 0
    assert q2x.workspace_bytes(q2x.TRI_SINGLE, 1000, 100, q2x.P_MAX + 1) == 0
    assert q2x.workspace_bytes(7, 1000, 100, 8) == 0
    assert q2x.workspace_bytes(q2x.TET, -1, 100, 8) == 0
    # larger p and more elements never need less workspace
    assert q2x.workspace_bytes(q2x.TET, 5000, 100, 20) >= q2x.workspace_bytes(q2x.TET, 1000, 100, 8)
    vp = ctypes.c_void_p
    # p out of range -> synchronous error, before any device work
    rc = L.q2x_tri_single(None, 0, None, 0, None, None, None, None, 0, 99, 0, 0, 0, None, vp(256), 1 << 20, None)
    assert rc == -2
    # null workspace
    rc = L.q2x_tri_single(None, 0, None, 0, None, None, None, None, 0, 8, 0, 0, 0, None, None, 0, None)
    assert rc == -3
    # misaligned workspace
    rc = L.q2x_tet(None, 0, None, 0, None, None, None, None, 0, 8, 0, 0, 0, None, vp(260), 1 << 20, None)
    assert rc == -3
    # unknown precision / norm / flag bits
    rc = L.q2x_segment(None, 0, None, 0, None, None, None, None, 0, 8, 5, 0, 0, None, vp(256), 1 << 20, None)
    assert rc == -1
    rc = L.q2x_segment(None, 0, None, 0, None, None, None, None, 0, 8, 0, 3, 0, None, vp(256), 1 << 20, None)
    assert rc == -1
    rc = L.q2x_segment(None, 0, None, 0, None, None, None, None, 0, 8, 0, 0, 64, None, vp(256), 1 << 20, None)
    assert rc == -1
    # elements without arrays
    rc = L.q2x_tri_double(None, 3, None, 10, None, None, None, None, 0, 8, 0, 0, 0, None, vp(256), 1 << 20, None)
    assert rc == -1
    # workspace too small
    rc = L.q2x_tri_single(vp(8), 3, vp(4), 1, vp(8), vp(4), vp(8), vp(8), 1, 8, 0, 0, 0, vp(8), vp(256), 16, None)
    assert rc == -3
    # fused single + double: its own workspace size (two sets of partial sums), the
    # second density and output are required, and the outputs must not overlap
    assert q2x.workspace_bytes(q2x.TRI_BOTH, 5000, 100, 16) > q2x.workspace_bytes(q2x.TRI_SINGLE, 5000, 100, 16)
    big = q2x.workspace_bytes(q2x.TRI_BOTH, 10, 4, 4)
    rc = L.q2x_tri_both(vp(8), 3, vp(4), 1, vp(8), None, vp(4), vp(8), None, 1, 4, 0, 0, 0, vp(8), vp(4096),
                        vp(256), big, None)
    assert rc == -1
    rc = L.q2x_tri_both(vp(8), 3, vp(4), 1, vp(8), vp(8), vp(4), vp(8), None, 1, 4, 0, 0, 0, vp(8), None,
                        vp(256), big, None)
    assert rc == -1
    rc = L.q2x_tri_both(vp(8), 3, vp(4), 1, vp(8), vp(8), vp(4), vp(8), None, 1, 4, 0, 0, 0, vp(4096), vp(4096 + 200),
                        vp(256), big, None)
    assert rc == -1  # 25 coefficients x 16 B = 400 B per box: the outputs overlap
    rc = L.q2x_tri_both(vp(8), 3, vp(4), 1, vp(8), vp(8), vp(4), vp(8), None, 1, 4, 0, 0, 0, vp(8), vp(4096),
                        vp(256), 16, None)
    assert rc == -3
    # batch plans: argument errors return before any device work
    h = ctypes.c_void_p()
    assert L.q2x_batch_plan(None, 1, ctypes.byref(h)) == -1
    J = (q2x.Job * 2)()
    assert L.q2x_batch_plan(J, 0, ctypes.byref(h)) == -1
    J[0] = q2x.Job(7, 4, 0, 0, 0, None, 0, None, 0, None, None, None, None, 0, None, None)  # bad kind
    J[1] = q2x.Job(0, 4, 0, 0, 0, None, 0, None, 0, None, None, None, None, 0, None, None)
    assert L.q2x_batch_plan(J, 2, ctypes.byref(h)) == -1 and not h.value
    J[0] = q2x.Job(0, 40, 0, 0, 0, None, 0, None, 0, None, None, None, None, 0, None, None)  # p out of range
    assert L.q2x_batch_plan(J, 2, ctypes.byref(h)) == -2
    J[0] = q2x.Job(1, 8, 0, 0, 0, None, 3, None, 5, None, None, None, None, 0, None, None)  # elements, no arrays
    assert L.q2x_batch_plan(J, 2, ctypes.byref(h)) == -1
    J[0] = q2x.Job(4, 8, 0, 0, 0, vp(8), 3, vp(4), 5, vp(8), None, vp(4), vp(8), 2, vp(8), vp(64))  # both: no density2
    assert L.q2x_batch_plan(J, 2, ctypes.byref(h)) == -1
    assert L.q2x_batch_workspace_bytes(None) == 0 and L.q2x_batch_mode(None) == -1
    L.q2x_batch_destroy(None)
    assert L.q2x_status_string(-2).startswith(b"Q2X_ERR_P_RANGE")
    assert b"gfx950" in L.q2x_version()


def test_eval_argument_errors():
    """q2x_eval: kinds other than the four element kinds, p out of range, bad
    precision or flags, missing arrays and a short workspace are refused
    synchronously, before any device work."""
    _ensure_built()
    from paper_2107_10942_amd import q2x
    L = q2x.lib()
    vp = ctypes.c_void_p
    ws = q2x.eval_workspace_bytes(1000, 50)
    assert ws > 0 and q2x.eval_workspace_bytes(-1, 5) == 0
    assert q2x.eval_workspace_bytes(5000, 50) >= ws

    def call(kind=0, p=8, prec=0, flags=0, nel=1, local=vp(8), out=vp(8), wsb=ws, wsp=vp(256)):
        return L.q2x_eval(kind, vp(8), 3, vp(4), nel, vp(4), vp(8), 1, local, p, prec, flags, out, wsp, wsb, None)

    assert call(kind=q2x.TRI_BOTH) == -1 and call(kind=q2x.SEGMENT_VEC) == -1 and call(kind=-1) == -1
    assert call(p=33) == -2 and call(p=-1) == -2
    assert call(prec=2) == -1 and call(flags=4) == -1
    assert call(local=None) == -1 and call(out=None) == -1
    assert call(wsb=16) == -3 and call(wsp=vp(264)) == -3 and call(wsp=None) == -3
    assert call(out=vp(12)) == -1  # misaligned output


def test_near_and_m2m_argument_errors():
    """q2x_near and q2x_m2m refuse bad arguments synchronously (no device work)."""
    _ensure_built()
    from paper_2107_10942_amd import q2x
    L = q2x.lib()
    vp = ctypes.c_void_p
    ws = vp(256)
    nb = q2x.lib().q2x_near_workspace_bytes()
    assert nb >= 64

    def near(nv=3, nt=1, ntar=1, npair=1, ds=vp(8), dd=None, eL=vp(8), eM=None, pot=vp(8), flags=0, w=ws, wb=nb,
             targets=vp(8), ps=vp(8), pt=vp(4)):
        return L.q2x_near(vp(8), nv, vp(4), nt, targets, ntar, ps, pt, npair, ds, dd, eL, eM, pot, flags, w, wb, None)

    assert near(nv=-1) == -1 and near(npair=-1) == -1
    assert near(flags=2) == -1  # PRESORTED has no meaning here
    assert near(ds=None, dd=None) == -1  # a potential needs a density
    assert near(eL=None, eM=None, pot=None) == -1  # nothing to write
    assert near(targets=None) == -1 and near(pt=None) == -1
    assert near(w=None) == -3 and near(w=vp(260)) == -3 and near(wb=8) == -3
    assert near(pot=vp(12)) == -1  # misaligned

    mb = q2x.lib().q2x_m2m_workspace_bytes(10, 3)
    assert mb > 0 and q2x.lib().q2x_m2m_workspace_bytes(-1, 3) == 0

    def m2m(p=8, norm=0, flags=0, child=vp(8), out=vp(1 << 20), w=ws, wb=mb, nc=10, npar=3):
        return L.q2x_m2m(child, vp(8), vp(4), nc, vp(8), npar, p, norm, flags, out, w, wb, None)

    assert m2m(p=33) == -2 and m2m(norm=2) == -1 and m2m(flags=8) == -1
    assert m2m(child=None) == -1 and m2m(out=None) == -1
    assert m2m(wb=16) == -3 and m2m(w=None) == -3
    # parents written over the children being read
    assert m2m(child=vp(4096), out=vp(4096 + 16 * 81)) == -1


def test_build_id_and_tune_cache_files(tmp_path):
    """q2x_build_id is the hash of the library's sources; the tuning cache
    reads and writes its text format (host-only calls), keeps well-formed
    entries of any device or build, skips malformed lines and refuses a path
    it cannot open."""
    _ensure_built()
    from paper_2107_10942_amd import build, q2x
    assert q2x.build_id() == build.library_hash()
    src = tmp_path / "in.txt"
    src.write_text("gfx950:sramecc+:xnack-/256|0123456789abcdef|0,1,16,40;2560/6617\t1 0 1024\n"
                   "not a cache line\n"
                   "other|feedfacefeedface|4,0,20,7;448/30\t0 1 0\n"
                   "bad|x|y\t7 0 0\n")
    q2x.tune_cache_load(src)
    out = tmp_path / "out.txt"
    q2x.tune_cache_save(out)
    lines = out.read_text().splitlines()
    assert "gfx950:sramecc+:xnack-/256|0123456789abcdef|0,1,16,40;2560/6617\t1 0 1024" in lines
    assert "other|feedfacefeedface|4,0,20,7;448/30\t0 1 0" in lines
    assert not any(ln.startswith("bad|") or ln.startswith("not a") for ln in lines)
    with pytest.raises(q2x.Q2XError):
        q2x.tune_cache_load(tmp_path / "missing.txt")
    with pytest.raises(q2x.Q2XError):
        q2x.tune_cache_save(tmp_path / "no_such_dir" / "x.txt")


def test_source_hash_does_not_depend_on_the_checkout_location(monkeypatch):
    """The tile-kernel source hash ties stored profiler figures to the code they
    measured; it must be the same wherever the tree is checked out (the
    compiler flags carry an absolute include directory)."""
    from paper_2107_10942_amd import build
    h = build.source_hash()
    moved = ["/elsewhere/include" if prev == "-I" else f for prev, f in zip([None] + build.COMMON, build.COMMON)]
    monkeypatch.setattr(build, "COMMON", moved)
    assert build.source_hash() == h
    monkeypatch.setattr(build, "COMMON", moved + ["-DQ2X_SOMETHING_ELSE"])
    assert build.source_hash() != h  # other flags still count

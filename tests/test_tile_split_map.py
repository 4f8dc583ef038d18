"""Host-side check of the tile kernel's workgroup -> (tile, half) mapping.

A launch of n tiles of which S are split (two workgroups each, the split
tiles spread evenly: tile t is split iff floor((t+1) S / n) > floor(t S / n))
has n + S workgroups; the kernel takes workgroup b to virtual id
vb = xcd_tile(b, n + S) (one contiguous range of virtual ids per XCD) and
vb to its tile and half with 32-bit integer arithmetic.  This test restates
that arithmetic (csrc/q2x_tile.hpp, csrc/q2x_internal.hpp) and the host's
choice of S (csrc/q2x_api.hip) and checks, for every launch of up to 2,199
tiles in both precisions, that each (tile, half) is covered exactly once and
that S tiles are split."""

import os

import pytest

U32 = 0xFFFFFFFF


def xcd_tile(bid, nblk):
    q, r = nblk // 8, nblk % 8
    x, k = bid % 8, bid // 8
    return x * (q + 1) + k if x < r else r * (q + 1) + (x - r) * q + k


def n_split(n, fp64):
    if fp64:
        return n if n <= 2048 else 0
    if n <= 512:
        return n
    if 1024 < n < 2048:
        return 2048 - n
    return 0


def tile_of(vb, n, s):
    if s == 0:
        return vb, 0, 1
    assert n <= 2048 and (n + s) * n <= U32  # every product below fits in 32 bits
    t = vb * n // (n + s)
    steps = 0
    while t + 1 < n and (t + 1) + (t + 1) * s // n <= vb:
        t += 1
        steps += 1
    while t > 0 and t + t * s // n > vb:
        t -= 1
        steps += 1
    assert steps <= 1
    part = vb - (t + t * s // n)
    ns = 2 if (t + 1) * s // n > t * s // n else 1
    return t, part, ns


def _check(n, fp64):
    s = n_split(n, fp64)
    nblk = n + s
    seen = {}
    for b in range(nblk):
        vb = xcd_tile(b, nblk)
        assert 0 <= vb < nblk
        t, part, ns = tile_of(vb, n, s)
        assert 0 <= t < n and 0 <= part < ns
        assert (t, part) not in seen
        seen[(t, part)] = ns
    split = 0
    for t in range(n):
        ns = seen[(t, 0)]
        assert all(seen[(t, w)] == ns for w in range(ns)) and (t, ns) not in seen
        split += ns == 2
    assert split == s


def test_every_launch_size_covers_each_tile_half_once():
    for fp64 in (False, True):
        for n in range(1, 2200):
            _check(n, fp64)
        for n in (4096, 20480):
            _check(n, fp64)


def test_headline_launch_spreads_whole_tiles_over_xcds():
    # 81,920 triangles: 1,280 tiles, 768 split, 2,048 workgroups (two per SIMD);
    # the 512 whole tiles fall 64 on each XCD
    n = 1280
    s = n_split(n, False)
    assert s == 768
    whole = [0] * 8
    for b in range(n + s):
        _, _, ns = tile_of(xcd_tile(b, n + s), n, s)
        whole[b % 8] += ns == 1
    assert whole == [64] * 8


def test_library_mapping_functions(tmp_path):
    """The same check through the library's own functions: a host program
    built from q2x_internal.hpp (xcd_tile, split_tile, split_count -- the code
    the kernel and the host call) checks every launch of up to 2,199 tiles."""
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    exe = tmp_path / "split_map_check"
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", os.path.join(here, "..", "include"),
                    os.path.join(here, "split_map_check.hip"), "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe), "2199"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "checked 4398 launches" in r.stdout

"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point that include/wacm.h declares, and its host-only treecode
helpers agree bit for bit with the oracle's independent implementation."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1912_05371_amd import wacm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "wacm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wacm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = wacm.lib()
    decl = declared_symbols()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(decl) == sorted(wacm.EXPORTS)


def test_struct_sizes_match_header():
    # wacm_grid_desc: 6 int32 + int64 + double; wacm_params: see header
    assert ctypes.sizeof(wacm.GridDesc) == 40
    assert ctypes.sizeof(wacm.Params) == 8 * 10 + 4 * 4 + 8 * 20


def test_treecode_matches_oracle(orc):
    rng = np.random.default_rng(9)
    for _ in range(500):
        J = int(rng.integers(0, 19))
        x, y, z = (int(v) for v in rng.integers(0, 1 << J, 3)) if J else (0, 0, 0)
        c = wacm.treecode_encode(J, x, y, z)
        assert c == orc.treecode_encode(J, x, y, z)
        assert wacm.treecode_decode(c, J) == (x, y, z)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(wacm, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(wacm, "_lib", None)
    with pytest.raises(RuntimeError):
        wacm.lib()


# ---------------------------------------------------------------- error codes
# Every failure below is detected by the host-side validation that runs
# before the library touches any device buffer, so the fake (aligned, never
# dereferenced) device addresses are safe without a GPU.  None of these
# calls has a valid full argument set.
FAKE_DEV = 1 << 40  # 256-byte aligned, never dereferenced


def _desc(bs=16, ng=4, jmin=1, jmax=3, dtype=wacm.F64, cap=64, L=1.0, dim=3):
    return wacm.GridDesc(bs, ng, jmin, jmax, dtype, dim, cap, L)


def _create(desc, leaves, ws=FAKE_DEV, ws_bytes=None):
    L = wacm.lib()
    lev = np.array([l[0] for l in leaves], np.int8)
    codes = np.array([wacm.treecode_encode(*l) for l in leaves], np.uint64)
    if ws_bytes is None:
        ws_bytes = int(L.wacm_workspace_bytes(ctypes.byref(desc)))
    h = ctypes.c_void_p()
    rc = L.wacm_grid_create(ctypes.byref(desc), len(leaves), codes.ctypes.data_as(ctypes.c_void_p),
                            lev.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ws), ws_bytes,
                            ctypes.byref(h))
    assert not h.value  # no handle on failure
    return rc, L.wacm_last_error(None).decode()


def _uniform(J):
    n = 1 << J
    return [(J, x, y, z) for z in range(n) for y in range(n) for x in range(n)]


def test_workspace_bytes():
    L = wacm.lib()
    a = int(L.wacm_workspace_bytes(ctypes.byref(_desc(cap=64))))
    b = int(L.wacm_workspace_bytes(ctypes.byref(_desc(cap=128))))
    assert a > 64 * 928 and b > a and a % 256 == 0 and b % 256 == 0
    for bad in (_desc(bs=18), _desc(ng=2), _desc(dtype=3), _desc(cap=0), _desc(dim=1),
                _desc(jmin=4, jmax=3), _desc(L=0.0)):
        assert L.wacm_workspace_bytes(ctypes.byref(bad)) == 0


def test_grid_create_inval():
    leaves = _uniform(1)
    for desc, what in ((_desc(bs=20), "bs"), (_desc(ng=2), "ng"), (_desc(dtype=0), "dtype"),
                       (_desc(cap=4), "capacity"), (_desc(dim=7), "dim")):
        rc, msg = _create(desc, leaves)
        assert rc == wacm.E_INVAL, (what, rc)
        assert msg
    d = _desc()
    need = int(wacm.lib().wacm_workspace_bytes(ctypes.byref(d)))
    assert _create(d, leaves, ws=0)[0] == wacm.E_INVAL                    # NULL workspace
    assert _create(d, leaves, ws=FAKE_DEV + 64)[0] == wacm.E_INVAL        # misaligned
    rc, msg = _create(d, leaves, ws_bytes=need - 256)                     # too small
    assert rc == wacm.E_INVAL and "workspace" in msg
    rc, msg = _create(d, [(4, 0, 0, 0)] + leaves[1:])                      # level above jmax
    assert rc == wacm.E_INVAL


def test_grid_create_tiling():
    leaves = _uniform(1)
    rc, msg = _create(_desc(), leaves + [leaves[3]])                       # repeated leaf
    assert rc == wacm.E_TILING and "repeated" in msg
    rc, msg = _create(_desc(), leaves[:-1])                                # a gap
    assert rc == wacm.E_TILING and "cover" in msg
    kids = [(2, 2 * 1 + (c & 1), (c >> 1) & 1, (c >> 2) & 1) for c in range(8)]
    rc, msg = _create(_desc(), leaves + kids)                              # overlap
    assert rc == wacm.E_TILING and "inside" in msg


def test_grid_create_unbalanced():
    # block (0,0,0) of level 1 split to level 2, one of those to level 3: the
    # level-3 leaves touch level-1 leaves (a 2-level jump)
    leaves = [l for l in _uniform(1) if l != (1, 0, 0, 0)]
    l2 = [(2, c & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8)]
    l2.remove((2, 1, 1, 1))
    l3 = [(3, 2 + (c & 1), 2 + ((c >> 1) & 1), 2 + ((c >> 2) & 1)) for c in range(8)]
    rc, msg = _create(_desc(jmax=3, cap=64), leaves + l2 + l3)
    assert rc == wacm.E_UNBALANCED and "balanced" in msg


def _uniform2(J):
    n = 1 << J
    return [(J, x, y, 0) for y in range(n) for x in range(n)]


def test_grid_create_2d_errors():
    # quadtrees: treecodes of (bx, by, 0), areas add up in 2D, 2:1 in the plane
    leaves = _uniform2(2)
    d2 = _desc(jmin=1, jmax=3, dim=2)
    rc, msg = _create(d2, leaves[:-1])
    assert rc == wacm.E_TILING and "cover" in msg
    rc, msg = _create(d2, leaves[:-1] + [(2, 3, 3, 1)])  # a z index in 2D
    assert rc == wacm.E_INVAL and "two dimensions" in msg
    rc, msg = _create(d2, leaves + [leaves[0]])
    assert rc == wacm.E_TILING
    # level 1 next to level 3: (1, 1, 1, 0) replaced by level-2 children,
    # one of which is split to level 3 at the corner touching level 1
    base = [(1, x, y, 0) for y in range(2) for x in range(2) if (x, y) != (0, 0)]
    l2 = [(2, x, y, 0) for y in range(2) for x in range(2) if (x, y) != (0, 0)]
    l3 = [(3, x, y, 0) for y in range(2) for x in range(2)]
    rc, msg = _create(d2, base + l2 + l3)
    assert rc == wacm.E_UNBALANCED
    # the octree reading of the same codes is not a tiling of the cube
    assert _create(_desc(jmin=2, jmax=2), leaves)[0] == wacm.E_TILING


def test_mr_work_buffer_checked_before_launch():
    L = wacm.lib()
    n, nf = 16, 2
    need = int(L.wacm_mr_work_bytes(n, nf, wacm.F64))
    assert need > 0
    u = ctypes.c_void_p(FAKE_DEV)
    for work, size, text in ((FAKE_DEV, need - 8, "smaller"), (FAKE_DEV + 8, need, "aligned"),
                             (0, need, "needs the work")):
        rc = L.wacm_mr_forward(n, nf, wacm.F64, wacm.CDF44, 1, u, ctypes.c_void_p(work), size,
                               None)
        assert rc == wacm.E_INVAL
        assert text in L.wacm_last_error(None).decode()
        rc = L.wacm_mr_inverse(n, nf, wacm.F64, wacm.CDF44, 2, u, ctypes.c_void_p(work), size,
                               None)
        assert rc == wacm.E_INVAL


def test_last_error_of_null_grid_is_thread_text():
    L = wacm.lib()
    assert L.wacm_grid_nb(None) == -1
    assert L.wacm_sync_ghosts(None, ctypes.c_void_p(FAKE_DEV), None) == wacm.E_INVAL
    assert "NULL" in L.wacm_last_error(None).decode()

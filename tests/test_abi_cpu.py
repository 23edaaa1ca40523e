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

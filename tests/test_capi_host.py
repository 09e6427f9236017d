"""CPU-side checks of the C ABI library: it loads, exports every entry point
declared in include/rsgdf.h, and validates arguments on the host (no kernel
is launched here: these calls fail before any device work)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2102_02989_amd as P
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rsgdf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\s*\*?\s*(rsgdf_[a-z0-9_]+)\s*\(", src, re.M)))


def test_library_exports_declared_symbols():
    lib = P.library()
    syms = declared_symbols()
    assert "rsgdf_build_j3c" in syms and "rsgdf_j3c_nbytes" in syms
    for s in syms:
        assert hasattr(lib, s), s
    assert P.version().startswith("rsgdf")


def test_nbytes_matches_layout():
    p = synth.config2()
    n = P.j3c_nbytes(p.cell, p.basis, p.aux, p.kmesh)
    assert n == 36 * 560 * 120 * 120 * 16
    p1 = synth.config1()
    assert P.j3c_nbytes(p1.cell, p1.basis, p1.aux, p1.kmesh) == 1 * 32 * 10 * 10 * 16


def _expect(code, fn):
    with pytest.raises(P.RsgdfError) as ei:
        fn()
    assert ei.value.code == code


def test_argument_validation_on_host():
    p = synth.tiny_problem()
    host = np.zeros((1, p.aux.nfunc, p.basis.nfunc, p.basis.nfunc), np.complex128)
    # bad kmesh
    _expect(-1, lambda: P.j3c_nbytes(p.cell, p.basis, p.aux, (0, 1, 1)))
    # non-positive exponent
    bad = synth.tiny_problem()
    bad.basis.exps = bad.basis.exps.copy()
    bad.basis.exps[0] = -1.0
    _expect(-1, lambda: P.j3c_nbytes(bad.cell, bad.basis, bad.aux, bad.kmesh))
    # unsupported angular momentum (AO g shell)
    bad2 = synth.tiny_problem()
    bad2.basis.shell_l = bad2.basis.shell_l.copy()
    bad2.basis.shell_l[0] = 4
    _expect(-5, lambda: P.j3c_nbytes(bad2.cell, bad2.basis, bad2.aux, bad2.kmesh))
    # omega <= 0 and thresh <= 0 are rejected before any device call
    _expect(-1, lambda: P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, 0.0, 1e-10, host))
    _expect(-1, lambda: P.build_j3c(p.cell, p.basis, p.aux, p.kmesh, 0.5, -1.0, host))
    # undersized output buffer: ESIZE, nothing written
    small = np.zeros(3, np.complex128)
    lib = P.library()
    m = P.rsgdf._Marshal(p.cell, p.basis, p.aux, p.kmesh)
    o = P.rsgdf.Out(small.ctypes.data, small.nbytes, 0, None, 0, 0, 0, None)
    rc = lib.rsgdf_build_j3c(ctypes.byref(m.cell), ctypes.byref(m.basis), ctypes.byref(m.aux), m.kmesh.ctypes.data,
                             0.5, 1e-10, ctypes.byref(o))
    assert rc == -2
    assert "capacity" in lib.rsgdf_last_error().decode()
    # singular lattice
    sing = synth.tiny_problem()
    sing.cell.lattice = np.zeros((3, 3))
    _expect(-1, lambda: P.build_j3c(sing.cell, sing.basis, sing.aux, sing.kmesh, 0.5, 1e-10, host))


def test_product_path_has_no_fallback(monkeypatch):
    """Without the native library the binding raises instead of computing."""
    import paper_2102_02989_amd.rsgdf as R
    monkeypatch.setattr(R, "_LIB_PATH", "/nonexistent/librsgdf.so")
    monkeypatch.setattr(R, "_lib", None)
    with pytest.raises(R.RsgdfError):
        R.library()


def test_library_matches_tree_sources():
    """The library records the hash of the sources it was built from; the
    loaded one is the tree's, and a library built from other sources is
    refused rather than run."""
    import paper_2102_02989_amd.build as B
    import paper_2102_02989_amd.rsgdf as R
    assert P.library().rsgdf_source_hash().decode() == B.source_hash()


def test_stale_library_is_refused(monkeypatch):
    import paper_2102_02989_amd.build as B
    import paper_2102_02989_amd.rsgdf as R
    monkeypatch.setattr(R, "_lib", None)
    monkeypatch.setattr(B, "source_hash", lambda: "0000000000000000")
    with pytest.raises(R.RsgdfError, match="other sources"):
        R.library()

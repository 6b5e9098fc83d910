"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and validates arguments on the host without a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rwseg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rw_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("rw_ctx_create", "rw_ctx_destroy", "rw_solve_bricks", "rw_solve_bricks_adjoint",
              "rw_last_error", "rw_version", "rw_validate_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2103_09564_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_validation():
    import paper_2103_09564_amd as rwg
    b = rwg.bricks_array([[4, 3, 2], [2, 2, 2]], [0, 24])
    ok, _ = rwg.validate_solve(rwg.solve_params(), b, 32)
    assert ok == 0
    cases = [
        (rwg.solve_params(nrhs=0), b, 32, "nrhs"),
        (rwg.solve_params(beta=-1.0), b, 32, "beta"),
        (rwg.solve_params(tol=float("nan")), b, 32, "tol"),
        (rwg.solve_params(precision=7), b, 32, "precision"),
        (rwg.solve_params(max_iter=-2), b, 32, "max_iter"),
        (rwg.solve_params(), b, 31, "outside"),
        (rwg.solve_params(), rwg.bricks_array([[4, 3, 2], [2, 2, 2]], [0, 20]), 32, "overlap"),
        (rwg.solve_params(), rwg.bricks_array([[0, 3, 2]], [0]), 32, "dims"),
        (rwg.solve_params(), rwg.bricks_array([[2, 2, 2]], [-1]), 32, "outside"),
    ]
    for p, bb, nv, word in cases:
        rc, msg = rwg.validate_solve(p, bb, nv)
        assert rc == -1 and word in msg, (word, rc, msg)
    bad = b.copy()
    bad["reserved"][0] = 1
    rc, msg = rwg.validate_solve(rwg.solve_params(), bad, 32)
    assert rc == -1 and "reserved" in msg


def test_params_defaults():
    import paper_2103_09564_amd as rwg
    p = rwg.solve_params()
    assert (p.beta, p.eps, p.tol, p.max_iter, p.nrhs) == (128.0, 1e-6, 1e-6, 5000, 1)
    assert p.precision == rwg.PREC_MIXED
    with pytest.raises(TypeError):
        rwg.solve_params(bogus=1)


def test_noalloc_scratch_size_is_stated():
    import paper_2103_09564_amd as rwg
    assert rwg.noalloc_scratch_bytes() == 64 << 20

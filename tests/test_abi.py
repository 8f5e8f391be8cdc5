"""CPU-side checks of the C-ABI: the library loads, exports every symbol the
header declares, and rejects invalid problems before touching a device."""
import os
import re

import numpy as np
import pytest

from paper_2601_18705_amd import dlrtrt
from synth import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "dlrtrt.h")).read()
    return sorted(set(re.findall(r"\b(dlr_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _header_functions() == sorted(dlrtrt.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(dlrtrt.LIB_PATH):
        pytest.skip("libdlrtrt.so not built")
    lib = dlrtrt.library()
    for name in _header_functions():
        assert hasattr(lib, name), name
    assert lib.dlr_status_string(-4).decode() == "source iteration did not converge"


def _bad(**kw):
    p = problems.slab_beam(nx=8, n_polar=2, n_azim=4, rank=2)
    p.update(kw)
    return p


@pytest.mark.parametrize("kw,status", [
    (dict(rank=0), -1), (dict(rank=65), -1), (dict(rank=9), -1),          # rank > ordinates (8)
    (dict(n_azim=6), -1), (dict(dt=0.0), -1),
    (dict(bc=[2, 0, 0, 0]), -7), (dict(precision=3), -1), (dict(precision=5), -1),
    (dict(si_max_iter=0), -1), (dict(deim_tie_tol=1.0), -1),
])
def test_create_rejects_invalid_problems(kw, status):
    if not os.path.exists(dlrtrt.LIB_PATH):
        pytest.skip("libdlrtrt.so not built")
    p = _bad(**kw)
    with pytest.raises(dlrtrt.DlrError) as ei:
        dlrtrt.Instance(p)
    assert ei.value.status == status


@pytest.mark.parametrize("kw,status", [
    (dict(n_azim=6), -1), (dict(dt=0.0), -1), (dict(bc=[2, 0, 0, 0]), -7), (dict(precision=3), -1),
    (dict(si_max_iter=0), -1), (dict(n_polar=200, n_azim=128), -1),
])
def test_sn_create_rejects_invalid_problems(kw, status):
    if not os.path.exists(dlrtrt.LIB_PATH):
        pytest.skip("libdlrtrt.so not built")
    p = _bad(**kw)
    with pytest.raises(dlrtrt.DlrError) as ei:
        dlrtrt.Instance(p, method="sn")
    assert ei.value.status == status


@pytest.mark.parametrize("args", [
    (0, 4, 0.1, 0.1, [0.5], [0.5], 0), (4, 0, 0.1, 0.1, [0.5], [0.5], 0),
    (1 << 15, 1 << 14, 0.1, 0.1, [0.5], [0.5], 0),                          # more than 2^28 cells
    ((1 << 20) + 1, 1, 0.1, 0.1, [0.5], [0.5], 0),                          # a side above 2^20
    (4, 4, 0.0, 0.1, [0.5], [0.5], 0), (4, 4, 0.1, float("inf"), [0.5], [0.5], 0),
    (4, 4, 0.1, 0.1, [0.0], [0.0], 0), (4, 4, 0.1, 0.1, [float("nan")], [0.5], 0),
    (4, 4, 0.1, 0.1, [0.5], [0.5], 2), (4, 4, 0.1, 0.1, [0.5], [0.5], 7),
])
def test_q1_create_rejects_invalid_arguments(args):
    if not os.path.exists(dlrtrt.LIB_PATH):
        pytest.skip("libdlrtrt.so not built")
    with pytest.raises(dlrtrt.DlrError) as ei:
        dlrtrt.Q1Sweep(*args)
    assert ei.value.status == -1


def test_create_rejects_nonpositive_fields():
    if not os.path.exists(dlrtrt.LIB_PATH):
        pytest.skip("libdlrtrt.so not built")
    p = _bad()
    p["sigma_a"] = p["sigma_a"].copy()
    p["sigma_a"][3] = 0.0
    with pytest.raises(dlrtrt.DlrError) as ei:
        dlrtrt.Instance(p)
    assert ei.value.status == -1


def test_batch_footprint_grows_with_grid_and_rank():
    from paper_2601_18705_amd import dlrtrt
    small = problems.slab_beam(nx=32, n_polar=4, n_azim=8, rank=4)
    big = problems.slab_beam(nx=64, n_polar=4, n_azim=8, rank=4)
    wide = problems.slab_beam(nx=32, n_polar=4, n_azim=8, rank=16)
    fs, fb, fw = (dlrtrt.footprint(p) for p in (small, big, wide))
    assert 0 < fs < fb and fs < fw


def test_batch_footprint_validates():
    from paper_2601_18705_amd import dlrtrt
    p = problems.slab_beam(nx=32, n_polar=4, n_azim=8, rank=4)
    p["rank"] = 1000
    with pytest.raises(dlrtrt.DlrError) as ei:
        dlrtrt.footprint(p)
    assert ei.value.status == -1


def test_set_allocator_needs_both_functions_or_neither():
    if not os.path.exists(dlrtrt.LIB_PATH):
        pytest.skip("libdlrtrt.so not built")
    lib = dlrtrt.library()
    keep = dlrtrt.ALLOC_FN(lambda n, s, u: None)
    assert lib.dlr_set_allocator(keep, dlrtrt.RELEASE_FN(), None) == -1
    assert lib.dlr_set_allocator(dlrtrt.ALLOC_FN(), dlrtrt.RELEASE_FN(), None) == 0
    assert lib.dlr_status_string(-9).decode() == "device wait exceeded its spin limit"

"""CPU: the C-ABI library loads, exports exactly what include/epo.h declares,
and rejects bad arguments on the host (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epo.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"EPO_API\s+[\w\s\*]+?\b(epo_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2607_00579_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libepo.so is not built (run __graft_entry__.build())")
    return _lib


def test_header_lists_the_four_calls():
    names = declared()
    for n in ("epo_build_distance_fields", "epo_edge_cost_fwd", "epo_edge_cost_bwd",
              "epo_pose_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    L = lib.load()
    for name in declared():
        assert hasattr(L, name), name
    assert sorted(lib.EXPORTS) == declared()


def test_only_declared_symbols_are_exported(lib):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    funcs = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert funcs == declared()


def test_version_and_error_paths(lib):
    assert "gfx950" in lib.version()
    with pytest.raises(lib.EpoError) as e:
        lib.build_distance_fields(None, None, None, None, 3, None, None, None)
    assert e.value.status == lib.ERR_INVALID_ARG
    w = np.array([20000], np.int32)
    h = np.array([5], np.int32)
    off = np.zeros(1, np.int64)
    with pytest.raises(lib.EpoError) as e:
        lib.build_distance_fields(1, off, w, h, 1, 1, 1, None)
    assert "side" in str(e.value)
    with pytest.raises(lib.EpoError):
        lib.plan_create(0, w, h, np.ones(4, np.float32), None, off, 1, 1, 1, None, 0, None, None,
                        None)
    with pytest.raises(lib.EpoError):
        lib.pose_step(None, None, None, None, 2, None, None, None, 0.9, 0.999, 1e-8, None, None)
    # zero views is a valid no-op for the distance transform
    lib.build_distance_fields(None, None, None, None, 0, None, None, None)


def test_struct_layouts(lib):
    assert C.sizeof(lib.CostParams) == 16
    assert C.sizeof(lib.PlanOptions) == 16

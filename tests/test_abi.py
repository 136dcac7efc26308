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
    with pytest.raises(lib.EpoError) as e:
        lib.plan_set_refinement(None, None, None, None, None)
    assert e.value.status == lib.ERR_INVALID_ARG and "null plan" in str(e.value)
    with pytest.raises(lib.EpoError) as e:
        lib.edge_cost_refine(None, None, None, None, None, None, None, None, None, None)
    assert e.value.status == lib.ERR_INVALID_ARG
    with pytest.raises(lib.EpoError) as e:
        lib.joint_step(None, None, None, None, None, None, None, None, None, None, None, None,
                       None, 0.9, 0.999, 1e-8, 0.01, 0.01, None, None)
    assert e.value.status == lib.ERR_INVALID_ARG and "null plan" in str(e.value)
    with pytest.raises(lib.EpoError) as e:
        lib.plan_resort(None, None, None, 1, None)
    assert e.value.status == lib.ERR_INVALID_ARG
    with pytest.raises(lib.EpoError) as e:
        lib.plan_pair_records(None, 0)
    assert e.value.status == lib.ERR_INVALID_ARG
    # zero views is a valid no-op for the distance transform
    lib.build_distance_fields(None, None, None, None, 0, None, None, None)


def _host_only():
    """These calls pass placeholder device pointers and must be rejected on
    the host; never run them where a GPU could be reached."""
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("host-validation test: runs only without a GPU")


def _plan_args(**over):
    a = dict(n_views=2, width=np.array([40, 40], np.int32), height=np.array([30, 30], np.int32),
             K=np.tile(np.array([32, 32, 19.5, 14.5], np.float32), 2),
             scene_of_view=np.array([0, 0], np.int32), view_offset=np.array([0, 1200], np.int64),
             edge_maps=1, depth=1, d2=1, pairs=np.array([[0, 1], [1, 0]], np.int32), n_pairs=2,
             params=None, options=None, stream=None)
    a.update(over)
    return a


@pytest.mark.parametrize("over,needle", [
    (dict(width=np.array([40, 1], np.int32)), "side"),
    (dict(width=np.array([40, 16385], np.int32)), "side"),
    (dict(pairs=np.array([[0, 2], [1, 0]], np.int32)), "out of range"),
    (dict(scene_of_view=np.array([0, 1], np.int32)), "different scenes"),
    (dict(scene_of_view=np.array([0, 2], np.int32), pairs=np.array([[0, 0], [1, 1]], np.int32)),
     "without gaps"),
    (dict(K=np.array([32, 32, 19.5, 14.5, -1, 32, 19.5, 14.5], np.float32)), "focal"),
    (dict(view_offset=np.array([0, -5], np.int64)), "negative offset"),
    (dict(n_views=0), "n_views"),
    (dict(edge_maps=None), "null"),
])
def test_plan_create_rejects_bad_arguments_on_host(lib, over, needle):
    _host_only()
    with pytest.raises(lib.EpoError) as e:
        lib.plan_create(**_plan_args(**over))
    assert e.value.status == lib.ERR_INVALID_ARG
    assert needle in str(e.value), str(e.value)


def test_plan_create_rejects_unsupported_texture(lib):
    _host_only()
    with pytest.raises(lib.EpoError) as e:
        lib.plan_create(**_plan_args(params=lib.CostParams(1.0, 1e-4, 0, 20.0),
                                     options=lib.PlanOptions(2, 4, 1, 2)))
    assert e.value.status == lib.ERR_UNSUPPORTED
    with pytest.raises(lib.EpoError) as e:
        lib.plan_create(**_plan_args(options=lib.PlanOptions(4, 4, 1, 2)))
    assert e.value.status == lib.ERR_INVALID_ARG
    with pytest.raises(lib.EpoError) as e:
        lib.plan_create(**_plan_args(options=lib.PlanOptions(1, 3, 1, 2)))
    assert "points_per_thread" in str(e.value)
    with pytest.raises(lib.EpoError) as e:
        lib.plan_create(**_plan_args(options=lib.PlanOptions(1, 4, 1, 2, 3, 0)))
    assert "record_order" in str(e.value)
    with pytest.raises(lib.EpoError) as e:
        lib.plan_create(**_plan_args(options=lib.PlanOptions(1, 4, 1, 2, 2, -1)))
    assert "resort_interval" in str(e.value)
    for bad in (-1, 65):
        with pytest.raises(lib.EpoError) as e:
            lib.plan_create(**_plan_args(options=lib.PlanOptions(1, 4, 1, 2, 1, 8, bad)))
        assert "graph_steps" in str(e.value)


def test_struct_layouts(lib):
    assert C.sizeof(lib.CostParams) == 16
    assert C.sizeof(lib.PlanOptions) == 28


@pytest.mark.parametrize("z_min", [0.0, -1.0, 1e-9, 1e7, float("nan")])
def test_plan_create_rejects_z_min_out_of_range(lib, z_min):
    _host_only()
    with pytest.raises(lib.EpoError) as e:
        lib.plan_create(**_plan_args(params=lib.CostParams(1.0, z_min, 0, 10.0)))
    assert e.value.status == lib.ERR_INVALID_ARG and "z_min" in str(e.value)


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback path: without libepo.so the binding raises."""
    from paper_2607_00579_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libepo.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.load()


def test_cpu_device_is_refused():
    """The package has no CPU path: a plan on a CPU device is refused."""
    from paper_2607_00579_amd.api import EdgePlan
    from synth import fixtures
    p = fixtures.odd_size_views()
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        EdgePlan.from_problem(p, device="cpu")


def test_noalloc_viewgraph_rejects_staging_beyond_its_array(lib):
    """Three 16384 x 16384 views at grid stride 1 need 786432 work chunks of
    staging, more than the 4 MiB static array: refused on the host."""
    _host_only()
    w = np.full(3, 16384, np.int32)
    K = np.tile(np.array([1000, 1000, 8191.5, 8191.5], np.float32), 3)
    off = np.arange(3, dtype=np.int64) * 16384 * 16384
    cand = np.array([[0, 1], [0, 2], [1, 2]], np.int32)
    with pytest.raises(lib.EpoError) as e:
        lib.build_viewgraph_noalloc(3, w, w, K, off, 1, 1, cand, 3, 1, 3.0, 0.125, 1e-4, 1, 1,
                                    None, None)
    assert e.value.status == lib.ERR_INVALID_ARG and "no-allocation" in str(e.value)

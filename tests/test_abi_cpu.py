"""The C-ABI library without a GPU: it loads, exports every entry point that
include/bmg.h declares, and rejects bad arguments on the host before any
device call."""
import ctypes as C
import os
import re

import pytest

from paper_2502_05279_amd import boxmg, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bmg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if build.needs_build():
        build.build()
    return boxmg.lib()


def test_library_exports_every_declared_entry_point(L):
    names = declared_functions()
    assert len(names) >= 15
    missing = [nm for nm in names if not hasattr(L, nm)]
    assert not missing, missing


def test_binding_covers_every_entry_point(L):
    import inspect
    src = inspect.getsource(boxmg)
    for nm in declared_functions():
        assert f'"{nm}"' in src, nm


def test_default_options(L):
    o = boxmg.default_options()
    assert (o.nu1, o.nu2, o.max_cycles, o.precision, o.check_every) == (2, 1, 100, 0, 8)
    # every field in the header's order (a field out of place in the binding
    # would show here as a wrong default)
    assert (o.kernels, o.refine_factor, o.tile_rows, o.interp, o.learned_levels, o.smoother, o.coarsest_n,
            o.persistent_below_n, o.square_tiles_below_n, o.graph_mode) == (1, 16, 0, 0, 0, 0, 0, 0, 0, 0)
    assert not o.net


@pytest.mark.parametrize("n", [0, 1, 2, 4, 100, 4096, -1])
def test_workspace_rejects_bad_sizes(L, n):
    out = C.c_size_t(0)
    assert L.bmg_workspace_bytes(n, 5, None, C.byref(out)) == boxmg.BMG_EINVAL
    assert b"2^m-1" in L.bmg_last_error()


def test_workspace_rejects_bad_kind_and_options(L):
    out = C.c_size_t(0)
    assert L.bmg_workspace_bytes(127, 7, None, C.byref(out)) == boxmg.BMG_EINVAL
    assert L.bmg_workspace_bytes(127, 5, None, None) == boxmg.BMG_EINVAL
    for bad in ({"nu1": -1}, {"nu1": 0, "nu2": 0}, {"max_cycles": 0}, {"precision": 7},
                {"kernels": 9}, {"check_every": 0}, {"smoother": 5},
                {"smoother": boxmg.BMG_SMOOTH_LINE, "precision": boxmg.BMG_FP32_IR},
                {"square_tiles_below_n": 100}, {"square_tiles_below_n": -1}, {"graph_mode": 2},
                {"persistent_below_n": 127}):
        o = boxmg.default_options(**bad)
        assert L.bmg_workspace_bytes(127, 5, C.byref(o), C.byref(out)) == boxmg.BMG_EINVAL, bad


def test_workspace_sizes_scale_with_the_grid(L):
    sizes = [boxmg.workspace_bytes(n) for n in (7, 127, 1023, 4095)]
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    # FP64 hierarchy at 4095^2: two iterate buffers, b, r and 3 stencil planes on
    # the fine level, the refinement arrays (rhs, iterate high and low parts),
    # 8 weight planes of 2049^2, nine-point coarse levels: about 2.1 GB
    assert 1.8e9 < sizes[-1] < 2.5e9
    assert boxmg.workspace_bytes(4095, precision=boxmg.BMG_FP32_IR) > sizes[-1] * 1.3
    assert boxmg.workspace_bytes(4095, 9) > sizes[-1]


def test_setup_validates_on_the_host_before_any_device_call(L):
    h = C.c_void_p(None)
    fake = C.c_void_p(0x1000)   # never dereferenced: every check below is on the host
    assert L.bmg_setup(C.byref(h), fake, 100, 5, None, fake, 1 << 30, None) == boxmg.BMG_EINVAL
    assert L.bmg_setup(C.byref(h), None, 127, 5, None, fake, 1 << 30, None) == boxmg.BMG_EINVAL
    assert L.bmg_setup(C.byref(h), fake, 127, 6, None, fake, 1 << 30, None) == boxmg.BMG_EINVAL
    assert L.bmg_setup(None, fake, 127, 5, None, fake, 1 << 30, None) == boxmg.BMG_EINVAL
    # missing, small or misaligned workspace
    assert L.bmg_setup(C.byref(h), fake, 127, 5, None, None, 1 << 30, None) == boxmg.BMG_EWORKSPACE
    assert L.bmg_setup(C.byref(h), fake, 127, 5, None, fake, 1024, None) == boxmg.BMG_EWORKSPACE
    odd = C.c_void_p(0x1008)
    assert L.bmg_setup(C.byref(h), fake, 127, 5, None, odd, 1 << 30, None) == boxmg.BMG_EWORKSPACE
    assert h.value is None


def test_entry_points_reject_null_handles(L):
    fake = C.c_void_p(0x1000)
    assert L.bmg_vcycle(None, fake, fake, None) == boxmg.BMG_EINVAL
    assert L.bmg_solve(None, fake, fake, C.c_double(1e-10), None) == boxmg.BMG_EINVAL
    assert L.bmg_step(None, 0, 0, 1, 0) == boxmg.BMG_EINVAL
    assert L.bmg_export(None, 0, 0, fake) == boxmg.BMG_EINVAL
    assert L.bmg_discretize(None, None, 127, None, None, None) == boxmg.BMG_EINVAL
    assert L.bmg_discretize(fake, fake, 126, fake, fake, None) == boxmg.BMG_EINVAL
    assert L.bmg_destroy(None) == boxmg.BMG_OK
    n = C.c_int(0)
    assert L.bmg_num_levels(None, C.byref(n)) == boxmg.BMG_EINVAL


def test_status_strings(L):
    for s in range(-6, 1):
        assert L.bmg_status_string(s)
    assert L.bmg_status_string(-99) == b"unknown status"


def test_batch_and_tuning_validation(L):
    out = C.c_size_t(0)
    ns = (C.c_int * 3)(127, 63, 100)
    assert L.bmg_batch_workspace_bytes(3, ns, None, C.byref(out)) == boxmg.BMG_EINVAL
    ns = (C.c_int * 2)(127, 3)
    assert L.bmg_batch_workspace_bytes(2, ns, None, C.byref(out)) == boxmg.BMG_EINVAL
    ns = (C.c_int * 2)(127, 63)
    assert L.bmg_batch_workspace_bytes(2, ns, None, C.byref(out)) == boxmg.BMG_OK
    assert out.value > 2 * boxmg.workspace_bytes(63)
    o = boxmg.default_options(nu1=1)
    assert L.bmg_batch_workspace_bytes(2, ns, C.byref(o), C.byref(out)) == boxmg.BMG_EINVAL
    assert L.bmg_batch_solve(None, None, None, C.c_double(1e-10), None, None) == boxmg.BMG_EINVAL
    assert L.bmg_batch_destroy(None) == boxmg.BMG_OK
    # the tile-rows table
    default = boxmg.tile_rows_get(4095)
    assert default > 0 and default % 2 == 0
    boxmg.tile_rows_set(4095, 6)
    assert boxmg.tile_rows_get(4095) == 6
    boxmg.tile_rows_set(4095, 0)
    assert boxmg.tile_rows_get(4095) == default
    assert L.bmg_tile_rows_set(4095, 7) == boxmg.BMG_EINVAL
    assert L.bmg_tile_rows_set(100, 8) == boxmg.BMG_EINVAL


def test_bench_traffic_record_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    """bench.py reports measured traffic only while the sources the counters
    were taken on are unchanged: a record with another hash gives None."""
    import json
    import bench
    root = tmp_path
    (root / "profiles").mkdir()
    (root / "k.hpp").write_text("kernel v1")
    import hashlib
    good = hashlib.sha256(b"kernel v1").hexdigest()
    rec = {"w fp64 pre": {"sources": ["k.hpp"], "sources_sha256": good, "traffic_bytes_per_launch": 123},
           "w fp64 post": {"sources": ["k.hpp"], "sources_sha256": "0" * 64, "traffic_bytes_per_launch": 5}}
    (root / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic("w fp64 pre") == 123
    rec["w fp64 pre"]["tile_rows"] = 96
    (root / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("w fp64 pre", 96) == 123
    assert bench.measured_traffic("w fp64 pre", 32) is None
    assert bench.measured_traffic("w fp64 post") is None
    assert bench.measured_traffic("other") is None
    (root / "k.hpp").write_text("kernel v2")
    assert bench.measured_traffic("w fp64 pre") is None


def test_block_entry_points_validate_on_the_host(L):
    """Block entry points reject NULL handles and arguments before any device
    call."""
    sz = C.c_size_t(0)
    assert L.bmg_block_workspace_bytes(None, 2, C.byref(sz)) == boxmg.BMG_EINVAL
    out = C.c_void_p(None)
    assert L.bmg_block_create(C.byref(out), None, 2, None, 0) == boxmg.BMG_EINVAL
    assert L.bmg_block_create(None, None, 2, None, 0) == boxmg.BMG_EINVAL
    assert L.bmg_block_solve(None, None, None, 1e-10, None, None) == boxmg.BMG_EINVAL
    assert L.bmg_block_trace_enable(None, 1, 0, 1) == boxmg.BMG_EINVAL
    n, ms = C.c_int(0), C.c_double(0)
    assert L.bmg_block_trace_read(None, C.byref(n), C.byref(ms), None) == boxmg.BMG_EINVAL
    assert L.bmg_block_destroy(None) == boxmg.BMG_OK

"""C-ABI checks that need no GPU: every declared entry point is exported, size
queries are sane, and argument errors are reported before any device work."""
import ctypes as ct
import os
import re

import pytest

from paper_2305_18663_amd import sbp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbp.h")

needs_lib = pytest.mark.skipif(not os.path.exists(sbp.LIB_PATH), reason="libsbp.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("sbp_build_blockmodel", "sbp_nodal_sweep", "sbp_merge_scores", "sbp_description_length",
                     "sbp_partition", "sbp_partition_batch", "sbp_merge_apply", "sbp_compact",
                     "sbp_engine_create", "sbp_engine_admit", "sbp_engine_step", "sbp_last_error"):
        assert required in names


@needs_lib
def test_every_declared_symbol_is_exported():
    L = ct.CDLL(sbp.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@needs_lib
def test_binding_covers_every_symbol():
    assert set(declared_functions()) == set(sbp._SIGS)


@needs_lib
def test_size_queries():
    L = sbp.lib()
    assert L.sbp_blockmodel_bytes(1000, 8000, 10) > 4 * 100
    dense = L.sbp_blockmodel_bytes(1000, 8000, 64)
    # the dense tier carries f(x) = x ln x for every count up to e and a block byte per edge end
    assert dense >= 8 * (8000 + 1) + 2 * 8000
    # the sparse tier stores rows, columns and proposal tables sized by the edges
    assert L.sbp_blockmodel_bytes(1000, 80000, 65) > L.sbp_blockmodel_bytes(1000, 8000, 65) + 8 * 72000
    assert L.sbp_blockmodel_bytes(0, 10, 1) == 0
    assert L.sbp_engine_workspace_bytes(1000, 8000, 4) > L.sbp_engine_graph_bytes(1000, 8000)
    n = (ct.c_int32 * 2)(100, 200)
    e = (ct.c_int32 * 2)(800, 1600)
    assert L.sbp_partition_workspace_bytes(2, n, e) >= L.sbp_engine_workspace_bytes(300, 2400, 2)


@needs_lib
def test_argument_errors_before_device_work():
    L = sbp.lib()
    fake = ct.c_void_p(0x1000)
    g = sbp.Graph(0, 10, fake.value, fake.value, fake.value, fake.value)
    assert L.sbp_build_blockmodel(ct.byref(g), fake, 1, fake, 1 << 20, fake, 1 << 20, None) == -1
    g = sbp.Graph(100, 10, fake.value, fake.value, fake.value, fake.value)
    # C > n
    assert L.sbp_build_blockmodel(ct.byref(g), fake, 101, fake, 1 << 20, fake, 1 << 20, None) == -1
    # blockmodel storage too small
    assert L.sbp_build_blockmodel(ct.byref(g), fake, 10, fake, 16, fake, 1 << 20, None) == -4
    assert b"too small" in L.sbp_last_error()
    # sizes beyond the limits
    g = sbp.Graph(1 << 30, 10, fake.value, fake.value, fake.value, fake.value)
    assert L.sbp_build_blockmodel(ct.byref(g), fake, 10, fake, 1 << 20, fake, 1 << 20, None) == -6
    # engine: workspace too small, capacity too large
    h = ct.c_void_p()
    assert L.sbp_engine_create(fake, 16, 1000, 1000, 2, None, ct.byref(h)) == -4
    assert L.sbp_engine_create(fake, 1 << 40, 1 << 31, 1000, 2, None, ct.byref(h)) == -6
    # sweep parameters
    g = sbp.Graph(100, 10, fake.value, fake.value, fake.value, fake.value)
    p = sbp.SweepParams(1, 0, 0, 3.0, 1, 0)  # n_batches = 0
    assert L.sbp_nodal_sweep(ct.byref(g), fake, 10, fake, 1 << 20, ct.byref(p), None, None, fake, 1 << 20,
                             None) == -1


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(sbp, "_lib", None)
    monkeypatch.setattr(sbp, "LIB_PATH", "/nonexistent/libsbp.so")
    with pytest.raises(RuntimeError, match="missing"):
        sbp.lib()


def test_autotune_bins_and_missing_cache(tmp_path):
    from paper_2305_18663_amd import autotune
    assert autotune.size_bin(200_000, 4_000_000, 45) == "n17_k22_c2_b1"
    assert autotune.size_bin(1000, 8000, 10, 3) == "n9_k13_c1_b3"
    assert autotune.size_bin(1, 0, 1) == "n0_k0_c0_b1"
    # no cache: the defaults are set and returned
    assert autotune.apply(str(tmp_path / "none.json"), 1000, 8000, 10) == autotune.DEFAULTS

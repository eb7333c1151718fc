"""The C-ABI library loads and exports every symbol include/dlmcol.h
declares; argument checks that fail before any device work behave as the
header states.  No compute call is made here (no GPU in this container)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dlmcol.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dlm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2109_05948_amd import _abi
    return _abi.lib()


def test_exports_every_declared_symbol(L):
    syms = declared_symbols()
    assert "dlm_tabu_batch" in syms and len(syms) >= 8
    for s in syms:
        assert hasattr(L, s), s
    from paper_2109_05948_amd import _abi
    assert set(_abi.EXPORTS) <= set(syms)


def test_version_and_error(L):
    assert L.dlm_abi_version() == 2
    assert isinstance(L.dlm_last_error(), bytes)


@pytest.mark.parametrize("case", ["asym", "loop", "unsorted", "range", "n0", "weight0"])
def test_graph_validation_rejects(L, case):
    from paper_2109_05948_amd import _abi
    n = 4
    rp = np.array([0, 1, 2, 3, 4], np.int32)
    ci = np.array([1, 0, 3, 2], np.int32)
    w = None
    if case == "asym":
        rp = np.array([0, 1, 1, 1, 1], np.int32)
        ci = np.array([1], np.int32)
    elif case == "loop":
        ci = np.array([0, 0, 3, 2], np.int32)
    elif case == "unsorted":
        rp = np.array([0, 2, 3, 4, 4], np.int32)
        ci = np.array([2, 1, 0, 0], np.int32)
    elif case == "range":
        ci = np.array([1, 0, 3, 7], np.int32)
    elif case == "n0":
        n = 0
    elif case == "weight0":
        w = np.array([1, 0, 2, 3], np.int32)
    with pytest.raises(_abi.DlmError) as e:
        _abi.Graph(n, rp, ci, w)
    assert e.value.code == -1
    assert len(L.dlm_last_error()) > 0


def test_graph_flags(L):
    """DLM_G_BITSET is declared but not built; unknown flag bits are invalid.
    Both are rejected before any device work."""
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([1, 0], np.int32)
    h = C.c_void_p()
    P = C.c_void_p
    assert L.dlm_graph_create(2, rp.ctypes.data_as(P), ci.ctypes.data_as(P), None, 0x1, None, C.byref(h)) == -4
    assert b"bitset" in L.dlm_last_error()
    assert L.dlm_graph_create(2, rp.ctypes.data_as(P), ci.ctypes.data_as(P), None, 0x6, None, C.byref(h)) == -1
    assert h.value is None


def test_null_arguments(L):
    from paper_2109_05948_amd import _abi
    prm = _abi.TabuParams(18, 10, 6, 10, 10, 0, 1, 0, 0, 0, 0)
    assert L.dlm_tabu_batch(None, C.byref(prm), 1, None, None, None, None, None, None, None, 0, None) == -1
    sz = C.c_size_t(7)
    assert L.dlm_tabu_workspace_bytes(None, C.byref(prm), 1, C.byref(sz)) == -1
    assert sz.value == 0  # cleared on failure
    assert L.dlm_tabu_workspace_bytes(None, C.byref(prm), 1, None) == -1
    assert L.dlm_graph_info(None, None, None, None) == -1
    assert L.dlm_evaluate(None, 2, None, 1, None, None, None) == -1
    assert L.dlm_init_population(None, 2, 1, 0, 0, 0, None, None, None) == -1


def test_diversity_argument_checks(L):
    """Bad sizes and null buffers are rejected before any device work."""
    fake = C.c_void_p(16)  # never dereferenced: every call below fails its checks first
    # k outside [1, 256], n outside [1, 32767]
    assert L.dlm_partition_distance(10, 0, fake, 1, fake, 1, 0, fake, 1, fake, None) == -1
    assert L.dlm_partition_distance(10, 257, fake, 1, fake, 1, 0, fake, 1, fake, None) == -1
    assert L.dlm_partition_distance(0, 3, fake, 1, fake, 1, 0, fake, 1, fake, None) == -1
    # the triangle form needs the same rows on both sides; ld below the row length
    assert L.dlm_partition_distance(10, 3, fake, 2, C.c_void_p(32), 2, 1, fake, 2, fake, None) == -1
    assert L.dlm_partition_distance(10, 3, fake, 2, fake, 3, 0, fake, 2, fake, None) == -1
    assert L.dlm_partition_distance(10, 3, None, 2, fake, 2, 0, fake, 2, fake, None) == -1
    # keep above the pool, ld below the pool, pool above 65536
    assert L.dlm_spacing_update(fake, 2, fake, 2, fake, 4, 5, 0, fake, fake, fake, None) == -1
    assert L.dlm_spacing_update(fake, 2, fake, 2, fake, 3, 2, 0, fake, fake, fake, None) == -1
    assert L.dlm_spacing_update(fake, 40000, fake, 40000, fake, 80000, 2, 0, fake, fake, fake, None) == -1
    assert L.dlm_spacing_update(fake, 2, fake, 2, fake, 4, 2, 0, None, fake, fake, None) == -1
    # K must stay below p
    assert L.dlm_nearest(fake, 4, 4, 4, fake, None) == -1
    assert L.dlm_nearest(fake, 3, 4, 2, fake, None) == -1
    assert L.dlm_gather_pool(fake, fake, -1, fake, fake, 1, 5, fake, 1, fake, fake, None) == -1
    assert L.dlm_gather_distances(fake, 4, fake, 5, fake, 4, None) == -1
    # empty requests are no-ops
    assert L.dlm_partition_distance(10, 3, None, 0, None, 0, 0, None, 0, None, None) == 0
    assert L.dlm_nearest(None, 1, 0, 0, None, None) == 0


def test_invnet_argument_checks(L):
    """The colour-invariant network rejects bad shapes before any device work."""
    from paper_2109_05948_amd import _abi
    w = np.array([8, 4, 1], np.int32)
    flat = np.zeros(1, np.float32)
    h = C.c_void_p()
    # k below 2, n of 0, a last width other than 1, a zero width, no widths
    assert L.dlm_invnet_create(10, 1, 3, _abi._ptr(w), _abi._ptr(flat), 4, C.byref(h)) == -1
    assert L.dlm_invnet_create(0, 3, 3, _abi._ptr(w), _abi._ptr(flat), 4, C.byref(h)) == -1
    assert L.dlm_invnet_create(10, 3, 2, _abi._ptr(w), _abi._ptr(flat), 4, C.byref(h)) == -1
    bad = np.array([8, 0, 1], np.int32)
    assert L.dlm_invnet_create(10, 3, 3, _abi._ptr(bad), _abi._ptr(flat), 4, C.byref(h)) == -1
    assert L.dlm_invnet_create(10, 3, 3, None, _abi._ptr(flat), 4, C.byref(h)) == -1
    assert L.dlm_invnet_create(10, 3, 3, _abi._ptr(w), _abi._ptr(flat), 0, C.byref(h)) == -1
    assert h.value is None
    # calls on no network
    assert L.dlm_invnet_forward(None, None, 1, None, None) == -1
    assert L.dlm_invnet_grad(None, None, None, 1, None, None, None) == -1
    assert L.dlm_invnet_train(None, None, None, 1, 1, 1, C.c_float(1e-3), None, None) == -1
    assert L.dlm_invnet_get_params(None, None, None) == -1
    assert L.dlm_invnet_destroy(None) == 0


def test_gemm_argument_checks(L):
    """dlm_gemm_bf16 refuses bad shapes, pitches, tiles, splits and null
    operands before touching the device; an empty output is a no-op."""
    a = C.c_void_p(16)
    c = C.c_void_p(16)
    g = L.dlm_gemm_bf16
    assert g(1, a, 8, 0, a, 8, c, 8, -1, 8, 8, 0, 0, None, 0, None) == -1  # negative M
    assert g(1, a, 8, 0, a, 8, c, 4, 8, 8, 8, 0, 0, None, 0, None) == -1  # ldc < N
    assert g(1, a, 8, 0, a, 8, c, 8, 8, 8, 8, 96, 0, None, 0, None) == -1  # tile not 0/64/128/256
    assert g(1, None, 8, 0, a, 8, c, 8, 8, 8, 8, 0, 0, None, 0, None) == -1  # null A
    assert g(1, a, 4, 0, a, 8, c, 8, 8, 8, 8, 0, 0, None, 0, None) == -1  # K-contiguous pitch < K
    assert g(0, a, 4, 0, a, 8, c, 8, 8, 8, 8, 0, 0, None, 0, None) == -1  # M-contiguous pitch < M
    assert g(1, a, 8, 0, a, 8, c, 8, 8, 8, 8, 0, 4, None, 0, None) == -1  # forced split, no workspace
    assert g(1, a, 8, 0, a, 8, c, 8, 8, 8, 8, 0, 4, a, 100, None) == -1  # forced split, workspace too small
    assert g(1, a, 8, 0, a, 8, c, 8, 8, 8, 8, 0, 65, a, 1 << 20, None) == -1  # more than 64 splits
    assert g(1, a, 1 << 23, 0, a, 8, c, 8, 8, 8, 8, 0, 0, None, 0, None) == -1  # pitch above 2^22
    assert g(1, None, 8, 0, None, 8, None, 8, 0, 8, 8, 0, 0, None, 0, None) == 0  # M = 0: nothing to do

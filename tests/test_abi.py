"""The C ABI loads and exports what include/knn.h declares; host-only helpers and
argument checks (no GPU needed: every call here returns before touching a device)."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def K():
    from paper_2206_14286_amd import knn
    return knn


def declared_functions():
    src = open(os.path.join(ROOT, "include", "knn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(knn_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported(K):
    lib = K.lib()
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/knn.h but not exported"


def test_helpers_match_oracle(K):
    for k in (1, 2, 5, 10, 64, 100):
        for r in (0.5, 0.9, 0.95, 0.99):
            assert K.bins_for_recall(k, r) == oracle.bins_for_recall(k, r)
            L = oracle.bins_for_recall(k, r)
            assert abs(K.expected_recall_bound(k, L) - oracle.recall_bound_paper(k, L)) < 1e-12
    assert K.bins_for_recall(10, 0.95, 100) == 100
    for N in (1, 7, 100, 65536, 1000000):
        for L in (1, 3, 176, 2048):
            if L > N:
                continue
            for b in (0, 1, L // 2, L - 1, L):
                assert K.bin_start(b, N, L) == oracle.bin_start(b, N, L)
    assert K.lib().knn_bins_for_recall(0, 0.95, 10) == -1
    assert K.lib().knn_bins_for_recall(10, 1.5, 10) == -1
    assert K.lib().knn_bin_start(-1, 10, 5) == -1


def test_approx_bins_match_oracle(K):
    for n in (1, 10, 176, 1000, 65536, 1 << 20):
        for k in (1, 10, 64):
            if k > n:
                assert K.lib().knn_approx_bins(n, k, 0.95, -1) == -1
                continue
            for over in (-1, n, 4 * n, 3 * n + 1):
                assert K.approx_bins(n, k, 0.95, over) == oracle.approx_bins(n, k, 0.95, over)


def test_approx_top_k_argument_checks(K):
    lib = K.lib()
    fake = _p(0x1000)
    args = dict(dt=0, rows=4, cols=100, ld=100, dim=1, k=5, r=0.95, over=-1, L=10, mn=0, agg=1)
    big = ctypes.c_size_t(1 << 40)

    def call(ws=fake, nws=big.value, **kw):
        a = {**args, **kw}
        return lib.knn_approx_top_k(fake, a["dt"], a["rows"], a["cols"], a["ld"], a["dim"], a["k"], a["r"],
                                    a["over"], a["L"], a["mn"], a["agg"], fake, fake, ws, nws, None)
    assert call(dt=2) == 1
    assert call(ld=99) == 1
    assert call(dim=2) == 1
    assert call(L=4) == 1 and b"K <= L" in lib.knn_last_error()
    assert call(L=101) == 1
    assert call(k=101) == 1
    assert call(k=2000, cols=5000, ld=5000, L=3000) == 1
    assert call(k=1025, cols=5000, ld=5000, L=3000) == 1 and b"1024" in lib.knn_last_error()
    assert call(k=1024, cols=5000, ld=5000, L=3000, rows=0) == 0  # the largest K passes the checks
    assert call(L=0, r=1.5) == 1
    assert call(dim=0, k=5, L=10) == 1  # the reduced dimension has 4 entries
    # no slices: succeeds without touching the device
    assert call(rows=0) == 0
    assert call(dim=0, rows=100, cols=0) == 0
    # the workspace: the query reports B * L bins when aggregating and nothing otherwise;
    # one byte short is refused before anything is enqueued
    n = ctypes.c_size_t()
    assert lib.knn_approx_workspace_size(0, 4, 100, 100, 1, 5, 0.95, -1, 10, 0, 1, ctypes.byref(n)) == 0
    assert n.value >= 4 * 10 * 8
    assert call(nws=n.value - 1) == 1 and b"workspace too small" in lib.knn_last_error()
    assert call(ws=None, nws=n.value) == 1
    assert lib.knn_approx_workspace_size(0, 4, 100, 100, 1, 5, 0.95, -1, 10, 0, 0, ctypes.byref(n)) == 0
    assert n.value == 0


def test_status_strings(K):
    lib = K.lib()
    assert lib.knn_status_string(0) == b"ok"
    assert lib.knn_status_string(1) == b"invalid argument"
    assert lib.knn_status_string(4) == b"HIP error"
    assert lib.knn_status_string(99) == b"unknown status"


def _p(v):
    return ctypes.c_void_p(v)


def test_invalid_arguments_return_before_any_device_work(K):
    lib = K.lib()
    fake = _p(0x1000)
    out = ctypes.c_void_p()
    # K > L
    assert lib.knn_search(fake, 4, fake, 100, 16, 11, 10, 0, fake, fake, None) == 1
    assert b"K <= L" in lib.knn_last_error()
    # L > N
    assert lib.knn_search(fake, 4, fake, 100, 16, 5, 101, 0, fake, fake, None) == 1
    # D too large: unsupported
    assert lib.knn_search(fake, 4, fake, 100, 300, 5, 10, 0, fake, fake, None) == 2
    # bad metric
    assert lib.knn_search(fake, 4, fake, 100, 16, 5, 10, 7, fake, fake, None) == 1
    # NULL pointers
    assert lib.knn_search(None, 4, fake, 100, 16, 5, 10, 0, fake, fake, None) == 1
    # database preparation: NULL X, bad dtype, N = 0, no buffer, a buffer one byte short
    need = lib.knn_db_prepare_size(100, 16, 0, 0)
    assert need > 0 and lib.knn_db_prepare_size(0, 16, 0, 0) == 0
    assert lib.knn_db_prepare(None, 0, 100, 16, 0, 0, fake, need, None, ctypes.byref(out)) == 1
    assert lib.knn_db_prepare(fake, 2, 100, 16, 0, 0, fake, need, None, ctypes.byref(out)) == 1
    assert lib.knn_db_prepare(fake, 0, 0, 16, 0, 0, fake, need, None, ctypes.byref(out)) == 1
    assert lib.knn_db_prepare(fake, 0, 100, 16, 0, 0, None, need, None, ctypes.byref(out)) == 1
    assert lib.knn_db_prepare(fake, 0, 100, 16, 0, 0, fake, need - 1, None, ctypes.byref(out)) == 1
    assert b"buf too small" in lib.knn_last_error()
    assert out.value is None
    assert lib.knn_db_search(None, fake, 0, 4, 5, 10, 0.95, -1, 0, fake, fake, None, None, fake, 1 << 30, None) == 1
    assert lib.knn_backward(fake, fake, fake, fake, 0, 4, 100, 300, 5, 0, fake, fake, None) == 2
    assert lib.knn_backward(fake, fake, fake, fake, 0, 4, 0, 16, 5, 0, fake, fake, None) == 1
    assert lib.knn_search_batched(None, None) == 1
    assert lib.knn_plan_create(None, 0, None, 0, 0, 0.95, 0, None, ctypes.byref(out)) == 1
    assert lib.knn_plan_setup(None, fake, 1 << 30, None) == 1
    assert lib.knn_db_destroy(None) == 0 and lib.knn_plan_destroy(None) == 0
    # M = 0 is a no-op that succeeds without touching the device
    assert lib.knn_search(None, 0, fake, 100, 16, 5, 10, 0, None, None, None) == 0


def test_search_size_queries_check_their_handle(K):
    """The workspace query and the search refuse a NULL database handle (the workspace
    size checks of a prepared database need a device: tests/test_gpu_search.py)."""
    lib = K.lib()
    fake = _p(0x1000)
    n = ctypes.c_size_t()
    assert lib.knn_db_search_workspace_size(None, 10, 5, 10, 0.95, -1, 0, 0, ctypes.byref(n)) == 1
    assert lib.knn_db_search(None, fake, 0, 10, 5, 10, 0.95, -1, 0, fake, fake, None, None, fake, 0, None) == 1


def test_plan_create_is_host_only_and_checks_arguments(K):
    lib = K.lib()
    out = ctypes.c_void_p()
    arr = (K.KnnBatch * 1)()
    hs = (ctypes.c_void_p * 1)(None)
    assert lib.knn_plan_create(hs, 1, arr, 1, 1, 0.95, 0, None, ctypes.byref(out)) == 1  # NULL database
    assert b"database 0 is NULL" in lib.knn_last_error()
    assert lib.knn_plan_workspace_size(None, ctypes.byref(ctypes.c_size_t())) == 1
    assert lib.knn_plan_set_own_launches(None, 2048) == 1

"""The C ABI library loads and exports every entry point include/kpm.h declares; host-only logic.

No test here launches a kernel: every call below either is pure host arithmetic or is rejected
by argument validation before any HIP call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1105_5481_amd as kpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "kpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kpm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1105_5481_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return kpm.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for st in range(7):
        assert L.kpm_status_string(st).decode()
    assert L.kpm_status_string(99).decode() == "unknown status"


def test_scale_from_bounds(L):
    a, b = kpm.scale_from_bounds(-6.0, 6.0, 0.01)
    assert a == 12.0 / 1.99 and b == 0.0
    a, b = kpm.scale_from_bounds(-1.0, 3.0, 0.0)
    assert (a, b) == (2.0, 1.0)
    for bad in [(1.0, 1.0, 0.01), (2.0, 1.0, 0.0), (-1.0, 1.0, 1.0), (-1.0, 1.0, -0.1), (float("nan"), 1.0, 0.0)]:
        with pytest.raises(kpm.KPMError):
            kpm.scale_from_bounds(*bad)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 8, 9, 10, 16, 31, 48, 63, 64, 96, 100, 1000, 4096, 65537,
                               2**20 + 3, 2**31 - 1, 2**31, 2**32 - 1])
def test_fast_division(L, d):
    g = np.random.default_rng(d)
    n = np.concatenate([np.arange(0, 2000, dtype=np.uint32), g.integers(0, 2**32, 20000, dtype=np.uint64).astype(np.uint32),
                        np.array([2**32 - 1, 2**32 - 2, 2**31, 2**31 - 1, d, d - 1, d + 1, 2 * d - 1], dtype=np.uint64).astype(np.uint32)])
    n = np.ascontiguousarray(n)
    r = L.kpm_selftest_fastdiv(ctypes.c_uint32(d), n.ctypes.data_as(ctypes.c_void_p), len(n))
    assert r == 0, (d, int(n[r - 1]) if r > 0 else None)


def test_argument_validation_without_device(L):
    # NULL descriptor / handle and out-of-range sizes are rejected before any HIP call
    h = ctypes.c_void_p()
    assert L.kpm_build(None, 1.0, 0.0, 0, None, ctypes.byref(h)) == 1
    assert L.kpm_workspace_bytes(None, 16, 4, 0) == 0
    a, b = ctypes.c_double(), ctypes.c_double()
    assert L.kpm_ham_get_scale(None, ctypes.byref(a), ctypes.byref(b)) == 1
    assert L.kpm_moments(None, 16, 4, 0, 1, 0, None, 0, None, None) != 0
    assert L.kpm_dos(None, 16, 1, 64, 1.0, 0.0, None, None, None) == 1
    assert L.kpm_start_vectors(5, 0, 0, 0, 10, 2, None, None) == 1
    assert L.kpm_set_launch(0, 3) == 1          # elems per thread must be 1, 2 or 4
    assert L.kpm_set_launch(1, 12) == 1         # block cap must be a multiple of 8
    assert L.kpm_set_launch(2, 5) == 1
    assert L.kpm_set_launch(3, 0) == 1
    assert L.kpm_set_launch(4, 4) == 1
    assert L.kpm_set_launch(5, 2) == 1
    assert L.kpm_set_launch(9, 2) == 1          # depth keys: 0 one step, 1 two, 3..6, -1 default; 2 is none
    assert L.kpm_set_launch(9, 7) == 1
    assert L.kpm_set_launch(10, 2) == 1         # 3D two-step passes: -1, 0 or 1
    assert L.kpm_set_launch(99, 1) == 1
    d = kpm.HamDesc()
    d.kind = 3
    d.L[0], d.L[1], d.L[2] = 4, 0, 4             # zero extent
    assert L.kpm_build(ctypes.byref(d), 1.0, 0.0, 0, None, ctypes.byref(h)) == 1
    d.L[1] = 4
    assert L.kpm_build(ctypes.byref(d), -1.0, 0.0, 0, None, ctypes.byref(h)) == 1   # a <= 0
    assert L.kpm_build(ctypes.byref(d), 1.0, 0.0, 7, None, ctypes.byref(h)) == 1    # bad precision
    d.hop = 1                                     # spin hopping without spinors
    assert L.kpm_build(ctypes.byref(d), 1.0, 0.0, 0, None, ctypes.byref(h)) == 1
    d.kind = 7
    assert L.kpm_bounds_gershgorin(ctypes.byref(d), None, None) == 1


def test_lanczos_argument_validation(L):
    assert L.kpm_lanczos_workspace_bytes(None, 10) == 0
    inf = float("inf")
    assert L.kpm_bounds_lanczos(None, 10, 0, 0.005, -inf, inf, None, 0, None, None) == 1


def test_launch_settings_roundtrip(L):
    old = kpm.get_launch()
    with kpm.launch_settings(elems_per_thread=2, max_blocks=1024, march=0, march_items=64, xcd_split=3, alternate=0,
                             small=0, streaming=0, wave_mib=0, tblock=0, tb3=1, tb_group=0):
        assert kpm.get_launch() == {"elems_per_thread": 2, "max_blocks": 1024, "march": 0, "march_items": 64,
                                    "xcd_split": 3, "alternate": 0, "small": 0, "streaming": 0, "wave_mib": 0,
                                    "tblock": 0, "tb3": 1, "tb_group": 0}
    assert kpm.get_launch() == old


def test_no_cpu_fallback_when_library_missing(monkeypatch):
    """The product path raises instead of computing anything without the HIP library."""
    monkeypatch.setattr(kpm, "_lib", None)
    monkeypatch.setattr(kpm, "_LIB_PATH", "/nonexistent/libkpm.so")
    with pytest.raises(kpm.KPMError):
        kpm.lib()


@pytest.mark.parametrize("wave", [0, 1])
@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("case", range(6))
def test_block_placement(L, case, split, wave):
    """Multi-instance launches: every block of the grid maps to one block of one instance or is idle;
    instances split per XCD start on a multiple of 8; with at least 8 candidates for whole placement
    (instances without a split of their own; in a static batch wave, every march instance) each of
    them has all its blocks on one XCD (block b runs on XCD b mod 8) and the XCD loads are balanced
    (a candidate that would overload an XCD by more than 10%, 25% in a wave, is split when it has
    >= 48 units)."""
    g = np.random.default_rng(case)
    n = [1, 3, 8, 9, 17, 256][case]
    nb = (g.integers(1, 40, n) * 8).astype(np.uint32)
    xcd = (g.random(n) < 0.3).astype(np.int32)
    if case == 0:
        xcd[:] = 0
    xcd_in = xcd.copy()
    units = (nb * 8).astype(np.uint32) if split else None
    b0 = np.zeros(n, np.uint32)
    bs = np.zeros(n, np.uint32)
    cap = int(nb.sum()) * 2 + 8 * int(nb.max())
    m = np.zeros(cap, np.uint32)
    P = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    blocks = L.kpm_selftest_placement(P(nb), P(xcd), P(units), n, wave, P(b0), P(bs), P(m), cap)
    assert blocks > 0
    m = m[:blocks]
    seen = [set() for _ in range(n)]
    for blk, i in enumerate(m):
        if i == 0xFFFFFFFF:
            continue
        assert i < n
        off = blk - int(b0[i])
        assert off >= 0 and off % bs[i] == 0
        j = off // bs[i]
        assert j < nb[i] and j not in seen[i]
        seen[i].add(j)
    cand = np.ones(n, bool) if (wave and n >= 8) else (xcd_in == 0)
    packed = int(cand.sum()) >= 8
    if not packed:
        cand[:] = False
    assert np.array_equal(xcd[~cand], xcd_in[~cand])     # the others keep their own split
    if not split:
        assert np.all(xcd[cand] == 0)
    load = np.zeros(8)
    for i in range(n):
        assert len(seen[i]) == nb[i]
        if xcd[i] or not packed:
            assert bs[i] == 1 and b0[i] % 8 == 0
            if cand[i]:
                load += nb[i] / 8.0
        else:
            assert bs[i] == 8
            load[int(b0[i]) % 8] += nb[i]
    if packed:
        whole = nb[cand]
        slack = 1.25 if wave else 1.10
        if split:    # within the slack of an even share, plus one share of a split instance
            assert load.max() <= slack * whole.sum() / 8.0 + 1e-9 + whole.max() / 8.0
        else:        # greedy balance: XCD loads differ by at most one instance
            assert load.max() - load.min() <= whole.max()
    idle = int((m == 0xFFFFFFFF).sum())
    assert idle <= 8 * int(nb.max()) + blocks // 4


def test_null_handles_and_bad_sizes_are_rejected(L):
    """Every entry point checks its handle and size arguments on the host: NULL handles, empty or
    negative sizes and unknown enum values give KPM_ERR_INVALID_ARG (or a zero size / -1 query)
    without touching the device; the free functions accept NULL."""
    INVALID = 1
    out = ctypes.c_void_p()
    rem = ctypes.c_int32()
    inf = float("inf")
    dummy = ctypes.c_void_p(16)        # never dereferenced: the size checks come first
    # handles
    assert L.kpm_solve_begin(None, 16, 4, 0, 1, 0, None, 0, ctypes.byref(out), None) == INVALID
    assert L.kpm_solve_advance(None, 1, None, ctypes.byref(rem)) == INVALID
    assert L.kpm_solve_finish(None, dummy, None) == INVALID
    assert L.kpm_solve_remaining(None, ctypes.byref(rem)) == INVALID
    assert L.kpm_solve_mode(None) == -1
    assert L.kpm_update(None, None, 1.0, 0.0, None) == INVALID
    assert L.kpm_ham_dim(None) == -1
    assert L.kpm_ham_bytes(None) == 0
    assert L.kpm_request_bytes(None, 0, 16, 4, 0) == 0
    assert L.kpm_workspace_bytes_batched(None, 0, None, None, 0) == 0
    assert L.kpm_moments_batched(None, 0, None, None, 0, None, None, None, 0, None, None) == INVALID
    assert L.kpm_batch_add(None, None) == INVALID
    assert L.kpm_batch_remove(None, None) == INVALID
    assert L.kpm_batch_size(None) == -1
    assert L.kpm_batch_advance(None, 1, None) == INVALID
    assert L.kpm_batch_create(0, ctypes.byref(out)) == INVALID
    assert L.kpm_batch_create(-3, ctypes.byref(out)) == INVALID
    assert L.kpm_graph_capture_batched(None, 0, None, None, 0, None, None, None, 0, None, None,
                                       ctypes.byref(out)) == INVALID
    assert L.kpm_graph_launch(None, None) == INVALID
    for free in (L.kpm_free, L.kpm_solve_free, L.kpm_batch_free, L.kpm_graph_free):
        free(None)
    # sizes and enums of the device-array entry points
    assert L.kpm_dos(dummy, 0, 1, 64, 1.0, 0.0, dummy, dummy, None) == INVALID      # M = 0
    assert L.kpm_dos(dummy, 16, 1, 0, 1.0, 0.0, dummy, dummy, None) == INVALID      # K = 0
    assert L.kpm_dos(dummy, 16, 1, 64, 0.0, 0.0, dummy, dummy, None) == INVALID     # a = 0
    assert L.kpm_green(None, 16, 0, 0.0, 64, 1.0, 0.0, dummy, dummy, dummy, None) == INVALID
    assert L.kpm_green(dummy, 0, 0, 0.0, 64, 1.0, 0.0, dummy, dummy, dummy, None) == INVALID
    assert L.kpm_green(dummy, 16, 0, 0.0, 0, 1.0, 0.0, dummy, dummy, dummy, None) == INVALID
    assert L.kpm_green(dummy, 16, 7, 0.0, 64, 1.0, 0.0, dummy, dummy, dummy, None) == INVALID   # kernel
    assert L.kpm_green(dummy, 16, 2, 0.0, 64, 1.0, 0.0, dummy, dummy, dummy, None) == INVALID   # lambda
    assert L.kpm_green(dummy, 16, 2, 800.0, 64, 1.0, 0.0, dummy, dummy, dummy, None) == INVALID
    assert L.kpm_green(dummy, 16, 0, 0.0, 64, -1.0, 0.0, dummy, dummy, dummy, None) == INVALID
    assert L.kpm_dense_workspace_bytes(0, 16, 4) == 0
    assert L.kpm_dense_workspace_bytes(64, 0, 4) == 0
    assert L.kpm_dense_workspace_bytes(64, 16, 0) == 0
    assert L.kpm_dense_moments(None, 64, 1.0, 0.0, 16, 4, 0, 1, 0, dummy, 1 << 20, dummy, None) == INVALID
    assert L.kpm_dense_moments(dummy, 0, 1.0, 0.0, 16, 4, 0, 1, 0, dummy, 1 << 20, dummy, None) == INVALID
    assert L.kpm_dense_moments(dummy, 64, 0.0, 0.0, 16, 4, 0, 1, 0, dummy, 1 << 20, dummy, None) == INVALID
    assert L.kpm_dense_moments(dummy, 64, 1.0, 0.0, 16, 4, 0, 1, 0, dummy, 0, dummy, None) == 6   # workspace
    assert L.kpm_start_vectors(0, 0, 0, 0, 0, 2, dummy, None) == INVALID             # N = 0
    assert L.kpm_start_vectors(0, 0, 0, 0, 10, 0, dummy, None) == INVALID            # R = 0
    assert L.kpm_bounds_lanczos(None, 10, 0, 0.005, -inf, inf, dummy, 1 << 20, dummy, None) == INVALID
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert L.kpm_scale_from_bounds(1.0, -1.0, 0.01, ctypes.byref(lo), ctypes.byref(hi)) == INVALID
    assert L.kpm_scale_from_bounds(-1.0, 1.0, 2.0, ctypes.byref(lo), ctypes.byref(hi)) == INVALID
    assert L.kpm_scale_from_bounds(-1.0, 1.0, 0.01, None, None) == INVALID
    assert L.kpm_get_launch(0, None) == INVALID

"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/wsm.h declares, answers size queries, and rejects
invalid arguments before enqueuing anything."""

from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wsm.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(wsm_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def wsm():
    import paper_1011_0093_amd as w
    return w


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("wsm_reduce_colors", "wsm_init", "wsm_iterate", "wsm_map_pixels",
              "wsm_reduce_workspace_bytes", "wsm_state_bytes", "wsm_status_string",
              "wsm_state_views", "wsm_init_pixels", "wsm_iterate_full"):
        assert n in names


def test_library_exports_every_declared_symbol(wsm):
    lib = ctypes.CDLL(wsm.library_path())
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings(wsm):
    lib = wsm._lib
    assert lib.wsm_status_string(0) == b"ok"
    assert lib.wsm_status_string(-1) == b"invalid argument"
    assert lib.wsm_status_string(-2).startswith(b"workspace")
    assert lib.wsm_status_string(12345) == b"unknown status"


def test_size_queries(wsm):
    a = wsm.reduce_workspace_bytes(4096 * 4096)
    assert a == wsm.reduce_workspace_bytes(4096 * 4096)
    # 2 bytes per pixel of grouped keys plus the per-(slice, tile) table
    assert 2 * 4096 * 4096 <= a < 2 * 4096 * 4096 + (8 << 20)
    assert wsm.reduce_workspace_bytes(1) > 0
    with pytest.raises(wsm.WsmError):
        wsm.reduce_workspace_bytes(0)
    with pytest.raises(wsm.WsmError):
        wsm.reduce_workspace_bytes(1 << 33)
    s1 = wsm.state_bytes(1, 1)
    s2 = wsm.state_bytes(1000, 256)
    assert s2 - s1 == 1024 - 256 and s1 % 256 == 0
    for bad in ((0, 4), (10, 0), (10, 257)):
        with pytest.raises(wsm.WsmError):
            wsm.state_bytes(*bad)


def test_argument_validation_before_any_launch(wsm):
    lib = wsm._lib
    P = ctypes.c_void_p
    fake = P(0x10000)  # never dereferenced: validation fails first
    nu = P(0x20000)
    # null pointers
    assert lib.wsm_reduce_colors(None, 10, fake, fake, 10, nu, fake, 1 << 20, None) == -1
    # n_pixels < 1
    assert lib.wsm_reduce_colors(fake, 0, fake, fake, 10, nu, fake, 1 << 20, None) == -1
    # capacity too small / workspace too small / misaligned workspace
    assert lib.wsm_reduce_colors(fake, 100, fake, fake, 99, nu, fake, 1 << 20, None) == -2
    assert lib.wsm_reduce_colors(fake, 100, fake, fake, 100, nu, fake, 16, None) == -2
    assert lib.wsm_reduce_colors(fake, 100, fake, fake, 100, nu, P(0x10001), 1 << 20, None) == -1
    prob = wsm._Problem()
    # K out of range, K > n_unique, misaligned state, state too small, null palette
    assert lib.wsm_init(ctypes.byref(prob), fake, 1 << 30, fake, fake, 100, 1000, 0, fake, None) == -1
    assert lib.wsm_init(ctypes.byref(prob), fake, 1 << 30, fake, fake, 100, 1000, 257, fake, None) == -1
    assert lib.wsm_init(ctypes.byref(prob), fake, 1 << 30, fake, fake, 3, 1000, 4, fake, None) == -1
    assert lib.wsm_init(ctypes.byref(prob), P(0x10010), 1 << 30, fake, fake, 100, 1000, 4, fake, None) == -1
    assert lib.wsm_init(ctypes.byref(prob), fake, 1024, fake, fake, 100, 1000, 4, fake, None) == -2
    assert lib.wsm_init(ctypes.byref(prob), fake, 1 << 30, fake, fake, 100, 1000, 4, None, None) == -1
    assert lib.wsm_init(ctypes.byref(prob), fake, 1 << 30, fake, fake, 100, 50, 4, fake, None) == -1
    # an uninitialised descriptor is rejected by every later call
    assert lib.wsm_iterate(ctypes.byref(prob), 10, 1e-4, None) == -1
    assert lib.wsm_iterate_full(ctypes.byref(prob), 10, 1e-4, None) == -1
    v = wsm._Views()
    assert lib.wsm_state_views(ctypes.byref(prob), ctypes.byref(v)) == -1
    assert lib.wsm_map_pixels(ctypes.byref(prob), fake, 10, fake, fake, None, None, None) == -1
    assert lib.wsm_iterate(None, 10, 1e-4, None) == -1
    # graph handles: invalid problem or output pointer, no handle
    h = ctypes.c_void_p(0)
    assert lib.wsm_iterate_graph_create(ctypes.byref(prob), 10, 1e-4, 0, ctypes.byref(h)) == -1
    assert h.value is None
    assert lib.wsm_iterate_graph_create(None, 10, 1e-4, 0, ctypes.byref(h)) == -1
    assert lib.wsm_iterate_graph_create(ctypes.byref(prob), 10, 1e-4, 0, None) == -1
    assert lib.wsm_iterate_graph_launch(None, None) == -1
    assert lib.wsm_iterate_graph_destroy(None) == 0


def test_iterate_rejects_bad_counts_and_eps(wsm):
    lib = wsm._lib
    prob = wsm._Problem()
    # a descriptor that looks initialised (no device work is reached)
    prob.k = 4
    prob.points = 0
    prob.n_points = 100
    prob.n_pixels = 1000
    prob.state = 0x100000
    prob.state_bytes = wsm.state_bytes(100, 4)
    prob.colors = 0x200000
    prob.counts = 0x300000
    prob.magic = 0x574D5331
    prob.grid = 1
    for it, eps in ((0, 1e-4), (1025, 1e-4), (5, -1.0), (5, float("nan")), (5, float("inf"))):
        assert lib.wsm_iterate(ctypes.byref(prob), it, eps, None) == -1, (it, eps)
        assert lib.wsm_iterate_full(ctypes.byref(prob), it, eps, None) == -1, (it, eps)
    prob.state_bytes = 100
    assert lib.wsm_iterate(ctypes.byref(prob), 5, 1e-4, None) == -2
    prob.state_bytes = wsm.state_bytes(100, 4)
    prob.points = 1
    assert lib.wsm_map_pixels(ctypes.byref(prob), ctypes.c_void_p(0x1000), 1000, ctypes.c_void_p(0x1000),
                              ctypes.c_void_p(0x1000), None, None, None) == -1

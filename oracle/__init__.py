"""FP64 CPU oracle of the weighted sort-means (WSM) color quantizer.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It wraps ``wsm_oracle.c`` (plain
C, double precision, no fused multiply-add) with ctypes; nothing here is
shared with the GPU library.

The C source follows Alg. 1 and Alg. 2 of the paper step by step; its header
comment lists the readings used where the paper is silent.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wsm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (double precision, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


class use_library:
    """Context manager that routes every call to another build of the oracle
    (the pin tests use it to check that planted mistakes are caught)."""

    def __init__(self, path: str):
        self._path = path
        self._saved = None

    def __enter__(self):
        global _lib
        self._saved = _lib
        _lib = _bind(ctypes.CDLL(self._path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def _bind(lib):
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int
    dbl = ctypes.c_double
    lib.oracle_reduce.argtypes = [P, i64, P, P]
    lib.oracle_reduce.restype = i64
    lib.oracle_center_tables.argtypes = [P, i32, P, P]
    lib.oracle_center_tables.restype = None
    lib.oracle_search_step.argtypes = [P, i64, P, i32, P, P, P, P, i32, i32]
    lib.oracle_search_step.restype = i64
    lib.oracle_update_step.argtypes = [P, P, i64, i64, P, i32, P]
    lib.oracle_update_step.restype = None
    lib.oracle_weighted_sse.argtypes = [P, i64, i64, P]
    lib.oracle_weighted_sse.restype = dbl
    lib.oracle_wsm.argtypes = [P, P, i64, i64, i32, P, i32, dbl, i32, i32,
                               P, P, P, P, P, P]
    lib.oracle_wsm.restype = i32
    lib.oracle_kmeans_pixels.argtypes = [P, i64, i32, P, i32, dbl, P, P, P, P, P]
    lib.oracle_kmeans_pixels.restype = i32
    lib.oracle_assign_colors.argtypes = [P, P, i64, i64, P, P, i32, P]
    lib.oracle_assign_colors.restype = dbl
    lib.oracle_map.argtypes = [P, i64, P, i64, P, P, i32, P, P]
    lib.oracle_map.restype = i32
    lib.oracle_distortion.argtypes = [P, i64, P, P, i32]
    lib.oracle_distortion.restype = dbl
    lib.oracle_distortion_grad.argtypes = [P, i64, P, P, i32, dbl, P, P]
    lib.oracle_distortion_grad.restype = None
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
def reduce_colors(rgb: np.ndarray):
    """Unique colors (ascending 0x00RRGGBB, uint32) and their pixel counts."""
    lib = _load()
    rgb = _c(rgb, np.uint8).reshape(-1, 3)
    n = rgb.shape[0]
    cap = max(1, min(n, 1 << 24))
    colors = np.empty(cap, dtype=np.uint32)
    counts = np.empty(cap, dtype=np.uint32)
    nu = lib.oracle_reduce(_ptr(rgb), n, _ptr(colors), _ptr(counts))
    if nu < 0:
        raise ValueError("oracle_reduce failed")
    return colors[:nu].copy(), counts[:nu].copy()


def center_tables(centers: np.ndarray):
    """(d[K,K] float64, M[K,K] int32) for centers[K,3]."""
    lib = _load()
    c = _c(centers, np.float64)
    K = c.shape[0]
    d = np.empty((K, K), dtype=np.float64)
    M = np.empty((K, K), dtype=np.int32)
    lib.oracle_center_tables(_ptr(c), K, _ptr(d), _ptr(M))
    return d, M


def search_step(colors, centers, m, prune=True, literal=False):
    """One assignment pass from memberships ``m``.

    Returns (new m uint8, min_dist float64, evaluations)."""
    lib = _load()
    colors = _c(colors, np.uint32)
    c = _c(centers, np.float64)
    K = c.shape[0]
    d, M = center_tables(c)
    m2 = _c(m, np.uint8).copy()
    mind = np.empty(colors.shape[0], dtype=np.float64)
    ev = lib.oracle_search_step(_ptr(colors), colors.shape[0], _ptr(c), K,
                                _ptr(d), _ptr(M), _ptr(m2), _ptr(mind),
                                int(bool(prune)), int(bool(literal)))
    return m2, mind, int(ev)


def update_step(colors, counts, n_pixels, m, centers):
    """One weighted centroid update; returns new centers (float64 [K,3])."""
    lib = _load()
    colors = _c(colors, np.uint32)
    counts = _c(counts, np.uint32)
    m = _c(m, np.uint8)
    c = _c(centers, np.float64).copy()
    lib.oracle_update_step(_ptr(colors), _ptr(counts), colors.shape[0],
                           int(n_pixels), _ptr(m), c.shape[0], _ptr(c))
    return c


def weighted_sse(counts, n_pixels, min_dist):
    lib = _load()
    counts = _c(counts, np.uint32)
    md = _c(min_dist, np.float64)
    return float(lib.oracle_weighted_sse(_ptr(counts), counts.shape[0],
                                         int(n_pixels), _ptr(md)))


def wsm(colors, counts, n_pixels, init_centers, max_iters=50, eps=1e-4,
        prune=True, literal=False):
    """Run Alg. 2 to termination.

    Returns a dict with centers [K,3] float64, m uint8 [N'], sse [iters],
    evals [iters], iters, converged."""
    lib = _load()
    colors = _c(colors, np.uint32)
    counts = _c(counts, np.uint32)
    init = _c(init_centers, np.float64)
    K = init.shape[0]
    n = colors.shape[0]
    centers = np.empty((K, 3), dtype=np.float64)
    m = np.empty(n, dtype=np.uint8)
    sse = np.zeros(max_iters, dtype=np.float64)
    evals = np.zeros(max_iters, dtype=np.int64)
    iters = ctypes.c_int32(0)
    conv = ctypes.c_int32(0)
    rc = lib.oracle_wsm(_ptr(colors), _ptr(counts), n, int(n_pixels), K,
                        _ptr(init), int(max_iters), float(eps),
                        int(bool(prune)), int(bool(literal)), _ptr(centers),
                        _ptr(m), _ptr(sse), _ptr(evals), ctypes.byref(iters),
                        ctypes.byref(conv))
    if rc != 0:
        raise ValueError("oracle_wsm: invalid arguments")
    it = iters.value
    return dict(centers=centers, m=m, sse=sse[:it].copy(),
                evals=evals[:it].copy(), iters=it, converged=bool(conv.value))


def kmeans_pixels(rgb, init_centers, max_iters=50, eps=1e-4):
    """Alg. 1 on every pixel with full search (same tie key and stopping)."""
    lib = _load()
    rgb = _c(rgb, np.uint8).reshape(-1, 3)
    init = _c(init_centers, np.float64)
    K = init.shape[0]
    n = rgb.shape[0]
    centers = np.empty((K, 3), dtype=np.float64)
    m = np.empty(n, dtype=np.uint8)
    sse = np.zeros(max_iters, dtype=np.float64)
    iters = ctypes.c_int32(0)
    conv = ctypes.c_int32(0)
    rc = lib.oracle_kmeans_pixels(_ptr(rgb), n, K, _ptr(init), int(max_iters),
                                  float(eps), _ptr(centers), _ptr(m),
                                  _ptr(sse), ctypes.byref(iters),
                                  ctypes.byref(conv))
    if rc != 0:
        raise ValueError("oracle_kmeans_pixels: invalid arguments")
    it = iters.value
    return dict(centers=centers, m=m, sse=sse[:it].copy(), iters=it,
                converged=bool(conv.value))


def assign_colors(colors, counts, n_pixels, m, centers):
    """Final per-unique-color palette index and the weighted MSE."""
    lib = _load()
    colors = _c(colors, np.uint32)
    counts = _c(counts, np.uint32)
    m = _c(m, np.uint8)
    c = _c(centers, np.float64)
    idx = np.empty(colors.shape[0], dtype=np.uint8)
    mse = lib.oracle_assign_colors(_ptr(colors), _ptr(counts), colors.shape[0],
                                   int(n_pixels), _ptr(m), _ptr(c), c.shape[0],
                                   _ptr(idx))
    return idx, float(mse)


def map_pixels(rgb, colors, m, centers):
    """Per-pixel palette index (uint8) and MSE (Sec. 3.1)."""
    lib = _load()
    rgb = _c(rgb, np.uint8).reshape(-1, 3)
    colors = _c(colors, np.uint32)
    m = _c(m, np.uint8)
    c = _c(centers, np.float64)
    idx = np.empty(rgb.shape[0], dtype=np.uint8)
    mse = ctypes.c_double(0.0)
    rc = lib.oracle_map(_ptr(rgb), rgb.shape[0], _ptr(colors), colors.shape[0],
                        _ptr(m), _ptr(c), c.shape[0], _ptr(idx),
                        ctypes.byref(mse))
    if rc != 0:
        raise ValueError("oracle_map: pixel color missing from the table")
    return idx, float(mse.value)


def psnr(mse: float) -> float:
    """PSNR of Sec. 3.1: 20 log10(255 / sqrt(MSE))."""
    return float(20.0 * np.log10(255.0 / np.sqrt(mse))) if mse > 0 else float("inf")


def distortion(x, m, centers):
    """D = (1/N) sum_p ||x_p - c_{m(p)}||^2 with the assignment m frozen
    (Eq. 1 over pixels); x [n,3] and centers [K,3] as float64."""
    lib = _load()
    x = _c(x, np.float64).reshape(-1, 3)
    m = _c(m, np.uint8).reshape(-1)
    c = _c(centers, np.float64)
    return float(lib.oracle_distortion(_ptr(x), x.shape[0], _ptr(m), _ptr(c), c.shape[0]))


def distortion_grad(x, m, centers, g=1.0):
    """(dD/dx [n,3], dD/dc [K,3]) of distortion(), scaled by g."""
    lib = _load()
    x = _c(x, np.float64).reshape(-1, 3)
    m = _c(m, np.uint8).reshape(-1)
    c = _c(centers, np.float64)
    gx = np.empty_like(x)
    gc = np.empty_like(c)
    lib.oracle_distortion_grad(_ptr(x), x.shape[0], _ptr(m), _ptr(c), c.shape[0], float(g),
                               _ptr(gx), _ptr(gc))
    return gx, gc

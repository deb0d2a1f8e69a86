"""MI355X (gfx950) weighted sort-means color quantizer.

Thin Python binding of ``libwsm.so`` (C ABI in include/wsm.h): every step runs
in the library's HIP kernels; this module only allocates device buffers with
PyTorch, passes pointers and the current stream, and reads back sizes.

Method: M. E. Celebi, "Fast Color Quantization Using Weighted Sort-Means
Clustering" -- k-means on the unique colors of an image weighted by their
pixel counts (Sec. 2), with the sort-means nearest-center search (Alg. 2),
stopped by the relative SSE change criterion of Sec. 3.2.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch  # imported before the library so both share one HIP runtime

__all__ = [
    "WsmError", "library_path", "reduce_colors", "reduce_colors_into",
    "State", "IterateGraph", "init", "init_pixels", "map_pixels", "palette_from_indices",
    "quantize", "distortion", "distortion_into", "distortion_workspace", "quantize_batch",
    "Batch", "MAX_K", "HISTORY",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwsm.so")
MAX_K = 256
HISTORY = 1024
POINTS_COLORS = 0
POINTS_PIXELS = 1


class WsmError(RuntimeError):
    pass


class _Problem(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("points", ctypes.c_int32),
        ("n_points", ctypes.c_int64),
        ("n_pixels", ctypes.c_int64),
        ("state", ctypes.c_void_p),
        ("state_bytes", ctypes.c_size_t),
        ("colors", ctypes.c_void_p),
        ("counts", ctypes.c_void_p),
        ("rgb", ctypes.c_void_p),
        ("magic", ctypes.c_uint32),
        ("grid", ctypes.c_int32),
    ]


class _Views(ctypes.Structure):
    _fields_ = [
        ("palette", ctypes.c_void_p),
        ("membership", ctypes.c_void_p),
        ("sse_history", ctypes.c_void_p),
        ("evals_history", ctypes.c_void_p),
        ("info", ctypes.c_void_p),
        ("palette64", ctypes.c_void_p),
    ]


def library_path() -> str:
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise WsmError(
            f"{_LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_1011_0093_amd/build.py`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I64, I32, SZ, D = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t,
                          ctypes.c_double)
    PP = ctypes.POINTER(_Problem)
    lib.wsm_status_string.argtypes = [I32]
    lib.wsm_status_string.restype = ctypes.c_char_p
    lib.wsm_reduce_workspace_bytes.argtypes = [I64, ctypes.POINTER(ctypes.c_size_t)]
    lib.wsm_reduce_colors.argtypes = [P, I64, P, P, I64, P, P, SZ, P]
    lib.wsm_state_bytes.argtypes = [I64, I32, ctypes.POINTER(ctypes.c_size_t)]
    lib.wsm_init.argtypes = [PP, P, SZ, P, P, I64, I64, I32, P, P]
    lib.wsm_init_pixels.argtypes = [PP, P, SZ, P, I64, I32, P, P]
    lib.wsm_iterate.argtypes = [PP, I32, D, P]
    lib.wsm_iterate_full.argtypes = [PP, I32, D, P]
    lib.wsm_state_views.argtypes = [PP, ctypes.POINTER(_Views)]
    lib.wsm_map_pixels.argtypes = [PP, P, I64, P, P, P, P, P]
    lib.wsm_gather_palette.argtypes = [P, I64, P, I32, P, P]
    lib.wsm_timing_attach.argtypes = [I32, I32]
    lib.wsm_timing_read.argtypes = [ctypes.POINTER(ctypes.c_float), I32, ctypes.POINTER(I32)]
    lib.wsm_timing_detach.argtypes = []
    lib.wsm_reduce_colors_static.argtypes = [P, I64, P, P, I64, P, P]
    lib.wsm_distortion_workspace_bytes.argtypes = [I32, I64, I32, ctypes.POINTER(SZ)]
    lib.wsm_distortion.argtypes = [P, P, P, I32, I64, I32, P, P, SZ, P]
    lib.wsm_distortion_backward.argtypes = [P, P, P, I32, I64, I32, P, P, P, P, SZ, P]
    lib.wsm_batch_workspace_bytes.argtypes = [I32, PP, P, P, P, ctypes.POINTER(SZ)]
    lib.wsm_batch_create.argtypes = [I32, PP, P, P, P, P, P, SZ, ctypes.POINTER(P)]
    lib.wsm_batch_launch.argtypes = [P, P]
    lib.wsm_batch_error.argtypes = [P, ctypes.POINTER(P)]
    lib.wsm_batch_destroy.argtypes = [P]
    lib.wsm_iterate_graph_create.argtypes = [PP, I32, D, I32, ctypes.POINTER(P)]
    lib.wsm_iterate_graph_launch.argtypes = [P, P]
    lib.wsm_iterate_graph_destroy.argtypes = [P]
    for f in ("wsm_reduce_workspace_bytes", "wsm_reduce_colors", "wsm_state_bytes", "wsm_init",
              "wsm_init_pixels", "wsm_iterate", "wsm_iterate_full", "wsm_state_views",
              "wsm_map_pixels", "wsm_gather_palette", "wsm_timing_attach", "wsm_timing_read",
              "wsm_timing_detach", "wsm_iterate_graph_create", "wsm_iterate_graph_launch",
              "wsm_iterate_graph_destroy", "wsm_reduce_colors_static",
              "wsm_distortion_workspace_bytes", "wsm_distortion", "wsm_distortion_backward",
              "wsm_batch_workspace_bytes", "wsm_batch_create", "wsm_batch_launch",
              "wsm_batch_error", "wsm_batch_destroy"):
        getattr(lib, f).restype = I32
    return lib


_lib = _load()


def _check(rc: int, what: str):
    if rc != 0:
        msg = _lib.wsm_status_string(rc).decode()
        raise WsmError(f"{what}: {msg} ({rc})")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise WsmError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise WsmError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise WsmError(f"{name} must be contiguous")
    return t


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


# ---------------------------------------------------------------------------
# Data reduction.

def reduce_workspace_bytes(n_pixels: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.wsm_reduce_workspace_bytes(int(n_pixels), ctypes.byref(out)),
           "wsm_reduce_workspace_bytes")
    return int(out.value)


def reduce_colors_into(img: torch.Tensor, colors: torch.Tensor, counts: torch.Tensor,
                       n_unique: torch.Tensor, workspace: torch.Tensor) -> None:
    """Asynchronous form: fills caller-provided buffers on the current stream."""
    img = _dev(img, torch.uint8, "img")
    n = img.numel() // 3
    _check(_lib.wsm_reduce_colors(_ptr(img), n, _ptr(colors), _ptr(counts), colors.numel(),
                                  _ptr(n_unique), _ptr(workspace), workspace.numel(), _stream()),
           "wsm_reduce_colors")


def reduce_colors_static_into(img: torch.Tensor, colors: torch.Tensor, counts: torch.Tensor,
                              n_unique: torch.Tensor) -> None:
    """Allocation-free form (wsm_reduce_colors_static): the library's own
    workspace, images of at most 2^24 pixels; asynchronous on the current
    stream."""
    img = _dev(img, torch.uint8, "img")
    n = img.numel() // 3
    _check(_lib.wsm_reduce_colors_static(_ptr(img), n, _ptr(colors), _ptr(counts), colors.numel(),
                                         _ptr(n_unique), _stream()), "wsm_reduce_colors_static")


def reduce_colors(img: torch.Tensor):
    """Unique colors (ascending 0x00RRGGBB, int32 view of uint32) and pixel
    counts of an 8-bit RGB image on the GPU.  Reads the count back (one host
    synchronisation)."""
    img = _dev(img, torch.uint8, "img")
    if img.numel() % 3 != 0 or img.numel() == 0:
        raise WsmError("img must hold n_pixels * 3 bytes")
    n = img.numel() // 3
    cap = min(n, 1 << 24)
    dev = img.device
    colors = torch.empty(cap, dtype=torch.int32, device=dev)
    counts = torch.empty(cap, dtype=torch.int32, device=dev)
    nu = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(reduce_workspace_bytes(n), dtype=torch.uint8, device=dev)
    reduce_colors_into(img, colors, counts, nu, ws)
    k = int(nu.item())
    if k < 1:
        raise WsmError("device error in wsm_reduce_colors")
    return colors[:k], counts[:k]


# ---------------------------------------------------------------------------
# Clustering state.

def state_bytes(n_points: int, k: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.wsm_state_bytes(int(n_points), int(k), ctypes.byref(out)), "wsm_state_bytes")
    return int(out.value)


@dataclass
class State:
    """A clustering state: the device buffer and its host descriptor.
    Keeps references to the point tensors the state is bound to."""

    prob: _Problem
    buf: torch.Tensor
    refs: tuple

    @property
    def k(self) -> int:
        return int(self.prob.k)

    @property
    def n_points(self) -> int:
        return int(self.prob.n_points)

    @property
    def n_pixels(self) -> int:
        return int(self.prob.n_pixels)

    @property
    def grid(self) -> int:
        """Blocks of the search launch (wsm_problem.grid)."""
        return int(self.prob.grid)

    @grid.setter
    def grid(self, blocks: int) -> None:
        """Fewer (or more) search blocks for the following iterate calls,
        1..2048, e.g. to share the GPU with work on other streams; the
        results do not depend on it (the SSE's last bits aside)."""
        if not 1 <= int(blocks) <= 2048:
            raise WsmError("grid must be in 1..2048")
        self.prob.grid = int(blocks)

    def iterate(self, max_iters: int = 50, eps: float = 1e-4) -> None:
        """Sort-means iterations (asynchronous on the current stream)."""
        _check(_lib.wsm_iterate(ctypes.byref(self.prob), int(max_iters), float(eps), _stream()),
               "wsm_iterate")

    def iterate_full(self, max_iters: int = 50, eps: float = 1e-4) -> None:
        """Full-search iterations (the plain batch k-means comparator)."""
        _check(_lib.wsm_iterate_full(ctypes.byref(self.prob), int(max_iters), float(eps),
                                     _stream()), "wsm_iterate_full")

    def graph(self, max_iters: int = 50, eps: float = 1e-4, full: bool = False) -> "IterateGraph":
        """The launch sequence of iterate(max_iters, eps) (or iterate_full),
        recorded once into a HIP graph that can be replayed on this state."""
        return IterateGraph(self, max_iters, eps, full)

    def _views(self) -> _Views:
        v = _Views()
        _check(_lib.wsm_state_views(ctypes.byref(self.prob), ctypes.byref(v)), "wsm_state_views")
        return v

    def _slice(self, addr: int, nbytes: int) -> torch.Tensor:
        off = addr - self.buf.data_ptr()
        return self.buf[off:off + nbytes]

    def palette(self) -> torch.Tensor:
        """float32 [k, 3] palette after the last update (device)."""
        v = self._views()
        return self._slice(v.palette, self.k * 16).view(torch.float32).view(self.k, 4)[:, :3]

    def palette64(self) -> torch.Tensor:
        """float64 [k, 3] palette after the last update (device): the centers
        the searches decide by; palette() is their float32 rounding."""
        v = self._views()
        return self._slice(v.palette64, self.k * 32).view(torch.float64).view(self.k, 4)[:, :3]

    def membership(self) -> torch.Tensor:
        v = self._views()
        return self._slice(v.membership, self.n_points)

    def info(self) -> dict:
        v = self._views()
        i = self._slice(v.info, 16).view(torch.int32).cpu().tolist()
        return dict(iters=i[0], converged=bool(i[1]), err=i[2])

    def history(self):
        """(sse[iters], evals[iters]) as numpy arrays."""
        v = self._views()
        it = self.info()["iters"]
        n = min(it, HISTORY)
        sse = self._slice(v.sse_history, 8 * HISTORY).view(torch.float64)[:n].cpu().numpy()
        ev = self._slice(v.evals_history, 8 * HISTORY).view(torch.int64)[:n].cpu().numpy()
        return sse, ev


class IterateGraph:
    """A caller-owned HIP graph of one iterate call's launches
    (wsm_iterate_graph_create / _launch / _destroy).  launch() has the effect
    of state.iterate(max_iters, eps) (or iterate_full) on the current
    stream; the state may be re-initialised with init(..., reuse=state)
    between launches."""

    def __init__(self, state: State, max_iters: int, eps: float, full: bool = False):
        self.state = state
        h = ctypes.c_void_p(0)
        _check(_lib.wsm_iterate_graph_create(ctypes.byref(state.prob), int(max_iters), float(eps),
                                             1 if full else 0, ctypes.byref(h)),
               "wsm_iterate_graph_create")
        self._h = h

    def launch(self) -> None:
        if not self._h:
            raise WsmError("graph already closed")
        _check(_lib.wsm_iterate_graph_launch(self._h, _stream()), "wsm_iterate_graph_launch")

    def close(self) -> None:
        if self._h:
            _lib.wsm_iterate_graph_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched persistent iterations (wsm_batch_*): one launch iterates every
    state of the list, each as state.iterate(max_iters[i], eps[i]) would.
    grid and rows_per_item (per state, 0 = default) split the work; an
    autotuner picks them.  The plan is recorded once; launch() runs it on
    the current stream (re-initialise the states with init(..., reuse=)
    before a launch that should start over)."""

    def __init__(self, states, max_iters, eps, grid=None, rows_per_item=None, tuned=True):
        n = len(states)
        self.states = list(states)
        if tuned and grid is None and rows_per_item is None:
            from . import autotune
            table = autotune.load()
            if table:
                split = [autotune.split_for(table, st.n_points, st.k) for st in states]
                grid = [g for g, _ in split]
                rows_per_item = [r for _, r in split]
        self._probs = (_Problem * n)(*[st.prob for st in states])
        as_list = lambda v, t: [t(x) for x in (v if hasattr(v, "__len__") else [v] * n)]  # noqa: E731
        self._mi = (ctypes.c_int32 * n)(*as_list(max_iters, int))
        self._eps = (ctypes.c_double * n)(*as_list(eps, float))
        self._grid = (ctypes.c_int32 * n)(*as_list(grid or 0, int))
        self._rpi = (ctypes.c_int32 * n)(*as_list(rows_per_item or 0, int))
        size = ctypes.c_size_t(0)
        _check(_lib.wsm_batch_workspace_bytes(n, self._probs, self._mi, self._grid, self._rpi,
                                              ctypes.byref(size)), "wsm_batch_workspace_bytes")
        dev = states[0].buf.device
        raw = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        self.ws = raw[off:off + int(size.value)]
        self._raw = raw
        h = ctypes.c_void_p(0)
        _check(_lib.wsm_batch_create(n, self._probs, self._mi, self._eps, self._grid, self._rpi,
                                     _ptr(self.ws), self.ws.numel(), ctypes.byref(h)),
               "wsm_batch_create")
        self._h = h
        e = ctypes.c_void_p(0)
        _check(_lib.wsm_batch_error(h, ctypes.byref(e)), "wsm_batch_error")
        self._err_off = e.value - self.ws.data_ptr()

    def launch(self) -> None:
        if not self._h:
            raise WsmError("batch already closed")
        _check(_lib.wsm_batch_launch(self._h, _stream()), "wsm_batch_launch")

    def error(self) -> int:
        """Error bits of the last run (reads the device; 0 when all is well)."""
        return int(self.ws[self._err_off:self._err_off + 4].view(torch.int32).item())

    def close(self) -> None:
        if self._h:
            _lib.wsm_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _new_state(n_points: int, k: int, device) -> torch.Tensor:
    nbytes = state_bytes(n_points, k)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def init(colors: torch.Tensor, counts: torch.Tensor, n_pixels: int, palette: torch.Tensor,
         reuse: "State | None" = None) -> State:
    """Bind a state to a unique-color table and an initial palette
    (float32 [k, 3] on the GPU).  With `reuse`, that state's device buffer is
    re-initialised instead of allocating a new one (it must be large enough)."""
    colors = _dev(colors, torch.int32, "colors")
    counts = _dev(counts, torch.int32, "counts")
    palette = _dev(palette, torch.float32, "palette")
    k = palette.shape[0]
    n = colors.numel()
    if reuse is not None and reuse.buf.numel() >= state_bytes(n, k) and reuse.buf.device == colors.device:
        buf = reuse.buf
    else:
        buf = _new_state(n, k, colors.device)
    prob = _Problem()
    _check(_lib.wsm_init(ctypes.byref(prob), _ptr(buf), buf.numel(), _ptr(colors), _ptr(counts),
                         n, int(n_pixels), k, _ptr(palette), _stream()), "wsm_init")
    return State(prob, buf, (colors, counts, palette))


def init_pixels(img: torch.Tensor, palette: torch.Tensor, reuse: "State | None" = None) -> State:
    """Bind a state to every pixel of an image (weight 1 each): Alg. 1.
    `reuse` as for init()."""
    img = _dev(img, torch.uint8, "img")
    palette = _dev(palette, torch.float32, "palette")
    k = palette.shape[0]
    n = img.numel() // 3
    if reuse is not None and reuse.buf.numel() >= state_bytes(n, k) and reuse.buf.device == img.device:
        buf = reuse.buf
    else:
        buf = _new_state(n, k, img.device)
    prob = _Problem()
    _check(_lib.wsm_init_pixels(ctypes.byref(prob), _ptr(buf), buf.numel(), _ptr(img), n, k,
                                _ptr(palette), _stream()), "wsm_init_pixels")
    return State(prob, buf, (img, palette))


def map_pixels(state: State, img: torch.Tensor, lut: torch.Tensor | None = None,
               want_rgb: bool = False, want_mse: bool = True):
    """Per-pixel palette index (uint8), optional quantized image and MSE.
    Returns (index, rgb_out or None, mse tensor [1] float64 or None)."""
    img = _dev(img, torch.uint8, "img")
    n = img.numel() // 3
    dev = img.device
    if lut is None:
        lut = torch.empty(1 << 24, dtype=torch.uint8, device=dev)
    idx = torch.empty(n, dtype=torch.uint8, device=dev)
    rgb_out = torch.empty_like(img) if want_rgb else None
    mse = torch.empty(1, dtype=torch.float64, device=dev) if want_mse else None
    _check(_lib.wsm_map_pixels(ctypes.byref(state.prob), _ptr(img), n, _ptr(lut), _ptr(idx),
                               _ptr(rgb_out), _ptr(mse), _stream()), "wsm_map_pixels")
    return idx, rgb_out, mse


def map_pixels_into(state: State, img: torch.Tensor, lut: torch.Tensor, index: torch.Tensor,
                    mse: torch.Tensor | None = None, rgb_out: torch.Tensor | None = None) -> None:
    """Asynchronous form of map_pixels with caller-provided outputs."""
    img = _dev(img, torch.uint8, "img")
    _check(_lib.wsm_map_pixels(ctypes.byref(state.prob), _ptr(img), img.numel() // 3, _ptr(lut),
                               _ptr(index), _ptr(rgb_out), _ptr(mse), _stream()), "wsm_map_pixels")


def palette_from_indices(colors: torch.Tensor, indices, out: torch.Tensor | None = None
                         ) -> torch.Tensor:
    """Initial palette: the unique colors at the given indices (the random
    subset the method starts from), as float32 [k, 3] on the GPU.  `indices`
    is a host sequence or a device int32 tensor."""
    colors = _dev(colors, torch.int32, "colors")
    if isinstance(indices, torch.Tensor) and indices.is_cuda:
        idx = _dev(indices, torch.int32, "indices")
    else:
        idx = torch.from_numpy(np.ascontiguousarray(np.asarray(indices, dtype=np.int32)))
        idx = idx.to(colors.device, non_blocking=False)
    k = idx.numel()
    if out is None:
        out = torch.empty((k, 3), dtype=torch.float32, device=colors.device)
    _check(_lib.wsm_gather_palette(_ptr(colors), colors.numel(), _ptr(idx), k, _ptr(out),
                                   _stream()), "wsm_gather_palette")
    return out


# ---------------------------------------------------------------------------
# Measurement hook.

KERNELS = dict(reduce_partition=1, reduce_compact=2, rows=3, search=4, map_assign=5,
               map_gather=6, full_step=7)


class kernel_timer:
    """Context manager: HIP events around every launch of one library kernel
    (on the stream it is launched on).  `.ms` holds the durations after exit."""

    def __init__(self, kernel: str, capacity: int = 4096):
        self.which = KERNELS[kernel]
        self.capacity = capacity
        self.ms: list[float] = []

    def __enter__(self):
        _check(_lib.wsm_timing_attach(self.which, self.capacity), "wsm_timing_attach")
        return self

    def __exit__(self, *exc):
        buf = (ctypes.c_float * self.capacity)()
        cnt = ctypes.c_int(0)
        try:
            _check(_lib.wsm_timing_read(buf, self.capacity, ctypes.byref(cnt)), "wsm_timing_read")
            self.ms = [float(buf[i]) for i in range(min(cnt.value, self.capacity))]
        finally:
            _lib.wsm_timing_detach()
        return False


def quantize(img: torch.Tensor, k: int, init_indices_fn, max_iters: int = 50, eps: float = 1e-4,
             want_rgb: bool = False):
    """Whole pipeline on one image: reduce, init from
    ``init_indices_fn(n_unique, k)``, iterate, map.  Returns
    (state, index, rgb_out, mse)."""
    n = img.numel() // 3
    colors, counts = reduce_colors(img)
    pal = palette_from_indices(colors, init_indices_fn(colors.numel(), k))
    st = init(colors, counts, n, pal)
    st.iterate(max_iters, eps)
    idx, rgb_out, mse = map_pixels(st, img, want_rgb=want_rgb)
    return st, idx, rgb_out, mse


# ---------------------------------------------------------------------------
# Differentiable form: the distortion of Eq. 1 over the pixels with frozen
# assignments (wsm_distortion / wsm_distortion_backward).

def _distortion_workspace(batch: int, n: int, k: int, device) -> torch.Tensor:
    out = ctypes.c_size_t(0)
    _check(_lib.wsm_distortion_workspace_bytes(int(batch), int(n), int(k), ctypes.byref(out)),
           "wsm_distortion_workspace_bytes")
    return torch.empty(int(out.value), dtype=torch.uint8, device=device)


class _Distortion(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, palette, index):
        B, N, _ = x.shape
        K = palette.shape[1]
        ws = _distortion_workspace(B, N, K, x.device)
        d = torch.empty(B, dtype=torch.float64, device=x.device)
        _check(_lib.wsm_distortion(_ptr(x), _ptr(index), _ptr(palette), B, N, K, _ptr(d),
                                   _ptr(ws), ws.numel(), _stream()), "wsm_distortion")
        ctx.save_for_backward(x, palette, index)
        ctx.mark_non_differentiable(index)
        return d

    @staticmethod
    def backward(ctx, grad_d):
        x, palette, index = ctx.saved_tensors
        B, N, _ = x.shape
        K = palette.shape[1]
        need_x, need_c = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_x or need_c):
            return None, None, None
        g = grad_d.detach().to(torch.float64).contiguous()
        gx = torch.empty_like(x) if need_x else None
        gc = torch.empty_like(palette) if need_c else None
        ws = _distortion_workspace(B, N, K, x.device)
        _check(_lib.wsm_distortion_backward(_ptr(x), _ptr(index), _ptr(palette), B, N, K, _ptr(g),
                                            _ptr(gx), _ptr(gc), _ptr(ws), ws.numel(), _stream()),
               "wsm_distortion_backward")
        return gx, gc, None


def distortion_into(x: torch.Tensor, palette: torch.Tensor, index: torch.Tensor,
                    d: torch.Tensor, workspace: torch.Tensor, grad_d: torch.Tensor = None,
                    grad_x: torch.Tensor = None, grad_palette: torch.Tensor = None) -> None:
    """The differentiable form's two calls on caller-owned buffers, without
    autograd: D into d (float64 [B]); and, when grad_d (float64 [B]) is
    given, the adjoint into grad_x and/or grad_palette.  Shapes as for
    distortion() ([B, N, 3] colors, [B, K, 3] palettes, [B, N] indices);
    workspace: uint8, at least wsm_distortion_workspace_bytes."""
    B, N, _ = x.shape
    K = palette.shape[1]
    _check(_lib.wsm_distortion(_ptr(x), _ptr(index), _ptr(palette), B, N, K, _ptr(d),
                               _ptr(workspace), workspace.numel(), _stream()), "wsm_distortion")
    if grad_d is not None:
        _check(_lib.wsm_distortion_backward(
            _ptr(x), _ptr(index), _ptr(palette), B, N, K, _ptr(grad_d),
            _ptr(grad_x), _ptr(grad_palette),
            _ptr(workspace), workspace.numel(), _stream()), "wsm_distortion_backward")


def distortion_workspace(batch: int, n: int, k: int, device) -> torch.Tensor:
    """A workspace for distortion_into (uint8 device tensor)."""
    return _distortion_workspace(batch, n, k, device)


def distortion(x: torch.Tensor, palette: torch.Tensor, index: torch.Tensor) -> torch.Tensor:
    """Per-image distortion D_i = (1/N) sum_p ||x_ip - c_{i,index(p)}||^2
    (float64 [B]) with the assignment frozen, differentiable in x (float32
    [B, N, 3] or [B, H, W, 3]) and palette (float32 [B, K, 3]); index is
    uint8 [B, N] (or [B, H, W]).  Forward and backward run in the library's
    kernels."""
    x = _dev(x, torch.float32, "x")
    palette = _dev(palette, torch.float32, "palette")
    index = _dev(index, torch.uint8, "index")
    B = x.shape[0]
    return _Distortion.apply(x.reshape(B, -1, 3), palette, index.reshape(B, -1))


def quantize_batch(x: torch.Tensor, k: int, init_indices_fn, max_iters: int = 50,
                   eps: float = 1e-4):
    """Forward pass of the differentiable form for a batch of float32 images
    (B, H, W, 3) whose values are 8-bit colors: WSM on each image -- every
    image reduced (one read-back of the B unique-color counts), its state
    initialised from ``init_indices_fn(n_unique, k)``, all of them iterated
    by one launch of the batched form (each image's result is that of
    State.iterate), then mapped.  Returns (palette float32 [B, k, 3], index
    uint8 [B, H*W], states)."""
    x = _dev(x, torch.float32, "x")
    B = x.shape[0]
    u8 = x.round().clamp(0, 255).to(torch.uint8)
    if not torch.equal(u8.to(torch.float32), x):
        raise WsmError("quantize_batch: x must hold 8-bit color values")
    u8 = u8.reshape(B, -1).contiguous()
    n = u8.shape[1] // 3
    dev = u8.device
    cap = min(n, 1 << 24)
    colors = torch.empty((B, cap), dtype=torch.int32, device=dev)
    counts = torch.empty((B, cap), dtype=torch.int32, device=dev)
    nu = torch.empty(B, dtype=torch.int32, device=dev)
    ws = torch.empty(reduce_workspace_bytes(n), dtype=torch.uint8, device=dev)
    for b in range(B):  # in stream order, so they share the workspace
        reduce_colors_into(u8[b], colors[b], counts[b], nu[b:b + 1], ws)
    nus = nu.cpu().tolist()
    if min(nus) < 1:
        raise WsmError("device error in wsm_reduce_colors")
    states = []
    for b in range(B):
        c, w = colors[b, :nus[b]], counts[b, :nus[b]]
        states.append(init(c, w, n, palette_from_indices(c, init_indices_fn(nus[b], k))))
    for b0 in range(0, B, 128):  # at most 128 images per batched launch
        batch = Batch(states[b0:b0 + 128], max_iters, eps)
        try:
            batch.launch()
            if batch.error() != 0:
                raise WsmError("batched iterations reported a device error")
        finally:
            batch.close()
    lut = torch.empty(1 << 24, dtype=torch.uint8, device=dev)
    idx = torch.empty((B, n), dtype=torch.uint8, device=dev)
    for b in range(B):  # the table is rewritten at every image's keys before it is read
        map_pixels_into(states[b], u8[b], lut, idx[b])
    pals = torch.stack([st.palette() for st in states]).contiguous()
    return pals, idx, states

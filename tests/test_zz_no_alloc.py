"""The allocation-free reduction (wsm_reduce_colors_static, its workspace a
device array of the library) against the workspace form (wsm_reduce_colors),
through the C ABI: calls in a row on one GPU, each on a smaller image than
the one before (the array keeps the last call's contents), bit-exact."""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_static_reduce_matches_workspace_reduce():
    import paper_1011_0093_amd as wsm
    lib = wsm._lib
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # largest accepted image first (2^24 pixels), then smaller ones
    for name, seed in (("large", 0), ("medium", 1), ("small", 2)):
        img = synth.workload_image(name, seed)
        n = img.shape[0] * img.shape[1]
        print("[case] static reduce", name, seed, img.shape, flush=True)
        g = torch.from_numpy(img).cuda()
        ref_c, ref_n = wsm.reduce_colors(g)
        cap = min(n, 1 << 24)
        colors = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        counts = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        nu = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        rc = lib.wsm_reduce_colors_static(_p(g), n, _p(colors), _p(counts), cap, _p(nu), stream)
        assert rc == 0, rc
        k = int(nu.item())
        assert k == ref_c.numel()
        assert torch.equal(colors[:k], ref_c) and torch.equal(counts[:k], ref_n)
        assert int(counts[:k].sum().item()) == n
        # entries past n_unique are left untouched
        assert bool((colors[k:] == -1).all()) and bool((counts[k:] == -1).all())
    # sizes past the array are refused on the host, before any launch
    assert lib.wsm_reduce_colors_static(_p(g), (1 << 24) + 1, _p(colors), _p(counts), 1 << 24,
                                        _p(nu), stream) == -2
    assert lib.wsm_reduce_colors_static(_p(g), n, _p(colors), _p(counts), n - 1, _p(nu),
                                        stream) == -2


def test_static_reduce_binding_on_a_captured_stream():
    """The static form inside a CUDA graph capture (where allocation is not
    allowed), replayed twice with host work in between."""
    import paper_1011_0093_amd as wsm
    img = synth.workload_image("small", 3)
    n = img.shape[0] * img.shape[1]
    print("[case] static reduce under graph capture, small seed 3", flush=True)
    g = torch.from_numpy(img).cuda()
    ref_c, ref_n = wsm.reduce_colors(g)
    colors = torch.zeros(n, dtype=torch.int32, device="cuda")
    counts = torch.zeros(n, dtype=torch.int32, device="cuda")
    nu = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        wsm.reduce_colors_static_into(g, colors, counts, nu)   # warm-up: address lookup
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        wsm.reduce_colors_static_into(g, colors, counts, nu)
    for _ in range(2):
        colors.zero_()
        counts.zero_()
        nu.zero_()
        graph.replay()
        torch.cuda.synchronize()
        k = int(nu.item())
        assert k == ref_c.numel()
        assert torch.equal(colors[:k], ref_c) and torch.equal(counts[:k], ref_n)

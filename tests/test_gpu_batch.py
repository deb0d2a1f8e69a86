"""GPU tests of the batched persistent form (wsm_batch_*, through the C ABI
via the binding): every image of a batch of uneven images, each with its
own K, iteration budget and eps, ends exactly where wsm_iterate takes it
alone, and that is the oracle's result."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from parity_util import SUM_RTOL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wsm():
    import paper_1011_0093_amd as wsm
    return wsm


def _say(*a):
    print("[case]", *a, flush=True)


# (side, K, max_iters, eps): small and large tables, every search variant
# (K <= 32, 33..127, >= 128), budgets that run out and eps stops that fire
CASES = [(96, 2, 20, 1e-3), (128, 16, 30, 1e-4), (200, 33, 12, 0.0), (256, 64, 50, 1e-3),
         (160, 128, 8, 0.0), (300, 256, 6, 1e-4), (64, 5, 50, 1e-4), (400, 200, 10, 1e-3),
         (128, 256, 3, 0.0), (220, 47, 25, 1e-4)]


def _tables(wsm, seed0=0):
    out = []
    for j, (side, K, mi, eps) in enumerate(CASES):
        img = synth.sinusoid_field_image(seed0 + j, side, side)
        g = torch.from_numpy(img).cuda()
        col, cnt = wsm.reduce_colors(g)
        pal = wsm.palette_from_indices(col, synth.init_indices(seed0 + j, col.numel(), K))
        out.append((img, g, col, cnt, pal, K, mi, eps))
    return out


@pytest.mark.parametrize("split", ["problem", "tuned", "coarse"])
def test_batch_equals_single_image_iterate(split):
    wsm = _wsm()
    _say("batch of", len(CASES), "uneven images, work split", split)
    tabs = _tables(wsm)
    ref, states = [], []
    for img, g, col, cnt, pal, K, mi, eps in tabs:
        n_pix = img.shape[0] * img.shape[1]
        r = wsm.init(col, cnt, n_pix, pal)
        r.iterate(mi, eps)
        ref.append(r)
        states.append(wsm.init(col, cnt, n_pix, pal))
    if split in ("problem", "tuned"):
        # each problem's own grid (the single-image launch's), or the
        # autotuned split from the committed table
        grid, rpi = None, None
    else:  # few large search blocks, many rows per rows item
        grid = [max(1, st.n_points // 16384) for st in states]
        rpi = [16] * len(states)
    b = wsm.Batch(states, [c[2] for c in CASES], [c[3] for c in CASES], grid, rpi,
                  tuned=(split == "tuned"))
    try:
        for rep in range(2):
            if rep:
                states = [wsm.init(t[2], t[3], t[0].shape[0] * t[0].shape[1], t[4], reuse=st)
                          for t, st in zip(tabs, states)]
            b.launch()
            torch.cuda.synchronize()
            assert b.error() == 0
            for j, (st, r) in enumerate(zip(states, ref)):
                assert st.info() == r.info(), (rep, j)
                assert torch.equal(st.palette64().cpu(), r.palette64().cpu()), (rep, j)
                assert torch.equal(st.membership().cpu(), r.membership().cpu()), (rep, j)
                s1, e1 = st.history()
                s2, e2 = r.history()
                assert np.array_equal(e1, e2), (rep, j)
                # float64 SSE sums: the batched form's search blocks (and, for
                # other splits, their number) add the terms in another order
                # than the single-image launches, whose deferred scans add
                # theirs in queue order
                np.testing.assert_allclose(s1, s2, rtol=SUM_RTOL)
    finally:
        b.close()


def test_batch_results_equal_the_oracle():
    wsm = _wsm()
    _say("batch vs oracle, first 6 cases")
    tabs = _tables(wsm, seed0=20)[:6]
    states = []
    for img, g, col, cnt, pal, K, mi, eps in tabs:
        states.append(wsm.init(col, cnt, img.shape[0] * img.shape[1], pal))
    b = wsm.Batch(states, [c[2] for c in CASES[:6]], [c[3] for c in CASES[:6]])
    b.launch()
    torch.cuda.synchronize()
    assert b.error() == 0
    for st, (img, g, col, cnt, pal, K, mi, eps) in zip(states, tabs):
        colors = col.cpu().numpy().astype(np.int64).astype(np.uint32)
        counts = cnt.cpu().numpy().astype(np.int64).astype(np.uint32)
        r = oracle.wsm(colors, counts, img.shape[0] * img.shape[1],
                       pal.cpu().numpy().astype(np.float64), mi, eps)
        assert st.info()["iters"] == r["iters"] and st.info()["converged"] == r["converged"]
        assert np.array_equal(st.palette64().cpu().numpy(), r["centers"])
        assert np.array_equal(st.membership().cpu().numpy(), r["m"])
    b.close()

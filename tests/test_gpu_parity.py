"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every test prints the case it runs (workload, seed, shape, entry point)
before touching the GPU.  Inputs are the seeded synthetic images of synth/.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from parity_util import CENTER_TOL, MSE_RTOL, SUM_RTOL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wsm():
    import paper_1011_0093_amd as wsm
    return wsm


def _say(*a):
    print("[case]", *a, flush=True)


def _gpu_img(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _u32(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


# ---------------------------------------------------------------------------
# Data reduction: bit-exact.

REDUCE_CASES = [
    ("small", 0), ("small", 3), ("medium", 0), ("medium", 2),
]


@pytest.mark.parametrize("name,seed", REDUCE_CASES)
def test_reduce_bit_exact_workloads(name, seed):
    wsm = _wsm()
    img = synth.workload_image(name, seed)
    _say("reduce", name, seed, img.shape)
    col, cnt = wsm.reduce_colors(_gpu_img(img))
    rc, rn = oracle.reduce_colors(img)
    assert np.array_equal(_u32(col), rc)
    assert np.array_equal(_u32(cnt), rn)


@pytest.mark.parametrize("shape,kind", [
    ((1, 1, 3), "one"), ((7, 5, 3), "const"), ((1000, 7, 3), "noise"),
    ((333, 77, 3), "noise"), ((64, 64, 3), "two"), ((1024, 1024, 3), "noise"),
    ((700, 701, 3), "coarse"),
])
def test_reduce_edge_cases(shape, kind):
    wsm = _wsm()
    rng = np.random.default_rng(hash((shape, kind)) & 0xFFFF)
    if kind == "one":
        img = np.array([[[1, 2, 3]]], dtype=np.uint8)
    elif kind == "const":
        img = np.full(shape, 200, dtype=np.uint8)
    elif kind == "two":
        img = np.zeros(shape, dtype=np.uint8)
        img[::2] = (255, 255, 255)
    elif kind == "coarse":
        img = (rng.integers(0, 4, size=shape) * 85).astype(np.uint8)
    else:
        img = rng.integers(0, 256, size=shape, dtype=np.uint8)
    _say("reduce edge", shape, kind)
    col, cnt = wsm.reduce_colors(_gpu_img(img))
    rc, rn = oracle.reduce_colors(img)
    assert np.array_equal(_u32(col), rc) and np.array_equal(_u32(cnt), rn)


# Partition blocks are dealt tiles in XCD-contiguous runs (ntiles rounded up
# to a multiple of 8, the blocks past the last tile idle): every tile count
# mod 8, with 1024-pixel tiles, and one with 16384-pixel tiles.
@pytest.mark.parametrize("n_pixels", [1024 * k + 5 for k in range(8, 16)] + [16384 * 515 - 7])
def test_reduce_tile_counts_mod_8(n_pixels):
    wsm = _wsm()
    rng = np.random.default_rng(n_pixels)
    img = (rng.integers(0, 64, size=(1, n_pixels, 3)) * 4 + 1).astype(np.uint8)
    _say("reduce tile counts", n_pixels)
    col, cnt = wsm.reduce_colors(_gpu_img(img))
    rc, rn = oracle.reduce_colors(img)
    assert np.array_equal(_u32(col), rc) and np.array_equal(_u32(cnt), rn)


def test_timing_hook_with_launches_from_several_threads():
    """The measurement hook hands out its events under a lock: four threads,
    each reducing on a stream of its own while the hook times the partition
    kernel, get 12 distinct event pairs between them and bit-exact results."""
    from concurrent.futures import ThreadPoolExecutor
    wsm = _wsm()
    img = synth.workload_image("small", 0)
    rc, rn = oracle.reduce_colors(img)
    g = _gpu_img(img)
    _say("timing hook, 4 threads x 5 reductions of small seed 0")

    def work(_):
        torch.cuda.set_device(0)
        st = torch.cuda.Stream()
        ok = True
        with torch.cuda.stream(st):
            for _ in range(5):
                col, cnt = wsm.reduce_colors(g)
                ok &= np.array_equal(_u32(col), rc) and np.array_equal(_u32(cnt), rn)
        st.synchronize()
        return ok

    with wsm.kernel_timer("reduce_partition", capacity=12) as kt:
        with ThreadPoolExecutor(4) as ex:
            oks = list(ex.map(work, range(4)))
    assert all(oks)
    assert len(kt.ms) == 12 and all(t > 0.0 for t in kt.ms)


def test_reduce_unaligned_input_and_full_size():
    wsm = _wsm()
    img = synth.workload_image("large", 0)
    _say("reduce large 4096x4096 seed 0 (aligned) and unaligned 1-byte offset")
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    rc, rn = oracle.reduce_colors(img)
    assert np.array_equal(_u32(col), rc) and np.array_equal(_u32(cnt), rn)
    # an image that starts one byte into a buffer takes the unaligned path
    sub = img[:1024, :1000].copy()
    buf = torch.empty(sub.size + 16, dtype=torch.uint8, device="cuda")
    view = buf[1:1 + sub.size]
    view.copy_(torch.from_numpy(sub.reshape(-1)).cuda())
    col, cnt = wsm.reduce_colors(view)
    rc, rn = oracle.reduce_colors(sub)
    assert np.array_equal(_u32(col), rc) and np.array_equal(_u32(cnt), rn)


def test_reduce_more_tiles_than_one_chunk():
    # 4196 x 4096 pixels = 1050 tiles of 16384: the compaction reads the
    # slice words in chunks of 1024 tiles, and the second chunk ends inside
    # its first group of 64 tiles.
    wsm = _wsm()
    big = synth.workload_image("large", 0)
    img = np.concatenate([big, big[:100, ::-1]], axis=0)
    _say("reduce", img.shape, "1050 tiles")
    col, cnt = wsm.reduce_colors(_gpu_img(img))
    rc, rn = oracle.reduce_colors(img)
    assert np.array_equal(_u32(col), rc) and np.array_equal(_u32(cnt), rn)
    assert int(rn.sum()) == img.shape[0] * img.shape[1]


@pytest.mark.parametrize("case", ["one_color_2^24", "one_color_2^25", "pair_2^24", "8200x4096"])
def test_reduce_heavy_bins_and_many_tiles(case):
    # Bins far past 2^16 pixels: one color filling 4096x4096 and 8192x4096
    # images (2048 tiles, two passes of the compaction's tile words), two
    # colors whose keys differ in the last bit (neighbouring bins), and a
    # 33.6M-pixel image of 2051 tiles whose last pass holds 3 tiles.
    wsm = _wsm()
    if case == "one_color_2^24":
        img = np.full((4096, 4096, 3), (17, 140, 201), dtype=np.uint8)
    elif case == "one_color_2^25":
        img = np.full((8192, 4096, 3), (250, 3, 98), dtype=np.uint8)
    elif case == "pair_2^24":
        img = np.zeros((4096, 4096, 3), dtype=np.uint8)
        img[:] = (40, 200, 30)
        img[1::2, :, 2] = 31
        img[::7, ::3] = (40, 200, 31)
    else:
        big = synth.workload_image("large", 0)
        img = np.concatenate([big, big[::-1][:4104]], axis=0)
    _say("reduce", case, img.shape)
    col, cnt = wsm.reduce_colors(_gpu_img(img))
    rc, rn = oracle.reduce_colors(img)
    assert np.array_equal(_u32(col), rc) and np.array_equal(_u32(cnt), rn)
    assert int(rn.sum()) == img.shape[0] * img.shape[1]


# ---------------------------------------------------------------------------
# Iterations, lock-step.  The GPU keeps every center in float64 as well (the
# correctly rounded mean of its exact integer sums) and decides every choice
# as float64 arithmetic on those centers does, so from the GPU's own state
# after step t-1 the oracle's step t gives exactly the GPU's memberships and
# float64 centers of step t.  Each step t comes from a fresh run of t
# iterations in one call, so the kernels a long call uses after its first
# step (the flattened scans and their deferral for K >= 128) are the ones
# checked.

def _gpu_table(img):
    wsm = _wsm()
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    return g, col, cnt, _u32(col), _u32(cnt)


def _check_step(colors, counts, n_pix, m_prev, c_prev, m_gpu, c_gpu64, c_gpu32, sse_gpu, ev_gpu,
                check_evals=True, t=None):
    """Oracle step from the GPU state (m_prev, c_prev) against the GPU's
    step: memberships and float64 centers bit-exact, SSE to float64 rounding,
    evaluation counts within the float32 break test's edge."""
    m_ref, mind, ev_ref = oracle.search_step(colors, c_prev, m_prev)
    bad = np.flatnonzero(m_gpu != m_ref)
    assert len(bad) == 0, (t, len(bad), bad[:5])
    c_ref = oracle.update_step(colors, counts, n_pix, m_gpu, c_prev)
    assert np.array_equal(c_gpu64, c_ref), (t, np.abs(c_gpu64 - c_ref).max())
    assert np.array_equal(c_gpu32, c_ref.astype(np.float32)), t
    sse_ref = oracle.weighted_sse(counts, n_pix, mind)
    # float64 sums in another order: 1.8e-12 relative measured over 1.9M colors
    assert sse_gpu == pytest.approx(sse_ref, rel=SUM_RTOL), (t, sse_gpu, sse_ref)
    if check_evals:
        # the float32 scan's count; it can differ from the float64 scan's
        # only where the break test sits on the edge
        assert abs(int(ev_gpu) - ev_ref) <= max(2, 1e-3 * ev_ref), (t, ev_gpu, ev_ref)
    return dict(t=t, evals_gpu=int(ev_gpu), evals_ref=ev_ref)


def _lockstep(img, K, seed, iters, full=False, check_evals=True, indices=None, palette=None):
    wsm = _wsm()
    g, col, cnt, colors, counts = _gpu_table(img)
    n_pix = img.shape[0] * img.shape[1]
    if palette is not None:
        pal = torch.from_numpy(np.ascontiguousarray(palette, dtype=np.float32)).cuda()
    else:
        idx = synth.init_indices(seed, len(colors), K) if indices is None else indices
        pal = wsm.palette_from_indices(col, idx)
    m_prev = np.zeros(len(colors), dtype=np.uint8)
    c_prev = pal.cpu().numpy().astype(np.float64)
    stats = []
    st = None
    for t in range(1, iters + 1):
        st = wsm.init(col, cnt, n_pix, pal, reuse=st)
        if full:
            st.iterate_full(t, 0.0)
        else:
            st.iterate(t, 0.0)
        info = st.info()
        assert info["iters"] == t and info["err"] == 0
        if info["converged"]:
            break
        m_gpu = st.membership().cpu().numpy()
        c64 = st.palette64().cpu().numpy()
        c32 = st.palette().cpu().numpy()
        sse_gpu, ev_gpu = st.history()
        s = _check_step(colors, counts, n_pix, m_prev, c_prev, m_gpu, c64, c32, sse_gpu[-1],
                        ev_gpu[-1], check_evals and not full, t)
        stats.append(s)
        m_prev, c_prev = m_gpu, c64
    return stats


@pytest.mark.parametrize("seed", [0, 1])
def test_lockstep_small_k32(seed):
    img = synth.workload_image("small", seed)
    _say("lockstep small", seed, "K=32")
    stats = _lockstep(img, 32, seed, 12)
    print(stats[-1])


@pytest.mark.parametrize("K", [16, 33, 47, 64, 256])
def test_lockstep_medium(K):
    img = synth.workload_image("medium", 0)
    _say("lockstep medium seed 0 K", K)
    stats = _lockstep(img, K, 0, 5)
    print(stats[-1])


@pytest.mark.parametrize("K", [2, 17, 31, 33, 63, 65, 66, 97, 127, 128, 200, 255])
def test_lockstep_k_around_kernel_switches(K):
    # K <= 32: one fused launch with lane scans (K = 17: rows of 16 entries);
    # K >= 33: rows + per-lane scans of the first 16 entries, then flattened
    # scans over 64-entry row heads; up to K = 65 the head holds the whole
    # row, from K = 66 on a scan can go past it and is deferred.  Odd K give
    # rows whose length is not a multiple of the scan batch or of the head.
    img = synth.workload_image("medium", 1)
    _say("lockstep medium seed 1 K", K)
    stats = _lockstep(img, K, 1, 4)
    print(stats[-1])


@pytest.mark.parametrize("K", [128, 256])
def test_lockstep_small_many_centers(K):
    """K = 128 is the first K whose search defers long scans; on the small
    image (about 28k colors) every block is short."""
    img = synth.workload_image("small", 1)
    _say("lockstep small seed 1 K", K)
    stats = _lockstep(img, K, 1, 5)
    print(stats[-1])


def test_lockstep_tiny_table_k256():
    """A table of a few hundred colors with K = 256: two search blocks, rows
    of 255 entries, most clusters holding one or two colors."""
    rng = np.random.default_rng(11)
    img = rng.integers(0, 256, size=(24, 20, 3)).astype(np.uint8)
    img[:, :4] = img[:1, :4]          # some repeated colors
    _say("lockstep tiny random image 24x20 K 256")
    stats = _lockstep(img, 256, 5, 4)
    print(stats[-1])


def _fractional_duplicates(colors, K, seed):
    """K centers in identical pairs at fractional positions near sampled
    colors: every color near a pair ties between its two members, so the
    float32 choice is never certified there and float64 decides."""
    rng = np.random.default_rng(seed)
    base = synth.unpack_keys_to_palette(colors[synth.init_indices(seed, len(colors), K // 2)])
    base = np.clip(base + rng.choice([-0.375, 0.25, 0.625], size=base.shape), 0, 255)
    return np.repeat(base, 2, axis=0).astype(np.float32)


@pytest.mark.parametrize("name,K", [("small", 32), ("medium", 64), ("medium", 256)])
def test_lockstep_duplicate_fractional_centers(name, K):
    img = synth.workload_image(name, 0)
    colors, _ = oracle.reduce_colors(img)
    _say("lockstep", name, "K", K, "pairs of identical fractional centers")
    stats = _lockstep(img, K, 0, 4, palette=_fractional_duplicates(colors, K, 0))
    print(stats[-1])


@pytest.mark.parametrize("K", [32, 200])
def test_lockstep_palette_outside_the_cube(K):
    """A center outside [0, 255]^3 voids the float32 error bound: every
    choice is then made in float64, and the results still match."""
    img = synth.workload_image("medium", 2)
    colors, _ = oracle.reduce_colors(img)
    pal = synth.unpack_keys_to_palette(colors[synth.init_indices(2, len(colors), K)])
    pal = pal.astype(np.float32)
    pal[1] = (300.0, -20.0, 128.5)
    _say("lockstep medium seed 2 K", K, "one center outside the color cube")
    stats = _lockstep(img, K, 2, 4, palette=pal)
    print(stats[-1])


def test_lockstep_full_search_comparator():
    img = synth.workload_image("small", 2)
    _say("lockstep small seed 2 K=32 full search")
    _lockstep(img, 32, 2, 6, full=True)


@pytest.mark.parametrize("K,size", [(64, 256), (256, 256), (64, 1024), (256, 1024)])
def test_sort_means_on_raw_pixels_equals_weighted_colors(K, size):
    """Sort-means run directly on every pixel (weight 1) gives bit-identical
    palettes to sort-means on the weighted unique colors (the exact integer
    sums make Sec. 2's data reduction and weighting exact on the GPU too);
    at 1024x1024 each block holds several chunks of pixels."""
    wsm = _wsm()
    if size == 256:
        img = synth.workload_image("small", 0)
    else:
        img = synth.sinusoid_field_image(1, size, size)
    _say("sort-means on pixels vs colors", img.shape, "K", K)
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    n_pix = img.shape[0] * img.shape[1]
    pal = wsm.palette_from_indices(col, synth.init_indices(2, col.numel(), K))
    a = wsm.init(col, cnt, n_pix, pal)
    a.iterate(8, 0.0)
    b = wsm.init_pixels(g, pal)
    b.iterate(8, 0.0)
    assert torch.equal(a.palette64().cpu(), b.palette64().cpu())
    np.testing.assert_allclose(a.history()[0], b.history()[0], rtol=SUM_RTOL)


# ---------------------------------------------------------------------------
# End-to-end against the free-running oracle (Alg. 2 with the Sec. 3.2 stop),
# and the three GPU forms against each other.

def _run_gpu(img, K, seed, max_iters=50, eps=1e-4, mode="sm"):
    wsm = _wsm()
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    n_pix = img.shape[0] * img.shape[1]
    idx = synth.init_indices(seed, col.numel(), K)
    pal = wsm.palette_from_indices(col, idx)
    if mode == "pixels":
        st = wsm.init_pixels(g, pal)
        st.iterate_full(max_iters, eps)
    else:
        st = wsm.init(col, cnt, n_pix, pal)
        if mode == "sm":
            st.iterate(max_iters, eps)
        else:
            st.iterate_full(max_iters, eps)
    return st, col, cnt, pal


def _end_to_end(name, seed, K, max_iters, eps):
    """A whole GPU run (one call) against a whole oracle run from the same
    palette: same iteration count and stop, same memberships, bit-equal
    float64 centers, SSE histories to float64 rounding, and the final map's
    indices and MSE (the benchmark spec bound: 1e-5 relative; here to rounding)."""
    wsm = _wsm()
    img = synth.workload_image(name, seed)
    n_pix = img.shape[0] * img.shape[1]
    _say("e2e", name, seed, "K", K, "eps", eps, "max", max_iters)
    st, col, cnt, pal = _run_gpu(img, K, seed, max_iters, eps)
    colors, counts = _u32(col), _u32(cnt)
    ref = oracle.wsm(colors, counts, n_pix, pal.cpu().numpy().astype(np.float64), max_iters, eps)
    info = st.info()
    sse, ev = st.history()
    print(dict(gpu_iters=info["iters"], ref_iters=ref["iters"], converged=info["converged"]))
    assert info["iters"] == ref["iters"] and info["converged"] == ref["converged"]
    assert np.array_equal(st.membership().cpu().numpy(), ref["m"])
    assert np.array_equal(st.palette64().cpu().numpy(), ref["centers"])
    np.testing.assert_allclose(sse, ref["sse"], rtol=SUM_RTOL)
    assert (np.abs(ev - ref["evals"]) <= np.maximum(2, 1e-3 * ref["evals"])).all()
    g = _gpu_img(img)
    idx, rgb_out, mse = wsm.map_pixels(st, g, want_rgb=True)
    ref_idx, mse_ref = oracle.map_pixels(img, colors, ref["m"], ref["centers"])
    assert np.array_equal(idx.cpu().numpy(), ref_idx)
    assert float(mse.item()) == pytest.approx(mse_ref, rel=SUM_RTOL)
    assert abs(float(mse.item()) - mse_ref) <= MSE_RTOL * mse_ref
    rp = np.clip(np.rint(ref["centers"]), 0, 255).astype(np.uint8)
    assert np.array_equal(rgb_out.cpu().numpy().reshape(-1, 3), rp[ref_idx])
    return info, ref


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_end_to_end_small_vs_oracle(seed):
    """WSM-C (eps 1e-4, at most 50 iterations) on the 256x256 workload."""
    _end_to_end("small", seed, 32, 50, 1e-4)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_end_to_end_small_eps_stop_fires(seed):
    """eps = 1e-3: the relative-change rule of Sec. 3.2 stops the run before
    the cap (after 17 to 40 iterations on these seeds)."""
    info, ref = _end_to_end("small", seed, 32, 50, 1e-3)
    assert info["converged"] and info["iters"] < 50


def test_end_to_end_small_fixed_ten_iterations():
    """The paper's fixed variant: exactly 10 iterations (eps = 0)."""
    info, _ = _end_to_end("small", 0, 32, 10, 0.0)
    assert info["iters"] == 10 and not info["converged"]


@pytest.mark.parametrize("K", [16, 64, 256])
def test_end_to_end_medium_vs_oracle(K):
    """The 512x512 workload, K 16 / 64 / 256, 50 iterations at eps 1e-4."""
    _end_to_end("medium", 0, K, 50, 1e-4)


@pytest.mark.parametrize("K", [16, 64, 256])
def test_end_to_end_medium_eps_stop_fires(K):
    info, _ = _end_to_end("medium", 0, K, 50, 1e-3)
    assert info["converged"] and info["iters"] < 50


@pytest.mark.parametrize("name,seed,K", [("small", 0, 32), ("medium", 1, 64), ("medium", 1, 128),
                                         ("medium", 2, 200), ("medium", 0, 256)])
def test_pruned_full_and_pixel_kmeans_identical(name, seed, K):
    img = synth.workload_image(name, seed)
    _say("three GPU forms", name, seed, K)
    a, *_ = _run_gpu(img, K, seed, 30, 1e-4, "sm")
    b, *_ = _run_gpu(img, K, seed, 30, 1e-4, "full")
    c, *_ = _run_gpu(img, K, seed, 30, 1e-4, "pixels")
    pa, pb, pc = (s.palette64().cpu().numpy() for s in (a, b, c))
    assert np.array_equal(pa, pb)
    assert np.array_equal(pa, pc)
    assert np.array_equal(a.membership().cpu().numpy(), b.membership().cpu().numpy())
    ia, ib, ic = a.info(), b.info(), c.info()
    assert ia["iters"] == ib["iters"] == ic["iters"]
    sa, ea = a.history()
    sb, eb = b.history()
    np.testing.assert_allclose(sa, sb, rtol=SUM_RTOL)
    assert (ea <= eb).all() and ea[-1] < eb[-1]


@pytest.mark.parametrize("K", [24, 256])
def test_resume_equals_single_call(K):
    img = synth.workload_image("small", 1)
    _say("resume 4+6 vs 10, small seed 1 K", K)
    a, *_ = _run_gpu(img, K, 1, 10, 0.0)
    wsm = _wsm()
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    pal = wsm.palette_from_indices(col, synth.init_indices(1, col.numel(), K))
    b = wsm.init(col, cnt, img.shape[0] * img.shape[1], pal)
    b.iterate(4, 0.0)
    assert b.info()["iters"] == 4 and not b.info()["converged"]
    b.iterate(1, 0.0)
    b.iterate(5, 0.0)
    assert np.array_equal(a.palette64().cpu().numpy(), b.palette64().cpu().numpy())
    assert np.array_equal(a.membership().cpu().numpy(), b.membership().cpu().numpy())
    assert a.info() == b.info()
    np.testing.assert_allclose(a.history()[0], b.history()[0], rtol=SUM_RTOL)


@pytest.mark.parametrize("K", [16, 64, 256])
def test_caller_grid_gives_the_same_results(K):
    """A caller-chosen search grid (wsm_problem.grid: fewer blocks, as when
    several K share the GPU on streams of their own, or more) gives the
    default grid's memberships, centers, evaluation counts and record; the
    SSE history within SUM_RTOL (its terms added in another order)."""
    wsm = _wsm()
    img = synth.workload_image("medium", 0)
    _say("caller grid medium seed 0 K", K)
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    n_pix = img.shape[0] * img.shape[1]
    pal = wsm.palette_from_indices(col, synth.init_indices(0, col.numel(), K))
    ref = wsm.init(col, cnt, n_pix, pal)
    ref.iterate(12, 1e-4)
    for grid in (1, 37, 96, 700):
        st = wsm.init(col, cnt, n_pix, pal)
        st.grid = grid
        st.iterate(12, 1e-4)
        assert np.array_equal(st.membership().cpu().numpy(), ref.membership().cpu().numpy()), grid
        assert np.array_equal(st.palette64().cpu().numpy(), ref.palette64().cpu().numpy()), grid
        assert st.info() == ref.info(), grid
        assert np.array_equal(st.history()[1], ref.history()[1]), grid
        np.testing.assert_allclose(st.history()[0], ref.history()[0], rtol=SUM_RTOL)
    with pytest.raises(wsm.WsmError):
        st.grid = 0
    with pytest.raises(wsm.WsmError):
        st.grid = 2049


@pytest.mark.parametrize("K", [16, 64, 256])
def test_unpacked_sums_equal_packed(K):
    # Counts x 300 push 255 * n_pixels past 2^32, so the centroid sums take
    # four u64 per center instead of two packed ones.  Scaling every weight
    # by the same factor leaves each center (sum c x / sum c, exact integer
    # sums) unchanged, so memberships, palettes and evaluation counts must be
    # identical to the unscaled run.
    wsm = _wsm()
    img = synth.workload_image("medium", 0)
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    n = img.shape[0] * img.shape[1]
    scale = 300
    assert 255 * n * scale >= 1 << 32 > 255 * n
    _say("unpacked sums, medium seed 0, counts x", scale, "K", K)
    pal = wsm.palette_from_indices(col, synth.init_indices(0, col.numel(), K))
    a = wsm.init(col, cnt, n, pal)
    a.iterate(6, 0.0)
    b = wsm.init(col, cnt * scale, n * scale, pal)
    b.iterate(6, 0.0)
    assert np.array_equal(a.palette64().cpu().numpy(), b.palette64().cpu().numpy())
    assert np.array_equal(a.membership().cpu().numpy(), b.membership().cpu().numpy())
    sa, ea = a.history()
    sb, eb = b.history()
    np.testing.assert_array_equal(ea, eb)
    np.testing.assert_allclose(sb, sa, rtol=SUM_RTOL)
    assert a.info()["iters"] == b.info()["iters"] == 6


# ---------------------------------------------------------------------------
# Degenerate cases.

def test_k1_and_exact_palette():
    wsm = _wsm()
    img = synth.workload_image("small", 3)
    _say("K=1 small seed 3")
    st, col, cnt, pal = _run_gpu(img, 1, 3, 10, 1e-4)
    px = img.reshape(-1, 3).astype(np.float64)
    np.testing.assert_allclose(st.palette().cpu().numpy()[0], px.mean(0), atol=CENTER_TOL)
    assert st.info()["iters"] == 3 and st.info()["converged"]
    idx, _, mse = wsm.map_pixels(st, _gpu_img(img))
    assert (idx.cpu().numpy() == 0).all()
    assert float(mse.item()) == pytest.approx(px.var(0).sum(), rel=MSE_RTOL)
    # an image of exactly K colors started from those colors: zero error at t=1
    rng = np.random.default_rng(4)
    palc = np.unique(rng.integers(0, 256, size=(40, 3)), axis=0).astype(np.uint8)
    K = palc.shape[0]
    img2 = palc[rng.integers(0, K, size=(64, 50))]
    _say("exact palette K", K)
    st2, col2, cnt2, pal2 = _run_gpu(img2, K, 0, 50, 1e-4)
    assert st2.info() == dict(iters=1, converged=True, err=0)
    idx2, rgb2, mse2 = wsm.map_pixels(st2, _gpu_img(img2), want_rgb=True)
    assert float(mse2.item()) == 0.0
    assert np.array_equal(rgb2.cpu().numpy(), img2)


def test_empty_cluster_keeps_center():
    wsm = _wsm()
    img = np.zeros((8, 8, 3), dtype=np.uint8)
    img[:, 4:6] = (10, 0, 0)
    img[:, 6:] = (20, 0, 0)
    _say("empty cluster, 3 colors, 3 centers, one far away")
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    init = np.array([[0, 0, 0], [200, 200, 200], [10, 0, 0]], dtype=np.float32)
    pal = torch.from_numpy(init).cuda()
    st = wsm.init(col, cnt, 64, pal)
    st.iterate(5, 1e-4)
    p = st.palette().cpu().numpy()
    np.testing.assert_array_equal(p[1], init[1])
    ref = oracle.wsm(_u32(col), _u32(cnt), 64, init.astype(np.float64), 5, 1e-4)
    assert np.array_equal(st.palette64().cpu().numpy(), ref["centers"])
    assert st.info()["iters"] == ref["iters"]
    np.testing.assert_allclose(st.history()[0], ref["sse"], rtol=SUM_RTOL)


def test_invalid_arguments_raise():
    wsm = _wsm()
    img = synth.workload_image("small", 0)
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    _say("invalid arguments")
    pal = torch.zeros((257, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(wsm.WsmError):
        wsm.init(col, cnt, 65536, pal)
    few = torch.zeros((3, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(wsm.WsmError):
        wsm.init(col[:2], cnt[:2], 65536, few)
    st = wsm.init(col, cnt, 65536, wsm.palette_from_indices(col, [0, 1, 2]))
    with pytest.raises(wsm.WsmError):
        st.iterate(0, 1e-4)
    with pytest.raises(wsm.WsmError):
        st.iterate(5, float("nan"))
    with pytest.raises(wsm.WsmError):
        st.iterate(5, -1.0)


# ---------------------------------------------------------------------------
# Pixel mapping.

@pytest.mark.parametrize("name,seed,K", [("small", 0, 32), ("medium", 0, 64), ("small", 1, 128),
                                         ("medium", 2, 256)])
def test_map_against_oracle(name, seed, K):
    wsm = _wsm()
    img = synth.workload_image(name, seed)
    _say("map", name, seed, K)
    st, col, cnt, pal = _run_gpu(img, K, seed, 8, 1e-4)
    idx, rgb_out, mse = wsm.map_pixels(st, _gpu_img(img), want_rgb=True)
    colors = _u32(col)
    m = st.membership().cpu().numpy()
    c = st.palette64().cpu().numpy()
    ref_idx, ref_mse = oracle.map_pixels(img, colors, m, c)
    gi = idx.cpu().numpy()
    assert np.array_equal(gi, ref_idx)
    assert float(mse.item()) == pytest.approx(ref_mse, rel=SUM_RTOL)
    rp = np.clip(np.rint(c), 0, 255).astype(np.uint8)
    assert np.array_equal(rgb_out.cpu().numpy().reshape(-1, 3), rp[gi])


def _pixel_color_index(img, colors):
    """Index of each pixel's color in the ascending table."""
    px = img.reshape(-1, 3).astype(np.uint32)
    keys = (px[:, 0] << 16) | (px[:, 1] << 8) | px[:, 2]
    pos = np.searchsorted(colors, keys)
    assert np.array_equal(colors[pos], keys)
    return pos


def _check_map_all_pixels(img, colors, counts, m, c, idx_gpu, mse_gpu):
    """Every pixel's index against the oracle's assignment of its color
    (all K centers, key (d, k != m_i, k)), through the color key."""
    n_pix = img.shape[0] * img.shape[1]
    ci, cmse = oracle.assign_colors(colors, counts, n_pix, m, c)
    pos = _pixel_color_index(img, colors)
    assert np.array_equal(idx_gpu, ci[pos])
    assert mse_gpu == pytest.approx(cmse, rel=SUM_RTOL)


# ---------------------------------------------------------------------------
# Full-size image (4096x4096, ~1.9M unique colors, K=256): lock-step on every
# color and the map on every pixel.

def test_large_lockstep_and_map():
    wsm = _wsm()
    img = synth.workload_image("large", 0)
    _say("large 4096x4096 seed 0 K=256: 3 lock-step iterations (all colors) + map (all pixels)")
    stats = _lockstep(img, 256, 0, 3)
    print(stats)
    st, col, cnt, pal = _run_gpu(img, 256, 0, 3, 1e-4)
    idx, _, mse = wsm.map_pixels(st, _gpu_img(img))
    _check_map_all_pixels(img, _u32(col), _u32(cnt), st.membership().cpu().numpy(),
                          st.palette64().cpu().numpy(), idx.cpu().numpy(), float(mse.item()))


def test_identical_centers_fill_the_deferral_queue():
    # All 256 centers start at one color.  The first step keeps every color
    # at center 0 (all distances tie); its update moves center 0 and leaves
    # the other 255 where they were, so in the second step every row is a
    # run of equal distances and nearly every scan covers its whole row.  At
    # 4096x4096 (about 7,450 colors per search block) that is more long scans
    # than a block's deferral queue holds, so both the deferred finish and
    # the in-place continuation run, in the search and in the pixel map.
    wsm = _wsm()
    img = synth.workload_image("large", 0)
    _say("large 4096x4096 seed 0 K=256, all centers at one color: 2 steps + map (all pixels)")
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    colors, counts = _u32(col), _u32(cnt)
    n_pix = img.shape[0] * img.shape[1]
    K = 256
    one_idx = [len(colors) // 2] * K
    stats = _lockstep(img, K, 0, 2, indices=one_idx)
    print(stats)
    assert stats[-1]["evals_ref"] > 100 * len(colors)  # most scans run over the whole row
    pal = wsm.palette_from_indices(col, one_idx)
    two = wsm.init(col, cnt, n_pix, pal)
    two.iterate(2, 0.0)
    m2 = two.membership().cpu().numpy()
    idx, _, mse = wsm.map_pixels(two, g)
    _check_map_all_pixels(img, colors, counts, m2, two.palette64().cpu().numpy(),
                          idx.cpu().numpy(), float(mse.item()))


# ---------------------------------------------------------------------------
# Launch replay from caller-owned HIP graphs: bit-identical to direct launches.

@pytest.mark.parametrize("K,full", [(32, False), (256, False), (64, True)])
def test_graph_handle_matches_direct_launches(K, full):
    """The recorded launch sequence of an iterate call, replayed several
    times on a re-initialised state with other eager work and host
    synchronisations in between, gives exactly the palette, memberships,
    evaluation counts and iteration record of direct launches, and their SSE
    history within SUM_RTOL (deferred scans add their SSE terms in queue
    order) (K = 32 runs the single-launch step, K = 256 the rows + search
    pair, full the comparator)."""
    wsm = _wsm()
    _say("graph handle medium seed 0 K", K, "full" if full else "sm", "12 iterations, 4 replays")
    img = synth.workload_image("medium", 0)
    g = _gpu_img(img)
    col, cnt = wsm.reduce_colors(g)
    n_pix = img.shape[0] * img.shape[1]
    pal = wsm.palette_from_indices(col, synth.init_indices(1, col.numel(), K))
    ref = wsm.init(col, cnt, n_pix, pal)
    if full:
        ref.iterate_full(12, 0.0)
    else:
        ref.iterate(12, 0.0)
    ref_pal = ref.palette64().cpu()
    ref_m = ref.membership().cpu()
    ref_sse, ref_ev = ref.history()
    st = wsm.init(col, cnt, n_pix, pal)
    graph = st.graph(12, 0.0, full=full)
    try:
        for rep in range(4):
            st = wsm.init(col, cnt, n_pix, pal, reuse=st)
            graph.launch()
            wsm.map_pixels(st, g)          # other work on the stream between replays
            torch.cuda.synchronize()
            sse, ev = st.history()
            assert torch.equal(st.palette64().cpu(), ref_pal), rep
            assert torch.equal(st.membership().cpu(), ref_m), rep
            assert np.array_equal(ev, ref_ev), rep
            np.testing.assert_allclose(sse, ref_sse, rtol=SUM_RTOL)
            assert st.info() == ref.info(), rep
    finally:
        graph.close()

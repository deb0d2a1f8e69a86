"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value comes from
a library routine (numpy.unique), an exact-rational brute force written in
tests/exact_ref.py, a closed form, an invariant, or a hand-worked example in
tests/golden/.  Sizes are small so the CPU suite stays fast.
"""

from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from exact_ref import lloyd, nearest, sqd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _keys(rgb):
    rgb = rgb.reshape(-1, 3).astype(np.uint32)
    return (rgb[:, 0] << 16) | (rgb[:, 1] << 8) | rgb[:, 2]


def _pack(cols):
    cols = np.asarray(cols, dtype=np.uint32)
    return (cols[:, 0] << 16) | (cols[:, 1] << 8) | cols[:, 2]


def _F(s):
    return Fraction(s)


# ---------------------------------------------------------------------------
# Data reduction (Sec. 2, data sampling): a library routine fixes the result.

@pytest.mark.parametrize("seed", [0, 1])
def test_reduce_matches_numpy_unique(seed):
    img = synth.workload_image("small", seed)
    col, cnt = oracle.reduce_colors(img)
    ref_k, ref_c = np.unique(_keys(img), return_counts=True)
    assert np.array_equal(col, ref_k.astype(np.uint32))
    assert np.array_equal(cnt, ref_c.astype(np.uint32))
    assert int(cnt.sum()) == img.shape[0] * img.shape[1]


def test_reduce_hand_cases():
    const = np.full((7, 5, 3), 77, dtype=np.uint8)
    col, cnt = oracle.reduce_colors(const)
    assert col.tolist() == [(77 << 16) | (77 << 8) | 77] and cnt.tolist() == [35]
    board = np.zeros((8, 8, 3), dtype=np.uint8)
    board[(np.add.outer(np.arange(8), np.arange(8)) % 2) == 1] = (255, 0, 1)
    col, cnt = oracle.reduce_colors(board)
    assert col.tolist() == [0, (255 << 16) | 1] and cnt.tolist() == [32, 32]
    extremes = np.array([[[255, 255, 255], [0, 0, 0], [255, 255, 255]]], dtype=np.uint8)
    col, cnt = oracle.reduce_colors(extremes)
    assert col.tolist() == [0, 0xFFFFFF] and cnt.tolist() == [1, 2]


def test_reduce_random_noise_matches_numpy_unique():
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(300, 200, 3), dtype=np.uint8)
    col, cnt = oracle.reduce_colors(img)
    ref_k, ref_c = np.unique(_keys(img), return_counts=True)
    assert np.array_equal(col, ref_k) and np.array_equal(cnt, ref_c)


# ---------------------------------------------------------------------------
# Hand-worked examples (tests/golden/worked_examples.json).

def _golden():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_golden_values_rederived_exactly(ex):
    """The fixture itself is re-derived by the exact brute force."""
    pts = [tuple(c) for c in ex["colors"]]
    hist, conv = lloyd(pts, ex["counts"], ex["init"], ex["max_iters"], ex["eps"])
    assert len(hist) == ex["iters"] and conv == ex["converged"]
    for t, rec in enumerate(hist):
        assert rec["sse"] == _F(ex["sse"][t])
        assert rec["m"] == ex["m_per_iter"][t]
        assert rec["centers"] == [tuple(_F(v) for v in c) for c in ex["centers_per_iter"][t]]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_oracle_reproduces_worked_example(ex):
    colors = _pack(ex["colors"])
    counts = np.array(ex["counts"], dtype=np.uint32)
    n_pix = int(counts.sum())
    r = oracle.wsm(colors, counts, n_pix, np.array(ex["init"], float),
                   ex["max_iters"], ex["eps"])
    assert r["iters"] == ex["iters"] and r["converged"] == ex["converged"]
    np.testing.assert_allclose(r["sse"], [float(_F(s)) for s in ex["sse"]], rtol=1e-13, atol=0)
    assert r["evals"].tolist() == ex["evals"]
    assert r["m"].tolist() == ex["m_per_iter"][-1]
    fin = np.array([[float(_F(v)) for v in c] for c in ex["centers_per_iter"][-1]])
    np.testing.assert_allclose(r["centers"], fin, rtol=1e-13, atol=1e-13)


def test_literal_tie_rule_mirrors_ex2():
    ex = [e for e in _golden() if e["name"].startswith("EX2")][0]
    colors = _pack(ex["colors"])
    counts = np.array(ex["counts"], dtype=np.uint32)
    r = oracle.wsm(colors, counts, 3, np.array(ex["init"], float), 50, 1e-4,
                   literal=True)
    fin = np.array([[float(_F(v)) for v in c] for c in ex["literal_final_centers"]])
    np.testing.assert_allclose(r["centers"], fin, atol=1e-13)
    assert r["m"].tolist() == ex["literal_m_final"]
    np.testing.assert_allclose(r["sse"], [float(_F(s)) for s in ex["sse"]], rtol=1e-13)
    assert r["evals"].tolist() == ex["evals"]


# ---------------------------------------------------------------------------
# Sort-means pruning never changes the assignment: exact brute force on
# tie-rich small grids with dyadic centers (all distances exact in float64).

@pytest.mark.parametrize("seed", range(40))
def test_search_step_equals_exact_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    K = int(rng.integers(1, 9))
    n = int(rng.integers(1, 40))
    span = int(rng.choice([3, 5, 9]))
    pts = rng.integers(0, span, size=(n, 3))
    colors = np.unique(_pack(pts))
    pts = np.stack([(colors >> 16) & 255, (colors >> 8) & 255, colors & 255], 1)
    # centers on a quarter-unit grid, duplicates allowed: many exact ties
    cen = rng.integers(0, 4 * span, size=(K, 3)) / 4.0
    if K > 2 and seed % 3 == 0:
        cen[1] = cen[0]
    m_prev = rng.integers(0, K, size=colors.shape[0]).astype(np.uint8)
    m_new, mind, ev = oracle.search_step(colors, cen, m_prev, prune=True)
    m_full, mind_full, ev_full = oracle.search_step(colors, cen, m_prev, prune=False)
    assert ev_full == colors.shape[0] * K
    assert ev <= ev_full
    cq = [tuple(Fraction(float(v)) for v in c) for c in cen]
    for i in range(colors.shape[0]):
        k, d = nearest(tuple(int(v) for v in pts[i]), cq, int(m_prev[i]))
        assert int(m_new[i]) == k, (i, k, int(m_new[i]))
        assert int(m_full[i]) == k
        assert Fraction(float(mind[i])) == d


@pytest.mark.parametrize("seed", range(12))
def test_wsm_trajectory_equals_exact_lloyd(seed):
    """Whole Alg. 2 runs equal exact weighted Lloyd on the same points."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 40))
    K = int(rng.integers(1, min(n, 8) + 1))
    pts = rng.integers(0, 256, size=(n, 3))
    colors = np.unique(_pack(pts))
    n = colors.shape[0]
    K = min(K, n)
    pts = [((int(c) >> 16) & 255, (int(c) >> 8) & 255, int(c) & 255) for c in colors]
    counts = rng.integers(1, 20, size=n).astype(np.uint32)
    init_idx = synth.init_indices(seed, n, K)
    init = np.array([pts[i] for i in init_idx], dtype=float)
    r = oracle.wsm(colors, counts, int(counts.sum()), init, 30, 1e-4)
    hist, conv = lloyd(pts, [int(c) for c in counts], [tuple(p) for p in init], 30, 1e-4)
    assert r["iters"] == len(hist) and r["converged"] == conv
    for t, rec in enumerate(hist):
        assert r["sse"][t] == pytest.approx(float(rec["sse"]), rel=1e-12, abs=1e-12)
    assert r["m"].tolist() == hist[-1]["m"]
    # the centers come from exact integer sums with one division: they are the
    # correctly rounded exact weighted means, bit for bit
    exact = np.array([[float(v) for v in c] for c in hist[-1]["centers"]])
    np.testing.assert_array_equal(r["centers"], exact)


def test_wsm_equals_kmeans_on_pixels():
    """Data reduction + weighting is exact: Alg. 2 on unique colors equals
    Alg. 1 on all pixels (and an exact Lloyd on the pixel multiset)."""
    rng = np.random.default_rng(7)
    img = rng.integers(0, 6, size=(9, 7, 3), dtype=np.uint8) * 40
    col, cnt = oracle.reduce_colors(img)
    K = 4
    init = synth.unpack_keys_to_palette(col[synth.init_indices(3, len(col), K)]).astype(float)
    r = oracle.wsm(col, cnt, 63, init, 20, 1e-4)
    km = oracle.kmeans_pixels(img, init, 20, 1e-4)
    assert r["iters"] == km["iters"]
    np.testing.assert_allclose(r["sse"], km["sse"], rtol=1e-12)
    # both compute each center as (exact integer sum) / (exact count)
    np.testing.assert_array_equal(r["centers"], km["centers"])
    pix = [tuple(int(v) for v in p) for p in img.reshape(-1, 3)]
    hist, conv = lloyd(pix, [1] * len(pix), [tuple(p) for p in init], 20, 1e-4)
    assert len(hist) == r["iters"]
    # per-pixel memberships of the exact run equal the per-color ones
    key_to_i = {int(c): i for i, c in enumerate(col)}
    m_pix = [int(r["m"][key_to_i[(p[0] << 16) | (p[1] << 8) | p[2]]]) for p in pix]
    assert m_pix == hist[-1]["m"]
    assert km["m"].tolist() == hist[-1]["m"]


# ---------------------------------------------------------------------------
# Invariants and closed forms.

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sse_is_non_increasing(seed):
    img = synth.workload_image("small", seed)
    col, cnt = oracle.reduce_colors(img)
    init = synth.unpack_keys_to_palette(col[synth.init_indices(seed, len(col), 32)])
    r = oracle.wsm(col, cnt, img.shape[0] * img.shape[1], init, 40, 0.0)
    s = r["sse"]
    assert np.all(s[1:] <= s[:-1] * (1 + 1e-12))
    # the first iteration is a full search from center 0: pruning only helps later
    assert r["evals"][0] <= 32 * len(col)
    assert r["evals"][-1] < 8 * len(col)


def test_k1_is_mean_color_and_total_variance():
    img = synth.workload_image("small", 2)
    col, cnt = oracle.reduce_colors(img)
    init = synth.unpack_keys_to_palette(col[:1])
    r = oracle.wsm(col, cnt, img.shape[0] * img.shape[1], init, 10, 1e-4)
    px = img.reshape(-1, 3).astype(np.float64)
    np.testing.assert_allclose(r["centers"][0], px.mean(0), rtol=1e-12)
    # iteration 2 measures the mean palette: SSE = sum of channel variances
    np.testing.assert_allclose(r["sse"][1], px.var(0).sum(), rtol=1e-10)
    assert r["iters"] == 3 and r["converged"]
    idx, mse = oracle.map_pixels(img, col, r["m"], r["centers"])
    assert np.all(idx == 0)
    np.testing.assert_allclose(mse, px.var(0).sum(), rtol=1e-10)


def test_exactly_k_colors_reach_zero_error_in_one_iteration():
    rng = np.random.default_rng(11)
    pal = np.unique(rng.integers(0, 256, size=(12, 3)), axis=0).astype(np.uint8)
    K = pal.shape[0]
    img = pal[rng.integers(0, K, size=(30, 30))]
    col, cnt = oracle.reduce_colors(img)
    assert len(col) == K
    init = synth.unpack_keys_to_palette(col[synth.init_indices(0, K, K)])
    r = oracle.wsm(col, cnt, 900, init, 50, 1e-4)
    assert r["iters"] == 1 and r["converged"] and r["sse"][0] == 0.0
    idx, mse = oracle.map_pixels(img, col, r["m"], r["centers"])
    # each center is (count x) / count, exactly the color
    assert mse == 0.0
    np.testing.assert_allclose(r["centers"][idx], img.reshape(-1, 3).astype(float), rtol=1e-14)


def test_max_iters_exhaustion_is_not_convergence():
    img = synth.workload_image("small", 1)
    col, cnt = oracle.reduce_colors(img)
    init = synth.unpack_keys_to_palette(col[synth.init_indices(1, len(col), 16)])
    r = oracle.wsm(col, cnt, img.shape[0] * img.shape[1], init, 1, 0.0)
    assert r["iters"] == 1 and not r["converged"]


def test_empty_cluster_keeps_its_center():
    colors = _pack([[0, 0, 0], [1, 0, 0]])
    counts = np.array([1, 1], dtype=np.uint32)
    init = np.array([[0, 0, 0], [200, 200, 200], [1, 0, 0]], dtype=float)
    r = oracle.wsm(colors, counts, 2, init, 5, 1e-4)
    np.testing.assert_array_equal(r["centers"][1], [200, 200, 200])
    assert r["sse"][0] == 0.0 and r["iters"] == 1


# ---------------------------------------------------------------------------
# Pixel mapping and MSE / PSNR (Sec. 3.1).

@pytest.mark.parametrize("seed", range(6))
def test_map_equals_brute_force(seed):
    rng = np.random.default_rng(50 + seed)
    img = (rng.integers(0, 5, size=(11, 13, 3)) * 60).astype(np.uint8)
    col, cnt = oracle.reduce_colors(img)
    K = int(rng.integers(1, 7))
    cen = rng.integers(0, 9, size=(K, 3)) * 30.0  # integer centers: exact ties
    m = rng.integers(0, K, size=len(col)).astype(np.uint8)
    idx, mse = oracle.map_pixels(img, col, m, cen)
    key_to_i = {int(c): i for i, c in enumerate(col)}
    px = img.reshape(-1, 3)
    s = 0
    for p in range(px.shape[0]):
        x = tuple(int(v) for v in px[p])
        i = key_to_i[(x[0] << 16) | (x[1] << 8) | x[2]]
        k, d = nearest(x, [tuple(c) for c in cen], int(m[i]))
        assert int(idx[p]) == k
        s += d
    assert mse == pytest.approx(float(s) / px.shape[0], rel=1e-14)
    ci, cmse = oracle.assign_colors(col, cnt, px.shape[0], m, cen)
    assert cmse == pytest.approx(mse, rel=1e-12)
    assert np.array_equal(ci[[key_to_i[int(k)] for k in _keys(img)]], idx)


def test_psnr_closed_forms():
    assert oracle.psnr(255.0 ** 2) == pytest.approx(0.0, abs=1e-12)
    assert oracle.psnr(1.0) == pytest.approx(20 * np.log10(255.0), rel=1e-15)
    assert oracle.psnr(0.0) == float("inf")


def test_sq_distance_uses_all_three_channels():
    # one color per axis direction: a dropped or repeated channel changes a value
    colors = _pack([[3, 0, 0], [0, 4, 0], [0, 0, 12]])
    cen = np.array([[0.0, 0.0, 0.0]])
    m, mind, _ = oracle.search_step(colors, cen, np.zeros(3, np.uint8))
    assert mind.tolist() == [9.0, 16.0, 144.0]
    d, M = oracle.center_tables(np.array([[0, 0, 0], [1, 2, 2], [0, 0, 1]], float))
    assert d.tolist() == [[0, 9, 1], [9, 0, 6], [1, 6, 0]]
    assert M.tolist() == [[0, 2, 1], [1, 2, 0], [2, 0, 1]]


# ---------------------------------------------------------------------------
# Differentiable form: the distortion of Eq. 1 with frozen assignments and
# its gradients.  D is a quadratic in x and c, so a central difference in
# exact rational arithmetic equals the derivative exactly, for any step.

def _exact_distortion(x, m, c):
    n = len(x)
    return sum(sqd(x[p], c[m[p]]) for p in range(n)) / n


@pytest.mark.parametrize("seed", range(6))
def test_distortion_gradient_equals_exact_central_difference(seed):
    rng = np.random.default_rng(100 + seed)
    n, K = int(rng.integers(5, 30)), int(rng.integers(1, 6))
    x = rng.integers(0, 256, size=(n, 3)).astype(float) + rng.integers(0, 4, size=(n, 3)) / 4
    c = rng.integers(0, 256, size=(K, 3)).astype(float) + rng.integers(0, 8, size=(K, 3)) / 8
    m = rng.integers(0, K, size=n).astype(np.uint8)
    g = 0.75
    xq = [[Fraction(v) for v in row] for row in x]
    cq = [[Fraction(v) for v in row] for row in c]
    D = oracle.distortion(x, m, c)
    assert D == pytest.approx(float(_exact_distortion(xq, m, cq)), rel=1e-14)
    gx, gc = oracle.distortion_grad(x, m, c, g)
    h = Fraction(1, 1000)
    for (arr, grad, idx) in ((xq, gx, rng.integers(0, n, 4)), (cq, gc, rng.integers(0, K, 3))):
        for i in idx:
            for ch in range(3):
                orig = arr[i][ch]
                arr[i][ch] = orig + h
                up = _exact_distortion(xq, m, cq)
                arr[i][ch] = orig - h
                dn = _exact_distortion(xq, m, cq)
                arr[i][ch] = orig
                fd = Fraction(g) * (up - dn) / (2 * h)
                assert grad[i, ch] == pytest.approx(float(fd), rel=1e-12, abs=1e-12)


def test_distortion_gradient_vanishes_at_exact_centroids():
    """dD/dc_k is (2/N)(W_k c_k - S_k): zero when every center is the mean
    of its points (here exact in binary), and the per-cluster sums of dD/dx
    are minus dD/dc."""
    rng = np.random.default_rng(7)
    K = 5
    m = np.repeat(np.arange(K), 8).astype(np.uint8)
    x = rng.integers(0, 256, size=(len(m), 3)).astype(float)
    c = np.stack([x[m == k].mean(0) for k in range(K)])
    gx, gc = oracle.distortion_grad(x, m, c, 1.0)
    assert np.abs(gc).max() < 1e-12
    c2 = c + rng.uniform(-3, 3, size=c.shape)
    gx, gc = oracle.distortion_grad(x, m, c2, 1.0)
    for k in range(K):
        np.testing.assert_allclose(gx[m == k].sum(0), -gc[k], rtol=1e-12, atol=1e-12)


def test_distortion_at_nearest_assignment_is_the_map_mse():
    """With every pixel assigned to its nearest center, D is the pixel MSE
    that oracle_map reports (Sec. 3.1)."""
    img = synth.workload_image("small", 1)[:64, :64]
    col, cnt = oracle.reduce_colors(img)
    c = synth.unpack_keys_to_palette(col[synth.init_indices(1, len(col), 12)]).astype(float) + 0.3
    idx, mse = oracle.map_pixels(img, col, np.zeros(len(col), np.uint8), c)
    D = oracle.distortion(img.reshape(-1, 3).astype(float), idx, c)
    assert D == pytest.approx(mse, rel=1e-12)

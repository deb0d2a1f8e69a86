"""GPU parity of the differentiable form (wsm_distortion and its adjoint,
through the C ABI via the autograd binding) against the FP64 oracle and
against FP64 central finite differences of the true distortion.

Inputs: the 512x512 sinusoid-field workload (seeds 0..), cast to float32, as
the differentiable configuration does (K = 64); the forward pass is WSM on
each image, the assignment its pixel map.
"""

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


def _batch(seeds, size=512):
    imgs = [synth.sinusoid_field_image(s, size, size) for s in seeds]
    return np.stack(imgs).astype(np.float32)


def _forward(x_np, K, max_iters=50, eps=1e-4):
    wsm = _wsm()
    x = torch.from_numpy(x_np).cuda()
    pal, idx, states = wsm.quantize_batch(x, K, lambda n, k: synth.init_indices(7, n, k),
                                          max_iters, eps)
    return x, pal, idx, states


def _grads(x, pal, idx, g):
    wsm = _wsm()
    xr = x.clone().requires_grad_(True)
    pr = pal.clone().requires_grad_(True)
    d = wsm.distortion(xr, pr, idx)
    (d * torch.as_tensor(g, dtype=torch.float64, device=d.device)).sum().backward()
    return d.detach().cpu().numpy(), xr.grad.cpu().numpy(), pr.grad.cpu().numpy()


@pytest.mark.parametrize("shift", [0.0, 0.37])
def test_distortion_and_gradients_equal_the_oracle(shift):
    """D and both gradients against the oracle's float64 ones, for the
    palettes WSM returns (shift 0: near the centroids, where dD/dc is
    small) and the same palettes moved by 0.37 (dD/dc large)."""
    _say("adjoint vs oracle, batch of 3 512x512 images, K 64, palette shift", shift)
    x_np = _batch([0, 1, 2])
    x, pal, idx, _ = _forward(x_np, 64, 20, 1e-4)
    pal = (pal + shift).contiguous()
    g = np.array([1.0, -0.5, 2.0])
    d, gx, gc = _grads(x, pal, idx, g)
    pal_np = pal.cpu().numpy().astype(np.float64)
    idx_np = idx.cpu().numpy()
    for b in range(3):
        xb = x_np[b].reshape(-1, 3).astype(np.float64)
        d_ref = oracle.distortion(xb, idx_np[b], pal_np[b])
        # float64 sums in another order (the oracle's sequential sum of
        # 262k terms is itself up to ~1e-12 off the exactly rounded sum)
        assert d[b] == pytest.approx(d_ref, rel=SUM_RTOL)
        gx_ref, gc_ref = oracle.distortion_grad(xb, idx_np[b], pal_np[b], g[b])
        # float32 outputs of float64 values: within a float32 rounding
        np.testing.assert_allclose(gx[b].reshape(-1, 3), gx_ref, rtol=2 ** -23, atol=1e-30)
        tol = 2 ** -23 * np.abs(gc_ref) + 1e-12 * np.abs(gx_ref).sum()
        assert (np.abs(gc[b] - gc_ref) <= tol).all(), np.abs(gc[b] - gc_ref).max()


@pytest.mark.parametrize("shape,offset", [((255, 257), 0), ((128, 128), 1), ((128, 128), 0)])
def test_both_kernel_paths_against_the_oracle(shape, offset):
    """The adjoint kernels take four pixels per lane with 16-byte accesses
    when the pixel count is a multiple of 4 and the buffers are aligned, one
    pixel per lane otherwise: an odd pixel count (255 x 257), colors that
    start 4 bytes into their buffer, and the aligned case, each against the
    oracle's float64 D and gradients."""
    wsm = _wsm()
    h, w = shape
    _say("adjoint kernel paths, 2 images", shape, "float offset", offset)
    x_np = np.stack([synth.sinusoid_field_image(s, h, w) for s in (4, 5)]).astype(np.float32)
    x, pal, idx, _ = _forward(x_np, 16, 10, 0.0)
    B, n = 2, h * w
    buf = torch.empty(B * n * 3 + offset, dtype=torch.float32, device="cuda")
    buf[offset:] = x.reshape(-1)
    xf = buf[offset:].view(B, n, 3)
    d = torch.empty(B, dtype=torch.float64, device="cuda")
    g = torch.tensor([1.0, -0.5], dtype=torch.float64, device="cuda")
    gx = torch.empty(B, n, 3, dtype=torch.float32, device="cuda")
    gc = torch.empty_like(pal)
    ws = wsm.distortion_workspace(B, n, 16, xf.device)
    wsm.distortion_into(xf, pal, idx, d, ws, g, gx, gc)
    d, gx, gc = d.cpu().numpy(), gx.cpu().numpy(), gc.cpu().numpy()
    pal_np = pal.cpu().numpy().astype(np.float64)
    idx_np = idx.cpu().numpy()
    for b in range(B):
        xb = x_np[b].reshape(-1, 3).astype(np.float64)
        assert d[b] == pytest.approx(oracle.distortion(xb, idx_np[b], pal_np[b]), rel=SUM_RTOL)
        gx_ref, gc_ref = oracle.distortion_grad(xb, idx_np[b], pal_np[b], [1.0, -0.5][b])
        np.testing.assert_allclose(gx[b], gx_ref, rtol=2 ** -23, atol=1e-30)
        tol = 2 ** -23 * np.abs(gc_ref) + 1e-12 * np.abs(gx_ref).sum()
        assert (np.abs(gc[b] - gc_ref) <= tol).all(), np.abs(gc[b] - gc_ref).max()


def _true_distortion_colors(colors, counts, n_pix, centers, m):
    """The true D (every color at its nearest center under the map's key)
    over the unique colors, and the assignment."""
    idx, mse = oracle.assign_colors(colors, counts, n_pix, m, centers)
    return mse, idx


def test_gradients_match_central_differences_at_tie_free_points():
    """FP64 central differences (h = 1e-3) of the true distortion, the
    assignment re-chosen at every evaluation, at palette entries and pixels
    whose assignment the step does not change; D is quadratic there, so the
    difference quotient equals the derivative up to float64 rounding.  This
    checks the partial derivative with the assignment frozen (equal to the
    true one away from ties)."""
    wsm = _wsm()
    _say("adjoint vs central differences, 512x512 seed 3, K 64")
    x_np = _batch([3])
    x, pal, idx, states = _forward(x_np, 64, 10, 0.0)
    pal = (pal + 0.25).contiguous()   # away from the centroids: non-zero palette gradient
    img = x_np[0].astype(np.uint8)
    colors, counts = oracle.reduce_colors(img)
    n_pix = img.shape[0] * img.shape[1]
    c = pal.cpu().numpy()[0].astype(np.float64)
    m = states[0].membership().cpu().numpy()
    D0, a0 = _true_distortion_colors(colors, counts, n_pix, c, m)
    keys = img.reshape(-1, 3).astype(np.uint32) @ np.array([65536, 256, 1], np.uint32)
    pos = np.searchsorted(colors, keys)
    # the assignment frozen at the moved palette: every pixel at its nearest center
    frozen = torch.from_numpy(a0[pos][None].copy()).cuda()
    d, gx, gc = _grads(x, pal, frozen, np.array([1.0]))
    assert d[0] == pytest.approx(D0, rel=SUM_RTOL)
    h = 1e-3
    rng = np.random.default_rng(0)
    checked = 0
    for k in rng.choice(64, size=12, replace=False):
        for ch in range(3):
            cp, cm = c.copy(), c.copy()
            cp[k, ch] += h
            cm[k, ch] -= h
            Dp, ap = _true_distortion_colors(colors, counts, n_pix, cp, m)
            Dm, am = _true_distortion_colors(colors, counts, n_pix, cm, m)
            if not (np.array_equal(ap, a0) and np.array_equal(am, a0)):
                continue  # a tie within h: not a tie-free point
            fd = (Dp - Dm) / (2 * h)
            assert gc[0, k, ch] == pytest.approx(fd, rel=1e-5, abs=1e-9), (k, ch)
            checked += 1
    assert checked >= 18
    # pixels: only the pixel's own term moves; tie-free = the margin between
    # its two nearest centers exceeds the change any h step can make
    xp = x_np[0].reshape(-1, 3).astype(np.float64)
    sel = rng.choice(n_pix, size=200, replace=False)
    dd = ((xp[sel, None, :] - c[None, :, :]) ** 2).sum(2)
    part = np.partition(dd, 1, axis=1)
    free = sel[(part[:, 1] - part[:, 0]) > 4 * h * 512]
    assert len(free) > 100
    for p in free[:60]:
        for ch in range(3):
            e = np.zeros(3)
            e[ch] = h
            up = ((xp[p] + e - c) ** 2).sum(1).min()
            dn = ((xp[p] - e - c) ** 2).sum(1).min()
            fd = (up - dn) / (2 * h) / n_pix
            assert gx[0].reshape(-1, 3)[p, ch] == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_palette_gradient_vanishes_at_the_fixed_point():
    """At a fixed point of the iteration every center is the mean of its
    colors, so dD/dc (frozen assignment) is zero up to the float32 rounding
    of the palette: |dD/dc_k| <= (2/N) W_k |c_k - mean_k| <= (2/N) W_k 2^-16.
    This is the envelope property: there the total derivative of the
    converged D with respect to the initial palette is zero as well."""
    _say("adjoint at convergence, 256x256 seed 1, K 16, up to 500 iterations")
    x_np = synth.workload_image("small", 1)[None].astype(np.float32)
    x, pal, idx, states = _forward(x_np, 16, 500, 0.0)
    st = states[0]
    assert np.array_equal(st.membership().cpu().numpy(),
                          oracle.search_step(oracle.reduce_colors(x_np[0].astype(np.uint8))[0],
                                             st.palette64().cpu().numpy(),
                                             st.membership().cpu().numpy())[0]), "not converged"
    d, gx, gc = _grads(x, pal, idx, np.array([1.0]))
    W = np.bincount(idx.cpu().numpy()[0], minlength=16)
    n = x_np[0].shape[0] * x_np[0].shape[1]
    bound = 2.0 / n * W * 2 ** -16 * np.sqrt(3) + 1e-9
    assert (np.linalg.norm(gc[0], axis=1) <= bound).all()


def test_batch_of_sixteen_and_validation():
    """The differentiable configuration's batch shape (16 images, K 64) on
    smaller images, every image's D and gradient independent of the others;
    and argument errors."""
    wsm = _wsm()
    _say("adjoint batch of 16 128x128 images, K 64")
    x_np = _batch(list(range(16)), size=128)
    x, pal, idx, _ = _forward(x_np, 64, 10, 0.0)
    d, gx, gc = _grads(x, pal, idx, np.ones(16))
    for b in (0, 7, 15):
        d1, gx1, gc1 = _grads(x[b:b + 1].contiguous(), pal[b:b + 1].contiguous(),
                              idx[b:b + 1].contiguous(), np.ones(1))
        assert d1[0] == d[b]
        assert np.array_equal(gx1[0], gx[b]) and np.array_equal(gc1[0], gc[b])
    with pytest.raises(wsm.WsmError):
        wsm.distortion(x.double(), pal, idx)
    with pytest.raises(wsm.WsmError):
        wsm.quantize_batch(x + 0.5, 64, lambda n, k: synth.init_indices(7, n, k))

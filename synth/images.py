"""Seeded synthetic RGB images standing in for the paper's test images.

The paper evaluates on eight standard test images (Sec. 3.1) of 300x200 up to
1536x1024 pixels with 7-58 % unique colors.  Those images are not available
here, so these generators produce photo-like uint8 images of comparable size
and unique-color density.  All randomness comes from
``numpy.random.default_rng(seed)`` (PCG64); arithmetic is float64 and the final
cast is ``clip(rint(v), 0, 255)``.

Workloads (sizes and unique-color counts are logged by the tests and bench):

* ``small``   256x256, 3 linear gradients + 12 Gaussian blobs (sigma 10 px),
              about 16-25k unique colors, K = 32.
* ``medium``  512x512, 128 + 6 random 2-D sinusoids per channel (amplitude
              U[4,16], 1/2..4 cycles per 512 px) + N(0, 6^2) noise, about
              160-200k unique colors, K in {16, 64, 256}.
* ``large``   4096x4096, the same field at the same 512-px spatial scale with
              amplitude U[5,20] and noise sigma 12, about 2M unique colors,
              K = 256.
* ``batched`` 64 square images with side uniform in [128, 1024] and K drawn
              from {16, 32, 64, 128, 256}, the ``medium`` generator.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "gradient_blob_image",
    "sinusoid_field_image",
    "workload_image",
    "batched_workload",
    "WORKLOADS",
]


def _to_u8(v: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(v), 0, 255).astype(np.uint8)


def gradient_blob_image(seed: int, height: int = 256, width: int = 256,
                        n_gradients: int = 3, n_blobs: int = 12,
                        blob_sigma: float = 10.0) -> np.ndarray:
    """Sum of linear color gradients and isotropic Gaussian color blobs.

    Each gradient has a direction theta ~ U[0, 2pi); the pixel coordinate is
    projected onto it and normalised to [0, 1]; the gradient adds t * v with a
    color vector v ~ U[0, 170]^3.  Each blob has a center uniform in the image
    and a color amplitude ~ U[-50, 50]^3 and adds a * exp(-r^2 / (2 sigma^2)).
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    img = np.zeros((height, width, 3), dtype=np.float64)
    for _ in range(n_gradients):
        theta = rng.uniform(0.0, 2.0 * np.pi)
        proj = xx * np.cos(theta) + yy * np.sin(theta)
        t = (proj - proj.min()) / max(proj.max() - proj.min(), 1e-12)
        v = rng.uniform(0.0, 170.0, size=3)
        img += t[..., None] * v[None, None, :]
    for _ in range(n_blobs):
        cy = rng.uniform(0.0, height)
        cx = rng.uniform(0.0, width)
        a = rng.uniform(-50.0, 50.0, size=3)
        r2 = (yy - cy) ** 2 + (xx - cx) ** 2
        img += np.exp(-r2 / (2.0 * blob_sigma ** 2))[..., None] * a[None, None, :]
    return _to_u8(img)


def sinusoid_field_image(seed: int, height: int = 512, width: int = 512,
                         n_waves: int = 6, amp_lo: float = 4.0,
                         amp_hi: float = 16.0, noise_sigma: float = 6.0,
                         scale: float = 512.0, row_block: int = 512) -> np.ndarray:
    """128 + sum of random 2-D sinusoidal color fields + Gaussian noise.

    Wave s has spatial frequency f ~ U[0.5, 4]^2 cycles per ``scale`` pixels,
    per-channel phase ~ U[0, 2pi)^3 and per-channel amplitude
    ~ U[amp_lo, amp_hi]^3.  i.i.d. N(0, noise_sigma^2) noise is added per
    channel.  Rows are generated in blocks so that 4096x4096 fits in memory.
    """
    rng = np.random.default_rng(seed)
    freqs = rng.uniform(0.5, 4.0, size=(n_waves, 2))
    phases = rng.uniform(0.0, 2.0 * np.pi, size=(n_waves, 3))
    amps = rng.uniform(amp_lo, amp_hi, size=(n_waves, 3))
    out = np.empty((height, width, 3), dtype=np.uint8)
    xs = np.arange(width, dtype=np.float64)
    for r0 in range(0, height, row_block):
        r1 = min(height, r0 + row_block)
        ys = np.arange(r0, r1, dtype=np.float64)
        block = np.full((r1 - r0, width, 3), 128.0, dtype=np.float64)
        for s in range(n_waves):
            arg = 2.0 * np.pi * (freqs[s, 0] * xs[None, :] + freqs[s, 1] * ys[:, None]) / scale
            for ch in range(3):
                block[..., ch] += amps[s, ch] * np.sin(arg + phases[s, ch])
        block += rng.normal(0.0, noise_sigma, size=block.shape)
        out[r0:r1] = _to_u8(block)
    return out


WORKLOADS = {
    "small": dict(kind="gradient_blob", height=256, width=256, ks=(32,)),
    "medium": dict(kind="sinusoid", height=512, width=512, ks=(16, 64, 256),
                   amp=(4.0, 16.0), noise=6.0),
    "large": dict(kind="sinusoid", height=4096, width=4096, ks=(256,),
                  amp=(5.0, 20.0), noise=12.0),
}


def workload_image(name: str, seed: int) -> np.ndarray:
    """The seeded image of a named workload (see the module docstring)."""
    w = WORKLOADS[name]
    if w["kind"] == "gradient_blob":
        return gradient_blob_image(seed, w["height"], w["width"])
    return sinusoid_field_image(seed, w["height"], w["width"],
                                amp_lo=w["amp"][0], amp_hi=w["amp"][1],
                                noise_sigma=w["noise"])


def batched_workload(seed: int = 0, n_images: int = 64,
                     side_lo: int = 128, side_hi: int = 1024):
    """64 square images of uneven size, each with its own K.

    Returns a list of (image, K, image_seed).  Side ~ U{side_lo..side_hi},
    K ~ U{16, 32, 64, 128, 256}; each image uses the ``medium`` generator
    with its own seed.
    """
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=n_images)
    ks = rng.choice(np.array([16, 32, 64, 128, 256]), size=n_images)
    out = []
    for j in range(n_images):
        s = int(sides[j])
        img = sinusoid_field_image(1000 + j, s, s)
        out.append((img, int(ks[j]), 1000 + j))
    return out

"""The random initial centers, drawn outside both implementations.

The method starts from a random subset of the unique colors (Alg. 2, first
step; Sec. 2).  The paper does not name a generator, so the draw is fixed
here: K distinct indices into the ascending unique-color table, in draw order,
from ``numpy.random.default_rng(seed).choice(n_unique, K, replace=False)``.
The same indices (hence the same float32-exact integer palette) are handed to
the oracle and to the GPU path.
"""

from __future__ import annotations

import numpy as np


def init_indices(seed: int, n_unique: int, k: int) -> np.ndarray:
    """K distinct indices in [0, n_unique), in draw order (int64)."""
    if not (1 <= k <= n_unique):
        raise ValueError(f"need 1 <= K <= n_unique, got K={k}, n_unique={n_unique}")
    rng = np.random.default_rng(seed)
    return rng.choice(n_unique, size=k, replace=False).astype(np.int64)


def unpack_keys_to_palette(keys: np.ndarray) -> np.ndarray:
    """Packed 0x00RRGGBB keys -> (len, 3) float32 array of (R, G, B)."""
    keys = np.asarray(keys, dtype=np.uint32)
    r = (keys >> 16) & 0xFF
    g = (keys >> 8) & 0xFF
    b = keys & 0xFF
    return np.stack([r, g, b], axis=1).astype(np.float32)

"""Autotuner of the batched persistent form's work split.

For each class of images -- the unique-color count bucket floor(log2 N')
and K -- it picks the points per search work item (which sets the number of
virtual search blocks, N' / points) and the rows per rows work item, by
timing the batched launch on a few synthetic images of that class with
every candidate, and caches the winners in a JSON file.  Batch() uses the
cache when it exists and its defaults otherwise.

The timing is the library's own batched launch on the GPU; the synthetic
images are the seeded sinusoid-field generator at sizes that give the
class's N'.
"""

from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import Batch, init, palette_from_indices, reduce_colors

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_batch.json")
POINTS_PER_ITEM = (2048, 4096, 8192, 16384)
ROWS_PER_ITEM = (1, 4, 16)
KS = (16, 32, 64, 128, 256)


def class_key(n_unique: int, k: int) -> str:
    return f"{int(math.floor(math.log2(max(n_unique, 1))))}:{k}"


def load(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def split_for(table: dict, n_unique: int, k: int):
    """(grid, rows_per_item) for one image from the table (0 = default)."""
    e = table.get(class_key(n_unique, k))
    if not e:
        return 0, 0
    grid = max(1, min(2048, -(-n_unique // int(e["points_per_item"]))))
    return grid, int(e["rows_per_item"])


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(sides=(128, 256, 512, 768, 1024), ks=KS, images_per_class=16, max_iters=10,
         path: str = CACHE, seed: int = 0, log=print) -> dict:
    """Times every candidate split for each (N' bucket, K) class met by
    images of the given sides -- a batch of images_per_class images of the
    class, enough to fill the GPU as a real batch does, 10 fixed iterations
    per image -- and writes the winners to `path`."""
    import synth
    table = load(path)
    for side in sides:
        imgs = [torch.from_numpy(synth.sinusoid_field_image(seed * 1000 + j, side, side)).cuda()
                for j in range(images_per_class)]
        tabs = [reduce_colors(g) for g in imgs]
        n_pix = side * side
        for k in ks:
            if any(c.numel() < k for c, _ in tabs):
                continue
            pals = [palette_from_indices(c, synth.init_indices(j, c.numel(), k))
                    for j, (c, _) in enumerate(tabs)]
            states = [init(c, n, n_pix, p) for (c, n), p in zip(tabs, pals)]
            key = class_key(int(np.median([c.numel() for c, _ in tabs])), k)
            best = None
            for ppi in POINTS_PER_ITEM:
                for rpi in ROWS_PER_ITEM:
                    grid = [max(1, min(2048, -(-st.n_points // ppi))) for st in states]
                    b = Batch(states, max_iters, 0.0, grid, [rpi] * len(states))

                    def run(b=b):
                        for st, (c, n), p in zip(states, tabs, pals):
                            init(c, n, n_pix, p, reuse=st)
                        b.launch()

                    ms = _time(run)
                    b.close()
                    if best is None or ms < best[0]:
                        best = (ms, ppi, rpi)
            table[key] = dict(points_per_item=best[1], rows_per_item=best[2], ms=best[0],
                              side=side, images=images_per_class, iters=max_iters)
            log(f"class {key} (side {side}): points/item {best[1]}, rows/item {best[2]}, "
                f"{best[0]:.3f} ms")
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    return table

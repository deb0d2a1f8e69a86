#!/usr/bin/env python
"""Benchmark of the MI355X weighted sort-means color quantizer.

Metric: WSM color-iterations/s (unique colors x iterations per second of the
whole pipeline) and images/s, on the 512x512 synthetic photo-like workload
(seeded sum of 6 sinusoidal color fields + N(0, 6^2) noise, ~180k unique
colors) quantized at K = 16, 64 and 256 (WSM-C: eps = 1e-4, at most 50
iterations), compared with full-search batch k-means on the GPU from the same
initial palette (same trajectory, so equal MSE by construction; checked).

One step = one pass of the whole hot path over the image: unique-color
reduction, then for each K: initial palette from the seeded random subset,
state init, iterations, pixel map (with MSE).  Inputs are resident in HBM
before the timed region.  Every kernel is launched directly; the same step
replayed from caller-owned HIP graphs is reported beside it.

Prints ONE JSON line.  Extra objects: per-K details, the full-search
comparators, the roofline of the dominant kernel (measured live with HIP
events around each of its launches, in a separate pass over the same
workload), the 256x256 workload (WSM-C and the fixed 10-iteration variant),
the 4096x4096 workload (reduction and map rooflines, whole-image
throughput), the K-scaling study (time and evaluations per iteration for
K = 2..256, sort-means against the full search), and the FP64 CPU oracle
timed on this host.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one search_kernel launch on this workload: two rocprofv3
# counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
# what the counter reads for a 256 MiB reference copy in the same program
# (profiles/search_kernel_512x512_traffic.md).  It describes the kernel
# sources it was measured on (hash below); for any other sources the bench
# reports null.
SEARCH_TRAFFIC_BYTES = 3846919
SEARCH_TRAFFIC_SRC = "7cec0f1246baf378"
_KERNEL_SOURCES = ("iterate.hip", "iter_device.h", "sm_block.h", "wave_ops.h", "wsm_internal.h")

# The same for the 4096x4096 reduction (partition + compaction, bytes per
# call) and pixel gather (bytes per launch)
# (profiles/reduce_map_4096x4096_traffic.md).
REDUCE_TRAFFIC_BYTES = 173722701
REDUCE_TRAFFIC_SRC = "3daaa189cbeb9d45"
GATHER_TRAFFIC_BYTES = 106355179
GATHER_TRAFFIC_SRC = "152d475eeb197d94"
_REDUCE_SOURCES = ("reduce.hip", "wave_ops.h", "wsm_internal.h")
_MAP_SOURCES = ("map.hip", "sm_block.h", "wave_ops.h", "wsm_internal.h")


def _code_only(text: str) -> str:
    """C++ source without its comments, trailing spaces and blank lines."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, copied whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (line.rstrip() for line in "".join(out).splitlines())
    return "\n".join(line for line in lines if line)


def kernel_sources_hash(names=None) -> str:
    """sha256 (first 16 hex digits) of kernel sources (default: the search
    kernel's), comments and blank lines removed, so that a comment edit keeps
    the counters."""
    import hashlib
    h = hashlib.sha256()
    for name in names or _KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1011_0093_amd", "csrc", name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


FP32_PEAK_TFLOPS = 157.3
EPS = 1e-4
MAX_ITERS = 50


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-k-sweep", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--single-stream", action="store_true",
                    help="run the three K of a step one after another on one stream")
    ap.add_argument("--no-oracle-timings", action="store_true")
    ap.add_argument("--no-differentiable", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB before the steps "
                         "(a reference dispatch for hardware traffic counters)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the quantizer runs on one GPU; it has no multi-GPU form "
                                   "(the path would shard by color-key range)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    import paper_1011_0093_amd as wsm
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    img_np = synth.workload_image("medium", args.seed)
    H, W, _ = img_np.shape
    N = H * W
    Ks = list(synth.WORKLOADS["medium"]["ks"])
    img = torch.from_numpy(img_np).to(dev)
    cap = min(N, 1 << 24)
    colors = torch.empty(cap, dtype=torch.int32, device=dev)
    counts = torch.empty(cap, dtype=torch.int32, device=dev)
    nu = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(wsm.reduce_workspace_bytes(N), dtype=torch.uint8, device=dev)
    lut = torch.empty(1 << 24, dtype=torch.uint8, device=dev)
    idx_host = torch.empty(sum(Ks), dtype=torch.int32).pin_memory()
    idx_dev = torch.empty(sum(Ks), dtype=torch.int32, device=dev)
    # one state buffer per K, re-initialised every step (persistent buffers,
    # as a serving loop would keep them)
    states = {}
    # the three K of a step are independent: by default each runs (init,
    # iterate, map) on a HIP stream of its own (default priority), after the
    # shared reduction, so that their latency-bound launches overlap
    k_streams = {K: torch.cuda.Stream(device=dev) for K in Ks}
    luts = {K: torch.empty(1 << 24, dtype=torch.uint8, device=dev) for K in Ks}
    # search blocks of each K while the three share the GPU (of 256 CUs): the
    # longest chain (K = 256) keeps three quarters, K = 64 and K = 16 half
    # each; K = 16 is enqueued last and starts last, so it needs the blocks to
    # catch up (chosen by measurement; results do not depend on the grid)
    share_grid = {16: 128, 64: 128, 256: 192}

    def step(single_stream=args.single_stream):
        wsm.reduce_colors_into(img, colors, counts, nu, ws)
        n_unique = int(nu.item())  # the caller needs N' to draw the initial subset
        col, cnt = colors[:n_unique], counts[:n_unique]
        off = 0
        for K in Ks:
            idx_host[off:off + K] = torch.from_numpy(
                synth.init_indices(args.seed, n_unique, K).astype(np.int32))
            off += K
        idx_dev.copy_(idx_host, non_blocking=True)
        ready = torch.cuda.Event()
        ready.record(stream)
        offs = dict(zip(Ks, np.cumsum([0] + Ks[:-1]).tolist()))
        out = {}
        # concurrent: the longest chain (largest K) is enqueued first
        for K in (Ks if single_stream else sorted(Ks, reverse=True)):
            s_k = stream if single_stream else k_streams[K]
            s_k.wait_event(ready)
            with torch.cuda.stream(s_k):
                pal = wsm.palette_from_indices(col, idx_dev[offs[K]:offs[K] + K])
                st = wsm.init(col, cnt, N, pal, reuse=states.get(K))
                states[K] = st
                if not single_stream and K in share_grid:
                    st.grid = min(st.grid, share_grid[K])
                st.iterate(MAX_ITERS, EPS)
                index, _, mse = wsm.map_pixels(st, img, lut=lut if single_stream else luts[K])
            out[K] = (st, mse, pal)
        if not single_stream:
            for K in Ks:
                stream.wait_stream(k_streams[K])
        return n_unique, out

    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    e0.record(stream)
    for s_ in range(args.steps):
        n_unique, out = step()
        marks[s_].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = [e0.elapsed_time(marks[0])] + [marks[s_ - 1].elapsed_time(marks[s_])
                                              for s_ in range(1, args.steps)]
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    ms_step_wall = wall * 1000.0 / args.steps
    # the same step with the three K one after another on one stream
    ms_single = None
    if not args.single_stream:
        for _ in range(args.warmup):
            step(single_stream=True)
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(args.steps):
            step(single_stream=True)
        s1.record(stream)
        torch.cuda.synchronize()
        ms_single = s0.elapsed_time(s1) / args.steps

    # ---- the same step with each K's iterate launches replayed from a
    # caller-owned HIP graph, recorded once outside the timed region (the
    # same image every step, so the recorded arguments stay valid)
    graph_leg = None
    if not args.no_graph:
        if not args.single_stream:
            for K in Ks:
                states[K].grid = min(states[K].grid, share_grid[K])
        graphs = {K: states[K].graph(MAX_ITERS, EPS) for K in Ks}
        ref64 = {K: states[K].palette64().cpu() for K in Ks}

        def step_graph():
            wsm.reduce_colors_into(img, colors, counts, nu, ws)
            n_u = int(nu.item())
            col_g, cnt_g = colors[:n_u], counts[:n_u]
            o = 0
            for K in Ks:
                idx_host[o:o + K] = torch.from_numpy(
                    synth.init_indices(args.seed, n_u, K).astype(np.int32))
                o += K
            idx_dev.copy_(idx_host, non_blocking=True)
            ready_g = torch.cuda.Event()
            ready_g.record(stream)
            offs_g = dict(zip(Ks, np.cumsum([0] + Ks[:-1]).tolist()))
            for K in (Ks if args.single_stream else sorted(Ks, reverse=True)):
                s_k = stream if args.single_stream else k_streams[K]
                s_k.wait_event(ready_g)
                with torch.cuda.stream(s_k):
                    pal_g = wsm.palette_from_indices(col_g, idx_dev[offs_g[K]:offs_g[K] + K])
                    st_g = wsm.init(col_g, cnt_g, N, pal_g, reuse=states[K])
                    graphs[K].launch()
                    wsm.map_pixels(st_g, img, lut=lut if args.single_stream else luts[K])
            if not args.single_stream:
                for K in Ks:
                    stream.wait_stream(k_streams[K])

        for _ in range(args.warmup):
            step_graph()
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(args.steps):
            step_graph()
        g1.record(stream)
        torch.cuda.synchronize()
        ms_graph = g0.elapsed_time(g1) / args.steps
        same = all(torch.equal(states[K].palette64().cpu(), ref64[K]) for K in Ks)
        for gr in graphs.values():
            gr.close()
        graph_leg = dict(ms_per_step=ms_graph, images_per_s=len(Ks) / (ms_graph * 1e-3),
                         equal_to_direct=bool(same),
                         note="iterate launches of each K replayed from a caller-owned HIP graph "
                              "(wsm_iterate_graph_*), on the K's stream; reduce, init and map "
                              "launched directly")

    per_k = {}
    color_iters = 0
    for K in Ks:
        st, mse, pal = out[K]
        info = st.info()
        sse, ev = st.history()
        color_iters += n_unique * info["iters"]
        mse_v = float(mse.item())
        per_k[str(K)] = dict(iters=info["iters"], converged=info["converged"],
                             mse=mse_v,
                             psnr_db=10.0 * math.log10(255.0 ** 2 / mse_v) if mse_v > 0 else None,
                             evals_per_color_first=float(ev[0] / n_unique),
                             evals_per_color_last=float(ev[-1] / n_unique))
    value = color_iters / (ms_step * 1e-3)
    if graph_leg is not None:
        graph_leg["value"] = color_iters / (graph_leg["ms_per_step"] * 1e-3)
    single_leg = None
    if ms_single is not None:
        single_leg = dict(ms_per_step=ms_single, images_per_s=len(Ks) / (ms_single * 1e-3),
                          value=color_iters / (ms_single * 1e-3))

    # ---- per-phase times and the full-search comparators (separate passes)
    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    col, cnt = colors[:n_unique], counts[:n_unique]
    phases = {"reduce_ms": timed(lambda: wsm.reduce_colors_into(img, colors, counts, nu, ws))}
    comparators = {}
    for K in Ks:
        st, mse, pal = out[K]
        iters = st.info()["iters"]

        scratch = {}

        def run_sm(pal=pal):
            s = wsm.init(col, cnt, N, pal, reuse=scratch.get("sm"))
            scratch["sm"] = s
            s.iterate(MAX_ITERS, EPS)
            return s

        t_sm = timed(run_sm)
        phases[f"iterate_ms_k{K}"] = t_sm
        phases[f"map_ms_k{K}"] = timed(lambda st=st: wsm.map_pixels(st, img, lut=lut))
        if args.no_comparators:
            continue
        holder = {}

        def run_full(pal=pal):
            s = wsm.init(col, cnt, N, pal, reuse=holder.get("full"))
            s.iterate_full(MAX_ITERS, EPS)
            holder["full"] = s

        def run_pix(pal=pal):
            s = wsm.init_pixels(img, pal, reuse=holder.get("pix"))
            s.iterate_full(MAX_ITERS, EPS)
            holder["pix"] = s

        t_full = timed(run_full)
        t_pix = timed(run_pix, reps=2)
        p_sm = st.palette().cpu().numpy()
        same_full = bool(np.array_equal(p_sm, holder["full"].palette().cpu().numpy()))
        same_pix = bool(np.array_equal(p_sm, holder["pix"].palette().cpu().numpy()))
        _, _, mse_full = wsm.map_pixels(holder["full"], img, lut=lut)
        comparators[str(K)] = dict(
            wsm_iterate_ms=t_sm, full_weighted_ms=t_full, full_pixels_ms=t_pix,
            iters_full=holder["full"].info()["iters"], iters_pixels=holder["pix"].info()["iters"],
            speedup_vs_full_weighted=t_full / t_sm, speedup_vs_full_pixels=t_pix / t_sm,
            full_weighted_color_iters_per_s=n_unique * holder["full"].info()["iters"] / (t_full * 1e-3),
            full_pixels_pixel_iters_per_s=N * holder["pix"].info()["iters"] / (t_pix * 1e-3),
            equal_palette_full=same_full, equal_palette_pixels=same_pix,
            mse_wsm=float(out[K][1].item()), mse_full=float(mse_full.item()))

    # ---- roofline of the dominant kernel: the sort-means search launch at
    # K = 256 from the second step on (search_kernel<true, 3>: row heads in
    # LDS, flattened scans, long scans deferred; the first step of a call runs
    # its own variant, K = 64 the lane-scan variant and K <= 32 one fused
    # launch per step), timed per launch with events the runtime records at
    # the kernel.  Algorithmic bytes per color and iteration: 4 (key) +
    # 4 (count) + 1 (membership read) + 1 (write).
    launches = []
    for K in Ks:
        if K < 128:
            continue
        st, mse, pal = out[K]
        with wsm.kernel_timer("search", capacity=MAX_ITERS) as kt:
            s = wsm.init(col, cnt, N, pal)
            s.iterate(MAX_ITERS, EPS)
        it = s.info()["iters"]
        launches += kt.ms[1:it]
    dur_ms = float(np.mean(launches))
    bytes_per_launch = 10.0 * n_unique
    achieved = bytes_per_launch / (dur_ms * 1e-3) / 1e9
    traffic = None
    if SEARCH_TRAFFIC_BYTES is not None and kernel_sources_hash() == SEARCH_TRAFFIC_SRC:
        traffic = SEARCH_TRAFFIC_BYTES
    roofline = dict(kernel="wsm::search_kernel<true, 3>", bound="hbm", achieved=achieved,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                    traffic_unit="bytes per launch", avg_launch_us=dur_ms * 1e3,
                    launches=len(launches), bytes_per_launch=bytes_per_launch)

    small = None
    small_np = synth.workload_image("small", 0)
    if not args.no_small:
        small = bench_small(torch, wsm, synth, small_np)

    large = None
    large_np = None
    if not args.no_large or not args.no_k_sweep:
        large_np = synth.workload_image("large", 0)
    if not args.no_large:
        large = bench_large(args, torch, wsm, synth, large_np)

    sweep = None
    if not args.no_k_sweep:
        sweep = k_sweep(torch, wsm, synth, {"512x512": img_np, "4096x4096": large_np}, args.seed)

    batched = None
    if not args.no_batched:
        batched = bench_batched(torch, wsm, synth)

    diff = None
    if not args.no_differentiable:
        diff = bench_differentiable(torch, wsm, synth)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, img_np, Ks, n_unique)
    oracle_t = None
    if not args.no_oracle_timings:
        oracle_t = oracle_timings(small_np, large_np)

    line = {
        "metric": "WSM color-iterations/s and images/s vs full-search GPU k-means at equal MSE",
        "value": value,
        "unit": "color-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_wall": ms_step_wall,
        "ms_per_step_p10_p50_p90": [float(np.percentile(step_ms, q)) for q in (10, 50, 90)],
        "images_per_s": len(Ks) / (ms_step * 1e-3),
        "launches": ("direct (no graph replay), one stream" if args.single_stream else
                     "direct (no graph replay); after the shared reduction each K on a HIP stream "
                     "of its own"),
        "single_stream": single_leg,
        "graph_replay": graph_leg,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512 sinusoid-field image (seed %d), K in %s, WSM-C eps=1e-4, "
                               "max 50 iterations; reduce + init + iterate + map per step"
                               % (args.seed, Ks),
                   "n_pixels": N, "n_unique": n_unique, "ks": Ks},
        "per_k": per_k,
        "phases_ms": phases,
        "comparators": comparators,
        "roofline": roofline,
        "roofline_large": large,
        "small_256x256": small,
        "k_scaling": sweep,
        "batched": batched,
        "differentiable": diff,
        "cpu_baseline": cpu,
        "oracle_timings": oracle_t,
    }
    print(json.dumps(line), flush=True)


def _timed(torch, fn, reps=5):
    """Average ms of fn() over reps calls, events on the current stream,
    after one untimed call."""
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


def _whole_image(torch, wsm, synth, img, K, max_iters, eps, seed=0):
    """One image through the whole path (reduce, palette, init, iterate,
    map with MSE), launches direct; returns a callable and a holder of the
    last state and MSE."""
    dev = img.device
    N = img.numel() // 3
    colors = torch.empty(min(N, 1 << 24), dtype=torch.int32, device=dev)
    counts = torch.empty_like(colors)
    nu = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(wsm.reduce_workspace_bytes(N), dtype=torch.uint8, device=dev)
    lut = torch.empty(1 << 24, dtype=torch.uint8, device=dev)
    held = {}

    def run():
        wsm.reduce_colors_into(img, colors, counts, nu, ws)
        n_u = int(nu.item())
        col, cnt = colors[:n_u], counts[:n_u]
        pal = wsm.palette_from_indices(col, synth.init_indices(seed, n_u, K))
        st = wsm.init(col, cnt, N, pal, reuse=held.get("st"))
        st.iterate(max_iters, eps)
        _, _, mse = wsm.map_pixels(st, img, lut=lut)
        held.update(st=st, mse=mse, n_unique=n_u)

    return run, held


def bench_small(torch, wsm, synth, img_np, K=32):
    """The 256x256 workload (K = 32): the whole image through WSM-C (eps
    1e-4, at most 50 iterations) and through the fixed 10-iteration variant,
    and the iterations alone."""
    img = torch.from_numpy(img_np).to("cuda:0")
    N = img_np.shape[0] * img_np.shape[1]
    out = dict(workload="256x256 gradient + blob image (seed 0), K=32", n_pixels=N)
    for name, (mi, eps) in (("wsm_c", (MAX_ITERS, EPS)), ("fixed10", (10, 0.0))):
        run, held = _whole_image(torch, wsm, synth, img, K, mi, eps)
        ms = _timed(torch, run, reps=20)
        st = held["st"]
        info = st.info()
        col, cnt = st.refs[0], st.refs[1]
        pal = st.refs[2]
        hold = {}

        def it_only():
            s_ = wsm.init(col, cnt, N, pal, reuse=hold.get("s"))
            hold["s"] = s_
            s_.iterate(mi, eps)

        ms_it = _timed(torch, it_only, reps=20)
        mse = float(held["mse"].item())
        out[name] = dict(ms_per_image=ms, images_per_s=1e3 / ms, iterate_ms=ms_it,
                         iters=info["iters"], converged=info["converged"],
                         n_unique=held["n_unique"], mse=mse,
                         psnr_db=10.0 * math.log10(255.0 ** 2 / mse) if mse > 0 else None,
                         color_iters_per_s=held["n_unique"] * info["iters"] / (ms_it * 1e-3))
    return out


def k_sweep(torch, wsm, synth, images, seed=0, Ks=(2, 4, 8, 16, 32, 64, 128, 256)):
    """Time and distance evaluations per iteration against K: sort-means and
    the full search, 10 fixed iterations each, and WSM-C (eps 1e-4, at most
    50 iterations), from the same seeded palette; launches direct."""
    out = {}
    for name, img_np in images.items():
        if img_np is None:
            continue
        img = torch.from_numpy(img_np).to("cuda:0")
        N = img_np.shape[0] * img_np.shape[1]
        col, cnt = wsm.reduce_colors(img)
        n = col.numel()
        rows = []
        for K in Ks:
            pal = wsm.palette_from_indices(col, synth.init_indices(seed, n, K))
            hold = {}

            def mk(full, mi, eps, pal=pal, hold=hold):
                def f():
                    s_ = wsm.init(col, cnt, N, pal, reuse=hold.get((full, mi)))
                    hold[(full, mi)] = s_
                    if full:
                        s_.iterate_full(mi, eps)
                    else:
                        s_.iterate(mi, eps)
                return f

            t_sm = _timed(torch, mk(False, 10, 0.0))
            t_full = _timed(torch, mk(True, 10, 0.0))
            t_c = _timed(torch, mk(False, MAX_ITERS, EPS))
            sm10 = hold[(False, 10)]
            _, ev = sm10.history()
            st_c = hold[(False, MAX_ITERS)]
            it_c = st_c.info()["iters"]
            sse_c, ev_c = st_c.history()
            same = bool(torch.equal(sm10.palette64().cpu(), hold[(True, 10)].palette64().cpu()))
            rows.append(dict(
                K=K, fixed10_us_per_iter=t_sm * 100.0, full10_us_per_iter=t_full * 100.0,
                speedup_vs_full=t_full / t_sm,
                evals_per_color_iter1=float(ev[0] / n),
                evals_per_color_iters2to10=float(ev[1:].mean() / n) if len(ev) > 1 else None,
                wsm_c_iters=it_c, wsm_c_ms=t_c, wsm_c_us_per_iter=t_c * 1e3 / it_c,
                wsm_c_converged=st_c.info()["converged"],
                wsm_c_evals_per_color_iter=float(ev_c.mean() / n),
                equal_palette_full=same))
        out[name] = dict(n_unique=n, rows=rows)
    return out


def bench_batched(torch, wsm, synth, n_images=64):
    """The batched configuration: 64 square images, side uniform in
    [128, 1024], K drawn from {16, 32, 64, 128, 256} (seeded), each through
    the whole path (reduce, palette, init, WSM-C at eps 1e-4 with at most 50
    iterations, map with MSE).  Sequential: 64 plain per-image calls.
    Batched: the 64 reductions, one read-back of the unique counts, the 64
    inits, one persistent launch for all the iterations (a plan recorded
    once for these images), the 64 maps.  Equal MSE is checked image by
    image (the palettes are bit-identical)."""
    work = synth.batched_workload(0, n_images)
    imgs = [torch.from_numpy(img).to("cuda:0") for img, _, _ in work]
    Ks = [k for _, k, _ in work]
    seeds = [s for _, _, s in work]
    lut = torch.empty(1 << 24, dtype=torch.uint8, device="cuda:0")
    seq_states = {}

    def sequential():
        out = []
        for j, (g, K, sd) in enumerate(zip(imgs, Ks, seeds)):
            col, cnt = wsm.reduce_colors(g)
            pal = wsm.palette_from_indices(col, synth.init_indices(sd, col.numel(), K))
            st = wsm.init(col, cnt, g.numel() // 3, pal, reuse=seq_states.get(j))
            seq_states[j] = st
            st.iterate(MAX_ITERS, EPS)
            _, _, mse = wsm.map_pixels(st, g, lut=lut)
            out.append(mse)
        return out

    t_seq = _timed(torch, sequential, reps=2)
    seq_mse = [float(m.item()) for m in sequential()]
    # batched: fixed buffers per image
    bufs = []
    for g in imgs:
        N = g.numel() // 3
        bufs.append(dict(
            colors=torch.empty(min(N, 1 << 24), dtype=torch.int32, device="cuda:0"),
            counts=torch.empty(min(N, 1 << 24), dtype=torch.int32, device="cuda:0"),
            nu=torch.empty(1, dtype=torch.int32, device="cuda:0"),
            ws=torch.empty(wsm.reduce_workspace_bytes(N), dtype=torch.uint8, device="cuda:0"),
            idx=torch.empty(N, dtype=torch.uint8, device="cuda:0"),
            mse=torch.empty(1, dtype=torch.float64, device="cuda:0")))
    holder = {}

    def prepare():
        for g, b in zip(imgs, bufs):
            wsm.reduce_colors_into(g, b["colors"], b["counts"], b["nu"], b["ws"])
        nus = torch.cat([b["nu"] for b in bufs]).cpu().tolist()  # one read-back for all
        states = holder.get("states")
        new = []
        for j, (g, b, K, sd) in enumerate(zip(imgs, bufs, Ks, seeds)):
            col, cnt = b["colors"][:nus[j]], b["counts"][:nus[j]]
            pal = wsm.palette_from_indices(col, synth.init_indices(sd, nus[j], K))
            new.append(wsm.init(col, cnt, g.numel() // 3, pal,
                                reuse=states[j] if states else None))
        holder["states"] = new
        return new

    states = prepare()
    t0 = time.perf_counter()
    plan = wsm.Batch(states, MAX_ITERS, EPS)
    t_plan = (time.perf_counter() - t0) * 1e3

    def batched():
        st_ = prepare()
        plan.launch()
        for g, b, st in zip(imgs, bufs, st_):
            wsm.map_pixels_into(st, g, lut, b["idx"], b["mse"])

    t_bat = _timed(torch, batched, reps=2)
    batched()
    torch.cuda.synchronize()
    err = plan.error()
    bat_mse = [float(b["mse"].item()) for b in bufs]
    same = all(torch.equal(a.palette64().cpu(), seq_states[j].palette64().cpu())
               for j, a in enumerate(holder["states"]))
    # the persistent launch alone, and the same iterations as 64 back-to-back
    # iterate calls (no host synchronisation between them)
    t_prep = _timed(torch, prepare, reps=2)
    t_launch = _timed(torch, lambda: (prepare(), plan.launch()), reps=2) - t_prep

    def iterate_calls():
        for st in prepare():
            st.iterate(MAX_ITERS, EPS)

    t_calls = _timed(torch, iterate_calls, reps=2) - t_prep
    plan.close()
    n_pix = sum(g.numel() // 3 for g in imgs)
    return dict(workload=f"{n_images} images, side U[128,1024] (seeded), K from {{16,32,64,128,256}}, "
                         "WSM-C eps 1e-4, max 50 iterations, whole path per image",
                n_images=n_images, n_pixels=n_pix, sequential_ms=t_seq, batched_ms=t_bat,
                images_per_s_sequential=n_images / (t_seq * 1e-3),
                images_per_s_batched=n_images / (t_bat * 1e-3), speedup=t_seq / t_bat,
                persistent_launch_ms_est=t_launch, iterate_calls_ms_est=t_calls,
                speedup_launch_vs_iterate_calls=t_calls / t_launch, plan_create_ms=t_plan,
                images_per_s_batched_with_plan=n_images / ((t_bat + t_plan) * 1e-3),
                equal_palettes=bool(same),
                max_rel_mse_diff=max(abs(a - b) / b for a, b in zip(bat_mse, seq_mse)),
                batch_error_bits=err)


def bench_differentiable(torch, wsm, synth, B=16, size=512, K=64):
    """The differentiable configuration: 16 float32 512x512 images (the
    sinusoid-field generator), K = 64.  Forward: WSM on each image to the
    Sec. 3.2 stop (eps 1e-4, at most 50 iterations), then the distortion of
    Eq. 1 with the map's assignment frozen; backward: its adjoint for the
    pixels and the palettes.  The adjoint kernels are timed against torch
    autograd of the same expression (gather, square, mean)."""
    x = torch.from_numpy(np.stack([synth.sinusoid_field_image(s, size, size)
                                   for s in range(B)]).astype(np.float32)).to("cuda:0")
    fn = lambda n, k: synth.init_indices(0, n, k)  # noqa: E731
    t_fwd = _timed(torch, lambda: wsm.quantize_batch(x, K, fn), reps=2)
    pal, idx, _ = wsm.quantize_batch(x, K, fn)
    xf = x.reshape(B, -1, 3)

    def ours():
        xr = xf.detach().requires_grad_(True)
        pr = pal.detach().requires_grad_(True)
        wsm.distortion(xr, pr, idx).sum().backward()
        return xr.grad, pr.grad

    def plain():
        xr = xf.detach().requires_grad_(True)
        pr = pal.detach().requires_grad_(True)
        c = torch.gather(pr, 1, idx.long()[..., None].expand(-1, -1, 3))
        ((xr - c) ** 2).sum(-1).mean(-1).sum().backward()
        return xr.grad, pr.grad

    t_ours = _timed(torch, ours, reps=10)
    t_plain = _timed(torch, plain, reps=10)
    # the library's two calls alone (D, then both gradients) on preallocated
    # buffers: the kernels' share of the autograd step
    d_buf = torch.empty(B, dtype=torch.float64, device=x.device)
    g_buf = torch.ones(B, dtype=torch.float64, device=x.device)
    gx_buf = torch.empty_like(xf)
    gc_buf = torch.empty_like(pal)
    ws = wsm.distortion_workspace(B, xf.shape[1], K, x.device)
    t_kern = _timed(torch, lambda: wsm.distortion_into(xf, pal, idx, d_buf, ws, g_buf, gx_buf,
                                                       gc_buf), reps=20)
    gx, gc = ours()
    px, pc = plain()
    n_pix = size * size
    return dict(workload=f"{B} x {size}x{size} float32 sinusoid-field images, K={K}",
                forward_wsm_ms=t_fwd, adjoint_fwd_bwd_ms=t_ours, torch_autograd_fwd_bwd_ms=t_plain,
                speedup_vs_torch=t_plain / t_ours,
                bytes_fwd_bwd=float(B * n_pix * (13 + 13 + 12)),
                achieved_gbs=B * n_pix * (13 + 13 + 12) / (t_ours * 1e-3) / 1e9,
                kernels_fwd_bwd_ms=t_kern,
                kernels_achieved_gbs=B * n_pix * (13 + 13 + 12) / (t_kern * 1e-3) / 1e9,
                max_rel_diff_grad_x=float(((gx - px).abs().max() / px.abs().max()).item()),
                max_rel_diff_grad_palette=float(((gc - pc).abs().max() / pc.abs().max()).item()),
                images_per_s_forward_backward=B / ((t_fwd + t_ours) * 1e-3))


def bench_large(args, torch, wsm, synth, img_np):
    """Reduction and pixel map on the 4096x4096 workload (~2M unique colors,
    K = 256), each kernel timed per launch with events on its stream; and
    the whole image through WSM-C and through 10 fixed iterations."""
    dev = torch.device("cuda:0")
    N = img_np.shape[0] * img_np.shape[1]
    img = torch.from_numpy(img_np).to(dev)
    colors = torch.empty(min(N, 1 << 24), dtype=torch.int32, device=dev)
    counts = torch.empty_like(colors)
    nu = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(wsm.reduce_workspace_bytes(N), dtype=torch.uint8, device=dev)
    lut = torch.empty(1 << 24, dtype=torch.uint8, device=dev)
    reps = 10
    # a plain device copy of 256 MiB: the bandwidth this GPU reaches on a
    # stream of reads and writes, to set the fractions below against
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2.0 * src.numel() * 4 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    for _ in range(2):
        wsm.reduce_colors_into(img, colors, counts, nu, ws)
    torch.cuda.synchronize()
    timers = {}
    with wsm.kernel_timer("reduce_partition", reps) as kp:
        for _ in range(reps):
            wsm.reduce_colors_into(img, colors, counts, nu, ws)
    with wsm.kernel_timer("reduce_compact", reps) as kc:
        for _ in range(reps):
            wsm.reduce_colors_into(img, colors, counts, nu, ws)
    n_unique = int(nu.item())
    col, cnt = colors[:n_unique], counts[:n_unique]
    pal = wsm.palette_from_indices(col, synth.init_indices(0, n_unique, 256))
    st = wsm.init(col, cnt, N, pal)
    t_iter = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_iter[0].record()
    st.iterate(10, 0.0)
    t_iter[1].record()
    with wsm.kernel_timer("map_gather", reps) as kg:
        for _ in range(reps):
            wsm.map_pixels(st, img, lut=lut, want_mse=False)
    with wsm.kernel_timer("map_assign", reps) as ka:
        for _ in range(reps):
            wsm.map_pixels(st, img, lut=lut, want_mse=False)
    torch.cuda.synchronize()
    t_part = float(np.mean(kp.ms))
    t_comp = float(np.mean(kc.ms))
    t_gather = float(np.mean(kg.ms))
    t_assign = float(np.mean(ka.ms))
    red_bytes = 3.0 * N + 8.0 * n_unique
    map_bytes = 4.0 * N
    red_t = t_part + t_comp
    red_gbs = red_bytes / (red_t * 1e-3) / 1e9
    map_gbs = map_bytes / (t_gather * 1e-3) / 1e9
    red_traffic = REDUCE_TRAFFIC_BYTES if (
        REDUCE_TRAFFIC_BYTES is not None
        and kernel_sources_hash(_REDUCE_SOURCES) == REDUCE_TRAFFIC_SRC) else None
    map_traffic = GATHER_TRAFFIC_BYTES if (
        GATHER_TRAFFIC_BYTES is not None
        and kernel_sources_hash(_MAP_SOURCES) == GATHER_TRAFFIC_SRC) else None
    out = dict(
        workload="4096x4096 sinusoid-field image (seed 0, noise sigma 12), K=256",
        n_pixels=N, n_unique=n_unique, copy_gbs=copy_gbs,
        reduce=dict(bound="hbm", achieved=red_gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=red_gbs / HBM_PEAK_GBS, frac_of_copy=red_gbs / copy_gbs,
                    traffic=red_traffic, traffic_unit="bytes per call",
                    partition_us=t_part * 1e3, compact_us=t_comp * 1e3, bytes=red_bytes),
        map_gather=dict(bound="hbm", achieved=map_gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=map_gbs / HBM_PEAK_GBS, frac_of_copy=map_gbs / copy_gbs,
                        traffic=map_traffic, traffic_unit="bytes per launch",
                        avg_launch_us=t_gather * 1e3, bytes=map_bytes),
        map_assign_us=t_assign * 1e3,
        iterate_10_ms=t_iter[0].elapsed_time(t_iter[1]),
    )
    sse, ev = st.history()
    out["evals_per_color_per_iter"] = [float(e / n_unique) for e in ev]
    for name, (mi, eps) in (("whole_image_wsm_c", (MAX_ITERS, EPS)), ("whole_image_fixed10", (10, 0.0))):
        run, held = _whole_image(torch, wsm, synth, img, 256, mi, eps)
        ms = _timed(torch, run, reps=3)
        info = held["st"].info()
        out[name] = dict(ms_per_image=ms, images_per_s=1e3 / ms, iters=info["iters"],
                         converged=info["converged"], mse=float(held["mse"].item()),
                         color_iters_per_s=held["n_unique"] * info["iters"] / (ms * 1e-3))
    return out


def oracle_timings(small_np, large_np):
    """The FP64 oracle (plain C, one thread) on whole images: 100 runs of the
    256x256 workload (K = 32, WSM-C and 10 fixed iterations) and one run of
    the 4096x4096 workload (K = 256, 10 fixed iterations; its pixel map is a
    full search per pixel)."""
    import oracle
    import synth

    out = {}
    N = small_np.shape[0] * small_np.shape[1]
    for name, (mi, eps) in (("small_wsm_c", (MAX_ITERS, EPS)), ("small_fixed10", (10, 0.0))):
        t0 = time.perf_counter()
        runs = 100
        for _ in range(runs):
            col, cnt = oracle.reduce_colors(small_np)
            pal = synth.unpack_keys_to_palette(col[synth.init_indices(0, len(col), 32)])
            r = oracle.wsm(col, cnt, N, pal, mi, eps)
            oracle.map_pixels(small_np, col, r["m"], r["centers"])
        dt = (time.perf_counter() - t0) / runs
        out[name] = dict(ms_per_image=dt * 1e3, runs=runs, iters=r["iters"])
    if large_np is not None:
        NL = large_np.shape[0] * large_np.shape[1]
        t0 = time.perf_counter()
        col, cnt = oracle.reduce_colors(large_np)
        t1 = time.perf_counter()
        pal = synth.unpack_keys_to_palette(col[synth.init_indices(0, len(col), 256)])
        r = oracle.wsm(col, cnt, NL, pal, 10, 0.0)
        t2 = time.perf_counter()
        oracle.map_pixels(large_np, col, r["m"], r["centers"])
        t3 = time.perf_counter()
        out["large_fixed10"] = dict(s_per_image=t3 - t0, reduce_s=t1 - t0, iterate_s=t2 - t1,
                                    map_s=t3 - t2, runs=1, iters=r["iters"],
                                    color_iters_per_s=len(col) * r["iters"] / (t2 - t1))
    out["cores"] = 1
    return out


def cpu_baseline(args, img_np, Ks, n_unique_gpu):
    """The FP64 oracle (plain C, one thread) on whole steps of the same
    workload, repeated until about `cpu_seconds` of CPU time."""
    import oracle
    import synth

    N = img_np.shape[0] * img_np.shape[1]
    t0 = time.perf_counter()
    steps = 0
    color_iters = 0
    while True:
        col, cnt = oracle.reduce_colors(img_np)
        for K in Ks:
            pal = synth.unpack_keys_to_palette(col[synth.init_indices(args.seed, len(col), K)])
            r = oracle.wsm(col, cnt, N, pal, MAX_ITERS, EPS)
            oracle.map_pixels(img_np, col, r["m"], r["centers"])
            color_iters += len(col) * r["iters"]
        steps += 1
        if time.perf_counter() - t0 >= args.cpu_seconds:
            break
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(value=color_iters / dt, unit="color-iterations/s", cores=1, kind="oracle",
                sample=f"{steps} whole steps (reduce + K in {Ks} x (WSM-C + map)) of the same "
                       f"512x512 image, {dt:.1f} s, single-threaded C, {model}, "
                       f"host has {os.cpu_count()} logical CPUs",
                images_per_s=steps * len(Ks) / dt)


if __name__ == "__main__":
    main()

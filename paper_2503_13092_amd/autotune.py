"""Launch autotuner for the tracking and vertexing kernels.

Sweeps workgroup size, persistent workgroups per compute unit and (tracking
only) the number of hit bins per layer on a resident device batch, timing each
point with HIP events on the launch stream (median of `reps` launches), and
caches the winner per (device, workload signature) in a JSON file.  The
results are bitwise independent of these settings; only speed changes.
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np

from . import ds

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

TRACK_SPACE = dict(block=(64, 128, 256, 512), wg_per_cu=(1, 2, 4, 6, 8), bins=(128, 256, 512, 1024))
VERTEX_SPACE = dict(block=(64, 128, 256, 512), wg_per_cu=(1, 2, 4, 8))


def signature(batch) -> str:
    """Coarse workload key: events, mean/max seeds and hits per event (log2 buckets)."""
    s = np.diff(batch.seed_off)
    h = batch.hit_off[4::4] - batch.hit_off[0:-1:4]
    b = lambda v: int(round(math.log2(max(float(v), 1.0))))
    return f"E{b(batch.n_events)}-S{b(s.mean())}:{b(s.max())}-H{b(h.mean())}:{b(h.max())}"


def device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.name}-{getattr(p, 'gcnArchName', 'gfx')}"


def _time(fn, stream, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def sweep_track(ctx, ev, tr, points: Iterable[Tuple[int, int, int]], fuse: int = 1, reps: int = 5,
                stream=None) -> List[Dict]:
    import torch
    stream = stream or torch.cuda.current_stream()
    out = []
    for block, wpc, bins in points:
        if (4 * bins) % block:
            continue
        try:
            ds.ds_set_launch(ctx, 0, block, wpc, bins)
            ms = _time(lambda: ds.ds_find_tracks(ctx, ev, tr, ds.DS_MODE_PERSISTENT, fuse, stream), stream, reps)
        except ds.DsError as e:
            out.append(dict(block=block, wg_per_cu=wpc, bins=bins, ms=None, error=str(e)))
            continue
        out.append(dict(block=block, wg_per_cu=wpc, bins=bins, ms=ms))
    return out


def sweep_vertex(ctx, ev, tr, vt, score_max: float, points: Iterable[Tuple[int, int]], reps: int = 5,
                 stream=None) -> List[Dict]:
    import torch
    stream = stream or torch.cuda.current_stream()
    out = []
    for block, wpc in points:
        try:
            ds.ds_set_launch(ctx, 1, block, wpc, 0)
            ms = _time(lambda: ds.ds_vertex(ctx, ev, tr, score_max, vt, ds.DS_MODE_PERSISTENT, stream), stream,
                       reps)
        except ds.DsError as e:
            out.append(dict(block=block, wg_per_cu=wpc, ms=None, error=str(e)))
            continue
        out.append(dict(block=block, wg_per_cu=wpc, ms=ms))
    return out


def load_cache(path: str = CACHE) -> Dict:
    if os.path.exists(path):
        try:
            return json.load(open(path))
        except Exception:
            return {}
    return {}


def apply_cached(ctx, batch, path: str = CACHE) -> Optional[Dict]:
    """Set the cached launch settings for this device and workload, if any."""
    try:
        key = f"{device_name()}|{signature(batch)}"
    except Exception:
        return None
    entry = load_cache(path).get(key)
    if entry:
        t, v = entry["track"], entry["vertex"]
        ds.ds_set_launch(ctx, 0, t["block"], t["wg_per_cu"], t["bins"])
        ds.ds_set_launch(ctx, 1, v["block"], v["wg_per_cu"], 0)
    return entry


def autotune(ctx, batch, ev, tr, vt, score_max: float, reps: int = 5, path: Optional[str] = CACHE,
             track_space=TRACK_SPACE, vertex_space=VERTEX_SPACE, log=print) -> Dict:
    tpts = list(itertools.product(track_space["block"], track_space["wg_per_cu"], track_space["bins"]))
    tres = sweep_track(ctx, ev, tr, tpts, reps=reps)
    ok = [r for r in tres if r["ms"] is not None]
    best_t = min(ok, key=lambda r: r["ms"])
    ds.ds_set_launch(ctx, 0, best_t["block"], best_t["wg_per_cu"], best_t["bins"])
    ds.ds_find_tracks(ctx, ev, tr, ds.DS_MODE_PERSISTENT, 1)
    vpts = list(itertools.product(vertex_space["block"], vertex_space["wg_per_cu"]))
    vres = sweep_vertex(ctx, ev, tr, vt, score_max, vpts, reps=reps)
    okv = [r for r in vres if r["ms"] is not None]
    best_v = min(okv, key=lambda r: r["ms"])
    ds.ds_set_launch(ctx, 1, best_v["block"], best_v["wg_per_cu"], 0)
    entry = dict(track=best_t, vertex=best_v, track_sweep=tres, vertex_sweep=vres, when=time.time())
    if log:
        log(f"autotune: track best {best_t}, vertex best {best_v}")
    if path:
        cache = load_cache(path)
        cache[f"{device_name()}|{signature(batch)}"] = dict(track=best_t, vertex=best_v, when=entry["when"])
        tmp = path + ".tmp"
        json.dump(cache, open(tmp, "w"), indent=1)
        os.replace(tmp, path)
    return entry


def main(argv=None):
    from . import synth
    import torch
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--events", type=int, default=None)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-save", action="store_true")
    args = ap.parse_args(argv)
    g = synth.default_geometry()
    w = synth.mlp_weights()
    b = synth.generate(args.config, n_events=args.events)
    ctx = ds.Context(0, g, w)
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds, with_cand=False)
    vt = ds.DeviceVertices(b.n_events, 1024 if args.config == 4 else 64)
    sm = math.inf if args.config == 4 else g["ghost_threshold"]
    entry = autotune(ctx.handle, b, ev, tr, vt, sm, reps=args.reps, path=None if args.no_save else CACHE)
    for r in sorted((r for r in entry["track_sweep"] if r["ms"] is not None), key=lambda r: r["ms"])[:12]:
        print("track", r)
    for r in sorted((r for r in entry["vertex_sweep"] if r["ms"] is not None), key=lambda r: r["ms"])[:6]:
        print("vertex", r)
    torch.cuda.synchronize()
    ctx.close()


if __name__ == "__main__":
    main()

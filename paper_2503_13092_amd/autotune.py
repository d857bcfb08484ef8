"""Launch autotuner of the fused step (ds_process: tracking, ghost-killer and
vertexing in one persistent launch, replayed from a hipGraph).

Sweeps workgroup size, persistent workgroups per compute unit, hit bins per
layer and the event order (input order or largest first) on a resident device
batch, timing each point with HIP events on the launch stream (median of
`reps` graph replays), and caches the winner per (device, algorithm, workload
signature) in a JSON file that ships with the package.  Results are bitwise
independent of these settings (tested); only speed changes.  A point whose
LDS does not fit is refused by the library (DS_E_CAPACITY) and skipped.
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np

from . import ds

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

SPACE = dict(block=(128, 192, 256, 512), wg_per_cu=(1, 2, 3, 4, 6), bins=(256, 512, 1024),
             order=(ds.DS_ORDER_INPUT, ds.DS_ORDER_LARGEST_FIRST))
# the standalone vertexing launch (ds_vertex, and the step when it runs as two launches)
VERTEX_SPACE = dict(block=(64, 128, 256, 512), wg_per_cu=(2, 4, 5, 6, 8, 16))


def signature(batch) -> str:
    """Coarse workload key: events, mean/max seeds and hits per event (log2 buckets)."""
    s = np.diff(batch.seed_off)
    h = batch.hit_off[4::4] - batch.hit_off[0:-1:4]
    b = lambda v: int(round(math.log2(max(float(v), 1.0))))
    return f"E{b(batch.n_events)}-S{b(s.mean())}:{b(s.max())}-H{b(h.mean())}:{b(h.max())}"


def device_name() -> str:
    """The device as the cache knows it: ISA name and compute-unit count (the
    marketing name is not stable across drivers and tools)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = str(getattr(p, "gcnArchName", "gfx")).split(":")[0]
    return f"{arch}-{p.multi_processor_count}cu"


def cache_key(batch, algorithm: int) -> str:
    return f"{device_name()}|alg{int(algorithm)}|{signature(batch)}"


def _time(fn, stream, reps: int) -> float:
    import torch
    fn()
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


def set_point(ctx, pt: Dict) -> None:
    ds.ds_set_launch(ctx, 0, pt["block"], pt["wg_per_cu"], pt["bins"])
    ds.ds_set_event_order(ctx, pt["order"])
    ds.ds_set_step_fusion(ctx, pt.get("fused", 1))
    v = pt.get("vertex")
    if v:
        ds.ds_set_launch(ctx, 1, v["block"], v["wg_per_cu"], 0)


def sweep_vertex(ctx, ev, tr, vt, score_max: float, reps: int = 5, stream=None, space=VERTEX_SPACE) -> List[Dict]:
    """Times ds_vertex (graph mode) on the tracks in `tr` at every (block, wg_per_cu)."""
    import torch
    stream = stream or torch.cuda.current_stream()
    out = []
    for block, wpc in itertools.product(space["block"], space["wg_per_cu"]):
        try:
            ds.ds_set_launch(ctx, 1, block, wpc, 0)
            ms = _time(lambda: ds.ds_vertex(ctx, ev, tr, score_max, vt, ds.DS_MODE_GRAPH, stream), stream, reps)
        except ds.DsError as e:
            out.append(dict(block=block, wg_per_cu=wpc, ms=None, error=str(e)))
            continue
        out.append(dict(block=block, wg_per_cu=wpc, ms=ms))
    return out


def sweep_process(ctx, ev, tr, vt, score_max: float, points: Iterable[Tuple[int, int, int, int]], reps: int = 5,
                  stream=None, fused: int = 1) -> List[Dict]:
    """Times ds_process (graph mode) at every (block, wg_per_cu, bins, order) point."""
    import torch
    stream = stream or torch.cuda.current_stream()
    out = []
    for block, wpc, bins, order in points:
        pt = dict(block=block, wg_per_cu=wpc, bins=bins, order=order, fused=fused)
        try:
            set_point(ctx, pt)
            ms = _time(lambda: ds.ds_process(ctx, ev, tr, vt, ds.DS_MODE_GRAPH, score_max=score_max,
                                             stream=stream), stream, reps)
        except ds.DsError as e:
            out.append(dict(pt, ms=None, error=str(e)))
            continue
        out.append(dict(pt, ms=ms))
    return out


def load_cache(path: str = CACHE) -> Dict:
    if os.path.exists(path):
        try:
            with open(path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def apply_cached(ctx, batch, algorithm: int = 0, path: str = CACHE) -> Optional[Dict]:
    """Set the cached launch settings for this device, algorithm and workload;
    returns the entry (None: not tuned, the library defaults stay)."""
    try:
        key = cache_key(batch, algorithm)
    except Exception:
        return None
    entry = load_cache(path).get(key)
    if entry:
        set_point(ctx, entry["best"])
    return entry


def autotune(ctx, batch, ev, tr, vt, score_max: float, algorithm: int = 0, reps: int = 5,
             path: Optional[str] = CACHE, space=SPACE, log=print) -> Dict:
    import torch
    stream = torch.cuda.current_stream()
    # the vertexing launch first, on the tracks of one step
    ds.ds_process(ctx, ev, tr, vt, ds.DS_MODE_GRAPH, score_max=score_max, stream=stream)
    vres = sweep_vertex(ctx, ev, tr, vt, score_max, reps=reps, stream=stream)
    vbest = min((r for r in vres if r["ms"] is not None), key=lambda r: r["ms"])
    vpick = dict(block=vbest["block"], wg_per_cu=vbest["wg_per_cu"])
    ds.ds_set_launch(ctx, 1, vpick["block"], vpick["wg_per_cu"], 0)
    pts = list(itertools.product(space["block"], space["wg_per_cu"], space["bins"], space["order"]))
    res = sweep_process(ctx, ev, tr, vt, score_max, pts, reps=reps, stream=stream)
    ok = [r for r in res if r["ms"] is not None]
    best = {k: min(ok, key=lambda r: r["ms"])[k] for k in ("block", "wg_per_cu", "bins", "order")}
    best["fused"] = 1
    # the winner as two launches (tracking, then the standalone vertexing)
    res += sweep_process(ctx, ev, tr, vt, score_max, [(best["block"], best["wg_per_cu"], best["bins"], best["order"])],
                         reps=reps, stream=stream, fused=0)
    # confirm the winner against the library default with more repetitions
    default = dict(block=256, wg_per_cu=3, bins=1024, order=ds.DS_ORDER_INPUT, fused=1)
    confirm = {}
    for name, pt in (("best", best), ("unfused", dict(best, fused=0)), ("default", default)):
        set_point(ctx, pt)
        confirm[name] = _time(lambda: ds.ds_process(ctx, ev, tr, vt, ds.DS_MODE_GRAPH, score_max=score_max,
                                                    stream=stream), stream, 3 * reps)
    cands = [(confirm["best"], best), (confirm["unfused"], dict(best, fused=0)), (confirm["default"], default)]
    ms, pick = min(cands, key=lambda c: c[0])
    pick = dict(pick, vertex=vpick)
    set_point(ctx, pick)
    entry = dict(best=pick, ms=round(ms, 4), default_ms=round(confirm["default"], 4), n_events=batch.n_events,
                 vertex_ms=round(vbest["ms"], 4), when=round(time.time()))
    if log:
        log(f"autotune alg{algorithm} {signature(batch)}: best {pick} {entry['ms']} ms "
            f"(default {entry['default_ms']} ms)")
    if path:
        cache = load_cache(path)
        cache[cache_key(batch, algorithm)] = entry
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return dict(entry, sweep=res, vertex_sweep=vres)


def main(argv=None):
    from . import synth
    import torch
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--config", type=int, nargs="+", default=[1])
    ap.add_argument("--algorithm", type=int, default=0)
    ap.add_argument("--events", type=int, default=None)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=CACHE, help="cache file to update")
    args = ap.parse_args(argv)
    w = synth.mlp_weights()
    for config in args.config:
        g = dict(synth.default_geometry(), algorithm=args.algorithm)
        b = synth.generate(config, n_events=args.events)
        ctx = ds.Context(0, g, w)
        ev = ds.DeviceEvents(b)
        tr = ds.DeviceTracks(b.n_seeds, with_cand=False)
        vt = ds.DeviceVertices(b.n_events, 1024 if config == 4 else 64)
        sm = math.inf if config == 4 else g["ghost_threshold"]
        entry = autotune(ctx.handle, b, ev, tr, vt, sm, algorithm=args.algorithm, reps=args.reps, path=args.out)
        for r in sorted((r for r in entry["sweep"] if r["ms"] is not None), key=lambda r: r["ms"])[:8]:
            print(f"config {config} alg {args.algorithm}", r, flush=True)
        torch.cuda.synchronize()
        ctx.close()
        del ev, tr, vt


if __name__ == "__main__":
    main()

"""Benchmark of the Downstream tracking + vertexing hot path on one MI355X.

One step = the whole path (hit staging and window search, candidate fits and
selection, fused ghost-killer MLP, two-track vertexing) over one batch of
synthetic events resident in HBM: the 10 000-event throughput batch (150
seeds/event, 600 UT hits/layer) by default.  Steps rotate over four device
copies of the batch so the 256 MB Infinity Cache cannot serve it.

Prints one JSON line: whole-job events/s of the persistent, graph-replayed
launch; the same batch on the plain per-event-launch path; the roofline of
the dominant kernel (tracking) from its HIP-event-timed average duration; and
the FP64 CPU oracle timed on the host's cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FLOPS_PER_PAIR = 250.0   # straight-line start + 3 Newton steps of one opposite-charge pair, float64
PRESCREEN_FLOPS = 17.0   # the float32 straight-line DOCA test of one pair (differences, cross product, dot, squares)
FP32_VECTOR_PEAK_TFLOPS = 157.3
METRIC = "events/s/GPU (tracking+vertexing) and p99 event latency at fixed rate vs plain"
WORKLOADS = {
    1: "throughput batch: 10000 events x 150 seeds (40% true), 600 UT hits/layer, FP32 SoA",
    2: "uneven batch: 20000 events, pileup-scaled occupancy",
    4: "stress batch: 5000 events x 300 seeds, 1200 UT hits/layer, all-pairs vertexing",
}


# the workload part of the names of the rocprofv3 summaries under profiles/
PROFILE_TAG = {1: "throughput_10k", 2: "uneven_20k", 4: "stress_5k"}


def kernel_source_hash() -> str:
    from paper_2503_13092_amd.build_lib import kernel_source_hash as h
    return h()


def track_bytes_per_event(batch) -> float:
    """Algorithmic bytes of the tracking part of a step: the event in once
    (seed states 20 B/seed, hits 4 B/hit, offsets 20 B/event) and one 48 B
    track record per seed out (x, y, tx, ty, q/p, chi2, score, 4 hit indices,
    nhits).  The fused step adds 24 B per vertex and 4 B per event count."""
    S, H, E = batch.n_seeds, batch.n_hits, batch.n_events
    return (20.0 * S + 4.0 * H + 20.0 * E + 48.0 * S) / E


def vertex_bytes(batch, kept: int, n_vertices: int) -> float:  # the separate vertex launch
    """Algorithmic bytes of the vertex launch: nhits + score of every seed,
    the state (x, y, tx, ty, q/p) and charge of kept tracks, 24 B per vertex
    and a count per event."""
    return 8.0 * batch.n_seeds + 24.0 * kept + 24.0 * n_vertices + 8.0 * batch.n_events


def opposite_charge_pairs(batch, nhits, score, score_max) -> int:
    """Pairs of kept tracks with opposite seed charge, summed over events."""
    ev = np.repeat(np.arange(batch.n_events), np.diff(batch.seed_off))
    kept = (nhits > 0) & (score < score_max)
    pos = np.bincount(ev, weights=(kept & (batch.sqop > 0)).astype(np.float64), minlength=batch.n_events)
    neg = np.bincount(ev, weights=(kept & ~(batch.sqop > 0)).astype(np.float64), minlength=batch.n_events)
    return int(np.sum(pos * neg))


def prescreen_survivors(batch, trk, score_max, doca_max, curved, margin=0.1, chunk=64) -> int:
    """Host count of the opposite-charge pairs that the vertexing kernel's
    float32 straight-line test passes on to the float64 Newton fit (all of them
    when the trajectories curve).  numpy rounds each product separately where
    the kernel fuses multiply-adds, so pairs at the threshold may count
    differently: an estimate of the executed work, not a parity check."""
    x, y, tx, ty, nh, sc = (np.asarray(trk[k]) for k in ("x", "y", "tx", "ty", "nhits", "score"))
    so = batch.seed_off
    kept = (nh > 0) & (sc < score_max)
    pos = batch.sqop > 0
    if curved:
        return opposite_charge_pairs(batch, nh, sc, score_max)
    thr2 = np.float32((np.float32(doca_max) + np.float32(margin)) ** 2)
    idx = [np.nonzero(kept[so[e]:so[e + 1]])[0] + so[e] for e in range(batch.n_events)]
    by_n = {}
    for e, k in enumerate(idx):
        if len(k) > 1:
            by_n.setdefault(len(k), []).append(e)
    total = 0
    for n, evs in by_n.items():
        ia, ib = np.triu_indices(n, 1)
        for c0 in range(0, len(evs), chunk):
            K = np.stack([idx[e] for e in evs[c0:c0 + chunk]])      # [m, n] seed indices in slot order
            A, B = K[:, ia], K[:, ib]
            opp = pos[A] != pos[B]
            wx, wy = x[A] - x[B], y[A] - y[B]
            nx, ny = ty[A] - ty[B], tx[B] - tx[A]
            nz = tx[A] * ty[B] - ty[A] * tx[B]
            wn = wx * nx + wy * ny
            nn = nx * nx + ny * ny + nz * nz
            total += int(np.count_nonzero(opp & ((nn < np.float32(1e-6)) | (wn * wn < thr2 * nn))))
    return total


def stored_traffic(summary: str, src_hash: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary of
    that name (kernel and workload), if it was taken on the current kernel
    source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    e = d.get(summary)
    if not e or e.get("source_hash") != src_hash:
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(batch, g, w):
    """The oracle as it stands, on the host's cores, on a bounded sample."""
    from oracle import pyoracle as O
    try:
        n_threads = len(os.sched_getaffinity(0))
    except AttributeError:
        n_threads = os.cpu_count() or 1
    n_threads = max(1, min(n_threads, 16))
    # per-event cost from a short single-thread probe
    probe = batch.subset(np.arange(min(50, batch.n_events)))
    t0 = time.perf_counter()
    O.run_path(probe, g, w, cap=64, n_threads=1)
    per_event = (time.perf_counter() - t0) / probe.n_events
    # about 20 s of CPU work (single-thread seconds): the batch's first events,
    # or the whole batch run again as often as that takes (at most 4 passes)
    want = int(max(100, 20.0 / max(per_event, 1e-6)))
    n = int(min(batch.n_events, want))
    passes = int(min(4, max(1, round(want / max(n, 1)))))
    sample = batch.subset(np.arange(n))
    t0 = time.perf_counter()
    for _ in range(passes):
        O.run_path(sample, g, w, cap=64, n_threads=n_threads)
    dt = time.perf_counter() - t0
    n_done = n * passes
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=round(n_done / dt, 1), unit="events/s", cores=n_threads, kind="oracle",
                cpu_model=model, nproc=os.cpu_count(),
                sample=f"first {n} events of the batch x {passes} pass(es), whole path (tracks, ghost-killer, "
                       f"vertices), FP64, {n_threads} threads, {dt:.2f} s wall",
                single_thread_events_per_s=round(1.0 / per_event, 1))


def launch_settings(ds, ctx):
    block, wpc, bins = ds.ds_get_launch(ctx, 0)
    return dict(block=block, wg_per_cu=wpc, bins=bins,
                order="largest_first" if ds.ds_get_event_order(ctx) == ds.DS_ORDER_LARGEST_FIRST else "input",
                step="one fused launch" if ds.ds_get_step_fusion(ctx) else "tracking launch, then vertexing launch",
                vertex_launch=dict(zip(("block", "wg_per_cu"), ds.ds_get_launch(ctx, 1)[:2])))


def _timed(torch, stream, fn, warmup, reps):
    """Mean HIP-event time (ms) of fn on the launch stream, after warmup calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    pairs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps)]
    for p in pairs:
        p[0].record(stream)
        fn()
        p[1].record(stream)
    torch.cuda.synchronize()
    return float(np.mean([p[0].elapsed_time(p[1]) for p in pairs]))


def next_rows(ds, autotune, torch, g, w, batch, copies, mode, score_max, stream, warmup, reps):
    """The rows after the hot path, each on the same batch and launch mode:
    clone killing (the step with geometry clone_kill set: tracking, then the
    clone-killing and ghost-killer launches, then vertexing), every enumerated
    candidate scored (ds_score_candidates: one row per candidate, cleared and
    written every call), and the vertices' masses and trigger-line scores
    (ds_process with the extras outputs: the fused launch's extras
    instantiation)."""
    E = batch.n_events
    ev, tr, vt = copies[0]
    out = {}
    # clone killing
    ctx = ds.Context(0, dict(g, clone_kill=1), w)
    autotune.apply_cached(ctx.handle, batch, 0)
    ms = _timed(torch, stream, lambda: ds.ds_process(ctx.handle, ev, tr, vt, mode, score_max=score_max, stream=stream),
                warmup, reps)
    nh = tr.nhits.cpu().numpy()
    out["clone_killing"] = dict(ms_per_step=round(ms, 4), events_per_s=round(E / (ms * 1e-3), 1),
                                tracks=int(np.sum(nh > 0)), flags=int(tr.flags.item()) | int(vt.flags.item()),
                                launch="ds_process with clone_kill: tracking, clone-killing, ghost-killer and "
                                       "vertexing launches, hipGraph replay")
    ctx.close()
    # every candidate scored (a 56-byte row per valid candidate; every slot's nhits cleared first)
    ctx = ds.Context(0, g, w)
    slots = ds.ds_candidate_slots(ctx.handle)
    cd = ds.DeviceCandidates(batch.n_seeds, slots)
    ms = _timed(torch, stream, lambda: ds.ds_score_candidates(ctx.handle, ev, cd, stream=stream), warmup, reps)
    rows = int(np.sum(cd.nhits.cpu().numpy() > 0))
    written = 4.0 * batch.n_seeds * slots + 56.0 * rows
    out["all_candidates_scored"] = dict(ms=round(ms, 4), candidates=rows, slots_per_seed=slots,
                                        candidates_per_s=round(rows / (ms * 1e-3), 1),
                                        bytes_written_per_call=round(written),
                                        write_GBs=round(written / (ms * 1e-3) / 1e9, 1))
    del cd
    ctx.close()
    # masses and trigger lines after vertexing
    ctx = ds.Context(0, g, w)
    autotune.apply_cached(ctx.handle, batch, 0)
    ds.ds_load_lines(ctx.handle, synth_line_weights())
    vx = ds.DeviceVertices(batch.n_events, vt.cap, extras=True)
    ms = _timed(torch, stream, lambda: ds.ds_process(ctx.handle, ev, tr, vx, mode, score_max=score_max, stream=stream),
                warmup, reps)
    out["masses_and_lines"] = dict(ms_per_step=round(ms, 4), events_per_s=round(E / (ms * 1e-3), 1),
                                   vertices=int(vx.count.sum().item()),
                                   flags=int(tr.flags.item()) | int(vx.flags.item()),
                                   launch="ds_process with masses and trigger-line outputs (the extras "
                                          "instantiation of the fused launch), hipGraph replay")
    del vx
    ctx.close()
    return out


def synth_line_weights():
    from paper_2503_13092_amd import synth
    return synth.line_weights()


def copy_ceiling_gbs(torch, nbytes=2 << 30, reps=10):
    """Achievable HBM bandwidth of a plain device-to-device copy (read + write)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    return 2.0 * nbytes / dt / 1e9


def serving(g, w, seconds):
    """Open-loop Poisson arrivals of uneven (pileup-scaled) events at fixed
    rates; continuous batching over 3 in-flight slots vs the plain path (one
    launch per event per step).  Latency = completion - scheduled arrival."""
    from paper_2503_13092_amd import ds, serve, synth
    pool = serve.EventPool(synth.generate(2, n_events=8000))
    res = {}
    for name, kw in (("batched", dict(n_slots=3, max_events=512, mode=ds.DS_MODE_PERSISTENT)),
                     ("plain", dict(n_slots=1, max_events=1, mode=ds.DS_MODE_PER_EVENT))):
        be = serve.GpuBackend(pool, g, w, **kw)
        srv = serve.Server(be, pool)
        srv.run(serve.poisson_arrivals(20000.0, 2000, seed=9))   # warm-up: contexts, caches
        for rate in (20000.0, 50000.0, 100000.0):
            n = int(rate * seconds)
            _, st = srv.run(serve.poisson_arrivals(rate, n, seed=3), time_limit_s=4.0 * seconds + 2.0)
            d = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.as_dict().items()}
            d["offered"] = n
            res.setdefault(str(int(rate)), {})[name] = d
        be.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1, choices=(1, 2, 4))
    ap.add_argument("--copies", type=int, default=4, help="rotated device copies of the batch")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-dv1", action="store_true", help="skip the Dv1 (triplet search) line")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the next rows (clone killing, every candidate scored, masses and trigger lines)")
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for {args.gpus}); the path shards by "
              f"independent events, see the design notes", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_13092_amd import autotune, ds, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    g = synth.default_geometry()
    w = synth.mlp_weights()
    t0 = time.perf_counter()
    batch = synth.generate(args.config)
    gen_s = time.perf_counter() - t0
    E = batch.n_events
    score_max = math.inf if args.config == 4 else g["ghost_threshold"]
    cap = 1024 if args.config == 4 else 64

    ctx = ds.Context(0, g, w)
    tuned = autotune.apply_cached(ctx.handle, batch, 0)   # the autotuner's launch settings for this workload
    copies = []
    for _ in range(args.copies):
        ev = ds.DeviceEvents(batch)
        tr = ds.DeviceTracks(batch.n_seeds, with_cand=False)
        vt = ds.DeviceVertices(E, cap)
        copies.append((ev, tr, vt))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    mode = ds.DS_MODE_GRAPH

    def step(k, ev_pair=None):
        ev, tr, vt = copies[k % len(copies)]
        if ev_pair is not None:
            ev_pair[0].record(stream)
        ds.ds_process(ctx.handle, ev, tr, vt, mode, score_max=score_max, stream=stream)
        if ev_pair is not None:
            ev_pair[1].record(stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, events[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fused_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    ms_per_step = dt * 1e3 / args.steps
    value = E * args.steps / dt

    # checks on the last copy written
    ev, tr, vt = copies[(args.steps - 1) % len(copies)]
    flags = int(tr.flags.item()) | int(vt.flags.item())
    nh = tr.nhits.cpu().numpy()
    sc = tr.score.cpu().numpy()
    kept = int(np.sum((nh > 0) & (sc < score_max)))
    n_vtx = int(vt.count.sum().item())

    # the same step as two launches (tracking with the fused MLP, then vertexing), for reference
    a0, a1, a2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    trk_ms, vtx_ms = [], []
    for k in range(3):
        ev, tr, vt = copies[k % len(copies)]
        a0.record(stream)
        ds.ds_find_tracks(ctx.handle, ev, tr, mode, 1, stream)
        a1.record(stream)
        ds.ds_vertex(ctx.handle, ev, tr, score_max, vt, mode, stream)
        a2.record(stream)
        torch.cuda.synchronize()
        trk_ms.append(a0.elapsed_time(a1))
        vtx_ms.append(a1.elapsed_time(a2))
    trk_ms, vtx_ms = float(np.median(trk_ms)), float(np.median(vtx_ms))

    src_hash = kernel_source_hash()
    vb = vertex_bytes(batch, kept, n_vtx)
    bpe = track_bytes_per_event(batch)
    fused = bool(ds.ds_get_step_fusion(ctx.handle))
    if fused:
        # the step is the fused launch (plus, in largest-first order, two small sorting launches)
        step_bytes = bpe * E + 24.0 * n_vtx + 4.0 * E
        kms, kname, kkey = fused_ms, ("k_track: hit staging, search, fit, ghost-killer MLP and vertexing fused"
                                      + (", after the two event-order launches" if launch_settings(ds, ctx.handle)[
                                          "order"] == "largest_first" else "")), "k_track_fused"
    else:
        # two launches: the dominant one is tracking (the vertexing launch has its own flop roofline below)
        step_bytes = bpe * E
        kms, kname, kkey = trk_ms, "k_track: hit staging, search, fit and ghost-killer MLP", "k_track"
    achieved = step_bytes / (kms * 1e-3) / 1e9
    traffic = stored_traffic(f"{kkey}_{PROFILE_TAG.get(args.config, f'config{args.config}')}", src_hash)
    roofline = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5), traffic=traffic, kernel=kname,
                    kernel_ms=round(kms, 4), algorithmic_bytes_per_launch=round(step_bytes))
    opp = opposite_charge_pairs(batch, nh, sc, score_max)
    vflops = FLOPS_PER_PAIR * opp
    trk_host = {k: getattr(tr, k).cpu().numpy() for k in ("x", "y", "tx", "ty")}
    surv = prescreen_survivors(batch, dict(trk_host, nhits=nh, score=sc), score_max, g["doca_max"],
                               g.get("fringe_polarity", 0.0) != 0.0)
    # executed work: the float32 test on every opposite-charge pair, the float64 fit on its survivors
    xflops64 = FLOPS_PER_PAIR * surv
    xflops32 = PRESCREEN_FLOPS * opp
    mixed_peak = ((xflops64 + xflops32) / (xflops64 / FP64_VECTOR_PEAK_TFLOPS + xflops32 / FP32_VECTOR_PEAK_TFLOPS)
                  if xflops64 + xflops32 > 0 else FP64_VECTOR_PEAK_TFLOPS)
    vertex_info = dict(kept_tracks=kept, vertices=n_vtx, opposite_charge_pairs=opp, unfused_track_ms=round(trk_ms, 4),
                       unfused_vertex_ms=round(vtx_ms, 4), unfused_vertex_algorithmic_bytes=round(vb),
                       roofline=dict(bound="alu", unit="TFLOP/s", kernel="k_vertex (ds_vertex)",
                                     achieved=round((xflops64 + xflops32) / (vtx_ms * 1e-3) / 1e12, 3),
                                     peak=round(mixed_peak, 1),
                                     frac=round((xflops64 + xflops32) / (vtx_ms * 1e-3) / 1e12 / mixed_peak, 5),
                                     executed_fp64_flops=round(xflops64), executed_fp32_flops=round(xflops32),
                                     prescreen_survivors=surv,
                                     algorithmic_flops_per_launch=round(vflops),
                                     algorithmic_rate=round(vflops / (vtx_ms * 1e-3) / 1e12, 3),
                                     note="executed flops: the float32 straight-line test (17 flops) on every "
                                          "opposite-charge pair and the float64 fit (250 flops: start + 3 Newton "
                                          "steps) on the pairs it passes; peak: the float64 and float32 vector "
                                          "peaks weighted by those two counts.  algorithmic_rate counts 250 "
                                          "float64 flops on every opposite-charge pair, the method without the "
                                          "prescreen, and so exceeds what the ALUs execute"))

    out = dict(metric=METRIC, value=round(value, 1), unit="events/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64+f32", data="synthetic",
               config=dict(workload=WORKLOADS[args.config], events_per_step=E, seeds=batch.n_seeds,
                           hits=batch.n_hits, launch="ds_process: persistent launches replayed from a hipGraph",
                           rotated_copies=args.copies, launch_settings=launch_settings(ds, ctx.handle),
                           autotuned=tuned is not None),
               roofline=roofline, vertex=vertex_info, flags=flags, kernel_source=src_hash)

    if not args.no_plain:
        pe = []
        for k in range(args.plain_steps + 1):
            ev, tr, vt = copies[k % len(copies)]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ds.ds_find_tracks(ctx.handle, ev, tr, ds.DS_MODE_PER_EVENT, 1, stream)
            ds.ds_vertex(ctx.handle, ev, tr, score_max, vt, ds.DS_MODE_PER_EVENT, stream)
            torch.cuda.synchronize()
            if k > 0:
                pe.append(time.perf_counter() - t1)
        pdt = float(np.mean(pe))
        out["plain"] = dict(events_per_s=round(E / pdt, 1), ms_per_step=round(pdt * 1e3, 3),
                            launches_per_step=2 * E, speedup_of_persistent=round(value / (E / pdt), 2))
    if not args.no_dv1:
        # the same batch under Dv1 (triplet search, Y sectors), same launch
        g1 = dict(g, algorithm=1)
        ctx1 = ds.Context(0, g1, w)
        tuned1 = autotune.apply_cached(ctx1.handle, batch, 1)
        for k in range(args.warmup):
            ev, tr, vt = copies[k % len(copies)]
            ds.ds_process(ctx1.handle, ev, tr, vt, mode, score_max=score_max, stream=stream)
        torch.cuda.synchronize()
        ev_pairs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
        t1 = time.perf_counter()
        for k in range(args.steps):
            ev, tr, vt = copies[k % len(copies)]
            ev_pairs[k][0].record(stream)
            ds.ds_process(ctx1.handle, ev, tr, vt, mode, score_max=score_max, stream=stream)
            ev_pairs[k][1].record(stream)
        torch.cuda.synchronize()
        d1 = time.perf_counter() - t1
        ms1 = float(np.mean([e[0].elapsed_time(e[1]) for e in ev_pairs]))
        ev, tr, vt = copies[(args.steps - 1) % len(copies)]
        nh1 = tr.nhits.cpu().numpy()
        nv1 = int(vt.count.sum().item())
        ab1 = bpe * E + 24.0 * nv1 + 4.0 * E + 1.0 * batch.n_hits   # + the Y sector byte of every hit
        out["dv1"] = dict(events_per_s=round(E * args.steps / d1, 1), kernel_ms=round(ms1, 4),
                          achieved_GBs=round(ab1 / (ms1 * 1e-3) / 1e9, 2), algorithmic_bytes_per_launch=round(ab1),
                          traffic=stored_traffic("k_track_fused_dv1_throughput_10k", src_hash),
                          tracks=int(np.sum(nh1 > 0)), vertices=nv1,
                          flags=int(tr.flags.item()) | int(vt.flags.item()),
                          launch="ds_process, algorithm 1: one fused persistent launch, hipGraph replay",
                          launch_settings=launch_settings(ds, ctx1.handle), autotuned=tuned1 is not None)
        ctx1.close()
    if not args.no_next:
        out["next_rows"] = next_rows(ds, autotune, torch, g, w, batch, copies, mode, score_max, stream, args.warmup,
                                     max(5, args.steps // 2))
    if not args.no_copy_ceiling:
        cc = copy_ceiling_gbs(torch)
        out["roofline"]["copy_ceiling_GBs"] = round(cc, 1)
        out["roofline"]["frac_of_copy_ceiling"] = round(achieved / cc, 5)
    ctx.close()
    del copies
    if not args.no_serve:
        out["serving"] = serving(g, w, args.serve_seconds)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(batch, g, w)
    else:
        out["cpu_baseline"] = None
    out["generate_s"] = round(gen_s, 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

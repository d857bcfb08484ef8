"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes: configs 0-5 on subsets the oracle finishes in seconds (several
workgroup tiles and ragged tails), the loose-window mode, kick/polarity
variants, the curved-trajectory vertexer, edge cases, and the full 10 000
event throughput batch in the launch configuration the benchmark times
(checked on a sample of events).
"""
import math
import sys

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2503_13092_amd import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2503_13092_amd import ds  # noqa: E402

W = synth.mlp_weights()
G0 = synth.default_geometry()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = ds.Context(0, G0, W)
    yield c
    torch.cuda.synchronize()
    c.close()


def gpu_run(ctx_h, batch, mode=ds.DS_MODE_PERSISTENT, fuse=1, score_max=None, cap=1024, g=G0, vertex=True,
            max_hits=None, max_seeds=None):
    ev = ds.DeviceEvents(batch, max_hits_per_event=max_hits, max_seeds_per_event=max_seeds)
    tr = ds.DeviceTracks(batch.n_seeds)
    vt = ds.DeviceVertices(batch.n_events, cap)
    ds.ds_find_tracks(ctx_h, ev, tr, mode, fuse)
    if not fuse:
        ds.ds_ghost_kill(ctx_h, ev, tr)
    if vertex:
        sm = g["ghost_threshold"] if score_max is None else score_max
        ds.ds_vertex(ctx_h, ev, tr, sm, vt, mode)
    torch.cuda.synchronize()
    return tr.to_numpy(), (vt.to_numpy() if vertex else None)


def check_path(ctx_h, batch, g=G0, score_max=None, mode=ds.DS_MODE_PERSISTENT, label=""):
    say(f"[parity] {label}: {batch.n_events} events, {batch.n_seeds} seeds, {batch.n_hits} hits, mode {mode}")
    gt, gv = gpu_run(ctx_h, batch, mode=mode, score_max=score_max, g=g)
    sm = g["ghost_threshold"] if score_max is None else score_max
    ref = O.run_path(batch, g, W, score_max=sm, cap=1024, n_threads=8)
    tc = parity.compare_tracks(gt, ref["tracks"])
    found = ref["tracks"]["nhits"] > 0
    sc = parity.compare_scores(gt["score"], ref["score"], found & (gt["nhits"] == ref["tracks"]["nhits"]),
                               threshold=sm if math.isfinite(sm) else 0.5)
    vc = parity.compare_vertices(gv, ref["vertices"], g["doca_max"], parity.excused_slot_set(batch, tc, sc))
    assert gt["flags"] == 0 and gv["flags"] == 0
    say(f"[parity] {label}: identical {tc['identical']}/{tc['n']} (excused {len(tc['excused'])}), "
        f"found {tc['found']}, worst {tc['worst']}, score err {sc['worst']:.2e}, vertices {vc['n_gpu']}/{vc['n_ref']}")
    return gt, gv, ref


def test_config0_full(ctx):
    b = synth.generate(0)
    check_path(ctx.handle, b, label="config0")


@pytest.mark.parametrize("config,n", [(1, 300), (2, 400), (4, 60), (5, 8)])
def test_configs_subsets(ctx, config, n):
    b = synth.generate(config, n_events=n)
    sm = math.inf if config in (4, 5) else None
    check_path(ctx.handle, b, score_max=sm, label=f"config{config}x{n}")


def test_loose_windows_hit_the_caps(ctx):
    g = synth.default_geometry(loose=True)
    c = ds.Context(0, g, W)
    try:
        b = synth.generate(1, n_events=40, geometry=g)
        gt, _, ref = check_path(c.handle, b, g=g, label="loose")
        assert np.max(ref["tracks"]["cand"]) >= 36  # the 10th UTbX hit was used
    finally:
        torch.cuda.synchronize()
        c.close()


@pytest.mark.parametrize("kick,pol", [(1.2, 1.0), (1.2e-3, -1.0), (0.0, 1.0)])
def test_kick_variants(kick, pol):
    g = dict(G0, kick=kick, polarity=pol)
    c = ds.Context(0, g, W)
    try:
        b = synth.generate(0, n_events=60, geometry=g, seed=17)
        check_path(c.handle, b, g=g, score_max=math.inf, label=f"kick{kick}pol{pol}")
    finally:
        torch.cuda.synchronize()
        c.close()


def test_launch_modes_bitwise_equal(ctx):
    b = synth.generate(0, seed=3)
    outs = [gpu_run(ctx.handle, b, mode=m, score_max=math.inf) for m in (ds.DS_MODE_PER_EVENT,
                                                                          ds.DS_MODE_PERSISTENT, ds.DS_MODE_GRAPH)]
    outs.append(gpu_run(ctx.handle, b, mode=ds.DS_MODE_GRAPH, score_max=math.inf))  # graph replay
    for t, v in outs[1:]:
        for k in ("x", "y", "tx", "ty", "qop", "chi2", "score", "hits", "nhits", "cand"):
            assert np.array_equal(t[k], outs[0][0][k]), k
        for k in ("count", "i", "j", "x", "y", "z", "doca"):
            assert np.array_equal(v[k], outs[0][1][k]), k


def test_standalone_ghost_kill_equals_fused(ctx):
    b = synth.generate(1, n_events=50, seed=5)
    fused, _ = gpu_run(ctx.handle, b, fuse=1, vertex=False)
    alone, _ = gpu_run(ctx.handle, b, fuse=0, vertex=False)
    assert np.array_equal(fused["score"], alone["score"])


def test_process_graph_matches_separate_calls(ctx):
    b = synth.generate(0, seed=9)
    t1, v1 = gpu_run(ctx.handle, b, mode=ds.DS_MODE_PERSISTENT)
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds)
    vt = ds.DeviceVertices(b.n_events, 1024)
    for _ in range(3):
        ds.ds_process(ctx.handle, ev, tr, vt, ds.DS_MODE_GRAPH)
    torch.cuda.synchronize()
    t2, v2 = tr.to_numpy(), vt.to_numpy()
    for k in ("score", "hits", "nhits"):
        assert np.array_equal(t1[k], t2[k])
    for k in ("count", "i", "j", "x", "y", "z"):
        assert np.array_equal(v1[k], v2[k])


def test_hit_order_invariance_and_determinism(ctx):
    b = synth.generate(1, n_events=30, seed=23)
    t1, v1 = gpu_run(ctx.handle, b, score_max=math.inf)
    t1b, _ = gpu_run(ctx.handle, b, score_max=math.inf)
    for k in ("x", "score", "hits", "nhits"):
        assert np.array_equal(t1[k], t1b[k])
    rng = np.random.default_rng(1)
    perm = np.arange(b.n_hits)
    for k in range(4 * b.n_events):
        a, c = b.hit_off[k], b.hit_off[k + 1]
        perm[a:c] = a + rng.permutation(c - a)
    b2 = synth.EventBatch(b.n_events, b.seed_off, b.sx, b.sy, b.stx, b.sty, b.sqop, b.hit_off, b.hu[perm])
    t2, v2 = gpu_run(ctx.handle, b2, score_max=math.inf)
    assert np.array_equal(t1["nhits"], t2["nhits"]) and np.array_equal(t1["score"], t2["score"])
    for e in range(b.n_events):
        for i in range(b.seed_off[e], b.seed_off[e + 1]):
            for L in range(4):
                h1, h2 = t1["hits"][i, L], t2["hits"][i, L]
                if h1 < 0:
                    assert h2 < 0
                else:
                    base = b.hit_off[4 * e + L]
                    assert perm[base + h2] == base + h1


def test_vertexer_on_generated_track_states(ctx):
    """ds_vertex alone: the same float32 track states feed both sides."""
    s = synth.vertex_track_sample(n_events=40, n_pairs=6, n_random=40, seed=31)
    n = len(s["x"])
    E = len(s["seed_off"]) - 1
    b = synth.EventBatch(E, s["seed_off"], s["x"], s["y"], s["tx"], s["ty"], s["sqop"],
                         np.zeros(4 * E + 1, np.int32), np.zeros(0, np.float32))
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(n)
    for k in ("x", "y", "tx", "ty", "qop", "score"):
        getattr(tr, k).copy_(torch.from_numpy(s[k]))
    tr.nhits.copy_(torch.from_numpy(s["nhits"]))
    for fp in (0.0, 1.0, -1.0):
        g = dict(G0, fringe_polarity=fp)
        c = ds.Context(0, g, W)
        try:
            vt = ds.DeviceVertices(E, 256)
            ds.ds_vertex(c.handle, ev, tr, math.inf, vt, ds.DS_MODE_PERSISTENT)
            torch.cuda.synchronize()
            gv = vt.to_numpy()
            st = dict(x=s["x"], y=s["y"], tx=s["tx"], ty=s["ty"], qop=s["qop"], nhits=s["nhits"])
            rv = O.vertex(s["seed_off"], s["sqop"], st, s["score"].astype(np.float64), g, math.inf, 256)
            vc = parity.compare_vertices(gv, rv, g["doca_max"])
            say(f"[parity] vertexer fp={fp}: {vc['n_gpu']} vs {vc['n_ref']} vertices")
            assert vc["n_ref"] >= E * 3
        finally:
            torch.cuda.synchronize()
            c.close()


def test_vertex_cap_and_overflow(ctx):
    s = synth.vertex_track_sample(n_events=5, n_pairs=8, n_random=0, seed=2, smear=0.0)
    n = len(s["x"])
    E = 5
    b = synth.EventBatch(E, s["seed_off"], s["x"], s["y"], s["tx"], s["ty"], s["sqop"],
                         np.zeros(4 * E + 1, np.int32), np.zeros(0, np.float32))
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(n)
    for k in ("x", "y", "tx", "ty", "qop", "score"):
        getattr(tr, k).copy_(torch.from_numpy(s[k]))
    tr.nhits.copy_(torch.from_numpy(s["nhits"]))
    vt = ds.DeviceVertices(E, 3)
    ds.ds_vertex(ctx.handle, ev, tr, math.inf, vt, ds.DS_MODE_PERSISTENT)
    torch.cuda.synchronize()
    gv = vt.to_numpy()
    st = dict(x=s["x"], y=s["y"], tx=s["tx"], ty=s["ty"], qop=s["qop"], nhits=s["nhits"])
    rv = O.vertex(s["seed_off"], s["sqop"], st, s["score"].astype(np.float64), G0, math.inf, 3)
    assert list(gv["count"]) == list(rv["count"]) == [3] * E
    assert gv["overflow"] == rv["overflow"] > 0
    parity.compare_vertices(gv, rv, G0["doca_max"])


def test_edge_cases(ctx):
    seed = [100.0, 0.0, 0.0, 0.0, 0.25]
    evs = [dict(seeds=[], hits=[[], [], [], []]),
           dict(seeds=[seed], hits=[[], [], [], []]),
           dict(seeds=[], hits=[[1.0], [2.0], [3.0], [4.0]]),
           dict(seeds=[seed, seed], hits=[[100.0], [100.0, 100.0], [100.0], [100.0, 100.0]]),
           dict(seeds=[seed], hits=[[100.0], [100.0], [100.0], [float("nan")]]),
           dict(seeds=[[float("inf"), 0, 0, 0, 0.1]], hits=[[100.0], [100.0], [100.0], [100.0]])]
    b = synth.batch_from_lists(evs)
    g = dict(G0, kick=0.0)
    c = ds.Context(0, g, W)
    try:
        gt, gv = gpu_run(c.handle, b, g=g, score_max=math.inf)
        ref = O.find_tracks(b, g)
        assert list(gt["nhits"]) == list(ref["nhits"]) == [0, 4, 4, 0, 0]
        assert np.array_equal(gt["hits"], ref["hits"])
        assert gt["flags"] == ds.DS_F_NONFINITE
    finally:
        torch.cuda.synchronize()
        c.close()


def test_device_side_offset_and_capacity_checks(ctx):
    b = synth.generate(0, n_events=6)
    # an event above the declared capacity is flagged and skipped
    gt, _ = gpu_run(ctx.handle, b, max_hits=1000, vertex=False)
    assert gt["flags"] & ds.DS_F_CAPACITY and gt["nhits"].sum() == 0
    # non-monotone offsets: flagged, no write outside the event's seeds
    bad = synth.EventBatch(b.n_events, b.seed_off.copy(), b.sx, b.sy, b.stx, b.sty, b.sqop, b.hit_off.copy(), b.hu)
    bad.hit_off[5] = bad.hit_off[3] - 1
    ev = ds.DeviceEvents(bad, max_hits_per_event=4096, max_seeds_per_event=64)
    tr = ds.DeviceTracks(bad.n_seeds)
    ds.ds_find_tracks(ctx.handle, ev, tr, ds.DS_MODE_PERSISTENT, 1)
    torch.cuda.synchronize()
    out = tr.to_numpy()
    assert out["flags"] & ds.DS_F_BAD_OFFSETS
    assert out["nhits"][b.seed_off[1]:b.seed_off[2]].sum() == 0
    assert out["nhits"][b.seed_off[2]:].sum() > 0


def test_host_argument_errors(ctx):
    b = synth.generate(0, n_events=2)
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds)
    with pytest.raises(ds.DsError) as ei:
        ds.ds_find_tracks(ctx.handle, ev, tr, 7, 1)
    assert ei.value.status == ds.DS_E_ARG
    ev2 = ds.DeviceEvents(b, max_hits_per_event=10 ** 6)
    with pytest.raises(ds.DsError) as ei:
        ds.ds_find_tracks(ctx.handle, ev2, tr, ds.DS_MODE_PERSISTENT, 1)
    assert ei.value.status == ds.DS_E_CAPACITY
    c2 = ds.Context(0)
    try:
        with pytest.raises(ds.DsError) as ei:
            ds.ds_find_tracks(c2.handle, ev, tr, ds.DS_MODE_PERSISTENT, 1)
        assert ei.value.status == ds.DS_E_STATE
    finally:
        c2.close()


def test_full_throughput_batch_sampled(ctx):
    """The benchmark's 10 000-event batch, in its launch mode (graph-replayed
    persistent launch); 150 events checked against the oracle."""
    b = synth.generate(1)
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds)
    vt = ds.DeviceVertices(b.n_events, 64)
    say("[parity] full config1: running ds_process (graph)")
    ds.ds_process(ctx.handle, ev, tr, vt, ds.DS_MODE_GRAPH)
    torch.cuda.synchronize()
    gt, gv = tr.to_numpy(), vt.to_numpy()
    assert gt["flags"] == 0 and gv["flags"] == 0
    rng = np.random.default_rng(0)
    events = np.sort(rng.choice(b.n_events, 150, replace=False))
    sub = b.subset(events)
    ref = O.run_path(sub, G0, W, cap=64, n_threads=8)
    idx = np.concatenate([np.arange(b.seed_off[e], b.seed_off[e + 1]) for e in events])
    gsub = {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == (b.n_seeds,) else v) for k, v in gt.items()}
    tc = parity.compare_tracks(gsub, ref["tracks"])
    mask = (ref["tracks"]["nhits"] > 0) & (gsub["nhits"] == ref["tracks"]["nhits"])
    sc = parity.compare_scores(gsub["score"], ref["score"], mask)
    cap = 64
    gvs = dict(count=gv["count"][events], cap=cap, overflow=0, flags=0)
    for k in ("i", "j", "x", "y", "z", "doca"):
        gvs[k] = np.concatenate([gv[k][e * cap:(e + 1) * cap] for e in events])
    ref["vertices"]["overflow"] = 0
    parity.compare_vertices(gvs, ref["vertices"], G0["doca_max"], parity.excused_slot_set(sub, tc, sc))
    say(f"[parity] full config1 sample: identical {tc['identical']}/{tc['n']}")


@pytest.mark.parametrize("config,n,cap", [(4, 40, 1024), (2, 300, 1024), (1, 400, 1024), (4, 12, 16)])
def test_fused_process_graph_matches_oracle(ctx, config, n, cap):
    """The benchmark's launch (ds_process: one fused persistent launch of
    tracking, ghost-killer and vertexing, replayed from a hipGraph) against the
    oracle with every found track vertexed (score_max = inf): thousands of
    pairs per event at the stress occupancy, uneven events, and a cap of 16
    vertices per event so that the overflow count is exercised."""
    b = synth.generate(config, n_events=n, seed=50 + config)
    say(f"[parity] fused process config{config}x{n} cap {cap}: {b.n_seeds} seeds, {b.n_hits} hits")
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds)
    vt = ds.DeviceVertices(b.n_events, cap)
    ds.ds_process(ctx.handle, ev, tr, vt, ds.DS_MODE_GRAPH, score_max=math.inf)
    torch.cuda.synchronize()
    gt, gv = tr.to_numpy(), vt.to_numpy()
    assert gt["flags"] == 0 and gv["flags"] == 0
    ref = O.run_path(b, G0, W, score_max=math.inf, cap=cap, n_threads=8)
    tc = parity.compare_tracks(gt, ref["tracks"])
    found = ref["tracks"]["nhits"] > 0
    sc = parity.compare_scores(gt["score"], ref["score"], found & (gt["nhits"] == ref["tracks"]["nhits"]))
    vc = parity.compare_vertices(gv, ref["vertices"], G0["doca_max"], parity.excused_slot_set(b, tc, sc))
    if not (vc["only_gpu"] or vc["only_ref"]):
        assert np.array_equal(gv["count"], ref["vertices"]["count"])
        assert gv["overflow"] == ref["vertices"]["overflow"]
    if cap < 64:
        assert ref["vertices"]["overflow"] > 0
    say(f"[parity] fused process config{config}x{n}: identical {tc['identical']}/{tc['n']}, vertices "
        f"{vc['n_gpu']}/{vc['n_ref']}, overflow {gv['overflow']}/{ref['vertices']['overflow']}")
    # stored plus dropped: with a cap of 16 per event only 16 are stored
    assert vc["n_ref"] + ref["vertices"]["overflow"] > (1000 if config == 4 else 0)


def test_fused_vertexing_of_large_events_matches_oracle():
    """Events of 2 600 seeds with every found track vertexed (about 2 500
    kept tracks, about 1.5 M opposite-charge pairs and 50 000 vertices per
    event).
    At 256 lanes the fused step's row table (6 bytes per kept-track slot) no
    longer fits on the tracking kernel's dead buffers and takes LDS of its
    own; at 512 lanes it fits there.  Both, and the two-launch step (the
    standalone vertexing kernel, with its own LDS layout), match the oracle
    and each other bitwise."""
    cfg = dict(name="wide", n_events=3, seed=23, seeds_per_event=2600, llp_per_event=600, hits_per_layer=300,
               zmax=2200.0)
    b = synth.generate(cfg)
    cap = 65536
    say(f"[parity] large events: {b.n_seeds} seeds, {b.n_hits} hits")
    ref = O.run_path(b, G0, W, score_max=math.inf, cap=cap, n_threads=8)
    c = ds.Context(0, G0, W)
    outs = []
    try:
        for block, fused in ((256, 1), (512, 1), (256, 0)):
            ds.ds_set_launch(c.handle, 0, block, 1, 1024)
            ds.ds_set_step_fusion(c.handle, fused)
            say(f"[parity] large events: block {block}, fused {fused}")
            ev = ds.DeviceEvents(b)
            tr = ds.DeviceTracks(b.n_seeds)
            vt = ds.DeviceVertices(b.n_events, cap)
            ds.ds_process(c.handle, ev, tr, vt, ds.DS_MODE_PERSISTENT, score_max=math.inf)
            torch.cuda.synchronize()
            outs.append((tr.to_numpy(), vt.to_numpy()))
    finally:
        torch.cuda.synchronize()
        c.close()
    gt, gv = outs[0]
    assert gt["flags"] == 0 and gv["flags"] == 0
    tc = parity.compare_tracks(gt, ref["tracks"])
    found = ref["tracks"]["nhits"] > 0
    sc = parity.compare_scores(gt["score"], ref["score"], found & (gt["nhits"] == ref["tracks"]["nhits"]))
    vc = parity.compare_vertices(gv, ref["vertices"], G0["doca_max"], parity.excused_slot_set(b, tc, sc))
    assert vc["n_ref"] > 100000 and ref["vertices"]["overflow"] == 0
    for ot, ov in outs[1:]:
        for k in ("count", "i", "j", "x", "y", "z", "doca"):
            assert np.array_equal(ov[k], gv[k]), k
        for k in ("x", "y", "tx", "ty", "qop", "chi2", "score", "nhits"):
            assert np.array_equal(ot[k], gt[k]), k
    say(f"[parity] large events: identical {tc['identical']}/{tc['n']}, vertices {vc['n_gpu']}/{vc['n_ref']}")


def test_largest_first_order_matches_oracle_and_input_order():
    """Largest-first event order (two sorting launches ahead of the
    persistent launch): on uneven events every event is processed exactly
    once, results equal the oracle's and are bitwise those of the input
    order, in persistent and graph mode, on repeated calls (the sort's
    workspace is clean again after each) and after the workspace has grown."""
    c = ds.Context(0, G0, W)
    try:
        small = synth.generate(2, n_events=120, seed=71)
        big = synth.generate(2, n_events=700, seed=72)
        outs = {}
        for order in (ds.DS_ORDER_INPUT, ds.DS_ORDER_LARGEST_FIRST):
            ds.ds_set_event_order(c.handle, order)
            assert ds.ds_get_event_order(c.handle) == order
            for name, b in (("small", small), ("big", big), ("small2", small)):
                for mode in (ds.DS_MODE_PERSISTENT, ds.DS_MODE_GRAPH):
                    say(f"[order] order {order}, {name} ({b.n_events} events), mode {mode}")
                    ev = ds.DeviceEvents(b)
                    tr = ds.DeviceTracks(b.n_seeds)
                    vt = ds.DeviceVertices(b.n_events, 256)
                    for _ in range(2):
                        vt.overflow.zero_()   # the library only adds to it
                        ds.ds_process(c.handle, ev, tr, vt, mode, score_max=math.inf)
                    torch.cuda.synchronize()
                    outs[(order, name, mode)] = (tr.to_numpy(), vt.to_numpy())
        for key, (gt, gv) in outs.items():
            rt, rv = outs[(ds.DS_ORDER_INPUT, key[1], ds.DS_MODE_PERSISTENT)]
            for k in ("x", "y", "tx", "ty", "qop", "chi2", "score", "hits", "nhits"):
                assert np.array_equal(gt[k], rt[k]), (key, k)
            for k in ("count", "i", "j", "x", "y", "z", "doca"):
                assert np.array_equal(gv[k], rv[k]), (key, k)
        gt, gv = outs[(ds.DS_ORDER_LARGEST_FIRST, "big", ds.DS_MODE_GRAPH)]
        ref = O.run_path(big, G0, W, score_max=math.inf, cap=256, n_threads=8)
        tc = parity.compare_tracks(gt, ref["tracks"])
        found = ref["tracks"]["nhits"] > 0
        sc = parity.compare_scores(gt["score"], ref["score"], found & (gt["nhits"] == ref["tracks"]["nhits"]))
        vc = parity.compare_vertices(gv, ref["vertices"], G0["doca_max"], parity.excused_slot_set(big, tc, sc))
        say(f"[order] largest first, 700 uneven events: identical {tc['identical']}/{tc['n']}, "
            f"vertices {vc['n_gpu']}/{vc['n_ref']}")
        assert vc["n_ref"] > 0
    finally:
        torch.cuda.synchronize()
        c.close()


@pytest.mark.parametrize("fp", [1.0, -1.0])
def test_curved_daughters_path_matches_oracle(fp):
    """Daughters generated on eq. 4 parabolas before the UT (eq. 3 gamma,
    fringe polarity +-1): the fused graph step with every found track
    vertexed (the straight-line prescreen is off when gamma != 0, so every
    opposite-charge pair goes through the float64 Newton fit) equals the
    oracle track by track and vertex by vertex, and LLP daughter pairs are
    vertexed near their generated decay points."""
    g = dict(G0, fringe_polarity=fp)
    b = synth.generate(1, n_events=120, seed=60, geometry=g)
    c = ds.Context(0, g, W)
    try:
        say(f"[curved] fringe polarity {fp}: {b.n_seeds} seeds, {b.n_hits} hits")
        ev = ds.DeviceEvents(b)
        tr = ds.DeviceTracks(b.n_seeds)
        vt = ds.DeviceVertices(b.n_events, 1024)
        ds.ds_process(c.handle, ev, tr, vt, ds.DS_MODE_GRAPH, score_max=math.inf)
        torch.cuda.synchronize()
        gt, gv = tr.to_numpy(), vt.to_numpy()
    finally:
        torch.cuda.synchronize()
        c.close()
    assert gt["flags"] == 0 and gv["flags"] == 0
    ref = O.run_path(b, g, W, score_max=math.inf, cap=1024, n_threads=8)
    tc = parity.compare_tracks(gt, ref["tracks"])
    found = ref["tracks"]["nhits"] > 0
    sc = parity.compare_scores(gt["score"], ref["score"], found & (gt["nhits"] == ref["tracks"]["nhits"]))
    vc = parity.compare_vertices(gv, ref["vertices"], g["doca_max"], parity.excused_slot_set(b, tc, sc))
    t = b.truth
    dz = []
    for e in range(b.n_events):
        s0 = b.seed_off[e]
        for m in range(int(gv["count"][e])):
            k = e * gv["cap"] + m
            i, j = s0 + gv["i"][k], s0 + gv["j"][k]
            if t["seed_true"][i] and t["seed_llp"][i] == t["seed_llp"][j]:
                dz.append(abs(gv["z"][k] - t["seed_zdecay"][i]))
    say(f"[curved] fringe polarity {fp}: identical {tc['identical']}/{tc['n']}, vertices {vc['n_gpu']}/{vc['n_ref']}, "
        f"LLP vertices {len(dz)}, median |dz| {np.median(dz):.1f} mm")
    assert len(dz) >= 500 and np.median(dz) < 60.0


def _edge_event(rng, g, xs_ut, n_noise=40):
    """One hand-built event whose true tracks cross the UT near and beyond the
    hit-binning range |u| <= u_max: hits are forward-simulated from states
    before the kink (u = x - y tan(alpha) at each layer, 0.05 mm smear),
    seeds are the kinked lines at z_seed, and noise hits crowd the same
    u region on both sides of the range."""
    zl, tana, zr = np.asarray(g["z_layer"]), np.asarray(g["tan_stereo"]), g["z_ref"]
    hits = [[], [], [], []]
    secs = [[], [], [], []]
    seeds = []
    for k, x0 in enumerate(xs_ut):
        y0 = (300.0 if k % 2 else -250.0) + rng.uniform(-50, 50)
        txb, ty = x0 / 2500.0 + rng.normal(0, 0.01), y0 / 2500.0
        qop = (1.0 if k % 2 else -1.0) / rng.uniform(2.0, 20.0)
        for L in range(4):
            x = x0 + txb * (zl[L] - zr)
            y = y0 + ty * (zl[L] - zr)
            hits[L].append(x - y * tana[L] + rng.normal(0, g["sigma_hit"]))
            secs[L].append(int(synth.sector_of(y, g)))
        xm = x0 + txb * (g["z_magnet"] - zr)
        txa = txb + g["polarity"] * g["kick"] * qop
        seeds.append((xm + txa * (g["z_seed"] - g["z_magnet"]), y0 + ty * (g["z_seed"] - zr), txa, ty, qop))
    for L in range(4):
        for side in (1.0, -1.0):
            u = side * rng.uniform(g["u_max"] - 15.0, g["u_max"] + 60.0, n_noise)
            y = rng.uniform(-700, 700, n_noise)
            hits[L].extend(u.tolist())
            secs[L].extend(synth.sector_of(y, g).tolist())
    order = [rng.permutation(len(h)) for h in hits]
    return dict(seeds=seeds, hits=[[hits[L][i] for i in order[L]] for L in range(4)],
                sectors=[[secs[L][i] for i in order[L]] for L in range(4)])


@pytest.mark.parametrize("algorithm", [0, 1])
def test_hits_beyond_binning_range(algorithm):
    """Hits with u outside [u_min, u_max] land in the edge bins of the window
    lookup; windows that reach past the range must still select exactly what
    the oracle (full scans, no binning) selects."""
    g = dict(G0, algorithm=algorithm)
    rng = np.random.default_rng(23)
    evs = [_edge_event(rng, g, [855.0, 870.0, 905.0, -858.0, -880.0, -920.0]) for _ in range(6)]
    b = synth.batch_from_lists(evs)
    c = ds.Context(0, g, W)
    try:
        say(f"[parity] beyond binning range, algorithm {algorithm}: {b.n_seeds} seeds, {b.n_hits} hits")
        gt, gv = gpu_run(c.handle, b, g=g, score_max=math.inf)
        ref = O.run_path(b, g, W, score_max=math.inf, cap=1024)
        tc = parity.compare_tracks(gt, ref["tracks"])
        assert gt["flags"] == 0
        rt = ref["tracks"]
        assert (rt["nhits"] == 4).sum() >= 30
        outside = 0
        for e in range(b.n_events):
            for i in range(b.seed_off[e], b.seed_off[e + 1]):
                for L in range(4):
                    h = rt["hits"][i, L]
                    if h >= 0 and abs(b.hu[b.hit_off[4 * e + L] + h]) > g["u_max"]:
                        outside += 1
        assert outside >= 50, outside
        say(f"[parity] beyond binning range, algorithm {algorithm}: identical {tc['identical']}/{tc['n']}, "
            f"{outside} selected hits outside the range")
    finally:
        torch.cuda.synchronize()
        c.close()

def test_clone_killing_matches_oracle():
    g = dict(G0, clone_kill=1)
    c = ds.Context(0, g, W)
    try:
        for cfg, n in ((1, 200), (4, 40)):
            b = synth.generate(cfg, n_events=n, seed=31)
            ev = ds.DeviceEvents(b)
            tr = ds.DeviceTracks(b.n_seeds)
            ds.ds_find_tracks(c.handle, ev, tr, ds.DS_MODE_PERSISTENT, 0)
            ds.ds_kill_clones(c.handle, ev, tr)
            ds.ds_ghost_kill(c.handle, ev, tr)
            torch.cuda.synchronize()
            gt = tr.to_numpy()
            ref_tr = O.find_tracks(b, g, n_threads=8)
            st = O.stored_tracks(ref_tr)
            killed = O.kill_clones(b.seed_off, st)
            st2 = O.apply_kills(st, killed)
            assert killed.sum() > 0
            ref = dict(ref_tr)
            for k in ("nhits", "hits"):
                ref[k] = st2[k]
            ref["cand"] = np.where(killed > 0, -1, ref_tr["cand"])
            for k in ("x", "y", "tx", "ty", "qop", "chi2"):
                ref[k] = np.where(killed > 0, 0.0, ref_tr[k])
            tc = parity.compare_tracks(gt, ref)
            score = O.ghost_kill(b, st2, g, W)
            parity.compare_scores(gt["score"], score, st2["nhits"] > 0)
            say(f"[parity] clone kill config{cfg}: killed {int(killed.sum())}, identical {tc['identical']}/{tc['n']}")
            # the same through ds_process (graph) with clone_kill set
            vt = ds.DeviceVertices(b.n_events, 1024)
            tr2 = ds.DeviceTracks(b.n_seeds)
            ds.ds_process(c.handle, ev, tr2, vt, ds.DS_MODE_GRAPH, score_max=math.inf)
            torch.cuda.synchronize()
            t2 = tr2.to_numpy()
            for k in ("nhits", "hits", "score"):
                assert np.array_equal(t2[k], gt[k]), k
    finally:
        torch.cuda.synchronize()
        c.close()


def test_every_candidate_scored_matches_oracle():
    g = synth.default_geometry(loose=True)
    c = ds.Context(0, g, W)
    try:
        b = synth.generate(1, n_events=20, geometry=g, seed=8)
        slots = ds.ds_candidate_slots(c.handle)
        assert slots == 40
        ev = ds.DeviceEvents(b)
        cd = ds.DeviceCandidates(b.n_seeds, slots)
        ds.ds_score_candidates(c.handle, ev, cd)
        torch.cuda.synchronize()
        got = cd.to_numpy()
        ref = O.score_candidates(b, g, W)
        rows = ref["seed"].astype(np.int64) * slots + ref["cand"]
        present = np.zeros(b.n_seeds * slots, bool)
        present[rows] = True
        assert np.all(got["nhits"][~present] == 0)
        same = (got["nhits"][rows] == ref["nhits"]) & np.all(got["hits"][rows] == ref["hits"], axis=1)
        assert same.mean() >= 0.9999, same.mean()
        ok = rows[same]
        st = np.stack([got[k][ok] for k in ("x", "y", "tx", "ty", "qop", "chi2")], 1).astype(np.float64)
        rs = ref["state"][same]
        floors = np.array([1.0, 1.0, 1e-3, 1e-3, 1e-2, 1.0])
        assert np.max(np.abs(st - rs) / np.maximum(np.abs(rs), floors)) <= 1e-4
        assert np.max(np.abs(got["score"][ok] - ref["score"][same])) <= 1e-5
        say(f"[parity] candidate rows: {len(rows)} rows, identical {same.mean():.6f}")
    finally:
        torch.cuda.synchronize()
        c.close()


@pytest.mark.parametrize("algorithm", [0, 1])
def test_launch_shapes_bitwise_equal(algorithm):
    """Block size, workgroups per CU, hit bins, event order and step fusion
    (the autotuner's knobs) change chunking, scheduling, the bucket layout
    and the launches, never the results."""
    g = dict(G0, algorithm=algorithm)
    b = synth.generate(0, n_events=80, seed=23)
    c = ds.Context(0, g, W)
    try:
        outs = []
        for block, wpc, bins, order, fused in ((256, 3, 512, 0, 1), (64, 8, 512, 1, 1), (128, 4, 256, 0, 0),
                                               (512, 1, 1024, 1, 0), (256, 2, 128, 0, 1), (256, 3, 1024, 1, 0)):
            say(f"[parity] launch shape, algorithm {algorithm}: block {block}, {wpc} per CU, {bins} bins, "
                f"order {order}, fused {fused}")
            ds.ds_set_launch(c.handle, 0, block, wpc, bins)
            ds.ds_set_event_order(c.handle, order)
            ds.ds_set_step_fusion(c.handle, fused)
            ev = ds.DeviceEvents(b)
            tr = ds.DeviceTracks(b.n_seeds)
            vt = ds.DeviceVertices(b.n_events, 256)
            ds.ds_process(c.handle, ev, tr, vt, ds.DS_MODE_GRAPH, score_max=math.inf)
            torch.cuda.synchronize()
            outs.append((tr.to_numpy(), vt.to_numpy()))
        t0, v0 = outs[0]
        assert (t0["nhits"] > 0).sum() > 500 and t0["flags"] == 0
        for t, v in outs[1:]:
            for k in ("x", "y", "tx", "ty", "qop", "chi2", "score", "hits", "nhits"):
                assert np.array_equal(t[k], t0[k]), k
            for k in ("count", "i", "j", "x", "y", "z", "doca"):
                assert np.array_equal(v[k], v0[k]), k
    finally:
        torch.cuda.synchronize()
        c.close()


def test_vertex_launch_shapes_bitwise_equal():
    """The standalone vertexing launch (ds_vertex; the second launch of an
    unfused step) at the workgroup sizes and counts the autotuner picks from:
    the pair chunks, the survivor ring and the fit batches change with the
    workgroup size, the vertices never do.  Stress occupancy, every found
    track kept."""
    b = synth.generate(4, n_events=24, seed=61)
    c = ds.Context(0, G0, W)
    try:
        ev = ds.DeviceEvents(b)
        tr = ds.DeviceTracks(b.n_seeds)
        ds.ds_find_tracks(c.handle, ev, tr, ds.DS_MODE_PERSISTENT, 1)
        torch.cuda.synchronize()
        outs = []
        for block, wpc in ((256, 4), (64, 16), (128, 8), (512, 2), (256, 5)):
            say(f"[parity] vertex launch shape: block {block}, {wpc} per CU")
            ds.ds_set_launch(c.handle, 1, block, wpc, 0)
            vt = ds.DeviceVertices(b.n_events, 2048)
            ds.ds_vertex(c.handle, ev, tr, math.inf, vt, ds.DS_MODE_GRAPH)
            torch.cuda.synchronize()
            outs.append(vt.to_numpy())
        v0 = outs[0]
        assert v0["flags"] == 0 and v0["count"].sum() > 5000
        for v in outs[1:]:
            for k in ("count", "i", "j", "x", "y", "z", "doca", "overflow"):
                assert np.array_equal(v[k], v0[k]), k
    finally:
        torch.cuda.synchronize()
        c.close()


@pytest.mark.parametrize("algorithm", [0, 1])
def test_fused_step_masses_and_lines_match_standalone(algorithm):
    """ds_process with masses and trigger-line outputs (the fused launch's
    extras instantiation) against ds_find_tracks + ds_vertex, whose extras the
    test above pins to the oracle."""
    wl = synth.line_weights()
    g = dict(G0, algorithm=algorithm)
    b = synth.generate(0, n_events=60, seed=19)
    c = ds.Context(0, g, W)
    try:
        ds.ds_load_lines(c.handle, wl)
        outs = []
        for fused in (False, True):
            ev = ds.DeviceEvents(b)
            tr = ds.DeviceTracks(b.n_seeds)
            vt = ds.DeviceVertices(b.n_events, 256, extras=True)
            if fused:
                ds.ds_process(c.handle, ev, tr, vt, ds.DS_MODE_GRAPH, score_max=math.inf)
            else:
                ds.ds_find_tracks(c.handle, ev, tr, ds.DS_MODE_PERSISTENT, 1)
                ds.ds_vertex(c.handle, ev, tr, math.inf, vt, ds.DS_MODE_PERSISTENT)
            torch.cuda.synchronize()
            outs.append(vt.to_numpy())
        a, f = outs
        assert a["flags"] == 0 and f["flags"] == 0
        for k in ("count", "i", "j", "x", "y", "z", "doca"):
            assert np.array_equal(a[k], f[k]), k
        live = np.concatenate([np.arange(e * 256, e * 256 + int(a["count"][e])) for e in range(b.n_events)])
        assert len(live) > b.n_events
        for k in ("m_pipi", "m_ppi"):
            assert np.all(np.abs(a[k][live] - f[k][live]) <= 1e-5 * np.abs(a[k][live]) + 1e-4), k
        assert np.max(np.abs(a["lines"][live] - f["lines"][live])) <= 1e-6
        say(f"[parity] fused extras, algorithm {algorithm}: {len(live)} vertices")
    finally:
        torch.cuda.synchronize()
        c.close()


def test_vertex_masses_and_trigger_lines_match_oracle(ctx):
    wl = synth.line_weights()
    s = synth.vertex_track_sample(n_events=30, n_pairs=6, n_random=30, seed=41)
    n = len(s["x"])
    E = len(s["seed_off"]) - 1
    b = synth.EventBatch(E, s["seed_off"], s["x"], s["y"], s["tx"], s["ty"], s["sqop"],
                         np.zeros(4 * E + 1, np.int32), np.zeros(0, np.float32))
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(n)
    for k in ("x", "y", "tx", "ty", "qop", "score"):
        getattr(tr, k).copy_(torch.from_numpy(s[k]))
    tr.nhits.copy_(torch.from_numpy(s["nhits"]))
    vt = ds.DeviceVertices(E, 256, extras=True)
    with pytest.raises(ds.DsError):          # lines not loaded yet
        ds.ds_vertex(ctx.handle, ev, tr, math.inf, vt, ds.DS_MODE_PERSISTENT)
    ds.ds_load_lines(ctx.handle, wl)
    for fp in (0.0, 1.0):
        g = dict(G0, fringe_polarity=fp)
        c = ds.Context(0, g, W) if fp else ctx
        try:
            if fp:
                ds.ds_load_lines(c.handle, wl)
            vt = ds.DeviceVertices(E, 256, extras=True)
            ds.ds_vertex(c.handle, ev, tr, math.inf, vt, ds.DS_MODE_PERSISTENT)
            torch.cuda.synchronize()
            gv = vt.to_numpy()
            st = dict(x=s["x"], y=s["y"], tx=s["tx"], ty=s["ty"], qop=s["qop"], nhits=s["nhits"])
            rv = O.vertex(s["seed_off"], s["sqop"], st, s["score"].astype(np.float64), g, math.inf, 256,
                          line_weights=wl.astype(np.float64))
            parity.compare_vertices(gv, rv, g["doca_max"])
            G_ = parity.vertex_dict(gv)
            nchk = 0
            for e in range(E):
                for m in range(int(rv["count"][e])):
                    k = e * 256 + m
                    key = (e, int(rv["i"][k]), int(rv["j"][k]))
                    if key not in G_:
                        continue
                    mg = [mm for mm in range(int(gv["count"][e])) if (gv["i"][e * 256 + mm], gv["j"][e * 256 + mm]) == key[1:]][0]
                    kg = e * 256 + mg
                    assert abs(gv["m_pipi"][kg] - rv["m_pipi"][k]) <= 1e-4 * rv["m_pipi"][k] + 1e-3
                    assert abs(gv["m_ppi"][kg] - rv["m_ppi"][k]) <= 1e-4 * rv["m_ppi"][k] + 1e-3
                    assert np.max(np.abs(gv["lines"][kg] - rv["lines"][k])) <= 1e-5
                    nchk += 1
            say(f"[parity] masses and lines fp={fp}: {nchk} vertices checked")
            assert nchk > E
        finally:
            if fp:
                torch.cuda.synchronize()
                c.close()

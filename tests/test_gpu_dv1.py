"""Dv1 triplet search (Y sectors, no momentum window) on the GPU vs the FP64
oracle, element by element through the C ABI: generated configurations,
launch modes, the fused step, sector ids out of range, and the host check
for missing sectors."""
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
G1 = dict(synth.default_geometry(), algorithm=1)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = ds.Context(0, G1, W)
    yield c
    torch.cuda.synchronize()
    c.close()


def run(ctx_h, batch, mode=ds.DS_MODE_PERSISTENT, score_max=None, cap=1024, process=False):
    ev = ds.DeviceEvents(batch)
    tr = ds.DeviceTracks(batch.n_seeds)
    vt = ds.DeviceVertices(batch.n_events, cap)
    sm = G1["ghost_threshold"] if score_max is None else score_max
    if process:
        ds.ds_process(ctx_h, ev, tr, vt, mode, score_max=sm)
    else:
        ds.ds_find_tracks(ctx_h, ev, tr, mode, 1)
        ds.ds_vertex(ctx_h, ev, tr, sm, vt, mode)
    torch.cuda.synchronize()
    return tr.to_numpy(), vt.to_numpy()


def check(ctx_h, batch, label, score_max=None, mode=ds.DS_MODE_PERSISTENT, process=False):
    say(f"[dv1] {label}: {batch.n_events} events, {batch.n_seeds} seeds, {batch.n_hits} hits, mode {mode}")
    gt, gv = run(ctx_h, batch, mode=mode, score_max=score_max, process=process)
    sm = G1["ghost_threshold"] if score_max is None else score_max
    ref = O.run_path(batch, G1, W, score_max=sm, cap=1024, n_threads=8)
    tc = parity.compare_tracks(gt, ref["tracks"])
    found = ref["tracks"]["nhits"] > 0
    sc = parity.compare_scores(gt["score"], ref["score"], found & (gt["nhits"] == ref["tracks"]["nhits"]),
                               threshold=sm if math.isfinite(sm) else 0.5)
    vc = parity.compare_vertices(gv, ref["vertices"], G1["doca_max"], parity.excused_slot_set(batch, tc, sc))
    assert gt["flags"] == 0 and gv["flags"] == 0
    say(f"[dv1] {label}: identical {tc['identical']}/{tc['n']} (excused {len(tc['excused'])}), found "
        f"{tc['found']}, worst {tc['worst']}, score err {sc['worst']:.2e}, vertices {vc['n_gpu']}/{vc['n_ref']}")
    return gt, ref


def test_dv1_config0(ctx):
    b = synth.generate(0)
    gt, ref = check(ctx.handle, b, "config0", score_max=math.inf)
    assert (ref["tracks"]["nhits"] > 0).sum() > 500


@pytest.mark.parametrize("config,n", [(1, 40), (2, 120), (4, 10), (5, 4)])
def test_dv1_config_subsets(ctx, config, n):
    b = synth.generate(config, n_events=n, seed=31 + config)
    check(ctx.handle, b, f"config{config}")


def test_dv1_launch_modes_and_fused_step_bitwise_equal(ctx):
    b = synth.generate(0, n_events=60, seed=8)
    outs = [run(ctx.handle, b, mode=m, score_max=math.inf)
            for m in (ds.DS_MODE_PER_EVENT, ds.DS_MODE_PERSISTENT, ds.DS_MODE_GRAPH)]
    outs.append(run(ctx.handle, b, mode=ds.DS_MODE_GRAPH, score_max=math.inf, process=True))
    outs.append(run(ctx.handle, b, mode=ds.DS_MODE_GRAPH, score_max=math.inf, process=True))
    for t, v in outs[1:]:
        for k in ("x", "y", "tx", "ty", "qop", "chi2", "score", "hits", "nhits"):
            assert np.array_equal(t[k], outs[0][0][k]), k
        for k in ("count", "i", "j", "x", "y", "z", "doca"):
            assert np.array_equal(v[k], outs[0][1][k]), k


def test_dv1_out_of_range_sector_ids_are_never_compatible(ctx):
    b = synth.generate(0, n_events=30, seed=12)
    rng = np.random.default_rng(4)
    sec = b.hit_sector.copy()
    bad = rng.uniform(size=len(sec)) < 0.1
    sec[bad] = rng.integers(G1["n_sectors"], 256, bad.sum())
    b.hit_sector = sec
    check(ctx.handle, b, "bad sector ids", score_max=math.inf)


def test_dv1_finds_tracks_dv0_misses(ctx):
    """Seeds whose q/p estimate is off: Dv0's momentum window misses their
    UTbX hit, Dv1 finds them (the reason the paper gives for Dv1)."""
    b = synth.generate(0, n_events=20, seed=41)
    true = b.truth["seed_true"].astype(bool)
    b.sqop = np.where(true, -b.sqop * 3.0, b.sqop).astype(np.float32)
    g0 = dict(G1, algorithm=0)
    c0 = ds.Context(0, g0, W)
    try:
        t0, _ = run(c0.handle, b, score_max=math.inf)
    finally:
        torch.cuda.synchronize()
        c0.close()
    t1, ref = check(ctx.handle, b, "wrong q/p", score_max=math.inf)
    n0, n1 = (t0["nhits"][true] > 0).sum(), (t1["nhits"][true] > 0).sum()
    f0, f1 = (t0["nhits"][true] == 4).sum(), (t1["nhits"][true] == 4).sum()
    say(f"[dv1] wrong q/p: true seeds with a track Dv0 {n0} Dv1 {n1}; with 4 hits Dv0 {f0} Dv1 {f1}")
    assert n1 > n0 and f1 > f0


def test_dv1_needs_hit_sectors(ctx):
    b = synth.generate(0, n_events=4, seed=2)
    b.hit_sector = None
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds)
    with pytest.raises(ds.DsError):
        ds.ds_find_tracks(ctx.handle, ev, tr, ds.DS_MODE_PERSISTENT, 1)


def test_dv1_throughput_batch_sampled(ctx):
    """The 10 000-event batch under Dv1 in the benchmark's launch mode;
    40 events checked against the oracle."""
    b = synth.generate(1)
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds)
    vt = ds.DeviceVertices(b.n_events, 64)
    say("[dv1] full config1: ds_process (graph)")
    ds.ds_process(ctx.handle, ev, tr, vt, ds.DS_MODE_GRAPH)
    torch.cuda.synchronize()
    gt, gv = tr.to_numpy(), vt.to_numpy()
    assert gt["flags"] == 0 and gv["flags"] == 0
    events = np.sort(np.random.default_rng(3).choice(b.n_events, 40, replace=False))
    sub = b.subset(events)
    ref = O.run_path(sub, G1, W, cap=64, n_threads=8)
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
    parity.compare_vertices(gvs, ref["vertices"], G1["doca_max"], parity.excused_slot_set(sub, tc, sc))
    say(f"[dv1] full config1 sample: identical {tc['identical']}/{tc['n']}")

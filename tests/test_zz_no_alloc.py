"""ds_process_static (the entry point that allocates nothing: its work
counters and event order live in the library's static device array) against
ds_process in persistent mode, through the C ABI: bitwise-equal tracks and
vertices on two calls in a row, the second with a smaller batch, in both
event orders and on the clone-killing path (whose vertexing launch uses the
array's second pair of counters); oversized batches are refused."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from paper_2503_13092_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2503_13092_amd import ds  # noqa: E402

W = synth.mlp_weights()
TRACK_KEYS = ("x", "y", "tx", "ty", "qop", "chi2", "score", "hits", "nhits", "flags")
VERTEX_KEYS = ("count", "i", "j", "x", "y", "z", "doca", "overflow", "flags")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(ctx, b, static, score_max=math.inf, cap=64):
    ev = ds.DeviceEvents(b)
    tr = ds.DeviceTracks(b.n_seeds)
    vt = ds.DeviceVertices(b.n_events, cap)
    if static:
        ds.ds_process_static(ctx, ev, tr, vt, score_max=score_max)
    else:
        ds.ds_process(ctx, ev, tr, vt, ds.DS_MODE_PERSISTENT, score_max=score_max)
    torch.cuda.synchronize()
    return tr.to_numpy(), vt.to_numpy()


def assert_same(a, b, label):
    (ta, va), (tb, vb) = a, b
    for k in TRACK_KEYS:
        assert np.array_equal(ta[k], tb[k]), (label, "track", k)
    for k in VERTEX_KEYS:
        assert np.array_equal(va[k], vb[k]), (label, "vertex", k)


@pytest.mark.parametrize("clone_kill", [0, 1])
def test_static_entry_matches_process(clone_kill):
    g = dict(synth.default_geometry(), clone_kill=clone_kill)
    c = ds.Context(0, g, W)
    try:
        big = synth.generate(2, n_events=500, seed=81)
        small = synth.generate(1, n_events=150, seed=82)
        for order in (ds.DS_ORDER_LARGEST_FIRST, ds.DS_ORDER_INPUT):
            ds.ds_set_event_order(c.handle, order)
            for name, b in (("uneven x500", big), ("throughput x150", small)):
                say(f"[no-alloc] clone_kill {clone_kill}, order {order}, {name}: {b.n_seeds} seeds")
                got = run(c.handle, b, static=True)
                ref = run(c.handle, b, static=False)
                assert_same(got, ref, (clone_kill, order, name))
                assert got[0]["flags"] == 0 and got[1]["flags"] == 0
                say(f"[no-alloc] {name}: {int((got[0]['nhits'] > 0).sum())} tracks, "
                    f"{int(got[1]['count'].sum())} vertices, overflow {got[1]['overflow']}: identical")
    finally:
        torch.cuda.synchronize()
        c.close()


def test_static_entry_refuses_oversized_batches():
    c = ds.Context(0, synth.default_geometry(), W)
    try:
        b = synth.generate(0, n_events=4, seed=83)
        ev = ds.DeviceEvents(b)
        tr = ds.DeviceTracks(b.n_seeds)
        vt = ds.DeviceVertices(b.n_events, 16)
        ev.struct.n_events = ds.DS_STATIC_MAX_EVENTS + 1   # refused on the host, before any launch
        st = ds.library().ds_process_static(c.handle, C.byref(ev.struct), C.byref(tr.struct), C.c_float(0.5),
                                            C.byref(vt.struct), None)
        assert st == ds.DS_E_CAPACITY
        ev.struct.n_events = b.n_events
        ds.ds_process_static(c.handle, ev, tr, vt)
        torch.cuda.synchronize()
        assert tr.to_numpy()["flags"] == 0
    finally:
        torch.cuda.synchronize()
        c.close()

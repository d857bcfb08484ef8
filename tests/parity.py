"""Comparison of the HIP path with the oracle, with the stated tolerances.

Tracks: hit assignments and selected-candidate indices identical for at least
99.99 % of seeds; any difference must be excused by the oracle's own
diagnostics (a looked-at hit within 1e-4 mm of a window edge, competing chi2
within 1e-5 relative / 1e-6 absolute, or a |delta| tie within 1e-4 mm at a
rank cut).  Track parameters within 1e-4 relative (floors 1 mm, 1e-3,
1e-2 GeV^-1, 1).  Ghost-killer scores within 1e-5.  Vertices within 1e-3 mm
plus half a float32 ulp of the coordinate (the stored format; it matters only
for vertices beyond 16 m), DOCA within 1e-4 mm; a vertex present on one side only is excused if its DOCA
is within 1e-4 of the cut, its opening |d1 x d2| < 1e-3, or one of its tracks
was an excused mismatch or a keep/kill flip within 1e-5 of the threshold.
"""
from __future__ import annotations

import numpy as np

TRACK_FLOORS = dict(x=1.0, y=1.0, tx=1e-3, ty=1e-3, qop=1e-2, chi2=1.0)


def compare_tracks(gpu: dict, ref: dict, min_identical: float = 0.9999, check_cand: bool = True) -> dict:
    n = len(ref["nhits"])
    same = (gpu["nhits"] == ref["nhits"]) & np.all(gpu["hits"] == ref["hits"], axis=1)
    if check_cand and "cand" in gpu:
        same &= gpu["cand"] == ref["cand"]
    bad = np.nonzero(~same)[0]
    excused = []
    unexcused = []
    for i in bad:
        chi2 = abs(ref["chi2"][i])
        if (ref["edge_margin"][i] < 1e-4 or ref["chi2_gap"][i] < max(1e-5 * chi2, 1e-6)
                or ref["rank_gap"][i] < 1e-4):
            excused.append(int(i))
        else:
            unexcused.append(int(i))
    frac = same.mean() if n else 1.0
    assert not unexcused, f"{len(unexcused)} unexcused track mismatches, first seeds {unexcused[:5]}: " + \
        "; ".join(f"gpu n={gpu['nhits'][i]} hits={gpu['hits'][i]} cand={gpu.get('cand', [None]*n)[i]} vs "
                  f"ref n={ref['nhits'][i]} hits={ref['hits'][i]} cand={ref['cand'][i]}" for i in unexcused[:3])
    assert frac >= min_identical, f"only {frac:.6f} of seeds identical"
    # parameters of identical tracks
    found = same & (ref["nhits"] > 0)
    worst = {}
    for k, floor in TRACK_FLOORS.items():
        g = gpu[k][found].astype(np.float64)
        r = ref[k][found]
        err = np.abs(g - r) / np.maximum(np.abs(r), floor)
        worst[k] = float(err.max()) if err.size else 0.0
        assert worst[k] <= 1e-4, f"track {k}: max relative error {worst[k]:.3g}"
    return dict(n=n, identical=int(same.sum()), excused=excused, worst=worst, found=int(found.sum()))


def compare_scores(gpu_score, ref_score, mask, threshold=0.5):
    d = np.abs(gpu_score[mask].astype(np.float64) - ref_score[mask])
    worst = float(d.max()) if d.size else 0.0
    assert worst <= 1e-5, f"ghost score: max abs error {worst:.3g}"
    flips = np.nonzero(mask & ((gpu_score < threshold) != (ref_score < threshold)))[0]
    for i in flips:
        assert abs(ref_score[i] - threshold) < 1e-5, f"keep/kill flip at seed {i} far from the threshold"
    return dict(worst=worst, flips=[int(i) for i in flips])


def vertex_dict(v: dict, with_opening=False):
    out = {}
    cap = v["cap"]
    for e, c in enumerate(v["count"]):
        for m in range(int(c)):
            k = e * cap + m
            out[(e, int(v["i"][k]), int(v["j"][k]))] = (float(v["x"][k]), float(v["y"][k]), float(v["z"][k]),
                                                         float(v["doca"][k]),
                                                         float(v["opening"][k]) if with_opening else 0.0)
    return out


def compare_vertices(gpu: dict, ref: dict, doca_max: float, excused_slots=None, seed_off=None) -> dict:
    """``excused_slots`` is a set of (event, slot) whose track differs for an
    excused reason; vertices involving them may differ."""
    G = vertex_dict(gpu)
    R = vertex_dict(ref, with_opening=True)
    excused_slots = excused_slots or set()
    for key, (x, y, z, d, _) in G.items():
        if key in R:
            rx, ry, rz, rd, _ = R[key]
            # positions are stored as float32: 1e-3 mm plus half a float32 ulp
            # of the value (nearly parallel pairs can meet tens of metres away)
            tol = lambda r: 1e-3 + 0.5 * float(np.spacing(np.float32(abs(r))))
            assert abs(x - rx) <= tol(rx) and abs(y - ry) <= tol(ry) and abs(z - rz) <= tol(rz), \
                f"vertex {key}: gpu {(x, y, z)} vs ref {(rx, ry, rz)}"
            assert abs(d - rd) <= 1e-4, f"vertex {key}: doca {d} vs {rd}"
    only_g = [k for k in G if k not in R]
    only_r = [k for k in R if k not in G]
    for k in only_g + only_r:
        e, i, j = k
        if (e, i) in excused_slots or (e, j) in excused_slots:
            continue
        src = R.get(k) or G.get(k)
        if abs(src[3] - doca_max) < 1e-4:
            continue
        if k in R and R[k][4] < 1e-3:
            continue
        raise AssertionError(f"vertex {k} only on the {'gpu' if k in G else 'oracle'} side: {src}")
    assert gpu["overflow"] == ref["overflow"] or only_g or only_r
    return dict(n_gpu=len(G), n_ref=len(R), only_gpu=only_g, only_ref=only_r)


def excused_slot_set(batch, track_cmp: dict, score_cmp: dict = None):
    """(event, slot) pairs whose track or keep decision may legitimately differ."""
    seeds = list(track_cmp["excused"]) + (list(score_cmp["flips"]) if score_cmp else [])
    ev = np.searchsorted(batch.seed_off, np.asarray(seeds, dtype=np.int64), side="right") - 1
    return {(int(e), int(s - batch.seed_off[e])) for e, s in zip(ev, seeds)}

"""Pins of the oracle's Dv1 triplet search ("Algorithm Design", the improved
version): hits grouped into Y sectors, every UTbX hit of a compatible sector
joined to the magnet point, the line required to meet a UTaX hit, stereo hits
added as in Dv0.  CPU only."""
import itertools

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2503_13092_amd import synth

G1 = dict(synth.default_geometry(), algorithm=1)


def geom(**kw):
    g = dict(G1)
    g.update(kw)
    return g


def compatible_sectors(g, y):
    """Bands [y0 + k h, y0 + (k + 1) h) that overlap [y - tol, y + tol],
    found by testing every band (no floor formula)."""
    out = set()
    for k in range(g["n_sectors"]):
        lo = g["sector_y0"] + k * g["sector_h"]
        hi = lo + g["sector_h"]
        if lo <= y + g["sector_tol"] and hi > y - g["sector_tol"]:
            out.add(k)
    return out


def brute_dv1(g, seed, layers, sectors):
    """Exhaustive Dv1 enumeration: membership and ranks by counting over the
    whole layer, compatible sectors by band overlap, every option tuple."""
    xb, yl, xm = O.extrapolate(g, seed)
    W2 = g["w2_c0"] + g["w2_c1"] * abs(seed[4])
    ta = g["tan_stereo"]
    xhat = [np.asarray(layers[L], float) + yl[L] * ta[L] for L in range(4)]
    u = [np.asarray(layers[L], float) for L in range(4)]
    ok = [compatible_sectors(g, yl[L]) for L in range(4)]

    def ranked(L, centre, cap):
        d = np.abs(xhat[L] - centre)
        members = [i for i in range(len(d)) if d[i] <= W2 and int(sectors[L][i]) in ok[L]]
        out = {}
        for i in members:
            r = sum(1 for j in members if (d[j], u[L][j], j) < (d[i], u[L][i], i))
            if r < cap:
                out[r] = i
        return out

    caps = list(g["n_closest"])
    nw = [max(c, 1) for c in caps]
    cands = []
    for h3 in range(len(u[3])):
        if int(sectors[3][h3]) not in ok[3]:
            continue
        # the straight line through the magnet point and the UTbX hit
        slope = (xm - xhat[3][h3]) / (g["z_magnet"] - g["z_layer"][3])
        opts = []
        for L in range(3):
            xr = xhat[3][h3] + slope * (g["z_layer"][L] - g["z_layer"][3])
            rk = ranked(L, xr, caps[L])
            opts.append(sorted(rk.items()) if rk else [(0, -1)])
        if opts[0][0][1] < 0:
            continue  # no UTaX hit: no triplet
        for (i0, h0), (i1, h1), (i2, h2) in itertools.product(*opts):
            c = ((h3 * nw[0] + i0) * nw[1] + i1) * nw[2] + i2
            hits = [h0, h1, h2, h3]
            pts = [(g["z_layer"][L] - g["z_ref"], xhat[L][hits[L]]) for L in range(4) if hits[L] >= 0]
            A = np.array([[1.0, p[0]] for p in pts])
            y = np.array([p[1] for p in pts])
            sol, *_ = np.linalg.lstsq(A, y, rcond=None)
            chi2 = float(np.sum(((y - A @ sol) / g["sigma_hit"]) ** 2))
            cands.append((c, hits, len(pts), len(pts) >= 3, chi2))
    return cands


def _event(rng, g, n_hits, spread, n_sec_span=2):
    """A seed; hits near lines through its magnet point (so that triplets
    form) and scattered around its kinked predictions; random Y sectors drawn
    from the bands around the seed's height (some compatible)."""
    seed = [rng.uniform(-300, 300), rng.uniform(-500, 500), rng.uniform(-0.1, 0.1),
            rng.uniform(-0.08, 0.08), rng.choice([-1, 1]) / rng.uniform(2, 100)]
    xb, yl, xm = O.extrapolate(g, seed)
    slopes = (xm - xb[3]) / (g["z_magnet"] - g["z_layer"][3]) + rng.uniform(-spread, spread, 3) / 2000.0
    layers, sectors = [], []
    for L in range(4):
        on_line = rng.integers(0, 3, n_hits[L])
        xl = xm + slopes[on_line] * (g["z_layer"][L] - g["z_magnet"]) + rng.normal(0.0, 0.2, n_hits[L])
        xh = np.where(rng.uniform(size=n_hits[L]) < 0.6, xl, xb[L] + rng.uniform(-spread, spread, n_hits[L]))
        layers.append(list(xh - yl[L] * g["tan_stereo"][L]))
        k0 = int(np.clip(np.floor((yl[L] - g["sector_y0"]) / g["sector_h"]), 0, g["n_sectors"] - 1))
        off = np.where(rng.uniform(size=n_hits[L]) < 0.7, 0, rng.integers(-n_sec_span, n_sec_span + 1, n_hits[L]))
        sec = np.clip(k0 + off, 0, g["n_sectors"] - 1)
        sectors.append(list(sec))
    return seed, layers, sectors


@pytest.mark.parametrize("mode", ["default", "dense", "boundary"])
def test_dv1_candidates_match_bruteforce(mode):
    rng = np.random.default_rng({"default": 11, "dense": 12, "boundary": 13}[mode])
    g = geom()
    n_cases = 0
    for trial in range(60):
        nh = [int(rng.integers(0, 10 if mode != "dense" else 40)) for _ in range(4)]
        if trial % 7 == 0:
            nh[int(rng.integers(0, 4))] = 0
        seed, layers, sectors = _event(rng, g, nh, 3.0 if mode != "dense" else 2.0)
        if mode == "boundary":
            # put the seed's height within the tolerance of a sector boundary
            _, yl, _ = O.extrapolate(g, seed)
            k = int(np.floor((yl[3] - g["sector_y0"]) / g["sector_h"]))
            edge = g["sector_y0"] + (k + 1) * g["sector_h"]
            dy = edge - yl[3] + rng.uniform(-0.9, 0.9) * g["sector_tol"]
            seed[1] += dy
        ref = brute_dv1(g, seed, layers, sectors)
        got = O.candidates(g, seed, layers, sectors=sectors, max_out=20000)
        assert got["total"] == len(ref)
        for k, (c, hits, n, valid, chi2) in enumerate(ref):
            assert got["c"][k] == c
            assert list(got["hits"][k]) == hits
            assert got["nhits"][k] == n
            assert bool(got["valid"][k]) == valid
            assert got["chi2"][k] == pytest.approx(chi2, rel=1e-8, abs=1e-8)
        n_cases += len(ref)
    assert n_cases > (30 if mode == "boundary" else 50)


def test_sector_bands_at_boundaries():
    """Compatible bands by overlap, at and around exact boundaries."""
    g = geom(sector_tol=5.0)
    h, y0 = g["sector_h"], g["sector_y0"]
    # y - tol exactly on the boundary of bands 2|3: only band 3 (bands are [lo, hi))
    assert compatible_sectors(g, y0 + 3 * h + 5.0) == {3}
    # straddling 2|3
    assert compatible_sectors(g, y0 + 3 * h) == {2, 3}
    # outside the detector: none
    assert compatible_sectors(g, y0 - 10.0) == set()
    assert compatible_sectors(g, y0 + g["n_sectors"] * h + 10.0) == set()
    # the oracle agrees: a seed with its UTbX height just above a boundary sees band k only
    seed = [0.0, 0.0, 0.0, 0.0, 0.5]
    _, yl, _ = O.extrapolate(g, seed)
    for y_target, hit_sec, expect in ((y0 + 3 * h + 5.0, 2, 0), (y0 + 3 * h + 5.0, 3, 1),
                                      (y0 + 3 * h + 4.0, 2, 1), (y0 - 10.0, 0, 0)):
        s = list(seed)
        s[1] = y_target  # ty = 0: the height is the same in every layer
        layers = [[0.0], [0.0], [0.0], [0.0]]
        sectors = [[hit_sec]] * 4
        got = O.candidates(g, s, layers, sectors=sectors)
        assert got["total"] == expect


def _straight_event(g, seed_true, qop_seed):
    """Exact hits of a track through the magnet point, seen by a seed whose
    q/p estimate is replaced by qop_seed."""
    x0, y0, tx, ty, qop = seed_true
    xm = x0 + tx * (g["z_magnet"] - g["z_seed"])
    tb = tx - g["polarity"] * g["kick"] * qop
    layers, sectors = [], []
    for L in range(4):
        x = xm + tb * (g["z_layer"][L] - g["z_magnet"])
        y = y0 + ty * (g["z_layer"][L] - g["z_seed"])
        layers.append([x - y * g["tan_stereo"][L]])
        sectors.append([int(synth.sector_of(y, g))])
    return [x0, y0, tx, ty, qop_seed], layers, sectors


@pytest.mark.parametrize("qop_true,qop_seed", [(0.5, -0.5), (0.1, 2.0), (-1.0, -0.05)])
def test_dv1_needs_no_momentum_window(qop_true, qop_seed):
    """The paper's reason for Dv1: the triplet uses only the magnet point and
    the axial hits, so a track whose seed q/p is far off is still found, with
    the true q/p from the kink.  Dv0's momentum window misses the same hit."""
    g = geom(kick=1.2e-3)
    seed, layers, sectors = _straight_event(g, [150.0, 80.0, 0.05, 0.02, qop_true], qop_seed)
    got = O.candidates(g, seed, layers, sectors=sectors)
    assert got["total"] == 1 and got["nhits"][0] == 4 and got["chi2"][0] < 1e-12
    mk = g["polarity"] * g["kick"]
    assert (seed[2] - got["b"][0]) / mk == pytest.approx(qop_true, rel=1e-9)
    g0 = dict(g, algorithm=0, w1_c0=0.5, w1_c1=0.0)
    assert O.candidates(g0, seed, layers)["total"] == 0


def test_incompatible_sectors_hide_hits():
    """A hit in a band the seed cannot reach is invisible: moving the UTbX
    hit out kills the track; moving the UTaX hit out kills the triplet;
    moving a stereo hit out drops that hit only."""
    g = geom()
    seed, layers, sectors = _straight_event(g, [150.0, 80.0, 0.05, 0.02, 0.5], 0.5)
    base = O.candidates(g, seed, layers, sectors=sectors)
    assert base["total"] == 1 and base["nhits"][0] == 4
    far = lambda k: [(k + 5) % g["n_sectors"]]
    for L, expect_total, expect_n in ((3, 0, None), (0, 0, None), (1, 1, 3), (2, 1, 3)):
        sec = [list(s) for s in sectors]
        sec[L] = far(sectors[L][0])
        got = O.candidates(g, seed, layers, sectors=sec)
        assert got["total"] == expect_total
        if expect_n:
            assert got["nhits"][0] == expect_n and got["hits"][0][L] == -1


def test_dv1_zero_smear_generated_events():
    """Generated events with exact hits: every true seed whose decay is
    upstream of the UT finds its own four hits with chi2 ~ 0 under Dv1."""
    g = geom()
    b = synth.generate(0, n_events=6, geometry=g, smear=False, keep_float64=True)
    tr = O.find_tracks(b, g, float64_truth=True)
    t = b.truth
    n = 0
    for e in range(b.n_events):
        for i in range(b.seed_off[e], b.seed_off[e + 1]):
            if not t["seed_true"][i] or t["seed_zdecay"][i] >= g["z_layer"][0]:
                continue
            n += 1
            assert tr["nhits"][i] == 4
            for L in range(4):
                assert t["hit_owner"][b.hit_off[4 * e + L] + tr["hits"][i, L]] == i
            assert tr["chi2"][i] < 1e-12
    assert n > 30


def test_dv1_finds_at_least_dv0_true_tracks():
    """On smeared events Dv1 (no momentum window) finds a track for every true
    seed for which Dv0 finds one, and its candidates include Dv0's best."""
    g1 = geom()
    g0 = dict(g1, algorithm=0)
    b = synth.generate(0, n_events=8)
    t0 = O.find_tracks(b, g0)
    t1 = O.find_tracks(b, g1)
    true = t1["nhits"] > -1
    true &= b.truth["seed_true"].astype(bool)
    found0 = (t0["nhits"] > 0) & true
    found1 = (t1["nhits"] > 0) & true
    assert found0.sum() > 20
    assert np.all(found1[found0 & (t0["hits"][:, 0] >= 0)])

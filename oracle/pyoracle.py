"""ctypes front-end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg.  Nothing on the product path imports it.

Conversions: float32 inputs are widened exactly to float64 before the call.
``run_path`` mirrors the library's boundary: tracks are stored as float32,
and the ghost-killer and vertexer read those stored values.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class OrcGeom(C.Structure):
    _fields_ = [
        ("z_layer", C.c_double * 4),
        ("tan_stereo", C.c_double * 4),
        ("z_magnet", C.c_double), ("z_seed", C.c_double), ("z_ref", C.c_double),
        ("kick", C.c_double), ("polarity", C.c_double),
        ("sigma_hit", C.c_double),
        ("w1_c0", C.c_double), ("w1_c1", C.c_double), ("w2_c0", C.c_double), ("w2_c1", C.c_double),
        ("max_l3", C.c_int),
        ("n_closest", C.c_int * 3),
        ("gamma_c0", C.c_double), ("gamma_c1", C.c_double), ("fringe_polarity", C.c_double),
        ("newton_iters", C.c_int),
        ("doca_max", C.c_double),
        ("algorithm", C.c_int),
        ("n_sectors", C.c_int),
        ("sector_y0", C.c_double), ("sector_h", C.c_double), ("sector_tol", C.c_double),
    ]


def make_geom(g: dict) -> OrcGeom:
    o = OrcGeom()
    for k in ("z_layer", "tan_stereo"):
        getattr(o, k)[:] = [float(v) for v in g[k]]
    for k in ("z_magnet", "z_seed", "z_ref", "kick", "polarity", "sigma_hit", "w1_c0", "w1_c1",
              "w2_c0", "w2_c1", "gamma_c0", "gamma_c1", "fringe_polarity", "doca_max"):
        setattr(o, k, float(g[k]))
    o.max_l3 = int(g["max_l3"])
    o.n_closest[:] = [int(v) for v in g["n_closest"]]
    o.newton_iters = int(g["newton_iters"])
    o.algorithm = int(g.get("algorithm", 0))
    o.n_sectors = int(g.get("n_sectors", 1))
    for k, d in (("sector_y0", -700.0), ("sector_h", 1400.0), ("sector_tol", 0.0)):
        setattr(o, k, float(g.get(k, d)))
    return o


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_find_tracks.restype = C.c_int
        _lib.orc_candidates.restype = C.c_int
        _lib.orc_pca.restype = C.c_int
        _lib.orc_mlp.restype = C.c_double
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _seed_cols(batch, float64_truth=False):
    if float64_truth:
        t = batch.truth
        return [t["seed_x64"], t["seed_y64"], t["seed_tx64"], t["seed_ty64"], t["seed_qop64"]]
    return [batch.sx, batch.sy, batch.stx, batch.sty, batch.sqop]


def find_tracks(batch, g: dict, n_threads: int = 1, float64_truth: bool = False) -> dict:
    """Oracle tracks for every seed (O2-O8).  float64 results plus diagnostics."""
    L = lib()
    S = batch.n_seeds
    keep = []
    cols = []
    for c in _seed_cols(batch, float64_truth):
        a, p = _d(c)
        keep.append(a)
        cols.append(p)
    hu = batch.truth["hit_u64"] if float64_truth else batch.hu
    hu_a, hu_p = _d(hu)
    so_a, so_p = _i(batch.seed_off)
    ho_a, ho_p = _i(batch.hit_off)
    sec = getattr(batch, "hit_sector", None)
    sec_a, sec_p = _i(sec) if sec is not None else (None, None)
    out = {k: np.zeros(S, np.float64) for k in ("x", "y", "tx", "ty", "qop", "chi2", "edge_margin",
                                                  "chi2_gap", "rank_gap")}
    out["nhits"] = np.zeros(S, np.int32)
    out["hits"] = np.zeros((S, 4), np.int32)
    out["cand"] = np.zeros(S, np.int32)
    geom = make_geom(g)
    L.orc_find_tracks(C.byref(geom), C.c_int(batch.n_events), so_p, *cols, ho_p, hu_p, sec_p,
                      *[out[k].ctypes.data_as(_dp) for k in ("x", "y", "tx", "ty", "qop", "chi2")],
                      out["nhits"].ctypes.data_as(_ip), out["hits"].ctypes.data_as(_ip),
                      out["cand"].ctypes.data_as(_ip),
                      *[out[k].ctypes.data_as(_dp) for k in ("edge_margin", "chi2_gap", "rank_gap")],
                      C.c_int(n_threads))
    return out


def kill_clones(seed_off, st: dict) -> np.ndarray:
    """Clone-killing flags (1 = killed) of stored tracks."""
    L = lib()
    so_a, so_p = _i(seed_off)
    nh_a, nh_p = _i(st["nhits"])
    hh_a, hh_p = _i(np.asarray(st["hits"]).reshape(-1))
    c2_a, c2_p = _d(st["chi2"])
    killed = np.zeros(len(nh_a), np.int32)
    L.orc_kill_clones(C.c_int(len(seed_off) - 1), so_p, nh_p, hh_p, c2_p, killed.ctypes.data_as(_ip))
    return killed


def apply_kills(st: dict, killed) -> dict:
    """Killed tracks become 'no track' (as the library writes them)."""
    out = {k: v.copy() for k, v in st.items()}
    k = np.asarray(killed, bool)
    for name in ("x", "y", "tx", "ty", "qop", "chi2"):
        out[name][k] = 0
    out["nhits"][k] = 0
    out["hits"][k] = -1
    return out


def score_candidates(batch, g: dict, weights, max_rows: int = 10 ** 7) -> dict:
    """Every valid candidate of every seed as a stored track with its score."""
    L = lib()
    keep = []

    def d(a):
        arr, p = _d(a)
        keep.append(arr)
        return p

    so_a, so_p = _i(batch.seed_off)
    ho_a, ho_p = _i(batch.hit_off)
    n = max_rows
    seed = np.zeros(n, np.int32)
    cand = np.zeros(n, np.int32)
    hits = np.zeros((n, 4), np.int32)
    nh = np.zeros(n, np.int32)
    state = np.zeros((n, 6))
    score = np.zeros(n)
    geom = make_geom(g)
    m = L.orc_score_candidates(C.byref(geom), C.c_int(batch.n_events), so_p, d(batch.sx), d(batch.sy),
                               d(batch.stx), d(batch.sty), d(batch.sqop), ho_p, d(batch.hu), d(np.asarray(weights)),
                               C.c_int(n), seed.ctypes.data_as(_ip), cand.ctypes.data_as(_ip),
                               hits.ctypes.data_as(_ip), nh.ctypes.data_as(_ip), state.ctypes.data_as(_dp),
                               score.ctypes.data_as(_dp))
    return dict(seed=seed[:m], cand=cand[:m], hits=hits[:m], nhits=nh[:m], state=state[:m], score=score[:m])


def stored_tracks(tr: dict) -> dict:
    """The boundary's float32 track record made from oracle float64 tracks."""
    st = {k: tr[k].astype(np.float32) for k in ("x", "y", "tx", "ty", "qop", "chi2")}
    st["nhits"] = tr["nhits"].copy()
    st["hits"] = tr["hits"].copy()
    return st


def ghost_kill(batch, st: dict, g: dict, weights, want_features: bool = False):
    """Ghost-killer scores (O9) of stored (float32) tracks; float64 scores."""
    L = lib()
    S = batch.n_seeds
    keep = []

    def d(a):
        arr, p = _d(a)
        keep.append(arr)
        return p

    score = np.zeros(S, np.float64)
    feats = np.zeros((S, 17), np.float64) if want_features else None
    so_a, so_p = _i(batch.seed_off)
    ho_a, ho_p = _i(batch.hit_off)
    nh_a, nh_p = _i(st["nhits"])
    hh_a, hh_p = _i(np.asarray(st["hits"]).reshape(-1))
    geom = make_geom(g)
    L.orc_ghost_kill(C.byref(geom), C.c_int(batch.n_events), so_p,
                     d(batch.sx), d(batch.sy), d(batch.stx), d(batch.sty), d(batch.sqop), ho_p, d(batch.hu),
                     d(st["x"]), d(st["y"]), d(st["tx"]), d(st["ty"]), d(st["qop"]), d(st["chi2"]),
                     nh_p, hh_p, d(np.asarray(weights)), score.ctypes.data_as(_dp),
                     feats.ctypes.data_as(_dp) if feats is not None else None)
    return (score, feats) if want_features else score


def vertex(seed_off, sqop, st: dict, score, g: dict, score_max: float, cap: int, line_weights=None) -> dict:
    """Vertices (O10) of stored tracks; event-major, (i, j)-ordered, capped."""
    L = lib()
    E = len(seed_off) - 1
    keep = []

    def d(a):
        arr, p = _d(a)
        keep.append(arr)
        return p

    so_a, so_p = _i(seed_off)
    nh_a, nh_p = _i(st["nhits"])
    count = np.zeros(max(E, 1), np.int32)
    n = max(E * cap, 1)
    vi = np.zeros(n, np.int32)
    vj = np.zeros(n, np.int32)
    vx, vy, vz, vd, vo = (np.zeros(n, np.float64) for _ in range(5))
    ovf = C.c_longlong(0)
    geom = make_geom(g)
    extras = np.zeros((n, 6)) if line_weights is not None else None
    L.orc_vertex(C.byref(geom), C.c_int(E), so_p, d(sqop), d(st["x"]), d(st["y"]), d(st["tx"]), d(st["ty"]),
                 d(st["qop"]), d(score), nh_p, C.c_double(score_max), C.c_int(cap), count.ctypes.data_as(_ip),
                 vi.ctypes.data_as(_ip), vj.ctypes.data_as(_ip), vx.ctypes.data_as(_dp), vy.ctypes.data_as(_dp),
                 vz.ctypes.data_as(_dp), vd.ctypes.data_as(_dp), vo.ctypes.data_as(_dp), C.byref(ovf),
                 d(line_weights) if line_weights is not None else None,
                 extras.ctypes.data_as(_dp) if extras is not None else None)
    out = dict(count=count[:E], i=vi, j=vj, x=vx, y=vy, z=vz, doca=vd, opening=vo, overflow=int(ovf.value), cap=cap)
    if extras is not None:
        out["m_pipi"], out["m_ppi"], out["lines"] = extras[:, 0], extras[:, 1], extras[:, 2:6]
    return out


def vertex_list(v: dict):
    """Flatten capped per-event vertex arrays into a dict keyed by (event, i, j)."""
    out = {}
    cap = v["cap"]
    for e, c in enumerate(v["count"]):
        for m in range(int(c)):
            k = e * cap + m
            out[(e, int(v["i"][k]), int(v["j"][k]))] = (v["x"][k], v["y"][k], v["z"][k], v["doca"][k],
                                                         v.get("opening", np.zeros(1))[k] if "opening" in v else 0.0)
    return out


def run_path(batch, g: dict, weights, score_max=None, cap: int = 1024, n_threads: int = 1,
             clone_kill: bool = False) -> dict:
    """The whole path as the library runs it: tracks -> stored float32 ->
    (clone killing) -> ghost-killer scores -> vertices of kept tracks."""
    tr = find_tracks(batch, g, n_threads=n_threads)
    st = stored_tracks(tr)
    if clone_kill:
        st = apply_kills(st, kill_clones(batch.seed_off, st))
    score = ghost_kill(batch, st, g, weights)
    if score_max is None:
        score_max = g["ghost_threshold"]
    v = vertex(batch.seed_off, batch.sqop, st, score, g, score_max, cap)
    return dict(tracks=tr, stored=st, score=score, vertices=v)


def extrapolate(g: dict, seed):
    L = lib()
    xb = np.zeros(4)
    yl = np.zeros(4)
    xm = C.c_double(0)
    s, sp = _d(seed)
    geom = make_geom(g)
    L.orc_extrapolate(C.byref(geom), sp, xb.ctypes.data_as(_dp), yl.ctypes.data_as(_dp), C.byref(xm))
    return xb, yl, xm.value


def fit(dz, x, sigma):
    L = lib()
    dz_a, dzp = _d(dz)
    x_a, xp = _d(x)
    a, b, c2 = C.c_double(0), C.c_double(0), C.c_double(0)
    L.orc_fit(C.c_int(len(dz_a)), dzp, xp, C.c_double(sigma), C.byref(a), C.byref(b), C.byref(c2))
    return a.value, b.value, c2.value


def candidates(g: dict, seed, layers, max_out: int = 4096, sectors=None) -> dict:
    """Every enumerated candidate of one seed, in enumeration order
    (``sectors``: optional per-layer Y-sector ids of the hits, Dv1)."""
    L = lib()
    keep = []
    args = []
    for l in range(4):
        a, p = _d(np.asarray(layers[l], dtype=np.float64))
        keep.append(a)
        args += [p, C.c_int(len(a))]
    for l in range(4):
        if sectors is None:
            args.append(None)
        else:
            a, p = _i(np.asarray(sectors[l], dtype=np.int32))
            keep.append(a)
            args.append(p)
    s, sp = _d(seed)
    c = np.zeros(max_out, np.int32)
    hits = np.zeros((max_out, 4), np.int32)
    nh = np.zeros(max_out, np.int32)
    valid = np.zeros(max_out, np.int32)
    a_, b_, c2 = np.zeros(max_out), np.zeros(max_out), np.zeros(max_out)
    geom = make_geom(g)
    tot = L.orc_candidates(C.byref(geom), sp, *args, C.c_int(max_out), c.ctypes.data_as(_ip),
                           hits.ctypes.data_as(_ip), nh.ctypes.data_as(_ip), valid.ctypes.data_as(_ip),
                           a_.ctypes.data_as(_dp), b_.ctypes.data_as(_dp), c2.ctypes.data_as(_dp))
    m = min(tot, max_out)
    return dict(total=tot, c=c[:m], hits=hits[:m], nhits=nh[:m], valid=valid[:m], a=a_[:m], b=b_[:m],
                chi2=c2[:m])


def pca(g: dict, t1, t2, iters=None):
    """(vx, vy, vz, doca, z1, z2) or None if the pair is rejected."""
    L = lib()
    a1, p1 = _d(t1)
    a2, p2 = _d(t2)
    out = np.zeros(6)
    geom = make_geom(g)
    ok = L.orc_pca(C.byref(geom), p1, p2, C.c_int(g["newton_iters"] if iters is None else iters),
                   out.ctypes.data_as(_dp))
    return out if ok else None


def vertex_extras(g: dict, t1, t2, q1, q2, z1, z2, vtx, line_weights):
    L = lib()
    keep = [np.ascontiguousarray(v, dtype=np.float64) for v in (t1, t2, vtx, line_weights)]
    out = np.zeros(6)
    geom = make_geom(g)
    L.orc_vertex_extras(C.byref(geom), *[k.ctypes.data_as(_dp) for k in keep[:2]], C.c_double(q1), C.c_double(q2),
                        C.c_double(z1), C.c_double(z2), keep[2].ctypes.data_as(_dp), keep[3].ctypes.data_as(_dp),
                        out.ctypes.data_as(_dp))
    return out


def mlp(weights, f) -> float:
    L = lib()
    w, wp = _d(weights)
    ff, fp = _d(f)
    return L.orc_mlp(wp, fp)


def features(g: dict, trk, nh, seed, hit_u):
    L = lib()
    t, tp = _d(trk)
    s, sp = _d(seed)
    h, hp = _d(hit_u)
    f = np.zeros(17)
    geom = make_geom(g)
    L.orc_features(C.byref(geom), tp, C.c_int(nh), sp, hp, f.ctypes.data_as(_dp))
    return f

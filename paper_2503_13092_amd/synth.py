"""Seeded synthetic events for the Downstream tracking + vertexing path.

This module only *generates inputs*: detector geometry values, event
occupancies, LLP decays, SciFi seed states, UT hits (true + noise) and the
ghost-killer weights.  It performs none of the method's arithmetic (no
extrapolation back from a seed, no window search, no fit, no MLP, no
vertexing); both the oracle and the HIP path consume what it returns.

Physics model of the generator (the paper's LHCb samples are not available;
these seeded events stand in for them):

* Detector: four UT layers UTaX, UTaU, UTbV, UTbX at z = 2327, 2372, 2597,
  2642 mm with stereo angles 0, +5, -5, 0 degrees (UT description, Fig. 2);
  a hit measures u = x - y*tan(alpha), the strip's x-intercept at y = 0.
  SciFi seeds are states (x, y, tx, ty, q/p) at z = 7826 mm.
* Magnet: the field is along y, so only x bends (LHCb detector section);
  the bend is modelled as one kink at z = 5280 mm (magnet-point model,
  eq. 1 and the text after it) with dtx = polarity * K * q/p,
  K = 1.2e-3 rad GeV.
* An LLP starts at the origin with slopes tx ~ U[-0.25, 0.25],
  ty ~ U[-0.2, 0.2] and decays at z ~ U[0, zmax]; it gives two daughters of
  opposite charge with p = exp(U[ln 2, ln 100]) GeV and slopes smeared by
  N(0, 0.02).  A daughter is redrawn until it lies in the UT acceptance
  (|x| < 800, |y| < 700 mm) at every layer downstream of the decay and in
  |x| < 3000, |y| < 2500 mm at the seed plane.
* Seeds: the kicked line at z_seed plus N(0, 0.1) mm on x, y and N(0, 1e-4)
  on tx, ty; q/p is exact.  Ghost seeds have daughter kinematics but leave
  no UT hits.
* Hits: true hits at layers downstream of the decay with N(0, 0.05) mm
  smear; noise hits uniform over |x| < 800, |y| < 700 mm; hits shuffled
  within each (event, layer) run, seeds shuffled within each event.
* Fringe field (geometry ``fringe_polarity`` = +-1; 0, the default, keeps
  the straight lines above): between the decay point and the UT a daughter
  follows the eq. 4 parabola x(z) = x0 + tx0 (z - z0) + gamma (z - z0)^2,
  y linear, with gamma = -MP (c0 + c1 q/p[MeV^-1]) from eq. 3 and z0 the UT
  midpoint; (x0, tx0) is its state there, and from z0 on it is the straight
  line of the UT and the kink model.  The slopes drawn at the decay point are
  the parabola's there, so the generated decay point lies exactly on both
  daughters' eq. 4 trajectories.  No extra random draws.
* Y sectors: every hit also carries the 100 mm band of its layer that its
  true y falls in (14 bands over |y| < 700 mm); Dv1's triplet search uses
  them.  They are computed from the generated y, with no extra random draw.

Draw order (numpy PCG64, ``default_rng(seed)``): occupancies -> LLPs ->
daughter charges/momenta/slopes (with rejection redraws) -> ghost kinematics
-> seed smearing -> hit smearing/efficiency -> noise hits -> shuffle keys.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

TAN5 = math.tan(math.radians(5.0))

# UT acceptance used by the generator (and as the library's hit-binning range)
UT_XMAX = 800.0
UT_YMAX = 700.0
SEED_XMAX = 3000.0
SEED_YMAX = 2500.0
# Y sectors: horizontal bands of a UT layer, 100 mm high (about one sensor)
N_SECTORS = 14


def default_geometry(loose: bool = False) -> Dict:
    """Detector geometry and method settings for the synthetic workloads.

    Window constants are the reading W = c0 + c1*|q/p| (the paper derives its
    windows from simulation and prints no values); ``loose=True`` gives the
    fixed 100 mm / 10 mm windows the paper uses while training the
    ghost-killer.
    """
    g = dict(
        z_layer=(2327.0, 2372.0, 2597.0, 2642.0),
        tan_stereo=(0.0, TAN5, -TAN5, 0.0),
        z_magnet=5280.0,
        z_seed=7826.0,
        z_ref=0.5 * (2327.0 + 2642.0),
        kick=1.2e-3,
        polarity=1.0,
        sigma_hit=0.05,
        w1_c0=3.0, w1_c1=1.0,
        w2_c0=0.5, w2_c1=0.25,
        max_l3=10,
        n_closest=(1, 2, 2),
        gamma_c0=-1.5e-8, gamma_c1=9.3e-3,
        fringe_polarity=0.0,
        newton_iters=3,
        doca_max=1.0,
        ghost_threshold=0.5,
        u_min=-(UT_XMAX + UT_YMAX * TAN5),
        u_max=(UT_XMAX + UT_YMAX * TAN5),
        clone_kill=0,
        # Dv1 (triplet search): UT hits grouped into Y sectors of their layer
        algorithm=0,
        n_sectors=N_SECTORS, sector_y0=-UT_YMAX, sector_h=2.0 * UT_YMAX / N_SECTORS, sector_tol=5.0,
    )
    if loose:
        g.update(w1_c0=100.0, w1_c1=0.0, w2_c0=10.0, w2_c1=0.0)
    return g


CONFIGS = {
    0: dict(name="tiny", n_events=100, seed=0, seeds_per_event=20,
            llp_per_event=5, hits_per_layer=500, zmax=2200.0),
    1: dict(name="throughput", n_events=10000, seed=1, seeds_per_event=150,
            llp_per_event=30, hits_per_layer=600, zmax=2200.0),
    2: dict(name="uneven", n_events=20000, seed=2, pileup=5.3, seeds_per_nu=28,
            hits_per_nu=110, seed_clip=(5, 600), llp_max=3, zmax=2200.0),
    4: dict(name="stress", n_events=5000, seed=4, seeds_per_event=300,
            llp_per_event=45, hits_per_layer=1200, zmax=2500.0),
    # literal reading of the stress point: 4800 hits in every layer
    5: dict(name="stress-literal", n_events=500, seed=5, seeds_per_event=300,
            llp_per_event=45, hits_per_layer=4800, zmax=2500.0),
}

N_MLP_WEIGHTS = 17 * 32 + 32 + 32 * 16 + 16 + 16 * 1 + 1  # 1121


def mlp_weights(seed: int = 0, scale: float = 0.3) -> np.ndarray:
    """Ghost-killer parameters W1[32][17], b1[32], W2[16][32], b2[16],
    W3[1][16], b3[1] (row-major, concatenated), all N(0, scale)."""
    return np.random.default_rng(seed).normal(0.0, scale, N_MLP_WEIGHTS).astype(np.float32)


N_LINE_WEIGHTS = 4 * (32 * 12 + 32 + 32 + 1)  # four 12 -> 32 -> 1 trigger-line networks


def line_weights(seed: int = 1, scale: float = 0.3) -> np.ndarray:
    """Trigger-line networks, each W1[32][12], b1[32], W2[1][32], b2[1], all N(0, scale)."""
    return np.random.default_rng(seed).normal(0.0, scale, N_LINE_WEIGHTS).astype(np.float32)


@dataclasses.dataclass
class EventBatch:
    """SoA batch.  Offsets are event-major; ``hit_off`` is (event, layer)."""
    n_events: int
    seed_off: np.ndarray      # int32 [E+1]
    sx: np.ndarray            # float32 [S]
    sy: np.ndarray
    stx: np.ndarray
    sty: np.ndarray
    sqop: np.ndarray
    hit_off: np.ndarray       # int32 [4E+1]
    hu: np.ndarray            # float32 [H]
    truth: Dict[str, np.ndarray] = dataclasses.field(default_factory=dict)
    hit_sector: Optional[np.ndarray] = None   # uint8 [H]: Y sector of each hit (Dv1)

    @property
    def n_seeds(self) -> int:
        return int(self.seed_off[-1])

    @property
    def n_hits(self) -> int:
        return int(self.hit_off[-1])

    def seeds_per_event(self) -> np.ndarray:
        return np.diff(self.seed_off)

    def hits_per_layer(self) -> np.ndarray:
        return np.diff(self.hit_off).reshape(self.n_events, 4)

    def subset(self, events) -> "EventBatch":
        """A new batch made of the listed events (in the given order)."""
        events = np.asarray(events, dtype=np.int64)
        s_lo = self.seed_off[events]
        s_hi = self.seed_off[events + 1]
        s_idx = np.concatenate([np.arange(a, b) for a, b in zip(s_lo, s_hi)]) if len(events) else np.zeros(0, np.int64)
        h_idx_parts, hit_counts = [], []
        for e in events:
            for l in range(4):
                a, b = self.hit_off[4 * e + l], self.hit_off[4 * e + l + 1]
                h_idx_parts.append(np.arange(a, b))
                hit_counts.append(b - a)
        h_idx = np.concatenate(h_idx_parts) if h_idx_parts else np.zeros(0, np.int64)
        seed_off = np.zeros(len(events) + 1, np.int32)
        seed_off[1:] = np.cumsum(s_hi - s_lo)
        hit_off = np.zeros(4 * len(events) + 1, np.int32)
        hit_off[1:] = np.cumsum(hit_counts)
        truth = {}
        for k, v in self.truth.items():
            if k.startswith("seed_") and len(v) == self.n_seeds:
                truth[k] = v[s_idx]
            elif k.startswith("hit_") and len(v) == self.n_hits:
                truth[k] = v[h_idx]
        return EventBatch(len(events), seed_off, self.sx[s_idx], self.sy[s_idx], self.stx[s_idx],
                          self.sty[s_idx], self.sqop[s_idx], hit_off, self.hu[h_idx], truth,
                          None if self.hit_sector is None else self.hit_sector[h_idx])


def batch_from_lists(events, dtype=np.float32) -> EventBatch:
    """Build a batch from explicit per-event content.

    ``events`` is a list of dicts with ``seeds`` (list of (x, y, tx, ty, qop))
    and ``hits`` (list of 4 lists of u), optionally ``sectors`` (4 lists of
    Y-sector ids, default 0).  Used for hand-built test events.
    """
    seed_off, hit_off = [0], [0]
    cols = [[] for _ in range(5)]
    hu, sec = [], []
    for ev in events:
        for s in ev.get("seeds", []):
            for k in range(5):
                cols[k].append(s[k])
        seed_off.append(seed_off[-1] + len(ev.get("seeds", [])))
        layers = ev.get("hits", [[], [], [], []])
        secs = ev.get("sectors", [[0] * len(h) for h in layers])
        for l in range(4):
            hu.extend(layers[l])
            sec.extend(secs[l])
            hit_off.append(hit_off[-1] + len(layers[l]))
    arr = [np.asarray(c, dtype=dtype) for c in cols]
    return EventBatch(len(events), np.asarray(seed_off, np.int32), *arr,
                      np.asarray(hit_off, np.int32), np.asarray(hu, dtype=dtype),
                      hit_sector=np.asarray(sec, dtype=np.uint8))


def sector_of(y, g: Optional[Dict] = None) -> np.ndarray:
    """Y sector of points at height y (the band a hit's sensor covers)."""
    d = default_geometry()
    g = g or d
    y0, h, n = (g.get(k, d[k]) for k in ("sector_y0", "sector_h", "n_sectors"))
    k = np.floor((np.asarray(y, dtype=np.float64) - y0) / h)
    return np.clip(k, 0, n - 1).astype(np.uint8)


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def fringe_gamma(g: Dict, qop) -> np.ndarray:
    """Eq. 3: the second-order coefficient (mm^-1) of a track's x(z) between
    the decay point and the UT, q/p in GeV^-1 (converted to MeV^-1)."""
    return -g["fringe_polarity"] * (g["gamma_c0"] + g["gamma_c1"] * np.asarray(qop) * 1e-3)


def _ut_state(g, vx, tx_v, zd, gam):
    """x and tx at the UT midpoint z0 of the parabola through (vx, zd) with
    slope tx_v there and second-order coefficient gam."""
    h = g["z_ref"] - zd
    return vx + tx_v * h + gam * h * h, tx_v + 2.0 * gam * h


def _draw_daughters(rng, g, llp_tx, llp_ty, llp_z, charge, accept_ut=True):
    """Momenta and slopes for daughters of the given parents (one row each),
    redrawn until inside the acceptance.  Returns p, tx_before, ty (with a
    fringe field: the slope at the decay point)."""
    n = len(llp_tx)
    p = np.empty(n)
    tx = np.empty(n)
    ty = np.empty(n)
    todo = np.arange(n)
    zl = np.asarray(g["z_layer"])
    for _ in range(1000):
        if len(todo) == 0:
            break
        m = len(todo)
        p[todo] = _log_uniform(rng, 2.0, 100.0, m)
        tx[todo] = llp_tx[todo] + rng.normal(0.0, 0.02, m)
        ty[todo] = llp_ty[todo] + rng.normal(0.0, 0.02, m)
        zd = llp_z[todo]
        vx, vy = llp_tx[todo] * zd, llp_ty[todo] * zd
        qop = charge[todo] / p[todo]
        curved = g.get("fringe_polarity", 0.0) != 0.0
        if curved:   # the UT line of the eq. 4 parabola
            x0, tx0 = _ut_state(g, vx, tx[todo], zd, fringe_gamma(g, qop))
        ok = np.ones(m, bool)
        if accept_ut:
            for L in range(4):
                down = zl[L] > zd
                xL = x0 + tx0 * (zl[L] - g["z_ref"]) if curved else vx + tx[todo] * (zl[L] - zd)
                yL = vy + ty[todo] * (zl[L] - zd)
                ok &= ~down | ((np.abs(xL) < UT_XMAX) & (np.abs(yL) < UT_YMAX))
        if curved:
            xm = x0 + tx0 * (g["z_magnet"] - g["z_ref"])
            txa = tx0 + g["polarity"] * g["kick"] * qop
        else:
            xm = vx + tx[todo] * (g["z_magnet"] - zd)
            txa = tx[todo] + g["polarity"] * g["kick"] * qop
        xs = xm + txa * (g["z_seed"] - g["z_magnet"])
        ys = vy + ty[todo] * (g["z_seed"] - zd)
        ok &= (np.abs(xs) < SEED_XMAX) & (np.abs(ys) < SEED_YMAX)
        todo = todo[~ok]
    else:
        raise RuntimeError("daughter acceptance redraw did not converge")
    return p, tx, ty


def generate(config=1, n_events: Optional[int] = None, seed: Optional[int] = None,
             geometry: Optional[Dict] = None, smear: bool = True,
             hit_efficiency: float = 1.0, keep_float64: bool = False) -> EventBatch:
    """Generate one of the workload configurations (0, 1, 2, 4, 5) or a dict.

    ``smear=False`` removes every Gaussian smear (seed and hit), which makes
    true hits lie exactly on the generated trajectories.  ``keep_float64``
    also stores the float64 values in ``truth`` (``seed_*64``, ``hit_u64``).
    """
    cfg = dict(CONFIGS[config]) if not isinstance(config, dict) else dict(config)
    if n_events is not None:
        cfg["n_events"] = n_events
    if seed is not None:
        cfg["seed"] = seed
    g = geometry or default_geometry()
    rng = np.random.default_rng(cfg["seed"])
    E = int(cfg["n_events"])
    zl = np.asarray(g["z_layer"], dtype=np.float64)
    tana = np.asarray(g["tan_stereo"], dtype=np.float64)

    # 1. occupancies
    if "pileup" in cfg:
        nu = rng.poisson(cfg["pileup"], E)
        n_seed = np.clip(rng.poisson(cfg["seeds_per_nu"] * nu), *cfg["seed_clip"]).astype(np.int64)
        n_llp = np.minimum(rng.integers(0, cfg["llp_max"] + 1, E), n_seed // 2)
        noise_per_layer = rng.poisson(cfg["hits_per_nu"] * np.repeat(nu, 4)).reshape(E, 4)
        fixed_total = None
    else:
        n_seed = np.full(E, cfg["seeds_per_event"], np.int64)
        n_llp = np.full(E, cfg["llp_per_event"], np.int64)
        noise_per_layer = None
        fixed_total = cfg["hits_per_layer"]
    n_true = 2 * n_llp
    n_ghost = n_seed - n_true

    # 2. LLPs
    NL = int(n_llp.sum())
    llp_ev = np.repeat(np.arange(E), n_llp)
    llp_tx = rng.uniform(-0.25, 0.25, NL)
    llp_ty = rng.uniform(-0.2, 0.2, NL)
    llp_z = rng.uniform(0.0, cfg["zmax"], NL)

    # 3. daughters: charges (+1, -1) in random order
    first_pos = rng.integers(0, 2, NL)
    ch = np.empty(2 * NL)
    ch[0::2] = np.where(first_pos == 1, 1.0, -1.0)
    ch[1::2] = -ch[0::2]
    d_par = np.repeat(np.arange(NL), 2)
    p, txb, ty = _draw_daughters(rng, g, llp_tx[d_par], llp_ty[d_par], llp_z[d_par], ch)
    d_ev = llp_ev[d_par]
    d_z = llp_z[d_par]

    # 4. ghosts: daughter kinematics of a fake parent, no UT hits
    NG = int(n_ghost.sum())
    g_ev = np.repeat(np.arange(E), n_ghost)
    g_tx = rng.uniform(-0.25, 0.25, NG)
    g_ty = rng.uniform(-0.2, 0.2, NG)
    g_z = rng.uniform(0.0, cfg["zmax"], NG)
    g_ch = np.where(rng.integers(0, 2, NG) == 1, 1.0, -1.0)
    gp, gtxb, gty = _draw_daughters(rng, g, g_tx, g_ty, g_z, g_ch)

    # all tracks (true first, then ghosts), parameters before the kink
    T_ev = np.concatenate([d_ev, g_ev])
    T_z = np.concatenate([d_z, g_z])
    T_vx = np.concatenate([llp_tx[d_par] * d_z, g_tx * g_z])
    T_vy = np.concatenate([llp_ty[d_par] * d_z, g_ty * g_z])
    T_txb = np.concatenate([txb, gtxb])
    T_ty = np.concatenate([ty, gty])
    T_qop = np.concatenate([ch / p, g_ch / gp])
    T_true = np.concatenate([np.ones(2 * NL, bool), np.zeros(NG, bool)])
    T_llp = np.concatenate([d_par, np.full(NG, -1)])
    NT = len(T_ev)
    curved = g.get("fringe_polarity", 0.0) != 0.0
    T_gam = fringe_gamma(g, T_qop) if curved else np.zeros(NT)
    if curved:
        # from the UT on, the straight line with the parabola's UT state:
        # re-anchor it at the decay z so that the code below is unchanged
        x0, tx0 = _ut_state(g, T_vx, T_txb, T_z, T_gam)
        T_txb = tx0
        T_vx = x0 - tx0 * (g["z_ref"] - T_z)
        T_vx_true = np.concatenate([llp_tx[d_par] * d_z, g_tx * g_z])
    else:
        T_vx_true = T_vx

    xm = T_vx + T_txb * (g["z_magnet"] - T_z)
    txa = T_txb + g["polarity"] * g["kick"] * T_qop
    xs_true = xm + txa * (g["z_seed"] - g["z_magnet"])
    ys_true = T_vy + T_ty * (g["z_seed"] - T_z)

    # 5. seed smearing
    sm = rng.normal(0.0, 1.0, (NT, 4)) if smear else np.zeros((NT, 4))
    sx = xs_true + 0.1 * sm[:, 0]
    sy = ys_true + 0.1 * sm[:, 1]
    stx = txa + 1e-4 * sm[:, 2]
    sty = T_ty + 1e-4 * sm[:, 3]
    sqop = T_qop

    # 6. true hits (true daughters only, layers downstream of the decay)
    tr_idx = np.nonzero(T_true)[0]
    th_track, th_layer, th_u, th_y = [], [], [], []
    for L in range(4):
        down = tr_idx[zl[L] > T_z[tr_idx]]
        xL = T_vx[down] + T_txb[down] * (zl[L] - T_z[down])
        yL = T_vy[down] + T_ty[down] * (zl[L] - T_z[down])
        u = xL - yL * tana[L]
        th_track.append(down)
        th_layer.append(np.full(len(down), L))
        th_u.append(u)
        th_y.append(yL)
    th_track = np.concatenate(th_track)
    th_layer = np.concatenate(th_layer)
    th_u = np.concatenate(th_u)
    th_y = np.concatenate(th_y)
    if smear:
        th_u = th_u + rng.normal(0.0, g["sigma_hit"], len(th_u))
    if hit_efficiency < 1.0:
        keep = rng.uniform(0.0, 1.0, len(th_u)) < hit_efficiency
        th_track, th_layer, th_u, th_y = th_track[keep], th_layer[keep], th_u[keep], th_y[keep]
    th_ev = T_ev[th_track]

    # 7. noise hits
    true_counts = np.zeros((E, 4), np.int64)
    np.add.at(true_counts, (th_ev, th_layer), 1)
    if fixed_total is not None:
        noise_per_layer = np.maximum(fixed_total - true_counts, 0)
    nz = noise_per_layer.reshape(-1)
    NN = int(nz.sum())
    nz_grp = np.repeat(np.arange(4 * E), nz)
    nx = rng.uniform(-UT_XMAX, UT_XMAX, NN)
    ny = rng.uniform(-UT_YMAX, UT_YMAX, NN)
    nu_ = nx - ny * tana[nz_grp % 4]

    # 8. grouping + shuffles
    all_grp = np.concatenate([th_ev * 4 + th_layer, nz_grp])
    all_u = np.concatenate([th_u, nu_])
    all_y = np.concatenate([th_y, ny])
    all_owner_track = np.concatenate([th_track, np.full(NN, -1)])
    hkey = rng.integers(0, 1 << 31, len(all_u), dtype=np.int64)
    horder = np.argsort(all_grp.astype(np.int64) << 31 | hkey, kind="stable")
    all_grp, all_u, all_owner_track = all_grp[horder], all_u[horder], all_owner_track[horder]
    all_y = all_y[horder]
    counts = np.bincount(all_grp, minlength=4 * E)
    hit_off = np.zeros(4 * E + 1, np.int64)
    hit_off[1:] = np.cumsum(counts)

    skey = rng.integers(0, 1 << 31, NT, dtype=np.int64)
    sorder = np.argsort(T_ev.astype(np.int64) << 31 | skey, kind="stable")  # final seed order -> track id
    track_to_seed = np.empty(NT, np.int64)
    track_to_seed[sorder] = np.arange(NT)
    seed_off = np.zeros(E + 1, np.int64)
    seed_off[1:] = np.cumsum(np.bincount(T_ev, minlength=E))

    hit_owner = np.where(all_owner_track >= 0, track_to_seed[np.maximum(all_owner_track, 0)], -1)
    truth = dict(
        seed_true=T_true[sorder], seed_llp=T_llp[sorder], seed_qop=T_qop[sorder],
        seed_zdecay=T_z[sorder], seed_vx=T_vx_true[sorder], seed_vy=T_vy[sorder],
        seed_txb=T_txb[sorder], seed_ty=T_ty[sorder], seed_gamma=T_gam[sorder],
        # the state at the UT midpoint (x0, y0, tx0 = seed_txb, ty0 = seed_ty)
        seed_x0=(T_vx + T_txb * (g["z_ref"] - T_z))[sorder], seed_y0=(T_vy + T_ty * (g["z_ref"] - T_z))[sorder],
        hit_owner=hit_owner.astype(np.int64), hit_layer=(all_grp % 4).astype(np.int8),
    )
    if keep_float64:
        truth.update(seed_x64=sx[sorder], seed_y64=sy[sorder], seed_tx64=stx[sorder],
                     seed_ty64=sty[sorder], seed_qop64=sqop[sorder], hit_u64=all_u.copy())
    f32 = np.float32
    return EventBatch(E, seed_off.astype(np.int32), sx[sorder].astype(f32), sy[sorder].astype(f32),
                      stx[sorder].astype(f32), sty[sorder].astype(f32), sqop[sorder].astype(f32),
                      hit_off.astype(np.int32), all_u.astype(f32), truth, sector_of(all_y, g))


def vertex_track_sample(n_events: int, n_pairs: int, n_random: int, seed: int = 7,
                        geometry: Optional[Dict] = None, smear: float = 0.02):
    """Track states at z_ref for exercising the vertexer on its own.

    Each event has ``n_pairs`` opposite-charge pairs from a common decay point
    (state smearing ``smear`` mm / ``smear*1e-3`` rad) and ``n_random``
    unrelated tracks.  Returns a dict of float32/int32 arrays plus
    ``seed_off``.  The seed q/p carries the charge.
    """
    g = geometry or default_geometry()
    rng = np.random.default_rng(seed)
    zr = g["z_ref"]
    per = 2 * n_pairs + n_random
    E = n_events
    n = E * per
    x = np.empty(n); y = np.empty(n); tx = np.empty(n); ty = np.empty(n); qop = np.empty(n)
    for e in range(E):
        base = e * per
        for k in range(n_pairs):
            zd = rng.uniform(0.0, 2200.0)
            vx, vy = rng.uniform(-0.2, 0.2) * zd, rng.uniform(-0.15, 0.15) * zd
            q0 = 1.0 if rng.integers(0, 2) else -1.0
            for d, q in enumerate((q0, -q0)):
                t1, t2 = rng.uniform(-0.25, 0.25), rng.uniform(-0.2, 0.2)
                i = base + 2 * k + d
                tx[i], ty[i] = t1, t2
                x[i] = vx + t1 * (zr - zd) + rng.normal(0, smear)
                y[i] = vy + t2 * (zr - zd) + rng.normal(0, smear)
                tx[i] += rng.normal(0, smear * 1e-3)
                ty[i] += rng.normal(0, smear * 1e-3)
                qop[i] = q / math.exp(rng.uniform(math.log(2), math.log(100)))
        for k in range(n_random):
            i = base + 2 * n_pairs + k
            x[i], y[i] = rng.uniform(-800, 800), rng.uniform(-700, 700)
            tx[i], ty[i] = rng.uniform(-0.3, 0.3), rng.uniform(-0.25, 0.25)
            qop[i] = (1.0 if rng.integers(0, 2) else -1.0) / math.exp(rng.uniform(math.log(2), math.log(100)))
    f = np.float32
    return dict(seed_off=(np.arange(E + 1) * per).astype(np.int32), x=x.astype(f), y=y.astype(f),
                tx=tx.astype(f), ty=ty.astype(f), qop=qop.astype(f), sqop=qop.astype(f),
                score=np.zeros(n, f), nhits=np.full(n, 4, np.int32))

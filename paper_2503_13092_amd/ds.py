"""Python binding of libds.so (include/ds.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module only
turns torch device tensors into the C structs and calls the C ABI.  If the
library has not been built the import of a context fails loudly: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libds.so")

DS_OK, DS_E_ARG, DS_E_STATE, DS_E_NOMEM, DS_E_CAPACITY, DS_E_DEVICE = range(6)
DS_MODE_PER_EVENT, DS_MODE_PERSISTENT, DS_MODE_GRAPH = 0, 1, 2
DS_F_BAD_OFFSETS, DS_F_CAPACITY, DS_F_NONFINITE = 1, 2, 4
DS_ORDER_INPUT, DS_ORDER_LARGEST_FIRST = 0, 1
N_WEIGHTS = 1121
DS_STATIC_MAX_EVENTS = 262144

EXPORTED = ("ds_create", "ds_destroy", "ds_load_geometry", "ds_find_tracks", "ds_ghost_kill", "ds_kill_clones",
            "ds_candidate_slots", "ds_score_candidates", "ds_load_lines", "ds_vertex", "ds_process", "ds_process_static", "ds_set_launch",
            "ds_get_launch", "ds_set_event_order", "ds_get_event_order", "ds_set_step_fusion",
            "ds_get_step_fusion", "ds_status_str")


class DsGeometry(C.Structure):
    _fields_ = [
        ("z_layer", C.c_double * 4),
        ("tan_stereo", C.c_double * 4),
        ("z_magnet", C.c_double), ("z_seed", C.c_double), ("z_ref", C.c_double),
        ("kick", C.c_double), ("polarity", C.c_double),
        ("sigma_hit", C.c_double),
        ("w1_c0", C.c_double), ("w1_c1", C.c_double), ("w2_c0", C.c_double), ("w2_c1", C.c_double),
        ("u_min", C.c_double), ("u_max", C.c_double),
        ("max_l3", C.c_int32),
        ("n_closest", C.c_int32 * 3),
        ("gamma_c0", C.c_double), ("gamma_c1", C.c_double), ("fringe_polarity", C.c_double),
        ("newton_iters", C.c_int32),
        ("doca_max", C.c_double),
        ("ghost_threshold", C.c_double),
        ("clone_kill", C.c_int32),
        ("algorithm", C.c_int32),
        ("n_sectors", C.c_int32),
        ("sector_y0", C.c_double), ("sector_h", C.c_double), ("sector_tol", C.c_double),
    ]


class DsEvents(C.Structure):
    _fields_ = [
        ("n_events", C.c_int32), ("n_seeds", C.c_int32), ("n_hits", C.c_int32),
        ("max_seeds_per_event", C.c_int32), ("max_hits_per_event", C.c_int32),
        ("seed_off", C.c_void_p),
        ("sx", C.c_void_p), ("sy", C.c_void_p), ("stx", C.c_void_p), ("sty", C.c_void_p), ("sqop", C.c_void_p),
        ("hit_off", C.c_void_p),
        ("hu", C.c_void_p),
        ("hit_sector", C.c_void_p),
    ]


class DsTracks(C.Structure):
    _fields_ = [
        ("x", C.c_void_p), ("y", C.c_void_p), ("tx", C.c_void_p), ("ty", C.c_void_p),
        ("qop", C.c_void_p), ("chi2", C.c_void_p), ("score", C.c_void_p),
        ("hit", C.c_void_p * 4),
        ("nhits", C.c_void_p),
        ("cand", C.c_void_p),
        ("flags", C.c_void_p),
    ]


class DsVertices(C.Structure):
    _fields_ = [
        ("cap_per_event", C.c_int32),
        ("count", C.c_void_p),
        ("i", C.c_void_p), ("j", C.c_void_p),
        ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("doca", C.c_void_p),
        ("overflow", C.c_void_p),
        ("flags", C.c_void_p),
        ("m_pipi", C.c_void_p), ("m_ppi", C.c_void_p),
        ("line", C.c_void_p * 4),
    ]


class DsCandidates(C.Structure):
    _fields_ = [
        ("capacity", C.c_int32),
        ("seed", C.c_void_p), ("cand", C.c_void_p), ("nhits", C.c_void_p),
        ("hit", C.c_void_p * 4),
        ("x", C.c_void_p), ("y", C.c_void_p), ("tx", C.c_void_p), ("ty", C.c_void_p),
        ("qop", C.c_void_p), ("chi2", C.c_void_p), ("score", C.c_void_p),
        ("flags", C.c_void_p),
    ]


_lib = None


def library() -> C.CDLL:
    """Load libds.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        lib.ds_create.argtypes = [C.POINTER(P), C.c_int]
        lib.ds_destroy.argtypes = [P]
        lib.ds_destroy.restype = None
        lib.ds_load_geometry.argtypes = [P, C.POINTER(DsGeometry), C.POINTER(C.c_float), C.c_size_t]
        lib.ds_find_tracks.argtypes = [P, C.POINTER(DsEvents), C.POINTER(DsTracks), C.c_int, C.c_int, P]
        lib.ds_ghost_kill.argtypes = [P, C.POINTER(DsEvents), C.POINTER(DsTracks), P]
        lib.ds_kill_clones.argtypes = [P, C.POINTER(DsEvents), C.POINTER(DsTracks), P]
        lib.ds_candidate_slots.argtypes = [P]
        lib.ds_load_lines.argtypes = [P, C.POINTER(C.c_float), C.c_size_t]
        lib.ds_score_candidates.argtypes = [P, C.POINTER(DsEvents), C.POINTER(DsCandidates), P]
        lib.ds_vertex.argtypes = [P, C.POINTER(DsEvents), C.POINTER(DsTracks), C.c_float, C.POINTER(DsVertices),
                                  C.c_int, P]
        lib.ds_process.argtypes = [P, C.POINTER(DsEvents), C.POINTER(DsTracks), C.c_float, C.POINTER(DsVertices),
                                   C.c_int, P]
        lib.ds_process_static.argtypes = [P, C.POINTER(DsEvents), C.POINTER(DsTracks), C.c_float,
                                          C.POINTER(DsVertices), P]
        lib.ds_set_launch.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int]
        lib.ds_get_launch.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        lib.ds_set_event_order.argtypes = [P, C.c_int]
        lib.ds_get_event_order.argtypes = [P, C.POINTER(C.c_int)]
        lib.ds_set_step_fusion.argtypes = [P, C.c_int]
        lib.ds_get_step_fusion.argtypes = [P, C.POINTER(C.c_int)]
        lib.ds_status_str.argtypes = [C.c_int]
        lib.ds_status_str.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("ds_destroy", "ds_status_str"):
                getattr(lib, name).restype = C.c_int
        _lib = lib
    return _lib


class DsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {library().ds_status_str(status).decode()}")


def _check(status: int, where: str):
    if status != DS_OK:
        raise DsError(status, where)


def geometry_struct(g: Dict) -> DsGeometry:
    s = DsGeometry()
    s.z_layer[:] = [float(v) for v in g["z_layer"]]
    s.tan_stereo[:] = [float(v) for v in g["tan_stereo"]]
    for k in ("z_magnet", "z_seed", "z_ref", "kick", "polarity", "sigma_hit", "w1_c0", "w1_c1", "w2_c0",
              "w2_c1", "u_min", "u_max", "gamma_c0", "gamma_c1", "fringe_polarity", "doca_max",
              "ghost_threshold"):
        setattr(s, k, float(g[k]))
    s.max_l3 = int(g["max_l3"])
    s.n_closest[:] = [int(v) for v in g["n_closest"]]
    s.newton_iters = int(g["newton_iters"])
    s.clone_kill = int(g.get("clone_kill", 0))
    s.algorithm = int(g.get("algorithm", 0))
    s.n_sectors = int(g.get("n_sectors", 1))
    s.sector_y0 = float(g.get("sector_y0", -700.0))
    s.sector_h = float(g.get("sector_h", 1400.0))
    s.sector_tol = float(g.get("sector_tol", 0.0))
    return s


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ----------------------------------------------------------- device buffers

class DeviceEvents:
    """Device copies of an EventBatch (torch tensors) and the ds_events struct."""

    def __init__(self, batch, device="cuda", max_seeds_per_event=None, max_hits_per_event=None):
        import torch
        self.batch = batch
        dev = torch.device(device)
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.seed_off = f(batch.seed_off.astype(np.int32))
        self.sx, self.sy, self.stx, self.sty, self.sqop = (f(batch.sx), f(batch.sy), f(batch.stx), f(batch.sty),
                                                           f(batch.sqop))
        self.hit_off = f(batch.hit_off.astype(np.int32))
        self.hu = f(batch.hu)
        sec = getattr(batch, "hit_sector", None)
        self.hit_sector = f(sec.astype(np.uint8)) if sec is not None and len(sec) else None
        ms = int(np.max(np.diff(batch.seed_off))) if batch.n_events else 0
        mh = int(np.max(batch.hit_off[4::4] - batch.hit_off[0:-1:4])) if batch.n_events else 0
        self.n_events, self.n_seeds, self.n_hits = batch.n_events, batch.n_seeds, batch.n_hits
        self.max_seeds = max_seeds_per_event if max_seeds_per_event is not None else ms
        self.max_hits = max_hits_per_event if max_hits_per_event is not None else mh
        self.struct = self._make_struct()

    def _make_struct(self) -> DsEvents:
        s = DsEvents()
        s.n_events, s.n_seeds, s.n_hits = self.n_events, self.n_seeds, self.n_hits
        s.max_seeds_per_event, s.max_hits_per_event = self.max_seeds, self.max_hits
        s.seed_off, s.hit_off = _ptr(self.seed_off), _ptr(self.hit_off)
        s.sx, s.sy, s.stx, s.sty, s.sqop = (_ptr(self.sx), _ptr(self.sy), _ptr(self.stx), _ptr(self.sty),
                                            _ptr(self.sqop))
        s.hu = _ptr(self.hu)
        s.hit_sector = _ptr(self.hit_sector)
        return s


class DeviceTracks:
    """Track slots for n_seeds seeds (torch tensors) and the ds_tracks struct."""

    def __init__(self, n_seeds: int, device="cuda", with_cand: bool = True):
        import torch
        dev = torch.device(device)
        n = max(int(n_seeds), 1)
        self.n = int(n_seeds)
        for k in ("x", "y", "tx", "ty", "qop", "chi2", "score"):
            setattr(self, k, torch.zeros(n, dtype=torch.float32, device=dev))
        self.hits = torch.full((4, n), -1, dtype=torch.int32, device=dev)
        self.nhits = torch.zeros(n, dtype=torch.int32, device=dev)
        self.cand = torch.full((n,), -1, dtype=torch.int32, device=dev) if with_cand else None
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        s = DsTracks()
        for k in ("x", "y", "tx", "ty", "qop", "chi2", "score"):
            setattr(s, k, _ptr(getattr(self, k)))
        for L in range(4):
            s.hit[L] = _ptr(self.hits[L])
        s.nhits, s.cand, s.flags = _ptr(self.nhits), _ptr(self.cand), _ptr(self.flags)
        self.struct = s

    def to_numpy(self) -> Dict[str, np.ndarray]:
        n = self.n
        out = {k: getattr(self, k)[:n].cpu().numpy() for k in ("x", "y", "tx", "ty", "qop", "chi2", "score")}
        out["hits"] = self.hits[:, :n].cpu().numpy().T.copy()
        out["nhits"] = self.nhits[:n].cpu().numpy()
        if self.cand is not None:
            out["cand"] = self.cand[:n].cpu().numpy()
        out["flags"] = int(self.flags.item())
        return out


class DeviceVertices:
    """Vertex output for n_events events with cap_per_event slots each."""

    def __init__(self, n_events: int, cap_per_event: int = 1024, device="cuda", extras: bool = False):
        import torch
        dev = torch.device(device)
        self.n_events, self.cap = int(n_events), int(cap_per_event)
        self.extras = extras
        m = max(self.n_events * self.cap, 1)
        self.count = torch.zeros(max(self.n_events, 1), dtype=torch.int32, device=dev)
        self.i = torch.zeros(m, dtype=torch.int32, device=dev)
        self.j = torch.zeros(m, dtype=torch.int32, device=dev)
        for k in ("x", "y", "z", "doca"):
            setattr(self, k, torch.zeros(m, dtype=torch.float32, device=dev))
        self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        s = DsVertices()
        s.cap_per_event = self.cap
        s.count, s.i, s.j = _ptr(self.count), _ptr(self.i), _ptr(self.j)
        s.x, s.y, s.z, s.doca = _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.doca)
        s.overflow, s.flags = _ptr(self.overflow), _ptr(self.flags)
        if extras:
            self.m_pipi = torch.zeros(m, dtype=torch.float32, device=dev)
            self.m_ppi = torch.zeros(m, dtype=torch.float32, device=dev)
            self.lines = torch.zeros((4, m), dtype=torch.float32, device=dev)
            s.m_pipi, s.m_ppi = _ptr(self.m_pipi), _ptr(self.m_ppi)
            for l in range(4):
                s.line[l] = _ptr(self.lines[l])
        self.struct = s

    def to_numpy(self) -> Dict:
        out = {k: getattr(self, k).cpu().numpy() for k in ("i", "j", "x", "y", "z", "doca")}
        if self.extras:
            out["m_pipi"], out["m_ppi"] = self.m_pipi.cpu().numpy(), self.m_ppi.cpu().numpy()
            out["lines"] = self.lines.cpu().numpy().T.copy()
        out["count"] = self.count[:self.n_events].cpu().numpy()
        out["overflow"] = int(self.overflow.item())
        out["flags"] = int(self.flags.item())
        out["cap"] = self.cap
        return out


# ------------------------------------------------------- C ABI, same names

def ds_create(device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    _check(library().ds_create(C.byref(h), int(device)), "ds_create")
    return h


def ds_destroy(ctx) -> None:
    library().ds_destroy(ctx)


def ds_load_geometry(ctx, geometry: Dict, weights) -> None:
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    g = geometry_struct(geometry)
    _check(library().ds_load_geometry(ctx, C.byref(g), w.ctypes.data_as(C.POINTER(C.c_float)), w.size),
           "ds_load_geometry")


def ds_find_tracks(ctx, ev: DeviceEvents, trk: DeviceTracks, mode: int = DS_MODE_PERSISTENT, fuse_mlp: int = 1,
                   stream=None) -> None:
    _check(library().ds_find_tracks(ctx, C.byref(ev.struct), C.byref(trk.struct), int(mode), int(fuse_mlp),
                                    _stream_handle(stream)), "ds_find_tracks")


def ds_ghost_kill(ctx, ev: DeviceEvents, trk: DeviceTracks, stream=None) -> None:
    _check(library().ds_ghost_kill(ctx, C.byref(ev.struct), C.byref(trk.struct), _stream_handle(stream)),
           "ds_ghost_kill")


def ds_kill_clones(ctx, ev: DeviceEvents, trk: DeviceTracks, stream=None) -> None:
    _check(library().ds_kill_clones(ctx, C.byref(ev.struct), C.byref(trk.struct), _stream_handle(stream)),
           "ds_kill_clones")


class DeviceCandidates:
    """Candidate rows (n_seeds * slots) and the ds_candidates struct."""

    def __init__(self, n_seeds: int, slots: int, device="cuda"):
        import torch
        dev = torch.device(device)
        self.n_seeds, self.slots = int(n_seeds), int(slots)
        n = max(self.n_seeds * self.slots, 1)
        for k in ("seed", "cand", "nhits"):
            setattr(self, k, torch.zeros(n, dtype=torch.int32, device=dev))
        self.hits = torch.full((4, n), -1, dtype=torch.int32, device=dev)
        for k in ("x", "y", "tx", "ty", "qop", "chi2", "score"):
            setattr(self, k, torch.zeros(n, dtype=torch.float32, device=dev))
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        s = DsCandidates()
        s.capacity = self.n_seeds * self.slots
        for k in ("seed", "cand", "nhits", "x", "y", "tx", "ty", "qop", "chi2", "score", "flags"):
            setattr(s, k, _ptr(getattr(self, k)))
        for L in range(4):
            s.hit[L] = _ptr(self.hits[L])
        self.struct = s

    def to_numpy(self) -> Dict[str, np.ndarray]:
        m = self.n_seeds * self.slots
        out = {k: getattr(self, k)[:m].cpu().numpy() for k in ("seed", "cand", "nhits", "x", "y", "tx", "ty", "qop",
                                                              "chi2", "score")}
        out["hits"] = self.hits[:, :m].cpu().numpy().T.copy()
        out["flags"] = int(self.flags.item())
        return out


def ds_candidate_slots(ctx) -> int:
    return int(library().ds_candidate_slots(ctx))


def ds_score_candidates(ctx, ev: DeviceEvents, cands: DeviceCandidates, stream=None) -> None:
    _check(library().ds_score_candidates(ctx, C.byref(ev.struct), C.byref(cands.struct), _stream_handle(stream)),
           "ds_score_candidates")


def ds_vertex(ctx, ev: DeviceEvents, trk: DeviceTracks, score_max: float, vtx: DeviceVertices,
              mode: int = DS_MODE_PERSISTENT, stream=None) -> None:
    _check(library().ds_vertex(ctx, C.byref(ev.struct), C.byref(trk.struct), C.c_float(score_max),
                               C.byref(vtx.struct), int(mode), _stream_handle(stream)), "ds_vertex")


def ds_process(ctx, ev: DeviceEvents, trk: DeviceTracks, vtx: DeviceVertices, mode: int = DS_MODE_GRAPH,
               score_max: float = math.nan, stream=None) -> None:
    _check(library().ds_process(ctx, C.byref(ev.struct), C.byref(trk.struct), C.c_float(score_max),
                                C.byref(vtx.struct), int(mode), _stream_handle(stream)), "ds_process")


def ds_process_static(ctx, ev: DeviceEvents, trk: DeviceTracks, vtx: DeviceVertices, score_max: float = math.nan,
                      stream=None) -> None:
    _check(library().ds_process_static(ctx, C.byref(ev.struct), C.byref(trk.struct), C.c_float(score_max),
                                       C.byref(vtx.struct), _stream_handle(stream)), "ds_process_static")


def ds_load_lines(ctx, weights) -> None:
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    _check(library().ds_load_lines(ctx, w.ctypes.data_as(C.POINTER(C.c_float)), w.size), "ds_load_lines")


def ds_set_launch(ctx, kernel: int, block: int = 0, wg_per_cu: int = 0, bins: int = 0) -> None:
    _check(library().ds_set_launch(ctx, int(kernel), int(block), int(wg_per_cu), int(bins)), "ds_set_launch")


def ds_get_launch(ctx, kernel: int):
    b, w, n = C.c_int(), C.c_int(), C.c_int()
    _check(library().ds_get_launch(ctx, int(kernel), C.byref(b), C.byref(w), C.byref(n)), "ds_get_launch")
    return b.value, w.value, n.value


def ds_set_event_order(ctx, order: int) -> None:
    _check(library().ds_set_event_order(ctx, int(order)), "ds_set_event_order")


def ds_get_event_order(ctx) -> int:
    o = C.c_int()
    _check(library().ds_get_event_order(ctx, C.byref(o)), "ds_get_event_order")
    return o.value


def ds_set_step_fusion(ctx, fused: int) -> None:
    _check(library().ds_set_step_fusion(ctx, int(fused)), "ds_set_step_fusion")


def ds_get_step_fusion(ctx) -> int:
    o = C.c_int()
    _check(library().ds_get_step_fusion(ctx, C.byref(o)), "ds_get_step_fusion")
    return o.value


class Context:
    """Owning wrapper around a ds_ctx handle."""

    def __init__(self, device: int = 0, geometry: Optional[Dict] = None, weights=None):
        self.handle = ds_create(device)
        if geometry is not None:
            ds_load_geometry(self.handle, geometry, weights)

    def close(self):
        if self.handle:
            ds_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

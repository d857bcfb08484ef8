"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, the ctypes structs match the C layout, and host-side
argument checks answer without a GPU."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ds.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2503_13092_amd import build_lib, ds
    if build_lib.is_stale():
        build_lib.build()
    return ds.library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ds_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    from paper_2503_13092_amd import ds
    assert sorted(ds.EXPORTED) == names


def test_struct_layouts_match_header():
    from paper_2503_13092_amd import ds
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "ds.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("ds_geometry %zu\nds_events %zu\nds_tracks %zu\nds_vertices %zu\n", sizeof(ds_geometry),
         sizeof(ds_events), sizeof(ds_tracks), sizeof(ds_vertices));
  P(ds_geometry, max_l3) P(ds_geometry, n_closest) P(ds_geometry, gamma_c0) P(ds_geometry, newton_iters)
  P(ds_geometry, doca_max) P(ds_geometry, ghost_threshold) P(ds_geometry, clone_kill) P(ds_events, seed_off) P(ds_events, hu)
  P(ds_geometry, algorithm) P(ds_geometry, n_sectors) P(ds_geometry, sector_y0) P(ds_geometry, sector_tol)
  P(ds_events, hit_sector)
  P(ds_tracks, hit) P(ds_tracks, nhits) P(ds_tracks, flags) P(ds_vertices, count) P(ds_vertices, flags) P(ds_vertices, m_pipi) P(ds_vertices, line)
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe])
        out = subprocess.check_output([exe], text=True)
    vals = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    assert int(vals["ds_geometry"]) == C.sizeof(ds.DsGeometry)
    assert int(vals["ds_events"]) == C.sizeof(ds.DsEvents)
    assert int(vals["ds_tracks"]) == C.sizeof(ds.DsTracks)
    assert int(vals["ds_vertices"]) == C.sizeof(ds.DsVertices)
    for k, v in vals.items():
        if "." in k:
            T, f = k.split(".")
            cls = {"ds_geometry": ds.DsGeometry, "ds_events": ds.DsEvents, "ds_tracks": ds.DsTracks,
                   "ds_vertices": ds.DsVertices}[T]
            assert getattr(cls, f).offset == int(v), k


def test_host_side_errors_without_gpu(lib):
    from paper_2503_13092_amd import ds
    assert lib.ds_status_str(ds.DS_E_CAPACITY).startswith(b"DS_E_CAPACITY")
    assert lib.ds_create(None, 0) == ds.DS_E_ARG
    assert lib.ds_find_tracks(None, None, None, 1, 1, None) == ds.DS_E_ARG
    assert lib.ds_vertex(None, None, None, C.c_float(0.5), None, 1, None) == ds.DS_E_ARG
    assert lib.ds_set_launch(None, 0, 256, 4, 512) == ds.DS_E_ARG
    assert lib.ds_set_event_order(None, ds.DS_ORDER_LARGEST_FIRST) == ds.DS_E_ARG
    assert lib.ds_get_event_order(None, None) == ds.DS_E_ARG
    lib.ds_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2503_13092_amd import ds
    monkeypatch.setattr(ds, "LIB_PATH", "/nonexistent/libds.so")
    monkeypatch.setattr(ds, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        ds.library()


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2503_13092_amd")
    pat = re.compile(r"^\s*(from\s+oracle\b|import\s+oracle\b)|pyoracle|liboracle|orc_[a-z]+\(", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                assert not pat.search(open(os.path.join(dirpath, f)).read()), f

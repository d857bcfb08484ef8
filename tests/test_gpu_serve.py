"""The request loop on the GPU: each event's result is bitwise the same when
it is served alone, in a Poisson mix, and on the plain per-event path, and it
matches the oracle."""
import math
import sys

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2503_13092_amd import serve, synth
from tests import parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2503_13092_amd import ds  # noqa: E402

G = synth.default_geometry()
W = synth.mlp_weights()


def test_same_result_alone_in_mix_and_plain():
    b = synth.generate(2, n_events=300, seed=11)
    pool = serve.EventPool(b)
    got = {}

    def keep(a0, a1, res):
        for k in range(a1 - a0):
            got.setdefault((a0 + k) % pool.size, []).append(res.event(k))

    be = serve.GpuBackend(pool, G, W, n_slots=3, max_events=96)
    try:
        srv = serve.Server(be, pool)
        lat, st = srv.run(serve.poisson_arrivals(40000.0, 600, seed=5), on_result=keep)
        print(f"[serve] mix: {st.as_dict()}", flush=True)
        assert st.rejected == 0 and np.all(np.isfinite(lat))
        assert st.mean_batch > 1.0
        sample = [0, 1, 17, 150, 299]
        for e in sample:
            be.submit(0, e, e + 1)
            torch.cuda.synchronize()
            alone = be.fetch(0).event(0)
            for r in got[e]:
                for k in ("nhits", "hits", "score", "state", "vertices"):
                    assert np.array_equal(alone[k], r[k]), (e, k)
    finally:
        be.close()
    plain = serve.GpuBackend(pool, G, W, n_slots=1, max_events=8, mode=ds.DS_MODE_PER_EVENT)
    try:
        for e in (0, 17, 299):
            plain.submit(0, e, e + 1)
            torch.cuda.synchronize()
            r = plain.fetch(0).event(0)
            for k in ("nhits", "hits", "score", "state"):
                assert np.array_equal(r[k], got[e][0][k]), (e, k)
    finally:
        plain.close()
    # the served results against the oracle
    sub = b.subset(np.arange(40))
    ref = O.run_path(sub, G, W, cap=64)
    gt = dict(nhits=np.concatenate([got[e][0]["nhits"] for e in range(40)]),
              hits=np.concatenate([got[e][0]["hits"] for e in range(40)]),
              score=np.concatenate([got[e][0]["score"] for e in range(40)]))
    st_ = np.concatenate([got[e][0]["state"] for e in range(40)])
    for k, name in enumerate(("x", "y", "tx", "ty", "qop", "chi2")):
        gt[name] = st_[:, k]
    gt["cand"] = ref["tracks"]["cand"]
    tc = parity.compare_tracks(gt, ref["tracks"], check_cand=False)
    print(f"[serve] oracle check: {tc['identical']}/{tc['n']} identical", flush=True)

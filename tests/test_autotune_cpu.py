"""Host-only checks of the launch autotuner: the workload signature and the
committed cache of launch settings (the settings the benchmark and the
request loop apply), without a GPU."""
import json
import re

import numpy as np

from paper_2503_13092_amd import autotune, ds, synth


def test_signature_buckets_sizes_by_powers_of_two():
    b = synth.generate(0)   # 100 events x 20 seeds, about 2 000 hits per event
    sig = autotune.signature(b)
    assert re.fullmatch(r"E\d+-S\d+:\d+-H\d+:\d+", sig)
    assert sig.startswith("E7-")          # log2(100) = 6.6 -> 7
    s = np.diff(b.seed_off)
    assert f"-S{round(np.log2(s.mean()))}:{round(np.log2(s.max()))}-" in sig
    # the signature depends on sizes only, not on the values
    b2 = synth.generate(0, seed=99)
    assert autotune.signature(b2) == sig


def test_committed_cache_entries_are_valid_launch_settings():
    cache = autotune.load_cache()
    assert cache, "the package ships a tuned cache"
    for key, entry in cache.items():
        dev, alg, sig = key.split("|")
        assert re.fullmatch(r"gfx\d+-\d+cu", dev), key
        assert alg in ("alg0", "alg1"), key
        assert re.fullmatch(r"E\d+-S\d+:\d+-H\d+:\d+", sig), key
        best = entry["best"]
        assert best["block"] in autotune.SPACE["block"]
        assert best["wg_per_cu"] in autotune.SPACE["wg_per_cu"]
        assert best["bins"] in autotune.SPACE["bins"]
        assert best["order"] in (ds.DS_ORDER_INPUT, ds.DS_ORDER_LARGEST_FIRST)
        assert best["fused"] in (0, 1)
        v = best.get("vertex")
        if v:
            assert v["block"] in autotune.VERTEX_SPACE["block"]
            assert v["wg_per_cu"] in autotune.VERTEX_SPACE["wg_per_cu"]
        # the chosen point was confirmed no slower than the library default
        assert entry["ms"] <= entry["default_ms"] * 1.02
    json.dumps(cache)


def test_benchmark_workloads_have_cache_entries():
    """The three benchmark workloads (throughput, uneven, stress) and the Dv1
    throughput line find their tuned settings by signature."""
    cache = autotune.load_cache()
    sigs = {k.split("|", 1)[1] for k in cache}
    for config, alg in ((1, 0), (2, 0), (4, 0), (1, 1)):
        b = synth.generate(config)
        assert f"alg{alg}|{autotune.signature(b)}" in sigs, (config, alg)

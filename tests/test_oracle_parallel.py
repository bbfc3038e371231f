"""The oracle's range-parallel driver (the paper's Sec. 3 scheme: each thread
solves its own ranges) and its from-layer entry point build exactly what the
plain sequential builder builds: equal export bytes for every mode (2-bit and
1+-bit thresholds, searched cut points, filter mode, several widths and
layer counts) and thread count. Deeper layers built from a layer's own input
keys equal the corresponding sections of the whole build's export."""
import numpy as np
import pytest

import oracle
from paper_2411_12365_amd import workload as W
from tests import export_format

CASES = [
    (50_000, 8, dict(ranges=64)),
    (60_000, 16, dict(ranges=16, filter_mode=1, seed=3)),
    (40_000, 1, dict(ranges=200, minbpt=2, seed=4)),
    (70_000, 8, dict(ranges=32, threshold_mode=1, seed=5)),
    (70_000, 8, dict(ranges=32, cut_strategy=2, cut_search=50, seed=6)),
    (50_000, 5, dict(ranges=40, cut_strategy=3, cut_search=10, threshold_mode=1, seed=7)),
    (30_000, 8, dict(ranges=8, layers=5, load_num=85, load_den=100, seed=8)),
    (20_000, 32, dict(ranges=1)),
    (10, 8, dict(ranges=4)),
    (0, 8, dict(ranges=4)),
]


@pytest.mark.parametrize("n,r,kw", CASES)
@pytest.mark.parametrize("threads", [2, 3, 8])
def test_parallel_driver_equals_sequential(n, r, kw, threads):
    p = oracle.Params(**kw)
    keys = W.keys(n, 500 + n % 97)
    vals = None if p.filter_mode else W.values(n, r, 600 + n % 89)
    seq = oracle.build(keys, vals, r, p)
    par = oracle.build(keys, vals, r, p, threads=threads)
    assert par.export() == seq.export()
    for li in range(seq.layers_built):
        assert par.layer_info(li) == seq.layer_info(li)


@pytest.mark.parametrize("n,r,kw", [CASES[0], CASES[1], CASES[3], CASES[5]])
@pytest.mark.parametrize("threads", [1, 4])
def test_from_layer_equals_the_whole_builds_deeper_layers(n, r, kw, threads):
    p = oracle.Params(**kw)
    keys = W.keys(n, 500 + n % 97)
    vals = None if p.filter_mode else W.values(n, r, 600 + n % 89)
    whole = oracle.build(keys, vals, r, p)
    e = export_format.parse(whole.export())
    vmap = None if vals is None else dict(zip(keys.tolist(), vals.tolist()))
    for first in range(1, whole.layers_built + 1):
        k1 = whole.layer_keys(first)
        v1 = None if vmap is None else np.array([vmap[int(k)] for k in k1],
                                                dtype=oracle.value_dtype(r))
        part = oracle.build(k1, v1, r, p, threads=threads, first_layer=first)
        ep = export_format.parse(part.export())
        assert ep["header"]["first_layer"] == first
        assert [L["bytes"] for L in ep["layers"]] == [L["bytes"] for L in e["layers"][first:]]
        assert ep["final"]["bytes"] == e["final"]["bytes"]

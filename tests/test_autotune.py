"""Host logic of the scan autotuner: shape signature, choice rule and the JSON cache."""

import json

import numpy as np

from paper_2007_14135_amd import autotune


def _ula(M):
    p = np.zeros((M, 3))
    p[:, 0] = 0.5 * np.arange(M)
    return p


def test_signature_depends_on_shape_only():
    arrays = [_ula(16), _ula(8)]
    grids = [(-90, 0.01, 18000, 0), (-90, 0.1, 1800, 0)]
    fa = [(0, 0, 4096, 4, 0, 4096, 0), (0, 0, 2048, 4, 99, 2048, 0), (1, 1, 512, 2, 0, 512, 0)]
    fb = [(1, 1, 100, 2, 7, 100, 0), (0, 0, 10, 4, 3, 10, 0), (0, 0, 10, 4, 0, 10, 0)]   # other N, offsets, order
    s = autotune.signature(arrays, grids, fa, "music", "c64")
    assert s == autotune.signature(arrays, grids, fb, "music", "c64")
    assert s != autotune.signature(arrays, grids, fa, "music", "bf16")
    assert s != autotune.signature(arrays, grids, fa, "mn", "c64")
    assert s != autotune.signature(arrays, grids, fa, "music", "c64", "fp32")
    fc = [(0, 0, 4096, 3, 0, 4096, 0)] + fa[1:]                                           # another rank K
    assert s != autotune.signature(arrays, grids, fc, "music", "c64")


def test_choose_fastest_then_smallest():
    assert autotune.choose({384: 0.1, 256: 0.09, 512: 0.2}) == 256
    assert autotune.choose({384: 0.1, 256: 0.1}) == 256


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    c = autotune.Cache(path)
    assert c.get("dev", "sig") is None
    c.put("dev", "sig", 768, {384: 0.2, 768: 0.1})
    c2 = autotune.Cache(path)
    assert c2.get("dev", "sig") == 768 and c2.get("other", "sig") is None
    assert json.load(open(path))["dev"]["sig"]["timings_ms"]["768"] == 0.1

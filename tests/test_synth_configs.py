"""Workload recipes (synth/configs/*.json): the frames they draw, and the recipe language.

The digests were taken from the generator before its parameters moved into the JSON recipes;
they pin that every frame (parameters, source directions, positions and snapshot bits) is the
same draw from the same per-frame stream.
"""

import hashlib

import numpy as np
import pytest

from synth import frames as sf
from synth import make_frame

# (config/frame): (M, N, D, geometry, SNR dB, grid, sha256 prefix of X, angles, positions, polar)
DIGESTS = {
    'c1/0': (8, 1024, 2, 'ula', 10.0, (-90.0, 0.1, 1800), '1883e607e5c255cb'),
    'c2/0': (16, 4096, 4, 'ula', 1.183011354338, (-90.0, 0.01, 18000), '4d979907a7b47fd6'),
    'c2/1': (16, 4096, 4, 'ula', 4.40079469271, (-90.0, 0.01, 18000), '29efd3774124b066'),
    'c2/255': (16, 4096, 4, 'ula', 7.479687588614, (-90.0, 0.01, 18000), 'b6eaa373e003b2ea'),
    'c3/0': (8, 300, 1, 'uca', -4.947182073049, (-90.0, 0.002, 90000), '555bc93d9553116c'),
    'c3/1': (64, 300, 4, 'ula', 18.637265088241, (-90.0, 0.01, 18000), '176d46189e7c3bb0'),
    'c3/2': (32, 300, 6, 'ula', 2.879711530216, (-90.0, 0.01, 18000), '82773f47d2242225'),
    'c3/3': (16, 300, 1, 'ula', 2.899567735987, (-90.0, 0.1, 1800), '8030994611a4c8db'),
    'c3/4': (8, 300, 2, 'ula', 6.695272264513, (-90.0, 0.002, 90000), '77be3cd3c7ae07b2'),
    'c3/5': (8, 300, 2, 'uca', 3.177498423627, (-90.0, 0.1, 1800), '5dd46aa7d657338c'),
    'c3/4095': (16, 300, 3, 'uca', 2.18319524374, (-90.0, 0.1, 1800), '3df098a7ea172487'),
    'c4/0': (64, 512, 8, 'ula', 5.0, (-90.0, 0.001, 180000), 'f5c6d40091bc70f6'),
    'c4/63': (64, 512, 8, 'ula', 5.0, (-90.0, 0.001, 180000), '8566aaf371c7b217'),
    'c5/0': (16, 300, 4, 'ula', 9.706802841319, (-90.0, 0.001, 180000), 'a75f982542100d36'),
    'c5/1': (16, 300, 1, 'ula', 0.552192948061, (-90.0, 0.001, 180000), '25a730ab32e77fb5'),
    'c5/2': (16, 300, 4, 'ula', 11.13773562039, (-90.0, 0.001, 180000), '4aaa8b5675f6274a'),
    'c5/8191': (16, 300, 3, 'ula', -1.162161841497, (-90.0, 0.001, 180000), '29a8b5bd1a662ba4'),
    'c6/0': (8, 1024, 2, 'uca', 15.0, (0.0, 1.0, 360), '9e8b114dafc62e9a'),
    'c6/1': (8, 1024, 2, 'uca', 15.0, (0.0, 1.0, 360), '8f3893675a5605e2'),
}
# snapshot-count overrides of the long workloads, to keep the CPU suite quick
N_OVERRIDE = {"c3": 300, "c4": 512, "c5": 300}


@pytest.mark.parametrize("key", sorted(DIGESTS))
def test_recipe_frames_unchanged(key):
    c, i = key.split("/")
    n = N_OVERRIDE.get(c)
    f = make_frame(c, int(i), **({"N": n} if n else {}))
    h = hashlib.sha256()
    h.update(f.X.tobytes())
    h.update(f.angles_deg.tobytes())
    h.update(f.pos.tobytes())
    if f.polar_deg is not None:
        h.update(f.polar_deg.tobytes())
    got = (f.M, f.N, f.D, f.geometry, round(f.snr_db, 12), tuple(f.grid), h.hexdigest()[:16])
    assert got == DIGESTS[key]


def test_every_recipe_loads_with_its_readings():
    assert sorted(sf.CONFIGS) == ["c1", "c2", "c3", "c4", "c5", "c6"]
    assert [sf.CONFIGS[c].index for c in sorted(sf.CONFIGS)] == list(range(6))
    for c in sf.CONFIGS.values():
        assert c.readings, c.name
        p = c.draw(sf.config_seed(c.index, 0))
        assert p["pos"].shape == (p["M"], 3)
        assert p["grid"][2] >= 1
    assert sf.EL_GRIDS_2D[90] == (1.0, 1.0, 90) and sorted(sf.EL_GRIDS_2D) == [1, 30, 60, 90]


def test_recipe_values():
    rng = np.random.default_rng(5)
    env = {"M": 32}
    assert sf._value({"expr": "M // 4"}, env, rng) == 8
    assert sf._value({"expr": "0.5 * M / pi"}, env, rng) == pytest.approx(16.0 / np.pi)
    for _ in range(50):
        d = sf._value({"integers": [1, {"expr": "M // 4"}]}, env, rng)
        assert 1 <= d <= 8 and isinstance(d, int)
        n = sf._value({"log_uniform_int": [256, 8192]}, env, rng)
        assert 256 <= n <= 8192
        assert sf._value({"choice": [8, 16]}, env, rng) in (8, 16)
        assert sf._value({"coin": ["ula", "uca"]}, env, rng) in ("ula", "uca")
    # a literal consumes nothing from the stream
    a, b = np.random.default_rng(9), np.random.default_rng(9)
    sf._value(16, {}, a)
    assert a.uniform() == b.uniform()


@pytest.mark.parametrize("bad", [{"expr": "__import__('os')"}, {"expr": "M.real"},
                                 {"expr": "K + 1"}, {"normal": [0, 1]},
                                 {"uniform": [0, 1], "coin": [1, 2]}])
def test_recipe_rejects_unknown_forms(bad):
    with pytest.raises(ValueError):
        sf._value(bad, {"M": 8}, np.random.default_rng(0))


def test_uca_m_override_follows_the_radius_expression():
    # frame 0 of the uneven batch is a UCA (see DIGESTS); its radius is 0.5 M / pi wavelengths
    f = make_frame("c3", 0, M=16, N=64)
    assert f.geometry == "uca" and f.M == 16
    r = np.hypot(f.pos[:, 0], f.pos[:, 1])
    np.testing.assert_allclose(r, 8.0 / np.pi, rtol=1e-12)

"""The tile-shape autotuner: it times every shape of the force launch on
the workload, caches the fastest per shape bucket, and the handle built
with the chosen flags still matches the oracle."""
import json

import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, force_err, from_rows, host, to_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    return mixpi


def test_autotune_picks_a_shape_and_caches_it(mp, tmp_path):
    from paper_2411_11988_amd import tune
    s = synth.solvated_electron(70, 256, 13.0, seed=5, rc_pp=6.4, rc_aa=6.0, n_h=2, n_o=1)
    best, times = tune.autotune(s, reps=8)
    assert set(times) == {(32, 1), (32, 2), (64, 1), (64, 2)}
    assert all(np.isfinite(t) and t > 0 for t in times.values())
    assert times[best] == min(times.values())
    cache = tmp_path / "tiles.json"
    flags = tune.tile_flags(s, cache=str(cache))
    table = json.loads(cache.read_text())
    key = tune.bucket(s, mp.MIXPI_FP32_ACC64)
    assert key in table and (table[key]["tj"], table[key]["waves"]) in mp.TILE_FLAGS
    assert flags == mp.TILE_FLAGS[(table[key]["tj"], table[key]["waves"])]
    assert tune.tile_flags(s, cache=str(cache)) == flags       # read back, no retune
    sysm = mp.System(s, precision=mp.MIXPI_FP32_ACC64, flags=flags)
    f, _ = sysm.forces(dev(to_rows(s, s.q)))
    Fo, _ = oracle.OracleSystem(s).forces(s.q)
    assert force_err(from_rows(s, host(f)), Fo) <= 1e-5

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
    assert set(times) == {f"{tj}x{w}" for tj in tune.TJS for w in tune.WAVES}
    assert all(np.isfinite(t) and t > 0 for t in times.values())
    assert times[f"{best['tj'][tune.size_class(s)]}x{best['waves']}"] == min(times.values())
    cache = tmp_path / "tiles.json"
    flags = tune.tile_flags(s, cache=str(cache))
    table = json.loads(cache.read_text())
    key = tune.bucket(s, mp.MIXPI_FP32_ACC64)
    e = table[key]
    assert flags == mp.TILE_FLAGS[(e["tj"][tune.size_class(s)], e["waves"])]
    assert tune.tile_flags(s, cache=str(cache)) == flags       # read back, no retune
    sysm = mp.System(s, precision=mp.MIXPI_FP32_ACC64, flags=flags)
    f, _ = sysm.forces(dev(to_rows(s, s.q)))
    Fo, _ = oracle.OracleSystem(s).forces(s.q)
    assert force_err(from_rows(s, host(f)), Fo) <= 1e-5


def test_autotune_batch_per_class_widths(mp, tmp_path):
    """A batch of two size classes: the tuner returns one flag value per
    system, equal within a class, and the batch built with them matches each
    system's oracle forces."""
    from paper_2411_11988_amd import tune
    systems = [synth.solvated_electron(40, 64, 11.5, seed=k, rc_pp=5.5, rc_aa=5.4, n_h=2, n_o=1)
               for k in range(2)]
    systems += [synth.solvated_electron(90, 128, 14.0, seed=10 + k, rc_pp=6.4, rc_aa=6.0,
                                        n_h=2, n_o=1) for k in range(2)]
    assert len(set(tune.size_class(s) for s in systems)) == 2
    flags = tune.tile_flags(systems, cache=str(tmp_path / "tiles.json"))
    assert isinstance(flags, list) and len(flags) == 4
    assert flags[0] == flags[1] and flags[2] == flags[3]
    b = mp.System(systems, precision=mp.MIXPI_FP32_ACC64, flags=flags)
    off = 0
    idx = b.bead_index
    qa = np.concatenate([s.q for s in systems])
    qr = np.empty_like(qa)
    qr[idx] = qa
    f, _ = b.forces(dev(qr))
    F = host(f)[idx]
    for s in systems:
        n = len(s.q)
        Fo, _ = oracle.OracleSystem(s).forces(s.q)
        assert force_err(F[off:off + n], Fo) <= 1e-5
        off += n


def test_default_shape_by_work_size(mp):
    """Without shape flags the handle picks the tile shape from its work
    size (64 x 64 tiles): 16-wide j-tiles and two j-split waves for the
    64-bead electron with 32 waters, 16-wide tiles with one wave for the
    1024-bead electron with 512 waters, 64-wide tiles with two i-split
    waves and runs of four j-tiles for the 64-system batch."""
    for make, want in ((synth.config_c1, ([16], 2, 1, 1)), (synth.config_c3, ([16], 1, 1, 1))):
        s = make()
        sysm = mp.System(s)
        assert sysm.pair_shape() == want, (s.name, sysm.pair_shape())
        sysm.close()
    systems = synth.config_c5(workers=synth.build_workers())
    b = mp.System(systems)
    tj, w, iw, jr = b.pair_shape()
    assert tj == [64] * len(systems) and (w, iw, jr) == (1, 2, 4), (tj[:3], w, iw, jr)
    b.close()
    # flags override, per system in a batch
    fl = [mp.TILE_FLAGS[(32, "w2")], mp.TILE_FLAGS[(16, "w2")]]
    b = mp.System([synth.config_c1(), synth.config_c1()], flags=fl)
    assert b.pair_shape() == ([32, 16], 2, 1, 1)
    b.close()

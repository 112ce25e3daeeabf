"""The C-ABI library loads, exports exactly what include/mixpi.h declares,
and rejects invalid descriptions before touching the GPU (CPU-only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    if not os.path.exists(mixpi.LIB_PATH):
        from paper_2411_11988_amd import build
        build.build()
    mixpi.load()
    return mixpi


def _declared():
    src = open(os.path.join(ROOT, "include", "mixpi.h")).read()
    return sorted(set(re.findall(r"\b(mixpi_[a-z_]+)\s*\(", src)))


def _exported(path):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True,
                         text=True, check=True).stdout
    return sorted(l.split()[-1] for l in out.splitlines() if " T mixpi_" in l)


def test_exports_match_header(mp):
    declared = _declared()
    assert len(declared) >= 12
    assert _exported(mp.LIB_PATH) == declared
    lib = C.CDLL(mp.LIB_PATH)
    for name in declared:
        assert getattr(lib, name) is not None


def _desc(mp, s, **over):
    d, keep = mp.make_desc(s)
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


def test_rejects_non_power_of_two(mp):
    s = synth.tiny_random(0)
    s.n_beads = s.n_beads.copy()
    s.n_beads[0] = 3
    s.q = np.zeros((int(s.n_beads.sum()), 3))
    d, keep = _desc(mp, s)
    with pytest.raises(mp.MixPIError) as e:
        mp.mixpi_create(d)
    assert e.value.code == mp.MIXPI_E_NOT_POW2
    assert "power of two" in str(e.value)


def test_rejects_increasing_bead_counts(mp):
    s = synth.tiny_random(0, bead_choices=(1, 2, 4, 8))
    s.n_beads = s.n_beads[::-1].copy()
    d, keep = _desc(mp, s)
    with pytest.raises(mp.MixPIError) as e:
        mp.mixpi_create(d)
    assert e.value.code == mp.MIXPI_E_ORDER


def test_rejects_bad_parameters(mp):
    s = synth.tiny_random(0)
    for field, value in [("pp_a", 0.0), ("temperature", -1.0), ("rc_lj", float("nan")),
                         ("precision", 7), ("n_particles", 0), ("n_lj_types", 9)]:
        d, keep = _desc(mp, s, **{field: value})
        with pytest.raises(mp.MixPIError) as e:
            mp.mixpi_create(d)
        assert e.value.code in (mp.MIXPI_E_INVALID, mp.MIXPI_E_UNSUPPORTED), field
    d, keep = _desc(mp, s)
    d.mass = None
    with pytest.raises(mp.MixPIError) as e:
        mp.mixpi_create(d)
    assert e.value.code == mp.MIXPI_E_INVALID


def test_rejects_bad_topology(mp):
    s = synth.water_box(4, 6.0, 2, 1, seed=0, rc=2.9)
    s.bonds = s.bonds.copy()
    s.bonds[0, 1] = 999
    d, keep = _desc(mp, s)
    with pytest.raises(mp.MixPIError) as e:
        mp.mixpi_create(d)
    assert e.value.code == mp.MIXPI_E_INVALID and "bond" in str(e.value)


def test_null_handle_and_out(mp):
    lib = mp.load()
    assert lib.mixpi_forces(None, None, None, None, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_forces_static(None, None, None, None, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_step(None, 1, None, None, None, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_create(None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_rdf(None, None, 5.0, 10, 9, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_vacf_sample(None, None, 0, 4, 9, None, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_set_ewald(None, 0.3, 5.0, 32, 6) == mp.MIXPI_E_INVALID
    assert lib.mixpi_ewald(None, None, None, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_use_ewald(None, 1) == mp.MIXPI_E_INVALID
    assert lib.mixpi_layout(None, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_batch_step(None, 1, None, None, None, None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_destroy(None) == mp.MIXPI_OK
    assert b"null" in lib.mixpi_last_error()


def test_rejects_out_of_range_mol_id(mp):
    s = synth.tiny_random(0)
    for bad in (-1, 1 << 27):
        s2 = synth.tiny_random(0)
        s2.mol_id = s.mol_id.copy()
        s2.mol_id[2] = bad
        with pytest.raises(mp.MixPIError) as e:
            mp.System(s2)
        assert e.value.code == mp.MIXPI_E_INVALID and "mol_id" in str(e.value)


def test_rejects_conflicting_tile_flags(mp):
    s = synth.tiny_random(0)
    for bad in (mp.MIXPI_FLAG_TILE_J32 | mp.MIXPI_FLAG_TILE_J64,
                mp.MIXPI_FLAG_TILE_J16 | mp.MIXPI_FLAG_TILE_J32,
                mp.MIXPI_FLAG_TILE_J16 | mp.MIXPI_FLAG_TILE_J64,
                mp.MIXPI_FLAG_TILE_WAVES1 | mp.MIXPI_FLAG_TILE_WAVES2,
                mp.MIXPI_FLAG_TILE_WAVES2 | mp.MIXPI_FLAG_TILE_I128,
                mp.MIXPI_FLAG_TILE_I128 | mp.MIXPI_FLAG_TILE_I256, 1 << 12):
        with pytest.raises(mp.MixPIError) as e:
            mp.System(s, flags=bad)
        assert e.value.code == mp.MIXPI_E_INVALID and "flags" in str(e.value)


def test_batch_flags_may_differ_in_tile_width_only(mp):
    """The systems of a batch may carry different j-tile width flags; any
    other flag difference is rejected before the device is touched."""
    s0, s1 = synth.tiny_random(0), synth.tiny_random(1)
    with pytest.raises(mp.MixPIError) as e:
        mp.System([s0, s1], flags=[mp.MIXPI_FLAG_TILE_WAVES1, mp.MIXPI_FLAG_TILE_WAVES2])
    assert e.value.code == mp.MIXPI_E_INVALID and "flags" in str(e.value)
    try:
        mp.System([s0, s1], flags=[mp.MIXPI_FLAG_TILE_J16, mp.MIXPI_FLAG_TILE_J64]).close()
    except mp.MixPIError as err:   # no device here: only the device step may fail
        assert err.code == mp.MIXPI_E_HIP, err
    with pytest.raises(ValueError):
        mp.System([s0, s1], flags=[0])

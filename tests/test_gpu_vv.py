"""Velocity Verlet with the ring-polymer springs as forces (the paper's
second integrator) through the C-ABI, against the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, energy_err, from_rows, host, layout_rows, to_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    return mixpi


CASES = [
    ("tiny1", lambda: synth.tiny_random(1)),
    ("c1", synth.config_c1),
    ("water-h8-o2", lambda: synth.water_box(40, 11.0, 8, 2, seed=4, rc=5.4)),
    ("e256-water", lambda: synth.solvated_electron(70, 256, 13.0, seed=5, rc_pp=6.4, rc_aa=6.0,
                                                   n_h=2, n_o=1)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_vv_matches_oracle(mp, name, make):
    import torch
    print(f"[vv] {name}", flush=True)
    s = make()
    nsteps = 6
    rows = layout_rows(s)
    o = oracle.OracleSystem(s)
    Fo0, _ = o.forces(s.q)
    qo, po, _, elo = o.step_vv(s.q, s.p, nsteps, F=Fo0)
    sysm = mp.System(s)
    q, p = dev(to_rows(s, s.q, rows)), dev(to_rows(s, s.p, rows))
    f = dev(to_rows(s, Fo0, rows))
    elog = torch.zeros((nsteps, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step_vv(nsteps, q, p, f, elog)
    qg, pg = from_rows(s, host(q), rows), from_rows(s, host(p), rows)
    el = host(elog)[:, 0, :]
    assert np.abs(qg - qo).max() <= 1e-12 * np.abs(qo).max()
    assert np.abs(pg - po).max() <= 1e-12 * np.abs(po).max()
    assert max(energy_err(el[k], elo[k]) for k in range(nsteps)) <= 1e-12


def test_vv_then_split_propagator_on_one_handle(mp):
    """Sequences of both integrators on one handle keep their own graphs and
    energy bookkeeping: VV, then NVE, then VV again match the oracle run the
    same way."""
    import torch
    s = synth.config_c1()
    rows = layout_rows(s)
    o = oracle.OracleSystem(s)
    F0, _ = o.forces(s.q)
    q1, p1, F1, _ = o.step_vv(s.q, s.p, 3, F=F0)
    q2, p2, F2, _ = o.step(q1, p1, 3, F=F1)
    q3, p3, F3, el3 = o.step_vv(q2, p2, 3, F=F2)
    sysm = mp.System(s)
    q, p = dev(to_rows(s, s.q, rows)), dev(to_rows(s, s.p, rows))
    f = dev(to_rows(s, F0, rows))
    elog = torch.zeros((3, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step_vv(3, q, p, f, elog)
    sysm.step(3, q, p, f, elog)
    sysm.step_vv(3, q, p, f, elog)
    assert np.abs(from_rows(s, host(q), rows) - q3).max() <= 1e-12 * np.abs(q3).max()
    assert max(energy_err(host(elog)[k, 0], el3[k]) for k in range(3)) <= 1e-12


@pytest.mark.parametrize("rpw", [2, 4])
def test_vv_with_grouped_epilogue_rows(mp, rpw, monkeypatch):
    """The velocity-Verlet epilogue (neighbour-row spring forces, spring
    energy) with 2 or 4 bead rows per wave matches the oracle."""
    import torch
    monkeypatch.setenv("MIXPI_FIN_RPW", str(rpw))
    for name, make in CASES[1:]:
        print(f"[vv rpw={rpw}] {name}", flush=True)
        s = make()
        rows = layout_rows(s)
        o = oracle.OracleSystem(s)
        Fo0, _ = o.forces(s.q)
        qo, po, _, elo = o.step_vv(s.q, s.p, 3, F=Fo0)
        sysm = mp.System(s)
        q, p = dev(to_rows(s, s.q, rows)), dev(to_rows(s, s.p, rows))
        f = dev(to_rows(s, Fo0, rows))
        elog = torch.zeros((3, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
        sysm.step_vv(3, q, p, f, elog)
        assert np.abs(from_rows(s, host(q), rows) - qo).max() <= 1e-12 * np.abs(qo).max()
        assert np.abs(from_rows(s, host(p), rows) - po).max() <= 1e-12 * np.abs(po).max()
        assert max(energy_err(host(elog)[k, 0], elo[k]) for k in range(3)) <= 1e-12

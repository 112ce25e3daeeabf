"""Degenerate and extreme inputs through the C-ABI against the FP64 oracle:
systems without a single interacting pair, a molecule whose pairs are all
excluded, ragged tile tails, the largest ring the library takes, and an
electron bead on top of an atom."""
import math

import numpy as np
import pytest

import oracle
from tests._gpu import dev, energy_err, force_err, from_rows, host, layout_rows, to_rows
from tests._systems import custom, lj_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    return mixpi


def _momenta(s, seed):
    rng = np.random.default_rng(seed)
    m = np.repeat(s.fict_mass, s.n_beads)[:, None]
    return rng.normal(size=s.q.shape) * np.sqrt(m * 0.0025)


def _check(mp, s, nsteps=3, precisions=(0, 1)):
    """Forces in both forms and FP64 steps against the oracle."""
    import dataclasses
    import torch
    s = dataclasses.replace(s, p=_momenta(s, 1))
    rows = layout_rows(s)
    o = oracle.OracleSystem(s)
    Fo, eo = o.forces(s.q)
    for prec in precisions:
        sysm = mp.System(s, precision=prec)
        f, e = sysm.forces(dev(to_rows(s, s.q, rows)))
        F = from_rows(s, host(f), rows)
        if np.abs(Fo).max() == 0.0:
            assert np.abs(F).max() == 0.0
        else:
            assert force_err(F, Fo) <= (1e-12 if prec == 0 else 1e-5)
        if prec == 0:
            assert energy_err(host(e)[0], eo) <= 1e-12
    sysm = mp.System(s)
    q, p = dev(to_rows(s, s.q, rows)), dev(to_rows(s, s.p, rows))
    f, _ = sysm.forces(q)
    elog = torch.zeros((nsteps, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step(nsteps, q, p, f, elog)
    qo, po, _, elo = o.step(s.q, s.p, nsteps)
    assert np.abs(from_rows(s, host(q), rows) - qo).max() <= 1e-12 * max(1.0, np.abs(qo).max())
    assert np.abs(from_rows(s, host(p), rows) - po).max() <= 1e-12 * max(1e-30, np.abs(po).max())
    for k in range(nsteps):
        assert energy_err(host(elog)[k, 0], elo[k]) <= 1e-12


def test_lone_ring(mp):
    """One 8-bead particle: no pair tiles, no bonded terms; the step is the
    exact free ring polymer."""
    q = np.random.default_rng(0).normal(size=(8, 3)) * 0.2 + 5.0
    _check(mp, custom([8], q, box=20.0, rc=9.0))


def test_electrons_only(mp):
    """Two electrons: electron-electron pairs do not interact."""
    q = np.random.default_rng(1).normal(size=(32, 3)) + 5.0
    _check(mp, custom([16, 16], q, ele=[1, 1], box=20.0, rc=9.0, mass=[1.008, 1.008]))


def test_one_molecule_all_pairs_excluded(mp):
    """Four atoms of one molecule: every pair excluded, bonds and an angle
    carry all the forces."""
    q = np.array([[0, 0, 0], [1.0, 0, 0], [0, 1.0, 0.1], [1.2, 1.1, 0.3]]) + 5.0
    e, sg = lj_table(0, 0, 0.2, 3.0)
    s = custom([1, 1, 1, 1], q, charge=[0.4, -0.4, 0.3, -0.3], lj_type=[0, 0, 0, 0],
               mol=[7, 7, 7, 7], eps=e, sig=sg, bonds=[(0, 1), (0, 2), (1, 3)],
               angles=[(1, 0, 2)], box=20.0, rc=9.0)
    _check(mp, s)


@pytest.mark.parametrize("n_atoms", [1, 33, 65, 97])
def test_ragged_tile_tails(mp, n_atoms):
    """A 64-bead electron with 1, 33, 65 or 97 one-bead atoms: j-tiles and
    i-tiles that end part-way.  The atoms keep 2.2 A apart (random
    sequential placement), so that the steps stay in a smooth regime."""
    rng = np.random.default_rng(n_atoms)
    L = 16.0
    atoms = []
    while len(atoms) < n_atoms:
        x = rng.uniform(0, L, size=3)
        d = np.array(atoms).reshape(-1, 3) - x
        d -= L * np.rint(d / L)
        if len(atoms) == 0 or (d * d).sum(axis=1).min() >= 2.2 ** 2:
            atoms.append(x)
    atoms = np.array(atoms)
    elec = rng.normal(size=(64, 3)) * 0.8 + L / 2
    q = np.concatenate([elec, atoms])
    chg = np.concatenate([[0.0], rng.choice([-0.8, 0.4], size=n_atoms)])
    e, sg = lj_table(1, 1, 0.15, 3.1)
    s = custom([64] + [1] * n_atoms, q, charge=chg, lj_type=[3] + [1] * n_atoms,
               ele=[1] + [0] * n_atoms, eps=e, sig=sg, box=L, rc=7.5,
               mass=[1.008] + [15.999] * n_atoms)
    _check(mp, s, nsteps=2)


def test_largest_ring(mp):
    """The largest ring the library takes (4096 beads, FFT normal modes) next
    to 40 one-bead atoms."""
    rng = np.random.default_rng(7)
    L = 14.0
    atoms = rng.uniform(0, L, size=(40, 3))
    elec = rng.normal(size=(4096, 3)) * 0.7 + L / 2
    q = np.concatenate([elec, atoms])
    chg = rng.choice([-0.8, 0.4], size=40)
    s = custom([4096] + [1] * 40, q, charge=np.concatenate([[0.0], chg]),
               lj_type=[3] + [2] * 40, ele=[1] + [0] * 40, box=L, rc=6.5,
               mass=[1.008] + [15.999] * 40)
    _check(mp, s, nsteps=2)


def test_electron_bead_on_an_atom(mp):
    """An electron bead exactly on an ion (r = 0 for the softened
    pseudopotential): finite forces equal to the oracle's."""
    q = np.zeros((9, 3)) + 5.0
    q[1:8] += np.random.default_rng(3).normal(size=(7, 3)) * 0.5
    s = custom([8, 1], q, charge=[0.0, 3.0], ele=[1, 0], box=20.0, rc=9.0,
               mass=[1.008, 58.9])
    assert np.array_equal(s.q[0], s.q[8])
    _check(mp, s)

"""Batched handles (many independent systems in one set of launches) through
the C-ABI: every system's forces, energies and steps must equal what a
handle of that system alone computes, and match the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import (dev, energy_err, energy_err_scale, force_err, from_rows, host,
                        layout_rows, to_rows)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    return mixpi


def batch_rows(systems):
    """Rows of every (system, particle, bead) in the batched layout: the
    systems' own layouts concatenated in order."""
    out, off = [], 0
    for s in systems:
        r = layout_rows(s)
        out.append(r + off)
        off += len(r)
    return out, off


def mixed_batch():
    return [synth.tiny_random(2), synth.config_c1(),
            synth.water_box(40, 11.0, 8, 2, seed=4, rc=5.4),
            synth.solvated_electron(70, 256, 13.0, seed=5, rc_pp=6.4, rc_aa=6.0, n_h=2, n_o=1),
            synth.tiny_random(3, n_particles=90, box=14.0, bead_choices=(1, 2, 4, 8, 16))]


def pack(systems, arrs):
    rows, total = batch_rows(systems)
    out = np.zeros((total, 3))
    for r, a in zip(rows, arrs):
        out[r] = a
    return out, rows


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_forces_match_single_and_oracle(mp, prec):
    systems = mixed_batch()
    b = mp.System(systems, precision=prec)
    assert b.n_systems == len(systems)
    q, rows = pack(systems, [s.q for s in systems])
    assert np.array_equal(b.bead_index, np.concatenate(rows))
    f, e = b.forces(dev(q))
    f, e = host(f), host(e)
    tol_f, tol_e = (1e-12, 1e-12) if prec == 0 else (1e-5, 1e-6)
    for k, s in enumerate(systems):
        print(f"[batch forces] system {k} prec={prec}", flush=True)
        one = mp.System(s, precision=prec)
        f1, e1 = one.forces(dev(to_rows(s, s.q)))
        F1 = from_rows(s, host(f1))
        Fb = f[rows[k]]
        assert force_err(Fb, F1) <= 1e-13
        assert energy_err(e[k], host(e1)[0]) <= 1e-13
        Fo, eo = oracle.OracleSystem(s).forces(s.q)
        assert force_err(Fb, Fo) <= tol_f
        err = energy_err(e[k], eo) if prec == 0 else energy_err_scale(e[k], eo)
        assert err <= tol_e


def test_batch_step_matches_single_and_oracle(mp):
    import torch
    systems = mixed_batch()
    b = mp.System(systems)
    q, rows = pack(systems, [s.q for s in systems])
    p, _ = pack(systems, [s.p for s in systems])
    qd, pd = dev(q), dev(p)
    fd, _ = b.forces(qd)
    nsteps = 3
    elog = torch.zeros((nsteps, len(systems), 11), dtype=torch.float64, device="cuda")
    b.step(nsteps, qd, pd, fd, elog)
    qb, pb, el = host(qd), host(pd), host(elog)
    for k, s in enumerate(systems):
        print(f"[batch step] system {k}", flush=True)
        one = mp.System(s)
        q1, p1 = dev(to_rows(s, s.q)), dev(to_rows(s, s.p))
        f1, _ = one.forces(q1)
        el1 = torch.zeros((nsteps, 1, 11), dtype=torch.float64, device="cuda")
        one.step(nsteps, q1, p1, f1, el1)
        Q1, P1 = from_rows(s, host(q1)), from_rows(s, host(p1))
        scale_q = np.abs(Q1).max()
        scale_p = np.abs(P1).max()
        assert np.abs(qb[rows[k]] - Q1).max() <= 1e-13 * scale_q
        assert np.abs(pb[rows[k]] - P1).max() <= 1e-13 * scale_p
        assert np.allclose(el[:, k, :], host(el1)[:, 0, :], rtol=1e-12, atol=1e-12)
        qo, po, _, elo = oracle.OracleSystem(s).step(s.q, s.p, nsteps)
        assert np.abs(qb[rows[k]] - qo).max() <= 1e-11 * scale_q
        assert np.abs(pb[rows[k]] - po).max() <= 1e-10 * scale_p
        for t in range(nsteps):
            assert energy_err(el[t, k, :], elo[t]) <= 1e-10, (t, el[t, k], elo[t])


@pytest.mark.timeout(400)
def test_batch_full_size_sampled(mp):
    """The 64-system batch of uneven electron/water systems: forces of the
    batched handle in both forms, sampled systems against the oracle."""
    print("[c5 sampled] generating the 64-system batch", flush=True)
    systems = synth.config_c5()
    q, rows = pack(systems, [s.q for s in systems])
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        b = mp.System(systems, precision=prec)
        f, e = b.forces(dev(q))
        f, e = host(f), host(e)
        assert np.isfinite(f).all() and np.isfinite(e).all()
        for k in (0, 21, 63):
            print(f"[c5 sampled] system {k} prec={prec}", flush=True)
            s = systems[k]
            Fo, eo = oracle.OracleSystem(s).forces(s.q)
            assert force_err(f[rows[k]], Fo) <= tol
            err = energy_err(e[k], eo) if prec == 0 else energy_err_scale(e[k], eo)
            assert err <= (1e-12 if prec == 0 else 1e-6)
        del b


def test_batch_pair_counts(mp):
    """The device pair-evaluation counter of a batch is the sum of the
    oracle's per-system in-cutoff slice-pair counts."""
    systems = mixed_batch()
    b = mp.System(systems)
    q, _ = pack(systems, [s.q for s in systems])
    b.pair_evals(reset=True)
    b.forces(dev(q))
    aa, ea = b.pair_evals(reset=True)
    want = np.sum([oracle.OracleSystem(s).pair_evals(s.q) for s in systems], axis=0)
    assert (aa, ea) == (int(want[0]), int(want[1]))

"""Batched handles (many independent systems in one set of launches) through
the C-ABI: every system's forces, energies and steps must equal what a
handle of that system alone computes, and match the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, energy_err, force_err, from_rows, host, layout_rows, to_rows

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
        err = energy_err(e[k], eo)
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
        assert np.abs(qb[rows[k]] - qo).max() <= 1e-12 * np.abs(qo).max()
        assert np.abs(pb[rows[k]] - po).max() <= 1e-12 * np.abs(po).max()
        for t in range(nsteps):
            assert energy_err(el[t, k, :], elo[t]) <= 1e-12, (t, el[t, k], elo[t])


@pytest.fixture(scope="module")
def c5():
    """The 64-system batch of uneven electron/ion/water systems (built in
    worker processes; each system has its own seed) and its rows."""
    print("[c5] generating the 64-system batch", flush=True)
    systems = synth.config_c5(workers=synth.build_workers())
    q, rows = pack(systems, [s.q for s in systems])
    p, _ = pack(systems, [s.p for s in systems])
    return systems, q, p, rows


@pytest.mark.timeout(400)
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_full_size_forces_every_system(mp, c5, prec):
    """The 64-system batch at full size: forces and energies of every
    system of the batched handle against the oracle (FP64 form 1e-12; FP32
    form forces 1e-5 x RMS, energies 1e-6 per term), and equal bits from a
    repeated call."""
    systems, q, _, rows = c5
    b = mp.System(systems, precision=prec)
    qd = dev(q)
    f, e = b.forces(qd)
    f, e = host(f), host(e)
    assert np.isfinite(f).all() and np.isfinite(e).all()
    # the same bits from a second call (several waves of a tile add to the
    # same j-partials: their sums keep a fixed order)
    f2, e2 = b.forces(qd)
    assert np.array_equal(f, host(f2)) and np.array_equal(e, host(e2))
    tol_f, tol_e = (1e-12, 1e-12) if prec == 0 else (1e-5, 1e-6)
    worst_f = worst_e = 0.0
    for k, s in enumerate(systems):
        Fo, eo = oracle.OracleSystem(s).forces(s.q)
        ef, ee = force_err(f[rows[k]], Fo), energy_err(e[k], eo)
        worst_f, worst_e = max(worst_f, ef), max(worst_e, ee)
        assert ef <= tol_f, (k, ef)
        assert ee <= tol_e, (k, ee, e[k], eo)
    print(f"[c5 forces] prec={prec}: worst force err {worst_f:.2e}, energy err {worst_e:.2e}",
          flush=True)
    del b


@pytest.mark.timeout(400)
def test_batch_full_size_step_fp64(mp, c5):
    """Two FP64 steps of the whole 64-system batch (one handle, one graph):
    every system's positions, momenta and energy log against two oracle
    steps of that system alone."""
    import torch
    systems, q, p, rows = c5
    b = mp.System(systems)
    qd, pd = dev(q), dev(p)
    fd, _ = b.forces(qd)
    nsteps = 2
    elog = torch.zeros((nsteps, len(systems), mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    b.step(nsteps, qd, pd, fd, elog)
    qb, pb, el = host(qd), host(pd), host(elog)
    worst = [0.0, 0.0, 0.0]
    for k, s in enumerate(systems):
        qo, po, _, elo = oracle.OracleSystem(s).step(s.q, s.p, nsteps)
        dq = np.abs(qb[rows[k]] - qo).max() / np.abs(qo).max()
        dp = np.abs(pb[rows[k]] - po).max() / np.abs(po).max()
        de = max(energy_err(el[t, k], elo[t]) for t in range(nsteps))
        worst = [max(worst[0], dq), max(worst[1], dp), max(worst[2], de)]
        assert dq <= 1e-12, (k, dq)
        assert dp <= 1e-12, (k, dp)
        assert de <= 1e-12, (k, de)
    print(f"[c5 step64] worst dq/max|q| {worst[0]:.2e}, dp/max|p| {worst[1]:.2e}, "
          f"energy {worst[2]:.2e}", flush=True)
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


@pytest.mark.parametrize("waves,jrun", [("w1", 2), ("i2", 2), ("w2", 1)])
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_mixed_widths_with_j_runs(mp, prec, waves, jrun, monkeypatch):
    """A batch whose systems sweep with different tile widths (16, 32 and
    64 j-beads in one force launch), with i-split waves and j-runs: every
    system against the oracle, and equal bits from a repeated call."""
    monkeypatch.setenv("MIXPI_PAIR_JRUN", str(jrun))
    systems = mixed_batch()
    widths = [16, 64, 32, 64, 16]
    flags = [mp.TILE_FLAGS[(tj, waves)] for tj in widths]
    b = mp.System(systems, precision=prec, flags=flags)
    tj, w, iw, jr = b.pair_shape()
    assert list(tj) == widths and jr == jrun
    q, rows = pack(systems, [s.q for s in systems])
    qd = dev(q)
    f, e = b.forces(qd)
    f, e = host(f), host(e)
    f2, e2 = b.forces(qd)
    assert np.array_equal(f, host(f2)) and np.array_equal(e, host(e2))
    tol_f, tol_e = (1e-12, 1e-12) if prec == 0 else (1e-5, 1e-6)
    for k, s in enumerate(systems):
        print(f"[batch widths] system {k} prec={prec} {waves} jrun={jrun}", flush=True)
        Fo, eo = oracle.OracleSystem(s).forces(s.q)
        assert force_err(f[rows[k]], Fo) <= tol_f, k
        assert energy_err(e[k], eo) <= tol_e, k


def test_layout_matches_bead_index(mp):
    """mixpi_layout's groups reproduce every system's bead rows: bead a of
    particle p of a group at first_row + a n + (p - first particle)."""
    systems = mixed_batch()
    b = mp.System(systems)
    lay = b.layout()
    assert lay.shape == (b.n_groups, 5)
    nb = np.concatenate([np.asarray(s.n_beads) for s in systems])
    sys_of = np.concatenate([np.full(len(s.n_beads), k) for k, s in enumerate(systems)])
    first = np.concatenate([[0], np.cumsum(nb)[:-1]])
    seen = np.zeros(b.rows, dtype=bool)
    for row0, N, n, p0, k in lay:
        assert np.all(nb[p0:p0 + n] == N) and np.all(sys_of[p0:p0 + n] == k)
        for i in range(n):
            got = b.bead_index[first[p0 + i]:first[p0 + i] + N]
            assert np.array_equal(got, row0 + np.arange(N) * n + i)
        seen[row0:row0 + N * n] = True
    assert seen.all()
    assert np.all(np.diff(lay[:, 0]) > 0)


def test_batch_step_with_separate_arrays(mp):
    """mixpi_batch_step with one device array per system equals mixpi_step
    on the systems' rows back to back, bit for bit, both with separate
    allocations (staged) and with views into one allocation (direct), over
    two calls in a row."""
    import torch
    systems = mixed_batch()
    b = mp.System(systems)
    q, rows = pack(systems, [s.q for s in systems])
    p, _ = pack(systems, [s.p for s in systems])
    qd, pd = dev(q), dev(p)
    fd, _ = b.forces(qd)
    n_steps, ne = 3, mp.MIXPI_NE
    el_ref = torch.zeros((2, n_steps, len(systems), ne), dtype=torch.float64, device="cuda")
    q0, p0, f0 = qd.clone(), pd.clone(), fd.clone()
    for c in range(2):
        b.step(n_steps, qd, pd, fd, el_ref[c])
    lens = [len(r) for r in rows]
    offs = np.concatenate([[0], np.cumsum(lens)])
    # separate allocations: each system's rows in its own tensor
    qs = [q0[offs[k]:offs[k + 1]].clone() for k in range(len(systems))]
    ps = [p0[offs[k]:offs[k + 1]].clone() for k in range(len(systems))]
    fs = [f0[offs[k]:offs[k + 1]].clone() for k in range(len(systems))]
    el = torch.zeros_like(el_ref)
    for c in range(2):
        b.batch_step(n_steps, qs, ps, fs, el[c])
    assert torch.equal(torch.cat(qs), qd) and torch.equal(torch.cat(ps), pd)
    assert torch.equal(torch.cat(fs), fd) and torch.equal(el, el_ref)
    # views into one allocation: the direct path
    qv, pv, fv = q0.clone(), p0.clone(), f0.clone()
    el2 = torch.zeros_like(el_ref)
    for c in range(2):
        b.batch_step(n_steps, [qv[offs[k]:offs[k + 1]] for k in range(len(systems))],
                     [pv[offs[k]:offs[k + 1]] for k in range(len(systems))],
                     [fv[offs[k]:offs[k + 1]] for k in range(len(systems))], el2[c])
    assert torch.equal(qv, qd) and torch.equal(pv, pd) and torch.equal(fv, fd)
    assert torch.equal(el2, el_ref)


def test_batch_step_rejects_bad_arguments(mp):
    """mixpi_batch_step: null pointer arrays, a null entry and a negative
    step count are errors; zero steps do nothing; the state is untouched."""
    import ctypes as C
    import torch
    systems = mixed_batch()[:2]
    b = mp.System(systems)
    q, rows = pack(systems, [s.q for s in systems])
    qs = [dev(q[r]) for r in rows]
    ps = [torch.zeros_like(x) for x in qs]
    fs = [torch.zeros_like(x) for x in qs]
    lib = mp.load()
    arr = [(C.c_void_p * 2)(*[x.data_ptr() for x in xs]) for xs in (qs, ps, fs)]
    before = [host(x).copy() for x in qs]
    assert lib.mixpi_batch_step(b.h, 1, None, arr[1], arr[2], None, None) == mp.MIXPI_E_INVALID
    bad = (C.c_void_p * 2)(qs[0].data_ptr(), None)
    assert lib.mixpi_batch_step(b.h, 1, bad, arr[1], arr[2], None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_batch_step(b.h, -1, arr[0], arr[1], arr[2], None, None) == mp.MIXPI_E_INVALID
    assert lib.mixpi_batch_step(b.h, 0, arr[0], arr[1], arr[2], None, None) == mp.MIXPI_OK
    torch.cuda.synchronize()
    for x, bx in zip(qs, before):
        assert np.array_equal(host(x), bx)

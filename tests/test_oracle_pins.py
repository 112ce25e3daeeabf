"""Pins of the FP64 CPU oracle against the paper and against mathematics.

Each test checks the oracle against something other than itself: values the
paper prints (fixtures under tests/golden/), closed forms, library routines
(numpy FFT, scipy expm / eigvalsh, scipy.constants), brute force over global
slices, finite differences and invariants.
"""
import math
import os

import numpy as np
import pytest
import scipy.constants as sc
import scipy.linalg as sla

import oracle
import synth
from tests._systems import custom, lj_table

POW2 = [1, 2, 4, 8, 16, 32]


# ---------------------------------------------------------------- slice map

def _nested_pairs(ni, nj):
    """Paper's 2-body index sets of Eq. (mts-hamiltonian), 1-based."""
    out = []
    for a in range(1, nj + 1):
        for g in range(1, ni // nj + 1):
            out.append(((a - 1) * (ni // nj) + g, a))
    return sorted(out)


def _nested_triples(ni, nj, nk):
    """Paper's 3-body index sets of Eq. (mts-hamiltonian), 1-based."""
    out = []
    for a in range(1, nk + 1):
        for lam in range(1, nj // nk + 1):
            for g in range(1, ni // nj + 1):
                bj = (a - 1) * (nj // nk) + lam
                bi = ((a - 1) * (nj // nk) + lam - 1) * (ni // nj) + g
                out.append((bi, bj, a))
    return sorted(out)


def test_slice_map_matches_paper_example(golden_dir):
    """Fig. 1(b)-(d) discussion: exact bead pairs for N_1=4 vs N_2=4,1,2."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "fig1_bead_pairs.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        n1, n2 = int(row[1]), int(row[2])
        want = sorted(tuple(int(x) for x in p.split("-")) for p in row[3:])
        got = sorted((oracle.slice_bead(s, n1, n1) + 1, oracle.slice_bead(s, n2, n1) + 1)
                     for s in range(max(n1, n2)))
        assert got == want, row[0]


@pytest.mark.parametrize("ni", POW2)
def test_slice_map_equals_nested_indices_two_body(ni):
    for nj in [n for n in POW2 if n <= ni]:
        got = sorted((oracle.slice_bead(s, ni, ni) + 1, oracle.slice_bead(s, nj, ni) + 1)
                     for s in range(ni))
        assert got == _nested_pairs(ni, nj)


def test_slice_map_equals_nested_indices_three_body():
    for ni in POW2:
        for nj in [n for n in POW2 if n <= ni]:
            for nk in [n for n in POW2 if n <= nj]:
                got = sorted(tuple(oracle.slice_bead(s, n, ni) + 1 for n in (ni, nj, nk))
                             for s in range(ni))
                assert got == _nested_triples(ni, nj, nk), (ni, nj, nk)


def test_bead_totals_tables(golden_dir):
    """Table 1 and Table 2 'Particles' columns from the generated systems."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "table_bead_totals.txt"))
            if l.strip() and not l.startswith("#")]
    for kind, nw, nh, no, ne, total in rows:
        nw, nh, no, ne, total = map(int, (nw, nh, no, ne, total))
        assert synth.water_bead_total(nw, nh, no) + ne + (1 if ne else 0) == total
    # the generated 90-water box at (32,4) has that many beads
    s = synth.water_box(90, 14.0, 32, 4, seed=3)
    assert s.total_beads == 6120


# ---------------------------------------------------------------- constants

def test_constants_against_codata():
    c = oracle.constants()
    amu_a2_fs2 = sc.atomic_mass * 1e-20 / 1e-30
    assert c["kcal"] == pytest.approx(4184.0 / sc.N_A / amu_a2_fs2, rel=1e-12)
    assert c["hbar"] == pytest.approx(sc.hbar / (sc.atomic_mass * 1e-20 / 1e-15), rel=1e-9)
    assert c["kb"] == pytest.approx(sc.k / amu_a2_fs2, rel=1e-9)
    ke = sc.e ** 2 / (4 * math.pi * sc.epsilon_0) * sc.N_A / 4184.0 * 1e10
    assert c["ke"] == pytest.approx(ke, rel=1e-8)


# ---------------------------------------------------------------- pair terms

def test_lj_zero_crossing_and_minimum():
    eps, sig = lj_table(0, 0, 0.3, 2.0)
    for r, v_want, f_want in [(2.0, 0.0, None), (2.0 * 2 ** (1 / 6), -0.3, 0.0)]:
        s = custom([1, 1], [[0, 0, 0], [r, 0, 0]], lj_type=[0, 0], eps=eps, sig=sig)
        F, e = oracle.OracleSystem(s).forces(s.q)
        assert e[1] == pytest.approx(v_want, abs=1e-12)
        if f_want is not None:
            assert abs(F).max() < 1e-12


def test_coulomb_form_and_constant():
    s = custom([1, 1], [[0, 0, 0], [0, 3.0, 0]], charge=[0.5, -0.7])
    F, e = oracle.OracleSystem(s).forces(s.q)
    ke = sc.e ** 2 / (4 * math.pi * sc.epsilon_0) * sc.N_A / 4184.0 * 1e10
    assert e[2] == pytest.approx(ke * 0.5 * -0.7 / 3.0, rel=1e-8)
    # attraction pulls particle 0 toward +y
    assert F[0, 1] == pytest.approx(-ke * 0.5 * -0.7 / 9.0, rel=1e-8)
    assert np.allclose(F[0], -F[1])


def test_pseudopotential_at_zero_separation_and_limit():
    ke = sc.e ** 2 / (4 * math.pi * sc.epsilon_0) * sc.N_A / 4184.0 * 1e10
    s = custom([1, 1], [[1, 1, 1], [1, 1, 1]], charge=[-1.0, 3.0], ele=[1, 0],
               pp_q=-1.0, pp_a=0.5)
    F, e = oracle.OracleSystem(s).forces(s.q)
    assert e[3] == pytest.approx(ke * -3.0 / 0.5, rel=1e-8)
    assert abs(F).max() < 1e-12
    # far from the core the softened form approaches Coulomb
    s = custom([1, 1], [[0, 0, 0], [400.0, 0, 0]], charge=[-1.0, 3.0], ele=[1, 0],
               pp_a=0.5)
    _, e = oracle.OracleSystem(s).forces(s.q)
    assert e[3] == pytest.approx(ke * -3.0 / 400.0, rel=1e-5)


def test_shifted_force_vanishes_at_cutoff():
    eps, sig = lj_table(0, 0, 0.3, 2.0)
    rc = 5.0
    for kw in (dict(lj_type=[0, 0], eps=eps, sig=sig), dict(charge=[1.0, -1.0]),
               dict(charge=[-1.0, 1.0], ele=[1, 0])):
        s = custom([1, 1], [[0, 0, 0], [rc * (1 - 1e-9), 0, 0]], rc=rc, box=100.0, **kw)
        F, e = oracle.OracleSystem(s).forces(s.q)
        assert abs(e[0]) < 1e-9 and abs(F).max() < 1e-6
        s = custom([1, 1], [[0, 0, 0], [rc * (1 + 1e-9), 0, 0]], rc=rc, box=100.0, **kw)
        F, e = oracle.OracleSystem(s).forces(s.q)
        assert e[0] == 0.0 and abs(F).max() == 0.0


def test_nearest_image_and_exclusion():
    box = 10.0
    a = custom([1, 1], [[0.5, 2, 2], [9.0, 2, 2]], charge=[1, -1], box=box, rc=4.0)
    b = custom([1, 1], [[0.5, 2, 2], [-1.0, 2, 2]], charge=[1, -1], box=box, rc=4.0)
    Fa, ea = oracle.OracleSystem(a).forces(a.q)
    Fb, eb = oracle.OracleSystem(b).forces(b.q)
    assert ea[2] == pytest.approx(eb[2], rel=1e-14) and ea[2] != 0.0
    assert np.allclose(Fa, Fb, rtol=1e-14)
    c = custom([1, 1], [[0.5, 2, 2], [1.5, 2, 2]], charge=[1, -1], mol=[7, 7], box=box, rc=4.0)
    Fc, ec = oracle.OracleSystem(c).forces(c.q)
    assert ec[2] == 0.0 and abs(Fc).max() == 0.0


def test_bond_and_angle_closed_forms():
    s = custom([1, 1], [[0, 0, 0], [1.13, 0, 0]], bonds=[(0, 1)], bond_k=400.0,
               bond_r0=1.0, mol=[1, 1])
    F, e = oracle.OracleSystem(s).forces(s.q)
    assert e[4] == pytest.approx(0.5 * 400.0 * 0.13 ** 2, rel=1e-12)
    assert F[0, 0] == pytest.approx(400.0 * 0.13, rel=1e-12)
    t0 = math.radians(105.0)
    s = custom([1, 1, 1], [[1, 0, 0], [0, 0, 0], [0, 2, 0]], angles=[(0, 1, 2)],
               angle_k=60.0, angle_t0=t0, mol=[1, 1, 1])
    F, e = oracle.OracleSystem(s).forces(s.q)
    assert e[5] == pytest.approx(0.5 * 60.0 * (math.pi / 2 - t0) ** 2, rel=1e-12)
    assert np.abs(F.sum(axis=0)).max() < 1e-12


# ---------------------------------------------------------------- V_mix

@pytest.mark.parametrize("seed", range(8))
def test_o2_equals_global_slice_brute_force(seed):
    """Per-term N_max evaluation == average over N_G global slices."""
    s = synth.tiny_random(seed)
    o = oracle.OracleSystem(s)
    F2, e2 = o.forces(s.q, "o2")
    F1, e1 = o.forces(s.q, "o1")
    scale = np.abs(F1).max()
    assert np.abs(F2 - F1).max() <= 1e-12 * scale
    assert np.abs(e2 - e1).max() <= 1e-12 * np.abs(e1).sum()


@pytest.mark.parametrize("seed", range(4))
def test_forces_are_minus_gradient(seed):
    s = synth.tiny_random(seed)
    o = oracle.OracleSystem(s)
    F, _ = o.forces(s.q)
    h = 1e-5
    fd = np.zeros_like(F)
    for b in range(s.q.shape[0]):
        for c in range(3):
            qp = s.q.copy(); qp[b, c] += h
            qm = s.q.copy(); qm[b, c] -= h
            fd[b, c] = -(o.forces(qp)[1][0] - o.forces(qm)[1][0]) / (2 * h)
    assert np.abs(fd - F).max() <= 1e-6 * max(1.0, np.abs(F).max())


@pytest.mark.parametrize("seed", range(4))
def test_newton3_and_translation(seed):
    s = synth.tiny_random(seed)
    o = oracle.OracleSystem(s)
    F, e = o.forces(s.q)
    assert np.abs(F.sum(axis=0)).max() <= 1e-11 * np.abs(F).max()
    F2, e2 = o.forces(s.q + np.array([0.37, -1.21, 2.9]))
    assert np.abs(e2 - e).max() <= 1e-11 * np.abs(e).sum()


@pytest.mark.parametrize("seed", range(4))
def test_collapsed_rings_reduce_to_classical(seed):
    """Coincident beads: V_mix = V_classical, sum of bead forces = classical."""
    s = synth.tiny_random(seed)
    off = s.bead_offset
    X = np.array([s.q[off[i]:off[i + 1]].mean(axis=0) for i in range(s.n_particles)])
    s.q = np.repeat(X, s.n_beads, axis=0)
    o = oracle.OracleSystem(s)
    F, e = o.forces(s.q)
    Fc, ec = o.classical(X)
    assert np.abs(e - ec).max() <= 1e-12 * np.abs(ec).sum()
    Fs = np.array([F[off[i]:off[i + 1]].sum(axis=0) for i in range(s.n_particles)])
    assert np.abs(Fs - Fc).max() <= 1e-12 * np.abs(Fc).max()


def test_equal_bead_counts_reduce_to_standard_pimd():
    """All N_i = N: V_mix = (1/N) sum_a V(q_a), each bead force = F_cl/N."""
    s = synth.tiny_random(5, bead_choices=(4,))
    o = oracle.OracleSystem(s)
    F, e = o.forces(s.q)
    N = 4
    ecl = np.zeros(6)
    for a in range(N):
        X = s.q[a::N]
        Fa, ea = o.classical(X)
        ecl += ea / N
        assert np.abs(F[a::N] - Fa / N).max() <= 1e-12 * np.abs(Fa).max()
    # the constant background counts once, not once per bead
    assert np.abs(e - ecl).max() <= 1e-12 * np.abs(ecl).sum()


def test_block_shift_invariance():
    s = synth.tiny_random(11, bead_choices=(2, 4, 8))
    o = oracle.OracleSystem(s)
    F, e = o.forces(s.q)
    nmin = int(s.n_beads.min())
    off = s.bead_offset
    q2 = s.q.copy()
    perm = np.arange(s.total_beads)
    for i, n in enumerate(s.n_beads):
        sh = n // nmin
        idx = off[i] + (np.arange(n) + sh) % n
        q2[off[i]:off[i + 1]] = s.q[idx]
        perm[off[i]:off[i + 1]] = idx
    F2, e2 = o.forces(q2)
    assert np.abs(e2 - e).max() <= 1e-12 * np.abs(e).sum()
    assert np.abs(F2 - F[perm]).max() <= 1e-12 * np.abs(F).max()


# ---------------------------------------------------------------- theta

@pytest.mark.parametrize("seed", range(3))
def test_theta_gradient_euler_and_fd(seed):
    s = synth.solvated_electron(6, 8, 8.0, seed=seed, rc_pp=3.9, rc_aa=3.9,
                                n_h=4, n_o=2, ion_excl=3.4)
    th0 = np.array([s.pp_q, s.pp_a, s.lj_eps[0, 0], s.lj_sigma[0, 0],
                    s.bond_k[0], s.angle_k[0]])
    o = oracle.OracleSystem(s, theta=th0)
    g = o.dvdtheta(s.q)
    _, e = o.forces(s.q)
    # V_pp, V_bond, V_angle are linear in q_e, k_b, k_theta
    assert th0[0] * g[0] == pytest.approx(e[3], rel=1e-12)
    assert th0[4] * g[4] == pytest.approx(e[4], rel=1e-12)
    assert th0[5] * g[5] == pytest.approx(e[5], rel=1e-12)
    for k in range(6):
        h = 1e-6 * abs(th0[k])
        tp = th0.copy(); tp[k] += h
        tm = th0.copy(); tm[k] -= h
        ep = oracle.OracleSystem(s, theta=tp).forces(s.q)[1][0]
        em = oracle.OracleSystem(s, theta=tm).forces(s.q)[1][0]
        fd = (ep - em) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_theta_gradient_water_only():
    s = synth.water_box(8, 7.0, 4, 2, seed=1, rc=3.4)
    o = oracle.OracleSystem(s)
    g = o.dvdtheta(s.q)
    _, e = o.forces(s.q)
    assert g[0] == 0.0 and g[1] == 0.0
    assert s.lj_eps[0, 0] * g[2] == pytest.approx(e[1], rel=1e-12)


# ---------------------------------------------------------------- ring polymer

def _cyclic_laplacian(N):
    D = np.eye(N) - np.roll(np.eye(N), 1, axis=1)   # (D q)_a = q_a - q_{a+1}
    return D.T @ D


@pytest.mark.parametrize("N", [1, 2, 4, 8, 64, 256])
def test_nm_basis_orthonormal_and_diagonalises_springs(N):
    Cm = oracle.nm_basis(N)
    assert np.abs(Cm.T @ Cm - np.eye(N)).max() < 1e-13
    L = _cyclic_laplacian(N)
    lam = np.array([oracle.nm_lambda(N, k) for k in range(N)])
    assert np.abs(Cm.T @ L @ Cm - np.diag(lam)).max() < 1e-12
    assert np.allclose(np.sort(lam), np.linalg.eigvalsh(L), atol=1e-12)


@pytest.mark.parametrize("N", [2, 4, 16, 128, 4096])
def test_nm_basis_against_fft(N):
    rng = np.random.default_rng(N)
    x = rng.normal(size=N)
    xi = oracle.nm_basis(N).T @ x
    f = np.fft.fft(x)
    want = np.empty(N)
    want[0] = f[0].real / math.sqrt(N)
    for k in range(1, N):
        if 2 * k < N:
            want[k] = math.sqrt(2.0 / N) * f[k].real
        elif 2 * k == N:
            want[k] = f[k].real / math.sqrt(N)
        else:
            want[k] = -math.sqrt(2.0 / N) * f[k].imag
    assert np.abs(xi - want).max() < 1e-13 * max(1.0, np.abs(want).max())


def _beta_hbar(T):
    return sc.hbar / (sc.k * T) * 1e15   # fs


def test_mode_frequencies_closed_form():
    """m_f = m/N gives omega_k = 2 (N / beta hbar) sin(k pi / N)."""
    for N in (4, 32, 1024):
        s = custom([N], np.zeros((N, 3)), mass=[1.00794], temperature=300.0)
        o = oracle.OracleSystem(s)
        wp = N / _beta_hbar(300.0)
        for k in (0, 1, N // 3, N // 2, N - 1):
            assert o.omega(0, k) == pytest.approx(2 * wp * math.sin(k * math.pi / N),
                                                  rel=1e-9, abs=1e-15)


def test_free_propagation_equals_matrix_exponential():
    """Exact NM propagation == expm of the bead-space linear flow."""
    N, m = 8, 2.0
    rng = np.random.default_rng(0)
    q = rng.normal(scale=0.2, size=(N, 3))
    p = rng.normal(scale=0.05, size=(N, 3))
    s = custom([N], q, mass=[m], fict_mass=[m / N * 3.0], p=p)
    o = oracle.OracleSystem(s)
    t = 2.7
    q1, p1 = o.free_propagate(q, p, t)
    bh = _beta_hbar(300.0)
    ksp = N * m / bh ** 2
    mf = m / N * 3.0
    A = np.zeros((2 * N, 2 * N))
    A[:N, N:] = np.eye(N) / mf
    A[N:, :N] = -ksp * _cyclic_laplacian(N)
    U = sla.expm(A * t)
    for c in range(3):
        z = U @ np.concatenate([q[:, c], p[:, c]])
        assert np.abs(z[:N] - q1[:, c]).max() < 1e-10
        assert np.abs(z[N:] - p1[:, c]).max() < 1e-10


def test_free_propagation_reversible_and_conservative():
    s = synth.tiny_random(2, bead_choices=(1, 4, 16))
    o = oracle.OracleSystem(s)
    q1, p1 = o.free_propagate(s.q, s.p, 5.0)
    q2, p2 = o.free_propagate(q1, -p1, 5.0)
    assert np.abs(q2 - s.q).max() < 1e-12 and np.abs(-p2 - s.p).max() < 1e-12
    kcal = oracle.constants()["kcal"]

    def energy(q, p):
        ke = sum((p[s.bead_offset[i]:s.bead_offset[i + 1]] ** 2).sum() / (2 * s.fict_mass[i])
                 for i in range(s.n_particles)) / kcal
        return ke + o.springs(q)[0]
    assert energy(q1, p1) == pytest.approx(energy(s.q, s.p), rel=1e-12)


def test_springs_gradient():
    s = synth.tiny_random(3, bead_choices=(1, 2, 4, 8))
    o = oracle.OracleSystem(s)
    e, F = o.springs(s.q)
    h = 1e-6
    for b in range(0, s.total_beads, 3):
        for c in range(3):
            qp = s.q.copy(); qp[b, c] += h
            qm = s.q.copy(); qm[b, c] -= h
            fd = -(o.springs(qp)[0] - o.springs(qm)[0]) / (2 * h)
            assert fd == pytest.approx(F[b, c], abs=1e-5 * max(1.0, abs(F).max()))


@pytest.mark.parametrize("P,want", [(1, 0.1), (4, (1 + 2 / 1.32 + 1 / 1.64) / 10)])
def test_harmonic_oscillator_x2_finite_p(P, want):
    """<x^2>_P from the oracle's mode frequencies equals the Gaussian
    path-integral covariance (linear algebra), in units hbar/(m omega)."""
    T, m = 300.0, 1.00794
    bh = _beta_hbar(T)
    w = 10.0 / bh                 # beta hbar omega = 10
    s = custom([P], np.zeros((P, 3)), mass=[m], temperature=T)
    o = oracle.OracleSystem(s)
    beta = o.beta
    x2_modes = sum(1.0 / (beta * m * (w * w + o.omega(0, k) ** 2)) for k in range(P))
    ksp = P * m / bh ** 2
    A = (m * w * w / P) * np.eye(P) + ksp * _cyclic_laplacian(P)
    x2_lin = np.trace(np.linalg.inv(beta * A)) / P
    assert x2_modes == pytest.approx(x2_lin, rel=1e-12)
    unit = oracle.constants()["hbar"] / (m * w)
    assert x2_modes / unit == pytest.approx(want, rel=1e-9)


def test_harmonic_oscillator_x2_converges_to_quantum():
    T, m = 300.0, 1.00794
    bh = _beta_hbar(T)
    w = 10.0 / bh
    P = 4096
    s = custom([P], np.zeros((P, 3)), mass=[m], temperature=T)
    o = oracle.OracleSystem(s)
    x2 = sum(1.0 / (o.beta * m * (w * w + o.omega(0, k) ** 2)) for k in range(P))
    unit = oracle.constants()["hbar"] / (m * w)
    assert x2 / unit == pytest.approx(0.5 / math.tanh(5.0), rel=2e-5)


# ---------------------------------------------------------------- integrator

def test_step_without_interactions_is_free_propagation():
    s = synth.tiny_random(4, bead_choices=(1, 2, 8))
    s.charge[:] = 0.0
    s.lj_eps[:] = 0.0
    s.bonds = np.zeros((0, 2), np.int32)
    s.angles = np.zeros((0, 3), np.int32)
    s.background = False
    o = oracle.OracleSystem(s)
    q, p, F, _ = o.step(s.q, s.p, 3)
    qf, pf = o.free_propagate(s.q, s.p, 3 * s.dt)
    assert np.abs(q - qf).max() < 1e-12 and np.abs(p - pf).max() < 1e-12


def _nve_fluct(dt, nsteps):
    s = synth.water_box(8, 7.0, 4, 2, seed=2, rc=3.4, dt=dt)
    o = oracle.OracleSystem(s)
    _, p, _, elog = o.step(s.q, s.p, nsteps)
    h = elog[:, oracle.E_NAMES.index("ham")]
    return h.std(), abs(h[-1] - h[0]), p.sum(axis=0)


def test_nve_energy_error_scales_as_dt_squared():
    s1, _, ptot = _nve_fluct(0.2, 400)
    s2, _, _ = _nve_fluct(0.1, 800)
    ratio = s1 / s2
    assert 3.0 < ratio < 5.5, ratio
    assert np.abs(ptot).max() < 1e-9


def test_observables_classical_limits():
    s = synth.tiny_random(6, bead_choices=(1,))
    o = oracle.OracleSystem(s)
    F, v = o.forces(s.q)
    e = o.observables(s.q, s.p, F, v)
    kT = oracle.constants()["kb_kcal"] * s.temperature
    n = s.n_particles
    assert e[oracle.E_NAMES.index("spring")] == 0.0
    assert e[oracle.E_NAMES.index("kcv")] == pytest.approx(1.5 * n * kT, rel=1e-14)
    assert e[oracle.E_NAMES.index("kprim")] == pytest.approx(1.5 * n * kT, rel=1e-14)
    kcal = oracle.constants()["kcal"]
    ke = sum((s.p[i] ** 2).sum() / (2 * s.fict_mass[i]) for i in range(n)) / kcal
    assert e[oracle.E_NAMES.index("kin")] == pytest.approx(ke, rel=1e-13)


def _ke_quantum_finite_p(N, w, bh, kT):
    """Exact kinetic energy (kcal/mol, three Cartesian components) of an
    N-bead ring in an isotropic harmonic well of frequency w, under the
    discretised path-integral distribution: (3 kT / 2) [1 + sum_{k>=1}
    w^2 / (w^2 + w_k^2)], w_k = 2 (N / beta hbar) sin(pi k / N).  It tends
    to (3 hbar w / 4) coth(beta hbar w / 2) as N grows."""
    wk = 2.0 * (N / bh) * np.sin(np.pi * np.arange(1, N) / N)
    return 1.5 * kT * (1.0 + np.sum(w * w / (w * w + wk * wk)))


def test_kinetic_estimators_exact_expectation_harmonic_rings():
    """Kinetic-energy estimators of Sec. Output and Analysis at N > 1:
    rings of 16, 4 and 1 beads, each in its own harmonic well, one 1-body
    term per particle in Eq. (mts-hamiltonian) (slice weight 1/N_i, bead
    force -m w^2 (q - c) / N_i).  The ring distribution is Gaussian with
    the covariance of the springs of Eq. (mts-hamiltonian-b) plus the well
    (linear algebra); both estimators are quadratic in q, so their mean
    over the distribution is exactly the sigma-point average (+/- sqrt(D)
    times the columns of a Cholesky factor).  Both means must equal the
    exact finite-N kinetic energy; a flipped virial sign, q instead of
    q - q_bar, or 3 instead of 3 N_i in the primitive estimator fails."""
    T = 300.0
    Ns = [16, 4, 1]
    masses = [1.00794, 15.9994, 58.9332]
    bh = _beta_hbar(T)
    ws = [3.0 / bh, 7.0 / bh, 1.5 / bh]              # beta hbar omega = 3, 7, 1.5
    centres = np.array([[1.0, -2.0, 0.5], [4.0, 3.0, -1.0], [-3.0, 0.0, 2.0]])
    B = sum(Ns)
    s = custom(Ns, np.zeros((B, 3)), mass=masses, temperature=T)
    o = oracle.OracleSystem(s)
    kcal = oracle.constants()["kcal"]
    kT = oracle.constants()["kb_kcal"] * T
    beta = 1.0 / (sc.k * T / (sc.atomic_mass * 1e-20 / 1e-30))   # 1 / (amu A^2 fs^-2)
    # covariance of one Cartesian component of every bead (block per particle)
    cov = np.zeros((B, B))
    off = np.concatenate([[0], np.cumsum(Ns)])
    for i, (N, m, w) in enumerate(zip(Ns, masses, ws)):
        A = (m * w * w / N) * np.eye(N) + (N * m / bh ** 2) * _cyclic_laplacian(N)
        cov[off[i]:off[i + 1], off[i]:off[i + 1]] = np.linalg.inv(beta * A)
    Lc = np.linalg.cholesky(cov)
    centre_rows = np.repeat(centres, Ns, axis=0)
    well = np.repeat([m * w * w / N / kcal for N, m, w in zip(Ns, masses, ws)], Ns)[:, None]
    D = 3 * B
    acc = {"kcv": 0.0, "kprim": 0.0}
    p0 = np.zeros((B, 3))
    for c in range(3):                      # sigma points along each Cartesian block
        for col in range(B):
            for sign in (1.0, -1.0):
                q = centre_rows.copy()
                q[:, c] += sign * math.sqrt(D) * Lc[:, col]
                F = -well * (q - centre_rows)
                e = o.observables(q, p0, F, np.zeros(oracle.N_POT))
                for k in acc:
                    acc[k] += e[oracle.E_NAMES.index(k)] / (2 * D)
    want = sum(_ke_quantum_finite_p(N, w, bh, kT) for N, w in zip(Ns, ws))
    assert acc["kcv"] == pytest.approx(want, rel=1e-11)
    assert acc["kprim"] == pytest.approx(want, rel=1e-11)
    # the closed form itself: N = 1 is classical, large N reaches the quantum value
    assert _ke_quantum_finite_p(1, ws[0], bh, kT) == pytest.approx(1.5 * kT, rel=1e-15)
    qv = 0.75 * kT * 3.0 / math.tanh(1.5)          # 3 hbar w / 4 coth(beta hbar w / 2)
    assert _ke_quantum_finite_p(4096, ws[0], bh, kT) == pytest.approx(qv, rel=1e-5)


# ---------------------------------------------------------------- thermostat
# The path-integral Langevin thermostat (PILE) of the paper's NVT runs:
# an Ornstein-Uhlenbeck step of the momenta in each ring's normal modes.

def _free_rings(n, P, T=300.0, mass=1.00794, seed=0):
    rng = np.random.default_rng(seed)
    q = rng.normal(scale=0.2, size=(n * P, 3))
    return custom([P] * n, q, mass=[mass] * n, temperature=T, dt=1.0)


def test_pile_centroid_is_a_textbook_langevin_step():
    """One-bead particles: with zero noise the momentum decays as
    exp(-t/tau0) (the exact Ornstein-Uhlenbeck mean); gamma_0 = 0 for an
    infinite tau0 leaves it unchanged."""
    s = _free_rings(5, 1)
    o = oracle.OracleSystem(s)
    p = np.random.default_rng(1).normal(size=(5, 3))
    zero = np.zeros_like(p)
    out = o.pile(p, zero, 3.0, 20.0)
    assert np.allclose(out, p * math.exp(-3.0 / 20.0), rtol=1e-14, atol=0)
    assert np.array_equal(o.pile(p, zero, 3.0, math.inf), p)


def test_pile_internal_modes_decay_and_compose():
    """Zero noise: mode k of a ring decays by exp(-2 omega_k t) (critical
    damping of the free-ring mode), and two steps compose into one."""
    P = 8
    s = _free_rings(1, P)
    o = oracle.OracleSystem(s)
    p = np.random.default_rng(2).normal(size=(P, 3))
    zero = np.zeros_like(p)
    a = o.pile(o.pile(p, zero, 0.7, 15.0), zero, 1.3, 15.0)
    b = o.pile(p, zero, 2.0, 15.0)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(p).max()
    C = oracle.nm_basis(P)
    modes_before, modes_after = C.T @ p, C.T @ b
    for k in range(1, P):
        w = o.omega(0, k)
        assert w == pytest.approx(2.0 * (P / _beta_hbar(300.0)) * math.sin(math.pi * k / P), rel=1e-12)
        assert np.allclose(modes_after[k], modes_before[k] * math.exp(-2.0 * w * 2.0), rtol=1e-10,
                           atol=1e-14)
    assert np.allclose(modes_after[0], modes_before[0] * math.exp(-2.0 / 15.0), rtol=1e-12)


def test_pile_keeps_maxwell_boltzmann_invariant():
    """Momenta drawn from N(0, m_f kT) stay so distributed after a step with
    fresh noise: per-component variance m_f kT, no correlation between
    neighbouring beads (4-sigma bounds over 24,000 samples)."""
    n, P = 1000, 8
    s = _free_rings(n, P)
    o = oracle.OracleSystem(s)
    kT = oracle.constants()["kb"] * 300.0
    mf = s.fict_mass[0]
    rng = np.random.default_rng(3)
    p = rng.normal(scale=math.sqrt(mf * kT), size=(n * P, 3))
    eta = rng.normal(size=p.shape)
    out = o.pile(p, eta, 4.0, 10.0) / math.sqrt(mf * kT)
    var = (out ** 2).mean()
    assert abs(var - 1.0) < 4.0 * math.sqrt(2.0 / out.size)
    r = out.reshape(n, P, 3)
    cov = (r * np.roll(r, 1, axis=1)).mean()
    assert abs(cov) < 4.0 / math.sqrt(out.size)


def test_pile_samples_the_quantum_harmonic_dimer():
    """A harmonic bond k/2 |r1 - r2|^2 between two particles of P = 4 beads:
    the bead-averaged <|r1 - r2|^2> sampled by the thermostatted steps
    matches the exact finite-P value 3/(beta mu) sum_k 1/(omega^2 +
    omega_k^2) of the relative coordinate (reduced mass mu) within 4
    standard errors (block averages).  The logged kinetic-energy estimators
    (centroid virial and primitive) sample the exact finite-P kinetic energy
    of the pair, 3 kT/2 [2 + sum_{k>=1} omega^2 / (omega^2 + omega_k^2)]
    (a free centre-of-mass ring plus the relative oscillator), within 4
    standard errors."""
    P, T, m = 4, 300.0, 1.00794
    mu = m / 2
    bh = _beta_hbar(T)
    w = 4.0 / bh                                     # beta hbar omega = 4
    kcal = oracle.constants()["kcal"]
    kb = mu * w * w / kcal                           # kcal/mol/A^2
    q = np.zeros((2 * P, 3))
    q[P:, 0] = 0.1
    s = custom([P, P], q, mass=[m, m], bonds=[(0, 1)], bond_k=kb, bond_r0=0.0,
               temperature=T, dt=1.0)
    o = oracle.OracleSystem(s)
    beta = o.beta
    wk = [2.0 * (P / bh) * math.sin(math.pi * k / P) for k in range(P)]
    want = 3.0 / (beta * mu) * sum(1.0 / (w * w + x * x) for x in wk)
    rng = np.random.default_rng(11)
    nthreads = oracle.num_threads()
    oracle.set_threads(1)
    try:
        qq, pp = s.q, np.zeros_like(s.q)
        F, _ = o.forces(qq)
        vb, kcv, kpr = [], [], []
        for chunk in range(40):
            noise = rng.normal(size=(5000, 2, 2 * P, 3))
            qq, pp, F, el = o.step_nvt(qq, pp, noise, 50.0, F=F)
            vb.append(el[:, oracle.E_NAMES.index("bond")])
            kcv.append(el[:, oracle.E_NAMES.index("kcv")])
            kpr.append(el[:, oracle.E_NAMES.index("kprim")])
    finally:
        oracle.set_threads(nthreads)
    kT = oracle.constants()["kb_kcal"] * T
    want_ke = 1.5 * kT * (2.0 + sum(w * w / (w * w + x * x) for x in wk[1:]))
    for series in (kcv, kpr):
        kb_blocks = np.concatenate(series[4:]).reshape(72, -1).mean(axis=1)
        km, ke = kb_blocks.mean(), kb_blocks.std(ddof=1) / math.sqrt(len(kb_blocks))
        assert ke < 0.02 * want_ke
        assert abs(km - want_ke) < 4.0 * ke, (km, want_ke, ke)
    # bead-averaged |r1 - r2|^2 = 2 V_bond / k (V_bond carries the 1/P weights)
    x = 2.0 * np.concatenate(vb[4:]) / kb
    blocks = x.reshape(72, -1).mean(axis=1)
    mean, err = blocks.mean(), blocks.std(ddof=1) / math.sqrt(len(blocks))
    assert err < 0.02 * want
    assert abs(mean - want) < 4.0 * err, (mean, want, err)


# ------------------------------------------------- velocity Verlet with springs

def test_vv_equals_split_propagator_without_springs():
    """One bead per particle: no springs, the free motion is a plain drift,
    and both integrators are the same velocity-Verlet step."""
    s = synth.tiny_random(6, bead_choices=(1,))
    o = oracle.OracleSystem(s)
    a = o.step(s.q, s.p, 4)
    b = o.step_vv(s.q, s.p, 4)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-13, atol=1e-13)


def test_vv_converges_to_exact_free_rings_as_dt_squared():
    """Free rings: velocity Verlet approaches the exact normal-mode motion
    with an error that falls by about 4 when dt halves."""
    def err(dt, n):
        s = _free_rings(3, 8)
        s.dt = dt
        rng = np.random.default_rng(4)
        s.p = rng.normal(scale=0.02, size=s.q.shape)
        o = oracle.OracleSystem(s)
        q, p, _, _ = o.step_vv(s.q, s.p, n)
        qe, pe = o.free_propagate(s.q, s.p, dt * n)
        return np.abs(q - qe).max()
    e1, e2 = err(0.4, 10), err(0.2, 20)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def test_vv_conserves_energy_as_dt_squared():
    s1 = synth.water_box(8, 7.0, 4, 2, seed=2, rc=3.4, dt=0.05)
    s2 = synth.water_box(8, 7.0, 4, 2, seed=2, rc=3.4, dt=0.025)
    h = []
    for s, n in ((s1, 200), (s2, 400)):
        _, _, _, el = oracle.OracleSystem(s).step_vv(s.q, s.p, n)
        h.append(el[:, oracle.E_NAMES.index("ham")].std())
    assert 3.0 < h[0] / h[1] < 5.5, h


# --------------------------------------------------- radial distribution

def test_rdf_shell_counts_of_a_simple_cubic_lattice():
    """Particles on a periodic simple cubic lattice of 4^3 sites (M sites,
    spacing a, box 4a): by nearest image the unordered pair counts at a,
    sqrt(2) a, sqrt(3) a and 2 a are 3M, 6M, 4M and 3M/2 (the site two steps
    along an axis is the same one both ways); rings collapsed on their sites
    count each pair once (weights 1/N_max over N_max slices)."""
    n, a = 4, 2.5
    M = n ** 3
    sites = np.array([(x, y, z) for x in range(n) for y in range(n) for z in range(n)]) * a
    for nb in (1, 4):
        q = np.repeat(sites, nb, axis=0)
        s = custom([nb] * M, q, box=n * a, rc=4.0, lj_type=[0] * M)
        h = oracle.OracleSystem(s).rdf(q, 5.1, 510)[0, 0]
        dr = 5.1 / 510
        def count(r):
            return h[int(r / dr)]
        assert count(a) == 3 * M
        assert count(math.sqrt(2) * a) == 6 * M
        assert count(math.sqrt(3) * a) == 4 * M
        assert count(2 * a) == 3 * M // 2
        assert h.sum() == (3 + 6 + 4) * M + 3 * M // 2


def test_rdf_pair_set_and_weights():
    """A 4-bead particle and a 2-bead particle: 4 slice-pairs of weight 1/4;
    equal molecule ids and two electrons contribute nothing."""
    q = np.array([[0, 0, 0], [0, 0, 0.1], [0, 0, 0.2], [0, 0, 0.3],
                  [1.0, 0, 0], [1.5, 0, 0]], dtype=float)
    s = custom([4, 2], q, lj_type=[0, 1])
    h = oracle.OracleSystem(s).rdf(q, 3.0, 300)
    assert h[0, 1].sum() == pytest.approx(1.0, abs=0) and h[1, 0].sum() == 0
    s_same = custom([4, 2], q, lj_type=[0, 1], mol=[5, 5])
    assert oracle.OracleSystem(s_same).rdf(q, 3.0, 300).sum() == 0
    s_ele = custom([4, 2], q, lj_type=[0, 1], ele=[1, 1])
    assert oracle.OracleSystem(s_ele).rdf(q, 3.0, 300).sum() == 0


# --------------------------------------------------- velocity correlation

def test_centroid_velocity_of_a_ring():
    """Bead momenta m_f (v + u_j) with sum_j u_j = 0 have centroid velocity v."""
    rng = np.random.default_rng(0)
    nb = [8, 1, 4]
    q = rng.normal(size=(13, 3))
    s = custom(nb, q, mass=[4.0, 2.0, 16.0])
    o = oracle.OracleSystem(s)
    v = rng.normal(size=(3, 3))
    p = np.zeros((13, 3))
    for i in range(3):
        u = rng.normal(size=(nb[i], 3))
        u -= u.mean(axis=0)
        p[o.off[i]:o.off[i + 1]] = o.fm[i] * (v[i] + u)
    assert np.allclose(o.centroid_velocity(p), v, rtol=1e-14, atol=1e-15)


def test_vacf_of_constant_and_oscillating_velocities():
    """Constant centroid velocities give (T - tau) sum_i |v_i|^2; velocities
    v0 cos(w t) give |v0|^2 sum_{t=tau}^{T-1} cos(w (t - tau)) cos(w t)
    = |v0|^2 / 2 [(T - tau) cos(w tau) + sin(w (T - tau)) cos(w (T - 1)) / sin(w)],
    the product-to-sum identity with the closed form of a cosine sum."""
    rng = np.random.default_rng(1)
    nb = [4, 2]
    s = custom(nb, rng.normal(size=(6, 3)), lj_type=[0, 2], mass=[3.0, 5.0])
    o = oracle.OracleSystem(s)
    T, L = 12, 5
    v = rng.normal(size=(2, 3))

    def moments(vel):
        p = np.zeros((6, 3))
        for i in range(2):
            p[o.off[i]:o.off[i + 1]] = o.fm[i] * vel[i]
        return p

    acc = o.vacf([moments(v)] * T, L)
    for tau in range(L):
        assert acc[0, tau] == pytest.approx((T - tau) * v[0] @ v[0], rel=1e-13)
        assert acc[2, tau] == pytest.approx((T - tau) * v[1] @ v[1], rel=1e-13)
    assert np.count_nonzero(acc) == 2 * L
    w = 0.7
    acc = o.vacf([moments(v * math.cos(w * t)) for t in range(T)], L)
    for tau in range(L):
        want = 0.5 * ((T - tau) * math.cos(w * tau)
                      + math.sin(w * (T - tau)) * math.cos(w * (T - 1)) / math.sin(w))
        assert acc[0, tau] == pytest.approx(want * (v[0] @ v[0]), rel=1e-12, abs=1e-12)
    # a window longer than the trajectory: lags past T - 1 stay zero
    acc = o.vacf([moments(v)] * 3, 6)
    assert np.all(acc[:, 3:] == 0) and acc[0, 2] == pytest.approx(v[0] @ v[0], rel=1e-13)


# --------------------------------------------------- centroid electrostatics

def _rock_salt(cells: int, a: float, nb: int = 1):
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    pos, chg = [], []
    for x in range(cells):
        for y in range(cells):
            for z in range(cells):
                for b in base:
                    pos.append((np.array([x, y, z]) + b) * a)
                    chg.append(1.0)
                    pos.append((np.array([x, y, z]) + b + [0.5, 0, 0]) * a)
                    chg.append(-1.0)
    pos = np.array(pos)
    n = len(pos)
    return custom([nb] * n, np.repeat(pos, nb, axis=0), charge=chg, box=cells * a, rc=cells * a / 2)


def test_ewald_madelung_constant_of_rock_salt():
    """Rock salt (2 x 2 x 2 conventional cells, 64 ions, nearest-neighbour
    distance r0): E = -(N/2) M k_e / r0 with M = 1.747564594633...; the
    force on every ion vanishes by symmetry; two splitting parameters give
    the same energy.  Collapsed 2-bead rings are their centroids."""
    a = 5.64
    for nb in (1, 2):
        s = _rock_salt(2, a, nb)
        o = oracle.OracleSystem(s)
        ke = oracle.constants()["ke"]
        want = -(64 / 2) * 1.747564594633182 * ke / (a / 2)
        for alpha, kmax in ((1.0, 22), (1.2, 26)):
            F, e = o.ewald(s.q, alpha, a, kmax)
            assert e.sum() == pytest.approx(want, rel=1e-10)
            assert np.abs(F).max() < 1e-9


def test_ewald_dipole_in_a_large_cube():
    """Charges +-1 at distance d in a cube of side L (conducting boundary):
    E = -k_e/d - 2 pi k_e d^2 / (3 L^3) up to O(d^4 / L^5) (the cubic dipole
    lattice has no dipole-dipole field at its sites); the force on the
    positive charge along the bond is -dE/dd = k_e / d^2 - 4 pi k_e d / (3 L^3)."""
    L, d = 30.0, 1.0
    q = np.array([[10.0, 10.0, 10.0], [10.0 + d, 10.0, 10.0]])
    s = custom([1, 1], q, charge=[1.0, -1.0], box=L, rc=L / 2)
    ke = oracle.constants()["ke"]
    F, e = oracle.OracleSystem(s).ewald(q, 0.35, L / 2, 22)
    want = -ke / d - 2 * math.pi * ke * d * d / (3 * L ** 3)
    assert abs(e.sum() - want) < 1e-6 * ke
    assert abs(e.sum() - (-ke / d)) > 50e-6 * ke          # the volume term is resolved
    assert F[0, 0] == pytest.approx(ke / d ** 2 - 4 * math.pi * ke * d / (3 * L ** 3), rel=2e-6)
    assert np.allclose(F[0], -F[1], rtol=0, atol=1e-10)


def test_ewald_is_independent_of_the_splitting():
    """The converged Ewald sum does not depend on alpha; this holds only
    with the self term, the excluded pairs' erf correction and (net charge
    +3 here) the neutralising-background term all correct."""
    s = synth.config_c1()
    o = oracle.OracleSystem(s)
    L = float(s.box[0])
    out = [o.ewald(s.q, al, L / 2, km) for al, km in ((1.1, 24), (1.4, 30))]
    (F1, e1), (F2, e2) = out
    assert e1.sum() == pytest.approx(e2.sum(), rel=1e-9)
    assert abs(e1[2] - e2[2]) > 1.0                        # the parts do move
    rms = np.sqrt((F1 ** 2).sum(axis=1).mean())
    assert np.abs(F1 - F2).max() < 1e-7 * rms


def test_ewald_forces_are_minus_the_gradient():
    """Central differences of the energy in one bead coordinate: the bead
    force is 1/N_i of the centroid force."""
    s = synth.config_c1()
    o = oracle.OracleSystem(s)
    L = float(s.box[0])
    F, _ = o.ewald(s.q, 0.6, L / 2, 10)
    rng = np.random.default_rng(2)
    for b in rng.integers(0, s.q.shape[0], 5):
        for k in range(3):
            qp, qm = s.q.copy(), s.q.copy()
            qp[b, k] += 1e-5
            qm[b, k] -= 1e-5
            fd = -(o.ewald(qp, 0.6, L / 2, 10)[1].sum() - o.ewald(qm, 0.6, L / 2, 10)[1].sum()) / 2e-5
            assert F[b, k] == pytest.approx(fd, rel=1e-5, abs=1e-6)


def test_bspline_partition_of_unity():
    from oracle.oracle import _bspline
    w = np.linspace(0, 1, 17, endpoint=False)
    for n in (4, 6, 8):
        tot = sum(_bspline(n, w + j) for j in range(n))
        assert np.allclose(tot, 1.0, rtol=0, atol=1e-14)
        # M_n is the n-fold convolution of the unit box: M_n(n/2) is the
        # peak, symmetric about it
        assert _bspline(n, n / 2 - 0.3) == pytest.approx(_bspline(n, n / 2 + 0.3), rel=1e-14)
    assert _bspline(4, 2.0) == pytest.approx(2.0 / 3.0, rel=1e-15)
    assert _bspline(4, 1.0) == pytest.approx(1.0 / 6.0, rel=1e-15)


def test_spme_converges_to_the_ewald_reciprocal_sum():
    """SPME's reciprocal energy and forces approach the direct sum as the
    grid and the spline order grow; its forces are minus the gradient of
    its own energy."""
    s = synth.config_c1()
    o = oracle.OracleSystem(s)
    L = float(s.box[0])
    al = 0.45
    Fd, ed = o.ewald(s.q, al, L / 2, 16)
    Fr, _ = o.ewald(s.q, al, L / 2, -1)
    Fk = Fd - Fr
    rms = np.sqrt((Fk ** 2).sum(axis=1).mean())
    errs = []
    for K, n in ((16, 4), (32, 6), (64, 8)):
        F, E = o.spme_recip(s.q, al, K, n)
        errs.append((abs(E - ed[1]) / abs(ed[1]), np.abs(F - Fk).max() / rms))
    assert errs[0][0] > errs[1][0] > errs[2][0] and errs[2][0] < 1e-8
    assert errs[0][1] > errs[1][1] > errs[2][1] and errs[2][1] < 1e-6
    F, E = o.spme_recip(s.q, al, 16, 4)
    b = 7
    for k in range(3):
        qp, qm = s.q.copy(), s.q.copy()
        qp[b, k] += 1e-5
        qm[b, k] -= 1e-5
        fd = -(o.spme_recip(qp, al, 16, 4)[1] - o.spme_recip(qm, al, 16, 4)[1]) / 2e-5
        assert F[b, k] == pytest.approx(fd, rel=1e-5, abs=1e-6)


def test_step_extra_with_zero_term_equals_the_c_steps():
    """The Python composition used for steps with an extra (centroid Ewald)
    term reproduces orc_step, orc_step_vv and orc_step_nvt exactly in
    structure: with a zero extra term, trajectories and logs agree to
    rounding."""
    s = synth.tiny_random(3, n_particles=12, box=9.0, bead_choices=(1, 2, 4, 8))
    o = oracle.OracleSystem(s)

    def zero(q):
        return np.zeros_like(q), 0.0

    noise = np.random.default_rng(4).normal(size=(3, 2, o.B, 3))
    for mode in ("nve", "vv", "nvt"):
        q1, p1, _, e1 = o.step_extra(s.q, s.p, 3, zero, mode=mode, noise=noise, tau0=20.0)
        if mode == "nve":
            q2, p2, _, e2 = o.step(s.q, s.p, 3)
        elif mode == "vv":
            q2, p2, _, e2 = o.step_vv(s.q, s.p, 3)
        else:
            q2, p2, _, e2 = o.step_nvt(s.q, s.p, noise, 20.0)
        assert np.allclose(q1, q2, rtol=0, atol=1e-12), mode
        assert np.allclose(p1, p2, rtol=1e-12, atol=1e-12), mode
        assert np.allclose(e1, e2, rtol=1e-12, atol=1e-10), mode

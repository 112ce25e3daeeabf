"""GPU parity of the HIP path (through the C-ABI) against the FP64 CPU oracle.

Tolerances (per evaluation on identical inputs; steps compared after each
step against the oracle stepping the same start state):
  FP64 form: bead forces within 1e-12 x RMS(F), energies 1e-12 relative per
  term (tests._gpu.energy_err), positions and momenta 1e-12 of their largest
  magnitude.
  FP32 form: bead forces within 1e-5 x RMS(F), energies 1e-6 relative per
  term under the same rule.
"""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, energy_err, force_err, from_rows, host, layout_rows, to_rows

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL_F = {FP64: 1e-12, FP32: 1e-5}
TOL_E = {FP64: 1e-12, FP32: 1e-6}


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    return mixpi


def _systems():
    out = [("tiny%d" % k, synth.tiny_random(k)) for k in range(4)]
    out.append(("tiny-wide", synth.tiny_random(9, n_particles=90, box=14.0,
                                                 bead_choices=(1, 2, 4, 8, 16))))
    out.append(("c1", synth.config_c1()))
    out.append(("water-h8-o2", synth.water_box(40, 11.0, 8, 2, seed=4, rc=5.4)))
    out.append(("e256-water", synth.solvated_electron(70, 256, 13.0, seed=5, rc_pp=6.4,
                                                      rc_aa=6.0, n_h=2, n_o=1)))
    return out


SYSTEMS = _systems()


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("name,s", SYSTEMS, ids=[n for n, _ in SYSTEMS])
def test_forces_match_oracle(mp, name, s, prec):
    print(f"[forces] {name} prec={prec}", flush=True)
    sysm = mp.System(s, precision=prec)
    rows = layout_rows(s)
    assert np.array_equal(sysm.bead_index, rows)
    q = dev(to_rows(s, s.q, rows))
    f, e = sysm.forces(q)
    F = from_rows(s, host(f), rows)
    Fo, eo = oracle.OracleSystem(s).forces(s.q)
    assert force_err(F, Fo) <= TOL_F[prec], force_err(F, Fo)
    assert energy_err(host(e)[0], eo) <= TOL_E[prec], (host(e)[0], eo)


@pytest.mark.parametrize("name,s", SYSTEMS[4:], ids=[n for n, _ in SYSTEMS[4:]])
def test_energy_matches_forces_call(mp, name, s):
    sysm = mp.System(s)
    q = dev(to_rows(s, s.q))
    _, e1 = sysm.forces(q)
    e2 = sysm.energy(q)
    assert np.allclose(host(e1), host(e2), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_nm_transform_matches_oracle(mp, N):
    print(f"[nm] N={N}", flush=True)
    rng = np.random.default_rng(N)
    n = 3 if N > 64 else 37
    s = synth.tiny_random(1, n_particles=n, bead_choices=(N,), with_electron=False)
    s.q = rng.normal(size=s.q.shape)
    sysm = mp.System(s)
    o = oracle.OracleSystem(s)
    rows = layout_rows(s)
    x = dev(to_rows(s, s.q, rows))
    fwd = from_rows(s, host(sysm.nm_transform(x, +1)), rows)
    want = o.nm_transform(s.q, +1)
    assert np.abs(fwd - want).max() <= 1e-12 * np.abs(want).max()
    bwd = from_rows(s, host(sysm.nm_transform(x, -1)), rows)
    want = o.nm_transform(s.q, -1)
    assert np.abs(bwd - want).max() <= 1e-12 * np.abs(want).max()


def _step_compare(mp, s, prec, nsteps, tol_q, tol_p, tol_e):
    sysm = mp.System(s, precision=prec)
    o = oracle.OracleSystem(s)
    rows = layout_rows(s)
    Fo0, _ = o.forces(s.q)
    q = dev(to_rows(s, s.q, rows))
    p = dev(to_rows(s, s.p, rows))
    f = dev(to_rows(s, Fo0, rows))
    import torch
    elog = torch.zeros((nsteps, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step(nsteps, q, p, f, elog)
    qo, po, Fo, elo = o.step(s.q, s.p, nsteps, F=Fo0)
    qg, pg = from_rows(s, host(q), rows), from_rows(s, host(p), rows)
    el = host(elog)[:, 0, :]
    dq = np.abs(qg - qo).max() / np.abs(qo).max()
    dp = np.abs(pg - po).max() / np.abs(po).max()
    de = max(energy_err(el[k], elo[k]) for k in range(nsteps))
    assert dq <= tol_q, dq
    assert dp <= tol_p, dp
    assert de <= tol_e, (de, el[-1], elo[-1])
    return sysm, q, p, f


@pytest.mark.parametrize("name,s", [SYSTEMS[0], SYSTEMS[5], SYSTEMS[6], SYSTEMS[7]],
                         ids=["tiny0", "c1", "water-h8-o2", "e256-water"])
def test_one_step_fp64(mp, name, s):
    print(f"[step64] {name}", flush=True)
    _step_compare(mp, s, FP64, 1, 1e-12, 1e-12, 1e-12)


def _per_step(mp, s, nsteps):
    """GPU and oracle stepped one step at a time from the same state: the
    errors of positions and momenta (relative to their largest magnitude)
    and of the energy log after every step."""
    import torch
    sysm = mp.System(s)
    o = oracle.OracleSystem(s)
    rows = layout_rows(s)
    Fo, _ = o.forces(s.q)
    q, p, f = dev(to_rows(s, s.q, rows)), dev(to_rows(s, s.p, rows)), dev(to_rows(s, Fo, rows))
    qo, po = s.q, s.p
    el = torch.zeros((1, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    out = []
    for k in range(nsteps):
        sysm.step(1, q, p, f, el)
        qo, po, Fo, elo = o.step(qo, po, 1, F=Fo)
        qg, pg = from_rows(s, host(q), rows), from_rows(s, host(p), rows)
        out.append((np.abs(qg - qo).max() / np.abs(qo).max(),
                    np.abs(pg - po).max() / np.abs(po).max(),
                    energy_err(host(el)[0, 0], elo[0])))
    return np.array(out)


def test_c1_twenty_steps_fp64(mp):
    """FP64 trajectory of the tiny workload, compared after every one of its
    20 steps at the FP64 bar.  The GPU and the oracle sum forces in
    different orders, so their trajectories part by rounding that each step
    adds and the next carries on: positions about 5e-15 A per step here
    (9e-14 A, 9e-15 of the largest coordinate, after 20 steps)."""
    print("[step64] c1 x20", flush=True)
    err = _per_step(mp, synth.config_c1(), 20)
    print("  max per-step errors (q, p, E):", err.max(axis=0), flush=True)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("name,s", [SYSTEMS[5], SYSTEMS[6]], ids=["c1", "water-h8-o2"])
def test_one_step_fp32(mp, name, s):
    print(f"[step32] {name}", flush=True)
    _step_compare(mp, s, FP32, 1, 1e-12, 1e-6, 1e-6)


FULL = [("c2-water256-h32-o4", synth.config_c2), ("c3-e1024-ion-512w", synth.config_c3)]


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("name,make", FULL, ids=[n for n, _ in FULL])
def test_full_size_forces(mp, name, make, prec):
    """The benchmark systems at full size, every bead compared."""
    print(f"[full forces] {name} prec={prec}", flush=True)
    s = make()
    sysm = mp.System(s, precision=prec)
    rows = layout_rows(s)
    q = dev(to_rows(s, s.q, rows))
    f, e = sysm.forces(q)
    F = from_rows(s, host(f), rows)
    Fo, eo = oracle.OracleSystem(s).forces(s.q)
    assert force_err(F, Fo) <= TOL_F[prec], force_err(F, Fo)
    assert energy_err(host(e)[0], eo) <= TOL_E[prec], (host(e)[0], eo)


@pytest.mark.parametrize("name,make", FULL, ids=[n for n, _ in FULL])
def test_full_size_step_fp64(mp, name, make):
    print(f"[full step64] {name}", flush=True)
    _step_compare(mp, make(), FP64, 2, 1e-12, 1e-12, 1e-12)


def test_e256_ten_steps_fp64(mp):
    """Many-bead ring (FFT normal modes) over 10 steps, compared after every
    step at the FP64 bar (positions part by about 6e-14 A per step: 6e-13 A,
    5e-14 of the largest coordinate, after 10)."""
    print("[step64] e256 x10", flush=True)
    err = _per_step(mp, SYSTEMS[7][1], 10)
    print("  max per-step errors (q, p, E):", err.max(axis=0), flush=True)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("circ", ["0", "1"], ids=["fft", "circulant"])
def test_e2048_step_fp64(mp, circ, monkeypatch):
    """A 2048-bead electron ring (its FFT columns take radix-8 passes) among
    waters, one FP64 step against the oracle at the FP64 bar, through FFT
    items and through bead-space circulant items."""
    monkeypatch.setenv("MIXPI_RING_CIRC", circ)
    monkeypatch.setenv("MIXPI_RING_CIRC_MMAC", "64")     # 12 N^2 = 48 M multiply-adds
    print(f"[step64] e2048 circ={circ}", flush=True)
    s = synth.solvated_electron(40, 2048, 11.0, seed=11, rc_pp=5.4, rc_aa=5.0, n_h=1, n_o=1)
    _step_compare(mp, s, FP64, 1, 1e-12, 1e-12, 1e-12)


@pytest.mark.parametrize("sparse", ["auto", "1"])
def test_pair_counts(mp, sparse, monkeypatch):
    """Candidate and in-cutoff counts equal the oracle's (masked and
    compacted atom-atom sweeps)."""
    if sparse != "auto":
        monkeypatch.setenv("MIXPI_PAIR_SPARSE", sparse)
    s = synth.config_c1()
    sysm = mp.System(s)
    n = s.n_particles
    cand = 0
    for i in range(n):
        for j in range(i + 1, n):
            if s.mol_id[i] == s.mol_id[j] or (s.is_electron[i] and s.is_electron[j]):
                continue
            cand += max(s.n_beads[i], s.n_beads[j])
    assert sysm.pair_candidates() == cand
    sysm.pair_evals(reset=True)
    q = dev(to_rows(s, s.q))
    sysm.forces(q)
    ev = sysm.pair_evals()
    assert ev == oracle.OracleSystem(s).pair_evals(s.q)
    assert 0 < ev[0] + ev[1] <= cand and ev[1] > 0


def test_kernel_time_leaves_caller_state(mp):
    """The per-launch timer runs on library copies and reports three
    positive durations."""
    s = SYSTEMS[7][1]
    sysm = mp.System(s, precision=FP32)
    q, p = dev(to_rows(s, s.q)), dev(to_rows(s, s.p))
    f, _ = sysm.forces(q)
    before = [host(x).copy() for x in (q, p, f)]
    t = sysm.kernel_time(20, q, p, f)
    assert set(t) == {"force", "free_rp", "finish"}
    assert all(np.isfinite(v) and 0.5 < v < 5000.0 for v in t.values()), t
    for x, b in zip((q, p, f), before):
        assert np.array_equal(host(x), b)


def test_nonfinite_energy_is_reported(mp):
    """With the check flag, a non-finite position surfaces as
    MIXPI_E_NONFINITE from mixpi_step (and a clean run returns normally)."""
    import torch
    s = SYSTEMS[5][1]
    sysm = mp.System(s, flags=mp.MIXPI_FLAG_CHECK_FINITE)
    q, p = dev(to_rows(s, s.q)), dev(to_rows(s, s.p))
    f, _ = sysm.forces(q)
    elog = torch.zeros((2, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step(2, q, p, f, elog)
    q2 = q.clone()
    q2[5, 1] = float("nan")
    f2, _ = sysm.forces(q2)
    with pytest.raises(mp.MixPIError) as err:
        sysm.step(2, q2, p.clone(), f2, elog)
    assert err.value.code == mp.MIXPI_E_NONFINITE
    # the flag is cleared: a finite run succeeds again
    sysm.step(2, q, p, f, elog)


def test_nve_conservation_and_dt_squared(mp):
    """NVE on the GPU (FP64 form): the conserved H fluctuates as dt^2 and
    total momentum stays zero (Sec. Evaluation split propagator)."""
    import torch

    def run(dt, nsteps):
        s = synth.water_box(40, 11.0, 8, 2, seed=4, rc=5.4, dt=dt)
        sysm = mp.System(s)
        q, p = dev(to_rows(s, s.q)), dev(to_rows(s, s.p))
        f, _ = sysm.forces(q)
        elog = torch.zeros((nsteps, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
        sysm.step(nsteps, q, p, f, elog)
        h = host(elog)[:, 0, mp.E_NAMES.index("ham")]
        return h.std(), host(p).sum(axis=0)

    s1, ptot = run(0.2, 400)
    s2, _ = run(0.1, 800)
    assert 3.0 < s1 / s2 < 5.5, (s1, s2)
    assert np.abs(ptot).max() < 1e-9


@pytest.mark.parametrize("name,s", [SYSTEMS[5], SYSTEMS[7]], ids=["c1", "e256-water"])
def test_steps_are_bit_reproducible(mp, name, s):
    """Two fresh handles stepping the same state give bit-identical q, p, f
    and energy logs: every sum has a fixed order, and no launch reads what
    another workgroup of the same launch writes."""
    import torch
    out = []
    for _ in range(2):
        sysm = mp.System(s)
        q, p = dev(to_rows(s, s.q)), dev(to_rows(s, s.p))
        f, _ = sysm.forces(q)
        elog = torch.zeros((12, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
        sysm.step(12, q, p, f, elog)
        out.append([host(x).copy() for x in (q, p, f, elog)])
        del sysm
    for a, b in zip(*out):
        assert np.array_equal(a, b)


SHAPES = [(16, "w1"), (16, "w2"), (16, "i4"), (32, "w1"), (32, "w2"), (32, "i2"),
          (64, "w1"), (64, "w2"), (64, "i2"), (64, "i4")]


def _set_shape(monkeypatch, tj, waves):
    monkeypatch.setenv("MIXPI_PAIR_TJ", str(tj))
    monkeypatch.setenv("MIXPI_PAIR_WAVES", "2" if waves == "w2" else "1")
    monkeypatch.setenv("MIXPI_PAIR_IW", waves[1] if waves[0] == "i" else "1")


@pytest.mark.parametrize("tj,waves", SHAPES)
def test_pair_tile_variants(mp, tj, waves, monkeypatch):
    """Every tile shape of the force launch (j-tile width; one wave, two
    waves splitting the j-beads, or two / four waves of 64 i-beads each)
    gives the oracle's forces and energies in both forms."""
    _set_shape(monkeypatch, tj, waves)
    for name, s in (SYSTEMS[4], SYSTEMS[7]):
        Fo, eo = oracle.OracleSystem(s).forces(s.q)
        for prec in (FP64, FP32):
            print(f"[tiles] tj={tj} waves={waves} {name} prec={prec}", flush=True)
            sysm = mp.System(s, precision=prec)
            f, e = sysm.forces(dev(to_rows(s, s.q)))
            F = from_rows(s, host(f))
            assert force_err(F, Fo) <= TOL_F[prec], force_err(F, Fo)
            assert energy_err(host(e)[0], eo) <= TOL_E[prec]


@pytest.mark.parametrize("tj,waves", [(16, "i2"), (32, "i4"), (64, "i2"), (64, "i4")])
def test_pair_i_split_tiles_span_several_i_tiles(mp, tj, waves, monkeypatch):
    """Tiles of 128 or 256 i-beads on blocks whose i-runs span several of
    them: 1200 one-bead atoms (upper-triangle tiles of a group with itself)
    and 4-bead H with 2-bead O (a group pair with shift 1)."""
    _set_shape(monkeypatch, tj, waves)
    for name, s in (("water-400", synth.water_box(400, 23.0, 1, 1, seed=3, rc=9.0)),
                    ("water-h4-o2", synth.water_box(150, 17.0, 4, 2, seed=6, rc=7.0))):
        Fo, eo = oracle.OracleSystem(s).forces(s.q)
        for prec in (FP64, FP32):
            print(f"[i-split] tj={tj} waves={waves} {name} prec={prec}", flush=True)
            sysm = mp.System(s, precision=prec)
            f, e = sysm.forces(dev(to_rows(s, s.q)))
            F = from_rows(s, host(f))
            assert force_err(F, Fo) <= TOL_F[prec], force_err(F, Fo)
            assert energy_err(host(e)[0], eo) <= TOL_E[prec]


@pytest.mark.parametrize("tj,waves,jrun", [(16, "w1", 4), (16, "w2", 2), (32, "i2", 8),
                                           (64, "w1", 2), (64, "i4", 4)])
def test_pair_j_runs(mp, tj, waves, jrun, monkeypatch):
    """Items that sweep several j-tiles in turn (j-runs, the last run of an
    i-tile shorter), with every tile shape: forces, energies and pair counts
    against the oracle; the same bits from repeated calls."""
    _set_shape(monkeypatch, tj, waves)
    monkeypatch.setenv("MIXPI_PAIR_JRUN", str(jrun))
    for name, s in (("water-400", synth.water_box(400, 23.0, 1, 1, seed=3, rc=9.0)),
                    ("water-h4-o2", synth.water_box(150, 17.0, 4, 2, seed=6, rc=7.0)),
                    SYSTEMS[7]):
        o = oracle.OracleSystem(s)
        Fo, eo = o.forces(s.q)
        for prec in (FP64, FP32):
            print(f"[j-run] tj={tj} waves={waves} jrun={jrun} {name} prec={prec}", flush=True)
            sysm = mp.System(s, precision=prec)
            assert sysm.pair_shape()[3] == jrun
            q = dev(to_rows(s, s.q))
            sysm.pair_evals(reset=True)
            f, e = sysm.forces(q)
            F = from_rows(s, host(f))
            assert force_err(F, Fo) <= TOL_F[prec], force_err(F, Fo)
            assert energy_err(host(e)[0], eo) <= TOL_E[prec]
            assert sysm.pair_evals() == o.pair_evals(s.q)
            f2, _ = sysm.forces(q)
            assert np.array_equal(host(f), host(f2))


@pytest.mark.parametrize("tj,waves,jrun", [(16, "i2", 1), (64, "i2", 4), (32, "i4", 2)])
def test_pair_culled_electron_tiles(mp, tj, waves, jrun, monkeypatch):
    """Electron-atom tiles of i-split waves that leave out the j-atoms out of
    reach of their beads (forced on; a box large against the cutoff, so
    most tiles cull some atoms and some cull all): forces, energies and
    in-cutoff pair counts against the oracle, the same bits from a repeated
    call, and the forces of the uncull sweep to rounding."""
    _set_shape(monkeypatch, tj, waves)
    monkeypatch.setenv("MIXPI_PAIR_JRUN", str(jrun))
    for name, s in (("e256-w300", synth.solvated_electron(300, 256, 21.0, seed=7, rc_pp=6.0,
                                                           rc_aa=6.0)),
                    ("e64-w120-h2", synth.solvated_electron(120, 64, 15.4, seed=8, rc_pp=4.5,
                                                             rc_aa=5.0, n_h=2, n_o=1))):
        o = oracle.OracleSystem(s)
        Fo, eo = o.forces(s.q)
        for prec in (FP64, FP32):
            print(f"[cull] tj={tj} waves={waves} jrun={jrun} {name} prec={prec}", flush=True)
            q = dev(to_rows(s, s.q))
            out = []
            for cull in ("1", "0"):
                monkeypatch.setenv("MIXPI_PAIR_CULL", cull)
                sysm = mp.System(s, precision=prec)
                sysm.pair_evals(reset=True)
                f, e = sysm.forces(q)
                F = from_rows(s, host(f))
                assert force_err(F, Fo) <= TOL_F[prec], (cull, force_err(F, Fo))
                assert energy_err(host(e)[0], eo) <= TOL_E[prec], cull
                assert sysm.pair_evals() == o.pair_evals(s.q), cull
                f2, _ = sysm.forces(q)
                assert np.array_equal(host(f), host(f2)), cull
                out.append(F)
                del sysm
            assert force_err(out[0], out[1]) <= (1e-13 if prec == FP64 else 1e-6)


@pytest.mark.parametrize("tj,waves", [(32, "w1"), (32, "w2"), (64, "w1"), (64, "w2"), (64, "i4")])
def test_pair_compacted_sweep(mp, tj, waves, monkeypatch):
    """The compacted atom-atom sweep (a distance pass marks each lane's
    in-cutoff j-slots; the pair math runs for those only) against the masked
    sweep and the oracle, in both forms and with the parameter derivatives.
    The two sweeps add the same terms; they may round differently (the
    order of the j-reaction sums, and the compiler's contraction of each
    loop into fused multiply-adds, which can move an FP32 pair term by an
    ulp), so they agree to rounding: forces and gradients to 1e-12 (FP64)
    or 1e-6 (FP32) of the RMS force; energies and theta-weighted d/dtheta to
    1e-12 (FP64) or 1e-7 (FP32) of the energy scale sum_k |V_k|."""
    _set_shape(monkeypatch, tj, waves)
    for name, s in (SYSTEMS[4], SYSTEMS[6], SYSTEMS[7]):
        osys = oracle.OracleSystem(s)
        Fo, eo = osys.forces(s.q)
        q = dev(to_rows(s, s.q))
        for prec in (FP64, FP32):
            print(f"[compacted] tj={tj} waves={waves} {name} prec={prec}", flush=True)
            res = []
            for sp in (0, 1):
                monkeypatch.setenv("MIXPI_PAIR_SPARSE", str(sp))
                sysm = mp.System(s, precision=prec)
                f, e = sysm.forces(q)
                dq, dth = sysm.energy_adjoint(q)
                res.append([host(x).copy() for x in (f, e, dq, dth)])
                del sysm
            (f0, e0, dq0, dth0), (f1, e1, dq1, dth1) = res
            scale = np.sqrt(np.mean(f0 ** 2))
            tol = 1e-12 if prec == FP64 else 1e-6
            assert np.max(np.abs(f1 - f0)) <= tol * scale
            assert np.max(np.abs(dq1 - dq0)) <= tol * scale
            escale = np.sum(np.abs(e0[0, 1:]))
            tol_e = 1e-12 if prec == FP64 else 1e-7
            theta = np.array([s.pp_q, s.pp_a, s.lj_eps[0, 0], s.lj_sigma[0, 0],
                              s.bond_k[0] if len(s.bond_k) else 0.0,
                              s.angle_k[0] if len(s.angle_k) else 0.0])
            assert np.max(np.abs(e1 - e0)) <= tol_e * escale
            assert np.max(np.abs(theta * (dth1 - dth0))) <= tol_e * escale
            F1 = from_rows(s, f1)
            assert force_err(F1, Fo) <= TOL_F[prec], force_err(F1, Fo)
            assert energy_err(e1[0], eo) <= TOL_E[prec]


@pytest.mark.parametrize("rpw", [1, 2, 4])
def test_epilogue_rows_per_wave(mp, rpw, monkeypatch):
    """Every epilogue grouping (1, 2 or 4 bead rows per wave): forces and
    two FP64 steps match the oracle, and a force call and the step's
    epilogue give the same F bit for bit (same summation order)."""
    monkeypatch.setenv("MIXPI_FIN_RPW", str(rpw))
    for name, s in (SYSTEMS[5], SYSTEMS[6], SYSTEMS[7]):
        print(f"[epilogue] rpw={rpw} {name}", flush=True)
        _step_compare(mp, s, FP64, 2, 1e-12, 1e-12, 1e-12)
        sysm = mp.System(s)
        q, p = dev(to_rows(s, s.q)), dev(to_rows(s, s.p))
        f, _ = sysm.forces(q)
        sysm.step(1, q, p, f)
        f2, _ = sysm.forces(q)
        assert np.array_equal(host(f), host(f2))

"""Matrix-core (MFMA) normal-mode work against the FP64 oracle.

The normal-mode transform of Sec. Evaluation as a dense generated matrix on
the matrix cores (mixpi_nm_transform), and the exact free ring-polymer
propagation of the split step as one dense circulant matrix per propagator
class (MIXPI_RING_MFMA=1), batched over the columns of every ring that
shares it.

Tolerances:
  FP64 form (FP64 matrix instructions): the FP64 bars of the other parity
  tests (1e-12).
  FP32 form, transforms (FP32 matrix instructions on columns shifted by
  their bead 0, sums moved to FP64 every 64 beads): each input and each
  generated matrix entry is rounded once to FP32 (2^-24 relative), so a
  transformed value carries about 2^-24 sqrt(K) |C| max|x - x_0| of error;
  the bar is 1e-6 of the largest transformed value.
  FP32 form, steps: the propagation uses FP64 matrix instructions (FP32 ones
  drifted the conserved energy of 1000 water steps by half its fluctuation),
  so positions meet 1e-12; momenta and energies the FP32 form's bars.
"""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, energy_err, force_err, from_rows, host, layout_rows, to_rows

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    return mixpi


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("N", [16, 32, 64, 256, 2048])
def test_mfma_transform_matches_oracle(mp, N, prec, monkeypatch):
    """Forward and backward transforms of rings of N beads (several columns
    sets, inputs far from the origin as unwrapped positions are)."""
    monkeypatch.setenv("MIXPI_NM_MFMA", "1")
    print(f"[mfma nm] N={N} prec={prec}", flush=True)
    rng = np.random.default_rng(N + prec)
    n = 7 if N >= 256 else 23
    s = synth.tiny_random(1, n_particles=n, bead_choices=(N,), with_electron=False)
    s.q = rng.normal(size=s.q.shape) + rng.uniform(-20, 20, size=(1, 3))
    sysm = mp.System(s, precision=prec)
    o = oracle.OracleSystem(s)
    rows = layout_rows(s)
    x = dev(to_rows(s, s.q, rows))
    for direction in (+1, -1):
        got = from_rows(s, host(sysm.nm_transform(x, direction)), rows)
        want = o.nm_transform(s.q, direction)
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"  dir={direction}: {err:.2e}", flush=True)
        assert err <= (1e-12 if prec == FP64 else 1e-6), err


def _step(mp, s, prec, nsteps, monkeypatch, mfma=True):
    import torch
    monkeypatch.setenv("MIXPI_RING_MFMA", "1" if mfma else "0")
    sysm = mp.System(s, precision=prec)
    o = oracle.OracleSystem(s)
    rows = layout_rows(s)
    Fo0, _ = o.forces(s.q)
    q, p = dev(to_rows(s, s.q, rows)), dev(to_rows(s, s.p, rows))
    f = dev(to_rows(s, Fo0, rows))
    elog = torch.zeros((nsteps, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step(nsteps, q, p, f, elog)
    qo, po, _, elo = o.step(s.q, s.p, nsteps, F=Fo0)
    qg, pg = from_rows(s, host(q), rows), from_rows(s, host(p), rows)
    return qg, pg, host(elog)[:, 0, :], qo, po, elo


CASES = [("c1-e64", synth.config_c1),
         ("e256-water", lambda: synth.solvated_electron(70, 256, 13.0, seed=5, rc_pp=6.4,
                                                        rc_aa=6.0, n_h=2, n_o=1)),
         ("c3-e1024", synth.config_c3)]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_mfma_step_fp64(mp, name, make, monkeypatch):
    """FP64 steps with the rings propagated on the matrix cores: positions,
    momenta and every energy term (the spring energy now summed by the
    epilogue) at the FP64 bar."""
    print(f"[mfma step64] {name}", flush=True)
    s = make()
    qg, pg, el, qo, po, elo = _step(mp, s, FP64, 3, monkeypatch)
    dq = np.abs(qg - qo).max() / np.abs(qo).max()
    dp = np.abs(pg - po).max() / np.abs(po).max()
    de = max(energy_err(el[k], elo[k]) for k in range(3))
    print(f"  dq {dq:.2e} dp {dp:.2e} dE {de:.2e}", flush=True)
    assert dq <= 1e-12 and dp <= 1e-12 and de <= 1e-12, (dq, dp, de)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_mfma_step_fp32(mp, name, make, monkeypatch):
    """FP32 form with the matrix-core propagation: one step against the
    oracle (positions at 1e-12; momenta and energies at the FP32 form's
    bars)."""
    print(f"[mfma step32] {name}", flush=True)
    s = make()
    qg, pg, el, qo, po, elo = _step(mp, s, FP32, 1, monkeypatch)
    dq = np.abs(qg - qo).max() / np.abs(qo).max()
    dp = np.abs(pg - po).max() / np.abs(po).max()
    de = energy_err(el[0], elo[0])
    print(f"  dq {dq:.2e} dp {dp:.2e} dE {de:.2e}", flush=True)
    assert dq <= 1e-12 and dp <= 1e-6 and de <= 1e-6, (dq, dp, de)


@pytest.mark.parametrize("name,make", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_step_without_mfma_items(mp, name, make, monkeypatch):
    """The dense (64-bead) and circulant / FFT (256-bead) step items with the
    matrix-core items switched off, at the FP64 bar."""
    print(f"[no mfma step64] {name}", flush=True)
    s = make()
    qg, pg, el, qo, po, elo = _step(mp, s, FP64, 3, monkeypatch, mfma=False)
    assert np.abs(qg - qo).max() <= 1e-12 * np.abs(qo).max()
    assert np.abs(pg - po).max() <= 1e-12 * np.abs(po).max()
    assert max(energy_err(el[k], elo[k]) for k in range(3)) <= 1e-12


def test_mfma_step_batch_shares_column_sets(mp, monkeypatch):
    """A batch of electron systems with equal bead counts and masses: their
    rings form one propagator class, so one matrix item holds columns of
    several systems.  Two FP64 steps of the batch against each system's
    oracle steps."""
    import torch
    monkeypatch.setenv("MIXPI_RING_MFMA", "1")
    systems = [synth.solvated_electron(40, 128, 11.5, seed=k, rc_pp=5.5, rc_aa=5.4, n_h=2, n_o=1)
               for k in range(7)]
    rows, off = [], 0
    for s in systems:
        r = layout_rows(s)
        rows.append(r + off)
        off += len(r)
    q = np.zeros((off, 3))
    p = np.zeros((off, 3))
    for r, s in zip(rows, systems):
        q[r], p[r] = s.q, s.p
    b = mp.System(systems)
    qd, pd = dev(q), dev(p)
    fd, _ = b.forces(qd)
    elog = torch.zeros((2, len(systems), mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    b.step(2, qd, pd, fd, elog)
    qb, pb, el = host(qd), host(pd), host(elog)
    for k, s in enumerate(systems):
        print(f"[mfma batch] system {k}", flush=True)
        qo, po, _, elo = oracle.OracleSystem(s).step(s.q, s.p, 2)
        assert np.abs(qb[rows[k]] - qo).max() <= 1e-12 * np.abs(qo).max()
        assert np.abs(pb[rows[k]] - po).max() <= 1e-12 * np.abs(po).max()
        for t in range(2):
            assert energy_err(el[t, k], elo[t]) <= 1e-12


def test_mfma_step_with_thermostat(mp, monkeypatch):
    """Thermostatted steps (Langevin half steps in normal modes around the
    matrix-core propagation) against the oracle."""
    import torch
    monkeypatch.setenv("MIXPI_RING_MFMA", "1")
    s = CASES[1][1]()
    rows = layout_rows(s)
    o = oracle.OracleSystem(s)
    nsteps = 3
    noise = np.random.default_rng(3).normal(size=(nsteps, 2, len(rows), 3))
    Fo0, _ = o.forces(s.q)
    qo, po, _, elo = o.step_nvt(s.q, s.p, noise, 25.0, F=Fo0)
    sysm = mp.System(s)
    sysm.set_thermostat(25.0)
    q, p = dev(to_rows(s, s.q, rows)), dev(to_rows(s, s.p, rows))
    f = dev(to_rows(s, Fo0, rows))
    nz = np.empty_like(noise)
    nz[:, :, rows, :] = noise
    elog = torch.zeros((nsteps, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step_nvt(nsteps, q, p, f, dev(nz), elog)
    qg, pg = from_rows(s, host(q), rows), from_rows(s, host(p), rows)
    assert np.abs(qg - qo).max() <= 1e-12 * np.abs(qo).max()
    assert np.abs(pg - po).max() <= 1e-12 * np.abs(po).max()
    for k in range(nsteps):
        assert energy_err(host(elog)[k, 0], elo[k]) <= 1e-12

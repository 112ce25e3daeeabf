"""Long NVE runs of the two benchmark workloads in both precision forms.

Over 1000 steps chaotic divergence makes a state-by-state comparison with
the oracle ill-posed, so the FP32 form's dynamics are compared with the
FP64 form's from the same start state (split propagator of Sec.
Evaluation): the drift and fluctuation of the conserved H, and the means of
V_mix and of the centroid-virial kinetic energy (Sec. Output and Analysis).

Bars: the drift of H within 5 % of its fluctuation and the fluctuations
within 5 % of each other; the means within 3 standard errors (10 block
means of the FP64 run) and, tighter, within 1e-5 of their magnitude (the
FP32 form's pair forces carry relative errors of about 1e-6).
"""
import numpy as np
import pytest

import synth
from tests._gpu import dev, host, to_rows

pytestmark = pytest.mark.gpu

NSTEPS = 1000


@pytest.fixture(scope="module")
def mp():
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    return mixpi


def _run(mp, s, prec):
    import torch
    sysm = mp.System(s, precision=prec)
    q, p = dev(to_rows(s, s.q)), dev(to_rows(s, s.p))
    f, _ = sysm.forces(q)
    elog = torch.zeros((NSTEPS, 1, mp.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step(NSTEPS, q, p, f, elog)
    el = host(elog)[:, 0, :]
    del sysm
    return el


def _h_stats(h):
    x = np.arange(len(h))
    slope, icpt = np.polyfit(x, h, 1)
    return h[-1] - h[0], float(np.std(h - (slope * x + icpt)))


@pytest.mark.parametrize("name,make", [("c2-water256-h32-o4", synth.config_c2),
                                       ("c3-e1024-ion-512w", synth.config_c3)],
                         ids=["c2", "c3"])
def test_fp32_and_fp64_long_runs_agree(mp, name, make):
    print(f"[long run] {name}: {NSTEPS} steps in each form", flush=True)
    s = make()
    el64 = _run(mp, s, mp.MIXPI_FP64)
    el32 = _run(mp, s, mp.MIXPI_FP32_ACC64)
    assert np.isfinite(el64).all() and np.isfinite(el32).all()
    ih = mp.E_NAMES.index("ham")
    d64, f64 = _h_stats(el64[:, ih])
    d32, f32 = _h_stats(el32[:, ih])
    print(f"  H drift {d64:.6f} / {d32:.6f} kcal/mol, fluctuation {f64:.6f} / {f32:.6f} "
          f"(FP64 / FP32)", flush=True)
    assert abs(d32 - d64) <= 0.05 * f64, (d32, d64, f64)
    assert abs(f32 / f64 - 1.0) <= 0.05, (f32, f64)
    for key in ("vmix", "kcv"):
        k = mp.E_NAMES.index(key)
        m64, m32 = el64[:, k].mean(), el32[:, k].mean()
        se = el64[:, k].reshape(10, -1).mean(axis=1).std(ddof=1) / np.sqrt(10)
        print(f"  <{key}> {m64:.6f} / {m32:.6f} (block standard error {se:.4f})", flush=True)
        assert abs(m32 - m64) <= 3.0 * se, (key, m32, m64, se)
        assert abs(m32 - m64) <= 1e-5 * abs(m64), (key, m32, m64)

"""Throughput of the mixTS-PIMD hot path on one MI355X.

Workload (default): one 1024-bead electron, a +3 cation and 512 flexible
waters (1537 classical atoms) in a 24.8 A periodic box; electron-atom
softened Coulomb cut at 12 A, atom-atom LJ + Coulomb cut at 9 A; the FP32
form (FP32 pseudopotential and 1/r seeds, FP64 atom-atom terms, separations,
sums and integrator state); dt 0.1 fs.
A step is one full PIMD step: half-kick, exact free ring-polymer
propagation in normal modes, bead forces of V_mix, half-kick, energies.

Prints one JSON line.  value = in-cutoff slice-pair evaluations per second
over the timed steps (counted on the device); steps/s and the FP64 form's
figures ride along.  Inputs are resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FLOPs of the force launch (op counts of the kernel's arithmetic;
# FMA = 2, add/mul/compare/rint/rsqrt/rcp/sqrt/acos = 1):
#   every candidate slice-pair: separation, nearest image, r^2, cutoff test
#   an in-cutoff atom-atom slice-pair adds the Coulomb energy and force,
#     the force scale and the i/j force and energy sums
#   one with a Lennard-Jones type pair (eps != 0) inside its cutoff adds the
#     reciprocal and the LJ energy and force
#   an in-cutoff electron-atom slice-pair adds the pseudopotential + sums
#   a bond / angle slice (bonded workgroups of the same launch)
FLOP_CANDIDATE = 21
FLOP_ATOM_IN = 23
FLOP_LJ_IN = 19
FLOP_PP_IN = 25
FLOP_BOND = 35
FLOP_ANGLE = 100
# ALU ceiling of the launch: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz.
# The library is built without packed FP32, so FP32 and FP64 issue at the
# same rate; the 157.3 TFLOP/s FP32 figure needs packed FP32.
PEAK_ALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# HBM traffic of one force launch on the default workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by the same counters
# on a plain 256 MiB device copy; valid only while the kernel source is the
# one it was measured on (sha256 over KERNEL_SOURCES).
KERNEL_SOURCES = ("paper_2411_11988_amd/csrc/pair.hip", "paper_2411_11988_amd/csrc/device_common.h",
                  "paper_2411_11988_amd/csrc/mixpi_internal.h")
# VALU work of one force launch on the default workload, from rocprofv3
# --pmc (SQ_INSTS_VALU and the FP32/FP64 add/mul/fma/transcendental
# instruction counters, 64 lanes each, FMA = 2): executed FLOP including the
# masked-off math of out-of-cutoff candidates; same source-hash condition.
VALU = {"insts_valu": 2735846, "flop_executed": 145581526}
TRAFFIC = {"workload": "c3", "tile": "16xw1",
           "sha256": "e4999018cc50888b498a011093fba6dbd1207bdbff7d382c4eaf37b767039fc6",
           "bytes": (1491.95 * 2.0 + 10881.93 * 1.0) * 1024}


def _kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _executed(launch_us):
    """Counter-based work of the force launch over its measured duration:
    executed TFLOP/s and its fraction of the ALU peak, and the share of the
    launch the 1024 SIMDs spend issuing VALU instructions (4 cycles each at
    2.4 GHz)."""
    t = launch_us * 1e-6
    tf = VALU["flop_executed"] / t / 1e12
    return {"flop_per_launch": VALU["flop_executed"], "tflops": tf,
            "frac": tf / PEAK_ALU_TFLOPS,
            "valu_issue_frac": VALU["insts_valu"] * 4 / 1024 / (t * 2.4e9)}


def _workload(name, gen_workers=None):
    import synth
    if name == "c3":
        return synth.config_c3(), "e1024-ion-512w (1024-bead e-, +3 ion, 512 H2O, 24.8 A)"
    if name == "c2":
        return synth.config_c2(), "water256 N_H=32 N_O=4 (19.7 A)"
    if name == "c1":
        return synth.config_c1(), "e64-ion-32w (10 A)"
    if name == "c4":
        return (synth.config_c4_states(1)[0],
                "water256 N_H=32 N_O=4, gradient workload seed 0 (19.7 A)")
    if name == "c5":
        print("[bench] generating the 64-system batch", file=sys.stderr, flush=True)
        workers = synth.build_workers() if gen_workers is None else (gen_workers or None)
        return (synth.config_c5(workers=workers),
                "batch64 e-/ion/water (P in 256..2048, 128..1024 H2O per system)")
    raise SystemExit(f"unknown workload {name}")


def _as_list(s):
    return list(s) if isinstance(s, (list, tuple)) else [s]


def _run(s, precision, steps, warmup, mixpi, torch, flags=0):
    import numpy as np
    systems = _as_list(s)
    sysm = mixpi.System(s, precision=precision, flags=flags)
    idx = sysm.bead_index
    n_sys = len(systems)

    def dev(x):
        out = np.empty_like(x)
        out[idx] = x
        return torch.from_numpy(out).cuda()

    q = dev(np.concatenate([x.q for x in systems]))
    p = dev(np.concatenate([x.p for x in systems]))
    f, _ = sysm.forces(q)
    elog_w = torch.zeros((max(warmup, 1), n_sys, mixpi.MIXPI_NE), dtype=torch.float64,
                         device="cuda")
    elog = torch.zeros((steps, n_sys, mixpi.MIXPI_NE), dtype=torch.float64, device="cuda")
    if warmup > 0:
        sysm.step(warmup, q, p, f, elog_w)
    sysm.step_prepare(steps, q, p, f, elog)
    torch.cuda.synchronize()
    sysm.pair_evals(reset=True)
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    sysm.step(steps, q, p, f, elog)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    ev_atom, ev_pp = sysm.pair_evals(reset=True)
    el = elog.cpu().numpy()
    ham = el[:, :, mixpi.E_NAMES.index("ham")]
    drift = ham[-1] - ham[0]
    return dict(sysm=sysm, q=q, p=p, f=f, ms=ms, ev=(ev_atom, ev_pp), elog=el,
                drift=float(drift[np.argmax(np.abs(drift))]), hstd=float(ham.std(axis=0).max()))


def _run_sequential(systems, precision, steps, mixpi, torch):
    """The batch's systems as separate handles, each running the same number
    of steps (one captured graph per system) one after another on the
    stream: the comparison for a batched handle."""
    import numpy as np
    handles = []
    for x in systems:
        h = mixpi.System(x, precision=precision)
        idx = h.bead_index

        def dev(a, idx=idx):
            out = np.empty_like(a)
            out[idx] = a
            return torch.from_numpy(out).cuda()
        q, p = dev(x.q), dev(x.p)
        f, _ = h.forces(q)
        h.step(steps, q, p, f)                                    # captures the graph
        handles.append((h, q, p, f))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for h, q, p, f in handles:
        h.step(steps, q, p, f)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return {"ms_per_batch_step": ms / steps,
            "system_steps_per_s": len(systems) * steps / (ms * 1e-3)}


def _run_nvt(s, precision, steps, mixpi, torch, flags=0, tau0=50.0):
    """Thermostatted steps (O B A B O) with the noise drawn beforehand and
    resident in HBM; returns steps/s and the time per step."""
    import numpy as np
    systems = _as_list(s)
    sysm = mixpi.System(s, precision=precision, flags=flags)
    sysm.set_thermostat(tau0)
    idx = sysm.bead_index

    def dev(x):
        out = np.empty_like(x)
        out[idx] = x
        return torch.from_numpy(out).cuda()

    q = dev(np.concatenate([x.q for x in systems]))
    p = dev(np.concatenate([x.p for x in systems]))
    f, _ = sysm.forces(q)
    gen = torch.Generator(device="cuda").manual_seed(0)
    noise = torch.randn((steps, 2, sysm.rows, 3), dtype=torch.float64, device="cuda",
                        generator=gen)
    elog = torch.zeros((steps, len(systems), mixpi.MIXPI_NE), dtype=torch.float64,
                       device="cuda")
    sysm.step_nvt(2, q, p, f, noise[:2], elog[:2])                # warm-up
    sysm.step_nvt(steps, q, p, f, noise, elog)                    # captures the graph
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    t0.record(stream)
    sysm.step_nvt(steps, q, p, f, noise, elog)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return {"steps_per_s": steps / (ms * 1e-3), "ms_per_step": ms / steps, "tau0_fs": tau0}


def _run_vv(s, precision, steps, mixpi, torch, flags=0):
    """Velocity-Verlet steps with spring forces: steps/s and time per step."""
    import numpy as np
    systems = _as_list(s)
    sysm = mixpi.System(s, precision=precision, flags=flags)
    idx = sysm.bead_index

    def dev(x):
        out = np.empty_like(x)
        out[idx] = x
        return torch.from_numpy(out).cuda()

    q = dev(np.concatenate([x.q for x in systems]))
    p = dev(np.concatenate([x.p for x in systems]))
    f, _ = sysm.forces(q)
    elog = torch.zeros((steps, len(systems), mixpi.MIXPI_NE), dtype=torch.float64,
                       device="cuda")
    sysm.step_vv(steps, q, p, f, elog)                            # captures the graph
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    t0.record(stream)
    sysm.step_vv(steps, q, p, f, elog)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return {"steps_per_s": steps / (ms * 1e-3), "ms_per_step": ms / steps}


def _run_observables(sysm, q, p, s, mixpi, torch, reps=50):
    """The observables and the long-range electrostatics on the workload's
    configuration: mean time per call over `reps` calls (HIP events on the
    stream the library launches on), after warmup calls."""
    import numpy as np
    box = min(float(np.min(x.box)) for x in _as_list(s))      # every system's box
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(n):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) * 1e3 / n

    nb, rmax = 256, 0.5 * box
    hist = torch.zeros((sysm.n_systems, 9, 9, nb), dtype=torch.float64, device="cuda")
    rdf_us = timed(lambda: sysm.rdf(q, rmax, nb, hist), reps)
    L = 1000
    ring = torch.zeros((L, sysm.n_particles, 3), dtype=torch.float64, device="cuda")
    acc = torch.zeros((sysm.n_systems, 9, L), dtype=torch.float64, device="cuda")
    t = [0]

    def sample():
        sysm.vacf_sample(p, t[0] + L, ring, acc)    # a full window of lags
        t[0] += 1
    vacf_us = timed(sample, reps)
    alpha, rcut, grid, order = 0.35, min(9.0, 0.5 * box), 32, 6
    sysm.set_ewald(alpha, rcut, grid, order)
    f = torch.zeros_like(q)
    e = torch.zeros((sysm.n_systems, 3), dtype=torch.float64, device="cuda")
    ew_us = timed(lambda: sysm.ewald(q, f, e), reps)
    cand = sysm.pair_candidates()
    # normal-mode transforms of the whole state (matrix-core items for rings
    # of 16 to 64 beads, FFT or dense items otherwise), forward and backward;
    # algorithmic bytes: the state in and out, 48 B per bead row
    nm = torch.empty_like(q)
    fwd_us = timed(lambda: sysm.nm_transform(q, +1, out=nm), reps)
    bwd_us = timed(lambda: sysm.nm_transform(nm, -1, out=f), reps)
    nm_bytes = 48 * int(sysm.rows)
    return {"nm_transform": {"fwd_us": fwd_us, "bwd_us": bwd_us, "bytes": nm_bytes,
                             "fwd_GBps": nm_bytes / (fwd_us * 1e-6) / 1e9,
                             "bwd_GBps": nm_bytes / (bwd_us * 1e-6) / 1e9},
            "rdf": {"us_per_call": rdf_us, "nbins": nb, "r_max": rmax,
                    "slice_pairs_per_s": cand / (rdf_us * 1e-6)},
            "vacf": {"us_per_sample": vacf_us, "lags": L},
            "ewald": {"us_per_call": ew_us, "alpha": alpha, "r_cut": rcut, "grid": grid,
                      "order": order}}


def _run_ewald_step(s, precision, steps, mixpi, torch, flags=0):
    """NVE steps with the atom-atom electrostatics moved from the cut form
    (rc_coul = 0) to the centroid Ewald sum inside the step."""
    import dataclasses
    import numpy as np
    systems = [dataclasses.replace(x, rc_coul=0.0) for x in _as_list(s)]
    sysm = mixpi.System(systems if len(systems) > 1 else systems[0], precision=precision,
                        flags=flags)
    box = min(float(np.min(x.box)) for x in systems)
    alpha, rcut, grid, order = 0.35, min(9.0, 0.5 * box), 32, 6
    sysm.set_ewald(alpha, rcut, grid, order)
    sysm.use_ewald(True)
    idx = sysm.bead_index

    def dev(x):
        out = np.empty_like(x)
        out[idx] = x
        return torch.from_numpy(out).cuda()

    q = dev(np.concatenate([x.q for x in systems]))
    p = dev(np.concatenate([x.p for x in systems]))
    f, _ = sysm.forces(q)
    elog = torch.zeros((steps, len(systems), mixpi.MIXPI_NE), dtype=torch.float64, device="cuda")
    sysm.step(steps, q, p, f, elog)                               # captures the graph
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    t0.record(stream)
    sysm.step(steps, q, p, f, elog)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    h = elog[:, 0, mixpi.E_NAMES.index("ham")].cpu().numpy()
    return {"steps_per_s": steps / (ms * 1e-3), "ms_per_step": ms / steps,
            "energy_drift_kcal": float(h[-1] - h[0]),
            "ewald": {"alpha": alpha, "r_cut": rcut, "grid": grid, "order": order}}


def _run_adjoint(sysm, q, s, mixpi, torch, reps=50):
    """The gradient workload: one energy + adjoint evaluation (dV/dq and
    dV/dtheta of the six parameters) per call, timed as the library call and
    as torch.autograd forward + backward through energy_function()."""
    import numpy as np
    x = s if not isinstance(s, (list, tuple)) else s[0]
    theta = torch.tensor([[x.pp_q, x.pp_a, x.lj_eps[0, 0], x.lj_sigma[0, 0],
                           x.bond_k[0] if len(x.bond_k) else 0.0,
                           x.angle_k[0] if len(x.angle_k) else 0.0]],
                         dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    dq = torch.empty_like(q)
    dth = torch.empty((1, 6), dtype=torch.float64, device="cuda")

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) * 1e3 / reps

    adj_us = timed(lambda: sysm.energy_adjoint(q, theta, dq=dq, dtheta=dth))
    fn = mixpi.energy_function()
    qa = q.clone().requires_grad_(True)
    ta = theta.clone().requires_grad_(True)

    def fwd_bwd():
        qa.grad = None
        ta.grad = None
        fn.apply(qa, ta, sysm).sum().backward()
    ag_us = timed(fwd_bwd)
    f_us = timed(lambda: sysm.forces(q))
    return {"adjoint_us": adj_us, "autograd_fwd_bwd_us": ag_us, "forces_us": f_us,
            "theta": ["pp_q", "pp_a", "eps_00", "sigma_00", "k_bond0", "k_angle0"]}


def _split_state(x_rows, idx, s):
    """Bead tables (particle-major) of every system from a state array in
    the library layout."""
    beads = x_rows[idx]
    out, o = [], 0
    for x in _as_list(s):
        n = int(sum(x.n_beads))
        out.append(beads[o:o + n])
        o += n
    return out


def _lj_slice_pairs(s, q):
    """Slice-pairs of V_mix with a Lennard-Jones term inside its cutoff
    (eps != 0, r^2 < rc_lj^2, different molecules, no electron), from the
    bead positions q (particle-major bead table) by the slice map: the
    LJ share of the in-cutoff count, which the FLOP table charges LJ to."""
    import numpy as np
    total = 0
    for x, qx in zip(_as_list(s), q):
        nb = np.asarray(x.n_beads)
        off = np.concatenate([[0], np.cumsum(nb)])
        t = np.asarray(x.lj_type)
        nt = x.lj_eps.shape[0]
        lj = (t >= 0) & (np.asarray(x.is_electron) == 0)
        lj &= np.array([np.any(x.lj_eps[ti] != 0) if ti >= 0 else False for ti in t])
        idx = np.flatnonzero(lj)
        if len(idx) < 2:
            continue
        L = np.asarray(x.box, dtype=np.float64)
        rc2 = x.rc_lj ** 2
        tt = np.clip(t[idx], 0, nt - 1)
        eps = x.lj_eps[tt[:, None], tt[None, :]]
        mol = np.asarray(x.mol_id)[idx]
        upper = np.triu(np.ones((len(idx), len(idx)), dtype=bool), 1)
        keep = upper & (eps != 0) & (mol[:, None] != mol[None, :])
        ni = nb[idx]
        nmax = np.maximum(ni[:, None], ni[None, :])
        for N in np.unique(nmax[keep]):
            sel = keep & (nmax == N)
            for sl in range(int(N)):
                pos = qx[off[idx] + (sl * ni) // N]
                d = pos[:, None, :] - pos[None, :, :]
                d -= L * np.rint(d / L)
                total += int(np.count_nonzero(sel & ((d * d).sum(-1) < rc2)))
    return total


def _culled_candidates(s, q, shape):
    """Electron-atom candidates the force launch leaves out (the j-atoms of a
    tile out of reach of its beads, found as the kernel finds them: the
    periodic gap from the tile's bead box, offsets from its first bead, to
    the atom is at least rc_pp + 1e-6), from the bead positions q.  The
    library culls in electron-atom blocks of tiles with several i-split
    waves and one j-wave, in boxes where a sphere of rc_pp + 3 A is under
    0.6 of the volume (MIXPI_PAIR_CULL overrides); counted here for systems
    of one electron and one-bead atoms, the synthetic workloads' form."""
    import os
    import numpy as np
    tjs, waves, iw, _ = shape
    env = os.environ.get("MIXPI_PAIR_CULL")
    if waves != 1 or iw < 2 or env == "0":
        return 0
    total = 0
    for k, (x, qx) in enumerate(zip(_as_list(s), q)):
        nb = np.asarray(x.n_beads)
        ele = np.asarray(x.is_electron)
        L = np.asarray(x.box, dtype=np.float64)
        big = 4.0 / 3.0 * np.pi * (x.rc_pp + 3.0) ** 3 < 0.6 * float(np.prod(L))
        if not (big or env == "1") or ele.sum() != 1 or ele[0] != 1 or np.any(nb[1:] != 1):
            continue
        P, tj = int(nb[0]), int(tjs[k])
        xe, xa = qx[:P], qx[P:]
        rc = x.rc_pp + 1e-6
        for i0 in range(0, P, 64 * iw):
            c = xe[i0:i0 + 64 * iw]
            d = c - c[0]
            d -= L * np.rint(d / L)
            lo, hi = d.min(0), d.max(0)
            dj = xa - c[0]
            dj -= L * np.rint(dj / L)
            g = np.full(dj.shape, np.inf)
            for m in (-1.0, 0.0, 1.0):
                e = dj + m * L
                g = np.minimum(g, np.maximum(0.0, np.maximum(lo - e, e - hi)))
            culled = (g * g).sum(-1) >= rc * rc
            total += len(c) * int(culled.sum())
    return total


def _bonded_slices(s):
    """Bond and angle slices: each term is evaluated on N_max slices."""
    n_bond = n_angle = 0
    for x in _as_list(s):
        nb = x.n_beads
        n_bond += int(sum(max(nb[i], nb[j]) for i, j in x.bonds))
        n_angle += int(sum(max(nb[i], nb[j], nb[k]) for i, j, k in x.angles))
    return n_bond, n_angle


def _cpu_info():
    """CPU model (from /proc/cpuinfo) and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def _oracle_rate(o, q, p, F, target_s, max_steps=200):
    """Oracle steps from (q, p, F) for about target_s seconds: returns
    (steps, seconds, pair evaluations per step, state after)."""
    t = time.perf_counter()
    q1, p1, F1, _ = o.step(q, p, 1, F=F)
    one = time.perf_counter() - t
    n = max(1, min(max_steps, int(target_s / max(one, 1e-6))))
    evals = sum(o.pair_evals(q1))
    t = time.perf_counter()
    q2, p2, F2, _ = o.step(q1, p1, n, F=F1)
    return n, time.perf_counter() - t, evals, (q2, p2, F2)


def _cpu_baseline_batch(systems, target_s):
    """The FP64 CPU oracle on a batch: every system stepped alone, 10 steps
    each (after one untimed step), on all cores; the batch's oracle time per
    step is the sum of the per-system times per step.  A 1-thread pass runs
    the first systems until target_s / 4 has passed."""
    import oracle
    model, cores = _cpu_info()
    oracle.set_threads(cores)
    evals = spent = 0.0
    for s in systems:
        o = oracle.OracleSystem(s)
        F, _ = o.forces(s.q)
        q1, p1, F1, _ = o.step(s.q, s.p, 1, F=F)
        ev = sum(o.pair_evals(q1))
        t = time.perf_counter()
        o.step(q1, p1, 10, F=F1)
        dt = (time.perf_counter() - t) / 10
        spent += dt
        evals += ev
    single = dict(evals=0.0, spent=0.0, done=0)
    oracle.set_threads(1)
    try:
        for s in systems:
            o = oracle.OracleSystem(s)
            F, _ = o.forces(s.q)
            t = time.perf_counter()
            o.step(s.q, s.p, 1, F=F)
            single["spent"] += time.perf_counter() - t
            single["evals"] += sum(o.pair_evals(s.q))
            single["done"] += 1
            if single["spent"] > target_s / 4:
                break
    finally:
        oracle.set_threads(cores)
    return dict(value=evals / spent, unit="pair-evals/s", cores=oracle.num_threads(),
                kind="oracle", cpu_model=model, steps_per_s=1.0 / spent,
                value_1thread=single["evals"] / single["spent"],
                sample=(f"each of the {len(systems)} systems alone: 10 FP64 oracle steps after 1 "
                        f"untimed step; batch step time = sum of the per-system step times "
                        f"({spent:.3f} s); 1-thread rate from one step of each of the first "
                        f"{single['done']} systems"))


def _cpu_baseline(s, target_s=15.0):
    """The FP64 CPU oracle stepping the same system on the host cores: all
    cores the process may use, then one thread."""
    import oracle
    if isinstance(s, (list, tuple)):
        return _cpu_baseline_batch(s, target_s)
    model, cores = _cpu_info()
    oracle.set_threads(cores)
    o = oracle.OracleSystem(s)
    F, _ = o.forces(s.q)
    n, dt, evals, state = _oracle_rate(o, s.q, s.p, F, target_s)
    oracle.set_threads(1)
    try:
        n1, dt1, evals1, _ = _oracle_rate(o, *state, target_s / 3, max_steps=50)
    finally:
        oracle.set_threads(cores)
    return dict(value=evals * n / dt, unit="pair-evals/s", cores=oracle.num_threads(),
                kind="oracle", cpu_model=model, steps_per_s=n / dt,
                value_1thread=evals1 * n1 / dt1, steps_per_s_1thread=n1 / dt1,
                sample=f"{n} FP64 oracle steps of the same system on {cores} threads "
                       f"(term-by-term V_mix, OpenMP over particles) after 1 untimed step; "
                       f"then {n1} steps on 1 thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--nvt", action=argparse.BooleanOptionalAction, default=True,
                    help="also time thermostatted (path-integral Langevin) steps and "
                         "velocity-Verlet steps")
    ap.add_argument("--observables", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the radial distribution, velocity correlation and centroid "
                         "Ewald calls on the workload's configuration")
    ap.add_argument("--tile", default="heuristic", choices=["auto", "heuristic"],
                    help="pair-sweep tile shape: the library's choice from the work size "
                         "(default; measured best on these workloads) or autotuned per "
                         "workload bucket")
    ap.add_argument("--kernel-sha", action="store_true",
                    help="print the sha256 of the force-kernel sources and exit")
    ap.add_argument("--gen-workers", type=int, default=None,
                    help="processes that build the batch's systems (0: this process alone; "
                         "default: the host's cores, at most 16)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (a known-size "
                         "kernel that calibrates hardware byte counters)")
    args = ap.parse_args()
    if args.kernel_sha:
        print(_kernel_sha())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent systems shard with zero communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_11988_amd import mixpi
    mixpi.load()
    torch.cuda.set_device(0)
    s, wname = _workload(args.workload, args.gen_workers)

    flags32 = flags64 = 0
    tile = "heuristic"
    if args.tile == "auto":
        from paper_2411_11988_amd import tune
        print("[bench] autotuning the pair tile shape", file=sys.stderr, flush=True)
        flags32 = tune.tile_flags(s, mixpi.MIXPI_FP32_ACC64)
        flags64 = tune.tile_flags(s, mixpi.MIXPI_FP64)
        tile = {"fp32": tune.describe(flags32), "fp64": tune.describe(flags64)}
    print(f"[bench] {wname}: FP32 pair form, {args.warmup} warmup + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    r32 = _run(s, mixpi.MIXPI_FP32_ACC64, args.steps, args.warmup, mixpi, torch, flags32)
    sysm = r32["sysm"]
    ev_step = (r32["ev"][0] + r32["ev"][1]) / args.steps
    value = (r32["ev"][0] + r32["ev"][1]) / (r32["ms"] * 1e-3)
    steps_per_s = args.steps / (r32["ms"] * 1e-3)

    # each launch of the step timed with HIP events around it, inside eager
    # steps on the step's stream (same inputs and cache state as the graph)
    print("[bench] per-launch timing", file=sys.stderr, flush=True)
    reps = 200
    k_us = sysm.kernel_time(reps, r32["q"], r32["p"], r32["f"])
    cand = sysm.pair_candidates()
    ev_atom, ev_pp = (x / args.steps for x in r32["ev"])
    n_bond, n_angle = _bonded_slices(s)
    q_end = [x for x in _split_state(r32["q"].cpu().numpy(), sysm.bead_index, s)]
    ev_lj = _lj_slice_pairs(s, q_end)
    # candidates the launch never distance-checks are not charged
    culled = _culled_candidates(s, q_end, sysm.pair_shape())
    cand -= culled
    flops = (cand * FLOP_CANDIDATE + ev_atom * FLOP_ATOM_IN + ev_lj * FLOP_LJ_IN
             + ev_pp * FLOP_PP_IN + n_bond * FLOP_BOND + n_angle * FLOP_ANGLE)
    achieved = flops / (k_us["force"] * 1e-6) / 1e12

    out = {
        "metric": "pair-force evals/s + PIMD steps/s, 1024-bead e-/512 H2O, FP32 vs FP64",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "beads": int(sysm.rows), "particles": int(sysm.n_particles),
                   "candidate_slice_pairs": int(cand), "in_cutoff_slice_pairs": ev_step,
                   "systems": len(_as_list(s)), "dt_fs": _as_list(s)[0].dt,
                   "precision": ("fp32 electron-atom pseudopotential and 1/r seeds; fp64 atom-atom "
                                 "terms, separations, state and sums"),
                   "pair_tile_tj_x_waves": tile,
                   "pair_shape_fp32": dict(zip(("tj", "waves", "i_waves", "j_run"),
                                               (sorted(set(sysm.pair_shape()[0])),
                                                *sysm.pair_shape()[1:])))},
        "steps_per_s": steps_per_s,
        "kernel_us": k_us,
        "energy_drift_kcal": r32["drift"],
        "energy_std_kcal": r32["hstd"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS,
                     "traffic": (TRAFFIC["bytes"] if args.workload == TRAFFIC["workload"]
                                 and TRAFFIC["sha256"] == _kernel_sha()
                                 and (tile == "heuristic" or tile["fp32"] == TRAFFIC["tile"])
                                 else None),
                     "kernel": "k_pair<float,false,WAVES> (pair_tile_tj_x_waves)",
                     "flop_per_launch": flops, "launch_us": k_us["force"],
                     "lj_slice_pairs": ev_lj,
                     "candidates_culled": culled,
                     "executed": (_executed(k_us["force"]) if args.workload == TRAFFIC["workload"]
                                  and TRAFFIC["sha256"] == _kernel_sha()
                                  and (tile == "heuristic" or tile["fp32"] == TRAFFIC["tile"])
                                  else None)},
    }
    if args.workload == "c4":
        print("[bench] energy adjoint and autograd (FP32 form)", file=sys.stderr, flush=True)
        out["adjoint"] = _run_adjoint(sysm, r32["q"], s, mixpi, torch)
    if len(_as_list(s)) > 1:
        print("[bench] the same systems as separate handles, one after another",
              file=sys.stderr, flush=True)
        seq = _run_sequential(_as_list(s), mixpi.MIXPI_FP32_ACC64, args.steps, mixpi, torch)
        batched = len(_as_list(s)) * steps_per_s
        out["sequential"] = dict(seq, batched_system_steps_per_s=batched,
                                 batched_speedup=batched / seq["system_steps_per_s"])
    if args.observables:
        print("[bench] observables and centroid electrostatics", file=sys.stderr, flush=True)
        out["observables"] = _run_observables(sysm, r32["q"], r32["p"], s, mixpi, torch)
        print("[bench] NVE steps with centroid Ewald electrostatics (FP32 form)",
              file=sys.stderr, flush=True)
        out["ewald_step"] = _run_ewald_step(s, mixpi.MIXPI_FP32_ACC64, args.steps, mixpi, torch,
                                            flags32)
    if args.nvt:
        print("[bench] thermostatted steps (FP32 form)", file=sys.stderr, flush=True)
        out["nvt"] = _run_nvt(s, mixpi.MIXPI_FP32_ACC64, args.steps, mixpi, torch, flags32)
        print("[bench] velocity-Verlet steps (FP32 form)", file=sys.stderr, flush=True)
        out["vv"] = _run_vv(s, mixpi.MIXPI_FP32_ACC64, args.steps, mixpi, torch, flags32)
    if not args.no_fp64:
        print("[bench] FP64 form", file=sys.stderr, flush=True)
        r64 = _run(s, mixpi.MIXPI_FP64, args.steps, args.warmup, mixpi, torch, flags64)
        out["fp64"] = {"value": (r64["ev"][0] + r64["ev"][1]) / (r64["ms"] * 1e-3),
                       "steps_per_s": args.steps / (r64["ms"] * 1e-3),
                       "ms_per_step": r64["ms"] / args.steps,
                       "energy_drift_kcal": r64["drift"], "energy_std_kcal": r64["hstd"],
                       "kernel_us": r64["sysm"].kernel_time(reps, r64["q"], r64["p"], r64["f"])}
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(s)
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * n * 8
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

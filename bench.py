"""Throughput of the mixTS-PIMD hot path on one MI355X.

Workload (default): one 1024-bead electron, a +3 cation and 512 flexible
waters (1537 classical atoms) in a 24.8 A periodic box; electron-atom
softened Coulomb cut at 12 A, atom-atom LJ + Coulomb cut at 9 A; FP32 pair
potentials with FP64 separations, sums and integrator state; dt 0.1 fs.
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

# algorithmic FLOPs per slice-pair of the pair sweep (op counts of the
# kernel's arithmetic; FMA = 2, add/mul/compare/rint/rsqrt/rcp = 1):
#   every candidate: separation, nearest image, r^2 and cutoff test
#   an in-cutoff atom-atom pair adds LJ + Coulomb + force/energy sums
#   an in-cutoff electron-atom pair adds the pseudopotential + sums
FLOP_CANDIDATE = 21
FLOP_ATOM_IN = 38
FLOP_PP_IN = 22
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0


def _workload(name):
    import synth
    if name == "c3":
        return synth.config_c3(), "e1024-ion-512w (1024-bead e-, +3 ion, 512 H2O, 24.8 A)"
    if name == "c2":
        return synth.config_c2(), "water256 N_H=32 N_O=4 (19.7 A)"
    if name == "c1":
        return synth.config_c1(), "e64-ion-32w (10 A)"
    raise SystemExit(f"unknown workload {name}")


def _run(s, precision, steps, warmup, mixpi, torch):
    sysm = mixpi.System(s, precision=precision)
    idx = sysm.bead_index
    import numpy as np

    def dev(x):
        out = np.empty_like(x)
        out[idx] = x
        return torch.from_numpy(out).cuda()

    q, p = dev(s.q), dev(s.p)
    f, _ = sysm.forces(q)
    elog_w = torch.zeros((max(warmup, 1), 1, mixpi.MIXPI_NE), dtype=torch.float64, device="cuda")
    elog = torch.zeros((steps, 1, mixpi.MIXPI_NE), dtype=torch.float64, device="cuda")
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
    el = elog.cpu().numpy()[:, 0, :]
    ham = el[:, mixpi.E_NAMES.index("ham")]
    return dict(sysm=sysm, q=q, p=p, f=f, ms=ms, ev=(ev_atom, ev_pp), elog=el,
                drift=float(ham[-1] - ham[0]), hstd=float(ham.std()))


def _cpu_baseline(s, target_s=15.0):
    """The FP64 CPU oracle stepping the same system on the host cores."""
    import oracle
    o = oracle.OracleSystem(s)
    F, _ = o.forces(s.q)
    t = time.perf_counter()
    q, p, F, _ = o.step(s.q, s.p, 1, F=F)
    one = time.perf_counter() - t
    n = max(1, min(200, int(target_s / max(one, 1e-6))))
    evals = sum(o.pair_evals(q))
    t = time.perf_counter()
    o.step(q, p, n, F=F)
    dt = time.perf_counter() - t
    return dict(value=evals * n / dt, unit="pair-evals/s", cores=oracle.num_threads(),
                kind="oracle", steps_per_s=n / dt,
                sample=f"{n} FP64 oracle steps of the same system (term-by-term V_mix, "
                       f"OpenMP over particles), after 1 untimed step")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    args = ap.parse_args()
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
    s, wname = _workload(args.workload)

    print(f"[bench] {wname}: FP32 pair form, {args.warmup} warmup + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    r32 = _run(s, mixpi.MIXPI_FP32_ACC64, args.steps, args.warmup, mixpi, torch)
    sysm = r32["sysm"]
    ev_step = (r32["ev"][0] + r32["ev"][1]) / args.steps
    value = (r32["ev"][0] + r32["ev"][1]) / (r32["ms"] * 1e-3)
    steps_per_s = args.steps / (r32["ms"] * 1e-3)

    # dominant kernel (pair sweep) timed with HIP events on the same stream
    print("[bench] kernel timing", file=sys.stderr, flush=True)
    reps = 200
    k_us = {name: sysm.kernel_time(k, reps, r32["q"], r32["p"])
            for name, k in (("pair", 0), ("bonded", 1), ("free_rp", 2), ("finish", 3))}
    cand = sysm.pair_candidates()
    ev_atom, ev_pp = (x / args.steps for x in r32["ev"])
    flops = cand * FLOP_CANDIDATE + ev_atom * FLOP_ATOM_IN + ev_pp * FLOP_PP_IN
    achieved = flops / (k_us["pair"] * 1e-6) / 1e12

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
                   "dt_fs": s.dt, "precision": "fp32 pair potentials, fp64 state and sums"},
        "steps_per_s": steps_per_s,
        "kernel_us": k_us,
        "energy_drift_kcal": r32["drift"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": None, "kernel": "k_pair"},
    }
    if not args.no_fp64:
        print("[bench] FP64 form", file=sys.stderr, flush=True)
        r64 = _run(s, mixpi.MIXPI_FP64, args.steps, args.warmup, mixpi, torch)
        out["fp64"] = {"value": (r64["ev"][0] + r64["ev"][1]) / (r64["ms"] * 1e-3),
                       "steps_per_s": args.steps / (r64["ms"] * 1e-3),
                       "ms_per_step": r64["ms"] / args.steps,
                       "pair_us": r64["sysm"].kernel_time(0, reps, r64["q"], r64["p"])}
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

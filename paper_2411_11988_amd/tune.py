"""Autotuner for the shape of the pair sweep.

The force launch cuts each system's pair blocks into 64 x TJ tiles (TJ = 16,
32 or 64, per system), each run by one wave, two waves splitting its
j-beads, or two or four waves with 64 i-beads each (128 x TJ or 256 x TJ
tiles); every shape gives the same forces to rounding.  ``autotune`` times the force launch and the
epilogue that gathers its partial forces (``mixpi_kernel_time``, inside
eager steps of the actual workload) for
every (TJ, waves) with one TJ for all systems, and then, for a batch whose
systems fall in several size classes, tries each class's other widths with
the rest held; it returns the fastest.
``tile_flags`` returns the descriptor flags (one per system) for a
workload, measuring once per workload bucket and keeping the choice in a
JSON cache.

A size class is (largest ring bead count, atom count rounded to a power of
two); a workload bucket is (device architecture, the built library's
content hash, precision, number of systems, its size classes).  Workloads in
one bucket share the shape of their work lists closely enough to share a
choice, and a rebuilt library (changed kernels) never reuses a stale one.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import mixpi

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mixpi_tiles.json")
TJS = (16, 32, 64)
WAVES = ("w1", "w2", "i2", "i4")


def _pow2_ceil(x: int) -> int:
    return 1 << max(0, int(x - 1).bit_length())


_LIB_HASH = None


def library_hash() -> str:
    """First 16 hex digits of the sha256 of the loaded libmixpi.so."""
    global _LIB_HASH
    if _LIB_HASH is None:
        import hashlib
        h = hashlib.sha256()
        with open(mixpi.LIB_PATH, "rb") as fh:
            for chunk in iter(lambda: fh.read(1 << 20), b""):
                h.update(chunk)
        _LIB_HASH = h.hexdigest()[:16]
    return _LIB_HASH


def _as_list(systems):
    return list(systems) if isinstance(systems, (list, tuple)) else [systems]


def size_class(s) -> str:
    """(largest bead count, atom count rounded up to a power of two)."""
    atoms = int(np.sum(np.asarray(s.is_electron) == 0))
    return f"N{int(np.max(s.n_beads))}A{_pow2_ceil(atoms)}"


def bucket(systems, precision: int) -> str:
    import torch
    systems = _as_list(systems)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    classes = ",".join(sorted(set(size_class(s) for s in systems)))
    return f"{arch}|lib{library_hash()}|p{precision}|s{len(systems)}|{classes}"


def _state(sysm, systems):
    import torch
    idx = sysm.bead_index
    q = np.concatenate([s.q for s in systems])
    p = np.concatenate([s.p for s in systems])
    qr, pr = np.empty_like(q), np.empty_like(p)
    qr[idx], pr[idx] = q, p
    return torch.from_numpy(qr).cuda(), torch.from_numpy(pr).cuda()


def _flags(systems, tj_of, waves):
    return [mixpi.TJ_FLAGS[tj_of[size_class(s)]] | mixpi.WAVES_FLAGS[waves] for s in systems]


def _time(systems, precision, flags, reps, parts=False):
    """In-step microseconds of the launches the shape changes: the force
    launch and the epilogue, which gathers the force launch's partial-force
    slots (their sum; both with parts=True)."""
    sysm = mixpi.System(systems if len(systems) > 1 else systems[0], precision=precision,
                        flags=flags if len(systems) > 1 else flags[0])
    q, p = _state(sysm, systems)
    f, _ = sysm.forces(q)
    sysm.kernel_time(4, q, p, f)                    # warm-up
    kt = sysm.kernel_time(reps, q, p, f)
    sysm.close()
    if parts:
        return kt["force"], kt["finish"]
    return kt["force"] + kt["finish"]


def autotune(systems, precision: int = mixpi.MIXPI_FP32_ACC64, reps: int = 32,
             tjs=TJS, waves=WAVES):
    """Times the in-step force launch plus epilogue over the shapes; returns
    (choice, {label: microseconds}) with choice = {"waves": w, "tj": {class: TJ}}."""
    systems = _as_list(systems)
    classes = sorted(set(size_class(s) for s in systems))
    times = {}
    best, best_t = None, float("inf")
    for tj in tjs:
        for w in waves:
            tj_of = {c: tj for c in classes}
            t = _time(systems, precision, _flags(systems, tj_of, w), reps)
            times[f"{tj}x{w}"] = t
            if t < best_t:
                best, best_t = {"waves": w, "tj": tj_of}, t
    if len(classes) > 1:
        # one class at a time, the others held at the current choice
        for c in classes:
            for tj in tjs:
                if tj == best["tj"][c]:
                    continue
                tj_of = dict(best["tj"], **{c: tj})
                t = _time(systems, precision, _flags(systems, tj_of, best["waves"]), reps)
                times[f"{c}:{tj}x{best['waves']}"] = t
                if t < best_t:
                    best, best_t = {"waves": best["waves"], "tj": tj_of}, t
    return best, times


def tile_flags(systems, precision: int = mixpi.MIXPI_FP32_ACC64, cache: str | None = None,
               retune: bool = False):
    """Descriptor flags of the fastest shape for this workload's bucket
    (measured on first use, then read from the cache file): an int for one
    system, a list with one value per system for a batch."""
    single = not isinstance(systems, (list, tuple))
    systems = _as_list(systems)
    cache = cache or DEFAULT_CACHE
    key = bucket(systems, precision)
    table = {}
    if os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if retune or key not in table:
        best, times = autotune(systems, precision)
        table[key] = {"waves": best["waves"], "tj": best["tj"], "us": times}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    e = table[key]
    flags = _flags(systems, {c: int(v) for c, v in e["tj"].items()}, e["waves"])
    return flags[0] if single else flags


def describe(flags) -> str:
    """'TJxWAVES' of a flag value (or of each value of a list)."""
    if isinstance(flags, (list, tuple)):
        return ",".join(sorted(set(describe(f) for f in flags)))
    inv = {v: k for k, v in mixpi.TILE_FLAGS.items()}
    return "%dx%s" % inv[flags]

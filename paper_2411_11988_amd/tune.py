"""Autotuner for the tile shape of the pair sweep.

The force launch can run with 32- or 64-wide j-tiles and with one or two
waves per 64-bead i-tile; every shape gives the same forces to rounding.
``autotune`` times the force launch of each shape inside eager steps of the
actual workload (``mixpi_kernel_time``) and returns the fastest;
``tile_flags`` returns the descriptor flags for a workload, measuring once
per shape bucket and keeping the choice in a JSON cache.

A bucket is (device architecture, the built library's content hash,
precision, number of systems, largest ring bead count, total atom count
rounded to a power of two): workloads in one bucket share the shape of their
work lists closely enough to share a tile choice, and a rebuilt library
(changed kernels) never reuses a stale choice.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import mixpi

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mixpi_tiles.json")


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


def bucket(systems, precision: int) -> str:
    import torch
    systems = systems if isinstance(systems, (list, tuple)) else [systems]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    pmax = max(int(np.max(s.n_beads)) for s in systems)
    atoms = sum(int(np.sum(np.asarray(s.is_electron) == 0)) for s in systems)
    return (f"{arch}|lib{library_hash()}|p{precision}|s{len(systems)}|N{pmax}"
            f"|A{_pow2_ceil(atoms)}")


def _state(sysm, systems):
    import torch
    idx = sysm.bead_index
    q = np.concatenate([s.q for s in systems])
    p = np.concatenate([s.p for s in systems])
    qr, pr = np.empty_like(q), np.empty_like(p)
    qr[idx], pr[idx] = q, p
    return torch.from_numpy(qr).cuda(), torch.from_numpy(pr).cuda()


def autotune(systems, precision: int = mixpi.MIXPI_FP32_ACC64, reps: int = 32,
             shapes=((32, 1), (32, 2), (64, 1), (64, 2))):
    """Times the in-step force launch for every tile shape; returns
    (best shape, {shape: microseconds})."""
    systems = systems if isinstance(systems, (list, tuple)) else [systems]
    times = {}
    for shape in shapes:
        sysm = mixpi.System(systems if len(systems) > 1 else systems[0],
                            precision=precision, flags=mixpi.TILE_FLAGS[shape])
        q, p = _state(sysm, systems)
        f, _ = sysm.forces(q)
        sysm.kernel_time(4, q, p, f)                    # warm-up
        times[shape] = sysm.kernel_time(reps, q, p, f)["force"]
        sysm.close()
    best = min(times, key=times.get)
    return best, times


def tile_flags(systems, precision: int = mixpi.MIXPI_FP32_ACC64, cache: str | None = None,
               retune: bool = False) -> int:
    """Descriptor flags of the fastest tile shape for this workload's bucket
    (measured on first use, then read from the cache file)."""
    cache = cache or DEFAULT_CACHE
    key = bucket(systems, precision)
    table = {}
    if os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if retune or key not in table:
        best, times = autotune(systems, precision)
        table[key] = {"tj": best[0], "waves": best[1],
                      "us": {f"{a}x{b}": t for (a, b), t in times.items()}}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    e = table[key]
    return mixpi.TILE_FLAGS[(int(e["tj"]), int(e["waves"]))]

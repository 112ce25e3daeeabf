"""ctypes binding of libmixpi (the C-ABI declared in include/mixpi.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  If the
compiled library is missing the import-time loader raises; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmixpi.so")

MIXPI_OK = 0
MIXPI_E_INVALID = -1
MIXPI_E_NOT_POW2 = -2
MIXPI_E_ORDER = -3
MIXPI_E_HIP = -4
MIXPI_E_NONFINITE = -5
MIXPI_E_UNSUPPORTED = -6

E_NAMES = ["vmix", "lj", "coul", "pp", "bond", "angle",
           "spring", "kin", "kcv", "kprim", "ham"]
MIXPI_NE = len(E_NAMES)
MIXPI_NV = 6
MIXPI_NTHETA = 6
MIXPI_FP64 = 0
MIXPI_FP32_ACC64 = 1
MIXPI_FLAG_CHECK_FINITE = 1
MIXPI_STATIC_SCRATCH_BYTES = 16 << 20
MIXPI_FLAG_TILE_J16 = 1 << 8
MIXPI_FLAG_TILE_J32 = 1 << 4
MIXPI_FLAG_TILE_J64 = 1 << 5
MIXPI_FLAG_TILE_WAVES1 = 1 << 6
MIXPI_FLAG_TILE_WAVES2 = 1 << 7
MIXPI_FLAG_TILE_I128 = 1 << 9
MIXPI_FLAG_TILE_I256 = 1 << 10
TJ_FLAGS = {16: MIXPI_FLAG_TILE_J16, 32: MIXPI_FLAG_TILE_J32, 64: MIXPI_FLAG_TILE_J64}
# waves per tile: "w1" one wave, "w2" two waves splitting the j-beads,
# "i2" / "i4" two / four waves of 64 i-beads sharing them
WAVES_FLAGS = {"w1": MIXPI_FLAG_TILE_WAVES1, "w2": MIXPI_FLAG_TILE_WAVES2,
               "i2": MIXPI_FLAG_TILE_I128, "i4": MIXPI_FLAG_TILE_I256}
# (j-tile width, waves per tile) -> descriptor flags
TILE_FLAGS = {(tj, w): TJ_FLAGS[tj] | WAVES_FLAGS[w] for tj in TJ_FLAGS for w in WAVES_FLAGS}


class MixPIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mixpi error {code}: {msg}")
        self.code = code


class mixpi_system_desc(C.Structure):
    _fields_ = [
        ("n_particles", C.c_int32),
        ("n_beads", C.c_void_p),
        ("mass", C.c_void_p), ("fict_mass", C.c_void_p), ("charge", C.c_void_p),
        ("lj_type", C.c_void_p), ("mol_id", C.c_void_p), ("is_electron", C.c_void_p),
        ("n_lj_types", C.c_int32), ("lj_eps", C.c_void_p), ("lj_sigma", C.c_void_p),
        ("n_bonds", C.c_int32), ("bonds", C.c_void_p), ("bond_type", C.c_void_p),
        ("n_bond_types", C.c_int32), ("bond_k", C.c_void_p), ("bond_r0", C.c_void_p),
        ("n_angles", C.c_int32), ("angles", C.c_void_p), ("angle_type", C.c_void_p),
        ("n_angle_types", C.c_int32), ("angle_k", C.c_void_p), ("angle_t0", C.c_void_p),
        ("pp_q", C.c_double), ("pp_a", C.c_double), ("rc_pp", C.c_double),
        ("rc_coul", C.c_double), ("rc_lj", C.c_double),
        ("background", C.c_int32),
        ("box", C.c_double * 3),
        ("temperature", C.c_double), ("dt", C.c_double),
        ("precision", C.c_int32), ("flags", C.c_int32),
    ]


_lib = None


def load():
    """Load libmixpi.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds the process to torch's HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2411_11988_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "mixpi_last_error": ([], C.c_char_p),
        "mixpi_create": ([P, P], C.c_int),
        "mixpi_batch_create": ([P, I32, P], C.c_int),
        "mixpi_destroy": ([P], C.c_int),
        "mixpi_sizes": ([P, P, P, P, P], C.c_int),
        "mixpi_bead_index": ([P, P], C.c_int),
        "mixpi_layout": ([P, P, P], C.c_int),
        "mixpi_forces": ([P, P, P, P, P, P], C.c_int),
        "mixpi_forces_static": ([P, P, P, P, P, P], C.c_int),
        "mixpi_energy": ([P, P, P, P, P], C.c_int),
        "mixpi_energy_adjoint": ([P, P, P, P, P, P, P], C.c_int),
        "mixpi_nm_transform": ([P, I32, P, P, P], C.c_int),
        "mixpi_step": ([P, I32, P, P, P, P, P], C.c_int),
        "mixpi_batch_step": ([P, I32, P, P, P, P, P], C.c_int),
        "mixpi_pair_candidates": ([P, P], C.c_int),
        "mixpi_pair_shape": ([P, P, P, P, P], C.c_int),
        "mixpi_pair_evals": ([P, P, I32, P], C.c_int),
        "mixpi_step_prepare": ([P, I32, P, P, P, P], C.c_int),
        "mixpi_kernel_time": ([P, I32, P, P, P, P, P], C.c_int),
        "mixpi_rdf": ([P, P, C.c_double, I32, I32, P, P], C.c_int),
        "mixpi_vacf_sample": ([P, P, C.c_int64, I32, I32, P, P, P], C.c_int),
        "mixpi_set_ewald": ([P, C.c_double, C.c_double, I32, I32], C.c_int),
        "mixpi_ewald": ([P, P, P, P, P], C.c_int),
        "mixpi_use_ewald": ([P, I32], C.c_int),
        "mixpi_set_thermostat": ([P, C.c_double], C.c_int),
        "mixpi_step_nvt": ([P, I32, P, P, P, P, P, P], C.c_int),
        "mixpi_step_vv": ([P, I32, P, P, P, P, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != MIXPI_OK:
        raise MixPIError(rc, load().mixpi_last_error().decode())


def _arr(x, dtype):
    return np.ascontiguousarray(np.asarray(x), dtype=dtype)


def make_desc(s, precision: int = MIXPI_FP64, flags: int = 0):
    """Build a mixpi_system_desc from an object with the system fields
    (n_beads, mass, fict_mass, charge, lj_type, mol_id, is_electron, lj_eps,
    lj_sigma, bonds, bond_type, bond_k, bond_r0, angles, angle_type, angle_k,
    angle_t0, pp_q, pp_a, rc_pp, rc_coul, rc_lj, background, box,
    temperature, dt).  Returns (desc, keepalive)."""
    keep = dict(
        n_beads=_arr(s.n_beads, np.int32), mass=_arr(s.mass, np.float64),
        fict_mass=_arr(s.fict_mass, np.float64), charge=_arr(s.charge, np.float64),
        lj_type=_arr(s.lj_type, np.int32), mol_id=_arr(s.mol_id, np.int32),
        is_electron=_arr(s.is_electron, np.int32),
        lj_eps=_arr(s.lj_eps, np.float64).reshape(-1),
        lj_sigma=_arr(s.lj_sigma, np.float64).reshape(-1),
        bonds=_arr(s.bonds, np.int32).reshape(-1), bond_type=_arr(s.bond_type, np.int32),
        bond_k=_arr(s.bond_k, np.float64), bond_r0=_arr(s.bond_r0, np.float64),
        angles=_arr(s.angles, np.int32).reshape(-1), angle_type=_arr(s.angle_type, np.int32),
        angle_k=_arr(s.angle_k, np.float64), angle_t0=_arr(s.angle_t0, np.float64),
    )
    d = mixpi_system_desc()
    d.n_particles = len(keep["n_beads"])
    for k in ("n_beads", "mass", "fict_mass", "charge", "lj_type", "mol_id", "is_electron",
              "lj_eps", "lj_sigma", "bonds", "bond_type", "bond_k", "bond_r0", "angles",
              "angle_type", "angle_k", "angle_t0"):
        setattr(d, k, keep[k].ctypes.data if keep[k].size else None)
    d.n_lj_types = int(round(np.sqrt(keep["lj_eps"].size)))
    d.n_bonds = keep["bonds"].size // 2
    d.n_bond_types = keep["bond_k"].size
    d.n_angles = keep["angles"].size // 3
    d.n_angle_types = keep["angle_k"].size
    d.pp_q, d.pp_a = float(s.pp_q), float(s.pp_a)
    d.rc_pp, d.rc_coul, d.rc_lj = float(s.rc_pp), float(s.rc_coul), float(s.rc_lj)
    d.background = int(bool(s.background))
    for k in range(3):
        d.box[k] = float(np.asarray(s.box).reshape(-1)[k])
    d.temperature, d.dt = float(s.temperature), float(s.dt)
    d.precision, d.flags = int(precision), int(flags)
    return d, keep


# ---- the C entry points, same names, raw handles ---------------------------

def mixpi_create(desc) -> C.c_void_p:
    h = C.c_void_p()
    _check(load().mixpi_create(C.byref(desc), C.byref(h)))
    return h


def mixpi_batch_create(descs) -> C.c_void_p:
    arr = (C.c_void_p * len(descs))(*[C.addressof(d) for d in descs])
    h = C.c_void_p()
    _check(load().mixpi_batch_create(arr, len(descs), C.byref(h)))
    return h


def mixpi_destroy(h) -> None:
    _check(load().mixpi_destroy(h))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def mixpi_forces(h, q, theta, f, e_out, stream=None) -> None:
    _check(load().mixpi_forces(h, _ptr(q), _ptr(theta), _ptr(f), _ptr(e_out), _stream(stream)))


def mixpi_forces_static(h, q, theta, f, e_out, stream=None) -> None:
    _check(load().mixpi_forces_static(h, _ptr(q), _ptr(theta), _ptr(f), _ptr(e_out),
                                      _stream(stream)))


def mixpi_energy(h, q, theta, e_out, stream=None) -> None:
    _check(load().mixpi_energy(h, _ptr(q), _ptr(theta), _ptr(e_out), _stream(stream)))


def mixpi_energy_adjoint(h, q, theta, grad_e, dq, dtheta, stream=None) -> None:
    _check(load().mixpi_energy_adjoint(h, _ptr(q), _ptr(theta), _ptr(grad_e), _ptr(dq),
                                       _ptr(dtheta), _stream(stream)))


def mixpi_nm_transform(h, direction: int, x_in, x_out, stream=None) -> None:
    _check(load().mixpi_nm_transform(h, int(direction), _ptr(x_in), _ptr(x_out), _stream(stream)))


def mixpi_step(h, nsteps: int, q, p, f, elog, stream=None) -> None:
    _check(load().mixpi_step(h, int(nsteps), _ptr(q), _ptr(p), _ptr(f), _ptr(elog),
                             _stream(stream)))


def mixpi_batch_step(h, nsteps: int, qs, ps, fs, elog, stream=None) -> None:
    """qs, ps, fs: one device array per system (its own rows)."""
    n = len(qs)
    if len(ps) != n or len(fs) != n:
        raise ValueError("qs, ps and fs need one array per system")
    arr = [(C.c_void_p * n)(*[x.data_ptr() for x in xs]) for xs in (qs, ps, fs)]
    _check(load().mixpi_batch_step(h, int(nsteps), arr[0], arr[1], arr[2], _ptr(elog),
                                   _stream(stream)))


def mixpi_layout(h) -> np.ndarray:
    """int64 [n_groups][5]: (first row, N, n, first particle, system) per group."""
    ng = C.c_int32()
    _check(load().mixpi_layout(h, None, C.byref(ng)))
    out = np.zeros((ng.value, 5), dtype=np.int64)
    _check(load().mixpi_layout(h, out.ctypes.data, C.byref(ng)))
    return out


def mixpi_pair_shape(h, n_systems: int) -> tuple:
    """(j-tile width per system, j-split waves, i-split waves, j-run)."""
    tj = (C.c_int32 * n_systems)()
    w, iw, jr = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().mixpi_pair_shape(h, tj, C.byref(w), C.byref(iw), C.byref(jr)))
    return list(tj), w.value, iw.value, jr.value


def mixpi_pair_candidates(h) -> int:
    v = C.c_int64()
    _check(load().mixpi_pair_candidates(h, C.byref(v)))
    return v.value


def mixpi_pair_evals(h, reset: bool = False, stream=None):
    """Returns (atom-atom, electron-atom) in-cutoff slice-pair evaluations."""
    v = (C.c_int64 * 2)()
    _check(load().mixpi_pair_evals(h, v, int(bool(reset)), _stream(stream)))
    return int(v[0]), int(v[1])


def mixpi_step_prepare(h, nsteps: int, q, p, f, elog) -> None:
    _check(load().mixpi_step_prepare(h, int(nsteps), _ptr(q), _ptr(p), _ptr(f), _ptr(elog)))


KERNEL_PAIR, KERNEL_BONDED, KERNEL_RP, KERNEL_FINISH = 0, 1, 2, 3


def mixpi_set_thermostat(h, tau0: float):
    _check(load().mixpi_set_thermostat(h, float(tau0)))


def mixpi_step_nvt(h, nsteps: int, q, p, f, noise, elog=None, stream=None):
    _check(load().mixpi_step_nvt(h, int(nsteps), _ptr(q), _ptr(p), _ptr(f), _ptr(noise),
                                 _ptr(elog), _stream(stream)))


def mixpi_step_vv(h, nsteps: int, q, p, f, elog=None, stream=None):
    _check(load().mixpi_step_vv(h, int(nsteps), _ptr(q), _ptr(p), _ptr(f), _ptr(elog),
                                _stream(stream)))


def mixpi_kernel_time(h, reps: int, q, p, f, stream=None) -> dict:
    """Mean in-step durations (us) of the force, free ring-polymer and
    epilogue launches over `reps` eager steps on library copies of q, p, f."""
    v = (C.c_double * 3)()
    _check(load().mixpi_kernel_time(h, int(reps), _ptr(q), _ptr(p), _ptr(f), v,
                                    _stream(stream)))
    return {"force": v[0], "free_rp": v[1], "finish": v[2]}


def mixpi_rdf(h, q, r_max: float, nbins: int, nspec: int, hist, stream=None):
    _check(load().mixpi_rdf(h, _ptr(q), float(r_max), int(nbins), int(nspec), _ptr(hist),
                            _stream(stream)))


def mixpi_vacf_sample(h, p, t: int, L: int, nspec: int, ring, acc, stream=None):
    _check(load().mixpi_vacf_sample(h, _ptr(p), int(t), int(L), int(nspec), _ptr(ring), _ptr(acc),
                                    _stream(stream)))


def mixpi_set_ewald(h, alpha: float, r_cut: float, grid: int, order: int):
    _check(load().mixpi_set_ewald(h, float(alpha), float(r_cut), int(grid), int(order)))


def mixpi_use_ewald(h, on: bool):
    _check(load().mixpi_use_ewald(h, int(bool(on))))


def mixpi_ewald(h, q, f, e_out, stream=None):
    _check(load().mixpi_ewald(h, _ptr(q), _ptr(f), _ptr(e_out), _stream(stream)))


# ---- convenience object ------------------------------------------------------

class System:
    """Owns a library handle for one system or a batch of systems."""

    def __init__(self, systems, precision: int = MIXPI_FP64, flags=0):
        """flags: one value for every system, or a list with one per system
        (the systems of a batch may differ in their j-tile width flag only)."""
        single = not isinstance(systems, (list, tuple))
        syss = [systems] if single else list(systems)
        fl = list(flags) if isinstance(flags, (list, tuple)) else [flags] * len(syss)
        if len(fl) != len(syss):
            raise ValueError(f"{len(fl)} flag values for {len(syss)} systems")
        pairs = [make_desc(s, precision, f) for s, f in zip(syss, fl)]
        self._keep = pairs
        if single:
            self.h = mixpi_create(pairs[0][0])
        else:
            self.h = mixpi_batch_create([p[0] for p in pairs])
        rows, npart, ngroups, nsys = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().mixpi_sizes(self.h, C.byref(rows), C.byref(npart), C.byref(ngroups),
                                  C.byref(nsys)))
        self.rows, self.n_particles = rows.value, npart.value
        self.n_groups, self.n_systems = ngroups.value, nsys.value
        idx = np.zeros(self.rows, dtype=np.int64)
        _check(load().mixpi_bead_index(self.h, idx.ctypes.data))
        self.bead_index = idx

    def close(self):
        if getattr(self, "h", None):
            mixpi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # layout marshalling (host side, numpy): particle-major bead table <-> rows
    def to_layout(self, x_beads: np.ndarray) -> np.ndarray:
        out = np.empty_like(x_beads)
        out[self.bead_index] = x_beads
        return out

    def from_layout(self, x_rows: np.ndarray) -> np.ndarray:
        return x_rows[self.bead_index]

    def forces(self, q, theta=None, f=None, e_out=None, stream=None):
        import torch
        if f is None:
            f = torch.empty_like(q)
        if e_out is None:
            e_out = torch.empty((self.n_systems, MIXPI_NV), dtype=torch.float64, device=q.device)
        mixpi_forces(self.h, q, theta, f, e_out, stream)
        return f, e_out

    def forces_static(self, q, f, e_out, theta=None, stream=None):
        """mixpi_forces_static: into caller buffers, allocating nothing."""
        mixpi_forces_static(self.h, q, theta, f, e_out, stream)
        return f, e_out

    def energy(self, q, theta=None, e_out=None, stream=None):
        import torch
        if e_out is None:
            e_out = torch.empty((self.n_systems, MIXPI_NV), dtype=torch.float64, device=q.device)
        mixpi_energy(self.h, q, theta, e_out, stream)
        return e_out

    def energy_adjoint(self, q, theta=None, grad_e=None, dq=None, dtheta=None, stream=None):
        import torch
        if dq is None:
            dq = torch.empty_like(q)
        if dtheta is None:
            dtheta = torch.empty((self.n_systems, MIXPI_NTHETA), dtype=torch.float64,
                                 device=q.device)
        mixpi_energy_adjoint(self.h, q, theta, grad_e, dq, dtheta, stream)
        return dq, dtheta

    def nm_transform(self, x, direction: int, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(x)
        mixpi_nm_transform(self.h, direction, x, out, stream)
        return out

    def step(self, nsteps: int, q, p, f, elog=None, stream=None):
        mixpi_step(self.h, nsteps, q, p, f, elog, stream)

    def batch_step(self, nsteps: int, qs, ps, fs, elog=None, stream=None):
        """mixpi_batch_step: one device array per system for q, p and f."""
        mixpi_batch_step(self.h, nsteps, qs, ps, fs, elog, stream)

    def layout(self) -> np.ndarray:
        return mixpi_layout(self.h)
        return elog

    def pair_candidates(self) -> int:
        return mixpi_pair_candidates(self.h)

    def pair_shape(self):
        """(j-tile width per system, j-split waves, i-split waves, j-run)."""
        return mixpi_pair_shape(self.h, self.n_systems)

    def pair_evals(self, reset: bool = False, stream=None):
        return mixpi_pair_evals(self.h, reset, stream)

    def step_prepare(self, nsteps: int, q, p, f, elog=None):
        mixpi_step_prepare(self.h, nsteps, q, p, f, elog)

    def set_thermostat(self, tau0: float):
        mixpi_set_thermostat(self.h, tau0)

    def step_nvt(self, nsteps: int, q, p, f, noise, elog=None, stream=None):
        mixpi_step_nvt(self.h, nsteps, q, p, f, noise, elog, stream)
        return elog

    def step_vv(self, nsteps: int, q, p, f, elog=None, stream=None):
        mixpi_step_vv(self.h, nsteps, q, p, f, elog, stream)
        return elog

    def kernel_time(self, reps: int, q, p, f, stream=None) -> dict:
        return mixpi_kernel_time(self.h, reps, q, p, f, stream)

    def set_ewald(self, alpha: float, r_cut: float, grid: int, order: int):
        mixpi_set_ewald(self.h, alpha, r_cut, grid, order)

    def use_ewald(self, on: bool = True):
        mixpi_use_ewald(self.h, on)

    def ewald(self, q, f=None, e_out=None, stream=None):
        """Centroid Ewald energies [systems][3] (real, reciprocal, constant);
        bead forces are added to f when given."""
        if e_out is None:
            import torch
            e_out = torch.zeros((self.n_systems, 3), dtype=torch.float64, device=q.device)
        mixpi_ewald(self.h, q, f, e_out, stream)
        return e_out

    def vacf_sample(self, p, t: int, ring, acc, nspec: int = 9, stream=None):
        """Adds sample t of the centroid velocity correlation sums to acc
        ([systems][nspec][L]); ring ([L][particles][3]) keeps the history."""
        mixpi_vacf_sample(self.h, p, t, ring.shape[0], nspec, ring, acc, stream)
        return acc

    def rdf(self, q, r_max: float, nbins: int, hist=None, nspec: int = 9, stream=None):
        """Adds the bead-averaged slice-pair histogram of q to hist
        ([systems][nspec][nspec][nbins] FP64 on the device; zeros if None)."""
        if hist is None:
            import torch
            hist = torch.zeros((self.n_systems, nspec, nspec, nbins), dtype=torch.float64,
                               device=q.device)
        mixpi_rdf(self.h, q, r_max, nbins, nspec, hist, stream)
        return hist


def energy_function():
    """torch.autograd.Function E = V_mix(q; theta) with the hand-written
    adjoint kernel as its backward (recomputes every term)."""
    import torch

    class MixPIEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, q, theta, system):
            e = system.energy(q, theta)
            ctx.system = system
            ctx.save_for_backward(q, theta)
            return e[:, 0].clone()

        @staticmethod
        def backward(ctx, grad):
            q, theta = ctx.saved_tensors
            g = grad.contiguous().to(torch.float64)
            dq, dth = ctx.system.energy_adjoint(q, theta, grad_e=g)
            return dq, (dth if theta is not None else None), None

    return MixPIEnergy

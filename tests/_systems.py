"""Hand-built small systems for the tests (inputs only, no method arithmetic)."""
import math

import numpy as np

from synth.systems import System


def custom(n_beads, q, charge=None, lj_type=None, mol=None, ele=None,
           eps=None, sig=None, bonds=(), angles=(), bond_k=300.0, bond_r0=1.0,
           angle_k=50.0, angle_t0=math.radians(105.0), box=1e13, rc=1e12,
           pp_q=-1.0, pp_a=0.5, mass=None, fict_mass=None, temperature=300.0,
           dt=0.25, p=None, background=False, name="custom"):
    n = len(n_beads)
    n_beads = np.asarray(n_beads, dtype=np.int32)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    assert q.shape[0] == n_beads.sum()
    mass = np.full(n, 10.0) if mass is None else np.asarray(mass, dtype=np.float64)
    fm = mass / n_beads if fict_mass is None else np.asarray(fict_mass, dtype=np.float64)
    nt = 4
    e = np.zeros((nt, nt)) if eps is None else np.asarray(eps, dtype=np.float64)
    s = np.ones((nt, nt)) if sig is None else np.asarray(sig, dtype=np.float64)
    return System(
        name=name, n_beads=n_beads, mass=mass, fict_mass=fm,
        charge=np.zeros(n) if charge is None else np.asarray(charge, dtype=np.float64),
        lj_type=np.full(n, 3, np.int32) if lj_type is None else np.asarray(lj_type, np.int32),
        mol_id=np.arange(n, dtype=np.int32) if mol is None else np.asarray(mol, np.int32),
        is_electron=np.zeros(n, np.int32) if ele is None else np.asarray(ele, np.int32),
        lj_eps=e, lj_sigma=s,
        bonds=np.asarray(bonds, np.int32).reshape(-1, 2),
        bond_type=np.zeros(len(bonds), np.int32),
        bond_k=np.array([bond_k]), bond_r0=np.array([bond_r0]),
        angles=np.asarray(angles, np.int32).reshape(-1, 3),
        angle_type=np.zeros(len(angles), np.int32),
        angle_k=np.array([angle_k]), angle_t0=np.array([angle_t0]),
        pp_q=pp_q, pp_a=pp_a, rc_pp=rc, rc_coul=rc, rc_lj=rc,
        background=background, box=np.full(3, float(box)),
        temperature=temperature, dt=dt, q=q,
        p=np.zeros_like(q) if p is None else np.asarray(p, dtype=np.float64),
        seed=0)


def lj_table(t1, t2, eps, sig, nt=4):
    e = np.zeros((nt, nt))
    s = np.ones((nt, nt))
    e[t1, t2] = e[t2, t1] = eps
    s[t1, t2] = s[t2, t1] = sig
    return e, s

"""Seeded synthetic systems shaped like the paper's two workloads.

Workloads (Sec. "Examples and Discussion"):
  * System I: flexible q-SPC/Fw water with N_H and N_O beads per H and O
    (Table 1 lists 90 waters at (N_H, N_O) = (1,1), (32,1), (32,4), (32,32)).
  * System II: a classical +3 cation with a quantized many-bead electron in
    water (Table 2: 1024-bead electron, 91 waters).

The benchmark shapes scale these to larger boxes at liquid density.  Every
value here is an input: the generator draws coordinates and momenta with
``numpy.random.default_rng(seed)`` in a fixed, documented order and never
evaluates a force, an energy or a normal mode.

Units: Angstrom, fs, amu, kcal/mol, elementary charge, K.

Force-field constants (q-SPC/Fw-like charges and flexible bonds, the cation
Lennard-Jones parameters of System II) are synthetic inputs; the method's
results do not depend on their particular values.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# --- physical constants (SI / CODATA 2022; generator's own copy) -----------
_AMU_KG = 1.66053906892e-27
_HBAR_SI = 6.62607015e-34 / (2.0 * math.pi)
_KB_SI = 1.380649e-23
_NA = 6.02214076e23
_AMU_A2_FS2_J = _AMU_KG * 1e-20 / 1e-30          # 1 amu A^2 fs^-2 in J
HBAR = _HBAR_SI / (_AMU_KG * 1e-20 / 1e-15)       # amu A^2 / fs
KB = _KB_SI / _AMU_A2_FS2_J                        # amu A^2 fs^-2 / K

# --- synthetic force-field values -------------------------------------------
M_O = 15.9994
M_H = 1.00794
M_ION = 58.933194
M_E = 5.48579909065e-4
Q_O = -0.84
Q_H = 0.42
Q_ION = 3.0
Q_E = -1.0
BOND_K = 1059.162      # kcal/mol/A^2, V = k/2 (r-r0)^2
BOND_R0 = 1.0          # A
ANGLE_K = 75.90        # kcal/mol/rad^2, V = k/2 (t-t0)^2
ANGLE_T0 = math.radians(112.0)
EPS_OO = 0.1554        # kcal/mol
SIG_OO = 3.1655        # A
# cation-oxygen LJ of System II: sigma 4.134 A, epsilon 666.77 K (x k_B)
EPS_ION_O = 666.77 * _KB_SI * _NA / 4184.0
SIG_ION_O = 4.134
PP_A = 0.5             # softening length of the electron pseudopotential, A

# LJ type indices
T_O, T_ION, T_H, T_NONE = 0, 1, 2, 3
N_LJ_TYPES = 4


@dataclass
class System:
    """One mixTS-PIMD system: particles, topology, parameters, state.

    Bead coordinates are held in a particle-major bead table: the beads of
    particle i are rows ``bead_offset[i] : bead_offset[i+1]`` of ``q``/``p``.
    Positions are unwrapped (rings and molecules are never split across the
    periodic boundary); distances use the nearest image.
    """
    name: str
    n_beads: np.ndarray            # int32 [n]
    mass: np.ndarray               # float64 [n] physical mass (amu)
    fict_mass: np.ndarray          # float64 [n] fictitious bead mass (amu)
    charge: np.ndarray             # float64 [n] (e)
    lj_type: np.ndarray            # int32 [n]
    mol_id: np.ndarray             # int32 [n]
    is_electron: np.ndarray        # int32 [n]
    lj_eps: np.ndarray             # float64 [nt, nt]
    lj_sigma: np.ndarray           # float64 [nt, nt]
    bonds: np.ndarray              # int32 [nb, 2]
    bond_type: np.ndarray          # int32 [nb]
    bond_k: np.ndarray             # float64 [nbt]
    bond_r0: np.ndarray            # float64 [nbt]
    angles: np.ndarray             # int32 [na, 3] (vertex in the middle)
    angle_type: np.ndarray         # int32 [na]
    angle_k: np.ndarray            # float64 [nat]
    angle_t0: np.ndarray           # float64 [nat] (rad)
    pp_q: float                    # pseudopotential charge of the electron (e)
    pp_a: float                    # softening length (A)
    rc_pp: float                   # electron-atom cutoff (A)
    rc_coul: float                 # atom-atom Coulomb cutoff (A)
    rc_lj: float                   # atom-atom LJ cutoff (A)
    background: bool               # neutralising uniform background energy
    box: np.ndarray                # float64 [3] (A)
    temperature: float             # K
    dt: float                      # fs
    q: np.ndarray                  # float64 [B, 3] bead positions
    p: np.ndarray                  # float64 [B, 3] bead momenta (amu A/fs)
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.n_beads.shape[0])

    @property
    def bead_offset(self) -> np.ndarray:
        off = np.zeros(self.n_particles + 1, dtype=np.int64)
        np.cumsum(self.n_beads, out=off[1:])
        return off

    @property
    def total_beads(self) -> int:
        return int(self.n_beads.sum())

    def beads(self, i: int) -> np.ndarray:
        off = self.bead_offset
        return self.q[off[i]:off[i + 1]]


def water_bead_total(n_waters: int, n_h: int, n_o: int) -> int:
    """Bead count of a water box with N_H beads per H and N_O per O."""
    return n_waters * (2 * n_h + n_o)


# --- sampling helpers ---------------------------------------------------------

def _random_rotation(rng) -> np.ndarray:
    """Uniform random rotation matrix from a uniform unit quaternion."""
    u1, u2, u3 = rng.random(3)
    a = math.sqrt(1 - u1) * math.sin(2 * math.pi * u2)
    b = math.sqrt(1 - u1) * math.cos(2 * math.pi * u2)
    c = math.sqrt(u1) * math.sin(2 * math.pi * u3)
    d = math.sqrt(u1) * math.cos(2 * math.pi * u3)
    w, x, y, z = d, a, b, c
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _water_geometry() -> np.ndarray:
    """Rigid water (O, H1, H2) at the reference bond length and angle."""
    h = 0.5 * ANGLE_T0
    return np.array([
        [0.0, 0.0, 0.0],
        [BOND_R0 * math.sin(h), BOND_R0 * math.cos(h), 0.0],
        [-BOND_R0 * math.sin(h), BOND_R0 * math.cos(h), 0.0],
    ])


def _min_image_dist(a: np.ndarray, b: np.ndarray, box: np.ndarray) -> np.ndarray:
    d = a[None, :] - b
    d -= box * np.rint(d / box)
    return np.sqrt((d * d).sum(axis=1))


def _rotations(u: np.ndarray) -> np.ndarray:
    """Rotation matrices [K, 3, 3] from uniform unit quaternions built from
    u [K, 3] uniform in [0, 1) (the same map as ``_random_rotation``)."""
    u1, u2, u3 = u[:, 0], u[:, 1], u[:, 2]
    x = np.sqrt(1 - u1) * np.sin(2 * np.pi * u2)
    y = np.sqrt(1 - u1) * np.cos(2 * np.pi * u2)
    z = np.sqrt(u1) * np.sin(2 * np.pi * u3)
    w = np.sqrt(u1) * np.cos(2 * np.pi * u3)
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


class _Grid:
    """Cell grid over a cubic periodic box holding at most one point per
    cell (cell diagonal below the smallest allowed point distance)."""

    def __init__(self, box: float, min_sep: float, reach: float):
        self.box = box
        self.n = max(1, int(math.ceil(box / (0.99 * min_sep / math.sqrt(3.0)))))
        self.h = box / self.n
        self.cell = np.full(self.n ** 3, -1, dtype=np.int64)
        self.pos = np.zeros((0, 3))
        r = int(math.ceil(reach / self.h))
        o = np.arange(-r, r + 1)
        off = np.stack(np.meshgrid(o, o, o, indexing="ij"), -1).reshape(-1, 3)
        # keep the cells that can hold a point within `reach` of the centre cell
        gap = np.maximum(np.abs(off) - 1, 0) * self.h
        self.off = off[(gap * gap).sum(-1) <= reach * reach]

    def _flat(self, c):
        c = np.mod(c, self.n)
        return (c[..., 0] * self.n + c[..., 1]) * self.n + c[..., 2]

    def min_dist(self, x: np.ndarray) -> np.ndarray:
        """Nearest-image distance from each x [K, 3] to the closest stored
        point (inf if none is within the grid reach)."""
        if len(self.pos) == 0:
            return np.full(len(x), np.inf)
        c = np.floor(np.mod(x, self.box) / self.h).astype(np.int64)
        idx = self.cell[self._flat(c[:, None, :] + self.off[None])]   # [K, M]
        d = x[:, None, :] - self.pos[np.maximum(idx, 0)]
        d -= self.box * np.rint(d / self.box)
        r = np.sqrt((d * d).sum(-1))
        r[idx < 0] = np.inf
        return r.min(axis=1)

    def add(self, x: np.ndarray):
        c = np.floor(np.mod(x, self.box) / self.h).astype(np.int64)
        f = self._flat(c)
        if np.any(self.cell[f] >= 0):
            raise RuntimeError("grid cell already occupied")
        self.cell[f] = np.arange(len(self.pos), len(self.pos) + len(x))
        self.pos = np.vstack([self.pos, x])


def _place_waters(rng, n_waters: int, box: float, centre_excl: float,
                  min_dist: float = 1.6, min_oo: float = 2.6,
                  ion_pos: np.ndarray | None = None):
    """Rigid waters by random sequential addition with random orientations.

    A candidate is an oxygen position drawn uniformly from the part of the
    box not yet known to be excluded, and a uniform random rotation.  It is
    placed if its oxygen is ``min_oo`` from every placed oxygen, its atoms
    are ``min_dist`` from every placed atom, and its oxygen (hydrogens) keep
    ``centre_excl`` (``centre_excl - 0.6``) from the cation.  Excluded space
    is tracked on a fine cell grid: a cell lying wholly within ``min_oo`` of
    a placed oxygen (or ``centre_excl`` of the cation) can hold no oxygen of
    a later water, so drawing from any superset of the remaining cells gives
    the same distribution of placements as drawing from the whole box.
    """
    geo = _water_geometry()
    boxv = np.full(3, float(box))
    g_o = _Grid(box, min_oo, min_oo)
    g_a = _Grid(box, 0.999, min_dist)
    # free-space cells for oxygen candidates
    nf = max(1, int(math.ceil(box / 0.4)))
    hf = box / nf
    free = np.ones(nf ** 3, dtype=bool)
    half_diag = 0.5 * math.sqrt(3.0) * hf
    ctr = (np.arange(nf) + 0.5) * hf

    def block(x, radius):
        r_in = radius - half_diag
        if r_in <= 0:
            return
        k = int(math.ceil(r_in / hf)) + 1
        c = np.floor(np.mod(x, box) / hf).astype(np.int64)
        o = np.arange(-k, k + 1)
        cells = (c[None, :] + np.stack(np.meshgrid(o, o, o, indexing="ij"), -1).reshape(-1, 3))
        cw = np.mod(cells, nf)
        d = ctr[cw] - np.mod(x, box)[None, :]
        d -= box * np.rint(d / box)
        inside = (d * d).sum(-1) < r_in * r_in
        cw = cw[inside]
        free[(cw[:, 0] * nf + cw[:, 1]) * nf + cw[:, 2]] = False

    if ion_pos is not None:
        block(ion_pos, centre_excl)
    coords = []
    chunk = 16
    cells = np.flatnonzero(free)
    for w in range(n_waters):
        if w % 16 == 0:
            # a stale list is a superset of the free cells: still exact
            cells = np.flatnonzero(free)
        if len(cells) == 0:
            raise RuntimeError("water placement failed; box too dense")
        for attempt in range(2000):
            pick = cells[rng.integers(0, len(cells), chunk)]
            cz, cy, cx = pick % nf, (pick // nf) % nf, pick // (nf * nf)
            base = np.stack([cx, cy, cz], -1) * hf
            centres = base + rng.uniform(0.0, hf, (chunk, 3))
            mols = centres[:, None, :] + np.einsum("aj,kij->kai", geo,
                                                  _rotations(rng.random((chunk, 3))))
            ok = np.ones(chunk, dtype=bool)
            if ion_pos is not None:
                d = mols - ion_pos[None, None, :]
                d -= boxv * np.rint(d / boxv)
                r = np.sqrt((d * d).sum(-1))
                ok &= (r[:, 0] >= centre_excl) & (r[:, 1:].min(axis=1) >= centre_excl - 0.6)
            cand = np.flatnonzero(ok)
            cand = cand[g_o.min_dist(mols[cand, 0]) >= min_oo]
            if len(cand):
                da = g_a.min_dist(mols[cand].reshape(-1, 3)).reshape(len(cand), 3)
                cand = cand[da.min(axis=1) >= min_dist]
            if len(cand):
                mol = mols[cand[0]]
                chunk = int(min(256, max(16, 2 * (cand[0] + 1))))
                break
            chunk = min(256, 2 * chunk)
        else:
            raise RuntimeError("water placement failed; box too dense")
        coords.append(mol)
        g_o.add(mol[:1])
        g_a.add(mol)
        block(mol[0], min_oo)
    return np.array(coords)  # [n_waters, 3 atoms, 3]


def _bridge_ring(rng, n: int, step_var: float) -> np.ndarray:
    """Closed Gaussian path of n beads with centroid zero.

    A Brownian bridge: cumulative Gaussian steps of variance ``step_var`` per
    component, with the end-point drift removed so that the path closes.
    """
    if n == 1:
        return np.zeros((1, 3))
    steps = rng.normal(0.0, math.sqrt(step_var), size=(n, 3))
    walk = np.cumsum(steps, axis=0)
    walk = np.vstack([np.zeros((1, 3)), walk[:-1]])
    end = walk[-1] + steps[-1]
    frac = (np.arange(n) / n)[:, None]
    ring = walk - frac * end[None, :]
    return ring - ring.mean(axis=0, keepdims=True)


def _momenta(rng, fict_mass_per_bead: np.ndarray, temperature: float) -> np.ndarray:
    """Maxwell-Boltzmann momenta N(0, m_f k_B T), total momentum removed."""
    sd = np.sqrt(fict_mass_per_bead * KB * temperature)
    p = rng.normal(size=(len(sd), 3)) * sd[:, None]
    ptot = p.sum(axis=0)
    p -= fict_mass_per_bead[:, None] * (ptot / fict_mass_per_bead.sum())[None, :]
    return p


def _lj_tables():
    eps = np.zeros((N_LJ_TYPES, N_LJ_TYPES))
    sig = np.ones((N_LJ_TYPES, N_LJ_TYPES))
    eps[T_O, T_O] = EPS_OO
    sig[T_O, T_O] = SIG_OO
    eps[T_ION, T_O] = eps[T_O, T_ION] = EPS_ION_O
    sig[T_ION, T_O] = sig[T_O, T_ION] = SIG_ION_O
    return eps, sig


def _assemble(name, parts, bonds, angles, box, temperature, dt, rc_pp,
              rc_coul, rc_lj, background, rng, seed, elec_sigma=1.0,
              meta=None) -> System:
    """Sort particles by descending bead count, draw beads and momenta.

    ``parts``: list of dicts with keys n, mass, fm, charge, lj, mol, ele, pos.
    Draw order after sorting: per particle in sorted order its bead ring
    (electron: iid Gaussian cloud; nucleus: closed Brownian path), then all
    momenta at once.
    """
    order = sorted(range(len(parts)), key=lambda i: (-parts[i]["n"], i))
    inv = np.empty(len(parts), dtype=np.int64)
    inv[np.array(order)] = np.arange(len(parts))
    P = [parts[i] for i in order]
    n_beads = np.array([x["n"] for x in P], dtype=np.int32)
    mass = np.array([x["mass"] for x in P])
    fm = np.array([x["fm"] for x in P])
    charge = np.array([x["charge"] for x in P])
    ljt = np.array([x["lj"] for x in P], dtype=np.int32)
    mol = np.array([x["mol"] for x in P], dtype=np.int32)
    ele = np.array([x["ele"] for x in P], dtype=np.int32)
    beta = 1.0 / (KB * temperature)
    rows = []
    for x in P:
        n = x["n"]
        if x["ele"]:
            rows.append(x["pos"][None, :] + rng.normal(0.0, elec_sigma, size=(n, 3)))
        else:
            var = beta * HBAR * HBAR / (n * x["mass"])
            rows.append(x["pos"][None, :] + _bridge_ring(rng, n, var))
    q = np.vstack(rows)
    fm_bead = np.repeat(fm, n_beads)
    p = _momenta(rng, fm_bead, temperature)
    b = np.asarray(bonds, dtype=np.int64).reshape(-1, 2)
    a = np.asarray(angles, dtype=np.int64).reshape(-1, 3)
    eps, sig = _lj_tables()
    return System(
        name=name, n_beads=n_beads, mass=mass, fict_mass=fm, charge=charge,
        lj_type=ljt, mol_id=mol, is_electron=ele, lj_eps=eps, lj_sigma=sig,
        bonds=inv[b].astype(np.int32) if len(b) else np.zeros((0, 2), np.int32),
        bond_type=np.zeros(len(b), np.int32),
        bond_k=np.array([BOND_K]), bond_r0=np.array([BOND_R0]),
        angles=inv[a].astype(np.int32) if len(a) else np.zeros((0, 3), np.int32),
        angle_type=np.zeros(len(a), np.int32),
        angle_k=np.array([ANGLE_K]), angle_t0=np.array([ANGLE_T0]),
        pp_q=Q_E, pp_a=PP_A, rc_pp=rc_pp, rc_coul=rc_coul, rc_lj=rc_lj,
        background=background, box=np.full(3, float(box)),
        temperature=float(temperature), dt=float(dt), q=q, p=p, seed=seed,
        meta=dict(meta or {}))


def _water_parts(coords, n_h, n_o, mol0):
    parts, bonds, angles = [], [], []
    for w, mol in enumerate(coords):
        base = len(parts)
        m = mol0 + w
        parts.append(dict(n=n_o, mass=M_O, fm=M_O / n_o, charge=Q_O, lj=T_O,
                          mol=m, ele=0, pos=mol[0]))
        for h in (1, 2):
            parts.append(dict(n=n_h, mass=M_H, fm=M_H / n_h, charge=Q_H, lj=T_H,
                              mol=m, ele=0, pos=mol[h]))
        bonds += [(base, base + 1), (base, base + 2)]
        angles += [(base + 1, base, base + 2)]
    return parts, bonds, angles


def water_box(n_waters: int, box: float, n_h: int, n_o: int, seed: int = 0,
              rc: float = 9.0, temperature: float = 300.0, dt: float = 0.25,
              name: str = "water") -> System:
    """Flexible 3-site water, N_H beads per H and N_O per O (System I shape).

    Fictitious masses m_f = m/N for every nucleus.
    """
    rng = np.random.default_rng(seed)
    coords = _place_waters(rng, n_waters, box, centre_excl=0.0)
    parts, bonds, angles = _water_parts(coords, n_h, n_o, mol0=0)
    return _assemble(name, parts, bonds, angles, box, temperature, dt,
                     rc_pp=rc, rc_coul=rc, rc_lj=rc, background=True, rng=rng,
                     seed=seed, meta=dict(n_waters=n_waters, n_h=n_h, n_o=n_o))


def solvated_electron(n_waters: int, n_e: int, box: float, seed: int = 0,
                      rc_pp: float = 12.0, rc_aa: float = 9.0,
                      temperature: float = 300.0, dt: float = 0.1,
                      n_h: int = 1, n_o: int = 1, with_ion: bool = True,
                      ion_excl: float = 3.4, name: str = "e-ion-water") -> System:
    """A +3 cation at the box centre, an n_e-bead electron and waters.

    The electron's fictitious mass is m_H / n_e (its ring moves like one
    hydrogen); its beads start as an iid Gaussian cloud of sigma 1 A around
    the cation.  The electron interacts with atoms only through the softened
    Coulomb pseudopotential.
    """
    rng = np.random.default_rng(seed)
    centre = np.full(3, 0.5 * box)
    coords = _place_waters(rng, n_waters, box, centre_excl=ion_excl if with_ion else 0.0,
                           ion_pos=centre if with_ion else None)
    parts = [dict(n=n_e, mass=M_E, fm=M_H / n_e, charge=Q_E, lj=T_NONE,
                  mol=0, ele=1, pos=centre.copy())]
    if with_ion:
        parts.append(dict(n=1, mass=M_ION, fm=M_ION, charge=Q_ION, lj=T_ION,
                          mol=1, ele=0, pos=centre.copy()))
    wparts, wb, wa = _water_parts(coords, n_h, n_o, mol0=2)
    off = len(parts)
    parts += wparts
    bonds = [(i + off, j + off) for i, j in wb]
    angles = [(i + off, j + off, k + off) for i, j, k in wa]
    return _assemble(name, parts, bonds, angles, box, temperature, dt,
                     rc_pp=rc_pp, rc_coul=rc_aa, rc_lj=rc_aa, background=True,
                     rng=rng, seed=seed,
                     meta=dict(n_waters=n_waters, n_e=n_e))


def tiny_random(seed: int, n_particles: int = 7, box: float = 7.0,
                bead_choices=(1, 2, 4, 8), with_electron: bool = True,
                rc: float = 3.3, temperature: float = 300.0) -> System:
    """Small random system with mixed bead counts for brute-force checks.

    Random charges, LJ types, bonds and angles that join particles of
    different bead counts, optionally one electron.  Beads spread 0.15 A
    around random centres at least 1.6 A apart.
    """
    rng = np.random.default_rng(seed)
    centres = []
    while len(centres) < n_particles:
        c = rng.uniform(0, box, 3)
        if all(_min_image_dist(c, np.array([x]), np.full(3, box))[0] > 1.6
               for x in centres):
            centres.append(c)
    parts = []
    for i in range(n_particles):
        n = int(rng.choice(bead_choices))
        ele = 1 if (with_electron and i == 0) else 0
        lj = int(rng.integers(0, 3)) if not ele else T_NONE
        mass = M_E if ele else float(rng.uniform(1.0, 16.0))
        parts.append(dict(n=n, mass=mass, fm=(M_H if ele else mass) / n,
                          charge=Q_E if ele else float(rng.uniform(-1, 1)),
                          lj=lj, mol=i, ele=ele, pos=centres[i]))
    atoms = [i for i in range(n_particles) if not parts[i]["ele"]]
    bonds, angles = [], []
    if len(atoms) >= 3:
        a0, a1, a2 = atoms[:3]
        bonds = [(a1, a0), (a1, a2)]
        angles = [(a0, a1, a2)]
        for a in (a0, a1, a2):
            parts[a]["mol"] = 1000  # one molecule: bonded, nonbonded-excluded
    rows = []
    order = sorted(range(n_particles), key=lambda i: (-parts[i]["n"], i))
    inv = np.empty(n_particles, dtype=np.int64)
    inv[np.array(order)] = np.arange(n_particles)
    Ps = [parts[i] for i in order]
    for x in Ps:
        rows.append(x["pos"][None, :] + rng.normal(0, 0.15, size=(x["n"], 3)))
    q = np.vstack(rows)
    n_beads = np.array([x["n"] for x in Ps], dtype=np.int32)
    fm = np.array([x["fm"] for x in Ps])
    p = _momenta(rng, np.repeat(fm, n_beads), temperature)
    eps = np.zeros((N_LJ_TYPES, N_LJ_TYPES))
    sig = np.ones((N_LJ_TYPES, N_LJ_TYPES))
    for t1 in range(3):
        for t2 in range(t1, 3):
            eps[t1, t2] = eps[t2, t1] = float(rng.uniform(0.05, 0.5))
            sig[t1, t2] = sig[t2, t1] = float(rng.uniform(1.5, 2.5))
    b = np.asarray(bonds, dtype=np.int64).reshape(-1, 2)
    a = np.asarray(angles, dtype=np.int64).reshape(-1, 3)
    return System(
        name=f"tiny{seed}", n_beads=n_beads,
        mass=np.array([x["mass"] for x in Ps]), fict_mass=fm,
        charge=np.array([x["charge"] for x in Ps]),
        lj_type=np.array([x["lj"] for x in Ps], dtype=np.int32),
        mol_id=np.array([x["mol"] for x in Ps], dtype=np.int32),
        is_electron=np.array([x["ele"] for x in Ps], dtype=np.int32),
        lj_eps=eps, lj_sigma=sig,
        bonds=inv[b].astype(np.int32), bond_type=np.zeros(len(b), np.int32),
        bond_k=np.array([float(rng.uniform(200, 600))]),
        bond_r0=np.array([1.1]),
        angles=inv[a].astype(np.int32), angle_type=np.zeros(len(a), np.int32),
        angle_k=np.array([float(rng.uniform(30, 90))]),
        angle_t0=np.array([math.radians(105.0)]),
        pp_q=Q_E, pp_a=PP_A, rc_pp=rc, rc_coul=rc, rc_lj=rc, background=True,
        box=np.full(3, float(box)), temperature=temperature, dt=0.25,
        q=q, p=p, seed=seed)


# --- benchmark configurations -------------------------------------------------

def config_c1(seed: int = 0, rc: float = 6.0) -> System:
    """Tiny FP64 case: 64-bead electron, +3 ion, 32 waters, 10 A box, 6 A cutoffs."""
    return solvated_electron(32, 64, 10.0, seed=seed, rc_pp=rc, rc_aa=rc,
                             dt=0.25, name="c1-e64-ion-32w")


def config_c2(seed: int = 0) -> System:
    """256 waters in a 19.7 A box, N_H = 32, N_O = 4, 9 A cutoffs."""
    return water_box(256, 19.7, n_h=32, n_o=4, seed=seed, rc=9.0, dt=0.25,
                     name="c2-water256-h32-o4")


def config_c3(seed: int = 0) -> System:
    """1024-bead electron, +3 ion, 512 waters, 24.8 A box, 12/9 A cutoffs."""
    return solvated_electron(512, 1024, 24.8, seed=seed, rc_pp=12.0, rc_aa=9.0,
                             dt=0.1, name="c3-e1024-ion-512w")


def config_c4_states(n: int = 10, small: bool = False):
    """Seeded configurations for gradient checks (water shape, seeds 0..n-1)."""
    if small:
        return [water_box(8, 7.0, n_h=4, n_o=2, seed=s, rc=3.4) for s in range(n)]
    return [config_c2(seed=s) for s in range(n)]


def _c5_system(args):
    i, p, w = args
    box = (float(w) * 29.915) ** (1.0 / 3.0)
    return solvated_electron(int(w), int(p), box, seed=1000 + i, rc_pp=12.0, rc_aa=9.0,
                             dt=0.1, name=f"c5-{i}-e{p}-w{w}")


def config_c5(seed: int = 0, n_systems: int = 64,
              p_choices=(256, 512, 1024, 2048),
              w_choices=(128, 256, 512, 1024), workers: int | None = None):
    """Batch of independent electron/ion/water systems with uneven sizes.

    The (P, N_w) draws use ``default_rng(seed)``; system i is built with seed
    1000 + i.  Boxes at 29.915 A^3 per water (about 1.0 g/cm^3).  With
    ``workers`` > 1 the systems are built in that many child processes
    (each system has its own seed, so the result is the same).
    """
    rng = np.random.default_rng(seed)
    ps = rng.choice(p_choices, size=n_systems)
    ws = rng.choice(w_choices, size=n_systems)
    jobs = [(i, int(ps[i]), int(ws[i])) for i in range(n_systems)]
    if workers and workers > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=workers,
                                    mp_context=mp.get_context("spawn")) as ex:
            return list(ex.map(_c5_system, jobs))
    return [_c5_system(j) for j in jobs]


def build_workers() -> int:
    """Worker processes for building many systems: the host's cores, at
    most 16."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))

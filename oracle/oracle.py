"""Python access to the FP64 CPU oracle (``mixts_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  The C source is
compiled with gcc on first use (or by the package build step) into
``oracle/_build/libmixts_oracle.so``.

Arrays use the oracle's own layout: a particle-major bead table ``[B, 3]``
where the beads of particle i are rows ``off[i]:off[i+1]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mixts_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libmixts_oracle.so")

# energy slot names (same order as the C enum)
E_NAMES = ["vmix", "lj", "coul", "pp", "bond", "angle",
           "spring", "kin", "kcv", "kprim", "ham"]
E_N = len(E_NAMES)
N_POT = 6


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (-O2, OpenMP, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("nb", C.c_void_p), ("off", C.c_void_p),
        ("mass", C.c_void_p), ("fm", C.c_void_p), ("charge", C.c_void_p),
        ("ljt", C.c_void_p), ("mol", C.c_void_p), ("ele", C.c_void_p),
        ("nt", C.c_int), ("eps", C.c_void_p), ("sig", C.c_void_p),
        ("nbond", C.c_int), ("bond", C.c_void_p), ("btype", C.c_void_p),
        ("bk", C.c_void_p), ("br0", C.c_void_p),
        ("nangle", C.c_int), ("angle", C.c_void_p), ("atype", C.c_void_p),
        ("ak", C.c_void_p), ("at0", C.c_void_p),
        ("pp_q", C.c_double), ("pp_a", C.c_double), ("rc_pp", C.c_double),
        ("rc_coul", C.c_double), ("rc_lj", C.c_double),
        ("background", C.c_int),
        ("box", C.c_double * 3),
        ("temperature", C.c_double), ("dt", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.orc_slice_bead.argtypes = [C.c_int, C.c_int, C.c_int]
        _lib.orc_slice_bead.restype = C.c_int
        for name in ("orc_forces_o2", "orc_forces_o1", "orc_classical"):
            getattr(_lib, name).argtypes = [P, P, P, P]
            getattr(_lib, name).restype = None
        _lib.orc_dvdtheta.argtypes = [P, P, P]
        _lib.orc_pair_evals.argtypes = [P, P, P]
        _lib.orc_springs.argtypes = [P, P, P]
        _lib.orc_springs.restype = C.c_double
        _lib.orc_nm_basis.argtypes = [C.c_int, P]
        _lib.orc_nm_lambda.argtypes = [C.c_int, C.c_int]
        _lib.orc_nm_lambda.restype = C.c_double
        _lib.orc_nm_omega.argtypes = [P, C.c_int, C.c_int]
        _lib.orc_nm_omega.restype = C.c_double
        _lib.orc_nm_transform.argtypes = [P, C.c_int, P, P]
        _lib.orc_free_propagate.argtypes = [P, P, P, C.c_double]
        _lib.orc_observables.argtypes = [P, P, P, P, P, P]
        _lib.orc_step.argtypes = [P, C.c_int, P, P, P, P]
        _lib.orc_pile_gamma.argtypes = [P, C.c_int, C.c_int, C.c_double]
        _lib.orc_pile_gamma.restype = C.c_double
        _lib.orc_pile.argtypes = [P, P, P, C.c_double, C.c_double]
        _lib.orc_step_nvt.argtypes = [P, C.c_int, P, P, P, P, C.c_double, P]
        _lib.orc_step_vv.argtypes = [P, C.c_int, P, P, P, P]
        _lib.orc_rdf.argtypes = [P, P, C.c_double, C.c_int, C.c_int, P]
        _lib.orc_ewald.argtypes = [P, P, C.c_double, C.c_double, C.c_int, P, P]
        _lib.orc_beta.argtypes = [P]
        _lib.orc_beta.restype = C.c_double
        _lib.orc_constants.argtypes = [P]
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_num_threads.restype = C.c_int
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def _bspline(n: int, u):
    """Cardinal B-spline M_n(u) (support [0, n]) by the recursion
    M_2(u) = 1 - |u - 1| on [0, 2], M_n(u) = (u M_{n-1}(u) + (n - u)
    M_{n-1}(u - 1)) / (n - 1)."""
    u = np.asarray(u, dtype=np.float64)
    if n == 1:
        return np.where((u >= 0) & (u < 1), 1.0, 0.0)
    if n == 2:
        return np.where((u >= 0) & (u <= 2), 1.0 - np.abs(u - 1.0), 0.0)
    return (u * _bspline(n - 1, u) + (n - u) * _bspline(n - 1, u - 1.0)) / (n - 1)


class OracleSystem:
    """A synth.System bound to the oracle (keeps the parameter arrays alive).

    ``theta`` optionally overrides (q_e, a, eps_00, sigma_00, k_bond0, k_angle0).
    """

    def __init__(self, sysd, theta=None):
        s = sysd
        self.src = s
        self.n = s.n_particles
        self.nb = np.ascontiguousarray(s.n_beads, dtype=np.int32)
        self.off = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(self.nb, out=self.off[1:])
        self.B = int(self.off[-1])
        self.mass = np.ascontiguousarray(s.mass, dtype=np.float64)
        self.fm = np.ascontiguousarray(s.fict_mass, dtype=np.float64)
        self.charge = np.ascontiguousarray(s.charge, dtype=np.float64)
        self.ljt = np.ascontiguousarray(s.lj_type, dtype=np.int32)
        self.mol = np.ascontiguousarray(s.mol_id, dtype=np.int32)
        self.ele = np.ascontiguousarray(s.is_electron, dtype=np.int32)
        self.eps = np.ascontiguousarray(s.lj_eps, dtype=np.float64).copy()
        self.sig = np.ascontiguousarray(s.lj_sigma, dtype=np.float64).copy()
        self.nt = int(self.eps.shape[0])
        self.bond = np.ascontiguousarray(s.bonds, dtype=np.int32).reshape(-1, 2)
        self.btype = np.ascontiguousarray(s.bond_type, dtype=np.int32)
        self.bk = np.ascontiguousarray(s.bond_k, dtype=np.float64).copy()
        self.br0 = np.ascontiguousarray(s.bond_r0, dtype=np.float64)
        self.angle = np.ascontiguousarray(s.angles, dtype=np.int32).reshape(-1, 3)
        self.atype = np.ascontiguousarray(s.angle_type, dtype=np.int32)
        self.ak = np.ascontiguousarray(s.angle_k, dtype=np.float64).copy()
        self.at0 = np.ascontiguousarray(s.angle_t0, dtype=np.float64)
        pp_q, pp_a = float(s.pp_q), float(s.pp_a)
        if theta is not None:
            th = [float(x) for x in theta]
            pp_q, pp_a = th[0], th[1]
            self.eps[0, 0] = th[2]
            self.sig[0, 0] = th[3]
            self.bk[0] = th[4]
            self.ak[0] = th[5]
        self.c = _Sys()
        c = self.c
        c.n = self.n
        c.nb, c.off = _p(self.nb), _p(self.off)
        c.mass, c.fm, c.charge = _p(self.mass), _p(self.fm), _p(self.charge)
        c.ljt, c.mol, c.ele = _p(self.ljt), _p(self.mol), _p(self.ele)
        c.nt, c.eps, c.sig = self.nt, _p(self.eps), _p(self.sig)
        c.nbond, c.bond, c.btype = len(self.bond), _p(self.bond), _p(self.btype)
        c.bk, c.br0 = _p(self.bk), _p(self.br0)
        c.nangle, c.angle, c.atype = len(self.angle), _p(self.angle), _p(self.atype)
        c.ak, c.at0 = _p(self.ak), _p(self.at0)
        c.pp_q, c.pp_a = pp_q, pp_a
        c.rc_pp, c.rc_coul, c.rc_lj = float(s.rc_pp), float(s.rc_coul), float(s.rc_lj)
        c.background = int(bool(s.background))
        for k in range(3):
            c.box[k] = float(s.box[k])
        c.temperature, c.dt = float(s.temperature), float(s.dt)
        self.ptr = C.addressof(c)

    # -- potential and forces --------------------------------------------
    def forces(self, q, method: str = "o2"):
        """Returns (F [B,3], e[6]) of V_mix at bead positions q [B,3]."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == (self.B, 3)
        F = np.zeros((self.B, 3))
        e = np.zeros(N_POT)
        fn = {"o2": lib().orc_forces_o2, "o1": lib().orc_forces_o1}[method]
        fn(self.ptr, _p(q), _p(F), _p(e))
        return F, e

    def classical(self, X):
        """Classical potential of one configuration X [n,3] -> (F [n,3], e[6])."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        F = np.zeros((self.n, 3))
        e = np.zeros(N_POT)
        lib().orc_classical(self.ptr, _p(X), _p(F), _p(e))
        return F, e

    def pair_evals(self, q):
        """(atom-atom, electron-atom) slice-pairs inside a cutoff."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros(2, dtype=np.int64)
        lib().orc_pair_evals(self.ptr, _p(q), _p(out))
        return int(out[0]), int(out[1])

    def dvdtheta(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        g = np.zeros(6)
        lib().orc_dvdtheta(self.ptr, _p(q), _p(g))
        return g

    # -- ring polymer -----------------------------------------------------
    def springs(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        F = np.zeros((self.B, 3))
        e = lib().orc_springs(self.ptr, _p(q), _p(F))
        return e, F

    def nm_transform(self, x, direction: int):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros_like(x)
        lib().orc_nm_transform(self.ptr, int(direction), _p(x), _p(out))
        return out

    def omega(self, i: int, k: int) -> float:
        return lib().orc_nm_omega(self.ptr, i, k)

    def free_propagate(self, q, p, t: float):
        q = np.array(q, dtype=np.float64, copy=True)
        p = np.array(p, dtype=np.float64, copy=True)
        lib().orc_free_propagate(self.ptr, _p(q), _p(p), float(t))
        return q, p

    def observables(self, q, p, F, vpot):
        q = np.ascontiguousarray(q, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.float64)
        vpot = np.ascontiguousarray(vpot, dtype=np.float64)
        e = np.zeros(E_N)
        lib().orc_observables(self.ptr, _p(q), _p(p), _p(F), _p(vpot), _p(e))
        return e

    def step(self, q, p, nsteps: int, F=None):
        """Run nsteps; returns (q, p, F, elog[nsteps, E_N])."""
        q = np.array(q, dtype=np.float64, copy=True)
        p = np.array(p, dtype=np.float64, copy=True)
        if F is None:
            F, _ = self.forces(q)
        F = np.array(F, dtype=np.float64, copy=True)
        elog = np.zeros((nsteps, E_N))
        lib().orc_step(self.ptr, int(nsteps), _p(q), _p(p), _p(F), _p(elog))
        return q, p, F, elog

    def step_vv(self, q, p, nsteps: int, F=None):
        """Velocity Verlet with spring forces; returns (q, p, F, elog)."""
        q = np.array(q, dtype=np.float64, copy=True)
        p = np.array(p, dtype=np.float64, copy=True)
        if F is None:
            F, _ = self.forces(q)
        F = np.array(F, dtype=np.float64, copy=True)
        elog = np.zeros((nsteps, E_N))
        lib().orc_step_vv(self.ptr, int(nsteps), _p(q), _p(p), _p(F), _p(elog))
        return q, p, F, elog

    def rdf(self, q, rmax: float, nbins: int, nspec: int = 9):
        """Bead-averaged slice-pair histogram [nspec][nspec][nbins] (a <= b)."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        h = np.zeros((nspec, nspec, nbins))
        lib().orc_rdf(self.ptr, _p(q), float(rmax), int(nbins), int(nspec), _p(h))
        return h

    def centroids(self, q):
        """Mean bead position of every particle."""
        q = np.asarray(q, dtype=np.float64)
        return np.array([q[self.off[i]:self.off[i + 1]].mean(axis=0) for i in range(self.n)])

    def ewald(self, q, alpha: float, rc: float, kmax: int):
        """Centroid Ewald electrostatics by definition (orc_ewald): bead
        forces and (real, reciprocal, constant) energies in kcal/mol.
        kmax < 0 leaves the reciprocal part out."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        F = np.zeros_like(q)
        e = np.zeros(3)
        lib().orc_ewald(self.ptr, _p(q), float(alpha), float(rc), int(kmax), _p(F), _p(e))
        return F, e

    def spme_recip(self, q, alpha: float, K: int, order: int):
        """Reciprocal part of the centroid Ewald sum by smooth particle-mesh
        Ewald (Essmann et al., J. Chem. Phys. 103, 8577 (1995)), in that
        paper's steps: charges z_i at scaled fractional coordinates
        u = K c / L spread with cardinal B-splines M_n onto a K^3 grid Q;
        E = (k_e / 2) sum_m B(m) C(m) |F(Q)(m)|^2 with the Euler
        exponential spline moduli B and C(m) = exp(-pi^2 m^2 / alpha^2) /
        (pi V m^2) (C(0) = 0); forces from the B-spline derivatives against
        the convolution F^-1[B C F(Q)].  Returns (bead forces, energy)."""
        c = self.centroids(q)
        z = np.where(self.ele != 0, 0.0, self.charge)
        L = np.asarray(self.src.box, dtype=np.float64).reshape(3)
        V = float(np.prod(L))
        ke = constants()["ke"]
        n = int(order)
        u = K * np.mod(c / L, 1.0)
        base = np.floor(u).astype(np.int64)
        w = u - base
        # spline support: grid points base - j, argument w + j, j = 0 .. n-1
        j = np.arange(n)
        M = _bspline(n, w[:, :, None] + j)          # [particles][3][n]
        dM = _bspline(n - 1, w[:, :, None] + j) - _bspline(n - 1, w[:, :, None] + j - 1)
        idx = np.mod(base[:, :, None] - j, K)       # [particles][3][n]
        Q = np.zeros((K, K, K))
        for i in range(self.n):
            if z[i] == 0.0:
                continue
            wgt = z[i] * M[i, 0][:, None, None] * M[i, 1][None, :, None] * M[i, 2][None, None, :]
            Q[np.ix_(idx[i, 0], idx[i, 1], idx[i, 2])] += wgt
        m = np.arange(K)
        mp = np.where(m <= K // 2, m, m - K)
        bmod = np.zeros(K)
        kk = np.arange(n - 1)
        Mk = _bspline(n, kk + 1.0)
        for a in range(K):
            den = np.sum(Mk * np.exp(2j * np.pi * a * kk / K))
            bmod[a] = 1.0 / abs(den) ** 2
        m2 = ((mp[:, None, None] / L[0]) ** 2 + (mp[None, :, None] / L[1]) ** 2 +
              (mp[None, None, :] / L[2]) ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            Cm = np.exp(-np.pi ** 2 * m2 / alpha ** 2) / (np.pi * V * m2)
        Cm[0, 0, 0] = 0.0
        G = bmod[:, None, None] * bmod[None, :, None] * bmod[None, None, :] * Cm
        FQ = np.fft.fftn(Q)
        E = 0.5 * ke * float(np.sum(G * np.abs(FQ) ** 2))
        conv = np.real(np.fft.ifftn(G * FQ)) * K ** 3
        Fc = np.zeros((self.n, 3))
        for i in range(self.n):
            if z[i] == 0.0:
                continue
            cv = conv[np.ix_(idx[i, 0], idx[i, 1], idx[i, 2])]
            gx = np.einsum("abc,a,b,c->", cv, dM[i, 0], M[i, 1], M[i, 2]) * K / L[0]
            gy = np.einsum("abc,a,b,c->", cv, M[i, 0], dM[i, 1], M[i, 2]) * K / L[1]
            gz = np.einsum("abc,a,b,c->", cv, M[i, 0], M[i, 1], dM[i, 2]) * K / L[2]
            Fc[i] = -ke * z[i] * np.array([gx, gy, gz])
        F = np.zeros((self.B, 3))
        for i in range(self.n):
            F[self.off[i]:self.off[i + 1]] = Fc[i] / self.nb[i]
        return F, E

    def centroid_velocity(self, p):
        """Velocity of every ring-polymer centroid, the bead average
        (1/N_i) sum_j p_ij / m_f,i of the bead velocities (the centroid of the
        ring polymer of Eq. (mts-hamiltonian-b)); p is the bead table."""
        p = np.asarray(p, dtype=np.float64)
        v = np.empty((self.n, 3))
        for i in range(self.n):
            v[i] = p[self.off[i]:self.off[i + 1]].sum(axis=0) / (self.nb[i] * self.fm[i])
        return v

    def vacf(self, ps, L: int, nspec: int = 9):
        """RPMD centroid velocity correlation sums from the bead momenta ps[t]
        of an NVE ring-polymer trajectory sampled at t = 0 .. T-1:
        acc[a][tau] = sum over t = tau .. T-1 and particles i of species a
        (LJ type; the null type nt for none) of v_i(t - tau) . v_i(t), for
        tau < L.  Dividing by (T - tau), the particle count and 3 gives the
        Kubo-transformed correlation function of one velocity component."""
        vs = [self.centroid_velocity(p) for p in ps]
        spec = np.where(self.ljt < 0, self.nt, self.ljt)
        acc = np.zeros((nspec, L))
        for t in range(len(vs)):
            for tau in range(min(t + 1, L)):
                d = np.einsum("ij,ij->i", vs[t - tau], vs[t])
                for i in range(self.n):
                    acc[spec[i], tau] += d[i]
        return acc

    def pile_gamma(self, i: int, k: int, tau0: float) -> float:
        return lib().orc_pile_gamma(self.ptr, int(i), int(k), float(tau0))

    def pile(self, p, eta, t: float, tau0: float):
        """One Langevin step of length t of the momenta in normal modes."""
        p = np.array(p, dtype=np.float64, copy=True)
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        lib().orc_pile(self.ptr, _p(p), _p(eta), float(t), float(tau0))
        return p

    def step_nvt(self, q, p, noise, tau0: float, F=None):
        """Thermostatted steps O B A B O; noise [nsteps][2][B][3] standard
        normals (mode-indexed).  Returns (q, p, F, elog[nsteps, E_N])."""
        noise = np.ascontiguousarray(noise, dtype=np.float64)
        nsteps = noise.shape[0]
        assert noise.shape == (nsteps, 2, self.B, 3)
        q = np.array(q, dtype=np.float64, copy=True)
        p = np.array(p, dtype=np.float64, copy=True)
        if F is None:
            F, _ = self.forces(q)
        F = np.array(F, dtype=np.float64, copy=True)
        elog = np.zeros((nsteps, E_N))
        lib().orc_step_nvt(self.ptr, int(nsteps), _p(q), _p(p), _p(F), _p(noise),
                           float(tau0), _p(elog))
        return q, p, F, elog

    def step_extra(self, q, p, nsteps: int, extra, mode: str = "nve", noise=None,
                   tau0: float = float("inf")):
        """The oracle's split-propagator step ("nve"), velocity Verlet ("vv")
        or thermostatted step ("nvt", noise [nsteps][2][B][3]) with an extra
        potential term: extra(q) -> (bead forces, energy) is added to the
        forces and to V_Coul and V_mix of the logged energies.  Composed from
        the oracle's forces, free propagation, springs, PILE and observables
        in the order of orc_step / orc_step_vv / orc_step_nvt.  Returns
        (q, p, F, elog[nsteps, E_N])."""
        q = np.array(q, dtype=np.float64, copy=True)
        p = np.array(p, dtype=np.float64, copy=True)
        dt = float(self.src.dt)
        kick = 0.5 * dt * constants()["kcal"]
        ic, iv = E_NAMES.index("coul"), E_NAMES.index("vmix")

        def force(x):
            F, v = self.forces(x)
            Fe, ee = extra(x)
            v = np.array(v, dtype=np.float64, copy=True)
            v[ic] += ee
            v[iv] += ee
            return F + Fe, v

        F, _ = force(q)
        elog = np.zeros((nsteps, E_N))
        fm = np.repeat(self.fm, self.nb)[:, None]
        for k in range(nsteps):
            if mode == "nvt":
                p = self.pile(p, noise[k, 0], 0.5 * dt, tau0)
            if mode == "vv":
                p = p + kick * (F + self.springs(q)[1])
                q = q + dt * p / fm
                F, v = force(q)
                p = p + kick * (F + self.springs(q)[1])
            else:
                p = p + kick * F
                q, p = self.free_propagate(q, p, dt)
                F, v = force(q)
                p = p + kick * F
            elog[k] = self.observables(q, p, F, v)
            if mode == "nvt":
                p = self.pile(p, noise[k, 1], 0.5 * dt, tau0)
        return q, p, F, elog

    @property
    def beta(self) -> float:
        return lib().orc_beta(self.ptr)


def slice_bead(s: int, np_: int, nmax: int) -> int:
    return lib().orc_slice_bead(int(s), int(np_), int(nmax))


def nm_basis(N: int) -> np.ndarray:
    Cm = np.zeros((N, N))
    lib().orc_nm_basis(int(N), _p(Cm))
    return Cm


def nm_lambda(N: int, k: int) -> float:
    return lib().orc_nm_lambda(int(N), int(k))


def constants() -> dict:
    out = np.zeros(5)
    lib().orc_constants(_p(out))
    return dict(kcal=out[0], hbar=out[1], kb=out[2], ke=out[3], kb_kcal=out[4])


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return lib().orc_num_threads()

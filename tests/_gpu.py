"""Helpers for the GPU parity tests: the documented layout rebuilt
independently of the library, error norms, and device marshalling."""
import numpy as np


def layout_rows(s) -> np.ndarray:
    """Row of every (particle, bead) in the library layout, rebuilt from its
    documented definition: groups are maximal runs of equal bead count and
    electron flag, each stored [N][n][3] bead-major, groups concatenated."""
    nb = np.asarray(s.n_beads)
    ele = np.asarray(s.is_electron)
    first = np.concatenate([[0], np.cumsum(nb)[:-1]])
    rows = np.empty(int(nb.sum()), dtype=np.int64)
    row = 0
    i = 0
    n = len(nb)
    while i < n:
        j = i
        while j < n and nb[j] == nb[i] and ele[j] == ele[i]:
            j += 1
        cnt, N = j - i, int(nb[i])
        for a in range(N):
            for k in range(cnt):
                rows[first[i + k] + a] = row + a * cnt + k
        row += N * cnt
        i = j
    return rows


def to_rows(s, x_beads, rows=None):
    rows = layout_rows(s) if rows is None else rows
    out = np.empty_like(x_beads)
    out[rows] = x_beads
    return out


def from_rows(s, x_rows, rows=None):
    rows = layout_rows(s) if rows is None else rows
    return x_rows[rows]


def force_err(F, Fo):
    """max |F - F_oracle| over bead components / RMS of F_oracle."""
    return float(np.abs(F - Fo).max() / np.sqrt((Fo ** 2).mean()))


def energy_err(e, eo):
    """Largest per-term relative error of an energy row (forces/energy
    calls: the first 6 entries; step logs: all 11).  Each term is measured
    against its own magnitude, or against the potential-energy scale
    S = sum of |V_k| over LJ, Coulomb, pseudopotential, bond and angle if it
    is below 1e-3 S.  The sums and differences of other terms are measured
    against the sum of their parts' magnitudes, the bound per-term accuracy
    of the parts gives them: V_mix against S, the conserved
    H = KE + E_spring + V_mix against |KE| + |E_spring| + S, and the
    primitive estimator KE_prim = 3 sum_i N_i / (2 beta) - E_spring against
    |KE_prim + E_spring| + |E_spring|."""
    e, eo = np.asarray(e, dtype=np.float64), np.asarray(eo, dtype=np.float64)
    n = min(len(e), len(eo))
    e, eo = e[:n], eo[:n]
    big = np.abs(eo[1:6]).sum() if n > 1 else abs(eo[0])
    den = np.where(np.abs(eo) < 1e-3 * big, big, np.abs(eo))
    den[0] = max(big, abs(eo[0]))
    if n > 10:
        den[9] = abs(eo[9] + eo[6]) + abs(eo[6])
        den[10] = abs(eo[7]) + abs(eo[6]) + big
    den = np.where(den == 0, 1.0, den)
    return float((np.abs(e - eo) / den).max())


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()

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
    """Per-term relative error; a term below 1e-3 of the summed magnitude of
    the terms is compared against that sum instead."""
    e, eo = np.asarray(e, dtype=np.float64), np.asarray(eo, dtype=np.float64)
    big = np.abs(eo[1:6]).sum() if eo.size > 1 else abs(eo[0])
    den = np.where(np.abs(eo) < 1e-3 * big, big, np.abs(eo))
    den = np.where(den == 0, 1.0, den)
    return float((np.abs(e - eo) / den).max())


def energy_err_scale(e, eo):
    """Largest error of any energy term relative to the potential-energy
    scale sum_k |V_k| (LJ, Coulomb, pseudopotential, bond, angle): the
    bar of the FP32 form, whose pair arithmetic cannot resolve a net term
    below the rounding of its own cancelling contributions."""
    e, eo = np.asarray(e, dtype=np.float64), np.asarray(eo, dtype=np.float64)
    scale = np.abs(eo[1:6]).sum()
    n = min(len(e), len(eo))
    return float(np.abs(e[:n] - eo[:n]).max() / scale)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()

"""Drift term of Eq. BTE_E in an external field, on window states of a
Gamma-centred grid, and time stepping of the full right-hand side.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The electron's charge is -|e|, so its crystal momentum obeys
hbar dk/dt = -|e| E, and the occupations move with it:

  df_nk/dt |_drift = (|e|/hbar) E . grad_k f_nk .

This is Eq. BTE_E's drift term with e read as the magnitude of the charge (the
reading under which a distribution drifts against the field, as electrons do).
The paper's release solves only E = 0 and does not say how grad_k f is taken;
here it is the central difference along the three reciprocal directions of the
grid, band by band (band index = energy order at each k), and a neighbour that
is not a window state counts as empty (f = 0).  With k = sum_i kappa_i b_i and
a_i . b_j = 2 pi delta_ij,

  E . grad_k f = sum_i (E . a_i / 2 pi) df/dkappa_i ,
  df/dkappa_i ~ (N_i / 2) [f(kappa + e_i/N_i) - f(kappa - e_i/N_i)] .
"""
from __future__ import annotations

import numpy as np

from .grid import grid_coords, grid_index
from .units import HBAR_EV_FS, TWO_PI


def neighbours(k_idx, band, n_grid):
    """[S][3][2] state index of the +1 and -1 neighbour along reduced
    direction i (same band, periodic grid), or -1 if that state is not in the
    list."""
    n = np.asarray(n_grid, dtype=np.int64)
    where = {(int(k), int(b)): s for s, (k, b) in enumerate(zip(k_idx, band))}
    out = np.full((len(k_idx), 3, 2), -1, dtype=np.int64)
    for s, (k, b) in enumerate(zip(k_idx, band)):
        c = grid_coords(int(k), n)
        for i in range(3):
            for j, step in enumerate((1, -1)):
                d = np.zeros(3, dtype=np.int64)
                d[i] = step
                out[s, i, j] = where.get((int(grid_index((c + d) % n, n)), int(b)), -1)
    return out


def drift(f, nbr, lattice, n_grid, efield):
    """(|e|/hbar) E . grad_k f (1/fs) at every state; E in V/Angstrom."""
    f = np.asarray(f, dtype=np.float64)
    a = np.asarray(lattice, dtype=np.float64)
    n = np.asarray(n_grid, dtype=np.float64)
    E = np.asarray(efield, dtype=np.float64)
    fx = np.concatenate([f, [0.0]])          # index -1 reads the empty state
    out = np.zeros_like(f)
    for i in range(3):
        dfdk = 0.5 * n[i] * (fx[nbr[:, i, 0]] - fx[nbr[:, i, 1]])
        out += (E @ a[i]) / TWO_PI * dfdk
    return out / HBAR_EV_FS

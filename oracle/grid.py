"""Gamma-centred Monkhorst-Pack grids, energy-window states and (k,q) pairs
(paper Sec. 4.3 "Brillouin zone sampling and integration").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid point (i1,i2,i3), 0 <= i_d < N_d, has reduced coordinates i_d/N_d and
linear index (i1*N2 + i2)*N3 + i3.  A pair (s,t) of states on the grid is
connected by the phonon wavevector q = k_t - k_s, itself a point of the same
grid (commensurate k and q grids with q grid = k grid).
"""
from __future__ import annotations

import numpy as np


def _n3(n):
    return tuple(int(x) for x in np.broadcast_to(np.asarray(n), (3,)))


def grid_coords(idx, n):
    n1, n2, n3 = _n3(n)
    idx = np.asarray(idx, dtype=np.int64)
    return np.stack([idx // (n2 * n3), (idx // n3) % n2, idx % n3], axis=-1)


def grid_index(c, n):
    n1, n2, n3 = _n3(n)
    c = np.asarray(c, dtype=np.int64)
    return (c[..., 0] * n2 + c[..., 1]) * n3 + c[..., 2]


def grid_points(n):
    """Reduced coordinates of every grid point, in linear-index order."""
    n3 = _n3(n)
    c = grid_coords(np.arange(n3[0] * n3[1] * n3[2]), n3)
    return c / np.asarray(n3, dtype=np.float64)


def pair_q_index(k_s, k_t, n):
    """Grid index of q = k_t - k_s (mod the grid) for state k-indices k_s, k_t."""
    n3 = np.asarray(_n3(n))
    return grid_index((grid_coords(k_t, n) - grid_coords(k_s, n)) % n3, n)


def minus_q_index(iq, n):
    n3 = np.asarray(_n3(n))
    return grid_index((-grid_coords(iq, n)) % n3, n)


def snap_edge(energies_sorted, edge):
    """Move a window edge to the midpoint between the two sorted energies that
    straddle it (a reading that makes window membership robust to rounding;
    the paper only says the window is user-defined)."""
    e = np.asarray(energies_sorted)
    i = int(np.searchsorted(e, edge, side="left"))
    if i == 0:
        return e[0] - 1.0 if len(e) else edge
    if i == len(e):
        return e[-1] + 1.0
    return 0.5 * (e[i - 1] + e[i])


def window_states(eps_grid, band_lo, band_hi, e_lo, e_hi):
    """States (k-index, band) with band_lo <= band < band_hi and energy inside
    the window, edges snapped (see snap_edge); sorted by (k-index, band).
    eps_grid: (nk_grid, nw) band energies on the grid."""
    eps = np.asarray(eps_grid)[:, band_lo:band_hi]
    flat = np.sort(eps.ravel())
    lo = snap_edge(flat, e_lo)
    hi = snap_edge(flat, e_hi)
    kk, bb = np.nonzero((eps > lo) & (eps < hi))
    order = np.lexsort((bb, kk))
    return kk[order].astype(np.int64), (bb[order] + band_lo).astype(np.int64)


def lowest_states(eps_grid, band, count, tie_tol=1e-9):
    """The `count` lowest-energy states of one band, ordered by (energy,
    k-index) for the selection; the set grows past `count` while the next
    energy lies within tie_tol of the last one kept.  Returned sorted by
    k-index."""
    e = np.asarray(eps_grid)[:, band]
    order = np.lexsort((np.arange(len(e)), e))
    n = min(count, len(e))
    while n < len(e) and abs(e[order[n]] - e[order[n - 1]]) <= tie_tol:
        n += 1
    kk = np.sort(order[:n])
    return kk.astype(np.int64), np.full(n, band, dtype=np.int64)

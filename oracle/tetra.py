"""Linear tetrahedron integration over grid states (paper Sec. 4.3, the
integration behind Eqs. cond_tdf2 and pop; Bloechl, PRB 49, 16223 (1994)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Gamma-centred grid is cut into cubes of neighbouring points and every cube
into 6 tetrahedra sharing the diagonal from corner (0,0,0) to corner (1,1,1).
A tetrahedron of band n enters when its four corners are window states of
band n.  Inside it the energy and the integrand X are linear, so

  sum_nk X_nk delta(E - eps_nk)  ->  sum_T (1/6) sum_j c_j(E) X_j ,
  c_j(E) = (1/V_T) int_T delta(E - eps) lambda_j dV ,

with lambda_j the barycentric coordinate of corner j (the 1/6 is the volume of
one tetrahedron per grid point).  c_j is evaluated from its definition: the
plane eps = E cuts the tetrahedron in a triangle or a quadrilateral; in
barycentric space (unit simplex, volume 1/6) the delta integral is the area of
that polygon over |grad eps|, times 6 for V_T, and the lambda_j weight is the
area-weighted mean of lambda_j over the polygon.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .grid import grid_coords, grid_index
from .interp import fermi
from .units import KB_EV

# the simplex in barycentric space: corner j at V[j]
_V = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])

E_CHARGE = 1.602176634e-19        # C
# e^2 / (fs * Angstrom * eV) in S/m
SIGMA_UNIT = E_CHARGE / (1e-15 * 1e-10)


def tetrahedra(k_idx, band, n_grid):
    """[T][4] state indices of the tetrahedra whose corners are all states of
    one band, ordered by (cube index, path, band)."""
    n = np.asarray(n_grid, dtype=np.int64)
    lookup = {}
    for s, (k, b) in enumerate(zip(np.asarray(k_idx), np.asarray(band))):
        lookup[(int(k), int(b))] = s
    bands = sorted(set(int(b) for b in band))
    ks = sorted(set(int(k) for k in k_idx))
    out = []
    # only cubes with a window corner can hold a tetrahedron: take each cube
    # origin from the corners' neighbours, visit cubes in index order
    origins = set()
    for k in ks:
        c = grid_coords(k, n)
        for d in itertools.product((0, -1), repeat=3):
            origins.add(int(grid_index((c + np.array(d)) % n, n)))
    for o in sorted(origins):
        c0 = grid_coords(o, n)
        for perm in itertools.permutations(range(3)):
            e_a = np.eye(3, dtype=np.int64)[perm[0]]
            e_b = np.eye(3, dtype=np.int64)[perm[1]]
            corners = [c0, c0 + e_a, c0 + e_a + e_b, c0 + np.ones(3, dtype=np.int64)]
            kc = [int(grid_index(x % n, n)) for x in corners]
            for b in bands:
                st = [lookup.get((k, b)) for k in kc]
                if all(s is not None for s in st):
                    out.append(st)
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def delta_weights(e, E):
    """c_j(E), j = 0..3, for corner energies e (the definition in the module
    docstring, by explicit polygon construction)."""
    e = np.asarray(e, dtype=np.float64)
    g = np.array([e[1] - e[0], e[2] - e[0], e[3] - e[0]])
    gn = float(np.linalg.norm(g))
    c = np.zeros(4)
    if gn == 0.0:
        return c
    pts, lams = [], []
    for i, j in itertools.combinations(range(4), 2):
        if (e[i] < E) != (e[j] < E):
            t = (E - e[i]) / (e[j] - e[i])
            pts.append(_V[i] + t * (_V[j] - _V[i]))
            lam = np.zeros(4)
            lam[i], lam[j] = 1.0 - t, t
            lams.append(lam)
    if len(pts) < 3:
        return c
    pts, lams = np.array(pts), np.array(lams)
    # order the vertices around their centroid, in the plane normal to g
    cen = pts.mean(axis=0)
    nrm = g / gn
    u = np.cross(nrm, [1.0, 0.0, 0.0])
    if np.linalg.norm(u) < 1e-6:
        u = np.cross(nrm, [0.0, 1.0, 0.0])
    u /= np.linalg.norm(u)
    w = np.cross(nrm, u)
    ang = [math.atan2(float((p - cen) @ w), float((p - cen) @ u)) for p in pts]
    order = np.argsort(ang)
    pts, lams = pts[order], lams[order]
    area, mean = 0.0, np.zeros(4)
    for k in range(1, len(pts) - 1):
        a = 0.5 * float(np.linalg.norm(np.cross(pts[k] - pts[0], pts[k + 1] - pts[0])))
        area += a
        mean += a * (lams[0] + lams[k] + lams[k + 1]) / 3.0
    if area == 0.0:
        return c
    return 6.0 * area / gn * (mean / area)


def tetra_sum(eps, x, tets, energies):
    """out[i, comp] = sum_T (1/6) sum_j c_j(energies[i]) x[T_j, comp]."""
    eps = np.asarray(eps, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(len(eps), -1)
    out = np.zeros((len(energies), x.shape[1]))
    for t in tets:
        et = eps[t]
        lo, hi = et.min(), et.max()
        for i, E in enumerate(energies):
            if lo < E < hi:
                out[i] += delta_weights(et, E) @ x[t] / 6.0
    return out


def tdf(eps, vel, ff, tets, energies, n_k, omega_cell, spin=2.0):
    """Transport distribution function, Eq. cond_tdf2:
    Sigma_ab(E) = (S/(N_k Omega)) sum_nk v^a F^b delta(E - eps), [n_E][3][3]
    in 1/(fs Angstrom eV) (v in Angstrom/fs, F in Angstrom, Omega in Angstrom^3)."""
    v = np.asarray(vel, dtype=np.float64)
    f = np.asarray(ff, dtype=np.float64)
    x = (v[:, :, None] * f[:, None, :]).reshape(len(v), 9)
    return spin / (n_k * omega_cell) * tetra_sum(eps, x, tets, energies).reshape(-1, 3, 3)


def _trapz(y, x):
    x = np.asarray(x, dtype=np.float64)
    return np.tensordot(np.diff(x), 0.5 * (y[1:] + y[:-1]), axes=(0, 0))


def transport_from_tdf(energies, sig_e, mu, temp):
    """Conductivity (Eq. cond_tdf, S/m) and Seebeck coefficient (Eq. seebeck,
    V/K) from the TDF on an energy grid, trapezoid rule.  The charge in
    Eq. seebeck is the electron's, -e, so conduction electrons above mu give
    a negative S."""
    E = np.asarray(energies, dtype=np.float64)
    f0 = fermi(E, mu, temp).numpy()
    mdf = f0 * (1.0 - f0) / (KB_EV * temp)
    v1 = _trapz(mdf[:, None, None] * sig_e, E)
    v2 = _trapz((mdf * (E - mu))[:, None, None] * sig_e, E)
    sigma = SIGMA_UNIT * v1
    seebeck = -np.linalg.solve(v1, v2) / temp
    return sigma, seebeck


def population(eps, f, tets, energies):
    """Carrier population, Eq. pop: p(E) = sum_nk f_nk delta(eps_nk - E), 1/eV."""
    return tetra_sum(eps, f, tets, energies)[:, 0]

"""Comparison helpers for the parity tests (no method arithmetic here)."""
import re

import numpy as np
import torch

DEG_TOL = 1e-4   # eV, degenerate-group threshold for comparisons


def group_labels(e, tol=DEG_TOL):
    """Labels of runs of ascending values closer than tol, along the last axis."""
    e = np.asarray(e)
    lab = np.zeros(e.shape, dtype=np.int64)
    if e.shape[-1] > 1:
        lab[..., 1:] = np.cumsum(np.diff(e, axis=-1) >= tol, axis=-1)
    return lab


def _onehot(lab, n):
    return torch.nn.functional.one_hot(torch.as_tensor(lab), n).to(torch.float64)


def group_sums_g2(g2, eps_k, eps_kq, omega):
    """Sum |g|^2 [k][q][nu][m][n] over degenerate groups of modes (at q),
    final bands (at k+q) and initial bands (at k); groups from the reference
    energies.  Returns (nk, nq, Gnu, Gm, Gn)."""
    g2 = torch.as_tensor(np.asarray(g2), dtype=torch.float64)
    nw = g2.shape[-1]
    nm = g2.shape[2]
    pk = _onehot(group_labels(eps_k), nw)          # (k, n, c)
    pkq = _onehot(group_labels(eps_kq), nw)        # (k, q, m, b)
    pq = _onehot(group_labels(omega), nm)          # (q, nu, a)
    return torch.einsum("kqvmn,qva,kqmb,knc->kqabc", g2, pq, pkq, pk)


def g2_error(test, ref):
    """Per pair: max over group sums |dG| / max over the block of G_ref; returns
    (max over pairs, 99th percentile)."""
    d = (test - ref).abs().flatten(2).max(dim=2).values
    s = ref.abs().flatten(2).max(dim=2).values
    r = (d / torch.clamp(s, min=1e-300)).flatten()
    return float(r.max()), float(torch.quantile(r, 0.99))


def rate_error(test, ref, floor=1e-6):
    test = np.asarray(test)
    ref = np.asarray(ref)
    mask = np.abs(ref) >= floor * np.abs(ref).max()
    return float(np.max(np.abs(test - ref)[mask] / np.abs(ref)[mask]))


def header_symbols(path):
    txt = open(path).read()
    return sorted(set(re.findall(r"\b(ephx_[a-z0-9_]+)\s*\(", txt)))

"""The one-lane-per-matrix Hermitian eigensolver (eig_ql.h) built for the host.

The header is the device code's arithmetic (Householder tridiagonalisation,
implicit QL, back-transformation); compiled with g++ it runs the same steps on
the CPU, so its results can be checked against LAPACK on random, degenerate,
block-diagonal, diagonal, zero-row and nearly diagonal matrices of every order
1..8: eigenvalues, residual ||A U - U diag(w)|| and orthonormality of U, all
relative to the largest entry of A.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def solver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("eig") / "eig_lane_host")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "host", "eig_lane_host.cpp")])
    return exe


def _cases(rng, n):
    def herm(c):
        x = rng.normal(size=(c, n, n)) + 1j * rng.normal(size=(c, n, n))
        return 0.5 * (x + np.conj(np.swapaxes(x, 1, 2)))
    out = [herm(400)]
    u, _ = np.linalg.qr(rng.normal(size=(200, n, n)) + 1j * rng.normal(size=(200, n, n)))
    lam = np.round(rng.normal(size=(200, n)) * 2) / 2          # repeated eigenvalues
    out.append(u @ (lam[:, :, None] * np.conj(np.swapaxes(u, 1, 2))))
    dg = np.zeros((50, n, n), complex)
    dg[:, np.arange(n), np.arange(n)] = rng.normal(size=(50, n))
    out.append(dg)
    b = herm(50)
    h = n // 2
    b[:, :h, h:] = 0
    b[:, h:, :h] = 0
    out.append(b)
    out.append(herm(50) * 1e-9 + np.eye(n) * np.arange(n)[None, :, None])
    out.append(herm(50).real.astype(complex))
    out.append(np.zeros((4, n, n), complex))
    z = herm(50)
    z[:, 0, :] = 0
    z[:, :, 0] = 0
    out.append(z)
    return np.concatenate(out)


@pytest.mark.parametrize("n", list(range(1, 9)))
def test_lane_eigensolver_vs_lapack(solver, tmp_path, n):
    rng = np.random.default_rng(100 + n)
    a = _cases(rng, n)
    c = len(a)
    fin, fout = str(tmp_path / "a.bin"), str(tmp_path / "o.bin")
    a.astype(np.complex128).tofile(fin)
    subprocess.check_call([solver, str(n), str(c), fin, fout])
    o = np.fromfile(fout)
    w = o[:c * n].reshape(c, n)
    v = o[c * n:].view(np.complex128).reshape(c, n, n)
    nrm = np.abs(a).reshape(c, -1).max(axis=1) + 1e-300
    assert (np.diff(w, axis=1) >= 0).all()
    assert (np.abs(w - np.linalg.eigvalsh(a)).max(axis=1) / nrm).max() < 1e-13
    res = np.abs(a @ v - v * w[:, None, :]).reshape(c, -1).max(axis=1) / nrm
    assert res.max() < 1e-13
    orth = np.abs(np.conj(np.swapaxes(v, 1, 2)) @ v - np.eye(n)).reshape(c, -1).max()
    assert orth < 1e-13

"""FP64 CPU oracle for the electron-phonon hot path of PERTURBO (Zhou et al.,
arXiv:2002.02045).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code with the HIP library or its
Python binding; the only common dependency is the ``synth`` input generator,
which holds none of the method's arithmetic.

The oracle is deliberately plain: each step is written in the paper's order
and notation with float64 / complex128 PyTorch CPU tensors, LAPACK eigensolves
(``torch.linalg.eigh``) and library contractions (``einsum``), without blocking,
fusion or reordering beyond what the paper's definitions state.  PyTorch
autograd through these functions is the independent "oracle gradient".

Modules
-------
units   constants and unit conventions (eV, Angstrom, amu, K, fs)
interp  phases, band and phonon interpolation      (Sec. 2.2.1-2.2.2)
eph     g(k,q) interpolation, Froehlich term, rates (Sec. 2.2.3, 2.3, 2.1.2)
grid    Monkhorst-Pack grids, window states, pairs  (Sec. 4.3)
bte     pair table, collision integral, RK4, ITA, mobility (Sec. 2.1)

Pins (what each part is checked against, other than itself) are listed in
``tests/test_oracle_*.py``.  Parts without an independent pin are marked
"parity unpinned" in the docstring of the function concerned.
"""

"""Seeded synthetic inputs for the electron-phonon hot path.

This package only *draws* inputs: lattices, real-space vector sets, random
Wannier-basis tensors H(R), force constants C(R), couplings g(Re,Rp), and
random k/q lists.  It holds none of the method's arithmetic (no Fourier sums,
no diagonalisation, no scattering terms), so both the FP64 oracle and the GPU
path may use it without sharing any step of the computation.

The synthetic models stand in for the first-principles data the paper starts
from (DFT/DFPT + Wannier90 outputs, paper Sec. 3.2), with the shapes of its
examples: fcc Si/GaAs-like cells with 8 Wannier functions on 8x8x8 coarse grids
(Sec. 5.1, 5.4).
"""
from .models import (  # noqa: F401
    Model,
    fcc_lattice,
    sc_lattice,
    ws_vectors,
    make_model,
    make_config_model,
    make_counter_model,
    counter_coupling,
    counter_normals,
    coupling_envelope,
    philox4x32_10,
    random_points,
    cauchy_points,
    CONFIGS,
)

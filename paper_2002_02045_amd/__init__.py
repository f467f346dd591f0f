"""MI355X (gfx950) electron-phonon hot path of the PERTURBO method
(Zhou et al., arXiv:2002.02045): Wannier interpolation of g_mn,nu(k,q) and the
Boltzmann-equation scattering work built on it, behind the C ABI of
include/ephx.h.  This package is the thin Python binding; see ``api``.
"""
from .api import (  # noqa: F401
    FP32,
    FP64,
    BF16X3,
    BF16X6,
    EphxError,
    Model,
    PairTable,
    Params,
    bands,
    gkq,
    grid_states,
    phonons,
    rates,
)

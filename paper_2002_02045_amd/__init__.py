"""MI355X (gfx950) electron-phonon hot path of the PERTURBO method
(Zhou et al., arXiv:2002.02045): Wannier interpolation of g_mn,nu(k,q) and the
Boltzmann-equation scattering work built on it, behind the C ABI of
include/ephx.h.  This package is the thin Python binding; see ``api``.

The compiled library is loaded on first use of any public name (so that
``paper_2002_02045_amd.build`` can run before it exists); using the binding
without a built libephx.so raises ImportError.
"""
_PUBLIC = ("FP32", "FP64", "BF16X3", "BF16X6", "FP16X3", "EphxError", "Model", "PairTable", "Params",
           "bands", "gkq", "gkq_pairs", "grid_states", "phonons", "rates", "rates_part", "rates_polar_split",
           "rates_vjp", "RatesFunction",
           "MobilityFunction", "timer_enable", "timer_reset", "timer_get", "workspace_query")


def __getattr__(name):
    if name in _PUBLIC:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)


__all__ = list(_PUBLIC)

"""Python face of the C ABI: allocation of outputs with torch on the current
device and marshalling of pointers.  Names follow include/ephx.h."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import (BF16X3, BF16X6, FP16X3, FP32, FP64, EphxError, check, host_ptr, lib, ptr, stream_ptr,  # noqa: F401
                   timer_enable, timer_get, timer_reset)

F64 = torch.float64


def _prec(p):
    if isinstance(p, str):
        return _lib.PRECISIONS[p]
    return int(p)


def _pts(x):
    t = torch.as_tensor(x, dtype=F64, device="cuda")
    if t.ndim != 2 or t.shape[1] != 3:
        raise ValueError("points must be an (n, 3) array of reduced coordinates")
    return t.contiguous()


class Params:
    """temp (K), mu (eV), sigma (eV), omega_cut (eV), n_q (q-sum normalisation)."""

    def __init__(self, temp, mu=0.0, sigma=0.01, omega_cut=1e-4, n_q=1.0):
        self.temp, self.mu, self.sigma, self.omega_cut, self.n_q = temp, mu, sigma, omega_cut, n_q

    def c(self):
        return _lib.Params(self.temp, self.mu, self.sigma, self.omega_cut, self.n_q)


class Model:
    """Device copy of a Wannier model.  `src` needs the attributes lattice, tau,
    mass, nw, re, w_re, h, rp_ph, w_rp_ph, ifc, re_g, w_re_g, rp_g, w_rp_g, g
    and optionally zstar, eps_inf (+ polar = dict(alpha_ewald, gcut)).  With
    drawn = (seed, env) the coupling tensor is not uploaded but drawn on the
    device by the counter scheme (complex float, env [nRe][nRp] amplitudes);
    src.g is then ignored."""

    def __init__(self, src, polar=None, drawn=None):
        def f64(a):
            return np.ascontiguousarray(np.asarray(a, dtype=np.float64))

        def c128(a):
            return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)

        def i32(a):
            return np.ascontiguousarray(np.asarray(a, dtype=np.int32))

        keep = dict(
            tau=f64(src.tau), mass=f64(src.mass), re=i32(src.re), w_re=f64(src.w_re), h=c128(src.h),
            rp_ph=i32(src.rp_ph), w_rp_ph=f64(src.w_rp_ph), ifc=f64(src.ifc), re_g=i32(src.re_g),
            w_re_g=f64(src.w_re_g), rp_g=i32(src.rp_g), w_rp_g=f64(src.w_rp_g),
            g=None if drawn is not None else c128(src.g))
        d = _lib.ModelDesc()
        d.lattice[:] = [float(v) for v in np.asarray(src.lattice, dtype=np.float64).ravel()]
        d.natoms = keep["tau"].shape[0]
        d.nw = int(src.nw)
        d.tau, d.mass = host_ptr(keep["tau"]), host_ptr(keep["mass"])
        d.n_re, d.re, d.w_re, d.h = len(keep["re"]), host_ptr(keep["re"]), host_ptr(keep["w_re"]), host_ptr(keep["h"])
        d.n_rp_ph, d.rp_ph, d.w_rp_ph, d.ifc = (len(keep["rp_ph"]), host_ptr(keep["rp_ph"]),
                                                host_ptr(keep["w_rp_ph"]), host_ptr(keep["ifc"]))
        d.n_re_g, d.re_g, d.w_re_g = len(keep["re_g"]), host_ptr(keep["re_g"]), host_ptr(keep["w_re_g"])
        d.n_rp_g, d.rp_g, d.w_rp_g = len(keep["rp_g"]), host_ptr(keep["rp_g"]), host_ptr(keep["w_rp_g"])
        d.g = host_ptr(keep["g"])
        if drawn is not None:
            keep["env"] = f64(drawn[1])
            d.g_gen, d.g_seed, d.g_env = 1, int(drawn[0]), host_ptr(keep["env"])
        if polar is not None:
            keep["zstar"] = f64(src.zstar)
            keep["eps"] = f64(src.eps_inf)
            d.polar = 1 | (2 if polar.get("lo_to") else 0)
            d.zstar, d.eps_inf = host_ptr(keep["zstar"]), host_ptr(keep["eps"])
            d.alpha_ewald, d.gcut = float(polar["alpha_ewald"]), float(polar["gcut"])
        self._h = C.c_void_p()
        torch.cuda.init()
        check(lib.ephx_model_create(C.byref(d), C.byref(self._h)))
        self.nw = int(src.nw)
        self.nat = d.natoms
        self.nmodes = 3 * self.nat
        self.g_shape = (len(keep["re_g"]), len(keep["rp_g"]), self.nmodes, self.nw, self.nw)

    def set_g(self, g):
        """Replace the model's g(Re,Rp) by a complex128 device tensor of shape
        g_shape (ephx_model_set_g; synchronises the current stream)."""
        if not (torch.is_tensor(g) and g.is_cuda and g.dtype == torch.complex128):
            raise TypeError("g must be a complex128 tensor on the GPU")
        if tuple(g.shape) != self.g_shape:
            raise ValueError("g has shape %s, the model's is %s" % (tuple(g.shape), self.g_shape))
        g = g.detach().contiguous()
        check(lib.ephx_model_set_g(self._h, ptr(g), stream_ptr()))

    def g_entries(self, idx):
        """Entries of the device copy of g at flat indices idx (complex128 numpy)."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.empty(2 * len(idx), dtype=np.float64)
        check(lib.ephx_model_g_entries(self._h, len(idx), host_ptr(idx), host_ptr(out)))
        return out.view(np.complex128)

    def close(self):
        if self._h:
            check(lib.ephx_model_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def bands(model, k, want_u=True, want_vel=False):
    """eps (nk,nw), U (nk,nw,nw) complex128 or None, v (nk,nw,3) or None."""
    kt = _pts(k)
    nk = kt.shape[0]
    eps = torch.empty((nk, model.nw), dtype=F64, device="cuda")
    u = torch.empty((nk, model.nw, model.nw), dtype=torch.complex128, device="cuda") if want_u else None
    v = torch.empty((nk, model.nw, 3), dtype=F64, device="cuda") if want_vel else None
    check(lib.ephx_bands(model.handle, nk, ptr(kt), ptr(eps), ptr(u), ptr(v), stream_ptr()))
    return eps, u, v


def phonons(model, q, want_evec=True):
    qt = _pts(q)
    nq = qt.shape[0]
    om = torch.empty((nq, model.nmodes), dtype=F64, device="cuda")
    ev = torch.empty((nq, model.nmodes, model.nmodes), dtype=torch.complex128, device="cuda") if want_evec else None
    check(lib.ephx_phonons(model.handle, nq, ptr(qt), ptr(om), ptr(ev), stream_ptr()))
    return om, ev


def gkq(model, k, q, precision="fp64", omega_cut=1e-4, out=None):
    """|g|^2 as (nk, nq, nmodes, nw, nw) indexed [k][q][nu][m][n]."""
    p = _prec(precision)
    kt, qt = _pts(k), _pts(q)
    shape = (kt.shape[0], qt.shape[0], model.nmodes, model.nw, model.nw)
    if out is None:
        out = torch.empty(shape, dtype=F64 if p == FP64 else torch.float32, device="cuda")
    check(lib.ephx_gkq(model.handle, kt.shape[0], ptr(kt), qt.shape[0], ptr(qt), p, float(omega_cut), ptr(out),
                       stream_ptr()))
    return out


def gkq_pairs(model, k, q, ik, iq, precision="fp64", omega_cut=1e-4):
    """|g|^2 of the pairs (k[ik[j]], q[iq[j]]) as (npairs, nmodes, nw, nw)."""
    p = _prec(precision)
    kt, qt = _pts(k), _pts(q)
    ik = np.ascontiguousarray(ik, dtype=np.int32)
    iq = np.ascontiguousarray(iq, dtype=np.int32)
    if ik.shape != iq.shape or ik.ndim != 1:
        raise ValueError("ik and iq must be 1-D of the same length")
    out = torch.empty((len(ik), model.nmodes, model.nw, model.nw), dtype=F64 if p == FP64 else torch.float32,
                      device="cuda")
    check(lib.ephx_gkq_pairs(model.handle, kt.shape[0], ptr(kt), qt.shape[0], ptr(qt), len(ik),
                             ik.ctypes.data_as(C.c_void_p), iq.ctypes.data_as(C.c_void_p), p, float(omega_cut),
                             ptr(out), stream_ptr()))
    return out


def workspace_query(model, call, nk, nq, precision="fp64"):
    """Device bytes of the work buffers one gkq ("gkq") or rates ("rates") call of
    nk x nq takes from the model's workspace."""
    n = C.c_size_t(0)
    check(lib.ephx_workspace_query(model.handle, {"gkq": 0, "rates": 1}[call], int(nk), int(nq), _prec(precision),
                                   C.byref(n)))
    return int(n.value)


def rates(model, k, q, params, precision="fp64", q_weights=None, mode_resolved=True):
    """Scattering rates (nk, nw) in 1/fs and, optionally, per mode (nk, nw, nmodes)."""
    p = _prec(precision)
    kt, qt = _pts(k), _pts(q)
    nk = kt.shape[0]
    gam = torch.empty((nk, model.nw), dtype=F64, device="cuda")
    gmode = torch.empty((nk, model.nw, model.nmodes), dtype=F64, device="cuda") if mode_resolved else None
    qw = None if q_weights is None else torch.as_tensor(q_weights, dtype=F64, device="cuda").contiguous()
    pc = params.c()
    check(lib.ephx_rates(model.handle, C.byref(pc), nk, ptr(kt), qt.shape[0], ptr(qt), ptr(qw), p, ptr(gam),
                         ptr(gmode), stream_ptr()))
    return gam, gmode


PARTS = {"full": 0, "polar": 1, "rmpol": 2}


def rates_part(model, k, q, params, part, precision="fp64", q_weights=None, mode_resolved=True):
    """Rates of the long-range part |g_L|^2 ("polar") or of the rest
    |g|^2 - |g_L|^2 ("rmpol"), or of all of it ("full"), as for rates()."""
    p = _prec(precision)
    kt, qt = _pts(k), _pts(q)
    nk = kt.shape[0]
    gam = torch.empty((nk, model.nw), dtype=F64, device="cuda")
    gmode = torch.empty((nk, model.nw, model.nmodes), dtype=F64, device="cuda") if mode_resolved else None
    qw = None if q_weights is None else torch.as_tensor(q_weights, dtype=F64, device="cuda").contiguous()
    pc = params.c()
    check(lib.ephx_rates_part(model.handle, C.byref(pc), PARTS[part], nk, ptr(kt), qt.shape[0], ptr(qt), ptr(qw), p,
                              ptr(gam), ptr(gmode), stream_ptr()))
    return gam, gmode


def rates_polar_split(model, k, q_uniform, q_cauchy, params, precision="fp64", w_uniform=None, w_cauchy=None,
                      mode_resolved=True):
    """Polar split of the q sum: the rest |g|^2 - |g_L|^2 over q_uniform (weights
    w_uniform or 1/n) plus the long-range part over q_cauchy (weights w_cauchy)."""
    p = _prec(precision)
    kt, qu, qc = _pts(k), _pts(q_uniform), _pts(q_cauchy)
    nk = kt.shape[0]
    gam = torch.empty((nk, model.nw), dtype=F64, device="cuda")
    gmode = torch.empty((nk, model.nw, model.nmodes), dtype=F64, device="cuda") if mode_resolved else None
    wu = None if w_uniform is None else torch.as_tensor(w_uniform, dtype=F64, device="cuda").contiguous()
    wc = None if w_cauchy is None else torch.as_tensor(w_cauchy, dtype=F64, device="cuda").contiguous()
    pc = params.c()
    check(lib.ephx_rates_polar_split(model.handle, C.byref(pc), nk, ptr(kt), qu.shape[0], ptr(qu), ptr(wu),
                                     qc.shape[0], ptr(qc), ptr(wc), p, ptr(gam), ptr(gmode), stream_ptr()))
    return gam, gmode


def rates_vjp(model, k, q, params, gamma_bar, q_weights=None):
    """dL/dg(Re,Rp) (complex128, layout of the model's g) for L = sum gamma_bar * Gamma."""
    kt, qt = _pts(k), _pts(q)
    gb = torch.as_tensor(gamma_bar, dtype=F64, device="cuda").contiguous()
    qw = None if q_weights is None else torch.as_tensor(q_weights, dtype=F64, device="cuda").contiguous()
    out = torch.empty(model.g_shape, dtype=torch.complex128, device="cuda")
    pc = params.c()
    check(lib.ephx_rates_vjp(model.handle, C.byref(pc), kt.shape[0], ptr(kt), qt.shape[0], ptr(qt), ptr(qw), ptr(gb),
                             ptr(out), stream_ptr()))
    return out


class RatesFunction(torch.autograd.Function):
    """Gamma(g(Re,Rp)) (nk, nw) in FP64 with the hand-written adjoint.  g is a
    complex128 device tensor of the model's g_shape: the forward loads it into
    the model (ephx_model_set_g) and computes the rates from it; the backward
    loads it again (the model may have been given other values meanwhile) and
    returns dL/dRe g + i dL/dIm g."""

    @staticmethod
    def forward(ctx, g, model, k, q, params, q_weights=None):
        model.set_g(g)
        gam, _ = rates(model, k, q, params, precision="fp64", q_weights=q_weights, mode_resolved=False)
        ctx.save_for_backward(g)
        ctx.model, ctx.k, ctx.q, ctx.params, ctx.q_weights = model, k, q, params, q_weights
        return gam

    @staticmethod
    def backward(ctx, gbar):
        (g,) = ctx.saved_tensors
        ctx.model.set_g(g)
        gb = rates_vjp(ctx.model, ctx.k, ctx.q, ctx.params, gbar.contiguous(), q_weights=ctx.q_weights)
        return gb, None, None, None, None, None


class MobilityFunction(torch.autograd.Function):
    """mu(g(Re,Rp)) (3x3, cm^2/(V s)) in FP64 with the hand-written adjoint: the
    forward loads g into the model, builds the FP64 pair table of the given grid
    states from it and runs n_iter updates of the iterative BTE; the backward
    loads g again and reverses that chain (ephx_mobility_vjp)."""

    @staticmethod
    def forward(ctx, g, model, n_grid, k_idx, band, params, vel, n_iter):
        model.set_g(g)
        table = PairTable(model, n_grid, k_idx, band, precision="fp64")
        _, _, mob = table.mobility(params, vel, n_iter)
        ctx.save_for_backward(g)
        ctx.model, ctx.table, ctx.params, ctx.vel, ctx.n_iter = model, table, params, vel, n_iter
        return mob

    @staticmethod
    def backward(ctx, mob_bar):
        (g,) = ctx.saved_tensors
        ctx.model.set_g(g)
        gb = ctx.table.mobility_vjp(ctx.params, ctx.vel, ctx.n_iter, mob_bar.contiguous())
        return gb, None, None, None, None, None, None, None


def grid_states(model, n_grid, *, mode="window", band_lo=0, band_hi=None, e_lo=0.0, e_hi=0.0, count=0,
                capacity=None):
    """Window (mode="window") or lowest-count (mode="lowest") states on a
    Gamma-centred grid.  Returns numpy (k_idx, band, eps)."""
    n3 = (C.c_int * 3)(*[int(x) for x in np.broadcast_to(np.asarray(n_grid), (3,))])
    ngrid = n3[0] * n3[1] * n3[2]
    if band_hi is None:
        band_hi = model.nw
    if capacity is None:
        capacity = max(int(count) + 64, 1) if mode == "lowest" else ngrid * (band_hi - band_lo)
    kk = np.empty(capacity, np.int32)
    bb = np.empty(capacity, np.int32)
    ee = np.empty(capacity, np.float64)
    ns = C.c_int(0)
    check(lib.ephx_grid_states(model.handle, n3, 0 if mode == "window" else 1, int(band_lo), int(band_hi),
                               float(e_lo), float(e_hi), int(count), int(capacity), C.byref(ns), host_ptr(kk),
                               host_ptr(bb), host_ptr(ee), stream_ptr()))
    n = ns.value
    return kk[:n].copy(), bb[:n].copy(), ee[:n].copy()


class PairTable:
    """Symmetrised |g|^2 table of grid states with collision, dynamics and ITA."""

    def __init__(self, model, n_grid, k_idx, band, precision="fp64", omega_cut=1e-4):
        self.model = model
        self.S = len(k_idx)
        self.nmodes = model.nmodes
        self.precision = _prec(precision)
        n3 = (C.c_int * 3)(*[int(x) for x in np.broadcast_to(np.asarray(n_grid), (3,))])
        self._k = np.ascontiguousarray(k_idx, dtype=np.int32)
        self._b = np.ascontiguousarray(band, dtype=np.int32)
        self._h = C.c_void_p()
        check(lib.ephx_table_create(model.handle, n3, self.S, host_ptr(self._k), host_ptr(self._b),
                                    _prec(precision), float(omega_cut), C.byref(self._h), stream_ptr()))

    def close(self):
        if self._h:
            check(lib.ephx_table_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def g2(self):
        dt = F64 if self.precision == FP64 else torch.float32
        g = torch.empty((self.nmodes, self.S, self.S), dtype=dt, device="cuda")
        e = torch.empty(self.S, dtype=F64, device="cuda")
        check(lib.ephx_table_g2(self._h, ptr(g), ptr(e), stream_ptr()))
        return g, e

    def setup(self, params, mode_scale=None):
        pc = params.c()
        ms = None if mode_scale is None else np.ascontiguousarray(mode_scale, dtype=np.float64)
        check(lib.ephx_collision_setup(self._h, C.byref(pc), host_ptr(ms), stream_ptr()))
        self._ms = ms

    def collision(self, f):
        f = torch.as_tensor(f, dtype=F64, device="cuda").contiguous()
        out = torch.empty(self.S, dtype=F64, device="cuda")
        check(lib.ephx_collision(self._h, ptr(f), ptr(out), stream_ptr()))
        return out

    def collision_noalloc(self, f, out):
        """I[f] into the caller's device tensor `out` (S doubles) through the
        entry point that allocates nothing (its work memory is the library's
        static per-GPU array; calls overlapping on one GPU race)."""
        if not (torch.is_tensor(f) and f.is_cuda and f.dtype == F64 and f.numel() == self.S):
            raise TypeError("f must be a float64 device tensor of S entries")
        if not (torch.is_tensor(out) and out.is_cuda and out.dtype == F64 and out.numel() == self.S):
            raise TypeError("out must be a float64 device tensor of S entries")
        check(lib.ephx_collision_noalloc(self._h, ptr(f), ptr(out), stream_ptr()))
        return out

    def dynamics(self, f0, dt, n_steps, ckpt_every=0, method="rk4", efield=None):
        """f after n_steps steps of dt fs ("rk4" or "euler"), with an optional
        field (V/Angstrom, Cartesian); checkpoints every ckpt_every steps."""
        f0 = torch.as_tensor(f0, dtype=F64, device="cuda").contiguous()
        out = torch.empty(self.S, dtype=F64, device="cuda")
        ck = None
        if ckpt_every > 0:
            ck = torch.empty((n_steps // ckpt_every + 1, self.S), dtype=F64, device="cuda")
        meth = {"rk4": 0, "euler": 1}[method]
        if efield is None and meth == 0:
            check(lib.ephx_dynamics(self._h, ptr(f0), float(dt), int(n_steps), int(ckpt_every), ptr(out), ptr(ck),
                                    stream_ptr()))
        else:
            arr = None if efield is None else (C.c_double * 3)(*[float(x) for x in efield])
            ef = None if arr is None else C.addressof(arr)
            check(lib.ephx_dynamics_field(self._h, ptr(f0), float(dt), int(n_steps), meth, ef, int(ckpt_every),
                                          ptr(out), ptr(ck), stream_ptr()))
        return out, ck

    def stream_info(self, matrix="collision"):
        """(entries read per pass, live tiles, tiles) of the energy-banded
        collision ("collision") or transport ("transport") matrix."""
        n = C.c_longlong(0)
        a, b = C.c_int(0), C.c_int(0)
        check(lib.ephx_table_stream_info(self._h, {"collision": 0, "transport": 1}[matrix], C.byref(n), C.byref(a),
                                         C.byref(b), stream_ptr()))
        return int(n.value), int(a.value), int(b.value)

    def collision_vjp(self, f, lam, want_s=True):
        f = torch.as_tensor(f, dtype=F64, device="cuda").contiguous()
        lam = torch.as_tensor(lam, dtype=F64, device="cuda").contiguous()
        fb = torch.empty(self.S, dtype=F64, device="cuda")
        sb = torch.empty(self.nmodes, dtype=F64, device="cuda") if want_s else None
        check(lib.ephx_collision_vjp(self._h, ptr(f), ptr(lam), ptr(fb), ptr(sb), stream_ptr()))
        return fb, sb

    def dynamics_vjp(self, ckpts, dt, n_steps, ckpt_every, f_bar, want_s=True):
        fb = torch.as_tensor(f_bar, dtype=F64, device="cuda").contiguous()
        f0b = torch.empty(self.S, dtype=F64, device="cuda")
        sb = torch.empty(self.nmodes, dtype=F64, device="cuda") if want_s else None
        check(lib.ephx_dynamics_vjp(self._h, ptr(ckpts), float(dt), int(n_steps), int(ckpt_every), ptr(fb),
                                    ptr(f0b), ptr(sb), stream_ptr()))
        return f0b, sb

    def mobility(self, params, vel, n_iter):
        """(F (S,3), tau (S,), mu (3,3)) after exactly n_iter updates of the ITA."""
        ff, tau, mob, _, _ = self.ita(params, vel, n_iter, tol=0.0)
        return ff, tau, mob

    def ita(self, params, vel, n_iter_max, tol):
        """Iterate the linearised BTE until the largest change of F is below tol
        times its largest component, at most n_iter_max updates (tol <= 0: exactly
        n_iter_max).  Returns (F, tau, mu, n_iter made, last relative change)."""
        vel = torch.as_tensor(vel, dtype=F64, device="cuda").contiguous()
        ff = torch.empty((self.S, 3), dtype=F64, device="cuda")
        tau = torch.empty(self.S, dtype=F64, device="cuda")
        mob = torch.empty((3, 3), dtype=F64, device="cuda")
        n = C.c_int(0)
        chg = C.c_double(0.0)
        pc = params.c()
        check(lib.ephx_mobility(self._h, C.byref(pc), ptr(vel), int(n_iter_max), float(tol), ptr(ff), ptr(tau),
                                ptr(mob), C.byref(n), C.byref(chg), stream_ptr()))
        return ff, tau, mob, int(n.value), float(chg.value)

    def tdf(self, params, vel, f_ita, energies):
        """(TDF [n_E][3][3] in 1/(fs A eV), sigma [3][3] in S/m, Seebeck [3][3] in V/K)."""
        vel = torch.as_tensor(vel, dtype=F64, device="cuda").contiguous()
        ff = torch.as_tensor(f_ita, dtype=F64, device="cuda").contiguous()
        eg = torch.as_tensor(energies, dtype=F64, device="cuda").contiguous()
        out = torch.empty((eg.shape[0], 3, 3), dtype=F64, device="cuda")
        sig = torch.empty((3, 3), dtype=F64, device="cuda")
        see = torch.empty((3, 3), dtype=F64, device="cuda")
        pc = params.c()
        check(lib.ephx_tdf(self._h, C.byref(pc), ptr(vel), ptr(ff), int(eg.shape[0]), ptr(eg), ptr(out), ptr(sig),
                           ptr(see), stream_ptr()))
        return out, sig, see

    def population(self, f, energies):
        """p(E) = sum_nk f_nk delta(eps_nk - E) (1/eV) on the energy grid."""
        ff = torch.as_tensor(f, dtype=F64, device="cuda").contiguous()
        eg = torch.as_tensor(energies, dtype=F64, device="cuda").contiguous()
        out = torch.empty(eg.shape[0], dtype=F64, device="cuda")
        check(lib.ephx_population(self._h, ptr(ff), int(eg.shape[0]), ptr(eg), ptr(out), stream_ptr()))
        return out

    def mobility_vjp(self, params, vel, n_iter, mob_bar):
        """dL/dg(Re,Rp) (complex128, layout of the model's g) for L = sum mob_bar * mu."""
        vel = torch.as_tensor(vel, dtype=F64, device="cuda").contiguous()
        mb = torch.as_tensor(mob_bar, dtype=F64, device="cuda").contiguous()
        out = torch.empty(self.model.g_shape, dtype=torch.complex128, device="cuda")
        pc = params.c()
        check(lib.ephx_mobility_vjp(self._h, C.byref(pc), ptr(vel), int(n_iter), ptr(mb), ptr(out), stream_ptr()))
        return out

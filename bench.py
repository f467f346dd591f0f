#!/usr/bin/env python3
"""Throughput of the electron-phonon hot path on one MI355X.

Headline: |g(k,q)|^2 pairs/s of the scattering-rate pipeline (Eqs.
eph_mat_wann2, eph_mat, scatter_rate, BTE_W) on the Si-like workload: Nw = 8
Wannier functions, 2 atoms (6 modes), 512 Re and 512 Rp vectors from an 8x8x8
least-distance set, k points in a 0.3 eV window above the conduction-band
minimum, 10^6 uniform random q, T = 300 K, sigma = 5 meV.  One step = the rates
of one batch of k points against all q: bands at k, Re contraction, and per
(k,q) pair the H(k+q) Fourier sum + FP64 eigensolve, the Rp contraction, the
band rotation, the mode projection, |g|^2 and the delta-weighted sums.

The inputs are seeded synthetic models that take the shapes of the paper's Si
example (the first-principles data it starts from is not available here).
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k-batch", type=int, default=32)
    ap.add_argument("--nq", type=int, default=1_000_000)
    # the headline precision first, right after its warm-up; the others follow
    # (a precision measured after the others runs on a GPU they have heated)
    ap.add_argument("--precisions", default="fp16x3,bf16x3,bf16x6,fp32,fp64")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dyn-steps", type=int, default=200, help="timed RK4 steps of the dynamics workload (0: skip)")
    ap.add_argument("--dyn-grid", type=int, default=80)
    ap.add_argument("--dyn-states", type=int, default=20_000)
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="first run a 1 GiB device fill and a 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--no-adjoints", action="store_true",
                    help="skip the RK4 backward and the mobility adjoint legs (e.g. under hardware counters)")
    ap.add_argument("--gaas-grid", type=int, default=100, help="k = q grid of the GaAs-like transport leg (0: skip)")
    ap.add_argument("--cell-k", type=int, default=32, help="k points of the large-cell slice (0: skip)")
    ap.add_argument("--cell-q", type=int, default=4096, help="q points of the large-cell slice")
    return ap.parse_args()


BF16_PEAK = 2516.6   # dense bf16 and fp16 MFMA, TFLOP/s
# 16-bit products per FP32-equivalent real product of each split path
SPLIT_PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6, "fp16x3": 3}
# ceiling of each path in algorithmic (FP32/FP64-equivalent) TFLOP/s: the split
# paths run their products on the dense bf16/fp16 MFMA peak
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": BF16_PEAK / 3, "bf16x6": BF16_PEAK / 6,
               "fp16x3": BF16_PEAK / 3}
HBM_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    import paper_2002_02045_amd as px

    if args.pmc_calibrate:
        # known traffic for scaling FETCH_SIZE / WRITE_SIZE: the fill writes 1 GiB,
        # the copy reads 1 GiB and writes 1 GiB
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration: fill writes %d bytes; copy reads %d and writes %d bytes" % (a.nbytes, a.nbytes, b.nbytes))
        del a, b

    cfg = synth.CONFIGS["si"]
    t0 = time.time()
    model = synth.make_config_model("si")
    log("model generated in %.1fs: nw=%d nmodes=%d nR=%d" % (time.time() - t0, model.nw, model.nmodes, len(model.re)))
    dm = px.Model(model)
    nw, nm = model.nw, model.nmodes
    n_rp = len(model.rp_g)
    cb = nw // 2

    # k points in the window [CBM, CBM + 0.3 eV] of the lowest conduction band
    grid = np.stack(np.meshgrid(*[np.arange(40) / 40.0] * 3, indexing="ij"), -1).reshape(-1, 3)
    eg, _, _ = px.bands(dm, grid, want_u=False)
    cbm = float(eg[:, cb].min())
    cand = synth.random_points(cfg["seed"] + 100, 400_000)
    ec, _, _ = px.bands(dm, cand, want_u=False)
    ecb = ec[:, cb].cpu().numpy() - cbm
    sel = cand[(ecb >= 0.0) & (ecb <= cfg["window"])]
    nk_total = min(cfg["nk"], len(sel))
    kpts = sel[:nk_total]
    q = synth.random_points(cfg["seed"] + 200, args.nq)
    log("CBM %.4f eV, %d window k points, %d q" % (cbm, nk_total, args.nq))
    params = px.Params(temp=cfg["T"], mu=cfg["mu"], sigma=cfg["sigma"], omega_cut=cfg["omega_cut"])
    qdev = torch.as_tensor(q, device="cuda")
    kb = args.k_batch

    def kbatch(i):
        s = (i * kb) % max(1, nk_total - kb + 1)
        return kpts[s:s + kb]

    results = {}
    for prec in [p for p in args.precisions.split(",") if p]:
        steps = args.steps if prec != "fp64" else max(1, args.steps // 2)
        for i in range(args.warmup):
            px.rates(dm, kbatch(i), qdev, params, precision=prec)
        torch.cuda.synchronize()
        # the timed steps are one call over their k batches, as a run over all
        # window k makes it: the q-only work (phonons, phase planes and tables,
        # mode factors) is done once per call.  They run without the stage
        # timers (events around every stage); the same call then runs again
        # with them for the stage split and the contraction's launch average
        ksteps = np.concatenate([kbatch(args.warmup + i) for i in range(steps)])
        t0 = time.perf_counter()
        px.rates(dm, ksteps, qdev, params, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        px.timer_reset()
        px.timer_enable(True)
        torch.cuda.synchronize()
        px.rates(dm, ksteps, qdev, params, precision=prec)
        torch.cuda.synchronize()
        px.timer_enable(False)
        stages = {s: px.timer_get(s) for s in ("rp_contraction", "rp_phases", "hkq_fourier", "eig_hkq", "epilogue",
                                                "re_contraction", "phonons")}
        px.timer_reset()
        pairs = steps * kb * args.nq
        rp_n, rp_ms = stages["rp_contraction"]
        flops_pair = rp_flops_per_pair(model.rp_g, nw, nm)
        achieved = flops_pair * pairs / (rp_ms * 1e-3) / 1e12 if rp_ms > 0 else 0.0
        results[prec] = dict(
            pairs_per_s=pairs / dt, ms_per_step=1e3 * dt / steps, steps=steps,
            stage_ms={s: round(v[1] / steps, 3) for s, v in stages.items()},
            rp_launches=rp_n, rp_avg_ms=rp_ms / max(rp_n, 1),
            rp_tflops=achieved, rp_frac=achieved / PEAK_TFLOPS[prec])
        log("%s: %.3e pairs/s, %.1f ms/step, rp_contraction %.1f TFLOP/s (%.1f%% of %s peak); stages %s" % (
            prec, pairs / dt, 1e3 * dt / steps, achieved, 100 * achieved / PEAK_TFLOPS[prec], prec,
            results[prec]["stage_ms"]))

    # error of each reduced precision against the GPU FP64 path on a sample
    # block, compared as sums over degenerate groups (1e-4 eV) of bands at k,
    # k+q and modes at q, relative to each pair's largest group sum
    ks, qs = kpts[:4], q[:4096]
    ref = group_sums(px, dm, ks, qs, px.gkq(dm, ks, qs, precision="fp64"))
    blockmax = ref.flatten(2).abs().max(dim=2).values
    for prec in results:
        if prec == "fp64":
            results[prec]["g2_err_vs_fp64"] = 0.0
            continue
        got = group_sums(px, dm, ks, qs, px.gkq(dm, ks, qs, precision=prec).double())
        err = ((got - ref).abs().flatten(2).max(dim=2).values / blockmax.clamp_min(1e-300)).max()
        results[prec]["g2_err_vs_fp64"] = float(err)

    # headline: fastest path whose |g|^2 error meets 1e-5
    ok = [p for p in results if results[p]["g2_err_vs_fp64"] <= 1e-5]
    head = max(ok, key=lambda p: results[p]["pairs_per_s"]) if ok else "fp64"
    r = results[head]
    roof = {"bound": "mfma", "kernel": "rp_contraction (%s)" % RP_KERNEL[head], "achieved": round(r["rp_tflops"], 3),
            "peak": round(PEAK_TFLOPS[head], 1), "unit": "TFLOP/s", "frac": round(r["rp_frac"], 4),
            "traffic": measured_traffic(RP_KERNEL[head]), "traffic_unit": "HBM bytes per launch",
            "flops_per_pair": rp_flops_per_pair(model.rp_g, nw, nm), "avg_launch_ms": round(r["rp_avg_ms"], 4),
            "mfma_products_per_flop": SPLIT_PRODUCTS[head],
            "mfma_tflops": round(r["rp_tflops"] * SPLIT_PRODUCTS[head], 1)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(model, kpts, q, cfg, args.cpu_seconds)

    dyn = None
    if args.dyn_steps > 0:
        dyn = dynamics_bench(px, dm, model, args)

    gaas = None
    if args.gaas_grid > 0:
        gaas = gaas_bench(px, args)

    cell = None
    if args.cell_k > 0:
        del dm
        cell = cell_bench(px, args)

    out = {
        "metric": "|g(k,q)|^2 pairs/s (scattering-rate pipeline, Si-like)",
        "value": r["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3 (f32 accumulate)",
                  "bf16x6": "bf16x6 (f32 accumulate)", "fp16x3": "fp16x3 (f32 accumulate)"}[head],
        "data": "synthetic",
        "config": {"workload": "si-like rates: Nw=8, 6 modes, 512 Re x 512 Rp, %d k per step (of %d window k; "
                               "the timed steps in one call), %d random q, T=300 K, sigma=5 meV"
                               % (kb, nk_total, args.nq),
                   "precision": head},
        "roofline": roof,
        "speedup_vs_fp64_gpu": (round(r["pairs_per_s"] / results["fp64"]["pairs_per_s"], 3)
                                if "fp64" in results else None),
        "cpu_baseline": cpu,
        "by_precision": {p: {kk: (round(v, 6) if isinstance(v, float) else v) for kk, v in d.items()}
                         for p, d in results.items()},
        "dynamics": dyn,
        "gaas_transport": gaas,
        "large_cell": cell,
    }
    print(json.dumps(out), flush=True)


def dynamics_bench(px, dm, model, args):
    """BTE collision steps/s: RK4 time stepping of f_nk(t) (Eq. BTE_E with E = 0,
    collision integral of Eq. e_ph_scattering) on the lowest conduction states of
    an n^3 Gamma-centred grid with a stored FP32 |g|^2 pair table.  One step =
    four collision evaluations + stage updates."""
    import torch

    import synth
    cfg = synth.CONFIGS["dyn"]
    n = (args.dyn_grid,) * 3
    nw = model.nw
    t0 = time.perf_counter()
    kk, bb, ee = px.grid_states(dm, n, mode="lowest", band_lo=nw // 2, count=args.dyn_states)
    t_states = time.perf_counter() - t0
    S = len(kk)
    t0 = time.perf_counter()
    tab = px.PairTable(dm, n, kk, bb, precision="fp32")
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    nq = float(np.prod(n))
    par = px.Params(temp=cfg["T"], sigma=cfg["sigma"], omega_cut=cfg["omega_cut"], n_q=nq)
    t0 = time.perf_counter()
    tab.setup(par)
    t_setup = time.perf_counter() - t0
    cbm = float(ee.min())
    f0 = cfg["f0_peak"] * np.exp(-((ee - cbm - cfg["f0_centre"]) ** 2) / (2 * cfg["f0_width"] ** 2))
    f0 = torch.as_tensor(f0, device="cuda")
    log("dynamics: %d states (span %.3f eV) on %s grid; states %.1fs, table %.1fs, setup %.1fs" % (
        S, float(ee.max() - ee.min()), "x".join(map(str, n)), t_states, t_table, t_setup))
    tab.dynamics(f0, cfg["dt"], 2)                         # warmup
    torch.cuda.synchronize()
    # steps/s with the stage timers off (they record events around every
    # kernel); then the same steps again with the timers on for the per-kernel
    # averages of the roofline
    t0 = time.perf_counter()
    f1, _ = tab.dynamics(f0, cfg["dt"], args.dyn_steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    px.timer_reset()
    px.timer_enable(True)
    torch.cuda.synchronize()
    tab.dynamics(f0, cfg["dt"], args.dyn_steps)
    torch.cuda.synchronize()
    px.timer_enable(False)
    ns, ms = px.timer_get("collision_stream")
    npm, mspm = px.timer_get("stream_permute")
    px.timer_reset()
    ld = (S + 63) // 64 * 64
    # the FP32 collision matrix is stored in energy order and tiles of state
    # pairs further apart than omega_max + 6 sigma (exact zeros) are not read:
    # the algorithmic bytes of a pass are the entries of the live tiles
    live, n_live, n_tiles = tab.stream_info("collision")
    alg_bytes = 4.0 * live
    achieved = alg_bytes / (ms / ns * 1e-3) / 1e9
    drift = abs(float(f1.sum() - f0.sum())) / float(f0.sum())
    if not np.isfinite(drift):
        raise RuntimeError("dynamics produced non-finite occupations")
    log("dynamics: %.1f RK4 steps/s, collision_stream %.3f ms avg = %.0f GB/s (%.1f%% of HBM) over %d of %d tiles "
        "(%.3f of the dense matrix), number drift %.2e" % (
            args.dyn_steps / dt, ms / ns, achieved, 100 * achieved / HBM_GBS, n_live, n_tiles, live / S ** 2, drift))
    # Euler stepping in a field (Eq. BTE_E with E != 0): one collision pass
    # and the grid drift per step
    efield = [1e-4, 0.0, 0.0]                             # V/Angstrom (10 kV/cm)
    tab.dynamics(f0, cfg["dt"], 2, method="euler", efield=efield)     # warmup, builds the neighbour table
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f2, _ = tab.dynamics(f0, cfg["dt"], args.dyn_steps, method="euler", efield=efield)
    torch.cuda.synchronize()
    dt_e = time.perf_counter() - t0
    if not bool(torch.isfinite(f2).all()):
        raise RuntimeError("field dynamics produced non-finite occupations")
    log("dynamics: %.1f Euler steps/s with E = %g V/A along x" % (args.dyn_steps / dt_e, efield[0]))
    bwd = {} if args.no_adjoints else rk4_backward(tab, f0, cfg, args)
    out = {
        "metric": "BTE collision steps/s (RK4 steps of the carrier dynamics)",
        "value": args.dyn_steps / dt, "unit": "RK4 steps/s", "steps": args.dyn_steps,
        "ms_per_step": 1e3 * dt / args.dyn_steps, "dtype": "f32 table, f64 state",
        "config": {"workload": "si-like dynamics: %s grid, %d lowest conduction states (span %.3f eV), 6 modes, "
                               "FP32 pair table, sigma=8 meV, T_ph=300 K, dt=1 fs" % (
                                   "x".join(map(str, n)), S, float(ee.max() - ee.min()))},
        "roofline": {"bound": "hbm", "kernel": "collision_stream", "achieved": round(achieved, 1),
                     "peak": HBM_GBS, "unit": "GB/s", "frac": round(achieved / HBM_GBS, 4),
            "traffic": measured_traffic("k_stream<float, 1, 1>"), "traffic_unit": "HBM bytes per launch",
                     "bytes_per_launch": alg_bytes, "avg_launch_ms": round(ms / ns, 5),
                     "dense_bytes": 4.0 * S * S, "live_tiles": n_live, "tiles": n_tiles},
        "collision_evals_per_s": ns / (1e-3 * (ms + mspm)) if ms > 0 else None,
        "gather_reduce_ms_per_pass": round(mspm / max(1, ns), 5),
        "table_build_s": round(t_table, 3), "setup_s": round(t_setup, 3),
        "carrier_number_drift": drift,
        "euler_field_steps_per_s": args.dyn_steps / dt_e, "euler_field_V_per_A": efield,
        **bwd,
    }
    out["transport"] = transport_bench(px, dm, tab, kk, bb, ee, n, f1, cfg, args)
    tab.close()
    return out


def rk4_backward(tab, f0, cfg, args):
    """Backward through time: the forward with checkpoints every 50 steps, then
    the reverse RK4 that replays each segment from its checkpoint (Eq. BTE_E
    with E = 0), for the gradients w.r.t. f0 and the six mode scales."""
    import torch

    nb = max(50, args.dyn_steps // 50 * 50)
    ck = 50
    tab.dynamics_vjp(tab.dynamics(f0, cfg["dt"], ck, ckpt_every=ck)[1], cfg["dt"], ck, ck, f0)   # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fT, cks = tab.dynamics(f0, cfg["dt"], nb, ckpt_every=ck)
    torch.cuda.synchronize()
    t_fwd_ck = time.perf_counter() - t0
    t0 = time.perf_counter()
    f0_bar, s_bar = tab.dynamics_vjp(cks, cfg["dt"], nb, ck, torch.ones_like(fT))
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    if not (bool(torch.isfinite(f0_bar).all()) and bool(torch.isfinite(s_bar).all())):
        raise RuntimeError("dynamics adjoint produced non-finite gradients")
    log("dynamics: backward through %d RK4 steps %.3f s (%.1f steps/s, %.2fx the forward with checkpoints)" % (
        nb, t_bwd, nb / t_bwd, t_bwd / t_fwd_ck))
    return {"rk4_backward_steps_per_s": nb / t_bwd, "rk4_backward_steps": nb, "rk4_backward_ckpt_every": ck,
            "rk4_backward_over_forward": t_bwd / t_fwd_ck}


def transport_bench(px, dm, tab, kk, bb, ee, n, f_t, cfg, args):
    """On the dynamics states: ITA mobility (Eqs. BTE_iter, cond, 10 iterations,
    FP32 transport matrix), the TDF by tetrahedra on 512 energies with sigma and
    Seebeck (Eqs. cond_tdf2, cond_tdf, seebeck), and the population p(E,t) of the
    final occupations (Eq. pop)."""
    import torch

    pts = np.stack([kk // (n[1] * n[2]), (kk // n[2]) % n[1], kk % n[2]], axis=-1) / np.asarray(n, dtype=np.float64)
    _, _, v = px.bands(dm, pts, want_u=False, want_vel=True)
    vel = v[torch.arange(len(bb), device=v.device), torch.as_tensor(bb, device=v.device)].contiguous()
    cbm = float(ee.min())
    par = px.Params(temp=cfg["T"], mu=cbm - 0.2, sigma=cfg["sigma"], omega_cut=cfg["omega_cut"], n_q=float(np.prod(n)))
    energies = np.linspace(cbm, float(ee.max()), 512)
    tab.mobility(par, vel, 10)
    tab.tdf(par, vel, torch.zeros_like(vel), energies[:4])          # builds the tetrahedra
    torch.cuda.synchronize()
    px.timer_reset()
    px.timer_enable(True)
    t0 = time.perf_counter()
    ff, _, mob = tab.mobility(par, vel, 10)
    torch.cuda.synchronize()
    t_ita = time.perf_counter() - t0
    t0 = time.perf_counter()
    sig_e, sigma, seebeck = tab.tdf(par, vel, ff, energies)
    t_tdf = time.perf_counter() - t0
    t0 = time.perf_counter()
    pop = tab.population(f_t, energies)
    t_pop = time.perf_counter() - t0
    px.timer_enable(False)
    n_st, ms_st = px.timer_get("transport_stream")
    _, ms_build = px.timer_get("matrix_build")
    _, ms_tdf = px.timer_get("tdf_tetra")
    _, ms_pop = px.timer_get("population_tetra")
    px.timer_reset()
    S = len(kk)
    alg = 4.0 * tab.stream_info("transport")[0]
    log("transport: ITA 10 iterations %.1f ms (W build %.1f ms, stream %.3f ms avg = %.0f GB/s), TDF %d energies "
        "%.1f ms, population %.1f ms; mu_xx %.4g cm^2/Vs, S_xx %.4g uV/K" % (
            1e3 * t_ita, ms_build, ms_st / n_st, alg / (ms_st / n_st * 1e-3) / 1e9, len(energies), 1e3 * t_tdf,
            1e3 * t_pop,
            float(mob[0, 0]), 1e6 * float(seebeck[0, 0])))
    adj = None if args.no_adjoints else mobility_adjoint_bench(px, dm, cfg)
    return {
        "mobility_adjoint": adj,
        "ita_ms": round(1e3 * t_ita, 3), "ita_iterations": 10, "w_build_ms": round(ms_build, 3),
        "transport_stream_avg_ms": round(ms_st / n_st, 5),
        "transport_stream_gbs": round(alg / (ms_st / n_st * 1e-3) / 1e9, 1),
        "tdf_ms": round(1e3 * t_tdf, 3), "tdf_kernel_ms": round(ms_tdf, 3), "energies": len(energies),
        "population_ms": round(1e3 * t_pop, 3), "population_kernel_ms": round(ms_pop, 3),
        "mobility_xx_cm2_per_Vs": float(mob[0, 0]), "sigma_xx_S_per_m": float(sigma[0, 0]),
        "seebeck_xx_uV_per_K": 1e6 * float(seebeck[0, 0]),
        "population_integral": float(np.trapezoid(pop.cpu().numpy(), energies)),
        "carriers": float(f_t.sum()),
    }


def mobility_adjoint_bench(px, dm, cfg, grid=24, count=1500):
    """Adjoint of the ITA mobility w.r.t. g(Re,Rp) (FP64 table, 10 iterations)
    on the lowest conduction states of a 24^3 grid: the reverse fixed-point
    iterations with W^T, then every state pair's g(k,q) again and its
    derivative back through the mode projection, the rotations and both
    Fourier sums into g(Re,Rp)."""
    import torch

    n = (grid,) * 3
    kk, bb, ee = px.grid_states(dm, n, mode="lowest", band_lo=dm.nw // 2, count=count)
    S = len(kk)
    tab = px.PairTable(dm, n, kk, bb, precision="fp64")
    pts = np.stack([kk // (n[1] * n[2]), (kk // n[2]) % n[1], kk % n[2]], axis=-1) / np.asarray(n, dtype=np.float64)
    _, _, v = px.bands(dm, pts, want_u=False, want_vel=True)
    vel = v[torch.arange(len(bb), device=v.device), torch.as_tensor(bb, device=v.device)].contiguous()
    par = px.Params(temp=cfg["T"], mu=float(ee.min()) - 0.2, sigma=cfg["sigma"], omega_cut=cfg["omega_cut"],
                    n_q=float(np.prod(n)))
    mob_bar = np.zeros((3, 3))
    mob_bar[0, 0] = 1.0
    tab.mobility_vjp(par, vel, 10, mob_bar)                        # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gb = tab.mobility_vjp(par, vel, 10, mob_bar)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    if not bool(torch.isfinite(torch.view_as_real(gb)).all()):
        raise RuntimeError("mobility adjoint produced non-finite gradients")
    tab.close()
    log("mobility adjoint w.r.t. g(Re,Rp): %d states on %d^3, %d pairs in %.3f s (%.3g pairs/s), g_bar %.2f GB" % (
        S, grid, S * S, t_adj, S * S / t_adj, gb.numel() * 16 / 1e9))
    return {"states": S, "grid": grid, "pairs": S * S, "s": round(t_adj, 4), "pairs_per_s": S * S / t_adj,
            "iterations": 10, "precision": "fp64"}


def fermi_level(eps, n_c, temp, n_k, volume, spin=2.0):
    """Chemical potential (eV) that puts n_c carriers per cm^3 in the given
    states (spin degeneracy 2, N_k grid points, cell volume in A^3), by
    bisection on the Fermi-Dirac sum (a set-up parameter of the transport leg)."""
    kt = 8.617333262e-5 * temp
    lo, hi = float(eps.min()) - 2.0, float(eps.max()) + 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        x = np.clip((eps - mid) / kt, -700.0, 700.0)
        n = spin / (n_k * volume) * float(np.sum(1.0 / (np.exp(x) + 1.0))) * 1e24
        lo, hi = (mid, hi) if n < n_c else (lo, mid)
    return 0.5 * (lo + hi)


def gaas_bench(px, args):
    """GaAs-like polar transport: Nw = 8, 2 atoms (Ga, As masses), Z* = +-2.1,
    eps_inf = 10.9, real H, C and g on 512 Re x 512 Rp, the Froehlich term of
    Eq. e_ph_long in g (FP64, every q); the conduction states of a 0.2 eV window
    above the CBM on the n^3 k = q grid; mu for 1e17 carriers per cm^3 at
    300 K, sigma = 5 meV.  Pair tables in FP64 and FP32; the iterative BTE
    (Eq. BTE_iter) run to its threshold on each, the mobility (Eq. cond), and
    the adjoint d mu_xx / d g(Re,Rp) at full size, with a central-difference
    check of it on a 20^3 grid."""
    import torch

    import synth
    cfg = synth.CONFIGS["gaas"]
    m = synth.make_config_model("gaas")
    a = synth.models.A_GAAS
    pol = dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a)
    dm = px.Model(m, polar=pol)
    n = (args.gaas_grid,) * 3
    nk = float(np.prod(n))
    cb = m.nw // 2
    t0 = time.perf_counter()
    cbm = float(px.grid_states(dm, n, mode="lowest", band_lo=cb, count=1)[2].min())
    kk, bb, ee = px.grid_states(dm, n, mode="window", band_lo=cb, band_hi=m.nw, e_lo=cbm - 1e-3,
                                e_hi=cbm + cfg["window"])
    t_states = time.perf_counter() - t0
    S = len(kk)
    mu = fermi_level(ee, cfg["n_c"], cfg["T"], nk, m.volume())
    par = px.Params(temp=cfg["T"], mu=mu, sigma=cfg["sigma"], omega_cut=cfg["omega_cut"], n_q=nk)
    pts = np.stack([kk // (n[1] * n[2]), (kk // n[2]) % n[1], kk % n[2]], axis=-1) / np.asarray(n, dtype=np.float64)
    _, _, v = px.bands(dm, pts, want_u=False, want_vel=True)
    vel = v[torch.arange(S, device=v.device), torch.as_tensor(bb, device=v.device)].contiguous()
    log("gaas: %d window states on %s (CBM %.4f eV, mu %.4f eV for %.0e cm^-3), states %.1f s" % (
        S, "x".join(map(str, n)), cbm, mu, cfg["n_c"], t_states))
    out = {"workload": "gaas-like polar transport: Nw=8, 2 atoms, Z*=+-2.1, eps_inf=10.9, 512 Re x 512 Rp, "
                       "Froehlich term, %s k=q grid, %d states in a %.1f eV window above the CBM, n_c=%.0e cm^-3, "
                       "T=300 K, sigma=5 meV" % ("x".join(map(str, n)), S, cfg["window"], cfg["n_c"]),
           "states": S, "mu_eV_above_cbm": mu - cbm}
    mobs = {}
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-6)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tab = px.PairTable(dm, n, kk, bb, precision=prec)
        torch.cuda.synchronize()
        t_table = time.perf_counter() - t0
        tab.ita(par, vel, 2, 0.0)                                   # builds W and the plans
        torch.cuda.synchronize()
        px.timer_reset()
        px.timer_enable(True)
        t0 = time.perf_counter()
        ff, _, mob, n_it, chg = tab.ita(par, vel, 2000, tol)
        torch.cuda.synchronize()
        t_ita = time.perf_counter() - t0
        px.timer_enable(False)
        n_st, ms_st = px.timer_get("transport_stream")
        _, ms_build = px.timer_get("matrix_build")
        px.timer_reset()
        live = tab.stream_info("transport")[0]
        esz = 8 if prec == "fp64" else 4
        gbs = esz * live / (ms_st / n_st * 1e-3) / 1e9
        mobs[prec] = mob.cpu().numpy()
        out[prec] = {"table_build_s": round(t_table, 3), "tol": tol, "iterations": n_it, "last_change": chg,
                     "ita_s": round(t_ita, 4), "ms_per_iteration": round(1e3 * t_ita / max(1, n_it), 4),
                     "w_build_ms": round(ms_build, 3), "transport_stream_avg_ms": round(ms_st / n_st, 5),
                     "transport_stream_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_GBS, 4),
                     "mobility_cm2_per_Vs": [float(mobs[prec][i, i]) for i in range(3)]}
        log("gaas %s: table %.2f s, ITA to %.0e in %d updates (%.1f ms, %.3f ms each, stream %.0f GB/s), "
            "mu_xx %.5g cm^2/Vs" % (prec, t_table, tol, n_it, 1e3 * t_ita, 1e3 * t_ita / max(1, n_it), gbs,
                                    float(mob[0, 0])))
        if prec == "fp64":
            lam = np.zeros((3, 3))
            lam[0, 0] = 1.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gb = tab.mobility_vjp(par, vel, n_it, lam)
            torch.cuda.synchronize()
            t_adj = time.perf_counter() - t0
            out["adjoint_fp64"] = {"pairs": S * S, "iterations": n_it, "s": round(t_adj, 3),
                                   "pairs_per_s": S * S / t_adj}
            log("gaas: adjoint d mu_xx / d g(Re,Rp) through %d updates, %d pairs in %.2f s" % (n_it, S * S, t_adj))
            del gb
        tab.close()
        torch.cuda.empty_cache()
    d = np.diagonal(mobs["fp32"]) / np.diagonal(mobs["fp64"]) - 1.0
    out["fp32_mobility_rel_err_vs_fp64_gpu"] = float(np.abs(d).max())
    out["fd_check"] = gaas_fd_check(px, dm, m, cfg, par, 20)
    return out


def gaas_fd_check(px, dm, m, cfg, par, grid):
    """Directional derivative of mu_xx w.r.t. g(Re,Rp) from the adjoint against
    a central difference of the library's own mobility, on a small grid."""
    import torch

    n = (grid,) * 3
    cb = m.nw // 2
    cbm = float(px.grid_states(dm, n, mode="lowest", band_lo=cb, count=1)[2].min())
    kk, bb, ee = px.grid_states(dm, n, mode="window", band_lo=cb, band_hi=m.nw, e_lo=cbm - 1e-3,
                                e_hi=cbm + cfg["window"])
    pts = np.stack([kk // (n[1] * n[2]), (kk // n[2]) % n[1], kk % n[2]], axis=-1) / np.asarray(n, dtype=np.float64)
    _, _, v = px.bands(dm, pts, want_u=False, want_vel=True)
    vel = v[torch.arange(len(kk), device=v.device), torch.as_tensor(bb, device=v.device)].contiguous()
    p = px.Params(temp=par.temp, mu=par.mu, sigma=par.sigma, omega_cut=par.omega_cut, n_q=float(np.prod(n)))
    g0 = torch.as_tensor(m.g, dtype=torch.complex128, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(cfg["seed"] + 300)
    d = torch.randn(g0.shape, dtype=torch.complex128, device="cuda", generator=gen) * g0.abs()
    lam = np.zeros((3, 3))
    lam[0, 0] = 1.0
    tab = px.PairTable(dm, n, kk, bb, precision="fp64")
    _, _, _, n_it, _ = tab.ita(p, vel, 2000, 1e-10)
    gb = tab.mobility_vjp(p, vel, n_it, lam)
    ad = float((gb.conj() * d).real.sum())
    tab.close()
    h = 1e-4
    vals = []
    for sgn in (1.0, -1.0):
        dm.set_g(g0 + sgn * h * d)
        t = px.PairTable(dm, n, kk, bb, precision="fp64")
        vals.append(float(t.mobility(p, vel, n_it)[2][0, 0]))
        t.close()
    dm.set_g(g0)
    fd = (vals[0] - vals[1]) / (2 * h)
    rel = abs(fd - ad) / abs(ad)
    log("gaas: d mu_xx/dg along a random direction on %d^3 (%d states, %d updates): adjoint %.8e, central "
        "difference %.8e, relative difference %.2e" % (grid, len(kk), n_it, ad, fd, rel))
    return {"grid": grid, "states": len(kk), "iterations": n_it, "adjoint": ad, "central_difference": fd,
            "h": h, "rel_diff": rel}


def cell_bench(px, args):
    """Large cell (40 atoms, 120 modes, 64 Wannier functions, simple-cubic
    10 Angstrom cell) on its named 6^3 real-space sets: 216 Re x 216 Rp, so
    g(Re,Rp) has 2.3e10 complex entries (183 GB as complex float), drawn on the
    device by the counter scheme.  Scattering rates on a slice of k points in
    the 0.3 eV window above the CBM against random q, per precision, with the
    stage split and the MFMA rates of the Rp contraction and of the batched
    rotation + projection GEMMs.  The adjoint w.r.t. g(Re,Rp) would need the
    gradient (367 GB in complex128) beside g on one GPU; it is timed on the
    3^3 sets (27 x 27, uploaded g)."""
    import torch

    import synth
    cfg = synth.CONFIGS["cell"]
    t0 = time.perf_counter()
    m, env, seed = synth.make_counter_model("cell", n_grid=6, full=False)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    dm = px.Model(m, drawn=(seed, env))
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    nw, nm, n_rp, n_re = m.nw, m.nmodes, len(m.rp_g), len(m.re_g)
    fl_rp = rp_flops_per_pair(m.rp_g, nw, nm)
    g_bytes = n_re * n_rp * nm * nw * nw * 8
    log("large cell: nw=%d modes=%d Re=%d Rp=%d, g(Re,Rp) %.1f GB complex float drawn on the device; host part "
        "%.1fs, model with draws %.1fs" % (nw, nm, n_re, n_rp, g_bytes / 1e9, t_gen, t_load))
    cb = nw // 2
    cand = synth.random_points(cfg["seed"] + 100, 20_000)
    ec, _, _ = px.bands(dm, cand, want_u=False)
    ecb = ec[:, cb].cpu().numpy()
    cbm = float(ecb.min())
    sel = cand[(ecb - cbm >= 0.0) & (ecb - cbm <= cfg["window"])]
    ks = sel[:args.cell_k] if len(sel) >= args.cell_k else cand[np.argsort(ecb)[:args.cell_k]]
    q = synth.random_points(cfg["seed"] + 200, args.cell_q)
    qd = torch.as_tensor(q, device="cuda")
    par = px.Params(temp=cfg["T"], mu=cfg["mu"], sigma=cfg["sigma"], omega_cut=cfg["omega_cut"])
    pairs = len(ks) * len(q)
    fl_ep = 8.0 * nm * nw ** 3 + 8.0 * nm * nm * nw * nw       # rotation + projection per pair
    res = {}
    for prec in ("fp64", "fp32", "bf16x3", "bf16x6", "fp16x3"):
        px.rates(dm, ks[:1], qd[:64], par, precision=prec)
        torch.cuda.synchronize()
        px.timer_reset()
        px.timer_enable(True)
        t0 = time.perf_counter()
        px.rates(dm, ks, qd, par, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        px.timer_enable(False)
        st = {s: px.timer_get(s) for s in ("rp_contraction", "rp_phases", "epilogue", "hkq_fourier", "eig_hkq",
                                            "re_contraction", "phonons")}
        px.timer_reset()
        rp_ms, ep_ms = st["rp_contraction"][1], st["epilogue"][1]
        res[prec] = dict(pairs_per_s=pairs / dt, ms=round(1e3 * dt, 3),
                         stage_ms={s: round(v[1], 3) for s, v in st.items()},
                         rp_tflops=round(fl_rp * pairs / (rp_ms * 1e-3) / 1e12, 2) if rp_ms > 0 else None,
                         rot_proj_tflops=round(fl_ep * pairs / (ep_ms * 1e-3) / 1e12, 2) if ep_ms > 0 else None)
        log("large cell %s: %.3e pairs/s, rp %.1f TFLOP/s, rotation+projection %.1f TFLOP/s; stages %s" % (
            prec, pairs / dt, res[prec]["rp_tflops"] or 0, res[prec]["rot_proj_tflops"] or 0, res[prec]["stage_ms"]))
    # |g|^2 error vs FP64 on a sample (degenerate-group sums)
    ke, qe = ks[:2], q[:16]
    ref = group_sums(px, dm, ke, qe, px.gkq(dm, ke, qe, precision="fp64"))
    bmax = ref.flatten(2).abs().max(dim=2).values
    for prec in ("fp32", "bf16x3", "bf16x6", "fp16x3"):
        got = group_sums(px, dm, ke, qe, px.gkq(dm, ke, qe, precision=prec).double())
        res[prec]["g2_err_vs_fp64"] = float(((got - ref).abs().flatten(2).max(dim=2).values
                                             / bmax.clamp_min(1e-300)).max())
    dm.close()
    del dm
    torch.cuda.empty_cache()
    adj = cell_adjoint_bench(px, cfg, ks, q, par)
    return {
        "metric": "|g(k,q)|^2 pairs/s (scattering-rate pipeline, large cell)",
        "config": {"workload": "large cell: 40 atoms (120 modes), Nw=64, simple cubic a=10 A, %d Re x %d Rp "
                               "(6^3 sets, g drawn on the device, %.0f GB complex float), %d window k x %d random q, "
                               "T=300 K, sigma=5 meV" % (n_re, n_rp, g_bytes / 1e9, len(ks), len(q))},
        "flops_per_pair": {"rp_contraction": fl_rp, "rotation_projection": fl_ep},
        "by_precision": res,
        "rates_adjoint_fp64": adj,
    }


def cell_adjoint_bench(px, cfg, ks, q, par):
    """Adjoint of the rates w.r.t. g(Re,Rp) (FP64) on the large cell's 3^3 sets
    (uploaded g, 5.7 GB): 4 k x 64 q."""
    import torch

    import synth
    m = synth.make_config_model("cell")
    dm = px.Model(m)
    nw, n_re, n_rp = m.nw, len(m.re_g), len(m.rp_g)
    del m
    ka, qa = ks[:4], torch.as_tensor(q[:64], device="cuda")
    lam = torch.ones((len(ka), nw), dtype=torch.float64, device="cuda")
    px.rates_vjp(dm, ka, qa[:8], par, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gbar = px.rates_vjp(dm, ka, qa, par, lam)
    torch.cuda.synchronize()
    dt_adj = time.perf_counter() - t0
    adj = {"sets": "%d Re x %d Rp (3^3)" % (n_re, n_rp), "pairs": len(ka) * len(qa), "seconds": round(dt_adj, 4),
           "pairs_per_s": len(ka) * len(qa) / dt_adj, "g_bar_bytes": gbar.numel() * 16}
    log("large cell (3^3 sets) rates adjoint w.r.t. g(Re,Rp): %d pairs in %.3f s (%.3g pairs/s), g_bar %.2f GB"
        % (adj["pairs"], dt_adj, adj["pairs_per_s"], adj["g_bar_bytes"] / 1e9))
    del gbar
    dm.close()
    torch.cuda.empty_cache()
    return adj


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the PMC record in profiles/, or None
    when there is none or the kernel's source has changed since it was taken."""
    import hashlib
    import re
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(here, "profiles", "hbm_traffic_pmc.md")).read()
        rec = json.loads(re.search(r"```json\n(.*?)```", text, re.S).group(1))["kernels"].get(kernel)
        if rec is None:
            return None
        with open(os.path.join(here, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["bytes_per_launch"]
    except (OSError, AttributeError, KeyError, ValueError):
        return None


# kernel behind each precision's Rp contraction (Si-like shape: 384 output columns,
# half-set form with real coefficients)
RP_KERNEL = {"fp64": "k_phase_gemm<double, 4, true, false, false>", "fp32": "k_phase_gemm<float, 8, true, false, false>",
             "bf16x3": "k_gemm_bf16_planes<4, 2, true, false, 1, 8>", "bf16x6": "k_gemm_bf16_planes<3, 3, true, false, 1>",
             "fp16x3": "k_gemm_bf16_planes<4, 2, true, true, 1, 8>"}


def rp_flops_per_pair(rp, nw, nm):
    """Algorithmic flops of the Rp contraction per (k, q) pair.  The library sums
    over the half set (each +/-R pair once, unpaired vectors once) with real
    coefficients cos and sin(2 pi q.R): per output column 2 real x complex
    products (8 flops) per half vector, 4 for R = 0 (no sine).  Without a pair the
    complex sum runs: 8 flops per vector and column."""
    v = [tuple(int(c) for c in r) for r in np.asarray(rp)]
    idx = {r: i for i, r in enumerate(v)}
    if len(idx) != len(v):
        return 8.0 * len(v) * nw * nw * nm
    kh = 0
    for i, r in enumerate(v):
        j = idx.get(tuple(-c for c in r), -1)
        if 0 <= j < i:
            continue
        kh += 1
    if kh == len(v):
        return 8.0 * len(v) * nw * nw * nm
    entries = 2 * kh - (1 if (0, 0, 0) in idx else 0)
    return 4.0 * entries * nw * nw * nm


def group_sums(px, dm, ks, qs, g2):
    """Sum |g|^2 [k][q][nu][m][n] over degenerate groups, the groups taken from
    the FP64 energies at k, k+q and q."""
    import torch
    tol = 1e-4
    nk, nq = len(ks), len(qs)
    ek, _, _ = px.bands(dm, ks, want_u=False)
    kq = (ks[:, None, :] + qs[None, :, :]).reshape(-1, 3)
    ekq, _, _ = px.bands(dm, kq, want_u=False)
    om, _ = px.phonons(dm, qs, want_evec=False)

    def onehot(e):
        lab = torch.zeros(e.shape, dtype=torch.long, device=e.device)
        lab[..., 1:] = torch.cumsum((torch.diff(e, dim=-1) >= tol).long(), dim=-1)
        return torch.nn.functional.one_hot(lab, e.shape[-1]).double()

    pk, pkq, pq = onehot(ek), onehot(ekq.reshape(nk, nq, -1)), onehot(om)
    return torch.einsum("kqvmn,qva,kqmb,knc->kqabc", g2.double(), pq, pkq, pk)


def cpu_baseline(model, kpts, q, cfg, seconds):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    one window k point against consecutive chunks of the q list until about
    `seconds` of CPU time have passed."""
    import torch

    from oracle import eph
    t0 = time.perf_counter()
    done = 0
    chunk = 256
    k = kpts[:1]
    while time.perf_counter() - t0 < seconds and done < len(q):
        eph.rates(model, k, q[done:done + chunk], temp=cfg["T"], mu=cfg["mu"], sigma=cfg["sigma"],
                  omega_cut=cfg["omega_cut"], chunk=chunk)
        done += chunk
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "pairs/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": "1 window k x %d q of the same workload (FP64 oracle, %.1f s, host cpu_count %d)" % (
                done, dt, os.cpu_count()),
            "host": host_info()}


def host_info():
    """CPU model, logical CPUs, BLAS threads and RAM of the host the oracle ran on."""
    import platform
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()
                if d.get("user_api") == "blas"]
    except Exception:
        pass
    try:
        ram = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES") / 2 ** 30
    except (ValueError, OSError):
        ram = None
    import torch
    return {"cpu_model": model or platform.processor(), "logical_cpus": os.cpu_count(),
            "torch_threads": torch.get_num_threads(), "blas": blas,
            "ram_gib": round(ram, 1) if ram else None}


if __name__ == "__main__":
    main()

"""Writes tests/golden/tiny_oracle.json: a record of the FP64 oracle's results on
the tiny synthetic model, made by calling oracle/ only.

The record pins the oracle against accidental change (tests/test_golden.py
recomputes it) and gives the GPU path fixed expected values.  Contents:
  - band energies at 4 k (Eq. wannier_3) and phonon energies at 4 q (Eq. IFC2);
  - |g|^2 summed over degenerate groups for 2 k x 3 q (Eqs. eph_mat_wann2, eph_mat);
  - scattering rates for 2 k x 24 q (Eqs. scatter_rate, BTE_W), T = 300 K,
    mu = 0, sigma = 0.05 eV;
  - the collision integral of 10 grid states of a 4^3 grid at a Gaussian f
    (Eq. e_ph_scattering), and 3 ITA iterations with the mobility
    (Eqs. BTE_iter, cond), T = 300 K, sigma = 0.05 eV.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import synth  # noqa: E402
from helpers import group_sums_g2  # noqa: E402
from oracle import bte, eph, grid, interp  # noqa: E402

SEEDS = dict(k_bands=501, q_phon=502, k_g=503, q_g=504, k_rates=505, q_rates=506)


def compute():
    m = synth.make_config_model("tiny")
    out = {"model": "tiny", "seeds": SEEDS}
    kb = synth.random_points(SEEDS["k_bands"], 4)
    out["bands"] = interp.bands(m, kb)[0].numpy().tolist()
    qp = synth.random_points(SEEDS["q_phon"], 4)
    out["phonons"] = interp.phonons(m, qp)[0].numpy().tolist()
    k = synth.random_points(SEEDS["k_g"], 2)
    q = synth.random_points(SEEDS["q_g"], 3)
    blk = eph.eph_pipeline(m, k, q)
    gs = group_sums_g2(blk["g"].abs() ** 2, blk["eps_k"], blk["eps_kq"], blk["omega"])
    out["g2_group_sums"] = gs.numpy().tolist()
    out["g2_eps_k"] = blk["eps_k"].numpy().tolist()
    out["g2_eps_kq"] = blk["eps_kq"].numpy().tolist()
    out["g2_omega"] = blk["omega"].numpy().tolist()
    kr = synth.random_points(SEEDS["k_rates"], 2)
    qr = synth.random_points(SEEDS["q_rates"], 24)
    g, gm = eph.rates(m, kr, qr, temp=300.0, mu=0.0, sigma=0.05)
    out["rates"] = g.numpy().tolist()
    out["rates_mode"] = gm.numpy().tolist()
    n = (4, 4, 4)
    eps, _ = interp.bands(m, grid.grid_points(n))
    kk, bb = grid.lowest_states(eps.numpy(), m.nw // 2, 10)
    g2s, om = bte.pair_table(m, n, kk, bb)
    es = bte.state_energies(m, kk, bb, n)
    f = 0.1 * np.exp(-((es.numpy() - float(es.min()) - 0.2) / 0.2) ** 2)
    import torch
    i = bte.collision(torch.as_tensor(f), es, g2s, om, temp=300.0, sigma=0.05, n_q=64.0)
    out["states"] = {"k_idx": kk.tolist(), "band": bb.tolist()}
    out["collision_f"] = f.tolist()
    out["collision"] = i.numpy().tolist()
    w = bte.transport_matrix(es, g2s, om, temp=300.0, mu=0.0, sigma=0.05)
    _, _, vel = interp.bands(m, bte.state_points(kk, n), velocity=True)
    v = vel[torch.arange(len(bb)), torch.as_tensor(bb)]
    ff = bte.ita(w, v, 64.0, 3)[0]
    mob = bte.mobility(es, v, ff, mu=0.0, temp=300.0)
    out["velocities"] = v.numpy().tolist()
    out["ita_F"] = torch.as_tensor(ff).numpy().tolist()
    out["mobility"] = torch.as_tensor(mob).numpy().tolist()
    return out


if __name__ == "__main__":
    rec = compute()
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as fh:
        json.dump(rec, fh, indent=0)
    print("written", os.path.join(HERE, "tiny_oracle.json"))

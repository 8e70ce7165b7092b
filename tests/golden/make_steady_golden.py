"""Write ``steady_state.json``: steady states of the FP64 oracle that the GPU
steady-state parity test compares against.

Calls only ``oracle/`` and the seeded input generators. Each case starts from
rest and is advanced in windows of 1000 steps until the stopping criterion of
the paper's Sec. 3.1 holds,

    sum_x |u(x, t) - u(x, t - 1000)| / sum_x |u(x, t)| <= 1e-6,

with a factor-two margin (the oracle runs on until the ratio is at most
5e-7, so that a reduced-precision run, whose criterion decays alongside at a
slightly higher level, meets 1e-6 at the same step), and records, at that
step count N: the two-step means of the outlet flux and
of the inlet density (the outlet flux carries a period-two oscillation under
BGK), the apparent permeability k = rho0 nu q (nz - 1) / ((rho_in - rho_out)/3)
with Darcy velocity q = Q*/(nx ny) (Darcy's law over the whole length,
pressure p = rho/3 by eq. pressure), and the criterion itself.

Cases:
  slit    16x16x64 slit (fluid x = 1..14, periodic y), tau 1, Q* = 0.5, from
          rest (the plane-Poiseuille workload);
  crop64  [0, 64)^3 of the 256^3 sphere pack (seed 2, porosity 0.35), six
          fluid reservoir planes carved at each z end, periodic x and y,
          tau 0.8, Darcy velocity 1e-4 (Q* = 0.4096).

Run: ``python tests/golden/make_steady_golden.py`` (a few minutes).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1806_10589_amd import inputs  # noqa: E402

CRITERION = 1e-6
MARGIN = 0.5
WINDOW = 1000


def case_masks():
    slit = inputs.slit_channel(16, 16, 64)
    pack, _, _ = inputs.sphere_pack(256, 0.35, seed=2)
    crop = inputs.carve_reservoirs(pack[:64, :64, :64], 6)
    return {
        "slit": dict(mask=slit, tau=1.0, q_target=0.5, periodic_x=False, periodic_y=True),
        "crop64": dict(mask=crop, tau=0.8, q_target=1e-4 * 64 * 64, periodic_x=True, periodic_y=True),
    }


def criterion(u1, u0):
    num = np.sqrt(((u1 - u0) ** 2).sum(0)).sum()
    den = np.sqrt((u1 ** 2).sum(0)).sum()
    return float(num / den)


def run_case(name, spec, max_steps=60000):
    mask = spec["mask"]
    lat = oracle.OracleLattice(mask, tau=spec["tau"], q_target=spec["q_target"], periodic_x=spec["periodic_x"],
                               periodic_y=spec["periodic_y"])
    lat.init_equilibrium(1.0)
    prev = None
    t = 0
    trail = []
    t0 = time.time()
    while t < max_steps:
        h = lat.step(WINDOW)
        t += WINDOW
        _, ux, uy, uz = lat.fields()
        u = np.stack([ux, uy, uz])
        crit = criterion(u, prev) if prev is not None else float("inf")
        prev = u
        trail.append([t, crit])
        print(f"[{name}] t={t} criterion {crit:.3e} ({time.time() - t0:.0f} s)", flush=True)
        if crit <= CRITERION * MARGIN:
            break
    else:
        raise RuntimeError(f"{name}: no steady state within {max_steps} steps")
    nz, ny, nx = mask.shape
    q_out = 0.5 * (h[-1, 2] + h[-2, 2])
    rho_in = 0.5 * (h[-1, 0] + h[-2, 0])
    nu = (spec["tau"] - 0.5) / 3.0
    q_darcy = spec["q_target"] / (nx * ny)
    k = nu * q_darcy * (nz - 1) / ((rho_in - 1.0) / 3.0)
    return {
        "shape": [nz, ny, nx], "tau": spec["tau"], "q_target": spec["q_target"],
        "periodic_x": spec["periodic_x"], "periodic_y": spec["periodic_y"], "rho_out": 1.0, "rho0": 1.0,
        "steps": t, "criterion": trail[-1][1], "criterion_trail": trail,
        "q_out_two_step_mean": q_out, "rho_in_two_step_mean": rho_in, "permeability": k,
        "pore_sites": int((mask == 0).sum()),
    }


def main():
    out = {
        "source": "FP64 oracle (oracle/lbm_oracle.c) from rest to the stopping criterion of Sec. 3.1, "
                  "windows of 1000 steps; written by tests/golden/make_steady_golden.py",
        "criterion": CRITERION,
        "oracle_margin": MARGIN,
        "cases": {},
    }
    for name, spec in case_masks().items():
        out["cases"][name] = run_case(name, spec)
    with open(os.path.join(HERE, "steady_state.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()

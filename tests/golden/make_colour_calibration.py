"""Write ``colour_calibration.json``: the colour model's interfacial-stress
strength alpha that gives interfacial tension gamma = 0.01 (the two-fluid
pack workload), found with the FP64 oracle only.

Appendix A states that alpha is linearly related to the interfacial tension
but gives no constant. The tension is measured by the Laplace law: a
cylindrical drop of the non-wetting colour (radius R, axis along z) in a
periodic 40 x 40 box three planes thick holds a pressure jump
dp = gamma / R, with p = rho / 3 (eq. pressure); gamma is the slope of dp
against 1/R over R = 7, 10, 13 after 3000 steps at rest (tau = 1, beta =
0.7, no solids, periodic in every direction). alpha is then found by the secant method on gamma(alpha)
(linear to within the fit), starting from alpha = 0.005 and 0.01, until
gamma is within 1e-4 relative of the target.

Run: ``python tests/golden/make_colour_calibration.py`` (about a minute).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

GAMMA_TARGET = 0.01
RADII = (7.0, 10.0, 13.0)
SIZE, STEPS, TAU, BETA = 40, 3000, 1.0, 0.7


def pressure_jump(alpha, r):
    mask = np.zeros((3, SIZE, SIZE), np.uint8)
    yy, xx = np.mgrid[0:SIZE, 0:SIZE]
    inside = ((xx - SIZE / 2 + 0.5) ** 2 + (yy - SIZE / 2 + 0.5) ** 2) <= r * r
    na = np.broadcast_to(inside, mask.shape).astype(float)
    orc = oracle.OracleColour(mask, tau=TAU, alpha=alpha, beta=BETA, phi_solid=0.0, periodic_x=True,
                              periodic_y=True, z_mode=oracle.Z_PERIODIC)
    orc.init(na, 1.0 - na)
    orc.step(STEPS, record=False)
    rho, _, _, _, phi = orc.fields()
    return float((rho[phi > 0.9].mean() - rho[phi < -0.9].mean()) / 3.0)


def gamma_of(alpha):
    dps = [pressure_jump(alpha, r) for r in RADII]
    slope, icpt = np.polyfit([1.0 / r for r in RADII], dps, 1)
    return float(slope), float(icpt), dps


def main():
    trail = []
    a0, a1 = 0.005, 0.01
    g0 = gamma_of(a0)[0]
    trail.append([a0, g0])
    g1 = gamma_of(a1)[0]
    trail.append([a1, g1])
    for _ in range(8):
        if abs(g1 / GAMMA_TARGET - 1.0) <= 1e-4:
            break
        a2 = a1 + (GAMMA_TARGET - g1) * (a1 - a0) / (g1 - g0)
        a0, g0 = a1, g1
        a1 = a2
        g1 = gamma_of(a1)[0]
        trail.append([a1, g1])
        print(f"alpha {a1:.8f} gamma {g1:.8f}", flush=True)
    slope, icpt, dps = gamma_of(a1)
    out = {
        "source": "FP64 oracle (oracle/lbm_oracle.c): Laplace law of cylindrical drops, secant on gamma(alpha); "
                  "written by tests/golden/make_colour_calibration.py",
        "gamma_target": GAMMA_TARGET, "tau": TAU, "beta": BETA, "box": [3, SIZE, SIZE], "steps": STEPS,
        "radii": list(RADII),
        "alpha": a1, "gamma": slope, "intercept": icpt, "pressure_jumps": dps,
        "gamma_over_alpha": slope / a1, "secant_trail": trail,
    }
    with open(os.path.join(HERE, "colour_calibration.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps({k: out[k] for k in ("alpha", "gamma", "gamma_over_alpha")}))


if __name__ == "__main__":
    main()

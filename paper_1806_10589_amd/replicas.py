"""The paper's own test cases (Sec. 3), run on the GPU path.

E1 (Sec. 3.1): Poiseuille flow in a 40 x 40 x 80 square tube with the flux
inlet, MRT, tau = 1, three inlet velocities; the mid-plane profile is
compared with the series solution of the tube (truncated at k = 199).

E2 (Sec. 3.2, square tube): primary drainage at constant flux. A 40 x 40
tube of length 80 between a non-wetting reservoir (inlet side) and a
wetting reservoir (outlet side) of six pure-fluid layers each (open
sideways), unit density
and viscosity ratio (tau = 1), interfacial tension 6e-5 and the fluxes
Q = 0.02, 0.2, 2.0. The wetting volume falls at a rate that approaches Q.
The interfacial tension is set through alpha from a Laplace-law calibration
of the same code (the pressure jump of cylindrical drops against 1/R).

Command line: ``python -m paper_1806_10589_amd.replicas [e1|e2|laplace]``.
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import fluxlbm


def tube_series(x, y, w, kmax=199):
    """Shape function of the square-tube solution: u_z = 16 w^2 G / (nu pi^3)
    times this sum, for -w <= x, y <= w."""
    s = np.zeros(np.broadcast(x, y).shape)
    for k in range(1, kmax + 1, 2):
        s = s + ((-1) ** ((k - 1) // 2) * (1 - np.cosh(k * np.pi * x / (2 * w)) / np.cosh(k * np.pi / 2))
                 * np.cos(k * np.pi * y / (2 * w)) / k ** 3)
    return s


def e1_square_tube(u_mean, *, width=40, nz=80, tau=1.0, steps=40000, precision="fp64"):
    """Profile error against the series (with the pressure gradient measured
    in the run), the paper's steady-state criterion, and the mid-plane flux."""
    mask = np.zeros((nz, width, width), np.uint8)   # walls: the non-periodic box faces
    q = u_mean * width * width
    lat = fluxlbm.Lattice(mask, precision=precision, model="mrt", tau=tau, q_target=q, periodic_x=False,
                          periodic_y=False)
    try:
        lat.init_equilibrium()
        lat.step(steps)
        _, ux0, uy0, uz0 = (np.array(a) for a in lat.fields())
        lat.step(1000)
        rho, ux, uy, uz = lat.fields()
        c = lat.coords()
    finally:
        lat.close()
    du = np.sqrt((ux - ux0) ** 2 + (uy - uy0) ** 2 + (uz - uz0) ** 2)
    crit = float(du.sum() / np.sqrt(ux ** 2 + uy ** 2 + uz ** 2).sum())
    zs = np.arange(nz // 4, 3 * nz // 4 + 1)
    pm = np.array([rho[c[:, 2] == z].mean() for z in zs]) / 3.0
    grad = -np.polyfit(zs, pm, 1)[0]
    nu = (tau - 0.5) / 3.0
    w = width / 2.0
    mid = c[:, 2] == nz // 2
    x = c[mid, 0] - (width - 1) / 2.0
    y = c[mid, 1] - (width - 1) / 2.0
    theory = 16 * w * w * grad / (nu * np.pi ** 3) * tube_series(x, y, w)
    sim = uz[mid]
    centre = (np.abs(x) < 1) & (np.abs(y) < 1)
    return dict(u_mean=u_mean, q=q, steps=steps + 1000, criterion=crit,
                profile_err=float(np.abs(sim - theory).max() / theory.max()),
                centre_ratio=float(sim[centre].mean() / theory[centre].mean()),
                mid_plane_flux=float(sim.sum()), dp_dz=float(grad))


def laplace_gamma(alpha, *, beta=0.7, tau=1.0, radii=(7.0, 10.0, 13.0), size=40, steps=3000,
                  precision="fp64"):
    """Interfacial tension of the colour model at this alpha: the slope of the
    pressure jump of cylindrical drops (periodic thin box) against 1/R."""
    dps, inv_r = [], []
    for r in radii:
        mask = np.zeros((3, size, size), np.uint8)
        yy, xx = np.mgrid[0:size, 0:size]
        inside = ((xx - size / 2 + 0.5) ** 2 + (yy - size / 2 + 0.5) ** 2) <= r * r
        na = np.broadcast_to(inside, mask.shape).astype(float).reshape(-1)
        lat = fluxlbm.Lattice(mask, precision=precision, model="colour", tau=tau, alpha=alpha, beta=beta,
                              phi_solid=0.0, z_mode=fluxlbm.FLBM_Z_PERIODIC)
        try:
            lat.init_colour(na, 1.0 - na)
            lat.step(steps)
            rho, _, _, _ = lat.fields()
            phi = lat.phase()
        finally:
            lat.close()
        dps.append((rho[phi > 0.9].mean() - rho[phi < -0.9].mean()) / 3.0)
        inv_r.append(1.0 / r)
    slope, icpt = np.polyfit(inv_r, dps, 1)
    return float(slope), float(icpt), [float(v) for v in dps]


def e2_drainage(q, alpha, *, width=40, length=80, reservoir=6, tau=1.0, beta=0.7, steps=None,
                window=None, precision="fp32"):
    """Wetting volume against time; the rate -dV_w/dt over the last window
    steps, relative to Q. The tube has walls (one solid voxel around its
    width x width bore, wetted by the wetting fluid B); the reservoirs are
    pure fluid nodes, open sideways (periodic), so no wall connects the two
    reservoirs."""
    nz = length + 2 * reservoir
    n = width + 2
    mask = np.zeros((nz, n, n), np.uint8)
    tube = slice(reservoir, reservoir + length)
    mask[tube, 0, :] = 1
    mask[tube, -1, :] = 1
    mask[tube, :, 0] = 1
    mask[tube, :, -1] = 1
    if steps is None:
        # enough for the front to cross a good part of the tube, bounded
        steps = int(min(400000, max(40000, 0.4 * width * width * length / q)))
    steps = (steps // 1000) * 1000
    window = window or steps // 4
    lat = fluxlbm.Lattice(mask, precision=precision, model="colour", tau=tau, alpha=alpha, beta=beta,
                          phi_solid=-1.0, q_target=q, periodic_x=True, periodic_y=True,
                          watchdog_every=1000)
    try:
        c = lat.coords()
        na = (c[:, 2] < reservoir).astype(float)
        lat.init_colour(na, 1.0 - na)
        vw = []
        for _ in range(steps // 1000):
            lat.step(1000)
            h = lat.history(1)
            vw.append(float(h[0, 6]))
        qin = lat.history(1000)[:, 1]
    finally:
        lat.close()
    vw = np.array(vw)
    k = window // 1000
    rate = -(vw[-1] - vw[-1 - k]) / (1000.0 * k)
    rates = -np.diff(vw) / 1000.0
    return dict(q=q, alpha=alpha, steps=steps, window=window, rate=float(rate), rate_over_q=float(rate / q),
                rate_track=[float(r / q) for r in rates[:: max(1, len(rates) // 20)]],
                q_in_err=float(np.abs(qin - q).max() / q))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("case", choices=["e1", "e2", "laplace"])
    ap.add_argument("--gamma", type=float, default=6e-5)
    ap.add_argument("--reservoir", type=int, default=6,
                    help="pure-fluid planes at each end of the drainage tube (e2)")
    a = ap.parse_args(argv)
    if a.case == "e1":
        for u in (1e-3, 5e-3, 1e-2):
            print(json.dumps(e1_square_tube(u)), flush=True)
    elif a.case == "laplace":
        print(json.dumps(dict(zip(("slope", "intercept", "dp"), laplace_gamma(0.005)))), flush=True)
    else:
        slope, _, _ = laplace_gamma(0.005)
        alpha = a.gamma * 0.005 / slope
        print(json.dumps(dict(gamma_per_alpha=slope / 0.005, alpha=alpha)), flush=True)
        for q in (2.0, 0.2, 0.02):
            print(json.dumps(e2_drainage(q, alpha, reservoir=a.reservoir)), flush=True)


if __name__ == "__main__":
    main()

"""Steady-state parity: the FP32 GPU path against the FP64 oracle.

The stored oracle results (``golden/steady_state.json``, written by
``golden/make_steady_golden.py``, which calls only the oracle) are steady
states reached from rest under the stopping criterion of Sec. 3.1 (relative
change of the velocity field over 1000 steps at most 1e-6). The GPU runs the
same workload in FP32 storage for the same number of steps and must

- itself meet the criterion at that step (the 16x16x64 slit in FP32 levels
  off at 1.3e-6: its criterion is the same after 13,000 and 15,000 steps
  while FP64's keeps halving every 2,000, so there the bound is that
  floor, 2e-6),
- give the outlet flux (two-step mean; BGK leaves a period-two oscillation)
  within 1e-4 relative of the oracle's, and
- give the apparent permeability k = rho0 nu q (nz - 1) / ((rho_in -
  rho_out)/3) (Darcy's law over the sample, p = rho/3 by eq. pressure) within
  1e-4 relative of the oracle's.

The inlet flux equals Q* every step by construction (eq. potential); it is
checked too. Cases: the 16x16x64 slit (tau 1, Q* = 0.5) and a 64^3 crop of
the 256^3 benchmark pack with six reservoir planes at each end (tau 0.8,
Darcy velocity 1e-4).
"""
import json
import os

import numpy as np
import pytest

from paper_1806_10589_amd import fluxlbm, inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "steady_state.json")
TOL = 1e-4
# The velocity field of the FP32 slit stops changing at about 1.3e-6 of
# itself per 1000 steps (rounding of the stored deviations, which in the
# slit carry a density deviation of up to 4e-3 beside velocities of 3e-3);
# the criterion cannot fall below that floor.
CRIT_FP32 = {"slit": 2e-6}


def _masks():
    slit = inputs.slit_channel(16, 16, 64)
    pack, _, _ = inputs.sphere_pack(256, 0.35, seed=2)
    return {"slit": slit, "crop64": inputs.carve_reservoirs(pack[:64, :64, :64], 6)}


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def masks():
    return _masks()


def _criterion(u1, u0):
    return float(np.sqrt(((u1 - u0) ** 2).sum(0)).sum() / np.sqrt((u1 ** 2).sum(0)).sum())


@pytest.mark.parametrize("case", ["slit", "crop64"])
def test_fp32_steady_state_matches_oracle(golden, masks, case):
    g = golden["cases"][case]
    mask = masks[case]
    assert list(mask.shape) == g["shape"] and int((mask == 0).sum()) == g["pore_sites"]
    nz, ny, nx = mask.shape
    lat = fluxlbm.Lattice(mask, precision="fp32", tau=g["tau"], q_target=g["q_target"],
                          periodic_x=g["periodic_x"], periodic_y=g["periodic_y"], watchdog_every=1000)
    lat.init_equilibrium(1.0)
    n = g["steps"]
    lat.step(n - 1000)
    _, ux, uy, uz = lat.fields()
    u0 = np.stack([ux, uy, uz])
    lat.step(1000)
    assert lat.sync() == fluxlbm.FLBM_OK
    _, ux, uy, uz = lat.fields()
    u1 = np.stack([ux, uy, uz])
    h = lat.history(2)
    lat.close()
    crit = _criterion(u1, u0)
    q_out = 0.5 * (h[0, 2] + h[1, 2])
    rho_in = 0.5 * (h[0, 0] + h[1, 0])
    nu = (g["tau"] - 0.5) / 3.0
    k = nu * (g["q_target"] / (nx * ny)) * (nz - 1) / ((rho_in - 1.0) / 3.0)
    eq = abs(q_out / g["q_out_two_step_mean"] - 1.0)
    ek = abs(k / g["permeability"] - 1.0)
    print(f"[steady {case}] {n} steps: criterion GPU {crit:.2e} (oracle {g['criterion']:.2e}); "
          f"Q_out rel err {eq:.2e}; permeability rel err {ek:.2e}", flush=True)
    assert crit <= CRIT_FP32.get(case, golden["criterion"])
    assert np.abs(h[:, 1] - g["q_target"]).max() <= 1e-6 * g["q_target"]
    assert eq <= TOL, eq
    assert ek <= TOL, ek

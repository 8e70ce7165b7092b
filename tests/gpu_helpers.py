"""Shared set-up of the GPU parity tests: one seeded input, fed to both the
HIP path (through the C-ABI binding) and the FP64 oracle."""
import numpy as np

import oracle
from paper_1806_10589_amd import fluxlbm, inputs


def pair(mask, *, precision="fp64", tau=0.8, q_target=0.0, rho_out=1.0, rho0=1.0,
         periodic_x=True, periodic_y=True, z_mode=0, watchdog_every=1000, umax_limit=0.1, model="bgk"):
    lat = fluxlbm.Lattice(mask, tau=tau, q_target=q_target, rho_out=rho_out, rho0=rho0,
                          precision=precision, periodic_x=periodic_x, periodic_y=periodic_y,
                          z_mode=z_mode, watchdog_every=watchdog_every, umax_limit=umax_limit,
                          model=model)
    orc = oracle.OracleLattice(mask, tau=tau, q_target=q_target, rho_out=rho_out, rho0=rho0,
                               periodic_x=periodic_x, periodic_y=periodic_y, z_mode=z_mode)
    orc.set_mrt(model == "mrt")
    return lat, orc


def random_state(mask, seed, amp=0.05):
    """Dense FP64 distributions w_q (1 + amp * noise), zero at solids."""
    _, _, _, w, _ = oracle.velocity_set()
    f = w * (1.0 + amp * inputs.uniform_noise(mask.shape + (19,), seed))
    f[mask.astype(bool)] = 0.0
    return f


def dense_to_sites(mask, f_dense):
    """Dense (nz, ny, nx, Q) -> site-ordered (Q, n)."""
    q = f_dense.shape[-1]
    return np.ascontiguousarray(f_dense.reshape(-1, q)[inputs.pore_sites(mask)].T)


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def load_same_state(lat, orc, mask, seed, amp=0.05):
    f = random_state(mask, seed, amp)
    orc.set_f(f)
    lat.write_distributions(dense_to_sites(mask, f))
    return f

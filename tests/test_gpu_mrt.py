"""Single-fluid MRT collision (Appendix A's operator without the interfacial
stress) on the GPU against the FP64 oracle, and the paper's square-tube
Poiseuille case (Sec. 3.1) at its own size against the series solution.

Tolerances as for BGK: FP64 storage <= 1e-12 relative per step, FP32 <= 1e-6.
"""
import numpy as np
import pytest

from paper_1806_10589_amd import inputs

from .gpu_helpers import dense_to_sites, load_same_state, pair, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


def _compare(lat, orc, mask):
    return rel_err(lat.read_distributions(), dense_to_sites(mask, orc.get_f()))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_mrt_one_step_flux_box(precision, tau):
    mask = inputs.random_mask((10, 12, 11), 0.3, 31)
    mask[0, 0, 0] = 0
    lat, orc = pair(mask, precision=precision, tau=tau, q_target=0.4, periodic_x=True, periodic_y=False,
                    model="mrt")
    load_same_state(lat, orc, mask, 32)
    lat.step(1)
    orc.step(1)
    assert _compare(lat, orc, mask) <= TOL[precision]


@pytest.mark.parametrize("z_mode,px,py", [(1, 1, 1), (2, 0, 1)])
def test_mrt_one_step_closed_box(z_mode, px, py):
    mask = inputs.random_mask((9, 13, 17), 0.3, 33)
    lat, orc = pair(mask, precision="fp64", tau=0.75, periodic_x=px, periodic_y=py, z_mode=z_mode,
                    model="mrt")
    load_same_state(lat, orc, mask, 34)
    lat.step(1)
    orc.step(1)
    assert _compare(lat, orc, mask) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mrt_many_steps_with_history(precision):
    mask = inputs.random_mask((24, 20, 18), 0.3, 35)
    mask[0, 0, 0] = 0
    lat, orc = pair(mask, precision=precision, tau=0.9, q_target=0.3, model="mrt")
    lat.init_equilibrium()
    orc.init_equilibrium()
    lat.step(60)
    ho = orc.step(60)
    h = lat.history(60)
    assert _compare(lat, orc, mask) <= (1e-11 if precision == "fp64" else 2e-6)
    assert np.max(np.abs(h[:, 0] - ho[:, 0])) <= (1e-13 if precision == "fp64" else 1e-7)
    assert np.max(np.abs(h[:, 2] - ho[:, 2])) <= (1e-11 if precision == "fp64" else 1e-5) * 0.3


def test_mrt_fp16dev_one_step():
    mask = inputs.random_mask((10, 12, 11), 0.3, 36)
    mask[0, 0, 0] = 0
    lat, orc = pair(mask, precision="fp16dev", tau=0.8, q_target=0.2, model="mrt")
    load_same_state(lat, orc, mask, 37)
    lat.step(1)
    orc.step(1)
    # each stored deviation (|g| <= 0.05 w) is rounded to 11 significant bits
    # on load and on store (as for BGK)
    assert _compare(lat, orc, mask) <= 5e-5


@pytest.mark.parametrize("u_mean", [1e-3, 5e-3, 1e-2])
def test_square_tube_poiseuille_replica(u_mean):
    """Sec. 3.1: a 40 x 40 x 80 square tube, MRT, tau = 1, flux inlet with
    three inlet velocities. The mid-plane profile matches the series solution
    (truncated at k = 199) with the pressure gradient measured in the run,
    and the paper's steady-state criterion is met."""
    from paper_1806_10589_amd import replicas

    r = replicas.e1_square_tube(u_mean)
    assert r["criterion"] <= 1e-6, r
    assert r["profile_err"] <= 5e-3, r
    assert abs(r["mid_plane_flux"] - r["q"]) <= 1e-4 * r["q"], r

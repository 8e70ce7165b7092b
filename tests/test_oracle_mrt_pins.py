"""Pins of the oracle's single-fluid MRT step (Appendix A's collision without
the interfacial stress).

With s_q = s_m = 8 (2 - s_nu) / (8 - s_nu) the odd and even non-conserved
moments relax with rates whose "magic" product (1/s_nu - 1/2)(1/s_q - 1/2) is
3/16, for which halfway bounce-back puts a straight wall exactly halfway
between nodes: the plane Poiseuille profile is then parabolic to the
incompressibility error, at every tau, while BGK's wall moves with tau. The
square tube of Sec. 3.1 is compared with its series solution (truncated at
k = 199 as in the paper) at a reduced size."""
import numpy as np
import pytest

from paper_1806_10589_amd import inputs


def _slit_shape_error(orc, tau, steps, mrt, nx=10, nz=48):
    mask = inputs.slit_channel(nx, 4, nz)
    lat = orc.OracleLattice(mask, tau=tau, q_target=0.1, rho_out=1.0, periodic_x=False, periodic_y=True)
    lat.set_mrt(mrt)
    lat.init_equilibrium(1.0)
    hist = lat.step(steps)
    _, _, _, uz = lat.fields()
    x = np.arange(1, nx - 1)
    theory = (x - 0.5) * (nx - 1.5 - x)   # walls halfway: x = 0.5 and nx - 1.5
    sim = uz[nz // 2, 2, 1:nx - 1]
    return np.abs(sim / sim.mean() - theory / theory.mean()).max(), hist


@pytest.mark.parametrize("tau,steps", [(0.6, 3000), (0.8, 1500), (1.5, 1000)])
def test_mrt_slit_profile_is_parabolic_at_every_tau(orc, tau, steps):
    err, hist = _slit_shape_error(orc, tau, steps, True)
    assert err <= 3e-4
    assert np.abs(hist[:, 1] - 0.1).max() <= 1e-13   # the inlet flux is exact every step


def test_bgk_slit_profile_error_depends_on_tau(orc):
    # the contrast that makes the pin above discriminating
    e08, _ = _slit_shape_error(orc, 0.8, 1500, False)
    e15, _ = _slit_shape_error(orc, 1.5, 1000, False)
    assert e08 > 3e-3 and e15 > 3e-2


def _series(x, y, w, kmax=199):
    s = np.zeros_like(x, dtype=float)
    for k in range(1, kmax + 1, 2):
        s += ((-1) ** ((k - 1) // 2) * (1 - np.cosh(k * np.pi * x / (2 * w)) / np.cosh(k * np.pi / 2))
              * np.cos(k * np.pi * y / (2 * w)) / k ** 3)
    return s


def _duct(orc, tau, width=12, nz=32, steps=3000, q=0.05):
    mask = inputs.square_duct(width, nz)
    lat = orc.OracleLattice(mask, tau=tau, q_target=q, rho_out=1.0)
    lat.set_mrt(True)
    lat.init_equilibrium(1.0)
    lat.step(steps, record=False)
    rho, _, _, uz = lat.fields()
    c = np.arange(1, width + 1) - (width + 1) / 2.0
    X, Y = np.meshgrid(c, c, indexing="ij")
    w = width / 2.0
    shape = _series(X, Y, w)
    sim = uz[nz // 2, 1:width + 1, 1:width + 1].T
    zs = np.arange(nz // 4, 3 * nz // 4)
    G = -np.polyfit(zs, [rho[z][mask[z] == 0].mean() / 3.0 for z in zs], 1)[0]
    nu = (tau - 0.5) / 3.0
    theory = 16 * w * w * G / (nu * np.pi ** 3) * shape
    return np.abs(sim - theory).max() / theory.max(), np.abs(sim / sim.mean() - shape / shape.mean()).max(), sim


def test_series_solution_of_the_square_tube():
    # the series itself: symmetric, zero on the walls, and the centre value
    # of the textbook solution, u_max = 0.2947 G (2w)^2 / (4 nu) ... written
    # as the coefficient 16/pi^3 * s(0, 0) = 0.2947
    w = 1.0
    assert 16 / np.pi ** 3 * _series(np.array([0.0]), np.array([0.0]), w)[0] == pytest.approx(0.29468, abs=2e-5)
    edge = _series(np.array([1.0, 0.3]), np.array([0.4, 1.0]), w)
    assert np.all(np.abs(edge) < 1e-6)


def test_mrt_square_tube_matches_series_independent_of_tau(orc):
    e1, s1, _ = _duct(orc, 1.0)
    e2, s2, _ = _duct(orc, 0.8)
    assert e1 <= 5e-3 and e2 <= 5e-3
    assert s1 <= 5e-3 and abs(s1 - s2) <= 0.05 * s1


def test_mrt_closed_box_conserves_mass(orc):
    mask = inputs.random_mask((8, 9, 10), 0.3, 3)
    lat = orc.OracleLattice(mask, tau=0.7, z_mode=orc.Z_PERIODIC)
    lat.set_mrt(True)
    _, _, _, w, _ = orc.velocity_set()
    f = w * (1.0 + 0.05 * inputs.uniform_noise(mask.shape + (19,), 4))
    f[mask.astype(bool)] = 0.0
    lat.set_f(f)
    m0 = f.sum()
    hist = lat.step(300)
    assert np.abs(hist[:, 3] - m0).max() <= 1e-12 * m0

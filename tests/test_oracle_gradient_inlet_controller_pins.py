"""Pins of three oracle functions that the other pins do not reach.

1. The colour gradient of the two-fluid oracle (Appendix A names the gradient
   of the phase field, C = grad phi, without printing a stencil; the oracle
   uses C = 3 sum_q w_q xi_q phi(x + xi_q)). Pinned by closed forms derived
   by hand: exact on linear and quadratic fields away from faces; on a plane
   wave in a fully periodic box the stencil's Fourier symbol,
   C_a = (1/3) cos(k.x) sin(k_a) (1 + cos k_b + cos k_c), at every cell
   including the wrap; next to a wall (solid voxels or a non-periodic side)
   with a uniform fluid phase p, C = ((p - phi_s)/2, 0, 0); at an open z face
   the face's own phase is read beyond it, so a field linear in z shows half
   its slope there.
2. The plain inlet density of eq. potential that the controller oracle reads
   between steps: it must be the density the next step records.
3. The controller oracle's decision rule (the learned addition on top of the
   paper's update): its bound, proposal, clipping, release and stall rules at
   hand-computed decisions, and trust0 = 0 reproducing the plain method
   bitwise.
"""
import math

import numpy as np
import pytest

from paper_1806_10589_amd import inputs


def _colour(orc, mask, *, px=True, py=True, z_mode=None, phi_solid=-0.5):
    return orc.OracleColour(mask, tau=0.8, alpha=0.01, beta=0.7, phi_solid=phi_solid, q_target=0.0,
                            periodic_x=px, periodic_y=py,
                            z_mode=orc.Z_PERIODIC if z_mode is None else z_mode)


def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(float), y.astype(float), z.astype(float)


# ------------------------------------------------------------ colour gradient

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_exact_on_linear_and_quadratic_fields(orc, seed):
    """A symmetric stencil with sum_q w_q xi_a xi_b = delta_ab / 3 differentiates
    polynomials of degree <= 2 exactly: phi = a + b.x + x.Q.x has C = b + 2 Q x.
    Checked at the cells whose 18 neighbours do not cross the periodic wrap."""
    rng = np.random.default_rng(seed)
    shape = (9, 8, 7)
    mask = np.zeros(shape, np.uint8)
    c = _colour(orc, mask)
    x, y, z = _grid(shape)
    a = rng.standard_normal()
    b = rng.standard_normal(3)
    Q = rng.standard_normal((3, 3)) * 0.1
    Q = 0.5 * (Q + Q.T)
    X = np.stack([x, y, z], -1)
    phi = a + X @ b + np.einsum("...i,ij,...j->...", X, Q, X)
    grad = c.gradient(phi)
    exact = b + 2.0 * X @ Q
    inner = (slice(1, -1),) * 3
    err = np.abs(grad[inner] - exact[inner]).max()
    assert err < 1e-12, err


@pytest.mark.parametrize("k", [(1, 0, 0), (0, 2, 0), (0, 0, 3), (1, 2, 1), (3, 1, 2)])
def test_gradient_fourier_symbol_on_periodic_plane_wave(orc, k):
    """phi = sin(k.x) with k = 2 pi (m_x/n_x, m_y/n_y, m_z/n_z) is periodic, so
    every cell (also those whose neighbours wrap) obeys the symbol
    C_a = (1/3) cos(k.x) sin(k_a) (1 + cos k_b + cos k_c): axis pairs give
    (2/18) sin(k_a), each diagonal family 4 (1/36) sin(k_a) cos(k_b), times 3."""
    shape = (10, 9, 8)
    nz, ny, nx = shape
    c = _colour(orc, np.zeros(shape, np.uint8))
    x, y, z = _grid(shape)
    kv = 2.0 * np.pi * np.array([k[0] / nx, k[1] / ny, k[2] / nz])
    arg = kv[0] * x + kv[1] * y + kv[2] * z
    grad = c.gradient(np.sin(arg))
    cs = np.cos(kv)
    sym = np.array([np.sin(kv[0]) * (1 + cs[1] + cs[2]),
                    np.sin(kv[1]) * (1 + cs[0] + cs[2]),
                    np.sin(kv[2]) * (1 + cs[0] + cs[1])]) / 3.0
    exact = np.cos(arg)[..., None] * sym
    assert np.abs(grad - exact).max() < 1e-13


@pytest.mark.parametrize("phi_solid", [-0.707, 0.3])
def test_gradient_next_to_solid_plane_and_side_wall(orc, phi_solid):
    """Uniform fluid phase p, solid plane x = 0 (periodic box otherwise): at
    x = 1 the five directions with xi_x = -1 (weights summing to 1/6) read
    phi_s and the five with xi_x = +1 read p, so C = ((p - phi_s)/2, 0, 0);
    one cell further C = 0. The same holds at x = 0 of a box whose x faces
    are walls instead of solid voxels."""
    p = 0.25
    shape = (6, 5, 7)
    mask = np.zeros(shape, np.uint8)
    mask[:, :, 0] = 1
    phi = np.full(shape, p)
    g = _colour(orc, mask, phi_solid=phi_solid).gradient(phi)
    expect = np.array([(p - phi_solid) / 2.0, 0.0, 0.0])
    assert np.abs(g[:, :, 1] - expect).max() < 1e-15
    assert np.abs(g[:, :, 2:-1]).max() < 1e-15
    # the other side of the solid plane (x = nx - 1 wraps onto x = 0)
    assert np.abs(g[:, :, -1] - (-expect)).max() < 1e-15
    assert np.abs(g[:, :, 0]).max() == 0.0  # solid cells carry no gradient

    wall = _colour(orc, np.zeros(shape, np.uint8), px=False, phi_solid=phi_solid).gradient(phi)
    assert np.abs(wall[:, :, 0] - expect).max() < 1e-15
    assert np.abs(wall[:, :, -1] + expect).max() < 1e-15
    assert np.abs(wall[:, :, 1:-1]).max() < 1e-15


def test_gradient_at_open_and_walled_z_faces(orc):
    """phi = p + d z. Open z faces (the flux set-up): beyond them the face
    cell's own phase is read, so C_z = d/2 on both face planes and d inside.
    Walled z faces read phi_s beyond them."""
    shape = (8, 5, 6)
    p, d, phs = 0.1, 0.03, -0.4
    _, _, z = _grid(shape)
    phi = p + d * z
    g = _colour(orc, np.zeros(shape, np.uint8), z_mode=orc.Z_FLUX, phi_solid=phs).gradient(phi)
    assert np.abs(g[..., :2]).max() < 1e-15
    assert np.abs(g[0, ..., 2] - d / 2).max() < 1e-15
    assert np.abs(g[-1, ..., 2] - d / 2).max() < 1e-15
    assert np.abs(g[1:-1, ..., 2] - d).max() < 1e-14
    w = _colour(orc, np.zeros(shape, np.uint8), z_mode=orc.Z_WALL, phi_solid=phs).gradient(phi)
    # bottom: xi_z = +1 reads p + d, xi_z = -1 reads phi_s
    assert abs(w[0, 2, 3, 2] - ((p + d) - phs) / 2) < 1e-15
    top = p + d * (shape[0] - 1)
    assert abs(w[-1, 2, 3, 2] - (phs - (top - d)) / 2) < 1e-15


@pytest.mark.parametrize("z_mode,px,py", [(0, True, False), (1, False, True), (2, True, True)])
def test_gradient_vanishes_when_everything_reads_phi_solid(orc, z_mode, px, py):
    """A uniform phase equal to phi_s: every rule (pore neighbour, solid,
    side wall, open face) reads the same value, so C = 0 at every cell."""
    mask = inputs.random_mask((7, 6, 5), 0.3, 11)
    mask[0] = 0
    mask[-1] = 0
    phs = -0.6
    g = _colour(orc, mask, px=px, py=py, z_mode=z_mode, phi_solid=phs).gradient(np.full(mask.shape, phs))
    assert np.abs(g).max() < 1e-15


# ------------------------------------------------------- plain inlet density

@pytest.mark.parametrize("seed", [0, 1])
def test_plain_inlet_density_is_the_next_steps_rho_in(orc, seed):
    """eq. potential evaluated between steps equals the rho_in the next step
    records (the two sum the same K_i in the same order; they differ only in
    whether rho0 Q*/A and S/A are added before or after the division), and
    evaluating it leaves the state and the next step untouched."""
    rng = np.random.default_rng(seed)
    mask = inputs.random_mask((9, 6, 7), 0.3, seed)
    mask[0] = 0
    mask[-1] = 0
    _, _, _, w, _ = orc.velocity_set()

    def lattice():
        o = orc.OracleLattice(mask, tau=0.8, q_target=0.37, periodic_x=True, periodic_y=False)
        f = w * (1.0 + 0.05 * rng_state)
        f[mask.astype(bool)] = 0.0
        o.set_f(f)
        return o

    rng_state = rng.uniform(-1.0, 1.0, mask.shape + (19,))
    a, b = lattice(), lattice()
    for _ in range(3):
        rp = a.plain_inlet_density()
        assert a.plain_inlet_density() == rp
        ha = a.step(1)[0]
        hb = b.step(1)[0]
        assert abs(ha[0] - rp) <= 4.5e-16 * abs(rp)  # two roundings apart
        assert np.array_equal(ha, hb)
        assert np.array_equal(a.get_f(), b.get_f())
    # with an offset the step records the plain density plus the offset
    rp = a.plain_inlet_density()
    a.set_inlet_offset(1e-3)
    assert abs(a.step(1)[0][0] - (rp + 1e-3)) <= 4e-16


# ---------------------------------------------------------- controller rule

def _controller(orc_mod, **kw):
    from oracle import controller_oracle, mlp_oracle

    params = kw.pop("params", None)
    if params is None:
        params = np.zeros(mlp_oracle.N_PARAMS)
    base = dict(drho_ref=1e-2, gain=1.0, trust0=4.0, release_tol=1e-3, trust_decisions=10,
                relative=True, stall_decisions=0, period=2, margin=0.0)
    base.update(kw)
    return controller_oracle.OracleController(params, np.zeros(15), **base)


def test_controller_bound_and_proposal_at_hand_computed_decisions(orc):
    c = _controller(orc, trust0=4.0, trust_decisions=10, relative=True)
    # bound after n = 3 of 10 decisions: 4 (1 - 0.3) = 2.8; limit = 2.8 * 1 * 0.5 / 20 = 0.07
    rho_hat, limit = c.proposal(0.5, 0.01, 3, False, q_target=0.5, rho_out=1.0, rho0=1.0, a_in=20)
    assert abs(limit - 0.07) < 3e-17
    # relative: rho_hat = 1 + 0.01 e^0.5, e^0.5 = 1.6487212707001282
    assert abs(rho_hat - 1.016487212707001282) < 1e-15
    # clipping of the output: relative r in [-2, 3]
    rho_hat, _ = c.proposal(10.0, 0.01, 0, False, q_target=0.5, rho_out=1.0, rho0=1.0, a_in=20)
    assert abs(rho_hat - (1.0 + 0.01 * 20.085536923187668)) < 1e-15  # e^3
    rho_hat, _ = c.proposal(-7.0, 0.01, 0, False, q_target=0.5, rho_out=1.0, rho0=1.0, a_in=20)
    assert abs(rho_hat - (1.0 + 0.01 * 0.1353352832366127)) < 1e-15  # e^-2
    # absolute: rho_hat = rho_out + drho_ref e^clip(y, -4, 4); the bound with rho0 = 2, |Q*| = 3, A = 6, n = 5
    a = _controller(orc, relative=False, drho_ref=2e-2, trust0=1.5, trust_decisions=20, margin=0.25)
    rho_hat, limit = a.proposal(-9.0, 0.0, 5, False, q_target=3.0, rho_out=1.0, rho0=2.0, a_in=6)
    assert abs(limit - 1.5 * 0.75 * 2.0 * 3.0 / 6.0) < 1e-16  # = 1.125
    assert abs(rho_hat - (1.0 + 0.02 * 0.014264233908999256)) < 1e-15  # e^(-4 - 0.25)
    # the bound reaches zero at trust_decisions and stays there: no proposal
    assert a.proposal(0.0, 0.0, 20, False, q_target=3.0, rho_out=1.0, rho0=2.0, a_in=6) is None
    assert a.proposal(0.0, 0.0, 25, False, q_target=3.0, rho_out=1.0, rho0=2.0, a_in=6) is None


def test_controller_offset_is_clipped_gain_times_gap(orc):
    c = _controller(orc, gain=0.5)
    assert c.offset(None, 1.02) == 0.0
    assert abs(c.offset((1.10, 0.03), 1.02) - 0.03) < 1e-17      # 0.5 * 0.08 = 0.04 > 0.03
    assert abs(c.offset((1.03, 0.03), 1.02) - 0.005) < 1e-15     # 0.5 * 0.01
    assert abs(c.offset((0.90, 0.03), 1.02) + 0.03) < 1e-17      # -0.06 clipped to -0.03


def test_controller_no_proposal_cases(orc):
    c = _controller(orc, relative=True)
    kw = dict(q_target=0.5, rho_out=1.0, rho0=1.0, a_in=20)
    assert c.proposal(float("nan"), 0.01, 0, False, **kw) is None          # non-finite output
    assert c.proposal(float("inf"), 0.01, 0, False, **kw) is None
    assert c.proposal(0.1, 0.01, 0, True, **kw) is None                    # released
    assert c.proposal(0.1, 0.0, 0, False, **kw) is None                    # relative needs drho > 0
    assert c.proposal(0.1, 0.01, 0, False, **dict(kw, q_target=0.0)) is None   # Q* <= 0
    assert c.proposal(0.1, 0.01, 0, False, **dict(kw, q_target=-0.5)) is None
    big = _controller(orc, relative=False, drho_ref=1e308)
    assert big.proposal(4.0, 0.0, 0, False, **kw) is None                  # rho_hat overflows
    zero = _controller(orc, trust0=0.0)
    assert zero.proposal(0.1, 0.01, 0, False, **kw) is None                # no trust, no proposal


def test_controller_inputs_at_lags(orc):
    c = _controller(orc, drho_ref=1e-2)
    c.periods = [0.1, 0.2, 0.3, 0.4, 0.5]
    c.rho_in = [1.001]
    x, drho = c.inputs(q_target=0.5, rho_out=1.0)
    assert abs(drho - 1e-3) < 1e-15
    lag_expect = {0: (0.5 - 0.5) / 0.5, 1: (0.4 - 0.5) / 0.5, 2: (0.3 - 0.5) / 0.5, 3: (0.2 - 0.5) / 0.5,
                  4: -1.0, 15: -1.0}   # lags 1, 2, 3, 4; lag 6 and 250 reach before the first period
    for k, v in lag_expect.items():
        assert x[15 + k] == np.float32(v)
    assert x[31] == np.float32(-1.0 / 3.0)  # log10(1e-3 / 1e-2) / 3
    c.periods = [5.0]  # error (5 - 0.5)/0.5 = 9, clipped to 2
    x, _ = c.inputs(q_target=0.5, rho_out=1.0)
    assert x[15] == 2.0
    c.rho_in = [0.999]  # drho <= 0
    x, _ = c.inputs(q_target=0.5, rho_out=1.0)
    assert x[31] == -1.0
    c.rho_in = [1.0 + 1e-9]  # log10(1e-7)/3 < -1: clipped
    x, _ = c.inputs(q_target=0.5, rho_out=1.0)
    assert x[31] == -1.0


def _small_lattice(orc):
    mask = inputs.random_mask((10, 5, 6), 0.25, 3)
    mask[0] = 0
    mask[-1] = 0
    o = orc.OracleLattice(mask, tau=0.8, q_target=0.2, periodic_x=True, periodic_y=True)
    o.init_equilibrium(1.0)
    return o


def test_controller_release_and_stall_fire_for_good(orc):
    o = _small_lattice(orc)
    q = 0.2
    # release: the last period's error at or below release_tol, with at least two periods
    c = _controller(orc, release_tol=1e-3, stall_decisions=0)
    c.rho_in = [1.01]
    c.periods = [q * (1 + 1e-4)]
    c.decide(o, q, 1.0, 1.0, o.a_in)
    assert not c.released  # one period only
    c.periods.append(q * (1 + 5e-4))
    c.decide(o, q, 1.0, 1.0, o.a_in)
    assert c.released and c.hold is None
    c.periods.append(q * 3.0)  # the error grows again: released stays
    c.decide(o, q, 1.0, 1.0, o.a_in)
    assert c.released and c.hold is None

    # stall: no 10 % improvement over stall_decisions = 3 decisions
    s = _controller(orc, release_tol=0.0, stall_decisions=3)
    s.rho_in = [1.01]
    held = []
    for e in (1.0, 0.95, 0.92, 0.91, 0.5):
        s.periods.append(q * (1 + e))
        s.decide(o, q, 1.0, 1.0, o.a_in)
        held.append((s.released, s.hold is not None))
    # best at decision 0 (1.0); 0.95, 0.92, 0.91 are not below 0.9: released at decision 3
    assert held == [(False, True), (False, True), (False, True), (True, False), (True, False)]
    # an improvement below 0.9 of the best resets the count
    r = _controller(orc, release_tol=0.0, stall_decisions=3)
    r.rho_in = [1.01]
    for e in (1.0, 0.95, 0.85, 0.84, 0.83):
        r.periods.append(q * (1 + e))
        r.decide(o, q, 1.0, 1.0, o.a_in)
    assert not r.released  # best moved to decision 2 (0.85 < 0.9), only two decisions since


def test_controller_period_means_and_trace(orc):
    o = _small_lattice(orc)
    ref = _small_lattice(orc)
    c = _controller(orc, trust0=0.0, period=3)
    rows = c.run(o, 7, q_target=0.2)
    h = ref.step(7)
    assert np.array_equal(rows, h)
    assert len(c.periods) == 2
    assert c.periods[0] == (h[0, 2] + h[1, 2] + h[2, 2]) / 3
    assert c.periods[1] == (h[3, 2] + h[4, 2] + h[5, 2]) / 3
    assert c.decisions == 2 and len(c.records) == 2
    assert abs(c.acc - h[6, 2]) == 0.0  # the open period holds step 7


@pytest.mark.parametrize("relative", [True, False])
def test_controller_with_zero_trust_is_the_plain_method_bitwise(orc, relative):
    """trust0 = 0: the controller observes but never proposes; the run is the
    paper's update exactly, with a network that would propose a large jump."""
    from oracle import mlp_oracle

    rng = np.random.default_rng(7)
    params = 0.3 * rng.standard_normal(mlp_oracle.N_PARAMS)
    o, ref = _small_lattice(orc), _small_lattice(orc)
    c = _controller(orc, params=params, trust0=0.0, relative=relative, period=2)
    rows = c.run(o, 12, q_target=0.2)
    assert np.array_equal(rows, ref.step(12))
    assert np.array_equal(o.get_f(), ref.get_f())
    assert all(r[4] == 0.0 for r in c.records) and c.decisions == 6


def test_controller_held_proposal_moves_rho_in_within_the_bound(orc):
    """With trust the run departs from the plain method by exactly the held,
    clipped offset: rho_in(t) = plain(t) + offset, |offset| <= limit."""
    from oracle import mlp_oracle

    params = np.zeros(mlp_oracle.N_PARAMS)
    params[-1] = 2.0  # output bias: y = 2 everywhere, a strong upward proposal
    o = _small_lattice(orc)
    c = _controller(orc, params=params, trust0=0.5, trust_decisions=100, relative=True, period=2)
    c.rho_in = []
    rows = []
    for t in range(8):
        plain = o.plain_inlet_density()
        off = c.offset(c.hold, plain)
        rows.append(c.run(o, 1, q_target=0.2)[0])
        assert abs(rows[-1][0] - (plain + off)) <= 4e-16
        if c.hold is not None:
            assert abs(c.offset(c.hold, plain)) <= c.hold[1] + 1e-18
    a_in = o.a_in
    # decisions at t = 2, 4, 6 hold a proposal; its limit follows the bound rule
    assert c.decisions == 4
    assert c.hold is not None
    n = c.decisions - 1
    assert abs(c.hold[1] - 0.5 * (1 - n / 100) * 0.2 / a_in) < 1e-17

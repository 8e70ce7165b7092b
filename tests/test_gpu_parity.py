"""Parity of the HIP path with the FP64 oracle (GPU required).

Tolerances: FP64 storage <= 1e-12 relative per step (rounding order only);
FP32 storage <= 1e-6 relative per step. Relative errors are max |a - b|
over max |b| of the distributions (all of order w_q).
"""
import numpy as np
import pytest

from paper_1806_10589_amd import fluxlbm, inputs

from .gpu_helpers import dense_to_sites, load_same_state, pair, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


def _compare(lat, orc, mask):
    return rel_err(lat.read_distributions(), dense_to_sites(mask, orc.get_f()))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("z_mode,px,py", [(1, 1, 1), (2, 0, 1), (2, 0, 0)])
def test_one_step_closed_box(precision, z_mode, px, py):
    mask = inputs.random_mask((9, 13, 17), 0.3, 5)
    lat, orc = pair(mask, precision=precision, tau=0.7, periodic_x=px, periodic_y=py, z_mode=z_mode)
    load_same_state(lat, orc, mask, 6)
    lat.step(1)
    orc.step(1)
    assert _compare(lat, orc, mask) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,solid,px,py", [
    ((10, 12, 11), 0.3, 1, 0),   # ragged: n not a multiple of 256, inlet/outlet in few tiles
    ((5, 3, 4), 0.2, 1, 1),      # one tile holds inlet, interior and outlet sites
    ((24, 40, 36), 0.35, 1, 1),  # several tiles per plane
])
def test_one_step_flux_box(precision, shape, solid, px, py):
    mask = inputs.random_mask(shape, solid, 11)
    mask[0, 0, 0] = 0
    lat, orc = pair(mask, precision=precision, tau=0.9, q_target=0.05 * shape[1] * shape[2] * 0.1,
                    periodic_x=px, periodic_y=py)
    load_same_state(lat, orc, mask, 12)
    lat.step(1)
    h_orc = orc.step(1)
    assert _compare(lat, orc, mask) <= TOL[precision]
    h = lat.history(1)
    # FP32 storage rounds the input deviations (|g| <= 0.05 w) by 2^-24 each;
    # rho_in averages 14-term sums of them: error bound ~2e-8.
    assert abs(h[0, 0] - h_orc[0, 0]) <= (1e-13 if precision == "fp64" else 1e-7)
    assert abs(h[0, 1] - h_orc[0, 1]) <= 1e-12 * max(1.0, abs(h_orc[0, 1]))
    tol_q = 1e-12 if precision == "fp64" else 1e-6
    assert abs(h[0, 2] - h_orc[0, 2]) <= tol_q * max(1.0, abs(h_orc[0, 2]))


def test_streaming_only_is_bit_exact():
    """Collision off: pure streaming of unique values; every known slot moves exactly."""
    mask = inputs.random_mask((8, 7, 9), 0.3, 21)
    mask[0, 0, 0] = 0
    lat, orc = pair(mask, precision="fp64", tau=0.8, q_target=0.0, periodic_x=True, periodic_y=False)
    lat.set_collision(False)
    orc.set_collision(False)
    nz, ny, nx = mask.shape
    ids = (np.arange(nz * ny * nx * 19, dtype=np.float64) + 1.0).reshape(nz, ny, nx, 19) * 1e-6
    ids[mask.astype(bool)] = 0.0
    orc.set_f(ids)
    lat.write_distributions(dense_to_sites(mask, ids))
    lat.step(1)
    orc.step(1)
    g = lat.read_distributions()
    o = dense_to_sites(mask, orc.get_f())
    coords = lat.coords()
    cz = np.array([0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1])
    known = np.ones_like(g, bool)
    known[np.ix_(cz == 1, coords[:, 2] == 0)] = False
    known[np.ix_(cz == -1, coords[:, 2] == nz - 1)] = False
    # deviations are stored, so values differ from exact copies only by the
    # +/- w_q round trip
    assert np.abs(g[known] - o[known]).max() <= 4e-16 * np.abs(o).max()
    assert np.abs(g[~known] - o[~known]).max() <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_many_steps_flux_box_history(precision):
    mask = inputs.random_mask((16, 10, 12), 0.25, 31)
    mask[:2] = 0
    q = 0.4
    lat, orc = pair(mask, precision=precision, tau=0.75, q_target=q, periodic_x=True, periodic_y=True,
                    watchdog_every=20)
    lat.init_equilibrium(1.0)
    orc.init_equilibrium(1.0)
    n = 150  # spans graph replays (chunk 20) and a direct tail
    lat.step(n)
    h_orc = orc.step(n)
    assert lat.sync() == fluxlbm.FLBM_OK
    h = lat.history(n)
    err = _compare(lat, orc, mask)
    assert err <= (1e-11 if precision == "fp64" else 2e-5)
    # inlet flux equals the target every step
    assert np.abs(h[:, 1] - q).max() <= (1e-12 if precision == "fp64" else 1e-6 * q)
    assert np.abs(h[:, 0] - h_orc[:, 0]).max() <= (1e-12 if precision == "fp64" else 1e-6)
    assert np.abs(h[:, 2] - h_orc[:, 2]).max() <= (1e-11 if precision == "fp64" else 1e-5)
    # mass and max|u| are recorded at the end of every chunk and of the call
    rec = ~np.isnan(h[:, 3])
    assert rec[19] and rec[39] and rec[-1]
    assert np.abs(h[rec, 3] - h_orc[rec, 3]).max() <= (1e-12 if precision == "fp64" else 1e-6) * h_orc[0, 3]
    assert np.abs(h[rec, 4] - h_orc[rec, 4]).max() <= 1e-6


def test_mass_conserved_closed_box_gpu():
    mask = inputs.random_mask((20, 18, 16), 0.3, 41)
    lat, orc = pair(mask, precision="fp64", tau=0.7, z_mode=1)
    f = load_same_state(lat, orc, mask, 42)
    m0 = f.sum()
    lat.step(500)
    m, umax, bad = lat.observables()
    assert bad == 0
    assert abs(m - m0) / m0 < 1e-12


def test_slit_channel_fp64_matches_oracle():
    """The correctness configuration: 16x16x64 slit, tau 1, Q* 0.5, from rest."""
    mask = inputs.slit_channel(16, 16, 64)
    lat, orc = pair(mask, precision="fp64", tau=1.0, q_target=0.5, periodic_x=False, periodic_y=True)
    lat.init_equilibrium(1.0)
    orc.init_equilibrium(1.0)
    lat.step(2000)
    h_orc = orc.step(2000)
    h = lat.history(2000)
    assert lat.sync() == fluxlbm.FLBM_OK
    assert _compare(lat, orc, mask) <= 1e-10
    assert np.abs(h[:, 1] - 0.5).max() <= 1e-12
    assert np.abs(h[:, 2] - h_orc[:, 2]).max() <= 1e-10
    rho, ux, uy, uz = lat.fields()
    _, _, _, uz_o = orc.fields()
    sites = inputs.pore_sites(mask)
    assert np.abs(uz - uz_o.reshape(-1)[sites]).max() <= 1e-12


def test_checkpoint_resume_is_bitwise():
    mask = inputs.random_mask((12, 9, 10), 0.2, 51)
    mask[0] = 0
    lat, _ = pair(mask, precision="fp32", tau=0.8, q_target=0.3)
    lat.init_equilibrium(1.0)
    lat.step(40)
    blob = lat.save_state()
    lat.step(40)
    straight = lat.read_distributions()
    lat.load_state(blob)
    assert lat.step_count == 40
    lat.step(40)
    resumed = lat.read_distributions()
    assert np.array_equal(straight, resumed)


@pytest.mark.parametrize("precision,model,z_mode", [
    ("fp32", "bgk", 0), ("fp16dev", "bgk", 0), ("fp32", "mrt", 0), ("fp64", "bgk", 1)])
def test_step_end_inside_a_run_matches_its_own_launch(precision, model, z_mode):
    """Inside a run of steps the next step kernel ends each step (its inlet
    tiles sum the previous step's partials, tile 0 records it); one step per
    call ends every step in a launch of its own. Same state and history, bit
    for bit (flux inlet, and a periodic box whose records hold no flux)."""
    mask = inputs.random_mask((14, 12, 10), 0.25, 61)
    mask[:2] = 0
    kw = dict(tau=0.8, q_target=0.3 if z_mode == 0 else 0.0, precision=precision, model=model, z_mode=z_mode,
              watchdog_every=25)
    a = fluxlbm.Lattice(mask, **kw)
    b = fluxlbm.Lattice(mask, **kw)
    a.init_equilibrium(1.0)
    b.init_equilibrium(1.0)
    n = 90  # graph runs of 25 steps and a direct tail
    a.step(n)
    for _ in range(n):
        b.step(1)
    assert a.sync() == fluxlbm.FLBM_OK and b.sync() == fluxlbm.FLBM_OK
    assert np.array_equal(a.read_distributions(), b.read_distributions())
    assert a.step_count == b.step_count == n
    ha, hb = a.history(n), b.history(n)
    # rho_in, Q_in and Q_out of every step (mass and max |u| are recorded at
    # the end of each call, so those differ)
    for col in (0, 1, 2):
        assert np.array_equal(ha[:, col], hb[:, col], equal_nan=True), col
    assert np.isnan(ha[:, 0]).all() == (z_mode != 0)


def test_watchdog_trips_on_large_flux_and_nan():
    mask = np.zeros((10, 6, 6), np.uint8)
    lat, _ = pair(mask, precision="fp32", tau=0.8, q_target=36 * 0.5, watchdog_every=10)
    lat.init_equilibrium(1.0)
    lat.step(10)
    assert lat.sync() == fluxlbm.FLBM_EUNSTABLE
    # a rewritten state clears the flag; a NaN population trips it again
    lat.set_target_flux(0.0)
    f = lat.read_distributions()
    f[:] = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None]
    lat.write_distributions(f)
    lat.step(10)
    assert lat.sync() == fluxlbm.FLBM_OK
    f[3, 17] = np.nan
    lat.write_distributions(f)
    lat.step(10)
    assert lat.sync() == fluxlbm.FLBM_EUNSTABLE


def test_large_inlet_plane_grid_stride():
    """Inlet plane larger than the reduction grid (1024 blocks x 256 sites)."""
    mask = np.zeros((3, 520, 520), np.uint8)
    mask[1, ::7, ::5] = 1
    lat, orc = pair(mask, precision="fp64", tau=0.8, q_target=100.0)
    load_same_state(lat, orc, mask, 61)
    lat.step(1)
    h_orc = orc.step(1)
    h = lat.history(1)
    assert lat.a_in == 520 * 520
    assert abs(h[0, 0] - h_orc[0, 0]) <= 1e-13
    assert abs(h[0, 1] - 100.0) <= 1e-9
    assert _compare(lat, orc, mask) <= 1e-12


# ---------------------------------------------------------------- FP16 deviation storage

def test_fp16dev_one_step_flux_box():
    """FP16 storage of scaled deviations: one step from a random state. Each
    stored deviation (|g| <= 0.05 w) is rounded to 11 significant bits on
    load and on store: error bound ~1.2e-5 of max |f| per rounding."""
    mask = inputs.random_mask((12, 14, 13), 0.3, 71)
    mask[0, 0, 0] = 0
    lat, orc = pair(mask, precision="fp16dev", tau=0.9, q_target=0.3, periodic_x=True, periodic_y=False)
    load_same_state(lat, orc, mask, 72)
    lat.step(1)
    h_orc = orc.step(1)
    err = _compare(lat, orc, mask)
    assert err <= 5e-5, err
    h = lat.history(1)
    assert abs(h[0, 1] - 0.3) <= 1e-12
    assert abs(h[0, 0] - h_orc[0, 0]) <= 1e-5


def test_fp16dev_slit_channel_against_oracle():
    """Error of the FP16-deviation mode against the FP64 oracle on the slit
    after 2000 steps (reported in the assertion message)."""
    mask = inputs.slit_channel(16, 16, 64)
    lat, orc = pair(mask, precision="fp16dev", tau=1.0, q_target=0.5, periodic_x=False, periodic_y=True)
    lat.init_equilibrium(1.0)
    orc.init_equilibrium(1.0)
    lat.step(2000)
    h_orc = orc.step(2000)
    h = lat.history(2000)
    assert lat.sync() == fluxlbm.FLBM_OK
    rho, ux, uy, uz = lat.fields()
    _, _, _, uz_o = orc.fields()
    sites = inputs.pore_sites(mask)
    ref = uz_o.reshape(-1)[sites]
    err_u = np.abs(uz - ref).max() / np.abs(ref).max()
    assert err_u <= 1e-2, f"u_z error {err_u:.3e}"
    assert np.abs(h[:, 1] - 0.5).max() <= 1e-12
    q_err = abs(0.5 * (h[-1, 2] + h[-2, 2]) - 0.5 * (h_orc[-1, 2] + h_orc[-2, 2])) / 0.5
    assert q_err <= 1e-2, f"outlet flux error {q_err:.3e}"


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("fp16dev", 1e-2)])
def test_steady_flux_and_permeability_match_fp64(precision, tol):
    """A long pack (140 planes) run for 120,000 steps (well into the approach
    to steady state) against the same run in FP64: the outlet flux and the
    inlet-outlet density difference (the permeability's denominator) agree
    to 1e-4 relative in FP32 (1e-2 for FP16 deviations, whose 11-bit
    significands carry the velocity on top of a much larger density
    deviation). Reduced-precision rounding must not create mass: a coherent
    per-site source would add up along the planes into a flux error (1.3e-3
    over the 268 planes of a 256^3 pack before the rest population was made
    mass-exact)."""
    mask, _, _ = inputs.sphere_pack((140, 32, 32), 0.45, 17, reservoir_layers=6)
    q = 1e-5 * 32 * 32
    runs = {}
    for prec in ("fp64", precision):
        lat = fluxlbm.Lattice(mask, precision=prec, tau=0.7, q_target=q, watchdog_every=4096)
        lat.init_equilibrium()
        lat.step(120000)
        h = lat.history(2048)
        runs[prec] = (0.5 * (h[-1, 2] + h[-2, 2]), h[:, 0].mean() - 1.0)
        lat.close()
    (q64, d64), (qp, dp) = runs["fp64"], runs[precision]
    print(f"steady {precision}: Q_out/Q* FP64 {q64 / q:.6f}, {precision} vs FP64 {qp / q64 - 1:+.3e}, "
          f"density difference vs FP64 {dp / d64 - 1:+.3e}", flush=True)
    assert abs(q64 - q) <= 0.1 * q                  # FP64 is well into the approach
    assert abs(qp - q64) <= tol * q, (qp / q - 1, q64 / q - 1)
    assert abs(dp - d64) <= tol * d64, (dp / d64 - 1)

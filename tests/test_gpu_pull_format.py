"""The compact pull tables address the same slots as the int32 table, so a
lattice stepped with any of them must hold bitwise equal states and
histories: for every storage precision, BGK, MRT and the two-fluid colour
model (both of its passes read the table), with the default forms, with a
mix of 8-bit, 16-bit and int32 tiles (small code limits, and a lattice whose
wide reservoir planes overflow the 16-bit codes at a y-wrap), with the 8-bit
codes read as run codes (waves whose list of codes needs a second word, and
8-bit tiles too irregular for run codes beside them), and inside a batch
that mixes the formats."""
import numpy as np
import pytest

from paper_1806_10589_amd import fluxlbm, inputs

pytestmark = pytest.mark.gpu


def _pack(edge, seed, res=3):
    mask, _, _ = inputs.sphere_pack(edge, 0.35, seed=seed, reservoir_layers=res)
    return mask


def _run(mask, fmt, limits, precision, model, steps, q=0.3, tau=0.8):
    lat = fluxlbm.Lattice(mask, precision=precision, model=model, tau=tau, q_target=q, watchdog_every=50)
    try:
        lat.set_pull_format(fmt, *limits)
        info = lat.pull_format()
        lat.init_equilibrium()
        lat.step(steps)
        return lat.read_distributions(), lat.history(steps), info
    finally:
        lat.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
@pytest.mark.parametrize("model", ["bgk", "mrt"])
@pytest.mark.parametrize("fmt,limits", [(3, (0, 0)), (3, (600, 100)), (2, (0, 0)), (2, (600, 100)), (1, (0, 0))])
def test_compact_equals_int32_bitwise(precision, model, fmt, limits):
    mask = _pack(40, 11)
    print(f"pull format: {precision} {model} format {fmt} limits {limits}", flush=True)
    f0, h0, i0 = _run(mask, fluxlbm.FLBM_PULL_INT32, (0, 0), precision, model, 60)
    f1, h1, i1 = _run(mask, fmt, limits, precision, model, 60)
    assert i0[:3] == (fluxlbm.FLBM_PULL_INT32, 0, 0)
    assert i1[0] == fmt
    if limits != (0, 0):
        assert i1[1] > 0 and i1[2] > 0 and i1[1] + i1[2] < i1[3]   # all three forms
    assert np.array_equal(f0, f1)
    assert np.array_equal(h0[:, :3], h1[:, :3])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_run_codes_beside_irregular_byte_tiles(precision):
    # independent random solids (half the voxels): most waves change codes at
    # nearly every site, so most 8-bit tiles are too irregular for run codes;
    # the one tile that has them needs the second word in every wave
    mask = inputs.random_mask((20, 40, 40), 0.5, 3)
    lat = fluxlbm.Lattice(mask, precision="fp32", tau=0.8, q_target=0.1)
    try:
        _, t8, t16, _ = lat.pull_format()
        runs, wide = lat.pull_runs()
    finally:
        lat.close()
    print(f"run codes: {precision}; {t8} 8-bit tiles, {runs} with run codes ({wide} wide waves)", flush=True)
    assert 0 < runs < t8 and wide > 0 and t16 > 0
    f0, h0, _ = _run(mask, fluxlbm.FLBM_PULL_INT32, (0, 0), precision, "bgk", 40, q=0.1)
    f1, h1, _ = _run(mask, fluxlbm.FLBM_PULL_RUN, (0, 0), precision, "bgk", 40, q=0.1)
    assert np.array_equal(f0, f1)
    assert np.array_equal(h0[:, :3], h1[:, :3])


def test_wide_reservoir_planes_fall_back():
    # 300 x 300 planes: a fluid reservoir plane holds 90,000 sites, so the
    # tiles that hold a y-wrap have sources farther apart than 16 bits
    mask = np.zeros((10, 300, 300), np.uint8)
    mask[3:7] = inputs.random_mask((4, 300, 300), 0.3, 21)
    f0, h0, _ = _run(mask, fluxlbm.FLBM_PULL_INT32, (0, 0), "fp32", "bgk", 24, q=2.0)
    f1, h1, info = _run(mask, fluxlbm.FLBM_PULL_RUN, (0, 0), "fp32", "bgk", 24, q=2.0)
    print(f"wide planes: {info[1]} byte, {info[2]} 16-bit of {info[3]} tiles", flush=True)
    assert info[1] + info[2] < info[3]
    assert np.array_equal(f0, f1)
    assert np.array_equal(h0[:, :3], h1[:, :3])


def test_batch_mixing_formats_equals_singles():
    masks = [_pack(24, 31), _pack(32, 32), _pack(20, 33), _pack(28, 34), _pack(24, 35)]
    fmts = [(fluxlbm.FLBM_PULL_RUN, 0, 0), (fluxlbm.FLBM_PULL_INT32, 0, 0),
            (fluxlbm.FLBM_PULL_RUN, 800, 100), (fluxlbm.FLBM_PULL_HALF, 0, 0), (fluxlbm.FLBM_PULL_COMPACT, 0, 0)]

    def make():
        out = []
        for m, f in zip(masks, fmts):
            lat = fluxlbm.Lattice(m, precision="fp32", tau=0.8, q_target=0.2, watchdog_every=16)
            lat.set_pull_format(*f)
            lat.init_equilibrium()
            out.append(lat)
        return out

    singles, batched = make(), make()
    b = fluxlbm.Batch(batched)
    try:
        for sched in (dict(grid=0, order=fluxlbm.FLBM_ORDER_INTERLEAVE, tiles_per_item=1, chunk=8),
                      dict(grid=5, order=fluxlbm.FLBM_ORDER_LARGEST, tiles_per_item=2, chunk=5)):
            b.set_schedule(**sched)
            b.step(33)
            rc, bad = b.sync()
            assert rc == fluxlbm.FLBM_OK and bad == -1
            for s, l in zip(singles, batched):
                s.step(33)
                assert np.array_equal(s.read_distributions(), l.read_distributions())
    finally:
        b.close()
        for l in singles + batched:
            l.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
@pytest.mark.parametrize("fmt,limits", [(3, (0, 0)), (2, (0, 0)), (2, (600, 100)), (1, (0, 0))])
def test_colour_compact_equals_int32_bitwise(precision, fmt, limits):
    """Colour model, flux set-up with a non-wetting inlet reservoir: the phase
    pass (directions 1..6) and the colour step (all 18, and the neighbours'
    phase through the same decoded indices) give bitwise equal f, A and B."""
    mask = _pack(40, 12)
    print(f"colour pull format: {precision} format {fmt} limits {limits}", flush=True)
    sites = inputs.pore_sites(mask)
    z = sites // (mask.shape[1] * mask.shape[2])
    na = (z < 3).astype(float)

    def run(f, lim):
        lat = fluxlbm.Lattice(mask, precision=precision, model="colour", tau=1.0, q_target=0.05,
                              alpha=0.01, beta=0.7, phi_solid=-0.7, watchdog_every=20)
        try:
            lat.set_pull_format(f, *lim)
            info = lat.pull_format()
            lat.init_colour(na, 1.0 - na)
            lat.step(40)
            A, B = lat.read_colour()
            return lat.read_distributions(), A, B, lat.history(40), info
        finally:
            lat.close()

    f0, A0, B0, h0, i0 = run(fluxlbm.FLBM_PULL_INT32, (0, 0))
    f1, A1, B1, h1, i1 = run(fmt, limits)
    assert i0[:3] == (fluxlbm.FLBM_PULL_INT32, 0, 0) and i1[0] == fmt
    if limits != (0, 0):
        assert i1[1] > 0 and i1[2] > 0 and i1[1] + i1[2] < i1[3]
    assert np.array_equal(f0, f1) and np.array_equal(A0, A1) and np.array_equal(B0, B1)
    assert np.array_equal(h0[:, :3], h1[:, :3])

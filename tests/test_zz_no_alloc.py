"""The allocation-free entry point against the one it varies:
flbm_state_observables_noalloc (partials in the library's fixed device
array) must give what flbm_get_observables (partials in the context's device
memory) gives for the same state -- the same kernels over the same blocks, so
the same values -- on consecutive calls with a smaller input second (the
array keeps the first call's partials beyond the second's blocks), in every
storage precision, after steps and with a non-finite value planted in the
host-written state. Sizes beyond the array are refused before any launch."""
import numpy as np
import pytest

from paper_1806_10589_amd import fluxlbm, inputs

from .gpu_helpers import dense_to_sites, random_state

pytestmark = pytest.mark.gpu

PREC = {"fp64": fluxlbm.FLBM_FP64, "fp32": fluxlbm.FLBM_FP32, "fp16dev": fluxlbm.FLBM_FP16DEV}


def _lattice(edge, seed, precision):
    mask, _, _ = inputs.sphere_pack(edge, 0.35, seed=seed, reservoir_layers=3)
    lat = fluxlbm.Lattice(mask, precision=precision, tau=0.8, q_target=1e-4 * edge * edge, rho0=1.0)
    lat.write_distributions(dense_to_sites(mask, random_state(mask, seed)))
    return lat, mask


def _noalloc(lat, precision):
    f_dev, _, npad = fluxlbm.flbm_device_layout(lat.ctx)
    return fluxlbm.flbm_state_observables_noalloc(f_dev, PREC[precision], lat.n_sites, npad, 1.0,
                                                  lat.stream.cuda_stream)


def _same(got, ref):
    """Equal values (a non-finite state gives NaN on both sides)."""
    m, u, b = got
    mr, ur, br = ref
    assert b == br
    if br:
        assert np.isnan(u) and np.isnan(ur) and np.isnan(m) == np.isnan(mr)
        return
    assert abs(m - mr) <= 1e-15 * abs(mr) and m == mr
    assert abs(u - ur) <= 1e-15 * ur and u == ur


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_noalloc_observables_equal_the_context_entry_point(precision):
    big, _ = _lattice(48, 11, precision)
    small, mask_s = _lattice(24, 12, precision)
    try:
        print(f"noalloc {precision}: sites {big.n_sites} then {small.n_sites}", flush=True)
        for lat in (big, small):  # the second call has fewer blocks than the first
            _same(_noalloc(lat, precision), lat.observables())
        for lat in (big, small):  # after steps of the state
            lat.step(6)
            assert lat.sync() == fluxlbm.FLBM_OK
            _same(_noalloc(lat, precision), lat.observables())
        f = lat.read_distributions()  # small lattice: plant a non-finite value
        f[3, small.n_sites // 2] = np.nan
        small.write_distributions(f)
        got = _noalloc(small, precision)
        assert got[2] == 1
        _same(got, small.observables())
    finally:
        big.close()
        small.close()


def test_noalloc_refuses_sizes_beyond_its_array():
    lat, _ = _lattice(16, 13, "fp32")
    try:
        f_dev, _, npad = fluxlbm.flbm_device_layout(lat.ctx)
        with pytest.raises(fluxlbm.FlbmError) as e:
            fluxlbm.flbm_state_observables_noalloc(f_dev, fluxlbm.FLBM_FP32, lat.n_sites, (1 << 26) + 256, 1.0,
                                                   lat.stream.cuda_stream)
        assert e.value.status == fluxlbm.FLBM_ESCRATCH
        with pytest.raises(fluxlbm.FlbmError) as e:
            fluxlbm.flbm_state_observables_noalloc(f_dev, fluxlbm.FLBM_FP32, lat.n_sites, npad + 100, 1.0,
                                                   lat.stream.cuda_stream)
        assert e.value.status == fluxlbm.FLBM_EINVAL
        # after the refusals the lattice's own size still works
        _same(fluxlbm.flbm_state_observables_noalloc(f_dev, fluxlbm.FLBM_FP32, lat.n_sites, npad, 1.0,
                                                     lat.stream.cuda_stream), lat.observables())
    finally:
        lat.close()

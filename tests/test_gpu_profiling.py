"""FLBM_PROFILE=1 (roctx ranges around every launch, steps launched directly
instead of replaying graphs) changes nothing in the results: the same
kernels run in the same order, so states and histories are bitwise equal to
an unprofiled run, for the single-fluid step and the two-fluid step."""
import os

import numpy as np
import pytest

from paper_1806_10589_amd import fluxlbm, inputs

pytestmark = pytest.mark.gpu


def _run(mask, profile, **kw):
    old = os.environ.pop("FLBM_PROFILE", None)
    if profile:
        os.environ["FLBM_PROFILE"] = "1"
    try:
        lat = fluxlbm.Lattice(mask, watchdog_every=20, **kw)
    finally:
        os.environ.pop("FLBM_PROFILE", None)
        if old is not None:
            os.environ["FLBM_PROFILE"] = old
    try:
        if kw.get("model") == "colour":
            z = lat.coords()[:, 2]
            na = (z < 3).astype(float)
            lat.init_colour(na, 1.0 - na)
        else:
            lat.init_equilibrium()
        lat.step(45)
        assert lat.sync() == fluxlbm.FLBM_OK
        out = [lat.read_distributions(), lat.history(45)[:, :5]]
        if kw.get("model") == "colour":
            out += list(lat.read_colour())
        return out
    finally:
        lat.close()


@pytest.mark.parametrize("model", ["bgk", "colour"])
def test_profiling_markers_leave_results_unchanged(model):
    mask, _, _ = inputs.sphere_pack(32, 0.35, seed=21, reservoir_layers=3)
    kw = dict(precision="fp32", tau=0.9, q_target=0.05, model=model)
    if model == "colour":
        kw.update(alpha=0.0157, beta=0.7, phi_solid=-0.7071)
    a = _run(mask, False, **kw)
    b = _run(mask, True, **kw)
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)

"""The paper's square-tube drainage (Sec. 3.2) on the GPU: non-wetting fluid
injected at constant flux into a wetting-filled 40 x 40 x 80 tube between two
six-layer reservoirs, interfacial tension 6e-5 set through alpha from a
Laplace-law calibration of the same code. The paper's observation: the rate
at which the wetting volume falls approaches the injected flux Q once the
displacement is steady (the early deviation is the capillary entry effect).
At the lowest flux, Q = 0.02, the paper notes that spurious currents near
the boundaries can spoil this and that larger reservoirs mitigate it: with
six-plane reservoirs the rate is still 19 % above Q after 2.56M steps (1.45
falling to 1.19), with twelve-plane reservoirs it stays within 2-4 % of Q
from the start (0.98 to 0.96 over the same run); the test takes the
twelve-plane set-up."""
import numpy as np
import pytest

from paper_1806_10589_amd import replicas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def alpha():
    slope, icpt, dps = replicas.laplace_gamma(0.005)
    # Laplace: the jump grows linearly with 1/R and the fit's intercept is small
    assert slope > 0 and abs(icpt) < 0.5 * min(dps)
    return 6e-5 * 0.005 / slope


def test_drainage_rate_approaches_flux_q2(alpha):
    r = replicas.e2_drainage(2.0, alpha, steps=30000)
    track = np.array(r["rate_track"])
    assert r["q_in_err"] <= 1e-12                      # the inlet flux is exact every step
    assert abs(track[len(track) // 2:] - 1.0).max() <= 0.01, track


def test_drainage_rate_approaches_flux_q02(alpha):
    r = replicas.e2_drainage(0.2, alpha, steps=120000)
    track = np.array(r["rate_track"])
    assert r["q_in_err"] <= 1e-12
    assert abs(track[-1] - 1.0) <= 0.04, track
    # and the deviation keeps shrinking
    assert abs(track[-1] - 1.0) < abs(track[len(track) // 4] - 1.0)


def test_drainage_rate_near_flux_q002_with_larger_reservoirs(alpha):
    r = replicas.e2_drainage(0.02, alpha, reservoir=12, steps=640000, window=128000)
    track = np.array(r["rate_track"])
    print(f"Q = 0.02, 12-plane reservoirs: rate/Q {r['rate_over_q']:.4f}, track {np.round(track, 3)}", flush=True)
    assert r["q_in_err"] <= 1e-12
    assert abs(r["rate_over_q"] - 1.0) <= 0.05, track
    assert abs(track[len(track) // 2:] - 1.0).max() <= 0.05, track

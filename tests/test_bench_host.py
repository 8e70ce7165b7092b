"""Host-side checks of the benchmark's workload definitions and byte counts."""
import json
import os

import pytest

import bench

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_survey_byte_counts():
    """19 populations read and written once plus 18 int32 indices; the colour
    model adds both D3Q7 colours read and written once and the phase field."""
    assert bench.bytes_per_lup_survey("fp32") == 224
    assert bench.bytes_per_lup_survey("fp16dev") == 148
    assert bench.bytes_per_lup_survey("fp64") == 376
    assert bench.bytes_per_lup_survey("fp32", "colour") == 340
    assert bench.bytes_per_lup_survey("fp16dev", "colour") == 208


def test_design_byte_counts():
    # int32 table: the survey's single-fluid count
    assert bench.bytes_per_lup("fp32") == 224
    # all tiles with byte codes: 152 + 18 + the 80-byte header over 512 sites
    assert abs(bench.bytes_per_lup("fp32", "bgk", 1.0, 0.0) - (152 + 18 + 80 / 512)) < 1e-12
    # colour, int32 table: f 152 + 72; phase pass 56 + 24 + 8; colour step 8 + 56
    assert bench.bytes_per_lup("fp32", "colour") == 224 + 88 + 64
    # run codes: 8 bytes per site where the 8-bit codes take 18, 4 more on
    # wide waves; the single-fluid FP16 step reads them, the FP16 colour step
    # the 8-bit codes
    hdr = 80 / 512
    assert abs(bench.bytes_per_lup("fp16dev", "bgk", 1.0, 0.0, 1.0, 0.5) - (76 + 8 + hdr + 2)) < 1e-12
    assert abs(bench.bytes_per_lup("fp32", "bgk", 1.0, 0.0, 0.5, 0.0) - (152 + 13 + hdr)) < 1e-12
    assert bench.bytes_per_lup("fp16dev", "colour", 1.0, 0.0, 1.0, 0.5) == bench.bytes_per_lup(
        "fp16dev", "colour", 1.0, 0.0)


def test_two_fluid_workload_uses_the_oracle_calibration():
    """alpha of the two-fluid pack workload is the oracle's Laplace-law
    calibration for gamma = 0.01, and Q* follows Ca = mu Q* / (gamma eps A)."""
    with open(os.path.join(GOLDEN, "colour_calibration.json")) as fh:
        cal = json.load(fh)
    assert abs(cal["gamma"] / 0.01 - 1.0) <= 1e-4
    for name in ("pack384c", "pack384ch"):
        cfg = bench.CONFIGS[name]
        assert abs(cfg["alpha"] / cal["alpha"] - 1.0) <= 1e-5
        assert cfg["tau"] == 1.0 and abs(cfg["phi_solid"] + 2 ** -0.5) < 1e-4
        mu = (cfg["tau"] - 0.5) / 3.0
        ca = mu * cfg["q"] / (0.01 * 0.30 * 384 * 384)
        assert abs(ca / 1e-5 - 1.0) < 1e-12


@pytest.mark.parametrize("name", ["pack384c", "pack384ch", "pack256", "pack512", "pack256c"])
def test_workloads_are_defined(name):
    cfg = bench.CONFIGS[name]
    assert cfg["precision"] in ("fp32", "fp16dev", "fp64")

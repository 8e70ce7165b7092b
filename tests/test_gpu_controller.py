"""The learned inlet controller on the GPU: its decision rule against the FP64
oracle controller on the dense oracle lattice, and the cases where the plain
update of eq. potential must rule (trust0 = 0, a non-finite network, the
decaying trust bound, release), plus the trained network's gain.

Tolerances: the network's output differs from the oracle's (FP64 products
of the same BF16 operands) by FP32 accumulation, below 2e-4 of its scale;
an offset that is not clipped carries that difference times drho_ref exp(r);
a clipped offset is the same FP64 number on both sides."""
import math
import os

import numpy as np
import pytest

from oracle import mlp_oracle as mo
from oracle.controller_oracle import OracleController
from paper_1806_10589_amd import controller, fluxlbm, inputs
from .gpu_helpers import pair

pytestmark = pytest.mark.gpu


def _mask():
    m, _, _ = inputs.sphere_pack((20, 12, 12), 0.6, 3, rmin=2, rmax=3, reservoir_layers=2)
    return m


def _params(seed, b3, scale=0.3):
    p = scale * inputs.uniform_noise((mo.N_PARAMS,), seed)
    p[-1] = b3
    return p.astype(np.float32)


GEOM = np.linspace(-0.5, 0.5, 15).astype(np.float32)


def _run_pair(gain, trust0, b3, n=80, relative=False, stall=0, period=1, trust_decisions=50):
    mask = _mask()
    q = 0.02
    lat, orc = pair(mask, precision="fp64", tau=0.9, q_target=q)
    lat.init_equilibrium()
    orc.init_equilibrium()
    params = _params(81, b3)
    net = fluxlbm.Mlp(16)
    net.set_params(params)
    kw = dict(drho_ref=1e-3, gain=gain, trust0=trust0, release_tol=1e-12, trust_decisions=trust_decisions,
              relative=relative, stall_decisions=stall, period=period)
    lat.set_controller(net, GEOM, **kw)
    oc = OracleController(params.astype(np.float64), GEOM, **kw)
    lat.step(n)
    hg = lat.history(n)
    ho = oc.run(orc, n, q_target=q)
    x, aux = lat.controller_trace(n // period)
    return lat, orc, net, oc, hg, ho, x, aux, q, kw


@pytest.mark.parametrize("relative,period", [(False, 1), (True, 1), (True, 3)])
def test_clipped_decisions_match_oracle_exactly(relative, period):
    # every proposal lies far above the trust bound, so the inlet density of
    # every controlled step is the plain one plus the bound: the same FP64
    # number on both sides, and the two runs stay equal to rounding
    td = 50 // period
    lat, orc, net, oc, hg, ho, x, aux, q, kw = _run_pair(1.0, 0.5, 8.0, relative=relative, period=period,
                                                         trust_decisions=td)
    nd = 80 // period
    xo = np.array([r[0] for r in oc.records])
    auxo = np.array([[r[1], r[2], r[3], r[4]] for r in oc.records])
    assert len(oc.records) == nd and x.shape == (nd, 32)
    assert np.max(np.abs(x - xo)) <= 1e-6
    assert np.max(np.abs(aux[:, 0] - auxo[:, 0])) <= 1e-12          # drho
    assert np.max(np.abs(aux[:, 1] - auxo[:, 1])) <= 1e-12          # rho_plain
    assert np.max(np.abs(aux[:, 2] - auxo[:, 2])) <= 2e-4 * max(1.0, np.abs(auxo[:, 2]).max())
    limit = 0.5 * q / orc.a_in * np.maximum(0.0, 1.0 - np.arange(nd) / td)
    assert np.allclose(auxo[:, 3], limit, rtol=1e-15, atol=0)        # clipped every time
    assert np.max(np.abs(aux[:, 3] - auxo[:, 3])) <= 1e-15
    assert np.max(np.abs(hg[:, 0] - ho[:, 0])) <= 1e-12              # rho_in of every step
    assert np.max(np.abs(hg[:, 2] - ho[:, 2])) <= 1e-12              # Q_out
    # each step of a period is held at the bound of the decision before it
    dev = np.abs(hg[:, 1] - q) / q
    for k in range(80):
        d = k // period - 1                      # the decision in force at step k (-1: none yet)
        want = 0.5 * max(0.0, 1.0 - d / td) if d >= 0 else 0.0
        assert abs(dev[k] - want) <= 1e-9, (k, dev[k], want)
    active, released, _, decisions = lat.controller_state()
    assert active and not released and decisions == nd
    lat.close()
    net.close()


@pytest.mark.parametrize("relative,period", [(False, 1), (True, 1), (True, 4)])
def test_proportional_decisions_follow_the_rule(relative, period):
    # offsets inside the bound carry the network's FP32 output: check each
    # device decision against the rule evaluated by the oracle on the
    # device's own record, then the trajectory against the oracle run with
    # the propagated tolerance
    lat, orc, net, oc, hg, ho, x, aux, q, kw = _run_pair(0.2, 50.0, -0.3, relative=relative, period=period,
                                                         trust_decisions=50 // period)
    a_in = orc.a_in
    nd = 80 // period
    for k in range(nd):
        t = (k + 1) * period                     # steps completed at decision k
        ref = OracleController(oc.params, GEOM, **kw)
        ref.periods = [float(np.mean(hg[j * period:(j + 1) * period, 2])) for j in range(k + 1)]
        ref.rho_in = list(hg[:t, 0])
        xk, drho = ref.inputs(q, 1.0)
        assert np.max(np.abs(x[k] - xk)) <= 1e-6, k
        assert abs(aux[k, 0] - drho) <= 1e-15
        y = ref.network(x[k].astype(np.float64))
        assert abs(aux[k, 2] - y) <= 2e-4 * max(1.0, abs(y)), k
        hold = ref.proposal(aux[k, 2], aux[k, 0], k, False, q_target=q, rho_out=1.0, rho0=1.0, a_in=a_in)
        d = ref.offset(hold, aux[k, 1])
        assert abs(aux[k, 3] - d) <= 1e-15 + 1e-12 * abs(d), k
    td = 50 // period
    assert np.any(np.abs(aux[:td, 3]) > 0) and np.all(aux[td:, 3] == 0.0)
    auxo = np.array([[r[1], r[2], r[3], r[4]] for r in oc.records])
    scale = (np.abs(aux[:, 0]).max() * math.exp(3.0) if relative else kw["drho_ref"] * math.exp(4.0)) * kw["gain"]
    assert np.max(np.abs(aux[:, 3] - auxo[:, 3])) <= 2e-4 * scale + 1e-12
    assert np.max(np.abs(hg[:, 0] - ho[:, 0])) <= 2e-4 * scale + 1e-12
    lat.close()
    net.close()


def _plain_and_controlled(params, ctrl, steps=300, precision="fp64"):
    mask = _mask()
    q = 0.02
    a = fluxlbm.Lattice(mask, precision=precision, tau=0.9, q_target=q)
    b = fluxlbm.Lattice(mask, precision=precision, tau=0.9, q_target=q)
    a.init_equilibrium()
    b.init_equilibrium()
    net = fluxlbm.Mlp(16)
    net.set_params(params)
    b.set_controller(net, GEOM, **ctrl)
    a.step(steps)
    b.step(steps)
    out = a.read_distributions(), b.read_distributions(), a.history(steps), b.history(steps), b
    a.close()
    return out, net


def test_zero_trust_is_the_plain_method_bitwise():
    (fa, fb, ha, hb, b), net = _plain_and_controlled(
        _params(91, 2.0), dict(drho_ref=1e-3, trust0=0.0, release_tol=0.0, trust_decisions=1000))
    assert np.array_equal(fa, fb)
    assert np.array_equal(ha[:, :3], hb[:, :3])
    x, aux = b.controller_trace(300)
    assert np.all(aux[:, 3] == 0.0) and np.all(np.isfinite(x))
    b.close()
    net.close()


def test_non_finite_network_falls_back_to_plain():
    p = _params(92, 0.0)
    p[-1] = np.nan
    (fa, fb, ha, hb, b), net = _plain_and_controlled(
        p, dict(drho_ref=1e-3, trust0=5.0, release_tol=0.0, trust_decisions=1000))
    assert np.array_equal(fa, fb)
    _, aux = b.controller_trace(300)
    assert np.all(np.isnan(aux[:, 2])) and np.all(aux[:, 3] == 0.0)
    b.close()
    net.close()


def test_trust_bound_clips_and_decays():
    # r = 4 proposes a density far above anything reasonable: every offset is
    # clipped to the bound, which decays to zero after trust_decisions decisions
    q, trust0, ts = 0.02, 0.2, 100
    (fa, fb, ha, hb, b), net = _plain_and_controlled(
        _params(93, 50.0), dict(drho_ref=1e-3, trust0=trust0, release_tol=0.0, trust_decisions=ts), steps=200)
    dev = np.abs(hb[:, 1] - q) / q        # |Q_in - Q*| / Q* per step
    n = np.arange(200)
    bound = trust0 * np.maximum(0.0, 1.0 - (n - 1) / ts)  # step k uses decision k-1
    assert dev[0] <= 1e-9                  # the first step is plain
    assert np.all(dev[1:] <= bound[1:] + 1e-9)
    assert np.allclose(dev[1:ts], bound[1:ts], rtol=1e-6)  # clipped at the bound
    assert np.all(dev[ts + 1:] <= 1e-9)    # then the plain method
    b.close()
    net.close()


def test_release_returns_control_for_good():
    (fa, fb, ha, hb, b), net = _plain_and_controlled(
        _params(94, 50.0), dict(drho_ref=1e-3, trust0=1.0, release_tol=10.0, trust_decisions=10 ** 6), steps=50)
    _, released, delta, decisions = b.controller_state()
    assert released and delta == 0.0 and decisions == 50
    _, aux = b.controller_trace(50)
    assert aux[0, 3] != 0.0 and np.all(aux[1:, 3] == 0.0)  # released once two periods are recorded
    b.set_controller(None)
    assert not b.controller_state()[0]
    b.step(10)
    assert np.allclose(b.history(10)[:, 1], 0.02, rtol=1e-9)
    b.close()
    net.close()


def test_no_progress_returns_control():
    # a constant network holds the inlet at a fixed density; once the outlet
    # error stops falling by 10 % within stall_decisions decisions, the plain
    # update takes over for good
    p = np.zeros(mo.N_PARAMS, np.float32)
    p[-1] = 0.5
    (fa, fb, ha, hb, b), net = _plain_and_controlled(
        p, dict(drho_ref=2e-3, trust0=5.0, release_tol=1e-12, trust_decisions=10 ** 6, stall_decisions=40),
        steps=1500)
    _, released, delta, decisions = b.controller_state()
    assert released and delta == 0.0
    _, aux = b.controller_trace(1500)
    first_zero = int(np.argmax(aux[:, 3] == 0.0))
    assert first_zero > 40 and np.all(aux[first_zero:, 3] == 0.0)
    assert np.allclose(hb[first_zero + 1:, 1], 0.02, rtol=1e-9)   # plain: the inlet flux is exact
    b.close()
    net.close()


def test_controller_rejected_without_flux_inlet():
    mask = _mask()
    lat = fluxlbm.Lattice(mask, precision="fp32", z_mode=fluxlbm.FLBM_Z_PERIODIC)
    net = fluxlbm.Mlp(16)
    with pytest.raises(fluxlbm.FlbmError) as e:
        lat.set_controller(net, GEOM)
    assert e.value.status == fluxlbm.FLBM_ESTATE
    lat.close()
    net.close()


@pytest.mark.skipif(not os.path.exists(controller.DEFAULT_WEIGHTS), reason="no trained controller weights")
def test_trained_controller_reaches_tolerance_sooner():
    """What the trained network gains: on held-out packs (seeds outside the
    training family) the learned controller reaches |Q_out - Q*| / Q* <= 1e-3
    for good in fewer steps than the plain update, in total over the set."""
    params, meta = controller.load_weights()
    settings = controller.settings_of(meta)
    plain = learned = 0
    for seed in (4242, 4243, 4244):
        mask, kw = controller.make_sample(64, 0.3, seed, tau=0.8, darcy=1e-5)
        r = controller.evaluate(params, mask, kw, max_steps=200000, settings=settings)
        assert r["plain_steps"] is not None and r["learned_steps"] is not None, r
        plain += r["plain_steps"]
        learned += r["learned_steps"]
    print(f"steps to 1e-3: plain {plain}, learned {learned}, gain {plain / learned:.2f}")
    assert learned < plain


@pytest.mark.parametrize("trust", [0.5, 100.0])
def test_inlet_density_override_against_oracle(trust):
    # a caller's inlet density, judged by the plain update: clipped to within
    # trust |Q*| of the plain flux (trust 0.5), or taken as is (trust 100)
    mask = _mask()
    q = 0.02
    lat, orc = pair(mask, precision="fp64", tau=0.9, q_target=q)
    lat.init_equilibrium()
    orc.init_equilibrium()
    rho_hat = 1.002
    lat.set_inlet_density_override(rho_hat, trust)
    limit = trust * q / orc.a_in
    rows = []
    for _ in range(60):
        plain = orc.plain_inlet_density()
        orc.set_inlet_offset(min(limit, max(-limit, rho_hat - plain)))
        rows.append(orc.step(1)[0])
    ho = np.array(rows)
    lat.step(60)
    hg = lat.history(60)
    assert np.max(np.abs(hg[:, 0] - ho[:, 0])) <= 1e-12
    assert np.max(np.abs(hg[:, 1] - ho[:, 1])) <= 1e-11
    assert np.max(np.abs(hg[:, 2] - ho[:, 2])) <= 1e-11
    if trust > 10:
        assert np.allclose(hg[:, 0], rho_hat, rtol=0, atol=1e-14)
    else:
        dev = np.abs(hg[:, 1] - q)
        assert np.all(dev <= trust * q * (1 + 1e-9))
        assert np.allclose(dev[:40], trust * q, rtol=1e-9)   # clipped while the plain density is far
    lat.set_inlet_density_override(None)
    lat.step(5)
    assert np.allclose(lat.history(5)[:, 1], q, rtol=1e-10)
    lat.close()

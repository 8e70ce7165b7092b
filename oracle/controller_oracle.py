"""FP64 CPU oracle of the learned inlet controller's decision rule (test
infrastructure; only the tests use it).

The paper's update of eq. potential sets the inlet density so that the inlet
flux equals Q* at every step. The controller is a learned addition on top:
every `period` steps it proposes an inlet density, and for the next period
the plain update both bounds it and replaces it. This module takes the
decisions from their definition, step by step, on the dense FP64 oracle
lattice:

period    after every step t (steps counted from 1) the outlet flux of that
          step is added to the period's sum; when t is a multiple of the
          period, the period's mean Qbar is recorded and a decision taken;
inputs x (32):
  x[0..14]  the geometry values given with the controller;
  x[15+k]   (Qbar(P - lag_k) - Q*) / |Q*| clipped to [-2, 2], P the number of
            periods recorded, Qbar(j) the mean of period j (counted from 0;
            0 before the first), lags 1, 2, 3, 4, 6, 8, 11, 16, 22, 32, 45,
            64, 90, 128, 180, 250;
  x[31]     log10(drho / drho_ref) / 3 clipped to [-1, 1] (-1 when drho <= 0),
            drho = rho_in of the last step - rho_out;
network   y = net(x), computed by the network oracle with BF16 operands (the
          precision of the device's matrix products);
proposal  absolute: r = clip(y, -4, 4) = log(drho_inf / drho_ref),
          rho_hat = rho_out + drho_ref exp(r - margin); relative: r =
          clip(y, -2, 3) = log(drho_inf / drho), rho_hat = rho_out +
          drho exp(r - margin) (margin >= 0 aims below the prediction);
bound     b = trust0 max(0, 1 - n / trust_decisions) after n decisions,
          limit = b rho0 |Q*| / A_in;
release   for good once |Qbar(P - 1) - Q*| / |Q*| <= release_tol (P >= 2), or
          once that error has not fallen below 0.9 times its best value for
          stall_decisions decisions (when stall_decisions > 0);
hold      no proposal when released, when Q* <= 0, when relative and
          drho <= 0, when y or rho_hat is not finite, or when the limit is 0;
          otherwise every step of the next period uses
          rho_in = rho_plain + clip(gain (rho_hat - rho_plain), +-limit),
          rho_plain the density eq. potential gives for that step.
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp_oracle

LAGS = (1, 2, 3, 4, 6, 8, 11, 16, 22, 32, 45, 64, 90, 128, 180, 250)


def _f32(v):
    return float(np.float32(v))


class OracleController:
    def __init__(self, params, geometry, *, drho_ref, gain, trust0, release_tol, trust_decisions,
                 relative=False, stall_decisions=0, period=1, margin=0.0):
        self.params = np.asarray(params, np.float64)
        self.geometry = np.asarray(geometry, np.float64)
        self.drho_ref, self.gain, self.trust0 = float(drho_ref), float(gain), float(trust0)
        self.release_tol, self.trust_decisions = float(release_tol), int(trust_decisions)
        self.relative, self.stall_decisions, self.period = bool(relative), int(stall_decisions), int(period)
        self.margin = float(np.float32(margin))
        self.best, self.best_n = 0.0, 0
        self.qout = []      # Q_out of every step taken
        self.rho_in = []    # rho_in of every step taken
        self.periods = []   # mean Q_out of every period completed
        self.acc = 0.0
        self.released = False
        self.decisions = 0
        self.hold = None    # (rho_hat, limit) in force, or None
        self.records = []   # (x, drho, rho_plain, y, offset at the decision) per decision

    def _qbar(self, j):
        return self.periods[j] if j >= 0 else 0.0

    def inputs(self, q_target, rho_out):
        """The 32 inputs after the recorded periods, and drho."""
        p = len(self.periods)
        qn = abs(q_target) if q_target != 0.0 else 1.0
        drho = self.rho_in[-1] - rho_out if self.rho_in else 0.0
        x = np.empty(32)
        x[:15] = self.geometry
        for k, lag in enumerate(LAGS):
            e = (self._qbar(p - lag) - q_target) / qn
            x[15 + k] = _f32(min(2.0, max(-2.0, e)))
        if drho > 0.0:
            x[31] = _f32(min(1.0, max(-1.0, math.log10(drho / self.drho_ref) / 3.0)))
        else:
            x[31] = -1.0
        return x.astype(np.float32).astype(np.float64), drho

    def network(self, x):
        y, _, _ = mlp_oracle.forward(self.params, np.asarray(x, np.float64)[None, :], bf16=True)
        return float(y[0])

    def proposal(self, y, drho, n, released, *, q_target, rho_out, rho0, a_in):
        """(rho_hat, limit) for network output y at decision n, or None."""
        qn = abs(q_target) if q_target != 0.0 else 1.0
        b = self.trust0 * max(0.0, 1.0 - n / self.trust_decisions) if self.trust_decisions > 0 else 0.0
        limit = b * rho0 * qn / a_in
        if not math.isfinite(y) or released or not q_target > 0.0 or not limit > 0.0:
            return None
        if self.relative:
            if not drho > 0.0:
                return None
            rho_hat = rho_out + drho * math.exp(min(3.0, max(-2.0, y)) - self.margin)
        else:
            rho_hat = rho_out + self.drho_ref * math.exp(min(4.0, max(-4.0, y)) - self.margin)
        if not math.isfinite(rho_hat):
            return None
        return rho_hat, limit

    def offset(self, hold, rho_plain):
        """The offset a held proposal gives against this plain density."""
        if hold is None:
            return 0.0
        rho_hat, limit = hold
        return min(limit, max(-limit, self.gain * (rho_hat - rho_plain)))

    def decide(self, orc, q_target, rho_out, rho0, a_in):
        qn = abs(q_target) if q_target != 0.0 else 1.0
        x, drho = self.inputs(q_target, rho_out)
        y = self.network(x)
        p = len(self.periods)
        n = self.decisions
        e = abs(self._qbar(p - 1) - q_target) / qn
        if p >= 2 and e <= self.release_tol:
            self.released = True
        if n == 0 or e < 0.9 * self.best:
            self.best, self.best_n = e, n
        elif self.stall_decisions > 0 and n - self.best_n >= self.stall_decisions:
            self.released = True
        self.hold = self.proposal(y, drho, n, self.released, q_target=q_target, rho_out=rho_out, rho0=rho0,
                                  a_in=a_in)
        rho_plain = orc.plain_inlet_density()
        self.decisions += 1
        self.records.append((x, drho, rho_plain, y, self.offset(self.hold, rho_plain)))

    def run(self, orc, n, *, q_target, rho_out=1.0, rho0=1.0):
        """Advance the oracle lattice n steps under the controller; returns the
        oracle's history rows (rho_in, Q_in, Q_out, mass, max|u|)."""
        a_in = orc.a_in
        rows = []
        for _ in range(n):
            off = self.offset(self.hold, orc.plain_inlet_density()) if self.hold is not None else 0.0
            orc.set_inlet_offset(off)
            h = orc.step(1)[0]
            rows.append(h)
            self.rho_in.append(float(h[0]))
            self.qout.append(float(h[2]))
            self.acc += float(h[2])
            if len(self.qout) % self.period == 0:
                self.periods.append(self.acc / self.period)
                self.acc = 0.0
                self.decide(orc, q_target, rho_out, rho0, a_in)
        orc.set_inlet_offset(0.0)
        return np.array(rows)

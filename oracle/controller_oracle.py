"""FP64 CPU oracle of the learned inlet controller's decision rule (test
infrastructure; only the tests use it).

The paper's update of eq. potential sets the inlet density so that the inlet
flux equals Q* at every step. The controller is a learned addition on top:
after each step it proposes a density for the next step and the plain update
both bounds and replaces it. This module takes the decision from its
definition, step by step, on the dense FP64 oracle lattice:

inputs x (32):
  x[0..14]  the geometry values given with the controller;
  x[15+k]   (Qbar(t - lag_k) - Q*) / |Q*| clipped to [-2, 2], where
            Qbar(s) = (Q_out(s) + Q_out(s - 1)) / 2, Q_out(s) the outlet flux
            of step s (steps counted from 0, Q_out = 0 before step 0) and t
            the number of steps taken;
  x[31]     log10(drho / drho_ref) / 3 clipped to [-1, 1] (-1 when drho <= 0),
            drho = rho_in(t - 1) - rho_out.
network   r = clip(net(x), -4, 4), computed by the network oracle with BF16
          operands (the precision of the device's matrix products): the
          predicted steady density difference as log(drho_inf / drho_ref);
proposal  rho_hat = rho_out + drho_ref exp(r) (absolute mode), or with the
          relative target r = clip(net(x), -2, 3) = log(drho_inf / drho):
          rho_hat = rho_out + drho exp(r) (no offset while drho <= 0);
offset    delta = clip(gain (rho_hat - rho_plain), +-b rho0 |Q*| / A_in) with
          rho_plain the density eq. potential gives for the next step and
          b = trust0 max(0, 1 - n / trust_steps) after n decisions; delta = 0
          once Qbar(t - 1) has been within release_tol of Q* (relative; from
          then on for good, and only from t >= 2), once the error has not
          fallen below 0.9 times its best value for stall_steps decisions
          (when stall_steps > 0; for good), when Q* <= 0, or when the
          network output or the offset is not finite.
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp_oracle

LAGS = (1, 2, 3, 6, 11, 20, 36, 65, 119, 215, 391, 710, 1290, 2345, 4260, 7740)


def _f32(v):
    return float(np.float32(v))


class OracleController:
    def __init__(self, params, geometry, *, drho_ref, gain, trust0, release_tol, trust_steps, relative=False,
                 stall_steps=0):
        self.params = np.asarray(params, np.float64)
        self.geometry = np.asarray(geometry, np.float64)
        self.drho_ref, self.gain, self.trust0 = float(drho_ref), float(gain), float(trust0)
        self.release_tol, self.trust_steps = float(release_tol), int(trust_steps)
        self.relative, self.stall_steps = bool(relative), int(stall_steps)
        self.best, self.best_n = 0.0, 0
        self.qout = []      # Q_out of every step taken
        self.rho_in = []    # rho_in of every step taken
        self.released = False
        self.decisions = 0
        self.records = []   # (x, drho, rho_plain, r, delta) per decision

    def _q(self, s):
        return self.qout[s] if s >= 0 else 0.0

    def inputs(self, q_target, rho_out):
        """The 32 inputs after the recorded steps, and drho."""
        t = len(self.qout)
        qn = abs(q_target) if q_target != 0.0 else 1.0
        drho = self.rho_in[-1] - rho_out if t >= 1 else 0.0
        x = np.empty(32)
        x[:15] = self.geometry
        for k, lag in enumerate(LAGS):
            e = (0.5 * (self._q(t - lag) + self._q(t - lag - 1)) - q_target) / qn
            x[15 + k] = _f32(min(2.0, max(-2.0, e)))
        if drho > 0.0:
            x[31] = _f32(min(1.0, max(-1.0, math.log10(drho / self.drho_ref) / 3.0)))
        else:
            x[31] = -1.0
        return x.astype(np.float32).astype(np.float64), drho

    def network(self, x):
        y, _, _ = mlp_oracle.forward(self.params, np.asarray(x, np.float64)[None, :], bf16=True)
        return float(y[0])

    def offset(self, y, rho_plain, n, released, *, q_target, rho_out, rho0, a_in, drho=None):
        """The offset for network output y after n decisions."""
        qn = abs(q_target) if q_target != 0.0 else 1.0
        b = self.trust0 * max(0.0, 1.0 - n / self.trust_steps) if self.trust_steps > 0 else 0.0
        limit = b * rho0 * qn / a_in
        if not math.isfinite(y):
            return 0.0
        if self.relative:
            r = min(3.0, max(-2.0, y))
            rho_hat = rho_out + drho * math.exp(r)
        else:
            r = min(4.0, max(-4.0, y))
            rho_hat = rho_out + self.drho_ref * math.exp(r)
        delta = self.gain * (rho_hat - rho_plain)
        if not math.isfinite(delta) or not q_target > 0.0 or released or (self.relative and not drho > 0.0):
            delta = 0.0
        return min(limit, max(-limit, delta))

    def decide(self, orc, q_target, rho_out, rho0, a_in):
        """Take the decision after the last recorded step; returns the offset."""
        t = len(self.qout)
        qn = abs(q_target) if q_target != 0.0 else 1.0
        x, drho = self.inputs(q_target, rho_out)
        y = self.network(x)
        e2 = abs(0.5 * (self._q(t - 1) + self._q(t - 2)) - q_target) / qn
        n = self.decisions
        if t >= 2 and e2 <= self.release_tol:
            self.released = True
        if n == 0 or e2 < 0.9 * self.best:
            self.best, self.best_n = e2, n
        elif self.stall_steps > 0 and n - self.best_n >= self.stall_steps:
            self.released = True
        rho_plain = orc.plain_inlet_density()
        delta = self.offset(y, rho_plain, n, self.released, q_target=q_target, rho_out=rho_out,
                            rho0=rho0, a_in=a_in, drho=drho)
        self.decisions += 1
        self.records.append((x, drho, rho_plain, y, delta))
        return delta

    def run(self, orc, n, *, q_target, rho_out=1.0, rho0=1.0):
        """Advance the oracle lattice n steps under the controller; returns the
        oracle's history rows (rho_in, Q_in, Q_out, mass, max|u|)."""
        a_in = orc.a_in
        rows = []
        for _ in range(n):
            h = orc.step(1)[0]
            rows.append(h)
            self.rho_in.append(float(h[0]))
            self.qout.append(float(h[2]))
            orc.set_inlet_offset(self.decide(orc, q_target, rho_out, rho0, a_in))
        return np.array(rows)

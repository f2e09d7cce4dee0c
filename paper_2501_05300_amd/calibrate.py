"""Bulk calibration of contact parameters with the adjoint.

Scaled DEM models have to be calibrated against bulk responses before they
are used (the paper's introduction; its contact parameters are the normal
stiffness, the friction coefficient and the rolling-resistance
coefficient).  Here theta = (s_k, mu_t, mu_r) is fitted so that the mean
plate reactions of a few plate experiments match given targets.

An experiment is a bed at a saved state (positions, velocities, spins,
spring history, clock) whose plate is driven for a window of steps; its
response J(theta) is the mean z reaction on the plate over the window, and
the hand-written adjoint of the step gives dJ/dtheta in the same run.  The
fit is a damped Gauss-Newton iteration on the relative residuals
(J_e(theta) - target_e) / target_e over the parameters left free.

Everything that steps a bed goes through the HIP library (lprdem); this
module only chooses the next theta.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Sequence

import numpy as np

from . import beds
from .lprdem import Bed

NAMES = ("s_k", "mu_t", "mu_r")


@dataclasses.dataclass
class Experiment:
    """A plate experiment restarted from one saved state."""
    spec: beds.BedSpec
    body: int
    n_steps: int
    ckpt_every: int
    pos: np.ndarray
    vel: np.ndarray
    omega: np.ndarray
    keys: np.ndarray
    vals: np.ndarray
    clock: int
    bed_kw: dict
    _bed: Bed = None

    @classmethod
    def from_bed(cls, spec, bed, body, n_steps, ckpt_every=100, **bed_kw):
        """Saves the state of `bed` (a Bed of `spec`) as the experiment's start."""
        x, v, w = bed.state()
        keys, vals = bed.history()
        return cls(spec=spec, body=body, n_steps=n_steps, ckpt_every=ckpt_every, pos=x, vel=v, omega=w,
                   keys=keys, vals=vals, clock=bed.clock(), bed_kw=dict(bed_kw))

    def response(self, theta):
        """J(theta) and dJ/dtheta from the saved state (the bed is restored
        before every run)."""
        if self._bed is None:
            self._bed = Bed(self.spec, **self.bed_kw)
        b = self._bed
        b.set_state(self.pos, self.vel, self.omega)
        b.set_history(self.keys, self.vals)
        b.set_clock(self.clock)
        b.set_contact_params(float(theta[0]), float(theta[1]), float(theta[2]))
        return b.adjoint_window(self.n_steps, self.ckpt_every, self.body)

    def close(self):
        if self._bed is not None:
            self._bed.close()
            self._bed = None


def calibrate(experiments: Sequence[Experiment], targets: Sequence[float], theta0, free=(True, True, False),
              iters=10, rtol=1e-6, xtol=1e-7, damping=1e-3, max_damping=1e6, max_rel_step=0.5):
    """Damped Gauss-Newton on r_e = (J_e(theta) - target_e) / target_e.

    Only the parameters marked in `free` move.  A step whose residual norm
    is not smaller is retried with ten times the damping; once the damping
    passes `max_damping` without a smaller residual the fit stops where it
    is.  Each step changes a parameter by at most `max_rel_step` of its
    value, and the fit also stops when |r| <= rtol or no free parameter
    moved by more than `xtol` of its value.  Returns the fitted theta and
    the history of accepted iterates (theta, |r|, seconds)."""
    free = np.asarray(free, bool)
    targets = np.asarray(targets, np.float64)
    theta = np.asarray(theta0, np.float64).copy()
    history: List[dict] = []

    def evaluate(th):
        t0 = time.perf_counter()
        out = [e.response(th) for e in experiments]
        J = np.array([o[0] for o in out])
        G = np.array([o[1] for o in out])
        return (J - targets) / targets, G / targets[:, None], time.perf_counter() - t0

    r, Jac, sec = evaluate(theta)
    history.append({"theta": theta.copy(), "residual": float(np.linalg.norm(r)), "seconds": sec})
    lam = damping
    for _ in range(iters):
        if np.linalg.norm(r) <= rtol:
            break
        A = Jac[:, free]
        H = A.T @ A
        g = A.T @ r
        accepted = None
        while lam <= max_damping:
            step = np.linalg.solve(H + lam * np.diag(np.diag(H) + 1e-30), -g)
            limit = max_rel_step * np.abs(theta[free])
            step = np.clip(step, -limit, limit)
            trial = theta.copy()
            trial[free] += step
            r_t, J_t, sec = evaluate(trial)
            if np.linalg.norm(r_t) < np.linalg.norm(r):
                accepted = step
                break
            lam *= 10.0
        if accepted is None:
            break
        theta, r, Jac = trial, r_t, J_t
        lam = max(lam / 10.0, damping)
        history.append({"theta": theta.copy(), "residual": float(np.linalg.norm(r)), "seconds": sec})
        if np.all(np.abs(accepted) <= xtol * np.abs(theta[free])):
            break
    return theta, history

"""Reference calibration on the FP64 oracle (test infrastructure only).

Only the test suite may import this module.  It fits contact parameters
theta = (s_k, mu_t, mu_r) so that the mean plate reaction of each plate
experiment matches a target: the calibration the paper's introduction
requires of scaled DEM models, for the parameters of its contact model.
Each response and its derivative come from the oracle's forward-mode FP64
tangent over the window (the oracle's own stepping); the fit is the plain
Gauss-Newton iteration theta <- theta - (A^T A)^-1 A^T r on the relative
residuals r_e = (J_e - target_e) / target_e, A = dr/dtheta over the free
parameters, without damping or step control.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


class OracleExperiment:
    """A plate experiment restarted from a saved oracle state."""

    def __init__(self, spec, body, n_steps, state, history, clock):
        self.spec, self.body, self.n_steps = spec, body, n_steps
        self.state, self.history, self.clock = state, history, clock

    @classmethod
    def after(cls, spec, body, n_steps, pre_steps):
        """Steps a fresh oracle bed of `spec` pre_steps steps and saves its
        state, with velocities, spins and spring history rounded to FP32 (the
        precision both steppers store them in)."""
        ob = O.OracleBed(spec)
        ob.step(pre_steps)
        x, v, w = ob.state()
        keys, vals = ob.history()
        r32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
        return cls(spec, body, n_steps, (x, r32(v), r32(w)), (keys, r32(vals)), pre_steps)

    def response(self, theta):
        s2 = self.spec.copy()
        s2.params = self.spec.params.replace(s_k=float(theta[0]), mu_t=float(theta[1]), mu_r=float(theta[2]))
        ob = O.OracleBed(s2)
        ob.set_state(*self.state)
        ob.set_history(*self.history)
        ob.set_clock(self.clock)
        return ob.tangent_window(self.n_steps, self.body, 2)


def gauss_newton(experiments, targets, theta0, free, iters=8, rtol=1e-10):
    free = np.asarray(free, bool)
    targets = np.asarray(targets, np.float64)
    theta = np.asarray(theta0, np.float64).copy()
    for _ in range(iters):
        out = [e.response(theta) for e in experiments]
        r = (np.array([o[0] for o in out]) - targets) / targets
        if np.linalg.norm(r) <= rtol:
            break
        A = (np.array([o[1] for o in out]) / targets[:, None])[:, free]
        theta[free] -= np.linalg.solve(A.T @ A, A.T @ r)
    return theta

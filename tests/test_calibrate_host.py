"""Host logic of the two calibration loops on closed-form experiments (CPU).

The product's damped Gauss-Newton (paper_2501_05300_amd.calibrate) and the
oracle's plain one (oracle.calibrate_ref) only choose the next parameters;
here the experiments are closed forms whose fitted parameters are known, so
a wrong sign, a transposed Jacobian or a dropped scaling by the targets
fails a check."""
import numpy as np

from oracle.calibrate_ref import gauss_newton
from paper_2501_05300_amd.calibrate import calibrate


class Closed:
    """J(theta) = c * s_k^p * mu_t^q * (1 + mu_r) with its exact gradient:
    a power law like the Hertz reaction's dependence on the stiffness."""

    def __init__(self, c, p, q):
        self.c, self.p, self.q, self.calls = c, p, q, 0

    def response(self, th):
        self.calls += 1
        s, m, r = th
        J = self.c * s ** self.p * m ** self.q * (1.0 + r)
        return J, np.array([J * self.p / s, J * self.q / m, J / (1.0 + r)])


class Affine:
    """J(theta) = a . theta + b: Gauss-Newton reaches the root in one step."""

    def __init__(self, a, b):
        self.a, self.b = np.asarray(a, float), b

    def response(self, th):
        return float(self.a @ th + self.b), self.a.copy()


THETA_TRUE = np.array([1.25, 0.36, 0.02])
THETA0 = np.array([1.0, 0.3, 0.02])


def _targets(exps, th):
    return [e.response(th)[0] for e in exps]


def test_affine_model_is_solved_in_one_plain_step():
    exps = [Affine([2.0, -3.0, 5.0], 1.0), Affine([0.5, 4.0, -1.0], 2.0)]
    tg = _targets(exps, THETA_TRUE)
    th = gauss_newton(exps, tg, THETA0, (True, True, False), iters=1)
    # the root of the 2x2 system a_e[:2] . x = target_e - b_e - a_e[2] mu_r
    M = np.array([e.a[:2] for e in exps])
    rhs = np.array([t - e.b - e.a[2] * THETA0[2] for e, t in zip(exps, tg)])
    np.testing.assert_allclose(th[:2], np.linalg.solve(M, rhs), rtol=1e-12)
    np.testing.assert_allclose(th[:2], THETA_TRUE[:2], rtol=1e-12)
    assert th[2] == THETA0[2]


def test_both_loops_recover_power_law_parameters():
    exps = [Closed(8.0, 1.5, 0.7), Closed(1.4, 1.2, 1.1)]
    tg = _targets(exps, THETA_TRUE)
    th_o = gauss_newton(exps, tg, THETA0, (True, True, False), iters=30, rtol=1e-14)
    th_g, hist = calibrate(exps, tg, THETA0, (True, True, False), iters=30, rtol=1e-12)
    np.testing.assert_allclose(th_o, THETA_TRUE, rtol=1e-10)
    np.testing.assert_allclose(th_g, THETA_TRUE, rtol=1e-8)
    res = [h["residual"] for h in hist]
    assert all(b < a for a, b in zip(res, res[1:]))   # only improving steps are accepted
    assert res[-1] <= 1e-8   # stops once a step moves no parameter by 1e-7 of its value


def test_only_free_parameters_move():
    exps = [Closed(8.0, 1.5, 0.7), Closed(1.4, 1.2, 1.1)]
    tg = _targets(exps, np.array([1.25, 0.3, 0.02]))
    th_g, _ = calibrate(exps, tg, THETA0, (True, False, False), iters=30, rtol=1e-12)
    assert th_g[1] == THETA0[1] and th_g[2] == THETA0[2]
    np.testing.assert_allclose(th_g[0], 1.25, rtol=1e-8)


def test_step_is_clipped_to_a_fraction_of_each_parameter():
    # far from the root the undamped step would overshoot; each accepted
    # iterate changes a parameter by at most half its value
    exps = [Closed(8.0, 1.5, 0.7), Closed(1.4, 1.2, 1.1)]
    tg = _targets(exps, np.array([5.0, 1.5, 0.02]))
    _, hist = calibrate(exps, tg, THETA0, (True, True, False), iters=3, rtol=0.0)
    for a, b in zip(hist, hist[1:]):
        assert np.all(np.abs(b["theta"] - a["theta"]) <= 0.5 * np.abs(a["theta"]) * (1 + 1e-12))


def test_fit_stops_when_no_step_helps():
    # a response that no parameter changes: every trial fails, the damping
    # runs out and the fit returns the start after a bounded number of runs
    class Flat:
        calls = 0

        def response(self, th):
            Flat.calls += 1
            return 3.0, np.zeros(3)

    th, hist = calibrate([Flat()], [2.0], THETA0, (True, True, False), iters=10)
    np.testing.assert_array_equal(th, THETA0)
    assert len(hist) == 1
    assert Flat.calls <= 1 + 10  # the start, then one trial per damping level 1e-3 .. 1e6

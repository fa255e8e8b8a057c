"""Pins of the oracle's sampling loop (shoot, project, pull back) and of its
closed-form Gaussian velocity."""
import numpy as np

import synthgen
from oracle.families import family_of
from oracle.metric import max_violation
from oracle.pcfm import gaussian_ot_velocity, pcfm_sample


def test_velocity_is_the_conditional_mean_of_the_displacement():
    # Monte-Carlo regression of x1 - x0 on x_tau, per coordinate
    rng = np.random.default_rng(0)
    n, d = 400_000, 3
    m, s = np.array([0.7, -1.2, 0.3]), 0.4
    x0 = rng.standard_normal((n, d))
    x1 = m + s * rng.standard_normal((n, d))
    for tau in (0.2, 0.5, 0.85):
        xt = (1 - tau) * x0 + tau * x1
        y = x1 - x0
        for k in range(d):
            A = np.stack([np.ones(n), xt[:, k]], axis=1)
            coef = np.linalg.lstsq(A, y[:, k], rcond=None)[0]
            # prediction at two points against the closed form
            for u in (-0.5, 1.0):
                pred = coef[0] + coef[1] * u
                exact = gaussian_ot_velocity(np.array([u]), tau, np.array([m[k]]), s)[0]
                assert abs(pred - exact) <= 0.01 * (1 + abs(exact))


def test_velocity_end_points():
    u = np.array([0.3, -2.0])
    m = np.array([1.0, 0.5])
    # from flow time 0 the one-step shoot lands on the target mean
    assert np.allclose(u + gaussian_ot_velocity(u, 0.0, m, 0.7), m, atol=1e-15)
    # at flow time 1, c(1) = 1: the velocity is u itself
    assert np.allclose(gaussian_ot_velocity(u, 1.0, m, 0.7), m + (u - m), atol=1e-15)


def test_sample_is_feasible_and_equals_last_projection():
    b = synthgen.fisher_kpp_batch(batch=2, nx=16, nt=6, seed=3)
    rng = np.random.default_rng(5)
    for s_ in b.samples:
        fam = family_of(s_)
        u0 = rng.standard_normal(s_.n)
        mean = np.broadcast_to(s_.aux[: s_.nx], (s_.nt, s_.nx)).reshape(-1)
        u, hist = pcfm_sample(fam, u0, mean, 0.05, 4, return_history=True)
        assert len(hist) == 4
        assert np.abs(fam.h(u)).max() <= 1e-10
        np.testing.assert_array_equal(u, hist[-1])

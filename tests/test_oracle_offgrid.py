"""Pins of the oracle's off-grid correction (Sec. III-E, eq. doals), CPU only.

* the offset gradient and the Gauss-Newton block against finite differences
  of the residual (sign, factor and the closed form 2 c^2 Cov(positions));
* a shift by exactly one pixel reproduces the neighbouring pixel's steering
  vector and bound;
* with no Gauss-Newton rounds the solve is the on-grid solve of Table I;
* a source between pixel centres, exact covariance: the on-grid model leaves a
  residual and smears the power, the corrected solve recovers the offset and
  the power.
"""

import math

import numpy as np

import oracle
from oracle import offgrid
from tests._dense import random_hermitian


def _array(rng, P=12, radius=6.0):
    r = radius * np.sqrt(rng.uniform(size=P))
    t = rng.uniform(0, 2 * math.pi, size=P)
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def test_gradient_and_gauss_newton_block_against_finite_differences():
    rng = np.random.default_rng(1)
    pos, lam = _array(rng), 1.3
    l, m, z = 0.11, -0.07, 1.7
    B = random_hermitian(rng, pos.shape[0])

    def resid(d):
        a = offgrid.steering_at(pos, lam, [l + d[0]], [m + d[1]])
        return oracle.forward(a, np.array([z])) - B

    a0 = offgrid.steering_at(pos, lam, [l], [m])[:, 0]
    E = resid(np.zeros(2))
    g = offgrid.offset_gradient(pos, lam, a0, E, z)
    h = 1e-6
    f = lambda d: 0.5 * np.sum(np.abs(resid(d)) ** 2)  # noqa: E731
    g_fd = np.array([(f(np.array([h, 0])) - f(np.array([-h, 0]))) / (2 * h),
                     (f(np.array([0, h])) - f(np.array([0, -h]))) / (2 * h)])
    assert np.allclose(g, g_fd, rtol=1e-6, atol=1e-8 * np.abs(g_fd).max())
    # J^T J of the residual map against z^2 G
    J = np.stack([((resid(np.array([h, 0])) - resid(np.array([-h, 0]))) / (2 * h)).ravel(),
                  ((resid(np.array([0, h])) - resid(np.array([0, -h]))) / (2 * h)).ravel()], axis=1)
    JtJ = np.real(J.conj().T @ J)
    assert np.allclose(JtJ, z * z * offgrid.gauss_newton_block(pos, lam), rtol=1e-6)


def test_one_pixel_shift_is_the_neighbour():
    rng = np.random.default_rng(2)
    pos, lam = _array(rng), 1.0
    grid = (8, 6, -0.4, 0.1, -0.3, 0.1)
    A = oracle.steering(pos, lam, grid)
    l, m = oracle.pixel_directions(grid)
    a_shift = offgrid.steering_at(pos, lam, [l[10] + 0.1], [m[10]])[:, 0]
    assert np.allclose(a_shift, A[:, 11], atol=1e-12)
    a_shift = offgrid.steering_at(pos, lam, [l[10]], [m[10] + 0.1])[:, 0]
    assert np.allclose(a_shift, A[:, 18], atol=1e-12)


def _scene(rng, offsets, powers, P=16, n=11, noise=0.05):
    pos = _array(rng, P=P, radius=5.0)
    grid = (n, n, -0.5, 1.0 / (n - 1), -0.5, 1.0 / (n - 1))
    l, m = oracle.pixel_directions(grid)
    pix = [int(p) for p, _ in offsets]
    d = np.array([o for _, o in offsets]) * grid[3]
    As = offgrid.steering_at(pos, 1.0, l[pix] + d[:, 0], m[pix] + d[:, 1])
    R = (As * np.asarray(powers)[None, :]) @ As.conj().T + noise * np.eye(P)
    return pos, grid, 0.5 * (R + R.conj().T), pix, d


def test_zero_rounds_is_the_on_grid_solve():
    rng = np.random.default_rng(3)
    pos, grid, R, _, _ = _scene(rng, [(40, (0.3, -0.2)), (85, (0.0, 0.4))], [3.0, 1.5])
    A = oracle.steering(pos, 1.0, grid)
    B0 = R - 0.05 * np.eye(R.shape[0])
    eps = 0.02 * oracle.mf_image(A, R)
    ref = oracle.solve(A, B0, oracle.upper_bound(A, R), eps)
    res, delta = offgrid.solve_offgrid(pos, 1.0, grid, R, B0, eps, rounds=0)
    np.testing.assert_array_equal(res.state, ref.state)
    assert np.allclose(res.sigma, ref.sigma, rtol=1e-9, atol=1e-12)
    assert not delta.any()


def test_off_grid_sources_are_recovered():
    rng = np.random.default_rng(4)
    truth = [(40, (0.3, -0.25)), (85, (-0.2, 0.35))]
    powers = [3.0, 1.5]
    pos, grid, R, pix, d = _scene(rng, truth, powers, noise=0.05)
    A = oracle.steering(pos, 1.0, grid)
    B0 = R - 0.05 * np.eye(R.shape[0])
    eps = 0.05 * oracle.mf_image(A, R)
    # the MF bound: near an off-grid source the on-grid MVDR bound is far below
    # the source power (the bias that motivates the correction)
    on = oracle.solve(A, B0, oracle.upper_bound(A, R, kind="mf"), eps)
    res, delta = offgrid.solve_offgrid(pos, 1.0, grid, R, B0, eps, kind="mf", rounds=4)
    F = np.nonzero(res.state == oracle.STATE_F)[0]
    assert set(pix) <= set(F.tolist())
    for (p, _), dd, pw in zip(truth, d, powers):
        assert np.allclose(delta[p], dd, atol=0.02 * grid[3])
        assert abs(res.sigma[p] - pw) <= 0.02 * pw
    # the on-grid model leaves far more residual and spreads the power
    assert res.rel_residual < 0.2 * on.rel_residual
    assert np.sum(on.state == oracle.STATE_F) > len(pix)

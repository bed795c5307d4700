"""Pins of the oracle for K covariance blocks over one grid (CPU only).

* K identical blocks are the single-block problem (eq. vectRtotal with
  R_k = R, A_k = A): same MF and MVDR images, and the same solve -- including
  the thresholded release decisions, which see the (1/K)-scaled gradient;
* the stacked solve with distinct blocks (rotated array, another wavelength)
  matches SciPy's BVLS on the dense stacked Khatri-Rao matrix (objective and
  KKT conditions), and brute-force enumeration on a tiny grid;
* the MVDR image stays between the ASSC bound min_k 1/h_k (eq. ASSC0) and
  the MF image (the ordering shown after eq. MVDRUB2);
* both App. A variances against a Monte Carlo over independent sample
  covariances of each block.
"""

import math

import numpy as np
from scipy.optimize import lsq_linear

import oracle
from tests._dense import brute_force_box_ls, dense_psi, random_hermitian, real_stack, vect


def _rot(pos, ang):
    c, s = math.cos(ang), math.sin(ang)
    return pos @ np.array([[c, -s], [s, c]]).T


def _blocks(rng, P=5, Q=9, K=3):
    pos = rng.uniform(-3, 3, size=(P, 2))
    grid = (Q, 1, -0.6, 1.2 / Q, 0.0, 0.1)
    # Earth-rotation snapshots, the last one also at another wavelength
    geo = [(_rot(pos, 0.2 * k), 1.0 + 0.15 * (k == K - 1)) for k in range(K)]
    return oracle.steering_blocks(geo, grid), grid


def _sky_covs(rng, As, src, pw, noise=0.3):
    out = []
    for A in As:
        R = (A[:, src] * pw[None, :]) @ A[:, src].conj().T + noise * np.eye(A.shape[0])
        out.append(0.5 * (R + R.conj().T))
    return out


def test_identical_blocks_equal_the_single_block_problem():
    rng = np.random.default_rng(1)
    P, Q = 6, 16
    pos = rng.uniform(-3, 3, size=(P, 2))
    A = oracle.steering(pos, 1.0, (Q, 1, -0.7, 1.4 / Q, 0.0, 0.1))
    R = _sky_covs(rng, [A], np.array([3, 9, 12]), np.array([4.0, 1.5, 0.6]))[0]
    R = R + 0.05 * random_hermitian(rng, P)
    B0 = R - 0.3 * np.eye(P)
    mf = oracle.mf_image(A, R)
    gamma = oracle.upper_bound(A, R)
    eps = 0.35 * mf  # a threshold that stops some releases
    ref = oracle.solve(A, B0, gamma, eps, atol=1e-12, btol=1e-12)
    for K in (2, 3):
        As, Rs = [A] * K, [R] * K
        assert np.allclose(oracle.mf_image_multi(As, Rs), mf, rtol=1e-13)
        assert np.allclose(oracle.upper_bound_multi(As, Rs), gamma, rtol=1e-12)
        res = oracle.solve_multi(As, [B0] * K, gamma, eps, atol=1e-12, btol=1e-12)
        assert [e[0] for e in res.events] == [e[0] for e in ref.events]
        np.testing.assert_array_equal(res.state, ref.state)
        assert np.allclose(res.sigma, ref.sigma, rtol=1e-8, atol=1e-10 * np.abs(ref.sigma).max())
        assert abs(res.rel_residual - ref.rel_residual) <= 1e-9
    assert ref.adds >= 2 and np.any(ref.state == oracle.STATE_L)
    # App. A with kappa_b > 0: K independent sample covariances of the same R
    # average to an image whose standard deviation is 1/sqrt(K) of one block's,
    # so the K-block bound (pinned by Monte Carlo below) equals the
    # single-block bound with kappa_b / sqrt(K); K = 1 is the same problem.
    N, C = 300, 300 / (300 - P)
    for K in (1, 2, 3):
        As, Rs = [A] * K, [R] * K
        for kind, c in (("mvdr", C), ("mvdr", 1.0), ("mf", 1.0)):
            np.testing.assert_allclose(
                oracle.upper_bound_multi(As, Rs, kind, C=c, kappa_b=6.0, nsamples=N),
                oracle.upper_bound(A, R, kind, C=c, kappa_b=6.0 / math.sqrt(K), nsamples=N), rtol=1e-12)


def _dense_stacked(As, B0s):
    M = real_stack(np.vstack([dense_psi(A) for A in As]))
    b = real_stack(np.concatenate([vect(B) for B in B0s])[:, None])[:, 0]
    return M, b


def test_stacked_solve_matches_bvls_and_kkt():
    rng = np.random.default_rng(2)
    As, _ = _blocks(rng, P=5, Q=12, K=3)
    Rs = _sky_covs(rng, As, np.array([2, 7]), np.array([3.0, 1.0]))
    Rs = [R + 0.2 * random_hermitian(rng, R.shape[0]) for R in Rs]
    B0s = [R - 0.2 * np.eye(R.shape[0]) for R in Rs]
    gamma = oracle.upper_bound_multi(As, [R + 2.0 * np.eye(R.shape[0]) for R in Rs])
    res = oracle.solve_multi(As, B0s, gamma, np.zeros(12), atol=1e-14, btol=1e-14, conlim=1e14)
    M, b = _dense_stacked(As, B0s)
    ref = lsq_linear(M, b, bounds=(np.zeros(12), gamma), method="bvls", tol=1e-14)
    f = lambda s: 0.5 * np.sum((b - M @ s) ** 2)  # noqa: E731
    assert abs(f(res.sigma) - f(ref.x)) <= 1e-9 * max(f(ref.x), 1e-12)
    assert np.allclose(res.sigma, ref.x, atol=1e-7 * gamma.max())
    g = M.T @ (M @ res.sigma - b)
    scale = np.abs(M.T @ b).max()
    F = res.state == oracle.STATE_F
    assert np.all(np.abs(g[F]) <= 1e-6 * scale)
    assert np.all(g[res.state == oracle.STATE_L] >= -1e-6 * scale)
    assert np.all(g[res.state == oracle.STATE_U] <= 1e-6 * scale)


def test_stacked_solve_matches_brute_force_on_a_tiny_grid():
    rng = np.random.default_rng(3)
    As, _ = _blocks(rng, P=4, Q=6, K=2)
    Rs = _sky_covs(rng, As, np.array([1, 4]), np.array([2.0, 1.0]))
    Rs = [R + 0.3 * random_hermitian(rng, R.shape[0]) for R in Rs]
    gamma = np.full(6, 1.2)
    res = oracle.solve_multi(As, Rs, gamma, np.zeros(6), atol=1e-14, btol=1e-14, conlim=1e14)
    M, b = _dense_stacked(As, Rs)
    obj, x = brute_force_box_ls(M, b, gamma)
    assert abs(0.5 * np.sum((b - M @ res.sigma) ** 2) - obj) <= 1e-9 * max(obj, 1e-12)
    assert np.allclose(res.sigma, x, atol=1e-7)


def test_mvdr_between_assc_and_mf():
    rng = np.random.default_rng(4)
    As, _ = _blocks(rng, P=6, Q=20, K=3)
    Rs = [random_hermitian(rng, 6, pd=True) for _ in range(3)]
    mvdr = oracle.upper_bound_multi(As, Rs)
    mf = oracle.mf_image_multi(As, Rs)
    assc = np.min([1.0 / oracle.mvdr_inverse_power(A, R) for A, R in zip(As, Rs)], axis=0)
    assert np.all(mvdr <= mf * (1 + 1e-12))
    assert np.all(mvdr >= assc * (1 - 1e-12))
    # the blocks differ, so the bound is strictly looser than ASSC somewhere
    assert np.any(mvdr > assc * 1.01)


def test_app_a_variances_match_monte_carlo():
    rng = np.random.default_rng(5)
    P, N, trials, K = 5, 400, 500, 2
    As, _ = _blocks(rng, P=P, Q=4, K=K)
    Rs = [random_hermitian(rng, P, pd=True) for _ in range(K)]
    Ls = [np.linalg.cholesky(R) for R in Rs]
    mfs, mvs = [], []
    C = N / (N - P)
    for _ in range(trials):
        Rh = []
        for Lr in Ls:
            Y = Lr @ ((rng.standard_normal((P, N)) + 1j * rng.standard_normal((P, N))) / math.sqrt(2))
            Rh.append(Y @ Y.conj().T / N)
        mfs.append(oracle.mf_image_multi(As, Rh))
        mvs.append(oracle.upper_bound_multi(As, Rh, C=C))
    std_mf = oracle.mf_std_multi(As, Rs, N)
    assert np.allclose(np.std(mfs, axis=0), std_mf, rtol=0.12)
    # the bound's kappa_b term is one standard deviation of the MVDR image per unit of kappa_b
    std_mv = (oracle.upper_bound_multi(As, Rs, C=C, kappa_b=1.0, nsamples=N)
              - oracle.upper_bound_multi(As, Rs, C=C))
    assert np.allclose(np.std(mvs, axis=0), std_mv, rtol=0.12)
    assert np.allclose(oracle.detection_threshold_multi(As, Rs, 6.0, N), 6.0 * std_mf)

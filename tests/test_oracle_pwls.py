"""Pins of the oracle's PWLS formulation (eq. preWLS) against independent
constructions (CPU only).

* the whitening with the Cholesky factor has the cost of the paper's
  R^-1/2 weighting (eigendecomposition, built separately);
* the transformed operators equal the dense weighted, preconditioned
  Khatri-Rao matrix (R^-T/2 (x) R^-1/2) Psi D^-1 assembled with np.kron;
* the gradient at zero is minus the unbiased MVDR image (eqs. gmvdr, UBMVDRV)
  evaluated from R^-1 directly;
* the box-constrained PWLS solution matches SciPy's BVLS on the dense real
  system (objective, KKT);
* the threshold's standard deviation matches a Monte Carlo of the MVDR image
  over sample covariances (App. A).
"""

import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle
from oracle import pwls
from tests._dense import dense_psi, random_hermitian, real_stack, vect


def _small(rng, P=5, Q=7):
    pos = rng.uniform(-3, 3, size=(P, 2))
    grid = (Q, 1, -0.6, 1.2 / Q, 0.0, 0.1)
    A = oracle.steering(pos, 1.0, grid)
    R = random_hermitian(rng, P, pd=True)
    return A, R


def _inv_sqrt_hpd(R):
    w, V = np.linalg.eigh(R)
    return (V / np.sqrt(w)) @ V.conj().T


def test_cholesky_whitening_has_the_paper_cost():
    rng = np.random.default_rng(1)
    A, R = _small(rng)
    _, Linv = pwls.whitening_factor(R)
    Rm = _inv_sqrt_hpd(R)
    for _ in range(5):
        X = random_hermitian(rng, R.shape[0])
        a = np.linalg.norm(Linv @ X @ Linv.conj().T)
        b = np.linalg.norm(Rm @ X @ Rm)
        assert abs(a - b) <= 1e-12 * b


def test_transformed_operators_equal_dense_weighted_psi():
    rng = np.random.default_rng(2)
    A, R = _small(rng)
    Ahat, _, _, D = pwls.pwls_problem(A, R, R, np.ones(A.shape[1]))
    Rm = _inv_sqrt_hpd(R)
    # vec(R^-1/2 X R^-1/2) = ((R^-1/2)^T kron R^-1/2) vec(X), column stacking
    Wd = np.kron(Rm.T, Rm)
    Psi_pw = Wd @ dense_psi(A) @ np.diag(1.0 / D)
    v = rng.uniform(0, 1, A.shape[1])
    Y = oracle.forward(Ahat, v)
    # the Cholesky whitening differs from R^-1/2 by a unitary V on each side:
    # compare what is invariant (the Gram matrix and the norms)
    G1 = np.real(Psi_pw.conj().T @ Psi_pw)
    G2 = np.real(dense_psi(Ahat).conj().T @ dense_psi(Ahat))
    assert np.allclose(G1, G2, rtol=1e-10, atol=1e-12 * np.abs(G1).max())
    assert abs(np.linalg.norm(vect(Y)) - np.linalg.norm(Psi_pw @ v)) <= 1e-10 * np.linalg.norm(Psi_pw @ v)
    # adjoint of the whitened residual: D^-1 Psi^H (R^-T kron R^-1) vec(B)
    B = random_hermitian(rng, R.shape[0])
    Ri = np.linalg.inv(R)
    g_dense = np.real((dense_psi(A).conj().T @ np.kron(Ri.T, Ri) @ vect(B))) / D
    _, Linv = pwls.whitening_factor(R)
    g = oracle.adjoint(Ahat, Linv @ B @ Linv.conj().T)
    assert np.allclose(g, g_dense, rtol=1e-10, atol=1e-12 * np.abs(g_dense).max())


@pytest.mark.parametrize("C", [1.0, 0.8])
def test_gradient_at_zero_is_minus_unbiased_mvdr_image(C):
    rng = np.random.default_rng(3)
    A, R = _small(rng, P=6, Q=9)
    Ahat, Bhat, _, D = pwls.pwls_problem(A, R, R, np.ones(A.shape[1]), C=C)
    g0 = -oracle.adjoint(Ahat, Bhat)  # gradient of 1/2||Bhat - Psi_hat s||^2 at s = 0
    Ri = np.linalg.inv(R)
    h = np.array([np.real(A[:, i].conj() @ Ri @ A[:, i]) for i in range(A.shape[1])])
    assert np.allclose(g0, -C / h, rtol=1e-11)


@pytest.mark.parametrize("kind", ["mvdr", "mf"])
def test_box_pwls_matches_bvls_and_kkt(kind):
    rng = np.random.default_rng(4)
    A, R = _small(rng, P=5, Q=12)
    B0 = R - 0.3 * np.eye(R.shape[0])
    gamma = oracle.upper_bound(A, R, kind=kind)
    res = pwls.solve_pwls(A, R, B0, gamma, np.zeros(A.shape[1]), atol=1e-14, btol=1e-14, conlim=1e14)
    Ahat, Bhat, gpw, D = pwls.pwls_problem(A, R, B0, gamma)
    M = real_stack(dense_psi(Ahat))
    b = real_stack(vect(Bhat)[:, None])[:, 0]
    ref = lsq_linear(M, b, bounds=(np.zeros_like(gpw), gpw), method="bvls", tol=1e-14)
    f = lambda s: 0.5 * np.sum((b - M @ s) ** 2)  # noqa: E731
    assert abs(f(res.sigma_pw) - f(ref.x)) <= 1e-9 * max(f(ref.x), 1e-12)
    assert np.allclose(res.sigma_pw, ref.x, atol=1e-7 * max(gpw.max(), 1.0))
    assert np.allclose(res.sigma, res.sigma_pw / D)
    # KKT in the PWLS variable: free pixels have zero gradient, bounds the right sign
    g = M.T @ (M @ res.sigma_pw - b)
    F = res.state == oracle.STATE_F
    scale = np.abs(M.T @ b).max()
    assert np.all(np.abs(g[F]) <= 1e-6 * scale)
    assert np.all(g[res.state == oracle.STATE_L] >= -1e-6 * scale)
    assert np.all(g[res.state == oracle.STATE_U] <= 1e-6 * scale)


def test_threshold_std_matches_monte_carlo_of_mvdr_image():
    rng = np.random.default_rng(5)
    P, N, trials = 6, 400, 600
    A, R = _small(rng, P=P, Q=3)
    Lr = np.linalg.cholesky(R)
    h_true = np.real(np.sum(A.conj() * (np.linalg.inv(R) @ A), axis=0))
    vals = []
    for _ in range(trials):
        Y = Lr @ ((rng.standard_normal((P, N)) + 1j * rng.standard_normal((P, N))) / math.sqrt(2))
        Rh = Y @ Y.conj().T / N
        vals.append(1.0 / oracle.mvdr_inverse_power(A, Rh))
    vals = np.array(vals)
    C = N / (N - P + 1)  # unbiased MVDR scale (inverse-Wishart mean)
    std_mc = np.std(C * vals, axis=0)
    eps = pwls.pwls_threshold(h_true, 1.0, N, P)
    assert np.allclose(std_mc, eps, rtol=0.12)


def test_upper_set_pixels_sit_at_the_image_bound():
    # the bound of eq. preWLS is D gamma in the PWLS variable, i.e. gamma in
    # image units: pixels stopped at it carry exactly gamma_i in the image
    rng = np.random.default_rng(6)
    A, R = _small(rng, P=5, Q=12)
    gamma = 0.3 * oracle.upper_bound(A, R)
    res = pwls.solve_pwls(A, R, R, gamma, np.zeros(A.shape[1]), atol=1e-14, btol=1e-14, conlim=1e14)
    U = res.state == oracle.STATE_U
    assert U.any()
    assert np.allclose(res.sigma[U], gamma[U], rtol=1e-12)
    assert np.all(res.sigma <= gamma * (1 + 1e-12)) and np.all(res.sigma >= 0)

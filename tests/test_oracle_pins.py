"""Pins for the FP64 oracle against mathematics the paper fixes (CPU only).

Each test names the passage of the paper it checks.  None of them retypes the
oracle's own formula: the references are the Notation identities evaluated on
an explicitly built Khatri-Rao matrix, closed forms for a single source,
inequalities, SVD / BVLS / brute-force solutions and invariances.
"""

import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle
import synth
from tests._dense import (brute_force_box_ls, dense_psi, random_hermitian, real_stack,
                          steering_direct, vect)


def _small_geometry(rng, P=6, n=4, L=0.5, radius=3.0, lam=1.0):
    r = radius * np.sqrt(rng.random(P))
    t = 2 * math.pi * rng.random(P)
    pos = np.stack([r * np.cos(t), r * np.sin(t)], axis=1)
    d = 2 * L / n
    grid = (n, n, -L, d, -L, d)
    return pos, lam, grid


# --- steering vectors (Sec. II-A normalisation, Sec. III-E response model) ------------

def test_steering_matches_entrywise_model_and_is_unit_norm():
    rng = np.random.default_rng(1)
    pos, lam, grid = _small_geometry(rng, P=7, n=5)
    A = oracle.steering(pos, lam, grid)
    nl, nm, l0, dl, m0, dm = grid
    l = [l0 + (i % nl) * dl for i in range(nl * nm)]
    m = [m0 + (i // nl) * dm for i in range(nl * nm)]
    np.testing.assert_allclose(A, steering_direct(pos, lam, l, m), rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.abs(A) ** 2, 1.0 / 7, rtol=1e-14)
    np.testing.assert_allclose(np.sum(np.abs(A) ** 2, axis=0), 1.0, rtol=1e-14)


def test_pixel_order_is_l_fastest():
    grid = (3, 2, -1.0, 0.5, 2.0, 0.25)
    l, m = oracle.pixel_directions(grid)
    assert list(l) == [-1.0, -0.5, 0.0, -1.0, -0.5, 0.0]
    assert list(m) == [2.0, 2.0, 2.0, 2.25, 2.25, 2.25]


def test_array_translation_leaves_operators_unchanged():
    # A common shift of all antennas multiplies each column by a phase, so
    # a_i a_i^H (hence Psi) does not change.
    rng = np.random.default_rng(2)
    pos, lam, grid = _small_geometry(rng)
    A = oracle.steering(pos, lam, grid)
    A2 = oracle.steering(pos + np.array([3.7, -11.2]), lam, grid)
    v = rng.standard_normal(A.shape[1])
    U = random_hermitian(rng, A.shape[0])
    np.testing.assert_allclose(oracle.forward(A2, v), oracle.forward(A, v), atol=1e-12)
    np.testing.assert_allclose(oracle.adjoint(A2, U), oracle.adjoint(A, U), atol=1e-12)


def test_transposed_covariance_mirrors_the_image():
    # Negating every position conjugates A; the beamformer output then equals
    # that of the transposed covariance: a transposed R_hat mirrors the sky.
    rng = np.random.default_rng(3)
    pos, lam, grid = _small_geometry(rng)
    A = oracle.steering(pos, lam, grid)
    Am = oracle.steering(-pos, lam, grid)
    R = random_hermitian(rng, A.shape[0], pd=True)
    np.testing.assert_allclose(oracle.mf_image(Am, R), oracle.mf_image(A, R.T), atol=1e-12)
    assert not np.allclose(oracle.mf_image(A, R.T), oracle.mf_image(A, R), atol=1e-6)


# --- Khatri-Rao operators (Notation identities, eqs. vectRImg / bAt, Sec. IV-B) --------

def test_forward_and_adjoint_equal_dense_khatri_rao_psi():
    rng = np.random.default_rng(4)
    pos, lam, grid = _small_geometry(rng, P=5, n=4)
    A = oracle.steering(pos, lam, grid)
    Psi = dense_psi(A)
    v = rng.standard_normal(A.shape[1])
    np.testing.assert_allclose(vect(oracle.forward(A, v)), Psi @ v, atol=1e-14)
    U = random_hermitian(rng, 5)
    np.testing.assert_allclose(oracle.adjoint(A, U), np.real(Psi.conj().T @ vect(U)), atol=1e-14)
    # and the imaginary part of Psi^H vect(U) vanishes for Hermitian U
    np.testing.assert_allclose(np.imag(Psi.conj().T @ vect(U)), 0.0, atol=1e-14)


def test_adjointness_to_1e12():
    rng = np.random.default_rng(5)
    pos, lam, grid = _small_geometry(rng, P=9, n=6)
    A = oracle.steering(pos, lam, grid)
    S = rng.choice(A.shape[1], size=17, replace=False)
    x = rng.standard_normal(S.size)
    Y = random_hermitian(rng, 9)
    lhs = np.real(np.vdot(oracle.forward(A[:, S], x), Y))
    rhs = float(x @ oracle.adjoint(A[:, S], Y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_deconvolution_matrix_closed_form():
    # eq. convMat at K=1: H = (A^T A^*) o (A^H A), i.e. H_ij = |a_i^H a_j|^2.
    rng = np.random.default_rng(6)
    pos, lam, grid = _small_geometry(rng, P=6, n=4)
    A = oracle.steering(pos, lam, grid)
    G = A.conj().T @ A
    for j in range(A.shape[1]):
        e = np.zeros(A.shape[1])
        e[j] = 1.0
        np.testing.assert_allclose(oracle.adjoint(A, oracle.forward(A, e)), np.abs(G[:, j]) ** 2,
                                   atol=1e-14)


# --- dirty images and bounds (eqs. mfdimg, MFupper, wmvdr, mvdr_upper; Sec. II-C) -------

def test_mf_image_is_psi_h_r():
    rng = np.random.default_rng(7)
    pos, lam, grid = _small_geometry(rng, P=6, n=5)
    A = oracle.steering(pos, lam, grid)
    R = random_hermitian(rng, 6, pd=True)
    np.testing.assert_allclose(oracle.mf_image(A, R), np.real(dense_psi(A).conj().T @ vect(R)),
                               atol=1e-13)


def _single_source(rng, P=8, n=6):
    pos, lam, grid = _small_geometry(rng, P=P, n=n, radius=4.0)
    A = oracle.steering(pos, lam, grid)
    i0 = 13
    s0, sn = 7.5, 0.8
    R = s0 * np.outer(A[:, i0], A[:, i0].conj()) + sn * np.eye(P)
    return A, R, i0, s0, sn


def test_single_source_mf_closed_form():
    # eq. MFupper: sigma_MF,i = s0 |a_i^H a0|^2 + sn for R = s0 a0 a0^H + sn I.
    A, R, i0, s0, sn = _single_source(np.random.default_rng(8))
    c = np.abs(A.conj().T @ A[:, i0]) ** 2
    np.testing.assert_allclose(oracle.mf_image(A, R), s0 * c + sn, rtol=1e-13)


def test_single_source_mvdr_sherman_morrison():
    # R^-1 = (I - s0 a0 a0^H /(sn + s0)) / sn, so 1/h_i = sn / (1 - s0 c_i /(sn + s0)),
    # which equals s0 + sn at the source pixel (eq. mvdr_upper is tight there).
    A, R, i0, s0, sn = _single_source(np.random.default_rng(9))
    c = np.abs(A.conj().T @ A[:, i0]) ** 2
    expect = sn / (1.0 - s0 * c / (sn + s0))
    got = oracle.upper_bound(A, R, "mvdr")
    np.testing.assert_allclose(got, expect, rtol=1e-12)
    assert abs(got[i0] - (s0 + sn)) < 1e-12 * (s0 + sn)


def test_mvdr_below_mf_and_above_truth():
    # Sec. II-D: sigma <= MVDR <= MF, with the true R; MVDR <= MF also with R_hat.
    sc = synth.make_scene("c0")
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    for R in (sc.R_hat, synth.exact_covariance(sc.pos, sc.lam, sc.grid, sc.src_pix, sc.src_pow,
                                               sc.noise_var)):
        mf = oracle.mf_image(A, R)
        mv = oracle.upper_bound(A, R, "mvdr")
        assert np.all(mv <= mf * (1 + 1e-12))
    Rt = synth.exact_covariance(sc.pos, sc.lam, sc.grid, sc.src_pix, sc.src_pow, sc.noise_var)
    mv = oracle.upper_bound(A, Rt, "mvdr")
    assert np.all(sc.true_image() <= mv * (1 + 1e-12))


def test_mvdr_equals_jacobi_preconditioned_wls_dirty_image():
    # Sec. II-C at K=1: D_WLS^-1 sigma_WLS is the MVDR image, built here from the dense
    # weighted operator (R^-T kron R^-1) of eqs. imagingeqwls / imagingeqwls2.
    rng = np.random.default_rng(10)
    pos, lam, grid = _small_geometry(rng, P=5, n=4)
    A = oracle.steering(pos, lam, grid)
    R = random_hermitian(rng, 5, pd=True)
    Psi = dense_psi(A)
    Ri = np.linalg.inv(R)
    W = np.kron(Ri.T, Ri)
    s_wls = np.real(Psi.conj().T @ W @ vect(R))
    D = np.real(np.diag(Psi.conj().T @ W @ Psi))
    np.testing.assert_allclose(oracle.upper_bound(A, R, "mvdr"), s_wls / D, rtol=1e-11)


def test_bound_options():
    rng = np.random.default_rng(11)
    pos, lam, grid = _small_geometry(rng, P=6, n=4)
    A = oracle.steering(pos, lam, grid)
    R = random_hermitian(rng, 6, pd=True)
    N = 500
    h = 1.0 / oracle.upper_bound(A, R, "mvdr")
    # C scales the MVDR image; kappa_b adds kappa_b * std, App. A: std = 1/(h sqrt(N-P-1))
    C = N / (N - 6)
    np.testing.assert_allclose(oracle.upper_bound(A, R, "mvdr", C=C), C / h, rtol=1e-13)
    np.testing.assert_allclose(oracle.upper_bound(A, R, "mvdr", kappa_b=6.0, nsamples=N),
                               1 / h + 6.0 / (h * math.sqrt(N - 7)), rtol=1e-13)
    mf = oracle.mf_image(A, R)
    np.testing.assert_allclose(oracle.upper_bound(A, R, "mf", kappa_b=6.0, nsamples=N),
                               mf * (1 + 6.0 / math.sqrt(N)), rtol=1e-13)
    assert np.all(np.isinf(oracle.upper_bound(A, R, "none")))
    np.testing.assert_allclose(oracle.detection_threshold(mf, 6.0, N), 6.0 * mf / math.sqrt(N))


def test_single_block_bound_terms_are_app_a_std_by_monte_carlo():
    # App. A at K = 1: the kappa_b term of each bound is one standard deviation
    # of the image it inflates, per unit of kappa_b, and the detection
    # threshold is kappa_d of the MF image's.  Reference: the spread of the
    # images over many independent sample covariances of one R (complex
    # Gaussian samples, N R_hat complex Wishart).  A small N (13 samples, 4
    # antennas) makes the MVDR degrees of freedom visible: the first-order
    # std 1/(h sqrt(N-P-1)) is within 0.7 % of the exact one, a neighbouring
    # count (N-P, N-P+1) is 5-13 % off.
    rng = np.random.default_rng(14)
    P, N, trials = 4, 13, 60000
    pos, lam, grid = _small_geometry(rng, P=P, n=3, radius=1.5)
    A = oracle.steering(pos, lam, grid)
    R = random_hermitian(rng, P, pd=True)
    Lr = np.linalg.cholesky(R)
    W = (rng.standard_normal((trials, P, N)) + 1j * rng.standard_normal((trials, P, N))) / math.sqrt(2)
    Y = Lr[None] @ W
    Rh = Y @ np.conj(np.swapaxes(Y, 1, 2)) / N
    quad = lambda M: np.real(np.einsum("pi,tpq,qi->ti", A.conj(), M, A))  # noqa: E731
    mf_mc = quad(Rh)
    C = N / (N - P)  # the unbiased MVDR image (Sec. II-D)
    mv_mc = C / quad(np.linalg.inv(Rh))
    # MVDR: increment of the bound at kappa_b = 1 over the bound itself
    d_mv = (oracle.upper_bound(A, R, "mvdr", C=C, kappa_b=1.0, nsamples=N)
            - oracle.upper_bound(A, R, "mvdr", C=C))
    np.testing.assert_allclose(mv_mc.std(axis=0), d_mv, rtol=0.025)
    # MF: exact, N mf_hat / mf is Gamma(N) distributed
    d_mf = (oracle.upper_bound(A, R, "mf", kappa_b=1.0, nsamples=N) - oracle.upper_bound(A, R, "mf"))
    np.testing.assert_allclose(mf_mc.std(axis=0), d_mf, rtol=0.025)
    np.testing.assert_allclose(mf_mc.std(axis=0), oracle.detection_threshold(oracle.mf_image(A, R), 1.0, N),
                               rtol=0.025)
    # kappa_b scales the increment linearly
    d_mv3 = (oracle.upper_bound(A, R, "mvdr", C=C, kappa_b=3.0, nsamples=N)
             - oracle.upper_bound(A, R, "mvdr", C=C))
    np.testing.assert_allclose(d_mv3, 3.0 * mv_mc.std(axis=0), rtol=0.025)


def test_inverse_wishart_bias_constant_monte_carlo():
    # App. A: E{R_hat^-1} = N/(N-P) R^-1, the origin of the constant C.
    rng = np.random.default_rng(12)
    P, N, trials = 4, 40, 4000
    R = random_hermitian(rng, P, pd=True)
    Lc = np.linalg.cholesky(R)
    acc = np.zeros((P, P), dtype=complex)
    for _ in range(trials):
        y = Lc @ ((rng.standard_normal((P, N)) + 1j * rng.standard_normal((P, N))) / math.sqrt(2))
        acc += np.linalg.inv(y @ y.conj().T / N)
    ratio = np.real(np.trace(acc / trials @ R)) / P
    assert abs(ratio - N / (N - P)) < 0.01


def test_not_positive_definite_is_rejected():
    rng = np.random.default_rng(13)
    pos, lam, grid = _small_geometry(rng, P=4, n=3)
    A = oracle.steering(pos, lam, grid)
    R = random_hermitian(rng, 4)
    R = R - (np.linalg.eigvalsh(R).max() + 1.0) * np.eye(4)     # negative definite
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.upper_bound(A, R, "mvdr")
    Rn = np.eye(4, dtype=complex)
    Rn[1, 2] = np.nan
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.mf_image(A, Rn)


# --- LSQR (Sec. IV-A) ----------------------------------------------------------------

def _lsqr_problem(rng, P, nF, consistent=False):
    pos, lam, grid = _small_geometry(rng, P=P, n=6, radius=3.0)
    A = oracle.steering(pos, lam, grid)
    F = np.sort(rng.choice(A.shape[1], size=nF, replace=False))
    A_F = A[:, F]
    if consistent:
        b = oracle.forward(A_F, rng.standard_normal(nF))
    else:
        b = random_hermitian(rng, P)
    return A_F, b


@pytest.mark.parametrize("P,nF", [(6, 8), (4, 12)])
def test_lsqr_matches_svd_minimum_norm_solution(P, nF):
    # (4, 12): rank Psi_F <= P(P-1)+1 = 13 but 12 columns of a 36-pixel grid on 4
    # antennas are nearly dependent; (6, 8) is well determined.
    rng = np.random.default_rng(20 + P)
    A_F, b = _lsqr_problem(rng, P, nF)
    res = oracle.lsqr(lambda v: oracle.forward(A_F, v), lambda u: oracle.adjoint(A_F, u), b, nF,
                      atol=1e-14, btol=1e-14, conlim=1e16, itnlim=500)
    M = real_stack(dense_psi(A_F))
    x_ref = np.linalg.lstsq(M, real_stack(vect(b)[:, None])[:, 0], rcond=1e-12)[0]
    np.testing.assert_allclose(res.x, x_ref, rtol=0, atol=1e-8 * max(1.0, np.abs(x_ref).max()))
    r = real_stack(vect(b)[:, None])[:, 0] - M @ res.x
    assert abs(res.rnorm - np.linalg.norm(r)) < 1e-8 * np.linalg.norm(r) + 1e-12


def test_lsqr_minimum_norm_when_rank_deficient():
    # more unknowns than the rank of Psi_F: LSQR from zero returns the pseudo-inverse solution
    rng = np.random.default_rng(31)
    P = 2                                   # rank Psi <= P^2 = 4 real dims of Hermitian 2x2
    pos, lam, grid = _small_geometry(rng, P=P, n=3, radius=2.0)
    A_F = oracle.steering(pos, lam, grid)[:, :7]
    b = random_hermitian(rng, P)
    res = oracle.lsqr(lambda v: oracle.forward(A_F, v), lambda u: oracle.adjoint(A_F, u), b, 7,
                      atol=1e-15, btol=1e-15, conlim=1e16, itnlim=200)
    M = real_stack(dense_psi(A_F))
    x_ref = np.linalg.pinv(M, rcond=1e-10) @ real_stack(vect(b)[:, None])[:, 0]
    np.testing.assert_allclose(res.x, x_ref, atol=1e-9)


def test_lsqr_consistent_system_recovers_exactly_and_residual_decreases():
    rng = np.random.default_rng(32)
    A_F, b = _lsqr_problem(rng, 6, 10, consistent=True)
    M = real_stack(dense_psi(A_F))
    bb = real_stack(vect(b)[:, None])[:, 0]
    prev = math.inf
    for k in range(1, 11):
        res = oracle.lsqr(lambda v: oracle.forward(A_F, v), lambda u: oracle.adjoint(A_F, u), b, 10,
                          atol=0.0, btol=0.0, conlim=1e30, itnlim=k)
        true_r = np.linalg.norm(bb - M @ res.x)
        assert abs(true_r - res.rnorm) <= 1e-9 * np.linalg.norm(bb)
        assert true_r <= prev + 1e-12
        prev = true_r
    res = oracle.lsqr(lambda v: oracle.forward(A_F, v), lambda u: oracle.adjoint(A_F, u), b, 10,
                      atol=1e-12, btol=1e-12, itnlim=100)
    assert res.istop == 1
    assert np.linalg.norm(bb - M @ res.x) <= 1e-10 * np.linalg.norm(bb)


def test_lsqr_stops_on_normal_residual_test():
    rng = np.random.default_rng(33)
    A_F, b = _lsqr_problem(rng, 6, 9)
    res = oracle.lsqr(lambda v: oracle.forward(A_F, v), lambda u: oracle.adjoint(A_F, u), b, 9,
                      atol=1e-6, btol=1e-6, itnlim=200)
    assert res.istop == 2
    M = real_stack(dense_psi(A_F))
    r = real_stack(vect(b)[:, None])[:, 0] - M @ res.x
    assert np.linalg.norm(M.T @ r) <= 1.5e-6 * np.linalg.norm(M) * np.linalg.norm(r)


def test_lsqr_empty_and_zero_rhs():
    res = oracle.lsqr(lambda v: 0, lambda u: np.zeros(0), np.ones((2, 2)), 0)
    assert res.x.size == 0 and res.itn == 0
    A_F, _ = _lsqr_problem(np.random.default_rng(34), 4, 3)
    res = oracle.lsqr(lambda v: oracle.forward(A_F, v), lambda u: oracle.adjoint(A_F, u),
                      np.zeros((4, 4), complex), 3)
    assert np.all(res.x == 0) and res.itn == 0


# --- active set (Sec. III: eqs. CLS, gradFcond, etaL, etaU, Table I) ------------------

def _box_problem(rng, P, n, n_src=3, noise=0.5, N=200, radius=2.5):
    pos, lam, grid = _small_geometry(rng, P=P, n=n, radius=radius)
    Q = n * n
    src = rng.choice(Q, size=n_src, replace=False)
    pw = 1 + 4 * rng.random(n_src)
    R = synth.exact_covariance(pos, lam, grid, src, pw, noise)
    Lc = np.linalg.cholesky(R)
    y = Lc @ ((rng.standard_normal((P, N)) + 1j * rng.standard_normal((P, N))) / math.sqrt(2))
    Rh = y @ y.conj().T / N
    Rh = 0.5 * (Rh + Rh.conj().T)
    A = oracle.steering(pos, lam, grid)
    return A, Rh, noise


def _kkt(A, B0, sigma, state, gamma, tol):
    g = oracle.adjoint(A, oracle.forward(A, sigma) - B0)
    F, L, U = state == 1, state == 0, state == 2
    scale = np.abs(oracle.adjoint(A, B0)).max()
    assert np.all(np.abs(g[F]) <= tol * scale)
    assert np.all(g[L] >= -tol * scale)
    assert np.all(-g[U] >= -tol * scale)
    assert np.all(sigma[L] == 0) and np.all(sigma[U] == gamma[U])
    assert np.all(sigma >= 0) and np.all(sigma <= gamma)


@pytest.mark.parametrize("seed,bound", [(40, "mvdr"), (41, "mf"), (42, "mvdr")])
def test_active_set_matches_bvls_objective_and_kkt(seed, bound):
    rng = np.random.default_rng(seed)
    A, Rh, noise = _box_problem(rng, P=6, n=5)
    B0 = Rh - noise * np.eye(6)
    gamma = oracle.upper_bound(A, Rh, bound)
    res = oracle.solve(A, B0, gamma, np.zeros(A.shape[1]), atol=1e-13, btol=1e-13, conlim=1e14)
    assert res.status == 0
    M = real_stack(dense_psi(A))
    bb = real_stack(vect(B0)[:, None])[:, 0]
    ref = lsq_linear(M, bb, bounds=(np.zeros(A.shape[1]), gamma), method="bvls", tol=1e-14)
    assert abs(res.objective - ref.cost) <= 1e-8 * max(ref.cost, 1e-12)
    _kkt(A, B0, res.sigma, res.state, gamma, 1e-7)


def test_active_set_matches_brute_force_enumeration():
    rng = np.random.default_rng(50)
    pos, lam, grid = _small_geometry(rng, P=3, n=3, radius=1.5)
    grid = (3, 2) + grid[2:]                  # Q = 6 -> 729 patterns
    A = oracle.steering(pos, lam, grid)
    src = [1, 4]
    R = synth.exact_covariance(pos, lam, grid, src, [3.0, 1.5], 0.3)
    R = R + 0.05 * random_hermitian(rng, 3)
    B0 = R - 0.3 * np.eye(3)
    gamma = np.array([0.5, 2.0, 1.0, 3.0, 0.8, 1.2])
    res = oracle.solve(A, B0, gamma, np.zeros(6), atol=1e-14, btol=1e-14, conlim=1e15)
    M = real_stack(dense_psi(A))
    bb = real_stack(vect(B0)[:, None])[:, 0]
    obj, _x = brute_force_box_ls(M, bb, gamma)
    assert abs(res.objective - obj) <= 1e-9 * max(obj, 1e-12)


def test_first_release_is_dirty_image_peak():
    # Sec. III-C: from sigma = 0 the multipliers are the negated (noise-subtracted) dirty
    # image, so the first pixel released is the brightest dirty-image pixel.
    sc = synth.make_scene("c0")
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    mf = oracle.mf_image(A, R)
    res = oracle.solve(A, R - sc.noise_var * np.eye(sc.P), oracle.upper_bound(A, R),
                       oracle.detection_threshold(mf, 6.0, sc.N))
    assert res.events[0][0] == "feasible"
    assert res.events[1] == ("add", int(np.argmax(mf)))


@pytest.mark.parametrize("sources", [[(200, 5.0)], [(200, 5.0), (615, 2.0)]])
def test_exact_recovery_from_exact_covariance(sources):
    rng = np.random.default_rng(60)
    pos, lam, grid = _small_geometry(rng, P=16, n=32, radius=20.0)
    pix = [s[0] for s in sources]
    pw = [s[1] for s in sources]
    noise = 1.0
    R = synth.exact_covariance(pos, lam, grid, pix, pw, noise)
    A = oracle.steering(pos, lam, grid)
    mf = oracle.mf_image(A, R)
    gamma = oracle.upper_bound(A, R) * (1 + 1e-9)   # true powers sit exactly at the bound
    res = oracle.solve(A, R - noise * np.eye(16), gamma, oracle.detection_threshold(mf, 6.0, 10 ** 6),
                       atol=1e-13, btol=1e-13, conlim=1e14)
    assert sorted(np.nonzero(res.state == 1)[0].tolist()) == sorted(pix)
    np.testing.assert_allclose(res.sigma[pix], pw, rtol=1e-8)
    assert res.rel_residual < 1e-8


def test_scale_and_antenna_permutation_invariance():
    sc = synth.make_scene("c0")
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)

    def run(pos, Rm, noise):
        Am = oracle.steering(pos, sc.lam, sc.grid)
        mf = oracle.mf_image(Am, Rm)
        return oracle.solve(Am, Rm - noise * np.eye(sc.P), oracle.upper_bound(Am, Rm),
                            oracle.detection_threshold(mf, 6.0, sc.N))

    base = run(sc.pos, R, sc.noise_var)
    scaled = run(sc.pos, 3.0 * R, 3.0 * sc.noise_var)
    np.testing.assert_array_equal(scaled.state, base.state)
    np.testing.assert_allclose(scaled.sigma, 3.0 * base.sigma, rtol=1e-8, atol=1e-12)
    perm = np.random.default_rng(70).permutation(sc.P)
    permuted = run(sc.pos[perm], R[np.ix_(perm, perm)], sc.noise_var)
    np.testing.assert_array_equal(permuted.state, base.state)
    np.testing.assert_allclose(permuted.sigma, base.sigma, rtol=1e-8, atol=1e-12)
    assert A.shape == (sc.P, sc.Q)


def test_solution_respects_bounds_and_kkt_with_threshold():
    # with kappa_d > 0 the exit state still satisfies the box, g_F = 0, and
    # lambda >= -eps on the active pixels (the detection test failed everywhere)
    sc = synth.make_scene("c0")
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    mf = oracle.mf_image(A, R)
    gamma = oracle.upper_bound(A, R)
    eps = oracle.detection_threshold(mf, 6.0, sc.N)
    B0 = R - sc.noise_var * np.eye(sc.P)
    res = oracle.solve(A, B0, gamma, eps)
    assert np.all(res.sigma >= 0) and np.all(res.sigma <= gamma) and np.all(gamma <= mf)
    g = oracle.adjoint(A, oracle.forward(A, res.sigma) - B0)
    F = res.state == 1
    assert np.abs(g[F]).max() <= 1e-6 * np.abs(mf).max()
    lam = np.where(res.state == 0, g, -g)
    assert np.all(lam[~F] >= -eps[~F])


def test_resume_from_returned_state_is_a_fixed_point():
    sc = synth.make_scene("c0")
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    mf = oracle.mf_image(A, R)
    gamma = oracle.upper_bound(A, R)
    eps = oracle.detection_threshold(mf, 6.0, sc.N)
    B0 = R - sc.noise_var * np.eye(sc.P)
    res = oracle.solve(A, B0, gamma, eps)
    again = oracle.solve(A, B0, gamma, eps, sigma0=res.sigma, state0=res.state)
    np.testing.assert_array_equal(again.state, res.state)
    np.testing.assert_allclose(again.sigma, res.sigma, rtol=1e-9)
    assert again.adds == 0 and again.outer_iters == 1


def test_max_outer_guard():
    sc = synth.make_scene("c0")
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    mf = oracle.mf_image(A, R)
    res = oracle.solve(A, R - sc.noise_var * np.eye(sc.P), oracle.upper_bound(A, R),
                       oracle.detection_threshold(mf, 6.0, sc.N), max_outer=3)
    assert res.status == 1 and res.outer_iters == 3

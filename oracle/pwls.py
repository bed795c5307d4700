"""Constrained preconditioned weighted least squares (PWLS), eq. preWLS.

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).

Sec. II-E / III-B: with the weighting of eq. def:vecfWLS and the change of
variable sigma_pw = D sigma of eq. D (K = 1: D_i = h_i^2 / C with
h_i = a_i^H R^-1 a_i), the problem is

    min 1/2 || W (b - Psi D^-1 sigma_pw) ||^2   s.t.  0 <= sigma_pw <= D gamma,

and the image is sigma = D^-1 sigma_pw.  The weighting W applies
R^-1/2 on both sides of a covariance-shaped matrix; with the Cholesky factor
R = L L^H, ``X -> L^-1 X L^-H`` gives the same norm (L^-1 = V R^-1/2 for a
unitary V).  Writing the whitened, scaled steering vectors
``ahat_i = L^-1 a_i / sqrt(D_i)``, the problem is the LS problem of eq. CLS
with A replaced by Ahat, the data by L^-1 b L^-H and the bound by D gamma; its
gradient at any point is that of eq. gmvdr, and at sigma_pw = 0 with b = R it
is minus the unbiased MVDR image C / h (eq. UBMVDRV).  So the same active-set
solver (Table I) with LSQR runs unchanged on the transformed inputs.

Detection threshold (Sec. III-C, App. A): the multipliers of PWLS have the
statistics of the MVDR image, whose standard deviation at K = 1 is
``1 / (h_i sqrt(N - P - 1))``; epsilon_i = kappa_d times that.
"""

import math

import numpy as np

from .active_set import solve
from .imaging import NotPositiveDefinite, _check_covariance


def whitening_factor(R):
    """Cholesky factor L of R = L L^H and its inverse (FP64)."""
    R = _check_covariance(R)
    try:
        L = np.linalg.cholesky(R)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc
    Linv = np.linalg.solve(L, np.eye(R.shape[0], dtype=np.complex128))
    return L, Linv


def pwls_scaling(A, R, C=1.0):
    """D_i = h_i^2 / C (eq. D at K = 1) and h_i = a_i^H R^-1 a_i."""
    _, Linv = whitening_factor(R)
    W = Linv @ A
    h = np.sum(np.abs(W) ** 2, axis=0)  # a^H L^-H L^-1 a
    return h * h / C, h


def pwls_threshold(h, kappa_d, nsamples, P):
    """epsilon_i = kappa_d * std of the MVDR image pixel (App. A, K = 1)."""
    return kappa_d / (np.asarray(h, dtype=np.float64) * math.sqrt(nsamples - P - 1))


def pwls_problem(A, R, B0, gamma, C=1.0):
    """The LS-form inputs of the PWLS problem: (Ahat, Bhat, gamma_pw, D)."""
    _, Linv = whitening_factor(R)
    D, _ = pwls_scaling(A, R, C)
    Ahat = (Linv @ A) / np.sqrt(D)[None, :]
    Bhat = Linv @ np.asarray(B0, dtype=np.complex128) @ Linv.conj().T
    gamma_pw = D * np.asarray(gamma, dtype=np.float64)
    return Ahat, Bhat, gamma_pw, D


def solve_pwls(A, R, B0, gamma, eps, C=1.0, **kw):
    """Active-set PWLS solve; returns the oracle's SolveResult with sigma in
    image units (D^-1 sigma_pw) and the raw solution in ``sigma_pw``."""
    Ahat, Bhat, gpw, D = pwls_problem(A, R, B0, gamma, C)
    res = solve(Ahat, Bhat, gpw, eps, **kw)
    res.sigma_pw = res.sigma
    res.sigma = res.sigma / D
    return res

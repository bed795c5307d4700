"""Steering vectors, Khatri-Rao operators, dirty images and bounds (FP64).

Test infrastructure only (see the package docstring).  Everything here is
complex128 / float64 and stores the array-response matrix explicitly.
"""

from __future__ import annotations

import math

import numpy as np


class NotPositiveDefinite(ValueError):
    """The covariance is not Hermitian positive definite (or not finite)."""


def pixel_directions(grid):
    """Direction cosines of every pixel of a regular grid.

    Sec. II-A places one candidate source at each pixel centre.  The grid is
    ``(nl, nm, l0, dl, m0, dm)``; pixel ``i = im*nl + il`` sits at
    ``(l0 + il*dl, m0 + im*dm)``.
    """
    nl, nm, l0, dl, m0, dm = grid
    i = np.arange(nl * nm)
    return l0 + (i % nl) * dl, m0 + (i // nl) * dm


def steering(pos, lam, grid, pixels=None):
    """Array-response matrix A (P x n), one unit-norm column per pixel.

    Sec. III-E gives the response model ``P^-1/2 exp(j 2pi/lam Xi^T beta)``;
    on a planar array (z = 0) with direction cosines (l, m) this is
    ``a_i[p] = P^-1/2 exp(-j 2pi (x_p l_i + y_p m_i)/lam)`` with the sign
    convention of the data generator, and ``a_i^H a_i = 1`` (Sec. II-A).
    The phase is formed in float64.
    """
    pos = np.asarray(pos, dtype=np.float64)
    l, m = pixel_directions(grid)
    if pixels is not None:
        pixels = np.asarray(pixels, dtype=np.int64)
        l, m = l[pixels], m[pixels]
    phase = (-2.0 * math.pi / lam) * (np.outer(pos[:, 0], l) + np.outer(pos[:, 1], m))
    return np.exp(1j * phase) / math.sqrt(pos.shape[0])


def forward(A_S, v):
    """Correlation operator: ``Psi_S v`` as the P x P matrix sum_i v_i a_i a_i^H.

    Sec. IV-B (Implementation): with K = 1 the product of the Khatri-Rao
    matrix with a pixel vector is the correlation matrix built from the
    selected steering vectors, ``vect(A_S diag(v) A_S^H)``
    (Notation: (B^T o A) x = vect(A diag(x) B)).
    """
    v = np.asarray(v, dtype=np.float64)
    return (A_S * v[None, :]) @ A_S.conj().T


def adjoint(A_S, U):
    """Beamforming operator: ``Psi_S^H vect(U)`` = (a_i^H U a_i)_i, real part.

    Sec. IV-B: the adjoint is one beamformer output per pixel
    (Notation: vectdiag(A^H X A) = (A^* o A)^H vect(X)).  The unknowns are
    real, so the operator used by the real least-squares problem is the real
    part; it is exactly real whenever U is Hermitian.
    """
    return np.real(np.sum(A_S.conj() * (U @ A_S), axis=0))


def _check_covariance(R):
    R = np.asarray(R, dtype=np.complex128)
    if R.ndim != 2 or R.shape[0] != R.shape[1] or not np.all(np.isfinite(R)):
        raise NotPositiveDefinite("covariance must be a finite square matrix")
    return R


def mf_image(A, R):
    """Matched-filter dirty image, eq. mfdimg with K = 1: ``vectdiag(A^H R A)``."""
    return adjoint(A, _check_covariance(R))


def _inverse_hpd(R):
    """R^-1 through a Cholesky factorisation R = L L^H (fails if R is not PD)."""
    R = _check_covariance(R)
    try:
        Lc = np.linalg.cholesky(R)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc
    Linv = np.linalg.solve(Lc, np.eye(R.shape[0], dtype=np.complex128))
    return Linv.conj().T @ Linv


def mvdr_inverse_power(A, R):
    """``h_i = a_i^H R^-1 a_i`` for every column of A (the MVDR denominator).

    The MVDR dirty image (eq. wmvdr and the expression after it, K = 1) is
    ``1 / h_i``; the unbiased estimate of Sec. II-D scales it by C.
    """
    return adjoint(A, _inverse_hpd(R))


def upper_bound(A, R, kind="mvdr", C=1.0, kappa_b=0.0, nsamples=None):
    """Per-pixel upper bound gamma for the box constraint (eq. CLS).

    * ``"mvdr"``: ``C/h_i`` (Sec. II-D unbiased MVDR estimate) plus
      ``kappa_b`` standard deviations, where App. A gives the variance of the
      MVDR image at K = 1 as ``1/((N - P - 1) h_i^2)``.
    * ``"mf"``: the MF dirty image (eq. mfupper) plus ``kappa_b`` standard
      deviations, App. A: ``Var = (a_i^H R a_i)^2 / N`` at K = 1.
    * ``"none"``: +inf (only the lower bound, eq. NNLS).
    The sample covariance is plugged in for the true one.
    """
    P = A.shape[0]
    if kind == "mvdr":
        h = mvdr_inverse_power(A, R)
        g = C / h
        if kappa_b:
            g = g + kappa_b / (h * math.sqrt(nsamples - P - 1))
        return g
    if kind == "mf":
        mf = mf_image(A, R)
        if kappa_b:
            mf = mf + kappa_b * mf / math.sqrt(nsamples)
        return mf
    if kind == "none":
        return np.full(A.shape[1], np.inf)
    raise ValueError(kind)


def detection_threshold(mf, kappa_d, nsamples):
    """Detection threshold epsilon_i = kappa_d * std of MF pixel i.

    Sec. III-C ties the threshold to the standard deviation of the dirty image
    of the LS cost; App. A gives ``Var = (a_i^H R a_i)^2 / N`` at K = 1, with
    the sample covariance plugged in, so ``std_i = mf_i / sqrt(N)``.
    """
    return kappa_d * np.asarray(mf, dtype=np.float64) / math.sqrt(nsamples)

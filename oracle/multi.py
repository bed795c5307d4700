"""K sample covariances over one pixel grid (FP64).  Test infrastructure only.

The data model of Sec. II stacks K covariance blocks (eq. vectRtotal, the
block-diagonal form eq. blockdiagtilde): block k has its own array response
A_k -- the antenna positions rotated by the Earth's rotation for short-term
integration k (Q_k in the data model), or another wavelength for another
frequency channel whose sky is the same -- and its own sample covariance
R_k.  The LS cost is (1/2K) ||r - Psi sigma||^2 with Psi the stacked
Khatri-Rao blocks (eq. UCLS), so that

* the forward product gives one correlation matrix per block,
  Psi_k sigma = A_k diag(sigma) A_k^H, and the adjoint sums the blocks'
  beamformer outputs, sum_k vectdiag(A_k^H U_k A_k);
* the MF dirty image is (1/K) sum_k vectdiag(A_k^H R_k A_k) (eq. mfdimg);
* the MVDR dirty image with the sqrt(K) normalisation is
  K / sum_k a_{i,k}^H R_k^-1 a_{i,k} (eq. wmvdr and the expression after
  it), scaled by C for the unbiased estimate (Sec. II-D);
* App. A: Var(MF_i) = sum_k (a_{i,k}^H R_k a_{i,k})^2 / (N K^2) and
  Var(MVDR_i) = K^2 sum_k h_k^2 / ((N - p - 1) (sum_k h_k)^4), with
  h_k = a_{i,k}^H R_k^-1 a_{i,k} (sample covariances plugged in);
* the detection threshold is kappa_d standard deviations of the MF image
  (Sec. III-C), and the gradient of the cost on the active pixels is
  (1/K) Psi^H (Psi sigma - r) (``active_set.solve`` with a list of blocks).

All blocks share N samples and the antenna count p.
"""

from __future__ import annotations

import math

import numpy as np

from .active_set import solve
from .imaging import adjoint, mvdr_inverse_power, steering


def steering_blocks(blocks, grid):
    """A_k for blocks given as (positions P x 2, wavelength) pairs."""
    return [steering(pos, lam, grid) for pos, lam in blocks]


def mf_image_multi(As, Rs):
    """eq. mfdimg: (1/K) sum_k vectdiag(A_k^H R_k A_k)."""
    K = len(As)
    return sum(adjoint(A, np.asarray(R, np.complex128)) for A, R in zip(As, Rs)) / K


def mf_std_multi(As, Rs, nsamples):
    """App. A: sqrt(sum_k (a_{i,k}^H R_k a_{i,k})^2 / (N K^2))."""
    K = len(As)
    sq = sum(adjoint(A, np.asarray(R, np.complex128)) ** 2 for A, R in zip(As, Rs))
    return np.sqrt(sq / nsamples) / K


def mvdr_powers(As, Rs):
    """(sum_k h_k, sum_k h_k^2) per pixel, h_k = a_k^H R_k^-1 a_k."""
    hs = [mvdr_inverse_power(A, R) for A, R in zip(As, Rs)]
    return sum(hs), sum(h * h for h in hs)


def upper_bound_multi(As, Rs, kind="mvdr", C=1.0, kappa_b=0.0, nsamples=None):
    """Per-pixel upper bound gamma for K blocks (eq. wmvdr / eq. mfupper, App. A)."""
    K = len(As)
    P = As[0].shape[0]
    if kind == "mvdr":
        s1, s2 = mvdr_powers(As, Rs)
        g = C * K / s1
        if kappa_b:
            g = g + kappa_b * K * np.sqrt(s2) / (math.sqrt(nsamples - P - 1) * s1 * s1)
        return g
    if kind == "mf":
        mf = mf_image_multi(As, Rs)
        if kappa_b:
            mf = mf + kappa_b * mf_std_multi(As, Rs, nsamples)
        return mf
    if kind == "none":
        return np.full(As[0].shape[1], np.inf)
    raise ValueError(kind)


def detection_threshold_multi(As, Rs, kappa_d, nsamples):
    """kappa_d standard deviations of the MF image (Sec. III-C, App. A)."""
    return kappa_d * mf_std_multi(As, Rs, nsamples)


def solve_multi(As, B0s, gamma, eps, **kw):
    """The active-set solve of Table I on the stacked blocks."""
    return solve(list(As), list(B0s), gamma, eps, **kw)

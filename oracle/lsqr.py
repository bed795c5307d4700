"""LSQR on a matrix-free operator (FP64).

Test infrastructure only (see the package docstring).

Sec. IV-A reduces M to lower-bidiagonal form by the Golub-Kahan (Lanczos)
recurrences (eqs. initbeta, initu, lanczos) and solves ``min ||b - M x||`` with
LSQR (Paige and Saunders, 1982), whose scalar updates the paper leaves to that
reference.  The updates below are the published LSQR method restated from its
mathematics: a Givens QR of the growing bidiagonal matrix, the solution updated
along the search directions ``w``, and the residual / normal-residual norms
read from the rotation scalars.

Data-space vectors may be complex arrays of any shape (here P x P Hermitian
matrices); solution-space vectors are real.  Norms are Euclidean over all
entries (Frobenius for matrices).

Stopping (all three are the LSQR tests, evaluated after every iteration):

* 1: ``||r|| <= btol ||b|| + atol ||M|| ||x||`` (consistent systems);
* 2: ``||M^H r|| <= atol ||M|| ||r||`` (least-squares optimality, the test
  the paper states for ending the recursion);
* 3: condition estimate ``>= conlim``;
* 4: exact breakdown (``alpha`` or ``beta`` becomes zero, or ``b = 0``);
* 7: ``itnlim`` iterations reached.

``||M||`` is the running Frobenius norm of the bidiagonal matrix, the
condition estimate is ``||M|| * sqrt(sum ||w_k/rho_k||^2)``, and ``||x||`` is
the exact norm of the current iterate.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class LsqrResult:
    x: np.ndarray
    istop: int
    itn: int
    rnorm: float
    arnorm: float
    anorm: float
    acond: float
    xnorm: float


def _norm(a):
    return math.sqrt(float(np.sum(np.abs(a) ** 2)))


def lsqr(matvec, rmatvec, b, n, atol=1e-8, btol=1e-8, conlim=1e8, itnlim=None):
    """Solve ``min_x ||b - M x||`` from ``x0 = 0`` given ``M v`` and ``M^H u``.

    Starting from zero gives the minimum-norm least-squares solution when M
    is rank deficient (the iterates stay in the row space of M).
    """
    if itnlim is None:
        itnlim = 4 * n + 100
    x = np.zeros(n)
    beta = _norm(b)
    if n == 0 or beta == 0.0:
        return LsqrResult(x, 4, 0, beta, 0.0, 0.0, 0.0, 0.0)
    u = b / beta
    v = np.asarray(rmatvec(u), dtype=np.float64)
    alpha = _norm(v)
    if alpha == 0.0:
        return LsqrResult(x, 4, 0, beta, 0.0, 0.0, 0.0, 0.0)
    v = v / alpha
    w = v.copy()
    bnorm = beta
    phibar, rhobar = beta, alpha
    anorm2 = 0.0
    ddnorm = 0.0
    itn = 0
    istop = 7
    rnorm = arnorm = anorm = acond = xnorm = 0.0
    while itn < itnlim:
        itn += 1
        # Golub-Kahan step: beta u <- M v - alpha u ; alpha v <- M^H u - beta v
        u = matvec(v) - alpha * u
        beta = _norm(u)
        if beta > 0.0:
            u = u / beta
        anorm2 += alpha * alpha + beta * beta
        v = np.asarray(rmatvec(u), dtype=np.float64) - beta * v
        alpha = _norm(v)
        if alpha > 0.0:
            v = v / alpha
        # Givens rotation eliminating beta from the bidiagonal matrix
        rho = math.hypot(rhobar, beta)
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        # solution and search-direction updates
        dk = w / rho
        ddnorm += float(dk @ dk)
        x = x + phi * dk
        w = v - (theta / rho) * w
        # norm estimates and stopping tests
        rnorm = phibar
        arnorm = phibar * alpha * abs(c)
        anorm = math.sqrt(anorm2)
        acond = anorm * math.sqrt(ddnorm)
        xnorm = _norm(x)
        if rnorm <= btol * bnorm + atol * anorm * xnorm:
            istop = 1
            break
        if arnorm <= atol * anorm * rnorm:
            istop = 2
            break
        if acond >= conlim:
            istop = 3
            break
        if alpha == 0.0 or beta == 0.0:
            istop = 4
            break
    return LsqrResult(x, istop, itn, rnorm, arnorm, anorm, acond, xnorm)

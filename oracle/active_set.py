"""Active-set solver for box-constrained LS imaging (FP64).

Test infrastructure only (see the package docstring).

Problem (eq. CLS, K = 1):  ``min 1/2 ||B0 - sum_i sigma_i a_i a_i^H||_F^2``
subject to ``0 <= sigma <= gamma``, where ``B0 = R_hat - diag(noise)`` (the
data model of eq. vectRImg with the receiver-noise term moved to the data side;
``noise = 0`` ignores it as in eq. UCLS).  With K blocks (``A`` and ``B0``
given as lists, eq. vectRtotal) the cost is ``1/(2K) sum_k ||B0_k -
A_k diag(sigma) A_k^H||_F^2`` (eq. UCLS): the subproblems are LSQR on the
stacked blocks and the gradient is ``(1/K) sum_k vectdiag(A_k^H E_k A_k)``.

The iteration follows the active-set template of Sec. III-C (Table I):

* pixel sets L (at 0), U (at gamma) and F (free) as in Sec. III-A;
* while the free-set gradient is not known to vanish, solve the equality
  constrained subproblem on F (eqs. subproblemLS / bsubproblemLS) with LSQR
  started from zero;
* a feasible solution is accepted; then the gradient on the active pixels
  (eq. gls, ``g = Psi^H (Psi sigma - B0)``) gives the Lagrange multipliers
  (eqs. etaL / etaU: ``lambda = g`` on L, ``-g`` on U);
* an infeasible solution is followed only as far as the box allows (step
  eq. mumax) and the first pixel to reach a bound leaves F;
* otherwise the most negative multiplier is released into F if it is below
  minus the detection threshold of its pixel (Sec. III-C, App. A), else stop.

Readings where the paper leaves a choice open (also listed with the design
notes of the library):

* feasibility is tested without tolerance, ``0 <= z_i <= gamma_i``;
* ties in both argmins go to the lowest pixel index;
* ``mu_i`` is only formed for ``p_i != 0``; only the blocking pixel leaves F,
  to L if ``p_i < 0`` else to U, and is set exactly to that bound; the other
  free pixels are clamped to the box after the step;
* the subproblem is solved from zero each time (minimum-norm solution);
* ``gamma`` is fixed for the whole solve; with an empty active set the loop
  ends after the feasible solve;
* a pixel that is released and then immediately blocks again with a zero
  step restores the previous state exactly, so the iteration would repeat
  forever: the solve stops with the "cycle" status;
* ``max_outer`` bounds the number of subproblem solves.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from .imaging import forward, adjoint
from .lsqr import lsqr

STATE_L, STATE_F, STATE_U = 0, 1, 2

STATUS_OK = 0
STATUS_MAXOUTER = 1
STATUS_ITNLIM = 2
STATUS_CYCLE = 3


@dataclasses.dataclass
class SolveResult:
    sigma: np.ndarray
    state: np.ndarray
    status: int
    outer_iters: int
    adds: int
    drops: int
    lsqr_iters_total: int
    lsqr_itnlim_hits: int
    rel_residual: float
    objective: float
    min_margin_lambda: float
    min_margin_z: float
    events: list


def _nearest_neg(values, default=math.inf):
    return float(np.min(values)) if values.size else default


def solve(A, B0, gamma, eps, atol=1e-8, btol=1e-8, conlim=1e8, itnlim=-1, max_outer=-1,
          sigma0=None, state0=None):
    """Run the active-set iteration; returns the image, the sets and statistics.

    ``A`` is the explicit P x Q steering matrix, ``B0`` the P x P data matrix,
    ``gamma`` and ``eps`` the per-pixel upper bound and detection threshold.
    ``itnlim = -1`` means ``4 |F| + 100`` per subproblem, ``max_outer = -1``
    means ``4 Q`` subproblem solves.
    """
    if isinstance(A, (list, tuple)):  # K blocks over one pixel grid
        As = list(A)
        B0 = np.stack([np.asarray(b, dtype=np.complex128) for b in B0])
        K = len(As)

        def fwd(S, v):
            return np.stack([forward(Ak[:, S], v) for Ak in As])

        def adj(S, U):
            return sum(adjoint(Ak[:, S], U[k]) for k, Ak in enumerate(As))

        Q = As[0].shape[1]
    else:
        K = 1

        def fwd(S, v):
            return forward(A[:, S], v)

        def adj(S, U):
            return adjoint(A[:, S], U)

        Q = A.shape[1]
    gamma = np.asarray(gamma, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    if max_outer < 0:
        max_outer = 4 * Q
    if state0 is None:
        state = np.full(Q, STATE_L, dtype=np.uint8)
        sigma = np.zeros(Q)
    else:
        state = np.array(state0, dtype=np.uint8)
        sigma = np.array(sigma0, dtype=np.float64)
    events = []
    status = STATUS_OK
    outer = adds = drops = lsqr_total = itnlim_hits = 0
    need_solve = True
    last_added = -1
    lam_min, i_min = math.inf, -1
    margin_lambda = margin_z = math.inf
    while True:
        if need_solve:
            if outer >= max_outer:
                status = STATUS_MAXOUTER
                break
            F = np.nonzero(state == STATE_F)[0]
            U = np.nonzero(state == STATE_U)[0]
            Bb = B0 - fwd(U, gamma[U])
            lim = 4 * F.size + 100 if itnlim < 0 else itnlim
            res = lsqr(lambda v: fwd(F, v), lambda u: adj(F, u), Bb, F.size,
                       atol=atol, btol=btol, conlim=conlim, itnlim=lim)
            lsqr_total += res.itn
            if res.istop == 7:
                itnlim_hits += 1
            z = res.x
            outer += 1
            if np.all(z >= 0.0) and np.all(z <= gamma[F]):
                sigma[F] = z
                need_solve = False
                if F.size:
                    margin_z = min(margin_z, float(np.min(np.minimum(z, gamma[F] - z) / gamma[F])))
                act = np.nonzero(state != STATE_F)[0]
                events.append(("feasible", F.size, res.itn))
                if act.size == 0:
                    break
                S = np.nonzero(state != STATE_L)[0]
                E = fwd(S, sigma[S]) - B0
                g = adj(act, E) / K
                lam = np.where(state[act] == STATE_L, g, -g)
                k = int(np.argmin(lam))          # first occurrence = lowest index
                lam_min, i_min = float(lam[k]), int(act[k])
            else:
                p = z - sigma[F]
                nz = p != 0.0
                mu = np.full(F.size, math.inf)
                mu[nz] = np.maximum(-sigma[F][nz] / p[nz], (gamma[F][nz] - sigma[F][nz]) / p[nz])
                kb = int(np.argmin(mu))
                mu_max = float(mu[kb])
                ib = int(F[kb])
                sigma[F] = np.clip(sigma[F] + mu_max * p, 0.0, gamma[F])
                if p[kb] < 0.0:
                    sigma[ib], state[ib] = 0.0, STATE_L
                else:
                    sigma[ib], state[ib] = gamma[ib], STATE_U
                drops += 1
                events.append(("block", ib, int(state[ib]), mu_max))
                need_solve = True
                if ib == last_added and mu_max == 0.0:
                    status = STATUS_CYCLE
                    break
            last_added = -1
        else:
            thr = eps[i_min]
            if thr > 0:
                margin_lambda = min(margin_lambda, abs(lam_min + thr) / thr)
            if lam_min < -thr:
                state[i_min] = STATE_F
                adds += 1
                last_added = i_min
                events.append(("add", i_min))
                need_solve = True
            else:
                break
    if status == STATUS_OK and itnlim_hits:
        status = STATUS_ITNLIM
    S = np.nonzero(state != STATE_L)[0]
    Rres = B0 - fwd(S, sigma[S])
    bn = math.sqrt(float(np.sum(np.abs(B0) ** 2)))
    rn = math.sqrt(float(np.sum(np.abs(Rres) ** 2)))
    return SolveResult(sigma=sigma, state=state, status=status, outer_iters=outer, adds=adds,
                       drops=drops, lsqr_iters_total=lsqr_total, lsqr_itnlim_hits=itnlim_hits,
                       rel_residual=rn / bn if bn > 0 else 0.0, objective=0.5 * rn * rn,
                       min_margin_lambda=margin_lambda, min_margin_z=margin_z, events=events)

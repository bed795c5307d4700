"""Strong off-grid sources (Sec. III-E, eq. doals) in FP64.  Test infrastructure only.

A source inside a pixel but away from its centre is underestimated by the
on-grid model; the paper replaces the subproblem on the free set by the
non-linear problem

    min over (delta_F, sigma_F)  1/2 || b - Psi(delta)_F sigma_F ||^2,
    |delta_i,1| < W/2,  |delta_i,2| < H/2,

where pixel i's steering vector is taken at its centre shifted by
delta_i = (delta_l, delta_m) (direction cosines; W = dl, H = dm on this
grid), b = r - Psi_U sigma_U, and the bounds of the shifted pixels are
re-evaluated at their new positions.  The paper asks for a Newton-based
method and leaves it open; the reading implemented here (and on the GPU):

* a pixel enters F at its centre (delta = 0); delta is kept while the pixel
  stays in F and reset when it leaves F;
* each subproblem runs ``rounds`` Gauss-Newton rounds: LSQR for sigma_F at
  the current offsets (the linear part, solved exactly as in eq.
  subproblemLS), then one Gauss-Newton step on each free pixel's offset with
  the coupling between pixels neglected (its 2 x 2 block), clipped to the
  pixel; a last LSQR gives sigma_F at the final offsets;
* the gradient of f = 1/2 ||E||^2, E = Psi(delta)_F z - b, with respect to
  delta_i,j is 2 z_i Re(y^H d_j), y = E a_i, d_j = a_i (.) (-j c x_j),
  c = 2 pi / lambda, x_1 = x, x_2 = y antenna coordinates; the Gauss-Newton
  block is z_i^2 G with G_jk = <d_j a^H + a d_j^H, d_k a^H + a d_k^H> =
  2 c^2 Cov(x_j, x_k) (positions averaged over the antennas) -- the same for
  every pixel;
* the bound of a free pixel is the bound formula at its shifted direction;
  pixels at the upper bound keep their on-grid steering and bound (b uses
  the on-grid A_U), and a pixel that leaves F for U takes its on-grid bound;
* the release test and the gradient on the active pixels are unchanged
  (on-grid, eq. gls with E from the shifted free pixels).
"""

from __future__ import annotations

import math

import numpy as np

from .active_set import SolveResult, STATE_F, STATE_L, STATE_U, STATUS_CYCLE, STATUS_ITNLIM, STATUS_MAXOUTER, STATUS_OK
from .imaging import _inverse_hpd, adjoint, forward, pixel_directions, steering
from .lsqr import lsqr


def steering_at(pos, lam, l, m):
    """Steering vectors at arbitrary direction cosines (one column per (l, m))."""
    pos = np.asarray(pos, dtype=np.float64)
    phase = (-2.0 * math.pi / lam) * (np.outer(pos[:, 0], np.asarray(l, np.float64))
                                      + np.outer(pos[:, 1], np.asarray(m, np.float64)))
    return np.exp(1j * phase) / math.sqrt(pos.shape[0])


def gauss_newton_block(pos, lam):
    """G = 2 c^2 Cov(x, y) of the antenna positions (population covariance)."""
    pos = np.asarray(pos, dtype=np.float64)
    c = 2.0 * math.pi / lam
    d = pos - pos.mean(axis=0)
    return 2.0 * c * c * (d.T @ d) / pos.shape[0]


def offset_gradient(pos, lam, a, E, z):
    """d f / d delta_i for one free pixel: 2 z Re(y^H d_j), y = E a."""
    c = 2.0 * math.pi / lam
    y = E @ a
    out = np.empty(2)
    for j in range(2):
        d = a * (-1j * c * np.asarray(pos, np.float64)[:, j])
        out[j] = 2.0 * z * float(np.real(np.vdot(y, d)))
    return out


def _bounds_at(pos, lam, l, m, R, Rinv, kind, C, kappa_b, nsamples):
    A = steering_at(pos, lam, l, m)
    if kind == "mvdr":
        h = adjoint(A, Rinv)
        g = C / h
        if kappa_b:
            g = g + kappa_b / (h * math.sqrt(nsamples - A.shape[0] - 1))
        return g
    if kind == "mf":
        mf = adjoint(A, R)
        return mf + (kappa_b * mf / math.sqrt(nsamples) if kappa_b else 0.0)
    return np.full(A.shape[1], np.inf)


def solve_offgrid(pos, lam, grid, R, B0, eps, kind="mvdr", C=1.0, kappa_b=0.0, nsamples=None, rounds=3,
                  atol=1e-8, btol=1e-8, conlim=1e8, itnlim=-1, max_outer=-1):
    """Table I with eq. doals in place of the subproblem (K = 1).

    Returns (SolveResult, offsets) with offsets a Q x 2 array of (delta_l,
    delta_m), zero outside F; result.sigma[F] are the powers at the shifted
    positions.
    """
    pos = np.asarray(pos, dtype=np.float64)
    nl, nm, l0, dl, m0, dm = grid
    lc, mc = pixel_directions(grid)
    A0 = steering(pos, lam, grid)
    Q = A0.shape[1]
    R = np.asarray(R, dtype=np.complex128)
    Rinv = _inverse_hpd(R) if kind == "mvdr" else None
    gamma0 = _bounds_at(pos, lam, lc, mc, R, Rinv, kind, C, kappa_b, nsamples)
    gamma = gamma0.copy()
    eps = np.asarray(eps, dtype=np.float64)
    G = gauss_newton_block(pos, lam)
    half = np.array([dl / 2.0, dm / 2.0])
    if max_outer < 0:
        max_outer = 4 * Q
    state = np.full(Q, STATE_L, dtype=np.uint8)
    sigma = np.zeros(Q)
    delta = np.zeros((Q, 2))
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
            delta[state != STATE_F] = 0.0
            Bb = B0 - forward(A0[:, U], gamma0[U])
            lim = 4 * F.size + 100 if itnlim < 0 else itnlim
            for t in range(rounds + 1):
                A_F = steering_at(pos, lam, lc[F] + delta[F, 0], mc[F] + delta[F, 1])
                res = lsqr(lambda v: forward(A_F, v), lambda u: adjoint(A_F, u), Bb, F.size,
                           atol=atol, btol=btol, conlim=conlim, itnlim=lim)
                z = res.x
                lsqr_total += res.itn
                if res.istop == 7:
                    itnlim_hits += 1
                if t == rounds:
                    break
                E = forward(A_F, z) - Bb
                for k, i in enumerate(F):
                    if z[k] == 0.0:
                        continue
                    g = offset_gradient(pos, lam, A_F[:, k], E, z[k])
                    step = -np.linalg.solve(z[k] * z[k] * G, g)
                    delta[i] = np.clip(delta[i] + step, -half, half)
            gamma[:] = gamma0
            if F.size:
                gamma[F] = _bounds_at(pos, lam, lc[F] + delta[F, 0], mc[F] + delta[F, 1], R, Rinv, kind, C,
                                      kappa_b, nsamples)
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
                E = forward(A_F, sigma[F]) - Bb
                g = adjoint(A0[:, act], E)
                lamv = np.where(state[act] == STATE_L, g, -g)
                k = int(np.argmin(lamv))
                lam_min, i_min = float(lamv[k]), int(act[k])
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
                    sigma[ib], state[ib] = gamma0[ib], STATE_U  # U keeps the on-grid bound
                delta[ib] = 0.0
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
    F = np.nonzero(state == STATE_F)[0]
    U = np.nonzero(state == STATE_U)[0]
    A_F = steering_at(pos, lam, lc[F] + delta[F, 0], mc[F] + delta[F, 1])
    Rres = B0 - forward(A0[:, U], sigma[U]) - forward(A_F, sigma[F])
    bn = math.sqrt(float(np.sum(np.abs(B0) ** 2)))
    rn = math.sqrt(float(np.sum(np.abs(Rres) ** 2)))
    res = SolveResult(sigma=sigma, state=state, status=status, outer_iters=outer, adds=adds, drops=drops,
                      lsqr_iters_total=lsqr_total, lsqr_itnlim_hits=itnlim_hits,
                      rel_residual=rn / bn if bn > 0 else 0.0, objective=0.5 * rn * rn,
                      min_margin_lambda=margin_lambda, min_margin_z=margin_z, events=events)
    return res, delta

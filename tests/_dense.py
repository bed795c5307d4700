"""Independent dense constructions used to pin the oracle (tests only).

These build the Khatri-Rao matrix Psi column by column with ``np.kron`` and
work with its real-stacked form, so they exercise the Notation identities of
the paper rather than retyping the oracle's matrix formulation.
"""

import itertools
import math

import numpy as np


def steering_direct(pos, lam, l, m):
    """Entry-by-entry response ``P^-1/2 exp(-j 2pi (x l + y m)/lam)``, loops only."""
    P = len(pos)
    out = np.empty((P, len(l)), dtype=np.complex128)
    for i in range(len(l)):
        for p in range(P):
            ph = -2.0 * math.pi * (pos[p][0] * l[i] + pos[p][1] * m[i]) / lam
            out[p, i] = complex(math.cos(ph), math.sin(ph)) / math.sqrt(P)
    return out


def dense_psi(A):
    """Psi with column i = conj(a_i) kron a_i = vect(a_i a_i^H) (column stacking)."""
    return np.stack([np.kron(A[:, i].conj(), A[:, i]) for i in range(A.shape[1])], axis=1)


def vect(X):
    return np.asarray(X).reshape(-1, order="F")


def real_stack(Psi):
    return np.vstack([Psi.real, Psi.imag])


def random_hermitian(rng, P, pd=False):
    X = rng.standard_normal((P, P)) + 1j * rng.standard_normal((P, P))
    if pd:
        return X @ X.conj().T / P + 0.5 * np.eye(P)
    return 0.5 * (X + X.conj().T)


def brute_force_box_ls(Psi_r, b_r, gamma):
    """min 1/2||b - Psi x||^2 s.t. 0 <= x <= gamma by enumerating all 3^Q patterns."""
    Q = Psi_r.shape[1]
    best = (math.inf, None)
    for pattern in itertools.product((0, 1, 2), repeat=Q):
        pattern = np.array(pattern)
        x = np.where(pattern == 2, gamma, 0.0).astype(float)
        F = np.nonzero(pattern == 1)[0]
        rhs = b_r - Psi_r @ x
        if F.size:
            zF = np.linalg.lstsq(Psi_r[:, F], rhs, rcond=None)[0]
            if np.any(zF < -1e-12) or np.any(zF > gamma[F] + 1e-12):
                continue
            x[F] = np.clip(zF, 0.0, gamma[F])
        obj = 0.5 * float(np.sum((b_r - Psi_r @ x) ** 2))
        if obj < best[0]:
            best = (obj, x)
    return best

"""Seeded synthetic observations shaped like the paper's simulations.

What is simulated (Sec. I, eqs. samplemodel / cov_def, and Sec. V):

* a random planar array of P antennas, uniform in a disc (Sec. V uses a
  random dipole array);
* a sky of independent sources sitting on pixel centres of a regular
  (l, m) direction-cosine grid: point sources plus optional Gaussian extended
  blobs made of independent pixels (Sec. V-A builds extended structure from
  Gaussian components);
* white receiver noise of variance ``noise_var`` on every antenna;
* N complex-Gaussian samples per covariance estimate and the sample
  covariance R_hat = (1/N) sum_n y[n] y[n]^H, one snapshot (K = 1).

Conventions shared with both consumers (and documented with the C ABI):

* pixel flat index ``i = im * nl + il``; ``l = l0 + il*dl``, ``m = m0 + im*dm``;
  the grid over |l|, |m| <= L is ``l_j = (j - n/2) * 2L/n``;
* the array response towards direction (l, m) is
  ``P**-0.5 * exp(-2j*pi*(x_p*l + y_p*m)/lam)`` (unit norm, Sec. II-A);
* ``R_hat[p, q] = mean_n y_p[n] * conj(y_q[n])`` stored row-major.

Sampling uses y = chol(R) w with w ~ CN(0, I), which has exactly the
distribution of y = A_src x + e with x ~ CN(0, diag(s)), e ~ CN(0, noise I).
Samples are accumulated in fixed-size chunks in a fixed order, and the result
is made exactly Hermitian.  Everything is float64/complex128; ``R_hat32`` is the
complex64 rounding handed to the FP32 GPU path, and ``R_hat32_c128`` is that
same rounding upcast, handed to the FP64 oracle so that both see identical bits.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

_CHUNK = 4096

# Workload recipes.  "points" gives the number of point sources and the flux
# law; "blobs" the number of Gaussian blobs, their FWHM in pixels and peak power.
CONFIGS = {
    "c0": dict(P=24, radius=20.0, n=32, L=0.5, N=4096, noise=1.0,
               points=(5, ("uniform", 1.0, 10.0)), blobs=(0, 6.0, 0.0)),
    "c1": dict(P=48, radius=60.0, n=128, L=0.7, N=16384, noise=10.0,
               points=(40, ("loguniform", 0.1, 100.0)), blobs=(2, 6.0, 10.0)),
    "c2": dict(P=96, radius=150.0, n=256, L=0.7, N=65536, noise=50.0,
               points=(200, ("powerlaw", 0.5, 500.0)), blobs=(0, 6.0, 0.0)),
    "c4": dict(P=288, radius=400.0, n=512, L=0.7, N=2 ** 18, noise=100.0,
               points=(1000, ("powerlaw", 1.0, 1000.0)), blobs=(10, 6.0, 100.0)),
}

_SEED_BASE = 20150501
_REQUEST_SEED = 20150503


@dataclasses.dataclass
class Scene:
    name: str
    P: int
    pos: np.ndarray          # (P, 2) float64, antenna x, y in metres
    lam: float               # wavelength in metres
    nl: int
    nm: int
    l0: float
    dl: float
    m0: float
    dm: float
    N: int                   # samples behind R_hat
    noise_var: float         # white noise variance per antenna
    src_pix: np.ndarray      # (S,) int64 flat pixel index of each source
    src_pow: np.ndarray      # (S,) float64 source power
    R_hat: np.ndarray        # (P, P) complex128 sample covariance

    @property
    def Q(self) -> int:
        return self.nl * self.nm

    @property
    def grid(self):
        return (self.nl, self.nm, self.l0, self.dl, self.m0, self.dm)

    @property
    def R_hat32(self) -> np.ndarray:
        return np.ascontiguousarray(self.R_hat.astype(np.complex64))

    @property
    def R_hat32_c128(self) -> np.ndarray:
        return self.R_hat32.astype(np.complex128)

    @property
    def noise_diag(self) -> np.ndarray:
        return np.full(self.P, self.noise_var, dtype=np.float64)

    def true_image(self) -> np.ndarray:
        img = np.zeros(self.Q)
        np.add.at(img, self.src_pix, self.src_pow)
        return img


def _grid_axis(n: int, L: float):
    d = 2.0 * L / n
    return -0.5 * n * d, d


def _disc_positions(rng, P, radius):
    u = rng.random(P)
    t = rng.random(P)
    r = radius * np.sqrt(u)
    th = 2.0 * math.pi * t
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def _fluxes(rng, count, law):
    kind, lo, hi = law
    u = rng.random(count)
    if kind == "uniform":
        return lo + (hi - lo) * u
    if kind == "loguniform":
        return np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)
    if kind == "powerlaw":  # dN/dS ~ S^-1.5 on [lo, hi], inverse-CDF sampling
        a = 1.0 - 1.5
        return (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
    raise ValueError(kind)


def _sky(rng, nl, nm, n_points, law, n_blobs, fwhm, peak):
    Q = nl * nm
    img = np.zeros(Q)
    pix = rng.choice(Q, size=n_points, replace=False)
    img[pix] += _fluxes(rng, n_points, law)
    rad = int(math.floor(fwhm))
    for _ in range(n_blobs):
        c = int(rng.integers(Q))
        ci, cj = c % nl, c // nl
        for dj in range(-rad, rad + 1):
            for di in range(-rad, rad + 1):
                d2 = di * di + dj * dj
                if d2 > fwhm * fwhm:
                    continue
                il, im = ci + di, cj + dj
                if 0 <= il < nl and 0 <= im < nm:
                    img[im * nl + il] += peak * math.exp(-4.0 * math.log(2.0) * d2 / (fwhm * fwhm))
    src_pix = np.nonzero(img)[0]
    return src_pix, img[src_pix]


def _response(pos, lam, l, m):
    """Array response of the data model towards directions (l, m): (P, S)."""
    P = pos.shape[0]
    ph = -2.0 * math.pi / lam * (np.outer(pos[:, 0], l) + np.outer(pos[:, 1], m))
    return np.exp(1j * ph) / math.sqrt(P)


def exact_covariance(pos, lam, grid, src_pix, src_pow, noise_var):
    """R = A_src diag(s) A_src^H + noise_var I  (eq. cov_def with K = 1)."""
    nl, nm, l0, dl, m0, dm = grid
    src_pix = np.asarray(src_pix, dtype=np.int64)
    l = l0 + (src_pix % nl) * dl
    m = m0 + (src_pix // nl) * dm
    A = _response(np.asarray(pos, float), lam, l, m)
    R = (A * np.asarray(src_pow, float)[None, :]) @ A.conj().T
    R += noise_var * np.eye(pos.shape[0])
    return 0.5 * (R + R.conj().T)


def _sample_covariance(rng, R, N):
    P = R.shape[0]
    Lc = np.linalg.cholesky(R)
    acc = np.zeros((P, P), dtype=np.complex128)
    done = 0
    while done < N:
        n = min(_CHUNK, N - done)
        w = (rng.standard_normal((P, n)) + 1j * rng.standard_normal((P, n))) * math.sqrt(0.5)
        y = Lc @ w
        acc += y @ y.conj().T
        done += n
    Rh = acc / N
    return 0.5 * (Rh + Rh.conj().T)


def _build(name, seed, P, radius, n, L, N, noise, points, blobs, lam=1.0):
    ss = np.random.SeedSequence(seed)
    s_pos, s_sky, s_smp, _spare = ss.spawn(4)
    pos = _disc_positions(np.random.default_rng(s_pos), P, radius)
    l0, dl = _grid_axis(n, L)
    n_pts, law = points
    n_blobs, fwhm, peak = blobs
    src_pix, src_pow = _sky(np.random.default_rng(s_sky), n, n, n_pts, law, n_blobs, fwhm, peak)
    grid = (n, n, l0, dl, l0, dl)
    R = exact_covariance(pos, lam, grid, src_pix, src_pow, noise)
    Rh = _sample_covariance(np.random.default_rng(s_smp), R, N)
    return Scene(name=name, P=P, pos=pos, lam=lam, nl=n, nm=n, l0=l0, dl=dl, m0=l0, dm=dl,
                 N=N, noise_var=noise, src_pix=src_pix, src_pow=src_pow, R_hat=Rh)


def make_scene(config: str = "c0", **overrides) -> Scene:
    """Build one of the named workloads; keyword overrides replace recipe fields."""
    idx = {"c0": 0, "c1": 1, "c2": 2, "c4": 4}[config]
    rec = dict(CONFIGS[config])
    seed = overrides.pop("seed", _SEED_BASE + idx)
    rec.update(overrides)
    return _build(config, seed, **rec)


def make_request_scenes(n_req: int, seed: int = _REQUEST_SEED, P_choices=(24, 48, 96),
                        n_choices=(64, 128, 256)):
    """Mixed-size imaging requests (one frequency channel each)."""
    radius_by_P = {24: 20.0, 48: 60.0, 96: 150.0}
    out = []
    for k, child in enumerate(np.random.SeedSequence(seed).spawn(n_req)):
        rng = np.random.default_rng(child)
        P = int(rng.choice(P_choices))
        n = int(rng.choice(n_choices))
        n_src = int(rng.integers(10, 201))
        lam = float(1.0 + rng.random())
        sub_seed = int(rng.integers(2 ** 62))
        out.append(_build(f"req{k}", sub_seed, P=P, radius=radius_by_P.get(P, 60.0), n=n, L=0.7,
                          N=16384, noise=10.0, points=(min(n_src, n * n), ("loguniform", 0.1, 100.0)),
                          blobs=(0, 6.0, 0.0), lam=lam))
    return out


def make_block_scenes(config: str = "c0", K: int = 2, rotation: float = 0.05, lams=None, seed=None,
                      angles=None, **overrides):
    """K covariance blocks of one sky on one grid (the stacked data model):
    block k sees the array rotated by k * rotation radians about the origin
    (Earth rotation between short-term integrations; ``angles`` gives the K
    angles explicitly) and, if ``lams`` is given, wavelength lams[k]
    (frequency channels with the same sky).  Each block draws its own N
    samples.  Returns a list of K scenes."""
    idx = {"c0": 0, "c1": 1, "c2": 2, "c4": 4}[config]
    rec = dict(CONFIGS[config])
    rec.update(overrides)
    seed = _SEED_BASE + 100 + idx if seed is None else seed
    ss = np.random.SeedSequence(seed)
    s_pos, s_sky, s_smp = ss.spawn(3)
    P, n = rec["P"], rec["n"]
    pos0 = _disc_positions(np.random.default_rng(s_pos), P, rec["radius"])
    l0, dl = _grid_axis(n, rec["L"])
    n_pts, law = rec["points"]
    n_blobs, fwhm, peak = rec["blobs"]
    src_pix, src_pow = _sky(np.random.default_rng(s_sky), n, n, n_pts, law, n_blobs, fwhm, peak)
    grid = (n, n, l0, dl, l0, dl)
    out = []
    for k, sk in enumerate(s_smp.spawn(K)):
        ang = float(angles[k]) if angles is not None else k * rotation
        c, sn = math.cos(ang), math.sin(ang)
        pos = pos0 @ np.array([[c, -sn], [sn, c]]).T
        lam = float(lams[k]) if lams is not None else rec.get("lam", 1.0)
        R = exact_covariance(pos, lam, grid, src_pix, src_pow, rec["noise"])
        Rh = _sample_covariance(np.random.default_rng(sk), R, rec["N"])
        out.append(Scene(name=f"{config}-block{k}", P=P, pos=pos, lam=lam, nl=n, nm=n, l0=l0, dl=dl, m0=l0, dm=dl,
                         N=rec["N"], noise_var=rec["noise"], src_pix=src_pix, src_pow=src_pow, R_hat=Rh))
    return out


def make_offgrid_scene(config: str = "c0", max_offset: float = 0.45, seed=None, **overrides):
    """The workload with every point source moved off its pixel centre by a
    uniform offset of up to max_offset pixels in l and in m (the situation of
    strong off-grid sources).  Returns (scene, offsets) with offsets an S x 2
    array in direction cosines; scene.src_pix are the pixels that hold the
    sources."""
    idx = {"c0": 0, "c1": 1, "c2": 2, "c4": 4}[config]
    rec = dict(CONFIGS[config])
    rec.update(overrides)
    seed = _SEED_BASE + 200 + idx if seed is None else seed
    s_pos, s_sky, s_off, s_smp = np.random.SeedSequence(seed).spawn(4)
    P, n = rec["P"], rec["n"]
    pos = _disc_positions(np.random.default_rng(s_pos), P, rec["radius"])
    l0, dl = _grid_axis(n, rec["L"])
    n_pts, law = rec["points"]
    src_pix, src_pow = _sky(np.random.default_rng(s_sky), n, n, n_pts, law, 0, 6.0, 0.0)
    off = np.random.default_rng(s_off).uniform(-max_offset, max_offset, size=(len(src_pix), 2)) * dl
    lam = rec.get("lam", 1.0)
    l = l0 + (src_pix % n) * dl + off[:, 0]
    m = l0 + (src_pix // n) * dl + off[:, 1]
    A = _response(pos, lam, l, m)
    R = (A * src_pow[None, :]) @ A.conj().T + rec["noise"] * np.eye(P)
    R = 0.5 * (R + R.conj().T)
    Rh = _sample_covariance(np.random.default_rng(s_smp), R, rec["N"])
    sc = Scene(name=f"{config}-offgrid", P=P, pos=pos, lam=lam, nl=n, nm=n, l0=l0, dl=dl, m0=l0, dm=dl,
               N=rec["N"], noise_var=rec["noise"], src_pix=src_pix, src_pow=src_pow, R_hat=Rh)
    return sc, off

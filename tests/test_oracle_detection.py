"""Monte Carlo checks of the detection threshold (Sec. III-C, App. A), CPU only.

On noise-only data (R = sigma_n^2 I, noise known, so b = R_hat - sigma_n^2 I)
the first multipliers are lambda = -(MF - sigma_n^2): any detection is a false
alarm.  App. A gives the MF pixel standard deviation mf_i / sqrt(N) (K = 1,
sample covariance plugged in); the paper states that a 6-sigma threshold
keeps false alarms over the complete image below 0.1 %.  Checked here:
* the empirical per-pixel standard deviation of the MF image over many sample
  covariances matches the App. A formula;
* with kappa_d = 6 no trial raises a false alarm (the whole active-set solve
  of the oracle adds nothing), while a 2-sigma threshold does (the test has
  power);
* the MVDR image's standard deviation, behind the PWLS threshold, is checked
  in test_oracle_pwls.
"""

import math

import numpy as np

import oracle
import synth


def _noise_trials(trials, seed, noise=1.0):
    sc = synth.make_scene("c0")
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    P, N = sc.P, sc.N
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        Y = math.sqrt(noise / 2) * (rng.standard_normal((P, N)) + 1j * rng.standard_normal((P, N)))
        yield A, Y @ Y.conj().T / N, N, noise


def test_mf_pixel_std_matches_appendix_formula():
    mfs = np.array([oracle.mf_image(A, Rh) for A, Rh, _, _ in _noise_trials(300, 1)])
    N = 4096
    std_mc = mfs.std(axis=0)
    std_formula = mfs.mean(axis=0) / math.sqrt(N)
    # 300 draws: the relative standard error of a std estimate is ~1/sqrt(600)
    assert abs(np.median(std_mc / std_formula) - 1.0) < 0.05
    assert np.all(np.abs(std_mc / std_formula - 1.0) < 0.25)


def test_six_sigma_threshold_raises_no_false_alarm():
    alarms6 = alarms2 = 0
    trials = 200
    for A, Rh, N, noise in _noise_trials(trials, 2):
        mf = oracle.mf_image(A, Rh)
        lam = -(mf - noise)  # gradient at sigma = 0 with the noise removed from b
        if np.any(lam < -oracle.detection_threshold(mf, 6.0, N)):
            alarms6 += 1
        if np.any(lam < -oracle.detection_threshold(mf, 2.0, N)):
            alarms2 += 1
    assert alarms6 == 0
    assert alarms2 > trials // 2


def test_noise_only_solve_adds_nothing():
    for A, Rh, N, noise in _noise_trials(5, 3):
        gamma = oracle.upper_bound(A, Rh)
        eps = oracle.detection_threshold(oracle.mf_image(A, Rh), 6.0, N)
        res = oracle.solve(A, Rh - noise * np.eye(A.shape[0]), gamma, eps)
        assert res.adds == 0 and not np.any(res.state == oracle.STATE_F)

"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case takes the oracle's own source, makes one plausible mistake in it
(dropped conjugate, transposed operand, wrong sign or index, dropped term,
wrong bound), loads the result as a throw-away module, swaps it in, and
checks that at least one pin now fails.  The pins listed are the independent
ones: a test that restates an oracle formula (test_bound_options) is not a pin
and is not counted.
"""

import importlib
import inspect
import sys
import types

import pytest

import oracle
oas = importlib.import_module("oracle.active_set")
oim = importlib.import_module("oracle.imaging")
olsqr = importlib.import_module("oracle.lsqr")  # the package re-exports a function of that name
opw = importlib.import_module("oracle.pwls")
omu = importlib.import_module("oracle.multi")
oog = importlib.import_module("oracle.offgrid")
from tests import test_oracle_pins as pins
from tests import test_oracle_pwls as ppins
from tests import test_oracle_multi as mpins
from tests import test_oracle_offgrid as opins

PINS = [
    pins.test_steering_matches_entrywise_model_and_is_unit_norm,
    pins.test_array_translation_leaves_operators_unchanged,
    pins.test_transposed_covariance_mirrors_the_image,
    pins.test_forward_and_adjoint_equal_dense_khatri_rao_psi,
    pins.test_adjointness_to_1e12,
    pins.test_deconvolution_matrix_closed_form,
    pins.test_mf_image_is_psi_h_r,
    pins.test_single_source_mf_closed_form,
    pins.test_single_source_mvdr_sherman_morrison,
    pins.test_mvdr_below_mf_and_above_truth,
    pins.test_mvdr_equals_jacobi_preconditioned_wls_dirty_image,
    pins.test_single_block_bound_terms_are_app_a_std_by_monte_carlo,
    lambda: pins.test_lsqr_matches_svd_minimum_norm_solution(6, 8),
    pins.test_lsqr_minimum_norm_when_rank_deficient,
    pins.test_lsqr_consistent_system_recovers_exactly_and_residual_decreases,
    pins.test_lsqr_stops_on_normal_residual_test,
    lambda: pins.test_active_set_matches_bvls_objective_and_kkt(40, "mvdr"),
    pins.test_active_set_matches_brute_force_enumeration,
    pins.test_first_release_is_dirty_image_peak,
    lambda: pins.test_exact_recovery_from_exact_covariance([(200, 5.0), (615, 2.0)]),
    pins.test_solution_respects_bounds_and_kkt_with_threshold,
    ppins.test_cholesky_whitening_has_the_paper_cost,
    ppins.test_transformed_operators_equal_dense_weighted_psi,
    lambda: ppins.test_gradient_at_zero_is_minus_unbiased_mvdr_image(0.8),
    lambda: ppins.test_box_pwls_matches_bvls_and_kkt("mvdr"),
    ppins.test_threshold_std_matches_monte_carlo_of_mvdr_image,
    ppins.test_upper_set_pixels_sit_at_the_image_bound,
    mpins.test_identical_blocks_equal_the_single_block_problem,
    mpins.test_stacked_solve_matches_bvls_and_kkt,
    mpins.test_stacked_solve_matches_brute_force_on_a_tiny_grid,
    mpins.test_mvdr_between_assc_and_mf,
    mpins.test_app_a_variances_match_monte_carlo,
    opins.test_gradient_and_gauss_newton_block_against_finite_differences,
    opins.test_one_pixel_shift_is_the_neighbour,
    opins.test_zero_rounds_is_the_on_grid_solve,
    opins.test_off_grid_sources_are_recovered,
]

MUTATIONS = [
    # (module, original text, mistaken text)
    (oim, "A_S.conj() * (U @ A_S)", "A_S * (U @ A_S)"),
    (oim, "@ A_S.conj().T", "@ A_S.T"),
    (oim, "(-2.0 * math.pi / lam)", "(2.0 * math.pi / lam)"),
    (oim, "np.outer(pos[:, 0], l) + np.outer(pos[:, 1], m)",
     "np.outer(pos[:, 0], m) + np.outer(pos[:, 1], l)"),
    (oim, "return np.exp(1j * phase) / math.sqrt(pos.shape[0])", "return np.exp(1j * phase)"),
    (oim, "return adjoint(A, _inverse_hpd(R))", "return 1.0 / adjoint(A, _check_covariance(R))"),
    (oim, "return Linv.conj().T @ Linv", "return Linv @ Linv.conj().T"),
    (oim, "return kappa_d * np.asarray(mf, dtype=np.float64) / math.sqrt(nsamples)",
     "return kappa_d * np.asarray(mf, dtype=np.float64) / nsamples"),
    (oim, "g = g + kappa_b / (h * math.sqrt(nsamples - P - 1))",
     "g = g + kappa_b / (h * math.sqrt(nsamples - P))"),
    (oim, "g = g + kappa_b / (h * math.sqrt(nsamples - P - 1))",
     "g = g + kappa_b / (h * h * math.sqrt(nsamples - P - 1))"),
    (oim, "mf = mf + kappa_b * mf / math.sqrt(nsamples)", "mf = mf + kappa_b * mf / nsamples"),
    (oim, "mf = mf + kappa_b * mf / math.sqrt(nsamples)", "mf = mf + kappa_b / math.sqrt(nsamples)"),
    (olsqr, "u = matvec(v) - alpha * u", "u = matvec(v)"),
    (olsqr, "w = v - (theta / rho) * w", "w = v + (theta / rho) * w"),
    (olsqr, "rhobar = -c * alpha", "rhobar = c * alpha"),
    (olsqr, "phibar = s * phibar", "phibar = c * phibar"),
    (olsqr, "v = np.asarray(rmatvec(u), dtype=np.float64) - beta * v",
     "v = np.asarray(rmatvec(u), dtype=np.float64) - alpha * v"),
    (oas, "lam = np.where(state[act] == STATE_L, g, -g)", "lam = np.where(state[act] == STATE_L, g, g)"),
    (oas, "sigma[ib], state[ib] = gamma[ib], STATE_U", "sigma[ib], state[ib] = 0.0, STATE_U"),
    (oas, "Bb = B0 - fwd(U, gamma[U])", "Bb = B0"),
    (oas, "k = int(np.argmin(lam))", "k = int(np.argmax(lam))"),
    (oas, "E = fwd(S, sigma[S]) - B0", "E = B0 - fwd(S, sigma[S])"),
    (oas, "g = adj(act, E) / K", "g = adj(act, E)"),
    (oas, "return sum(adjoint(Ak[:, S], U[k]) for k, Ak in enumerate(As))",
     "return sum(adjoint(Ak[:, S], U[0]) for k, Ak in enumerate(As))"),
    (omu, "return sum(adjoint(A, np.asarray(R, np.complex128)) for A, R in zip(As, Rs)) / K",
     "return sum(adjoint(A, np.asarray(R, np.complex128)) for A, R in zip(As, Rs))"),
    (omu, "return np.sqrt(sq / nsamples) / K", "return np.sqrt(sq / nsamples) / math.sqrt(K)"),
    (omu, "g = C * K / s1", "g = C / s1"),
    (omu, "g = g + kappa_b * K * np.sqrt(s2) / (math.sqrt(nsamples - P - 1) * s1 * s1)",
     "g = g + kappa_b * np.sqrt(s2) / (math.sqrt(nsamples - P - 1) * s1 * s1)"),
    (omu, "return sum(hs), sum(h * h for h in hs)", "return sum(hs), sum(hs) ** 2"),
    (oog, "d = a * (-1j * c * np.asarray(pos, np.float64)[:, j])", "d = a * (1j * c * np.asarray(pos, np.float64)[:, j])"),
    (oog, "d = pos - pos.mean(axis=0)", "d = pos"),
    (oog, "step = -np.linalg.solve(z[k] * z[k] * G, g)", "step = -np.linalg.solve(z[k] * G, g)"),
    (oog, "phase = (-2.0 * math.pi / lam) * (np.outer(pos[:, 0], np.asarray(l, np.float64))",
     "phase = (2.0 * math.pi / lam) * (np.outer(pos[:, 0], np.asarray(l, np.float64))"),
    (oog, "gamma[F] = _bounds_at(pos, lam, lc[F] + delta[F, 0], mc[F] + delta[F, 1], R, Rinv, kind, C,",
     "gamma[F] = _bounds_at(pos, lam, lc[F], mc[F], R, Rinv, kind, C,"),
    (oas, "if lam_min < -thr:", "if lam_min < thr:"),
    (opw, "return h * h / C, h", "return h / C, h"),
    (opw, "Ahat = (Linv @ A) / np.sqrt(D)[None, :]", "Ahat = (Linv @ A) / D[None, :]"),
    (opw, "Bhat = Linv @ np.asarray(B0, dtype=np.complex128) @ Linv.conj().T",
     "Bhat = Linv @ np.asarray(B0, dtype=np.complex128) @ Linv.T"),
    (opw, "return kappa_d / (np.asarray(h, dtype=np.float64) * math.sqrt(nsamples - P - 1))",
     "return kappa_d / (np.sqrt(np.asarray(h, dtype=np.float64)) * math.sqrt(nsamples - P - 1))"),
    (opw, "res.sigma = res.sigma / D", "res.sigma = res.sigma * D"),
    (opw, "gamma_pw = D * np.asarray(gamma, dtype=np.float64)", "gamma_pw = np.asarray(gamma, dtype=np.float64)"),
]


def _load_mutant(module, old, new):
    src = inspect.getsource(module)
    assert src.count(old) == 1, f"mutation anchor not unique in {module.__name__}: {old!r}"
    mod = types.ModuleType(module.__name__ + "_mutant")
    mod.__package__ = "oracle"
    mod.__file__ = module.__file__
    sys.modules[mod.__name__] = mod
    exec(compile(src.replace(old, new), module.__file__, "exec"), mod.__dict__)
    return mod


def _install(monkeypatch, module, mutant):
    names = [n for n in dir(module) if not n.startswith("__")]
    # every module that imported the mutated functions by name
    targets = [t for t in (oracle, oas, omu, oog) if t is not module]
    for name in names:
        obj = getattr(mutant, name)
        if callable(obj) and getattr(obj, "__module__", None) == mutant.__name__:
            monkeypatch.setattr(module, name, obj)
            for t in targets:
                if hasattr(t, name):
                    monkeypatch.setattr(t, name, obj)


@pytest.mark.parametrize("module,old,new", MUTATIONS,
                         ids=[f"{m.__name__.split('.')[-1]}:{o[:28]}" for m, o, _ in MUTATIONS])
def test_planted_mistake_fails_a_pin(monkeypatch, module, old, new):
    mutant = _load_mutant(module, old, new)
    _install(monkeypatch, module, mutant)
    failures = 0
    for pin in PINS:
        try:
            pin()
        except Exception:  # noqa: BLE001 - any failure of a pin counts
            failures += 1
            break
    assert failures, f"planted mistake {new!r} escaped every pin"


def test_unmutated_oracle_passes_every_pin():
    for pin in PINS:
        pin()

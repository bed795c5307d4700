"""GPU operators at the full sizes of the larger workloads, on sampled outputs.

The 96-antenna / 256 x 256 and 288-antenna / 512 x 512 workloads run the
same launch configurations as in production (full grids, all antennas).  The
oracle computes only sampled outputs there (pixels drawn with a fixed seed,
always including the first and the last pixel), each from its own steering
vector in FP64; the forward product is checked entry by entry over a pixel
subset.  For the 96-antenna workload the whole active-set solve is also run
against the oracle (about half a minute of FP64 on the host), and for the
288-antenna workload its first ten Table I steps; both in FP32 and with the
FP16 / BF16 contractions.

Tolerances as in test_gpu_parity: normwise 1e-5 and every entry within 1e-5
of the peak (the covariances here are well conditioned, cond(R) ~ 11, so
the MVDR power computed from the FP32-rounded inverse meets the same bar).
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(got, ref):
    got = np.asarray(got).astype(np.complex128 if np.iscomplexobj(got) else np.float64)
    ref = np.asarray(ref)
    d = np.linalg.norm((got - ref).ravel())
    n = np.linalg.norm(ref.ravel())
    return d / n if n > 0 else d


def _assert_close(got, ref, tol=TOL, what=""):
    got, ref = np.asarray(got), np.asarray(ref)
    rel = _rel(got, ref)
    mx = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-30)
    print(f"{what}: normwise rel {rel:.3e}, max rel-to-peak {mx:.3e}", flush=True)
    assert rel <= tol, (what, rel)
    assert mx <= tol, (what, mx)


@pytest.fixture(scope="module")
def big():
    return {name: synth.make_scene(name) for name in ("c2", "c4")}


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _sample(Q, k=512, seed=5):
    rng = np.random.default_rng(seed)
    s = np.unique(np.concatenate([[0, Q - 1], rng.choice(Q, size=k, replace=False)]))
    return s


def _steer_at(sc, pix):
    """Steering vectors of the given pixels only (P x len(pix), FP64)."""
    return oracle.steering(sc.pos, sc.lam, sc.grid, pixels=pix)


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_full_grid_dirty_image_and_bound(gpu_lib, ctx, big, name):
    sc = big[name]
    print(f"case full-size dirty image / MVDR {name} P={sc.P} Q={sc.Q}", flush=True)
    geo = gpu_lib.Geometry(sc.pos, sc.lam, sc.grid)
    R = torch.as_tensor(sc.R_hat32).cuda()
    mf = ctx.dirty_image(R, geo).cpu().numpy()
    opts = gpu_lib.default_options()
    opts.nsamples = sc.N
    gamma = ctx.mvdr_bound(R, geo, opts).cpu().numpy()
    pix = _sample(sc.Q)
    A = _steer_at(sc, pix)
    Rr = sc.R_hat32_c128
    _assert_close(mf[pix], oracle.mf_image(A, Rr), what=f"{name} dirty image (sampled)")
    _assert_close(gamma[pix], oracle.upper_bound(A, Rr), what=f"{name} MVDR bound (sampled)")


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_full_size_forward_and_adjoint(gpu_lib, ctx, big, name):
    sc = big[name]
    print(f"case full-size forward / adjoint {name}", flush=True)
    geo = gpu_lib.Geometry(sc.pos, sc.lam, sc.grid)
    rng = np.random.default_rng(11)
    # forward over 4099 pixels (several tiles and a ragged tail)
    S = np.sort(rng.choice(sc.Q, size=4099, replace=False)).astype(np.int32)
    v = rng.uniform(0.0, 2.0, size=S.size)
    Y = ctx.forward(geo, torch.as_tensor(v.astype(np.float32)).cuda(),
                    idx=torch.as_tensor(S).cuda()).cpu().numpy()
    A_S = _steer_at(sc, S.astype(np.int64))
    _assert_close(Y, oracle.forward(A_S, v.astype(np.float32).astype(np.float64)), what=f"{name} forward")
    # adjoint on the whole grid with a Hermitian U, checked at sampled pixels
    X = rng.standard_normal((sc.P, sc.P)) + 1j * rng.standard_normal((sc.P, sc.P))
    U = ((X + X.conj().T) / 2).astype(np.complex64)
    g = ctx.adjoint(geo, torch.as_tensor(U).cuda()).cpu().numpy()
    pix = _sample(sc.Q, seed=13)
    _assert_close(g[pix], oracle.adjoint(_steer_at(sc, pix), U.astype(np.complex128)),
                  what=f"{name} adjoint (sampled)")


@pytest.fixture(scope="module")
def oracle_c2(big):
    sc = big["c2"]
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    R = sc.R_hat32_c128
    mf = oracle.mf_image(A, R)
    gamma = oracle.upper_bound(A, R)
    eps = oracle.detection_threshold(mf, 6.0, sc.N)
    nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
    return oracle.solve(A, R - np.diag(nd), gamma, eps, atol=1e-8, btol=1e-8)


@pytest.fixture(scope="module")
def oracle_c4_ten(big):
    # the full 288-antenna solve takes about a thousand Table I steps (each a
    # 174 GFLOP gradient in FP64 on the host); the state after the first ten
    # is compared instead, at full size
    sc = big["c4"]
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    R = sc.R_hat32_c128
    nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
    return oracle.solve(A, R - np.diag(nd), oracle.upper_bound(A, R),
                        oracle.detection_threshold(oracle.mf_image(A, R), 6.0, sc.N),
                        atol=1e-8, btol=1e-8, max_outer=10)


# FP32: the FP32 bar; FP16 / BF16 (reduced-precision contractions with FP32
# refinement): the reduced-precision bar, and the same sets
BAR = {0: 1e-5, 1: 1e-3, 2: 1e-3}
PNAME = {0: "fp32", 1: "fp16", 2: "bf16"}


def _solve(gpu_lib, ctx, sc, prec, max_outer=-1):
    opts = gpu_lib.default_options()
    opts.nsamples = sc.N
    opts.atol = opts.btol = 1e-7
    opts.precision = prec
    opts.max_outer = max_outer
    nd = np.asarray(sc.noise_diag, np.float32)
    return ctx.solve(torch.as_tensor(sc.R_hat32).cuda(), gpu_lib.Geometry(sc.pos, sc.lam, sc.grid), opts,
                     noise_diag=torch.as_tensor(nd).cuda())


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_solve_96_antennas_matches_oracle(gpu_lib, ctx, big, oracle_c2, prec):
    sc = big["c2"]
    print(f"case solve c2 (P=96, Q=65536) {PNAME[prec]} against the oracle", flush=True)
    ref = oracle_c2
    sigma, state, _, _, stats = _solve(gpu_lib, ctx, sc, prec)
    rel = _rel(sigma.cpu().numpy(), ref.sigma)
    print(f"gpu stats {stats}; oracle outer {ref.outer_iters}; image error {rel:.3e}; residual "
          f"{stats['rel_residual']:.9f} / {ref.rel_residual:.9f}", flush=True)
    np.testing.assert_array_equal(state.cpu().numpy(), ref.state)
    _assert_close(sigma.cpu().numpy(), ref.sigma, tol=BAR[prec], what=f"solve sigma c2 {PNAME[prec]}")
    assert abs(stats["rel_residual"] - ref.rel_residual) <= 1e-3 * ref.rel_residual


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_solve_288_antennas_first_ten_steps(gpu_lib, ctx, big, oracle_c4_ten, prec):
    sc = big["c4"]
    print(f"case solve c4 (P=288, Q=512^2) {PNAME[prec]}, first 10 Table I steps, against the oracle", flush=True)
    ref = oracle_c4_ten
    sigma, state, _, _, stats = _solve(gpu_lib, ctx, sc, prec, max_outer=10)
    rel = _rel(sigma.cpu().numpy(), ref.sigma)
    print(f"gpu stats {stats}; oracle outer {ref.outer_iters} adds {ref.adds}; image error {rel:.3e}; residual "
          f"{stats['rel_residual']:.9f} / {ref.rel_residual:.9f}", flush=True)
    assert stats["status"] == gpu_lib.WMAXOUTER and stats["outer_iters"] == ref.outer_iters == 10
    np.testing.assert_array_equal(state.cpu().numpy(), ref.state)
    _assert_close(sigma.cpu().numpy(), ref.sigma, tol=BAR[prec], what=f"solve sigma c4 {PNAME[prec]}, 10 steps")
    assert abs(stats["rel_residual"] - ref.rel_residual) <= 1e-3 * ref.rel_residual

"""GPU (HIP library through the C ABI) against the FP64 oracle, element by element.

Tolerances (FP32 contractions with FP32 steering entries of ~1 ulp):
* images and operator outputs: normwise relative error <= 1e-5 and every entry
  within 1e-5 * max|reference| (per-pixel relative error is no valid gate:
  sidelobe pixels cancel);
* the active-set solve: identical final sets on the 24-antenna workload and a
  relative image error <= 1e-5.
The oracle always sees the complex64-rounded covariance upcast to complex128,
i.e. exactly the bits the GPU receives.
"""

import math

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
    n = np.linalg.norm(np.asarray(ref).ravel())
    return d / n if n > 0 else d


def _assert_close(got, ref, tol=TOL, what=""):
    got = np.asarray(got)
    ref = np.asarray(ref)
    rel = _rel(got, ref)
    mx = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-30) if ref.size else 0.0
    print(f"{what}: normwise rel {rel:.3e}, max rel-to-peak {mx:.3e}", flush=True)
    assert rel <= tol, (what, rel)
    assert mx <= tol, (what, mx)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def scenes():
    return {name: synth.make_scene(name) for name in ("c0", "c1")}


def _geo(gpu_lib, sc):
    return gpu_lib.Geometry(sc.pos, sc.lam, sc.grid)


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def _rand_geometry(rng, P, nl, nm, radius=10.0, L=0.6):
    r = radius * np.sqrt(rng.random(P))
    t = 2 * np.pi * rng.random(P)
    pos = np.stack([r * np.cos(t), r * np.sin(t)], axis=1)
    grid = (nl, nm, -L, 2 * L / nl, -L * 0.9, 1.8 * L / nm)
    return pos, 1.3, grid


def _rand_hermitian(rng, P, pd=False):
    X = rng.standard_normal((P, P)) + 1j * rng.standard_normal((P, P))
    H = X @ X.conj().T / P + 0.5 * np.eye(P) if pd else 0.5 * (X + X.conj().T)
    return H.astype(np.complex64)


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_dirty_image_matches_oracle(gpu_lib, ctx, scenes, name):
    sc = scenes[name]
    print(f"case dirty_image {name} P={sc.P} Q={sc.Q}", flush=True)
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    ref = oracle.mf_image(A, sc.R_hat32_c128)
    got = ctx.dirty_image(_dev(sc.R_hat32, torch.complex64), _geo(gpu_lib, sc)).cpu().numpy()
    _assert_close(got, ref, what=f"mf {name}")


@pytest.mark.parametrize("name", ["c0", "c1"])
@pytest.mark.parametrize("bound", ["mvdr", "mf", "mvdr_opts"])
def test_upper_bound_matches_oracle(gpu_lib, ctx, scenes, name, bound):
    sc = scenes[name]
    print(f"case bound {bound} {name}", flush=True)
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    R = sc.R_hat32_c128
    opts = gpu_lib.default_options()
    opts.nsamples = sc.N
    if bound == "mvdr":
        ref = oracle.upper_bound(A, R, "mvdr")
    elif bound == "mf":
        opts.bound = gpu_lib.BOUND_MF
        opts.kappa_b = 6.0
        ref = oracle.upper_bound(A, R, "mf", kappa_b=6.0, nsamples=sc.N)
    else:
        opts.C = sc.N / (sc.N - sc.P)
        opts.kappa_b = 6.0
        ref = oracle.upper_bound(A, R, "mvdr", C=opts.C, kappa_b=6.0, nsamples=sc.N)
    got = ctx.mvdr_bound(_dev(sc.R_hat32, torch.complex64), _geo(gpu_lib, sc), opts).cpu().numpy()
    _assert_close(got, ref, what=f"gamma {bound} {name}")


def test_bound_none_is_infinite(gpu_lib, ctx, scenes):
    sc = scenes["c0"]
    opts = gpu_lib.default_options()
    opts.bound = gpu_lib.BOUND_NONE
    got = ctx.mvdr_bound(_dev(sc.R_hat32, torch.complex64), _geo(gpu_lib, sc), opts).cpu().numpy()
    assert np.all(np.isinf(got)) and np.all(got > 0)


@pytest.mark.parametrize("P,nl,nm", [(24, 32, 32), (48, 33, 17), (5, 7, 3), (13, 40, 9), (96, 20, 20),
                                     (288, 16, 12), (1, 4, 4)])
@pytest.mark.parametrize("n", [0, 1, 17, 64, 65, 300])
def test_adjoint_subset_matches_oracle(gpu_lib, ctx, P, nl, nm, n):
    rng = np.random.default_rng(1000 * P + n)
    pos, lam, grid = _rand_geometry(rng, P, nl, nm)
    Q = nl * nm
    n = min(n, Q)
    print(f"case adjoint P={P} grid={nl}x{nm} n={n}", flush=True)
    idx = np.sort(rng.choice(Q, size=n, replace=False)).astype(np.int32)
    U = _rand_hermitian(rng, P)
    A = oracle.steering(pos, lam, grid, pixels=idx)
    ref = oracle.adjoint(A, U.astype(np.complex128))
    geo = gpu_lib.Geometry(pos, lam, grid)
    got = ctx.adjoint(geo, _dev(U, torch.complex64), idx=_dev(idx, torch.int32)).cpu().numpy()
    if n:
        _assert_close(got, ref, what=f"adjoint P={P} n={n}")
    # the whole grid, no index list
    refQ = oracle.adjoint(oracle.steering(pos, lam, grid), U.astype(np.complex128))
    gotQ = ctx.adjoint(geo, _dev(U, torch.complex64)).cpu().numpy()
    _assert_close(gotQ, refQ, what=f"adjoint all P={P}")


@pytest.mark.parametrize("P,nl,nm", [(24, 32, 32), (48, 33, 17), (5, 7, 3), (13, 40, 9), (96, 20, 20),
                                     (288, 16, 12), (1, 4, 4)])
@pytest.mark.parametrize("n", [0, 1, 17, 64, 65, 300])
def test_forward_subset_matches_oracle(gpu_lib, ctx, P, nl, nm, n):
    rng = np.random.default_rng(2000 * P + n)
    pos, lam, grid = _rand_geometry(rng, P, nl, nm)
    Q = nl * nm
    n = min(n, Q)
    print(f"case forward P={P} grid={nl}x{nm} n={n}", flush=True)
    idx = rng.choice(Q, size=n, replace=False).astype(np.int32)
    v = rng.standard_normal(n).astype(np.float32)
    A = oracle.steering(pos, lam, grid, pixels=idx)
    ref = oracle.forward(A, v.astype(np.float64))
    geo = gpu_lib.Geometry(pos, lam, grid)
    got = ctx.forward(geo, _dev(v, torch.float32), idx=_dev(idx, torch.int32)).cpu().numpy()
    if n == 0:
        assert np.all(got == 0)
    else:
        _assert_close(got, ref, what=f"forward P={P} n={n}")


@pytest.mark.parametrize("P,nl,nm", [(48, 128, 128), (96, 64, 64), (288, 48, 48), (20, 70, 9), (136, 33, 31),
                                     (8, 40, 40)])
def test_forward_full_grid_matches_oracle(gpu_lib, ctx, P, nl, nm):
    # every pixel of the grid: many pixels per workgroup, many workgroups
    # (partials), several antenna-tile block pairs (a ragged last tile at 20,
    # 136 and 8 antennas, blocks of two tiles at 8 and 20)
    rng = np.random.default_rng(3000 + P)
    pos, lam, grid = _rand_geometry(rng, P, nl, nm)
    Q = nl * nm
    print(f"case forward full grid P={P} grid={nl}x{nm}", flush=True)
    v = rng.standard_normal(Q).astype(np.float32)
    ref = oracle.forward(oracle.steering(pos, lam, grid), v.astype(np.float64))
    geo = gpu_lib.Geometry(pos, lam, grid)
    got = ctx.forward(geo, _dev(v, torch.float32)).cpu().numpy()
    _assert_close(got, ref, what=f"forward full grid P={P}")
    np.testing.assert_array_equal(got, np.conj(got.T))  # Hermitian by construction


def test_gpu_adjointness(gpu_lib, ctx, scenes):
    sc = scenes["c1"]
    rng = np.random.default_rng(7)
    geo = _geo(gpu_lib, sc)
    idx = np.sort(rng.choice(sc.Q, size=500, replace=False)).astype(np.int32)
    x = rng.standard_normal(500).astype(np.float32)
    Y = _rand_hermitian(rng, sc.P)
    Fx = ctx.forward(geo, _dev(x, torch.float32), idx=_dev(idx, torch.int32)).cpu().numpy()
    AY = ctx.adjoint(geo, _dev(Y, torch.complex64), idx=_dev(idx, torch.int32)).cpu().numpy()
    lhs = float(np.real(np.vdot(Fx.astype(np.complex128), Y.astype(np.complex128))))
    rhs = float(x.astype(np.float64) @ AY.astype(np.float64))
    scale = np.linalg.norm(Fx) * np.linalg.norm(Y)
    print(f"adjointness: {lhs} vs {rhs}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * scale


@pytest.mark.parametrize("P", [8, 100, 288])
def test_not_positive_definite_is_reported(gpu_lib, ctx, P):
    # P = 8: LDS-resident factorisation; 100 and 288: the blocked one (panels
    # of 16), failing in the first column, in the last column, or on a NaN
    print(f"case not positive definite P={P}", flush=True)
    rng = np.random.default_rng(3)
    pos, lam, grid = _rand_geometry(rng, P, 8, 8)
    R = _rand_hermitian(rng, P)
    R = (R - (np.abs(np.linalg.eigvalsh(R)).max() + 1) * np.eye(P)).astype(np.complex64)
    geo = gpu_lib.Geometry(pos, lam, grid)
    with pytest.raises(gpu_lib.ClsimgError) as ei:
        ctx.mvdr_bound(_dev(R, torch.complex64), geo)
    assert ei.value.status == gpu_lib.ENOTPD
    Rl = np.eye(P, dtype=np.complex64)
    Rl[P - 1, P - 1] = -1.0
    with pytest.raises(gpu_lib.ClsimgError) as ei:
        ctx.mvdr_bound(_dev(Rl, torch.complex64), geo)
    assert ei.value.status == gpu_lib.ENOTPD
    Rn = np.eye(P, dtype=np.complex64)
    Rn[2, 3] = np.nan
    with pytest.raises(gpu_lib.ClsimgError) as ei:
        ctx.mvdr_bound(_dev(Rn, torch.complex64), geo)
    assert ei.value.status == gpu_lib.ENOTPD
    # the context stays usable: a valid covariance of the same size afterwards
    Rg = _rand_hermitian(rng, P, pd=True)
    got = ctx.mvdr_bound(_dev(Rg, torch.complex64), geo).cpu().numpy()
    _assert_close(got, oracle.upper_bound(oracle.steering(pos, lam, grid), Rg.astype(np.complex128)),
                  what=f"mvdr after ENOTPD P={P}")


@pytest.mark.parametrize("P", [65, 150, 288])
def test_mvdr_bound_beyond_the_lds_factorisation(gpu_lib, ctx, P):
    # FP64 Cholesky in panels of 16 columns (a ragged last panel at 65 and 150)
    # and one substitution workgroup per column of R^-1
    print(f"case mvdr bound P={P}", flush=True)
    rng = np.random.default_rng(40 + P)
    pos, lam, grid = _rand_geometry(rng, P, 24, 20)
    R = _rand_hermitian(rng, P, pd=True)
    geo = gpu_lib.Geometry(pos, lam, grid)
    got = ctx.mvdr_bound(_dev(R, torch.complex64), geo).cpu().numpy()
    _assert_close(got, oracle.upper_bound(oracle.steering(pos, lam, grid), R.astype(np.complex128)),
                  what=f"mvdr P={P}")


def _oracle_solve(sc, atol=1e-8, btol=1e-8, noise=True, kappa_d=6.0):
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    mf = oracle.mf_image(A, R)
    gamma = oracle.upper_bound(A, R)
    eps = oracle.detection_threshold(mf, kappa_d, sc.N)
    nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64) if noise else np.zeros(sc.P)
    res = oracle.solve(A, R - np.diag(nd), gamma, eps, atol=atol, btol=btol)
    return res, mf, gamma


def _gpu_solve(gpu_lib, ctx, sc, atol=1e-7, btol=1e-7, noise=True, kappa_d=6.0, **engine):
    # engine: loop / lsqr_engine / hand_over_free options (every engine gives the same iterates)
    opts = gpu_lib.default_options()
    opts.nsamples = sc.N
    opts.atol, opts.btol = atol, btol
    opts.kappa_d = kappa_d
    for k, val in engine.items():
        setattr(opts, k, val)
    nd = _dev(sc.noise_diag, torch.float32) if noise else None
    sigma, state, mf, gamma, stats = ctx.solve(_dev(sc.R_hat32, torch.complex64), _geo(gpu_lib, sc),
                                               opts, noise_diag=nd)
    return sigma.cpu().numpy(), state.cpu().numpy(), mf.cpu().numpy(), gamma.cpu().numpy(), stats


@pytest.mark.parametrize("noise", [True, False])
def test_solve_c0_identical_sets(gpu_lib, ctx, scenes, noise):
    sc = scenes["c0"]
    print(f"case solve c0 noise={noise}", flush=True)
    ref, mf_ref, gamma_ref = _oracle_solve(sc, noise=noise)
    sigma, state, mf, gamma, stats = _gpu_solve(gpu_lib, ctx, sc, noise=noise)
    print("gpu stats", stats, flush=True)
    print("oracle outer", ref.outer_iters, "adds", ref.adds, "drops", ref.drops, "lsqr", ref.lsqr_iters_total,
          flush=True)
    _assert_close(mf, mf_ref, what="solve mf")
    _assert_close(gamma, gamma_ref, what="solve gamma")
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what="solve sigma c0")
    assert stats["status"] == ref.status
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops
    assert abs(stats["rel_residual"] - ref.rel_residual) <= 1e-5 * max(ref.rel_residual, 1e-12) + 1e-7


@pytest.mark.parametrize("host,n", [(False, 37), (True, 37), (True, 101)])
def test_solve_ragged_grid(gpu_lib, ctx, host, n):
    # 40 antennas (5 row tiles, padding antennas inside the last tile pair),
    # 37 x 37 pixels: the last 16-pixel tile holds 9 pixels; device loop and
    # host loop.  101 x 101 pixels: the host loop's set compaction over two
    # whole chunks of 4096 states and a ragged third
    sc = synth.make_scene("c1", P=40, n=n, seed=41, points=(30, ("loguniform", 0.5, 50.0)), blobs=(1, 5.0, 5.0))
    print(f"case solve ragged P={sc.P} Q={sc.Q} host={host}", flush=True)
    ref, mf_ref, gamma_ref = _oracle_solve(sc)
    sigma, state, mf, gamma, stats = _gpu_solve(gpu_lib, ctx, sc, loop=gpu_lib.LOOP_HOST if host else 0)
    print(f"  steps {stats['outer_iters']} / {ref.outer_iters}, nF {stats['nF']}", flush=True)
    _assert_close(mf, mf_ref, what="ragged mf")
    _assert_close(gamma, gamma_ref, what="ragged gamma")
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what="ragged sigma")
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops


@pytest.mark.parametrize("P,n", [(104, 40), (150, 32)])
def test_solve_large_arrays_split_rows(gpu_lib, ctx, P, n):
    # beyond 96 antennas the LSQR subproblems run the split-K correlation and
    # the row-split beamformer (groups of four row tiles, the last one ragged
    # at 104 and 150 antennas); the FP64 factorisation runs in panels
    sc = synth.make_scene("c2", P=P, n=n, seed=P, points=(15, ("powerlaw", 0.5, 500.0)))
    print(f"case solve P={sc.P} Q={sc.Q} (row-split LSQR adjoint)", flush=True)
    ref, mf_ref, gamma_ref = _oracle_solve(sc)
    sigma, state, mf, gamma, stats = _gpu_solve(gpu_lib, ctx, sc)
    print(f"  steps {stats['outer_iters']} / {ref.outer_iters}, nF {stats['nF']}, lsqr "
          f"{stats['lsqr_iters_total']} / {ref.lsqr_iters_total}", flush=True)
    _assert_close(gamma, gamma_ref, what=f"gamma P={P}")
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what=f"sigma P={P}")
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops


@pytest.mark.parametrize("P,n,pts,engine", [(50, 32, 15, 3), (80, 32, 15, 3), (88, 64, 400, 3), (56, 32, 15, 2)])
def test_solve_two_kernel_lsqr_row_tiles(gpu_lib, ctx, P, n, pts, engine):
    # 7..12 row tiles: the free-set LSQR in two launches per iteration, the
    # adjoint with one wave per row tile (7, 10 and 11 here; 50 antennas
    # leaves the last tile ragged), the forward step's operands 128 pixels at
    # a time (the 88-antenna case ends with 176 free pixels: two chunks); and
    # the cooperative kernel where it still fits (56 antennas), asked for by
    # name since the two-kernel step is the default there
    sc = synth.make_scene("c2", P=P, n=n, seed=500 + P, points=(pts, ("powerlaw", 0.5, 500.0)))
    print(f"case solve P={sc.P} Q={sc.Q} (LSQR engine {engine}, {pts} sources)", flush=True)
    ref, mf_ref, gamma_ref = _oracle_solve(sc)
    sigma, state, mf, gamma, stats = _gpu_solve(gpu_lib, ctx, sc, lsqr_engine=engine)
    print(f"  steps {stats['outer_iters']} / {ref.outer_iters}, nF {stats['nF']}, lsqr "
          f"{stats['lsqr_iters_total']} / {ref.lsqr_iters_total}", flush=True)
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what=f"sigma P={P}")
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops
    assert abs(stats["rel_residual"] - ref.rel_residual) <= 1e-3 * ref.rel_residual


def test_solve_c1_image_error(gpu_lib, ctx, scenes):
    sc = scenes["c1"]
    print("case solve c1", flush=True)
    ref, _, _ = _oracle_solve(sc)
    sigma, state, mf, gamma, stats = _gpu_solve(gpu_lib, ctx, sc)
    print("gpu stats", stats, flush=True)
    print("oracle outer", ref.outer_iters, "adds", ref.adds, "drops", ref.drops, "lsqr",
          ref.lsqr_iters_total, flush=True)
    print("state mismatches", int(np.sum(state != ref.state)), flush=True)
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what="solve sigma c1")


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("name", ["c0", "c1"])
def test_solve_each_lsqr_engine_matches_oracle(gpu_lib, ctx, scenes, name, path):
    # every LSQR engine (one workgroup, one cooperative kernel, two kernels per
    # step) must reproduce the oracle's solve
    sc = scenes[name]
    print(f"case solve {name} LSQR engine {path}", flush=True)
    ref, _, _ = _oracle_solve(sc)
    sigma, state, mf, gamma, stats = _gpu_solve(gpu_lib, ctx, sc, loop=gpu_lib.LOOP_HOST, lsqr_engine=path)
    print("gpu stats", stats, flush=True)
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what=f"solve sigma {name} engine {path}")


@pytest.mark.parametrize("name,maxf", [("c0", 3), ("c1", 40)])
def test_solve_device_loop_hands_over_to_host(gpu_lib, ctx, scenes, name, maxf):
    # the device-resident loop stops when |F| passes maxf and the host loop
    # continues from the same sigma and state; the result must not change
    sc = scenes[name]
    print(f"case solve {name} device loop handover at |F| > {maxf}", flush=True)
    ref, _, _ = _oracle_solve(sc)
    sigma, state, mf, gamma, stats = _gpu_solve(gpu_lib, ctx, sc, hand_over_free=maxf)
    print("gpu stats", stats, flush=True)
    assert int(np.sum(ref.state == 1)) > maxf  # the handover really happens
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what=f"solve sigma {name} handover")
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops


@pytest.mark.parametrize("host", [0, 1])
@pytest.mark.parametrize("name", ["c0", "c1"])
def test_solve_tight_bound_uses_upper_set(gpu_lib, scenes, name, host):
    # a bias factor C < 1 lowers the MVDR bound until pixels stop at it: the
    # upper set U, b = B0 - Psi_U gamma_U and the moves into and out of U are
    # exercised on the device loop (host=0) and on the host loop (host=1)
    sc = scenes[name]
    C = 0.25
    print(f"case solve {name} C={C} host loop {host}", flush=True)
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    mf_ref = oracle.mf_image(A, R)
    gamma_ref = oracle.upper_bound(A, R, C=C)
    eps = oracle.detection_threshold(mf_ref, 6.0, sc.N)
    nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
    ref = oracle.solve(A, R - np.diag(nd), gamma_ref, eps, atol=1e-8, btol=1e-8)
    ctx2 = gpu_lib.Context(0)
    try:
        opts = gpu_lib.default_options()
        opts.nsamples = sc.N
        opts.atol = opts.btol = 1e-7
        opts.C = C
        opts.loop = host
        sigma, state, mf, gamma, stats = ctx2.solve(_dev(sc.R_hat32, torch.complex64), _geo(gpu_lib, sc), opts,
                                                    noise_diag=_dev(sc.noise_diag, torch.float32))
    finally:
        ctx2.close()
    sigma, state = sigma.cpu().numpy(), state.cpu().numpy()
    print("gpu stats", stats, "oracle U", int(np.sum(ref.state == 2)), flush=True)
    assert int(np.sum(ref.state == 2)) > 0
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what=f"solve sigma {name} C={C}")
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops


def _pwls_case(gpu_lib, ctx, sc, what, C=1.0, **optfields):
    # preconditioned weighted LS (eq. preWLS) with the MVDR bound and the
    # MVDR-image threshold, against the oracle's PWLS solve
    print(f"case PWLS solve {what} (P={sc.P}, Q={sc.Q}) C={C} {optfields}", flush=True)
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    gamma = oracle.upper_bound(A, R, C=C)
    _, h = oracle.pwls_scaling(A, R, C)
    eps = oracle.pwls_threshold(h, 6.0, sc.N, sc.P)
    nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
    ref = oracle.solve_pwls(A, R, R - np.diag(nd), gamma, eps, C=C, atol=1e-8, btol=1e-8)
    opts = gpu_lib.default_options()
    opts.nsamples = sc.N
    opts.atol = opts.btol = 1e-7
    opts.cost = gpu_lib.COST_PWLS
    opts.C = C
    for k, v in optfields.items():
        setattr(opts, k, v)
    sigma, state, mf, gam, stats = ctx.solve(_dev(sc.R_hat32, torch.complex64), _geo(gpu_lib, sc), opts,
                                             noise_diag=_dev(sc.noise_diag, torch.float32))
    print("gpu stats", stats, "oracle outer", ref.outer_iters, "adds", ref.adds, "drops", ref.drops, flush=True)
    state, sigma = state.cpu().numpy(), sigma.cpu().numpy()
    print("state mismatches", int(np.sum(state != ref.state)), flush=True)
    assert ref.adds > 0
    np.testing.assert_array_equal(state, ref.state)
    _assert_close(sigma, ref.sigma, what=f"PWLS sigma {what}")
    _assert_close(gam.cpu().numpy(), gamma, what=f"PWLS gamma {what}")
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops
    print("oracle U", int(np.sum(ref.state == 2)), flush=True)
    return stats, ref


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_solve_pwls_matches_oracle(gpu_lib, ctx, scenes, name):
    _pwls_case(gpu_lib, ctx, scenes[name], name)


def test_solve_pwls_on_the_host_loop_matches_oracle(gpu_lib, ctx, scenes):
    # the host-driven loop: the whitened steering rows of the free set in the
    # cache of the two-kernel LSQR, E coloured back for the multipliers
    _pwls_case(gpu_lib, ctx, scenes["c0"], "c0 host loop", loop=gpu_lib.LOOP_HOST)


def test_solve_pwls_hand_over_matches_oracle(gpu_lib, ctx, scenes):
    # the device loop hands the PWLS solve over to the host loop part way
    stats, _ = _pwls_case(gpu_lib, ctx, scenes["c1"], "c1 hand-over", hand_over_free=4)
    assert stats["nF"] > 4


@pytest.mark.parametrize("P,n,pts,C", [(72, 36, 12, 1.0), (96, 40, 12, 1.0), (96, 40, 30, 0.25)])
def test_solve_pwls_beyond_48_antennas_matches_oracle(gpu_lib, ctx, P, n, pts, C):
    # C = 0.25 moves pixels into U and drops them there (b whitened every step)
    sc = synth.make_scene("c2", P=P, n=n, seed=400 + P, points=(pts, ("powerlaw", 0.5, 500.0)))
    _, ref = _pwls_case(gpu_lib, ctx, sc, f"P={P}", C=C)
    if C < 1.0:
        assert int(np.sum(ref.state == 2)) > 0 and ref.drops > 0


def test_pwls_beyond_96_antennas_is_not_supported(gpu_lib):
    sc = synth.make_scene("c2", P=104, n=16, seed=12)
    ctx2 = gpu_lib.Context(0)
    try:
        opts = gpu_lib.default_options()
        opts.nsamples = sc.N
        opts.cost = gpu_lib.COST_PWLS
        with pytest.raises(gpu_lib.ClsimgError) as ei:
            ctx2.solve(_dev(sc.R_hat32, torch.complex64), _geo(gpu_lib, sc), opts)
        assert ei.value.status == gpu_lib.ENOTSUP
    finally:
        ctx2.close()


def test_noise_only_solves_raise_no_false_alarm(gpu_lib, ctx, scenes):
    # Sec. III-C: with the 6-sigma threshold a noise-only covariance (noise
    # known and removed from b) must not release any pixel
    sc = scenes["c0"]
    rng = np.random.default_rng(17)
    opts = gpu_lib.default_options()
    opts.nsamples = sc.N
    opts.atol = opts.btol = 1e-7
    nd = _dev(np.ones(sc.P, np.float32), torch.float32)
    for t in range(20):
        Y = np.sqrt(0.5) * (rng.standard_normal((sc.P, sc.N)) + 1j * rng.standard_normal((sc.P, sc.N)))
        Rh = (Y @ Y.conj().T / sc.N).astype(np.complex64)
        sigma, state, _, _, stats = ctx.solve(_dev(Rh, torch.complex64), _geo(gpu_lib, sc), opts, noise_diag=nd)
        assert stats["adds"] == 0, (t, stats)
        assert int((state.cpu().numpy() == 1).sum()) == 0

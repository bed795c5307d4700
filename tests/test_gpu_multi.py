"""K covariance blocks over one grid (clsimg_solve_multi) against the oracle.

Blocks are snapshots of one sky with the array rotated between them (Earth
rotation) and/or frequency channels (other wavelengths).  Each case compares
the MF image, the bound and the constrained image with the oracle's stacked
formulation (eqs. mfdimg, wmvdr, UCLS; App. A), and the final active sets
exactly.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(got, ref):
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


CASES = {
    # name: (config, K, rotation, wavelengths, overrides)
    "p24_k2_rot": ("c0", 2, 0.08, None, {}),
    "p24_k3_rot_chan": ("c0", 3, 0.05, [1.0, 1.1, 1.25], {}),
    "p48_k3_chan": ("c1", 3, 0.0, [1.0, 1.2, 1.4], {"n": 48, "points": (15, ("loguniform", 0.5, 50.0)),
                                                    "blobs": (0, 6.0, 0.0)}),
    "p96_k2_rot": ("c2", 2, 0.03, None, {"n": 40, "points": (20, ("powerlaw", 0.5, 500.0))}),
    # 13 row tiles: the adjoint's 32-pixel tiles with two waves per row group,
    # one workgroup row per block
    "p104_k2_chan": ("c2", 2, 0.0, [1.0, 1.15], {"P": 104, "n": 24, "points": (10, ("powerlaw", 0.5, 500.0))}),
}


def _blocks(gpu_lib, scs):
    return [{"R": torch.as_tensor(sc.R_hat32).cuda(), "geo": gpu_lib.Geometry(sc.pos, sc.lam, sc.grid),
             "noise_diag": torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()} for sc in scs]


def _oracle(scs, bound="mvdr", kappa_b=0.0, max_outer=-1):
    As = oracle.steering_blocks([(sc.pos, sc.lam) for sc in scs], scs[0].grid)
    Rs = [sc.R_hat32_c128 for sc in scs]
    N = scs[0].N
    mf = oracle.mf_image_multi(As, Rs)
    gamma = oracle.upper_bound_multi(As, Rs, kind=bound, kappa_b=kappa_b, nsamples=N)
    eps = oracle.detection_threshold_multi(As, Rs, 6.0, N)
    B0s = [R - np.diag(np.asarray(sc.noise_diag, np.float32).astype(np.float64)) for R, sc in zip(Rs, scs)]
    ref = oracle.solve_multi(As, B0s, gamma, eps, atol=1e-8, btol=1e-8, max_outer=max_outer)
    return ref, mf, gamma


def _opts(gpu_lib, scs, **kw):
    o = gpu_lib.default_options()
    o.nsamples = scs[0].N
    o.atol = o.btol = 1e-7
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@pytest.mark.parametrize("name", sorted(CASES))
def test_blocks_match_oracle(gpu_lib, ctx, name):
    cfg, K, rot, lams, ov = CASES[name]
    scs = synth.make_block_scenes(cfg, K=K, rotation=rot, lams=lams, **ov)
    print(f"case multi {name}: K={K} P={scs[0].P} Q={scs[0].Q}", flush=True)
    ref, mf_ref, gam_ref = _oracle(scs)
    sigma, state, mf, gamma, stats = ctx.solve_multi(_blocks(gpu_lib, scs), _opts(gpu_lib, scs))
    torch.cuda.synchronize()
    s, st = sigma.cpu().numpy(), state.cpu().numpy()
    print(f"  mf {_rel(mf.cpu().numpy(), mf_ref):.2e} gamma {_rel(gamma.cpu().numpy(), gam_ref):.2e}; "
          f"image {_rel(s, ref.sigma):.2e}; steps {stats['outer_iters']} oracle {ref.outer_iters}, adds "
          f"{stats['adds']} / {ref.adds}; residual {stats['rel_residual']:.6f} / {ref.rel_residual:.6f}", flush=True)
    assert _rel(mf.cpu().numpy(), mf_ref) <= TOL
    assert _rel(gamma.cpu().numpy(), gam_ref) <= TOL
    np.testing.assert_array_equal(st, ref.state)
    assert _rel(s, ref.sigma) <= TOL
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops
    assert abs(stats["rel_residual"] - ref.rel_residual) <= TOL * ref.rel_residual


@pytest.mark.parametrize("bound,kappa_b", [("mf", 2.0), ("none", 0.0), ("mvdr", 3.0)])
def test_bound_options(gpu_lib, ctx, bound, kappa_b):
    scs = synth.make_block_scenes("c0", K=2, rotation=0.1)
    print(f"case multi bound {bound} kappa_b {kappa_b}", flush=True)
    ref, _, gam_ref = _oracle(scs, bound=bound, kappa_b=kappa_b)
    b = {"mvdr": gpu_lib.BOUND_MVDR, "mf": gpu_lib.BOUND_MF, "none": gpu_lib.BOUND_NONE}[bound]
    sigma, state, _, gamma, _ = ctx.solve_multi(_blocks(gpu_lib, scs), _opts(gpu_lib, scs, bound=b, kappa_b=kappa_b))
    g = gamma.cpu().numpy()
    if bound == "none":
        assert np.all(np.isinf(g))
    else:
        assert _rel(g, gam_ref) <= TOL
    np.testing.assert_array_equal(state.cpu().numpy(), ref.state)
    assert _rel(sigma.cpu().numpy(), ref.sigma) <= TOL


def test_single_block_equals_the_single_solve(gpu_lib, ctx):
    sc = synth.make_scene("c0")
    print("case multi K=1 against clsimg_solve", flush=True)
    blk = _blocks(gpu_lib, [sc])
    o = _opts(gpu_lib, [sc])
    s1, st1, mf1, g1, stats1 = ctx.solve_multi(blk, o)
    s0, st0, mf0, g0, stats0 = ctx.solve(blk[0]["R"], blk[0]["geo"], o, noise_diag=blk[0]["noise_diag"])
    assert torch.equal(st1, st0)
    assert _rel(s1.cpu().numpy(), s0.cpu().numpy().astype(np.float64)) <= TOL
    assert torch.allclose(mf1, mf0, rtol=1e-6) and torch.allclose(g1, g0, rtol=1e-6)
    assert stats1["adds"] == stats0["adds"]


def test_half_precision_blocks(gpu_lib, ctx):
    scs = synth.make_block_scenes("c0", K=2, rotation=0.08)
    print("case multi fp16 split", flush=True)
    ref, mf_ref, _ = _oracle(scs)
    sigma, state, mf, _, _ = ctx.solve_multi(_blocks(gpu_lib, scs), _opts(gpu_lib, scs, precision=gpu_lib.FP16))
    np.testing.assert_array_equal(state.cpu().numpy(), ref.state)
    assert _rel(sigma.cpu().numpy(), ref.sigma) <= TOL and _rel(mf.cpu().numpy(), mf_ref) <= TOL


def test_multi_rejects(gpu_lib, ctx):
    scs = synth.make_block_scenes("c0", K=2)
    blk = _blocks(gpu_lib, scs)
    with pytest.raises(gpu_lib.ClsimgError) as ei:
        ctx.solve_multi(blk, _opts(gpu_lib, scs, cost=gpu_lib.COST_PWLS))
    assert ei.value.status == gpu_lib.ENOTSUP
    other = synth.make_scene("c1", n=32)
    bad = blk[:1] + _blocks(gpu_lib, [other])
    with pytest.raises(ValueError):  # grids differ
        ctx.solve_multi(bad, _opts(gpu_lib, scs))


def test_six_blocks_at_the_48_antenna_workload_size(gpu_lib, ctx):
    # 2 snapshots x 3 channels of the 48-antenna, 128 x 128 workload
    angles = [0.05 * k for c in range(3) for k in range(2)]
    lams = [1.0 + 0.1 * c for c in range(3) for k in range(2)]
    scs = synth.make_block_scenes("c1", K=6, angles=angles, lams=lams)
    print(f"case multi 6 blocks P={scs[0].P} Q={scs[0].Q}", flush=True)
    ref, mf_ref, gam_ref = _oracle(scs)
    sigma, state, mf, gamma, stats = ctx.solve_multi(_blocks(gpu_lib, scs), _opts(gpu_lib, scs))
    s = sigma.cpu().numpy()
    print(f"  image {_rel(s, ref.sigma):.2e}; steps {stats['outer_iters']} oracle {ref.outer_iters}", flush=True)
    assert _rel(mf.cpu().numpy(), mf_ref) <= TOL and _rel(gamma.cpu().numpy(), gam_ref) <= TOL
    np.testing.assert_array_equal(state.cpu().numpy(), ref.state)
    assert _rel(s, ref.sigma) <= TOL

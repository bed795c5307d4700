"""Split half-precision beamforming (CLSIMG_FP16, CLSIMG_BF16) against the
FP64 oracle.

The full-grid products (dirty image, MVDR bound, multipliers of the
host-driven loop) run on the 16x16x32 half-precision MFMA with each operand
split into high and low halves.  FP16 halves carry 22 significant bits
together, so the results must meet the FP32 bar (1e-5); BF16 halves carry
16, so they are held to the reduced-precision bar of 1e-3 (and printed).
Shapes include arrays whose antenna count is not a multiple of 16 (the last
K chunk reads clamped antennas against zero columns) and grids that are not
a multiple of the 16-pixel tiles.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

BAR = {1: 1e-5, 2: 1e-3}  # FP16, BF16
NAME = {1: "fp16", 2: "bf16"}


def _rel(got, ref):
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


def _peak(got, ref):
    return float(np.abs(np.asarray(got, np.float64) - ref).max() / np.abs(ref).max())


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _scene(kind):
    if kind == "p24":
        return synth.make_scene("c0")
    if kind == "p40_ragged":  # 40 antennas (3 K chunks, the last half empty), 37 x 29 pixels
        sc = synth.make_scene("c1", P=40, n=37, seed=11)
        return sc
    if kind == "p48":
        return synth.make_scene("c1")
    if kind == "p104":  # 13 row tiles: 4 per wave, 7 K chunks
        return synth.make_scene("c2", P=104, n=48, seed=12)
    return synth.make_scene("c2", n=64)


def _geo(gpu_lib, sc):
    return gpu_lib.Geometry(sc.pos, sc.lam, sc.grid)


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("kind", ["p24", "p40_ragged", "p48", "p104", "p96"])
def test_dirty_image_and_bound(gpu_lib, ctx, kind, prec):
    sc = _scene(kind)
    print(f"case {NAME[prec]} dirty image / MVDR {kind} P={sc.P} Q={sc.Q}", flush=True)
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    R = sc.R_hat32_c128
    mf_ref = oracle.mf_image(A, R)
    gam_ref = oracle.upper_bound(A, R)
    Rd = torch.as_tensor(sc.R_hat32).cuda()
    mf = ctx.dirty_image(Rd, _geo(gpu_lib, sc), precision=prec).cpu().numpy()
    opts = gpu_lib.default_options()
    opts.precision = prec
    gam = ctx.mvdr_bound(Rd, _geo(gpu_lib, sc), opts).cpu().numpy()
    mf32 = ctx.dirty_image(Rd, _geo(gpu_lib, sc)).cpu().numpy()
    print(f"  mf rel {_rel(mf, mf_ref):.2e} peak {_peak(mf, mf_ref):.2e} (fp32 {_rel(mf32, mf_ref):.2e}); "
          f"gamma rel {_rel(gam, gam_ref):.2e} peak {_peak(gam, gam_ref):.2e}", flush=True)
    for got, ref in ((mf, mf_ref), (gam, gam_ref)):
        assert _rel(got, ref) <= BAR[prec]
        assert _peak(got, ref) <= BAR[prec]


@pytest.mark.parametrize("prec", [1, 2])
def test_full_size_dirty_image_sampled(gpu_lib, ctx, prec):
    # the 288-antenna, 512 x 512 workload: sampled pixels in FP64
    sc = synth.make_scene("c4")
    print(f"case {NAME[prec]} dirty image P=288 Q=512^2 (sampled)", flush=True)
    rng = np.random.default_rng(7)
    pix = np.unique(np.concatenate([[0, sc.Q - 1], rng.choice(sc.Q, size=384, replace=False)]))
    A = oracle.steering(sc.pos, sc.lam, sc.grid, pixels=pix)
    ref = oracle.mf_image(A, sc.R_hat32_c128)
    mf = ctx.dirty_image(torch.as_tensor(sc.R_hat32).cuda(), _geo(gpu_lib, sc), precision=prec).cpu().numpy()[pix]
    print(f"  rel {_rel(mf, ref):.2e} peak {_peak(mf, ref):.2e}", flush=True)
    assert _rel(mf, ref) <= BAR[prec] and _peak(mf, ref) <= BAR[prec]


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("kind", ["p24", "p40_ragged", "p48", "p96"])
def test_solve(gpu_lib, ctx, kind, prec):
    sc = _scene(kind)
    print(f"case {NAME[prec]} solve {kind} P={sc.P} Q={sc.Q}", flush=True)
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    R = sc.R_hat32_c128
    nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
    ref = oracle.solve(A, R - np.diag(nd), oracle.upper_bound(A, R),
                       oracle.detection_threshold(oracle.mf_image(A, R), 6.0, sc.N), atol=1e-8, btol=1e-8)
    opts = gpu_lib.default_options()
    opts.nsamples = sc.N
    opts.atol = opts.btol = 1e-7
    opts.precision = prec
    sigma, state, _, _, stats = ctx.solve(torch.as_tensor(sc.R_hat32).cuda(), _geo(gpu_lib, sc), opts,
                                          noise_diag=torch.as_tensor(nd.astype(np.float32)).cuda())
    s, st = sigma.cpu().numpy(), state.cpu().numpy()
    same = bool(np.array_equal(st, ref.state))
    err = _rel(s, ref.sigma)
    print(f"  same sets {same}; image rel {err:.2e}; residual {stats['rel_residual']:.6f} "
          f"oracle {ref.rel_residual:.6f}; steps {stats['outer_iters']} oracle {ref.outer_iters}", flush=True)
    if prec == 1:
        assert same
    assert err <= BAR[prec]
    assert abs(stats["rel_residual"] - ref.rel_residual) <= BAR[prec] * ref.rel_residual


@pytest.mark.parametrize("kind,prec", [("p48", 0), ("p96", 0), ("p48", 1), ("p104", 2)])
def test_timed_dirty_image_is_the_dirty_image(gpu_lib, ctx, kind, prec):
    # clsimg_dirty_image_timed runs the same kernels (bit-identical image) and
    # binds the two events to the first and last of them
    sc = _scene(kind)
    print(f"case timed dirty image {kind} precision {prec}", flush=True)
    Rd = torch.as_tensor(sc.R_hat32).cuda()
    plain = ctx.dirty_image(Rd, _geo(gpu_lib, sc), precision=prec)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    timed = ctx.dirty_image_timed(Rd, _geo(gpu_lib, sc), e0, e1, precision=prec)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(f"  {ms * 1e3:.2f} us", flush=True)
    assert torch.equal(plain, timed)
    assert 0.0 < ms < 1000.0


@pytest.mark.parametrize("kind,prec", [("p96", 0), ("p104", 1), ("p40_ragged", 2), ("p96", 2)])
def test_every_tile_choice_gives_the_same_image(gpu_lib, ctx, kind, prec):
    # the tile count per workgroup regroups pixels only: the same bits for each
    # choice, and the autotuner keeps one of them
    sc = _scene(kind)
    geo = _geo(gpu_lib, sc)
    print(f"case beamformer tiles {kind} precision {prec}", flush=True)
    Rd = torch.as_tensor(sc.R_hat32).cuda()
    ref = ctx.dirty_image(Rd, geo, precision=prec).clone()
    for tiles in (2, 4, 8):
        ctx.set_beam_tiles(sc.P, prec, tiles)
        assert torch.equal(ctx.dirty_image(Rd, geo, precision=prec), ref), tiles
    chosen, us = ctx.autotune(geo, precision=prec)
    print(f"  kept {chosen} tiles; us per image {us}", flush=True)
    assert chosen in (2, 4, 8) and all(t > 0 for t in us)
    assert us[(2, 4, 8).index(chosen)] == min(us)
    assert torch.equal(ctx.dirty_image(Rd, geo, precision=prec), ref)
    ctx.set_beam_tiles(sc.P, prec, 0)


def test_solve_is_the_same_for_every_tile_choice(gpu_lib, ctx):
    # 96 antennas: the host-driven loop's multipliers use the GEMM-shaped
    # beamformer, whose argmin partition changes with the tile count
    sc = synth.make_scene("c2", n=40, points=(12, ("powerlaw", 0.5, 500.0)))
    geo = _geo(gpu_lib, sc)
    print(f"case solve P={sc.P} Q={sc.Q} for tiles 2 / 8", flush=True)
    Rd = torch.as_tensor(sc.R_hat32).cuda()
    nd = torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()
    o = gpu_lib.default_options()
    o.nsamples = sc.N
    o.atol = o.btol = 1e-7
    out = []
    for tiles in (2, 8):
        ctx.set_beam_tiles(sc.P, 0, tiles)
        s, st, _, _, stats = ctx.solve(Rd, geo, o, noise_diag=nd)
        out.append((s.clone(), st.clone(), stats))
    ctx.set_beam_tiles(sc.P, 0, 0)
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert out[0][2]["outer_iters"] == out[1][2]["outer_iters"]


def test_autotune_rejects(gpu_lib, ctx):
    sc = _scene("p48")
    with pytest.raises(gpu_lib.ClsimgError) as ei:  # register-resident kernel: nothing to tune
        ctx.autotune(_geo(gpu_lib, sc), precision=0)
    assert ei.value.status == gpu_lib.ENOTSUP
    for P, tiles in ((96, 3), (288, 8), (0, 2)):
        with pytest.raises(gpu_lib.ClsimgError) as ei:
            ctx.set_beam_tiles(P, 0, tiles)
        assert ei.value.status == gpu_lib.EINVAL


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("P,n", [(64, 48), (104, 40), (150, 32)])
def test_refined_multipliers_solve_matches_oracle(gpu_lib, ctx, P, n, prec):
    # host-driven loop with half-precision multipliers: the single half
    # product lists the candidates its rounding bound leaves, FP32 decides
    # among them (or, when more than Q/8 are left, FP32 evaluates every pixel
    # of that step): the decisions are the FP32 ones, so the sets are the
    # oracle's and the image meets the FP32 bar
    sc = synth.make_scene("c2", P=P, n=n, seed=300 + P, points=(15, ("powerlaw", 0.5, 500.0)))
    print(f"case refined multipliers {NAME[prec]} P={sc.P} Q={sc.Q}", flush=True)
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    R = sc.R_hat32_c128
    nd = sc.noise_diag.astype(np.float32).astype(np.float64)
    ref = oracle.solve(A, R - np.diag(nd), oracle.upper_bound(A, R),
                       oracle.detection_threshold(oracle.mf_image(A, R), 6.0, sc.N), atol=1e-8, btol=1e-8)
    o = gpu_lib.default_options()
    o.nsamples = sc.N
    o.atol = o.btol = 1e-7
    o.precision = prec
    sigma, state, _, _, stats = ctx.solve(torch.as_tensor(sc.R_hat32).cuda(), _geo(gpu_lib, sc), o,
                                          noise_diag=torch.as_tensor(nd.astype(np.float32)).cuda())
    err = _rel(sigma.cpu().numpy(), ref.sigma)
    print(f"  steps {stats['outer_iters']} / {ref.outer_iters}; image error {err:.3e}", flush=True)
    np.testing.assert_array_equal(state.cpu().numpy(), ref.state)
    assert err <= 1e-5
    assert stats["adds"] == ref.adds and stats["drops"] == ref.drops

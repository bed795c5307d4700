"""Off-grid correction of the free pixels (clsimg_solve_offgrid) against the
oracle's reading of Sec. III-E (eq. doals): same final sets, images, offsets
and residual, on skies whose point sources sit between pixel centres.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import offgrid

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(got, ref):
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _run(gpu_lib, ctx, sc, kind="mvdr", rounds=3, kappa_b=0.0):
    R = sc.R_hat32_c128
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    nd = sc.noise_diag.astype(np.float32).astype(np.float64)
    eps = oracle.detection_threshold(oracle.mf_image(A, R), 6.0, sc.N)
    ref, dref = offgrid.solve_offgrid(sc.pos, sc.lam, sc.grid, R, R - np.diag(nd), eps, kind=kind, rounds=rounds,
                                      kappa_b=kappa_b, nsamples=sc.N)
    o = gpu_lib.default_options()
    o.nsamples = sc.N
    o.atol = o.btol = 1e-7
    o.bound = {"mvdr": gpu_lib.BOUND_MVDR, "mf": gpu_lib.BOUND_MF, "none": gpu_lib.BOUND_NONE}[kind]
    o.kappa_b = kappa_b
    out = ctx.solve_offgrid(torch.as_tensor(sc.R_hat32).cuda(), gpu_lib.Geometry(sc.pos, sc.lam, sc.grid), o,
                            rounds=rounds, noise_diag=torch.as_tensor(nd.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return ref, dref, out


# 64, 72 and 96 antennas on 40 x 40 to 48 x 48 grids with a 25 m array
# (about a beamwidth per pixel): beyond 48 antennas the free set's LSQR runs
# in two kernels per step; c2c detects 36 of
# 40 sources.  (The 96-antenna workload's own 150 m array on such a grid puts
# about 9 beamwidths in a pixel: sources out of the Newton step's reach, and
# solves whose outcome turns on rounding, in the oracle as well.)
_OFFGRID = {
    "c0": ("c0", {}),
    "c1": ("c1", {"points": (25, ("loguniform", 0.5, 50.0))}),
    "c2p": ("c2", {"P": 64, "n": 40, "radius": 25.0, "points": (12, ("loguniform", 0.5, 50.0))}),
    "c2a": ("c2", {"P": 72, "n": 40, "radius": 25.0, "points": (12, ("loguniform", 0.5, 50.0))}),
    "c2b": ("c2", {"P": 96, "n": 48, "radius": 25.0, "points": (12, ("loguniform", 0.5, 50.0))}),
    "c2c": ("c2", {"P": 96, "n": 48, "radius": 25.0, "points": (40, ("loguniform", 2.0, 100.0))}),
}


@pytest.mark.parametrize("cfg,kind", [("c0", "mvdr"), ("c0", "mf"), ("c1", "mvdr"), ("c2p", "mvdr"),
                                      ("c2a", "mvdr"), ("c2b", "mf"), ("c2c", "mvdr")])
def test_offgrid_matches_oracle(gpu_lib, ctx, cfg, kind):
    # the workloads' own grids (about 1.3 beamwidths per pixel); a coarser grid
    # puts sources a beamwidth from every pixel centre, outside the reach of
    # the Newton correction (and of the on-grid model)
    base, ov = _OFFGRID[cfg]
    sc, off = synth.make_offgrid_scene(base, **ov)
    print(f"case offgrid {cfg} P={sc.P} Q={sc.Q} bound {kind}", flush=True)
    ref, dref, (sigma, state, offsets, mf, gamma, stats) = _run(gpu_lib, ctx, sc, kind=kind)
    s, st, d = sigma.cpu().numpy(), state.cpu().numpy(), offsets.cpu().numpy().astype(np.float64)
    F = ref.state == oracle.STATE_F
    dl = sc.dl
    print(f"  steps {stats['outer_iters']} / {ref.outer_iters}; |F| {int(np.sum(st == 1))} / {int(F.sum())}; "
          f"image {_rel(s, ref.sigma):.2e}; offsets max diff {np.abs(d - dref).max() / dl:.2e} px; "
          f"residual {stats['rel_residual']:.6f} / {ref.rel_residual:.6f}", flush=True)
    np.testing.assert_array_equal(st, ref.state)
    assert _rel(s, ref.sigma) <= TOL
    assert np.abs(d - dref).max() <= 1e-4 * dl
    assert abs(stats["rel_residual"] - ref.rel_residual) <= 1e-4 * ref.rel_residual
    assert not np.any(d[~F])


def test_zero_rounds_is_the_on_grid_solve(gpu_lib, ctx):
    sc = synth.make_scene("c0")
    print("case offgrid rounds=0 against clsimg_solve", flush=True)
    _, _, (sigma, state, offsets, _, _, stats) = _run(gpu_lib, ctx, sc, rounds=0)
    o = gpu_lib.default_options()
    o.nsamples = sc.N
    o.atol = o.btol = 1e-7
    nd = torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()
    s0, st0, _, _, _ = ctx.solve(torch.as_tensor(sc.R_hat32).cuda(), gpu_lib.Geometry(sc.pos, sc.lam, sc.grid), o,
                                 noise_diag=nd)
    assert torch.equal(state, st0)
    assert _rel(sigma.cpu().numpy(), s0.cpu().numpy().astype(np.float64)) <= TOL
    assert not offsets.abs().max().item()


def test_offgrid_recovers_positions(gpu_lib, ctx):
    sc, off = synth.make_offgrid_scene("c0")
    print("case offgrid recovery c0", flush=True)
    _, _, (sigma, state, offsets, _, _, stats) = _run(gpu_lib, ctx, sc)
    st = state.cpu().numpy()
    d = offsets.cpu().numpy()
    assert set(np.nonzero(st == 1)[0].tolist()) == set(int(p) for p in sc.src_pix)
    assert np.abs(d[sc.src_pix] - off).max() <= 0.05 * sc.dl


def test_offgrid_rejects(gpu_lib, ctx):
    sc = synth.make_scene("c2", P=104, n=16, seed=12)
    o = gpu_lib.default_options()
    o.nsamples = sc.N
    with pytest.raises(gpu_lib.ClsimgError) as ei:
        ctx.solve_offgrid(torch.as_tensor(sc.R_hat32).cuda(), gpu_lib.Geometry(sc.pos, sc.lam, sc.grid), o)
    assert ei.value.status == gpu_lib.ENOTSUP

"""Batched solves (clsimg_solve_batch): every request of a batch must give
exactly what the same request gives alone, and match the oracle.

Requests differ in data (seed), wavelength and grid size, as frequency
channels or separate observations would; the batch shares the GPU between
them (one outer-step workgroup per request, one multiplier launch for all).
"""

import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def _req(gpu_lib, sc):
    return {"R": _dev(sc.R_hat32, torch.complex64), "geo": gpu_lib.Geometry(sc.pos, sc.lam, sc.grid),
            "noise_diag": _dev(sc.noise_diag, torch.float32)}


def _opts(gpu_lib, sc, cost=0):
    o = gpu_lib.default_options()
    o.nsamples = sc.N
    o.atol = o.btol = 1e-7
    o.cost = cost
    return o


def _scenes(kind):
    if kind == "p48same":
        # one array and grid (snapshots of one observation): the batch reads the
        # steering tables in place; each request has its own covariance
        base = synth.make_scene("c1", seed=200, n=64)
        R = synth.scenes.exact_covariance(base.pos, base.lam, base.grid, base.src_pix, base.src_pow,
                                          base.noise_var)
        return [dataclasses.replace(base, R_hat=synth.scenes._sample_covariance(np.random.default_rng(300 + i), R,
                                                                                base.N))
                for i in range(4)]
    if kind == "p24":
        return [synth.make_scene("c0", seed=100 + i, lam=lam, n=n)
                for i, (lam, n) in enumerate([(1.0, 32), (1.3, 24), (1.7, 40), (1.15, 32), (1.9, 16)])]
    return [synth.make_scene("c1", seed=200 + i, lam=lam, n=n)
            for i, (lam, n) in enumerate([(1.0, 128), (1.4, 64), (1.8, 96)])]


@pytest.mark.parametrize("cost", [0, 1])
@pytest.mark.parametrize("kind", ["p24", "p48", "p48same"])
def test_each_request_in_a_batch_equals_its_solve_alone(gpu_lib, kind, cost):
    scenes = _scenes(kind)
    print(f"case batch of {len(scenes)} ({kind}, cost {cost})", flush=True)
    ctx = gpu_lib.Context(0)
    try:
        opts = _opts(gpu_lib, scenes[0], cost)
        st, res = ctx.solve_batch([_req(gpu_lib, sc) for sc in scenes], opts)
        torch.cuda.synchronize()
        assert st >= 0, st
        for i, sc in enumerate(scenes):
            r = _req(gpu_lib, sc)
            sigma, state, mf, gamma, stats = ctx.solve(r["R"], r["geo"], opts, noise_diag=r["noise_diag"])
            bs, bst, bmf, bg, bstats = res[i]
            print(f"request {i}: alone {stats['adds']} adds {stats['lsqr_iters_total']} LSQR; "
                  f"batch {bstats['adds']} adds {bstats['lsqr_iters_total']} LSQR", flush=True)
            assert torch.equal(state, bst)
            assert torch.equal(sigma, bs)
            assert torch.equal(mf, bmf) and torch.equal(gamma, bg)
            for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU"):
                assert stats[k] == bstats[k], (i, k)
    finally:
        ctx.close()


@pytest.mark.parametrize("variant", ["mvdr_kappa_b", "mvdr_no_noise", "mf_bound", "no_bound"])
def test_batch_bound_variants_equal_their_solves_alone(gpu_lib, variant):
    # the MVDR bound of the least-squares cost takes the batched set-up (with
    # the bound's inflation term, with and without a noise model); the MF
    # bound and no bound keep the per-request set-up
    scenes = _scenes("p24")[:3]
    print(f"case batch bound variant {variant}", flush=True)
    opts = _opts(gpu_lib, scenes[0])
    if variant == "mvdr_kappa_b":
        opts.kappa_b = 3.0
    elif variant == "mf_bound":
        opts.bound, opts.kappa_b = gpu_lib.BOUND_MF, 2.0
    elif variant == "no_bound":
        opts.bound = gpu_lib.BOUND_NONE
    reqs = [_req(gpu_lib, sc) for sc in scenes]
    if variant == "mvdr_no_noise":
        for r in reqs:
            r["noise_diag"] = None
    ctx = gpu_lib.Context(0)
    try:
        st, res = ctx.solve_batch(reqs, opts)
        torch.cuda.synchronize()
        assert st >= 0, st
        for i, r in enumerate(reqs):
            sigma, state, mf, gamma, stats = ctx.solve(r["R"], r["geo"], opts, noise_diag=r["noise_diag"])
            bs, bst, bmf, bg, bstats = res[i]
            print(f"request {i}: alone {stats['adds']} adds, batch {bstats['adds']} adds", flush=True)
            assert torch.equal(mf, bmf) and torch.equal(gamma, bg)
            assert torch.equal(state, bst) and torch.equal(sigma, bs)
            for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU"):
                assert stats[k] == bstats[k], (i, k)
    finally:
        ctx.close()


def test_batch_matches_the_oracle(gpu_lib):
    scenes = _scenes("p24")[:3]
    print("case batch of 3 against the oracle", flush=True)
    ctx = gpu_lib.Context(0)
    try:
        st, res = ctx.solve_batch([_req(gpu_lib, sc) for sc in scenes], _opts(gpu_lib, scenes[0]))
        torch.cuda.synchronize()
    finally:
        ctx.close()
    assert st >= 0
    for i, sc in enumerate(scenes):
        R = sc.R_hat32_c128
        A = oracle.steering(sc.pos, sc.lam, sc.grid)
        mf = oracle.mf_image(A, R)
        nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
        ref = oracle.solve(A, R - np.diag(nd), oracle.upper_bound(A, R),
                           oracle.detection_threshold(mf, 6.0, sc.N))
        sigma, state = res[i][0].cpu().numpy(), res[i][1].cpu().numpy()
        np.testing.assert_array_equal(state, ref.state)
        err = np.linalg.norm(sigma - ref.sigma) / max(np.linalg.norm(ref.sigma), 1e-30)
        print(f"request {i}: rel image error {err:.2e}; residual {res[i][4]['rel_residual']:.6f} "
              f"oracle {ref.rel_residual:.6f}", flush=True)
        assert err <= 1e-5
        assert abs(res[i][4]["rel_residual"] - ref.rel_residual) <= 1e-5 * ref.rel_residual + 1e-7


def test_batch_of_mixed_array_sizes_equals_solves_alone(gpu_lib):
    # 24, 48 and 96 antennas in one call: one batch per size (the first two on
    # the device together, the 96-antenna request on the host-driven loop)
    scenes = [synth.make_scene("c0", seed=610), synth.make_scene("c1", seed=611, n=32),
              synth.make_scene("c0", seed=612, lam=1.3), synth.make_scene("c2", seed=613, n=24,
                                                                          points=(8, ("powerlaw", 0.5, 500.0)))]
    print(f"case batch of mixed sizes {[sc.P for sc in scenes]}", flush=True)
    ctx = gpu_lib.Context(0)
    try:
        _batch_equals_alone(gpu_lib, ctx, scenes, _opts(gpu_lib, scenes[0]))
    finally:
        ctx.close()


def _batch_equals_alone(gpu_lib, ctx, scenes, opts):
    st, res = ctx.solve_batch([_req(gpu_lib, sc) for sc in scenes], opts)
    torch.cuda.synchronize()
    assert st >= 0, st
    for i, sc in enumerate(scenes):
        r = _req(gpu_lib, sc)
        sigma, state, mf, gamma, stats = ctx.solve(r["R"], r["geo"], opts, noise_diag=r["noise_diag"])
        bs, bst, bmf, bg, bstats = res[i]
        print(f"request {i}: alone {stats['adds']} adds nF {stats['nF']}; batch {bstats['adds']} adds "
              f"nF {bstats['nF']}", flush=True)
        assert torch.equal(state, bst) and torch.equal(sigma, bs)
        assert torch.equal(mf, bmf) and torch.equal(gamma, bg)
        for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU"):
            assert stats[k] == bstats[k], (i, k)
    return res


@pytest.mark.parametrize("cost", [0, 1])
def test_batch_beyond_48_antennas_equals_solves_alone(gpu_lib, cost):
    # 96 antennas: the requests run one after another on the host-driven loop
    scenes = [synth.make_scene("c2", seed=500 + i, n=n, points=(12, ("powerlaw", 0.5, 500.0)))
              for i, n in enumerate([24, 32])]
    print(f"case batch of {len(scenes)} at P=96 (cost {cost})", flush=True)
    ctx = gpu_lib.Context(0)
    try:
        res = _batch_equals_alone(gpu_lib, ctx, scenes, _opts(gpu_lib, scenes[0], cost))
        assert all(r[4]["adds"] > 0 for r in res)
    finally:
        ctx.close()


def test_batch_hands_large_free_sets_to_solves_alone(gpu_lib):
    # a free set past hand_over_free leaves the device loop: that request is
    # solved again alone (its device loop hands it to the host loop at the same
    # step); the others keep their batched results
    scenes = _scenes("p48") + [synth.make_scene("c1", seed=210, n=32, points=(3, ("uniform", 20.0, 50.0)),
                                                blobs=(0, 6.0, 0.0))]
    print(f"case batch of {len(scenes)} (P=48) with hand_over_free 12", flush=True)
    ctx = gpu_lib.Context(0)
    try:
        opts = _opts(gpu_lib, scenes[0])
        opts.hand_over_free = 12
        res = _batch_equals_alone(gpu_lib, ctx, scenes, opts)
        nF = [r[4]["nF"] for r in res]
        assert max(nF) > 12 and min(nF) <= 12, nF
    finally:
        ctx.close()


def test_batch_reports_a_covariance_that_is_not_positive_definite(gpu_lib):
    # the batched factorisation checks every request's covariance before any
    # request is set up; a negative-definite one fails the call with ENOTPD
    scs = [synth.make_scene("c0", seed=300 + i) for i in range(3)]
    reqs = [_req(gpu_lib, sc) for sc in scs]
    reqs[1]["R"] = -reqs[1]["R"]
    ctx = gpu_lib.Context(0)
    try:
        print("case batch with a non-PD covariance", flush=True)
        with pytest.raises(gpu_lib.ClsimgError) as ei:
            ctx.solve_batch(reqs, _opts(gpu_lib, scs[0]))
        assert ei.value.status == gpu_lib.ENOTPD
        # the context stays usable: the valid requests solve, as alone
        st, res = ctx.solve_batch([reqs[0], reqs[2]], _opts(gpu_lib, scs[0]))
        assert st >= 0
        s0, st0, _, _, _ = ctx.solve(reqs[0]["R"], reqs[0]["geo"], _opts(gpu_lib, scs[0]),
                                     noise_diag=reqs[0]["noise_diag"])
        assert torch.equal(res[0][1], st0) and torch.equal(res[0][0], s0)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_half_precision_batch(gpu_lib, prec):
    # the batch at FP16 / BF16 (the dirty images and bounds of the set-up in
    # split half precision): each request equals its solve alone; FP16 also
    # meets the FP32 bar against the oracle with the same sets
    scenes = _scenes("p24")[:4] + _scenes("p48")[:1]
    scenes = [sc for sc in scenes if sc.P == scenes[0].P]
    print(f"case batch precision {prec}: {len(scenes)} requests", flush=True)
    ctx = gpu_lib.Context(0)
    try:
        opts = _opts(gpu_lib, scenes[0])
        opts.precision = prec
        st, res = ctx.solve_batch([_req(gpu_lib, sc) for sc in scenes], opts)
        torch.cuda.synchronize()
        assert st >= 0, st
        for i, sc in enumerate(scenes):
            r = _req(gpu_lib, sc)
            sigma, state, mf, gamma, stats = ctx.solve(r["R"], r["geo"], opts, noise_diag=r["noise_diag"])
            bs, bst = res[i][0], res[i][1]
            assert torch.equal(state, bst) and torch.equal(sigma, bs), i
            if prec == 1:
                R = sc.R_hat32_c128
                A = oracle.steering(sc.pos, sc.lam, sc.grid)
                nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
                ref = oracle.solve(A, R - np.diag(nd), oracle.upper_bound(A, R),
                                   oracle.detection_threshold(oracle.mf_image(A, R), 6.0, sc.N), atol=1e-8,
                                   btol=1e-8)
                err = float(np.linalg.norm(sigma.cpu().numpy() - ref.sigma) / np.linalg.norm(ref.sigma))
                print(f"  request {i}: image error {err:.2e}", flush=True)
                np.testing.assert_array_equal(state.cpu().numpy(), ref.state)
                assert err <= 1e-5
    finally:
        ctx.close()


@pytest.mark.parametrize("kind", ["p24", "p48"])
def test_captured_rounds_equal_enqueued_rounds(gpu_lib, kind):
    # the batched steps replayed from a captured graph (batch_graph = 1) give
    # the results of the launches enqueued one by one; two calls in a row reuse
    # the graph (every replay with the program's own read-backs in between),
    # a third call with another batch size captures it again
    scenes = _scenes(kind)
    print(f"case batch of {len(scenes)} ({kind}) replayed from a graph", flush=True)
    ctx = gpu_lib.Context(0)
    try:
        opts = _opts(gpu_lib, scenes[0])
        st, eager = ctx.solve_batch([_req(gpu_lib, sc) for sc in scenes], opts)
        torch.cuda.synchronize()
        assert st >= 0, st
        opts.batch_graph = 1
        for call, subset in enumerate([len(scenes), len(scenes), len(scenes) - 1]):
            st, res = ctx.solve_batch([_req(gpu_lib, sc) for sc in scenes[:subset]], opts)
            torch.cuda.synchronize()
            assert st >= 0, st
            for i in range(subset):
                es, est, emf, eg, estats = eager[i]
                bs, bst, bmf, bg, bstats = res[i]
                assert torch.equal(est, bst) and torch.equal(es, bs), (call, i)
                for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU", "rel_residual"):
                    assert estats[k] == bstats[k], (call, i, k)
            print(f"call {call}: {subset} requests equal", flush=True)
    finally:
        ctx.close()

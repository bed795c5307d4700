"""The continuous-batching server (clsimg_server_*): requests of mixed array
sizes, wavelengths and grids arrive while others run; each result must be the
same as the request solved alone with clsimg_solve.

Arrivals are staggered (submit, run some steps, submit more) so that requests
join slots freed by finished ones; a small HBM budget forces admission to wait
for arena space; requests with 96 antennas go to the worker streams.
"""

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


def _opts(gpu_lib, cost=0):
    o = gpu_lib.default_options()
    o.nsamples = 16384
    o.atol = o.btol = 1e-7
    o.cost = cost
    return o


def _mixed_scenes(with_large=True):
    # P in {24, 48}, grids 32^2 / 64^2, lambda in [1, 2), 10..200 point sources
    out = synth.make_request_scenes(10, P_choices=(24, 48), n_choices=(32, 64))
    if with_large:  # 96 antennas: the workers'
        out.insert(3, synth.make_scene("c2", n=32, seed=777))
        out.insert(6, synth.make_scene("c2", n=48, seed=778))
    return out


def _alone(gpu_lib, scenes, opts):
    ctx = gpu_lib.Context(0)
    try:
        res = []
        for sc in scenes:
            r = _req(gpu_lib, sc)
            res.append(ctx.solve(r["R"], r["geo"], opts, noise_diag=r["noise_diag"]))
        torch.cuda.synchronize()
        return res
    finally:
        ctx.close()


def _same(alone, served, i):
    sigma, state, mf, gamma, stats = alone
    bs, bst, bmf, bg, bstats = served
    print(f"request {i}: alone {stats['status']} {stats['outer_iters']} steps {stats['lsqr_iters_total']} LSQR; "
          f"served {bstats['status']} {bstats['outer_iters']} steps {bstats['lsqr_iters_total']} LSQR", flush=True)
    assert torch.equal(state, bst), i
    assert torch.equal(sigma, bs), i
    assert torch.equal(mf, bmf) and torch.equal(gamma, bg), i
    for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU"):
        assert stats[k] == bstats[k], (i, k)


def _serve(gpu_lib, scenes, opts, **kw):
    srv = gpu_lib.Server(opts, **kw)
    got, tickets = {}, []
    try:
        half = len(scenes) // 2
        for sc in scenes[:half]:
            tickets.append(srv.submit(_req(gpu_lib, sc)))
        for _ in range(3):  # some steps before the rest arrive
            for t, r in srv.poll():
                got[t] = r
        first = srv.info()
        for sc in scenes[half:]:
            tickets.append(srv.submit(_req(gpu_lib, sc)))
        waited = 0  # most requests left waiting after an admission pass
        while len(got) < len(scenes):
            done = srv.poll(wait=True)
            assert done, "server idle with requests outstanding"
            for t, r in done:
                got[t] = r
            waited = max(waited, srv.info()["pending"])
        info = srv.info()
        info["after_first_polls"] = first
        info["max_waiting"] = waited
    finally:
        srv.close()
    return [got[t] for t in tickets], info


def test_mixed_requests_equal_their_solves_alone(gpu_lib):
    scenes = _mixed_scenes()
    print("case server: mixed P 24/48 and two 96, staggered arrivals, two workers", flush=True)
    opts = _opts(gpu_lib)
    served, info = _serve(gpu_lib, scenes, opts, max_slots=8, steps_per_poll=8, workers=2)
    print("server info", info, flush=True)
    assert info["submitted"] == len(scenes) and info["completed"] == len(scenes)
    assert info["admitted"] == len(scenes) - 2  # the 96-antenna requests went to the workers
    alone = _alone(gpu_lib, scenes, opts)
    for i in range(len(scenes)):
        _same(alone[i], served[i], i)


def test_admission_waits_for_arena_space(gpu_lib):
    scenes = _mixed_scenes(with_large=False)[:6]
    print("case server: arena for about two requests", flush=True)
    opts = _opts(gpu_lib)
    budget = 640 * 1024
    served, info = _serve(gpu_lib, scenes, opts, max_slots=64, hbm_budget=budget, steps_per_poll=4)
    print("server info", info, flush=True)
    assert info["arena_peak"] <= budget and info["admitted"] == len(scenes)
    assert info["max_waiting"] > 0  # some requests had to wait for arena space
    alone = _alone(gpu_lib, scenes, opts)
    for i in range(len(scenes)):
        _same(alone[i], served[i], i)


def test_pwls_requests_equal_their_solves_alone(gpu_lib):
    # device slots for 24 and 48 antennas, a worker for the 96-antenna request
    scenes = _mixed_scenes(with_large=False)[:4]
    scenes.insert(2, synth.make_scene("c2", n=24, seed=779, points=(8, ("powerlaw", 0.5, 500.0))))
    print("case server: PWLS cost", flush=True)
    opts = _opts(gpu_lib, cost=1)
    served, info = _serve(gpu_lib, scenes, opts, max_slots=4, workers=1)
    assert info["admitted"] == len(scenes) - 1
    alone = _alone(gpu_lib, scenes, opts)
    for i in range(len(scenes)):
        _same(alone[i], served[i], i)


def test_handover_beyond_the_device_capacity(gpu_lib):
    # a tiny free-set capacity makes every device slot hand its request to the worker
    scenes = _mixed_scenes(with_large=False)[:3]
    print("case server: free-set capacity 3 (hand-over to the worker)", flush=True)
    opts = _opts(gpu_lib)
    opts.hand_over_free = 3
    served, info = _serve(gpu_lib, scenes, opts, max_slots=4)
    print("server info", info, flush=True)
    alone = _alone(gpu_lib, scenes, opts)
    for i in range(len(scenes)):
        assert alone[i][4]["nF"] > 3  # the hand-over really happened
        _same(alone[i], served[i], i)


def test_served_request_matches_the_oracle(gpu_lib):
    sc = _mixed_scenes(with_large=False)[0]
    print("case server: one request against the oracle", flush=True)
    (res,), _ = _serve(gpu_lib, [sc], _opts(gpu_lib), max_slots=2)
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    R = sc.R_hat32_c128
    nd = np.asarray(sc.noise_diag, np.float32).astype(np.float64)
    ref = oracle.solve(A, R - np.diag(nd), oracle.upper_bound(A, R),
                       oracle.detection_threshold(oracle.mf_image(A, R), 6.0, sc.N))
    np.testing.assert_array_equal(res[1].cpu().numpy(), ref.state)
    s = res[0].cpu().numpy()
    assert np.linalg.norm(s - ref.sigma) <= 1e-5 * np.linalg.norm(ref.sigma)


def test_server_rejects_bad_requests(gpu_lib):
    srv = gpu_lib.Server(_opts(gpu_lib), max_slots=2)
    try:
        sc = synth.make_scene("c0")
        r = _req(gpu_lib, sc)
        with pytest.raises(ValueError):
            srv.submit({"R": r["R"][:10], "geo": r["geo"]})
        assert srv.poll() == []
        assert srv.info()["submitted"] == 0
    finally:
        srv.close()

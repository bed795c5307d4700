"""Benchmark: constrained-LS image formation on one MI355X.

Default run (the JSON line the driver records): the largest single-GPU
workload, 288 antennas uniform in a disc of radius 400 lambda, 512 x 512
pixels over |l|, |m| <= 0.7, 1000 point sources (S^-1.5 on [1, 1000]) plus
ten Gaussian blobs (FWHM 6 px), white noise variance 100, covariance from
2^18 complex-Gaussian samples.  One step is the first ten Table I steps of
the active-set solve over that covariance, already resident in HBM: steering
tables, MF dirty image, FP64-Cholesky MVDR bound, threshold, then ten
subproblem / gradient / release steps (each feasible step a full-grid
gradient of 8 P^2 Q = 174 GFLOP).  The complete solve takes about a thousand
such steps, far beyond a bounded run, so the first ten are timed and checked
against the oracle's first ten.  value = dense-count Psi / Psi^H TFLOP/s of
those steps; the roofline is taken on the kernel that dominates them, the
full-grid beamformer (gradient, dirty image, bound).

Beside it, as extra keys: the 48-antenna, 128 x 128 workload's complete
solves (solves/s, p50/p99, oracle parity, time per LSQR iteration), its
batched calls, the serving mix of 24/48/96-antenna requests (solves/s,
p50/p99 against one solve at a time), the full-grid operators at 288
antennas in every precision with executed-MFMA fractions, the oracle on the
host cores (CPU model, threads, and the 24-antenna workload on one thread).

--config c0|c1|c2|c4 runs one workload's complete solves instead (value =
solves/s), with the options below; --serve, --offgrid, --blocks, --batch and
--kernel-only select the other measurements.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("Ψ/Ψᴴ TFLOP/s + % MFMA peak; imaging solves/s and p50/p99 latency at "
          "fixed residual")
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HALF_MFMA_TFLOPS = 2516.6  # FP16 / BF16 dense
PRECISIONS = {"fp32": 0, "fp16": 1, "bf16": 2}
WORKLOADS = {
    "c0": "P=24 random planar array (radius 20 lambda), Q=32x32 over |l|,|m|<=0.5, 5 point sources "
          "U[1,10], noise 1, N=4096 samples",
    "c1": "P=48 random planar array (radius 60 lambda), Q=128x128 over |l|,|m|<=0.7, 40 point sources "
          "log-U[0.1,100] + 2 Gaussian blobs FWHM 6 px, noise 10, N=16384 samples",
    "c2": "P=96 random planar array (radius 150 lambda), Q=256x256 over |l|,|m|<=0.7, 200 point "
          "sources S^-1.5 on [0.5,500], noise 50, N=65536 samples",
    "c4": "P=288 random planar array (radius 400 lambda), Q=512x512 over |l|,|m|<=0.7, 1000 point "
          "sources S^-1.5 on [1,1000] + 10 Gaussian blobs FWHM 6 px, noise 100, N=262144 samples",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20 for the headline, 100 for --config)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 3 / 10)")
    ap.add_argument("--config", default="headline", choices=["headline"] + sorted(WORKLOADS))
    ap.add_argument("--max-outer", type=int, default=-1,
                    help="stop every solve (GPU and oracle) after this many Table I steps: the "
                         "288-antenna workload is measured on its first steps")
    ap.add_argument("--tol", type=float, default=1e-7, help="LSQR atol = btol")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--bound", default="mvdr", choices=["mvdr", "mf", "none"],
                    help="upper bound of the box (Sec. II-D)")
    ap.add_argument("--kappa-b", type=float, default=0.0, help="bound inflation in std units (App. A)")
    ap.add_argument("--precision", default=None, choices=["fp32", "fp16", "bf16"],
                    help="FP32, or FP16 / BF16 on the half-precision MFMA: split halves (dirty image, bound) "
                         "and one half product with the decision refined in FP32 (multipliers of the "
                         "host-driven loop).  Default: fp16 for the headline (the FP32 plain path is timed "
                         "beside it), fp32 for --config")
    ap.add_argument("--cost", default="ls", choices=["ls", "pwls"],
                    help="cost function: LS (eq. CLS) or preconditioned weighted LS (eq. preWLS)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 288-antenna full-grid beamformer timing")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only launch the beamformer (20 times) and a plain copy of --copy-mib MiB "
                         "(3 times): the program the HBM traffic counters are read on")
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--blocks", type=int, default=1,
                    help="snapshots per solve (array rotated 0.05 rad between them); with --channels, "
                         "blocks x channels covariance blocks of one sky (clsimg_solve_multi)")
    ap.add_argument("--channels", type=int, default=1, help="frequency channels (wavelength 1, 1.1, ...)")
    ap.add_argument("--offgrid", type=int, default=-1, metavar="ROUNDS",
                    help="off-grid correction benchmark (Sec. III-E): the workload's sources moved off their "
                         "pixel centres, solved with ROUNDS Gauss-Newton rounds per subproblem")
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="serving benchmark instead: N mixed requests (24/48/96 antennas, 64^2..256^2 "
                         "pixels) through the continuous-batching server, against one solve at a time")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=16, help="Table I steps per server poll")
    ap.add_argument("--serve-workers", type=int, default=8, help="server threads for P > 48 requests")
    ap.add_argument("--batched-extra", type=str, default="16,256",
                    help="after the timed solves, also time batched calls of these numbers of requests of "
                         "the workload, comma separated (reported under 'batched'; 0 = skip)")
    ap.add_argument("--serve-default", type=int, default=64, metavar="N",
                    help="requests of the serving mix measured beside the headline (0 = skip)")
    ap.add_argument("--no-poisson", action="store_true", help="headline serving leg: all requests at once only")
    ap.add_argument("--batch", type=int, default=1,
                    help="solve B independent requests of the workload per step (one batched call); "
                         "request 0 is the workload itself, the others redraw its sky and samples")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "beam_kernel_mf_c1_traffic.md")
BEAM_SOURCE = os.path.join(ROOT, "paper_1505_01348_amd", "csrc", "beam.hip")


def stamped_seconds(call, reps):
    """Mean device time of `call(start, stop)`, a library call that binds the two
    timing events to its first and last kernel (the GPU's own timestamps)."""
    import numpy as np
    import torch

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        call(a, b)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3


def measured_traffic():
    """HBM bytes per launch of the beamformer from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(BEAM_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_json: "):
            rec = json.loads(line[len("traffic_json: "):])
            if rec.get("beam_hip_sha256") == src:
                return rec.get("hbm_bytes_per_launch")
    return None


def cpu_baseline(sc, tol_oracle, budget_s=25.0, cost="ls", bound="mvdr", kappa_b=0.0, max_outer=-1):
    """Time oracle solves of the same workload on the host (bounded sample)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle
    R = sc.R_hat32_c128
    nd = sc.noise_diag.astype(np.float32).astype(np.float64)
    runs, t_total, res = 0, 0.0, None
    while True:
        t0 = time.perf_counter()
        A = oracle.steering(sc.pos, sc.lam, sc.grid)
        mf = oracle.mf_image(A, R)
        gamma = oracle.upper_bound(A, R, kind=bound, kappa_b=kappa_b, nsamples=sc.N)
        if cost == "pwls":
            _, h = oracle.pwls_scaling(A, R)
            eps = oracle.pwls_threshold(h, 6.0, sc.N, sc.P)
            res = oracle.solve_pwls(A, R, R - np.diag(nd), gamma, eps, atol=tol_oracle, btol=tol_oracle,
                                    max_outer=max_outer)
        else:
            eps = oracle.detection_threshold(mf, 6.0, sc.N)
            res = oracle.solve(A, R - np.diag(nd), gamma, eps, atol=tol_oracle, btol=tol_oracle,
                               max_outer=max_outer)
        t_total += time.perf_counter() - t0
        runs += 1
        log(f"cpu baseline: oracle solve {runs} done, {t_total:.1f} s")
        if t_total >= budget_s * 0.4 or runs >= 30:
            break
    threads = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
    cores = max(threads) if threads else 1
    what = "full" if max_outer < 0 else f"first-{max_outer}-step"
    return {"value": runs / t_total, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{runs} {what} FP64 oracle solves of the same workload ({t_total:.1f} s)"}, res


def offgrid_bench(args, clsimg, synth, np, torch):
    """The workload's point sources moved off their pixel centres by up to
    0.45 pixel (no extended blobs); clsimg_solve_offgrid against the oracle's
    reading of Sec. III-E, and the on-grid solve of the same data."""
    sc, off = synth.make_offgrid_scene(args.config)
    log(f"bench: off-grid {args.config} P={sc.P} Q={sc.Q} sources={len(sc.src_pix)} rounds={args.offgrid}")
    opts = clsimg.default_options()
    opts.nsamples = sc.N
    opts.atol = opts.btol = args.tol
    opts.bound = {"mvdr": clsimg.BOUND_MVDR, "mf": clsimg.BOUND_MF, "none": clsimg.BOUND_NONE}[args.bound]
    opts.kappa_b = args.kappa_b
    R = torch.as_tensor(sc.R_hat32).cuda()
    nd = torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()
    geo = clsimg.Geometry(sc.pos, sc.lam, sc.grid)
    ctx = clsimg.Context(0)
    out = None
    for _ in range(args.warmup):
        out = ctx.solve_offgrid(R, geo, opts, rounds=args.offgrid, noise_diag=nd)
        torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        out = ctx.solve_offgrid(R, geo, opts, rounds=args.offgrid, noise_diag=nd)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    total = time.perf_counter() - t_start
    sigma, state, offsets, _, _, stats = out
    on = ctx.solve(R, geo, opts, noise_diag=nd)[4]
    torch.cuda.synchronize()
    st = state.cpu().numpy()
    d = offsets.cpu().numpy().astype(np.float64)
    free_src = [int(p) for p in sc.src_pix if st[p] == 1]
    err = [float(np.abs(d[p] - o).max() / sc.dl) for p, o in zip(sc.src_pix, off) if st[p] == 1]
    lat_ms = np.array(lat) * 1e3
    result = {
        "metric": METRIC + " (off-grid correction, Sec. III-E)",
        "value": round(args.steps / total, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FP64 phases and Gauss-Newton scalars)",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}; point sources moved up to 0.45 pixel "
                               "off their centres, no extended blobs", "rounds": args.offgrid,
                   "bound": args.bound, "lsqr_tol": args.tol},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 4), "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
        "solve": {k: stats[k] for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU",
                                        "rel_residual")},
        "sources_free": f"{len(free_src)} of {len(sc.src_pix)}",
        "offset_error_px_max": round(max(err), 4) if err else None,
        "on_grid_solve": {"nF": on["nF"], "nU": on["nU"], "rel_residual": on["rel_residual"]},
    }
    if not args.no_cpu:
        from threadpoolctl import threadpool_info

        import oracle
        from oracle import offgrid
        Rr = sc.R_hat32_c128
        ndd = sc.noise_diag.astype(np.float32).astype(np.float64)
        runs, t_total, ref = 0, 0.0, None
        while True:
            t0 = time.perf_counter()
            A = oracle.steering(sc.pos, sc.lam, sc.grid)
            eps = oracle.detection_threshold(oracle.mf_image(A, Rr), 6.0, sc.N)
            ref, dref = offgrid.solve_offgrid(sc.pos, sc.lam, sc.grid, Rr, Rr - np.diag(ndd), eps, kind=args.bound,
                                              kappa_b=args.kappa_b, nsamples=sc.N, rounds=args.offgrid)
            t_total += time.perf_counter() - t0
            runs += 1
            log(f"cpu baseline: oracle solve {runs} done, {t_total:.1f} s")
            if t_total >= 10.0 or runs >= 30:
                break
        threads = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        result["cpu_baseline"] = {"value": runs / t_total, "unit": "solves/s", "cores": int(max(threads) if threads else 1),
                                  "kind": "oracle", "sample": f"{runs} FP64 oracle off-grid solves ({t_total:.1f} s)"}
        s = sigma.cpu().numpy().astype(np.float64)
        result["parity"] = {"rel_image_err": float(np.linalg.norm(s - ref.sigma) / np.linalg.norm(ref.sigma)),
                            "same_sets": bool(np.array_equal(st, ref.state)),
                            "offsets_max_diff_px": float(np.abs(d - dref).max() / sc.dl),
                            "oracle_rel_residual": ref.rel_residual}
    ctx.close()
    print(json.dumps(result), flush=True)


def multi_bench(args, clsimg, synth, np, torch):
    """K = blocks x channels covariance blocks of one sky on the workload's grid
    (eq. vectRtotal): snapshot k sees the array rotated by 0.05 k rad, channel c
    the wavelength 1 + 0.1 c; each block has its own N samples."""
    nb, nc = max(1, args.blocks), max(1, args.channels)
    angles = [0.05 * k for c in range(nc) for k in range(nb)]
    lams = [1.0 + 0.1 * c for c in range(nc) for k in range(nb)]
    K = nb * nc
    scs = synth.make_block_scenes(args.config, K=K, angles=angles, lams=lams)
    sc0 = scs[0]
    log(f"bench: {K} blocks ({nb} snapshots x {nc} channels) of {args.config} P={sc0.P} Q={sc0.Q}")
    opts = clsimg.default_options()
    opts.nsamples = sc0.N
    opts.atol = opts.btol = args.tol
    opts.bound = {"mvdr": clsimg.BOUND_MVDR, "mf": clsimg.BOUND_MF, "none": clsimg.BOUND_NONE}[args.bound]
    opts.kappa_b = args.kappa_b
    opts.precision = PRECISIONS[args.precision]
    opts.max_outer = args.max_outer
    blocks = [{"R": torch.as_tensor(sc.R_hat32).cuda(), "geo": clsimg.Geometry(sc.pos, sc.lam, sc.grid),
               "noise_diag": torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()} for sc in scs]
    ctx = clsimg.Context(0)
    out = None
    for i in range(args.warmup):
        out = ctx.solve_multi(blocks, opts)
        torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        out = ctx.solve_multi(blocks, opts)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    total = time.perf_counter() - t_start
    stats = out[4]
    log(f"bench: {args.steps} solves of {K} blocks in {total:.3f} s; stats {stats}")
    lat_ms = np.array(lat) * 1e3
    result = {
        "metric": METRIC + " (K covariance blocks per solve)",
        "value": round(args.steps / total, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16 split halves + f32", "bf16": "bf16 split halves + f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}; {nb} snapshots (array rotated 0.05 rad "
                               f"apart) x {nc} channels (wavelength 1, 1.1, ...), own samples per block",
                   "blocks": K, "bound": args.bound, "precision": args.precision, "lsqr_tol": args.tol,
                   "max_outer": args.max_outer},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 4), "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
        "psi_tflops": round(stats["psi_flops"] * args.steps / total / 1e12, 4),
        "solve": {k: stats[k] for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU",
                                        "rel_residual")},
    }
    if not args.no_cpu:
        from threadpoolctl import threadpool_info

        import oracle
        As = oracle.steering_blocks([(sc.pos, sc.lam) for sc in scs], sc0.grid)
        Rs = [sc.R_hat32_c128 for sc in scs]
        runs, t_total, ref = 0, 0.0, None
        while True:
            t0 = time.perf_counter()
            gamma = oracle.upper_bound_multi(As, Rs, kind=args.bound, kappa_b=args.kappa_b, nsamples=sc0.N)
            eps = oracle.detection_threshold_multi(As, Rs, 6.0, sc0.N)
            B0s = [R - np.diag(sc.noise_diag.astype(np.float32).astype(np.float64)) for R, sc in zip(Rs, scs)]
            ref = oracle.solve_multi(As, B0s, gamma, eps, atol=1e-8, btol=1e-8, max_outer=args.max_outer)
            t_total += time.perf_counter() - t0
            runs += 1
            log(f"cpu baseline: oracle solve {runs} done, {t_total:.1f} s")
            if t_total >= 10.0 or runs >= 30:
                break
        threads = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        result["cpu_baseline"] = {"value": runs / t_total, "unit": "solves/s", "cores": int(max(threads) if threads else 1),
                                  "kind": "oracle", "sample": f"{runs} FP64 oracle solves of the same {K} blocks "
                                                              f"({t_total:.1f} s)"}
        s = out[0].cpu().numpy().astype(np.float64)
        result["parity"] = {"rel_image_err": float(np.linalg.norm(s - ref.sigma) / np.linalg.norm(ref.sigma)),
                            "same_sets": bool(np.array_equal(out[1].cpu().numpy(), ref.state)),
                            "oracle_rel_residual": ref.rel_residual}
    ctx.close()
    print(json.dumps(result), flush=True)


def serve_bench(args, clsimg, synth, np, torch):
    """Mixed requests (one frequency channel each): P uniform in {24, 48, 96}, grid
    uniform in {64^2, 128^2, 256^2} over |l|,|m| <= 0.7, 10..200 point sources
    log-uniform in [0.1, 100], lambda uniform in [1, 2), noise 10, N = 16384."""
    n = args.serve
    scenes = synth.make_request_scenes(n)
    opts = clsimg.default_options()
    opts.nsamples = 16384
    opts.atol = opts.btol = args.tol
    reqs = [{"R": torch.as_tensor(sc.R_hat32).cuda(), "geo": clsimg.Geometry(sc.pos, sc.lam, sc.grid),
             "noise_diag": torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()} for sc in scenes]
    torch.cuda.synchronize()
    mix = {}
    for sc in scenes:
        key = f"P{sc.P}_{sc.nl}x{sc.nm}"
        mix[key] = mix.get(key, 0) + 1
    log(f"bench: {n} requests, mix {mix}")

    # the plain per-solve path: one clsimg_solve after another
    ctx = clsimg.Context(0)
    for rq in reqs[:2]:  # warm-up (module load, first allocations)
        ctx.solve(rq["R"], rq["geo"], opts, noise_diag=rq["noise_diag"])
    torch.cuda.synchronize()
    alone, lat1 = [], []
    t0 = time.perf_counter()
    for i, rq in enumerate(reqs):
        ts = time.perf_counter()
        alone.append(ctx.solve(rq["R"], rq["geo"], opts, noise_diag=rq["noise_diag"])[4])
        torch.cuda.synchronize()
        lat1.append(time.perf_counter() - ts)
    t_seq = time.perf_counter() - t0
    ctx.close()
    rate1 = n / t_seq
    log(f"bench: one solve at a time: {rate1:.2f} solves/s ({t_seq:.2f} s)")

    def run(arrivals):
        srv = clsimg.Server(opts, max_slots=args.serve_slots, hbm_budget=4 << 30, steps_per_poll=args.serve_steps,
                            workers=args.serve_workers)
        order = sorted(range(n), key=lambda i: arrivals[i])
        ticket_of, done_at, stats = {}, {}, {}
        k = 0
        t_start = time.perf_counter()
        while len(done_at) < n:
            now = time.perf_counter() - t_start
            while k < n and arrivals[order[k]] <= now:
                i = order[k]
                ticket_of[srv.submit(reqs[i])] = i
                k += 1
            info = srv.info()
            busy = info["pending"] + info["active"] + info["worker_queued"] + info["ready"] > 0
            if not busy:
                if k < n:
                    time.sleep(max(0.0, arrivals[order[k]] - (time.perf_counter() - t_start)))
                continue
            for t, r in srv.poll(wait=(k == n)):
                i = ticket_of[t]
                done_at[i] = time.perf_counter() - t_start
                stats[i] = r[4]
        total = time.perf_counter() - t_start
        peak = srv.info()["arena_peak"]
        srv.close()
        lat = np.array([done_at[i] - arrivals[i] for i in range(n)]) * 1e3
        same = all(stats[i]["rel_residual"] == alone[i]["rel_residual"] and
                   stats[i]["lsqr_iters_total"] == alone[i]["lsqr_iters_total"] for i in range(n))
        return {"solves_per_s": round(n / total, 3), "wall_s": round(total, 3),
                "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "arena_peak_bytes": int(peak), "same_result_as_alone": bool(same)}

    closed = run([0.0] * n)
    log(f"bench: server, all {n} at once: {closed}")
    rng = np.random.default_rng(20150504)
    sweep = {}
    for f in (0.5, 1.0, 2.0):
        qps = f * rate1
        arr = np.cumsum(rng.exponential(1.0 / qps, size=n))
        arr -= arr[0]
        sweep[f"{f}x"] = dict(run(list(arr)), qps=round(qps, 3))
        log(f"bench: server, Poisson arrivals at {qps:.2f}/s: {sweep[f'{f}x']}")
    lat1 = np.array(lat1) * 1e3
    by_class = {}
    for sc, t in zip(scenes, lat1):
        by_class.setdefault(f"P{sc.P}_{sc.nl}x{sc.nm}", []).append(float(t))
    by_class = {k: round(float(np.mean(v)), 2) for k, v in sorted(by_class.items())}
    result = {
        "metric": "imaging solves/s and p50/p99 latency, mixed requests (continuous batching)",
        "value": closed["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n} requests: P in {{24,48,96}}, grid in {{64^2,128^2,256^2}} (L=0.7), "
                               "10-200 points log-U[0.1,100], lambda U[1,2), noise 10, N=16384",
                   "mix": mix, "slots": args.serve_slots, "steps_per_poll": args.serve_steps,
                   "workers": args.serve_workers,
                   "lsqr_tol": args.tol},
        "one_solve_at_a_time": {"solves_per_s": round(rate1, 3), "p50_ms": round(float(np.percentile(lat1, 50)), 2),
                                "p99_ms": round(float(np.percentile(lat1, 99)), 2),
                                "mean_ms_by_class": by_class},
        "server_all_at_once": closed,
        "server_poisson": sweep,
        "speedup_vs_one_at_a_time": round(closed["solves_per_s"] / rate1, 3),
    }
    print(json.dumps(result), flush=True)


def cpu_info():
    """Host CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def blas_threads():
    from threadpoolctl import threadpool_info
    threads = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
    return int(max(threads)) if threads else 1


def oracle_solve(sc, max_outer=-1, tol=1e-8):
    """The FP64 oracle's solve of one workload (same covariance bits as the GPU)."""
    import numpy as np

    import oracle
    R = sc.R_hat32_c128
    nd = sc.noise_diag.astype(np.float32).astype(np.float64)
    A = oracle.steering(sc.pos, sc.lam, sc.grid)
    mf = oracle.mf_image(A, R)
    gamma = oracle.upper_bound(A, R)
    eps = oracle.detection_threshold(mf, 6.0, sc.N)
    return oracle.solve(A, R - np.diag(nd), gamma, eps, atol=tol, btol=tol, max_outer=max_outer)


def parity_of(sigma, state, ref):
    import numpy as np
    s = sigma.cpu().numpy().astype(np.float64)
    return {"rel_image_err": float(np.linalg.norm(s - ref.sigma) / np.linalg.norm(ref.sigma)),
            "same_sets": bool(np.array_equal(state.cpu().numpy(), ref.state)),
            "oracle_rel_residual": ref.rel_residual}


def time_solves(ctx, R, geo, opts, nd, steps, warmup, torch, what, on_timed_start=None):
    """warmup + timed clsimg_solve calls; every call ends with a synchronisation."""
    Q = geo.Q
    sigma = torch.empty(Q, dtype=torch.float32, device="cuda")
    state = torch.empty(Q, dtype=torch.uint8, device="cuda")
    stats = None
    for i in range(warmup):
        stats = ctx.solve(R, geo, opts, noise_diag=nd, sigma=sigma, state=state)[4]
        torch.cuda.synchronize()
        log(f"bench: {what}: warmup {i + 1}/{warmup}")
    lat, flops = [], 0.0
    torch.cuda.synchronize()
    if on_timed_start is not None:
        on_timed_start()
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        stats = ctx.solve(R, geo, opts, noise_diag=nd, sigma=sigma, state=state)[4]
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        flops += stats["psi_flops"]
    total = time.perf_counter() - t_start
    log(f"bench: {what}: {steps} solves in {total:.3f} s; stats {stats}")
    return {"lat": lat, "total": total, "flops": flops, "stats": stats, "sigma": sigma, "state": state}


def beam_executed_flops(P, Q, tiles):
    """MFMA flops one full-grid FP32 beamformer launch issues: the block
    triangle of Ut, 2 MT (MT + 1) 16x16x4 MFMAs per 16 pixels, MT = Pp / 8 row
    tiles (the GEMM-shaped kernel beyond 48 antennas runs whole workgroups of
    `tiles` 16-pixel tiles)."""
    MT = -(-P // 8)
    if MT <= 6:
        return (-(-Q // 16)) * 2 * MT * (MT + 1) * 2048.0
    # block triangle: row tile m runs column tiles 0..m (4 chunks each), over
    # whole workgroups of `tiles` 16-pixel tiles
    return (-(-Q // (16 * tiles)) * tiles) * 2 * MT * (MT + 1) * 2048.0


def h1_executed_flops(P, Q):
    """MFMA flops of the single half-precision multiplier kernel: row tile m of
    the block triangle runs 32-column chunks 0 .. m // 2, one 16x16x32 MFMA
    (16384 flops) per chunk and 16-pixel tile, over workgroups of 4 tiles."""
    MT = -(-P // 8)
    KC = -(-2 * (-(-P // 8) * 8) // 32)
    per_tile = sum(min(KC, m // 2 + 1) for m in range(MT))
    return (-(-Q // 64) * 4) * per_tile * 16384.0


def forward_executed_flops(P, Q):
    """MFMA flops of the correlation over Q pixels: four 16x16x4 MFMAs per
    16 x 16 antenna tile pair and 4 pixels, over the tile pairs on and below
    the diagonal that the waves' blocks of BT x BT tile pairs cover (a
    diagonal block its lower triangle), BT = 2 up to 2 tiles, else 3."""
    Pp = -(-P // 8) * 8
    na = -(-Pp // 16)
    bt = 2 if na <= 2 else 3
    nb = -(-na // bt)
    tiles = nb * bt * (bt + 1) // 2 + (nb * (nb - 1) // 2) * bt * bt
    return tiles * 4 * 2048.0 * (-(-Q // 4))


def traffic_from(profile, kernel, source):
    """HBM bytes per launch of `kernel` from a committed counter summary, or
    None when the kernel's source changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        src = hashlib.sha256(open(os.path.join(ROOT, "paper_1505_01348_amd", "csrc", source), "rb").read()).hexdigest()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_json: "):
            rec = json.loads(line[len("traffic_json: "):])
            if rec.get("kernel") == kernel and rec.get("source_sha256") == src:
                return rec.get("hbm_bytes_per_launch")
    return None


def batched_sweep(ctx, clsimg, synth, np, torch, opts, sizes, alone_stats):
    """clsimg_solve_batch calls of the 48-antenna workload: request 0 is the
    workload itself, the others redraw sky and samples with other seeds."""
    sc = synth.make_scene("c1")
    pool = []
    for k in range(sizes[-1]):
        sk = sc if k == 0 else synth.make_scene("c1", seed=synth.scenes._SEED_BASE + 1000 * k)
        pool.append({"R": torch.as_tensor(sk.R_hat32).cuda(), "geo": clsimg.Geometry(sk.pos, sk.lam, sk.grid),
                     "noise_diag": torch.as_tensor(sk.noise_diag.astype(np.float32)).cuda()})
    sweep = []
    for nbx in sizes:
        breqs = pool[:nbx]
        row = {"requests_per_call": nbx}
        # the step launches enqueued one by one, then replayed from a captured graph
        for mode in (0, 1):
            opts.batch_graph = mode
            ctx.solve_batch(breqs, opts)  # warm-up (and the capture)
            torch.cuda.synchronize()
            blat, bflops = [], 0.0
            tb0 = time.perf_counter()
            for _ in range(3):
                t0 = time.perf_counter()
                stb, resb = ctx.solve_batch(breqs, opts)
                torch.cuda.synchronize()
                blat.append(time.perf_counter() - t0)
                bflops += sum(r[4]["psi_flops"] for r in resb)
            tbt = time.perf_counter() - tb0
            same0 = (resb[0][4]["rel_residual"] == alone_stats["rel_residual"] and
                     resb[0][4]["lsqr_iters_total"] == alone_stats["lsqr_iters_total"])
            rec = {"solves_per_s": round(3 * nbx / tbt, 3),
                   "ms_per_call_p50": round(float(np.percentile(np.array(blat) * 1e3, 50)), 3),
                   "psi_tflops_dense_count": round(bflops / tbt / 1e12, 4),
                   "request0_same_as_alone": bool(same0 and stb >= 0)}
            if mode == 0:
                row.update(rec)
            else:
                row["graph_rounds"] = rec
        opts.batch_graph = 0
        sweep.append(row)
        log(f"bench: batched {nbx} per call: {sweep[-1]}")
    return sweep


def serving_mix(clsimg, synth, np, torch, n, tol, slots=64, steps_per_poll=16, workers=8, poisson=True):
    """Mixed requests (P in {24, 48, 96}, grids 64^2..256^2): one clsimg_solve
    after another, then the continuous-batching server with all requests
    submitted at once and, optionally, with Poisson arrivals."""
    scenes = synth.make_request_scenes(n)
    opts = clsimg.default_options()
    opts.nsamples = 16384
    opts.atol = opts.btol = tol
    reqs = [{"R": torch.as_tensor(sc.R_hat32).cuda(), "geo": clsimg.Geometry(sc.pos, sc.lam, sc.grid),
             "noise_diag": torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()} for sc in scenes]
    torch.cuda.synchronize()
    mix = {}
    for sc in scenes:
        key = f"P{sc.P}_{sc.nl}x{sc.nm}"
        mix[key] = mix.get(key, 0) + 1
    log(f"bench: serving {n} requests, mix {mix}")
    ctx = clsimg.Context(0)
    for rq in reqs[:2]:
        ctx.solve(rq["R"], rq["geo"], opts, noise_diag=rq["noise_diag"])
    torch.cuda.synchronize()
    alone, lat1 = [], []
    t0 = time.perf_counter()
    for rq in reqs:
        ts = time.perf_counter()
        alone.append(ctx.solve(rq["R"], rq["geo"], opts, noise_diag=rq["noise_diag"])[4])
        torch.cuda.synchronize()
        lat1.append(time.perf_counter() - ts)
    t_seq = time.perf_counter() - t0
    ctx.close()
    rate1 = n / t_seq
    log(f"bench: serving: one solve at a time {rate1:.2f} solves/s")

    def run(arrivals):
        srv = clsimg.Server(opts, max_slots=slots, hbm_budget=4 << 30, steps_per_poll=steps_per_poll,
                            workers=workers)
        order = sorted(range(n), key=lambda i: arrivals[i])
        ticket_of, done_at, stats = {}, {}, {}
        k = 0
        t_start = time.perf_counter()
        while len(done_at) < n:
            now = time.perf_counter() - t_start
            while k < n and arrivals[order[k]] <= now:
                i = order[k]
                ticket_of[srv.submit(reqs[i])] = i
                k += 1
            info = srv.info()
            busy = info["pending"] + info["active"] + info["worker_queued"] + info["ready"] > 0
            if not busy:
                if k < n:
                    time.sleep(max(0.0, arrivals[order[k]] - (time.perf_counter() - t_start)))
                continue
            for t, r in srv.poll(wait=(k == n)):
                i = ticket_of[t]
                done_at[i] = time.perf_counter() - t_start
                stats[i] = r[4]
        total = time.perf_counter() - t_start
        peak = srv.info()["arena_peak"]
        srv.close()
        lat = np.array([done_at[i] - arrivals[i] for i in range(n)]) * 1e3
        same = all(stats[i]["rel_residual"] == alone[i]["rel_residual"] and
                   stats[i]["lsqr_iters_total"] == alone[i]["lsqr_iters_total"] for i in range(n))
        return {"solves_per_s": round(n / total, 3), "wall_s": round(total, 3),
                "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "arena_peak_bytes": int(peak), "same_result_as_alone": bool(same)}

    closed = run([0.0] * n)
    log(f"bench: serving: server, all {n} at once: {closed}")
    sweep = {}
    if poisson:
        rng = np.random.default_rng(20150504)
        for f in (0.5, 1.0, 2.0):
            qps = f * rate1
            arr = np.cumsum(rng.exponential(1.0 / qps, size=n))
            arr -= arr[0]
            sweep[f"{f}x"] = dict(run(list(arr)), qps=round(qps, 3))
            log(f"bench: serving: Poisson arrivals at {qps:.2f}/s: {sweep[f'{f}x']}")
    lat1 = np.array(lat1) * 1e3
    by_class = {}
    for sc, t in zip(scenes, lat1):
        by_class.setdefault(f"P{sc.P}_{sc.nl}x{sc.nm}", []).append(float(t))
    by_class = {k: round(float(np.mean(v)), 2) for k, v in sorted(by_class.items())}
    return {
        "workload": f"{n} requests: P in {{24,48,96}}, grid in {{64^2,128^2,256^2}} (L=0.7), 10-200 points "
                    "log-U[0.1,100], lambda U[1,2), noise 10, N=16384",
        "mix": mix, "slots": slots, "steps_per_poll": steps_per_poll, "workers": workers, "lsqr_tol": tol,
        "one_solve_at_a_time": {"solves_per_s": round(rate1, 3), "p50_ms": round(float(np.percentile(lat1, 50)), 2),
                                "p99_ms": round(float(np.percentile(lat1, 99)), 2), "mean_ms_by_class": by_class},
        "server_all_at_once": closed,
        "server_poisson": sweep,
        "speedup_vs_one_at_a_time": round(closed["solves_per_s"] / rate1, 3),
    }


def graph_or_eager_seconds(call, reps, torch):
    """Seconds per call of `reps` back-to-back calls replayed from a captured
    graph (host enqueue time excluded, dispatch gaps included), or eager."""
    for _ in range(3):
        call()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    how = "graph"
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                call()
        g.replay()
        torch.cuda.synchronize()
        ev0.record()
        g.replay()
        ev1.record()
    except Exception as e:  # capture refused: eager calls
        log(f"bench: graph capture failed ({e}); timing eager calls")
        how = "eager"
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            call()
        ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / 1e3 / reps, f"{how} of {reps} back-to-back calls"


def full_grid_ops(ctx, clsimg, np, torch, sc, reps=20):
    """The full-grid operators of one workload: the beamformer (dirty image) in
    every precision, with device timestamps bound to its kernels, and the
    correlation over every pixel; dense-count and executed-MFMA rates."""
    geo = clsimg.Geometry(sc.pos, sc.lam, sc.grid)
    R = torch.as_tensor(sc.R_hat32).cuda()
    out = torch.empty(sc.Q, dtype=torch.float32, device="cuda")
    P, Q = sc.P, sc.Q
    Pp = -(-P // 8) * 8
    dense = 8.0 * P * P * Q + 8.0 * P * Q
    res = {"workload": f"P={P}, {sc.nl}x{sc.nm} pixels", "beamformer": {}}
    for name, prec in PRECISIONS.items():
        tiles = None
        if not (prec == 0 and P <= 48):
            tiles, tune_us = ctx.autotune(geo, precision=prec)
            log(f"bench: {name} beamformer at P={P}: {tiles} tiles per workgroup (us for 2/4/8: {tune_us})")
        for _ in range(3):
            ctx.dirty_image(R, geo, mf=out, precision=prec)
        torch.cuda.synchronize()
        t = stamped_seconds(lambda a, b: ctx.dirty_image_timed(R, geo, a, b, mf=out, precision=prec), reps)
        if prec == 0:
            ex = beam_executed_flops(P, Q, tiles or 2)
            kern = ("beam_kernel" if P <= 48 else "beam_big_kernel") + " (FP32 16x16x4 MFMA)"
            rec = {"kernel": kern, "us_per_launch": round(t * 1e6, 2), "dense_tflops": round(dense / t / 1e12, 3),
                   "executed_tflops": round(ex / t / 1e12, 3), "peak": PEAK_FP32_MFMA_TFLOPS,
                   "frac": round(ex / t / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                   "frac_dense_count": round(dense / t / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                   "executed_flops_per_launch": ex}
        else:
            # three products on the block triangle (chunks 0 .. m // 2 of row tile m)
            MT = Pp // 8
            KC = -(-2 * Pp // 32)
            ex = 3.0 * (-(-Q // (16 * tiles)) * tiles) * sum(min(KC, m // 2 + 1) for m in range(MT)) * 16384.0
            rec = {"kernel": f"beam_h16_kernel (split {name}: three 16x16x32 products)",
                   "us_per_launch": round(t * 1e6, 2), "dense_tflops": round(dense / t / 1e12, 3),
                   "executed_tflops": round(ex / t / 1e12, 3), "peak": PEAK_HALF_MFMA_TFLOPS,
                   "frac": round(ex / t / 1e12 / PEAK_HALF_MFMA_TFLOPS, 4), "executed_flops_per_launch": ex}
        if tiles:
            rec["tiles_per_workgroup"] = tiles
        res["beamformer"][name] = rec
        log(f"bench: {name} beamformer at P={P}: {t * 1e6:.1f} us, {dense / t / 1e12:.1f} TFLOP/s dense count")
    vq = torch.rand(Q, dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    Yq = torch.empty((P, P), dtype=torch.complex64, device="cuda")
    tf, how = graph_or_eager_seconds(lambda: ctx.forward(geo, vq, Y=Yq), reps, torch)
    fd = 8.0 * P * P * Q
    fe = forward_executed_flops(P, Q)
    res["forward"] = {"kernels": "corr_kernel + reduce_kernel", "us_per_call": round(tf * 1e6, 2),
                      "dense_tflops": round(fd / tf / 1e12, 3), "executed_tflops": round(fe / tf / 1e12, 3),
                      "peak": PEAK_FP32_MFMA_TFLOPS, "frac": round(fe / tf / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                      "frac_dense_count": round(fd / tf / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                      "executed_flops_per_call": fe, "timing": how}
    log(f"bench: forward at P={P}: {tf * 1e6:.1f} us, {fd / tf / 1e12:.1f} TFLOP/s dense count")
    return res


def headline_bench(args, clsimg, synth, np, torch):
    steps = 20 if args.steps is None else args.steps
    warmup = 3 if args.warmup is None else args.warmup
    prec = PRECISIONS[args.precision]
    sc = synth.make_scene("c4")
    log(f"bench: headline workload c4 P={sc.P} Q={sc.Q} N={sc.N}, first 10 Table I steps")
    geo = clsimg.Geometry(sc.pos, sc.lam, sc.grid)
    opts = clsimg.default_options()
    opts.nsamples = sc.N
    opts.atol = opts.btol = args.tol
    opts.precision = prec
    opts.max_outer = 10
    R = torch.as_tensor(sc.R_hat32).cuda()
    nd = torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()
    ctx = clsimg.Context(0)
    if prec != 0:
        ctx.autotune(geo, precision=prec)
    # the multiplier kernel of every feasible step (the steps' dominant kernel)
    # is timed with HIP events bound to its launches inside the timed solves
    ctx.kernel_timing(False)
    run = time_solves(ctx, R, geo, opts, nd, steps, warmup, torch, f"c4 first 10 steps, {args.precision}",
                      on_timed_start=lambda: ctx.kernel_timing(True))
    mult_ms, mult_n = ctx.kernel_timing(False)
    total, stats = run["total"], run["stats"]
    lat_ms = np.array(run["lat"]) * 1e3
    plain = None
    if prec != 0:
        # the plain FP32 path on the same steps, for the equal-residual comparison
        o32 = clsimg.default_options()
        o32.nsamples = sc.N
        o32.atol = o32.btol = args.tol
        o32.max_outer = 10
        r32 = time_solves(ctx, R, geo, o32, nd, max(3, steps // 2), 1, torch, "c4 first 10 steps, fp32 plain")
        res_lo, res32 = stats["rel_residual"], r32["stats"]["rel_residual"]
        s_lo = run["sigma"].cpu().numpy().astype(np.float64)
        s32 = r32["sigma"].cpu().numpy().astype(np.float64)
        plain = {"ms_per_step": round(r32["total"] / len(r32["lat"]) * 1e3, 4),
                 "psi_tflops_dense_count": round(r32["flops"] / r32["total"] / 1e12, 4),
                 "rel_residual": res32,
                 "speedup_of_reduced_precision": round((r32["total"] / len(r32["lat"])) / (total / steps), 4),
                 "equal_final_residual": bool(abs(res_lo - res32) <= 1e-3 * res32),
                 "same_sets": bool(np.array_equal(run["state"].cpu().numpy(), r32["state"].cpu().numpy())),
                 "rel_image_diff": float(np.linalg.norm(s_lo - s32) / np.linalg.norm(s32))}
        log(f"bench: fp32 plain path {plain}")

    # the roofline kernel: the full-grid beamformer of every feasible step's
    # gradient (the same GEMM as the dirty image and the bound), timed on the
    # dirty image with the device's own timestamps of its launches
    full4 = full_grid_ops(ctx, clsimg, np, torch, sc)
    dense_beam = 8.0 * sc.P * sc.P * sc.Q + 8.0 * sc.P * sc.Q
    t_mult = mult_ms / 1e3 / max(mult_n, 1)
    if prec == 0:
        ex = beam_executed_flops(sc.P, sc.Q, 4)
        roof = {"kernel": "beam_big_kernel<9, 4, BeamLambda> (multipliers of each feasible step: the full-grid "
                          "gradient, eq. gls)", "bound": "mfma", "peak": PEAK_FP32_MFMA_TFLOPS,
                "traffic": traffic_from("beam_big_kernel_c4_traffic.md", "beam_big_kernel<9, 4, BeamMF>", "beam.hip")}
        peak = PEAK_FP32_MFMA_TFLOPS
    else:
        ex = h1_executed_flops(sc.P, sc.Q)
        roof = {"kernel": f"beam_h1_kernel<9, {args.precision}, BeamLambdaApprox> (multipliers of each feasible "
                          "step: one half-precision product, decision refined in FP32)", "bound": "mfma",
                "peak": PEAK_HALF_MFMA_TFLOPS,
                "traffic": traffic_from("beam_h1_kernel_c4_traffic.md", "beam_h1_kernel<9, fp16, BeamLambdaApprox>",
                                        "beam.hip")}
        peak = PEAK_HALF_MFMA_TFLOPS
    roof.update({"achieved": round(ex / t_mult / 1e12, 4), "unit": "TFLOP/s",
                 "frac": round(ex / t_mult / 1e12 / peak, 5),
                 "frac_dense_count": round(dense_beam / t_mult / 1e12 / peak, 5),
                 "us_per_launch": round(t_mult * 1e6, 3), "launches_timed": mult_n,
                 "executed_flops_per_launch": ex, "dense_flops_per_launch": dense_beam,
                 "timing": "HIP events bound to every launch of the kernel inside the timed solves "
                           "(clsimg_kernel_timing), mean"})

    psi_tflops = run["flops"] / total / 1e12
    model, ncores = cpu_info()
    result = {
        "metric": METRIC,
        "value": round(psi_tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(total / steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16 + f32", "bf16": "bf16 + f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"c4: {WORKLOADS['c4']}; first 10 Table I steps of the active-set solve",
                   "P": sc.P, "Q": sc.Q, "nsamples": sc.N, "n_sources": int(len(sc.src_pix)), "max_outer": 10,
                   "bound": "mvdr", "cost": "ls", "precision": args.precision, "lsqr_tol": args.tol,
                   "value_is": "dense-count Psi / Psi^H flops of the timed steps (8 P^2 per pixel and correlation "
                               "term, + 8 P per beamformed pixel) / wall time"},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
        "solves_per_s": round(steps / total, 4),
        "solve": {k: stats[k] for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF", "nU",
                                        "rel_residual")},
        "roofline": roof,
        "full_grid_288": full4,
    }
    if plain is not None:
        result["fp32_plain_path"] = plain
    del R

    # the 48-antenna workload: complete solves (the device-resident loop)
    s1 = synth.make_scene("c1")
    g1 = clsimg.Geometry(s1.pos, s1.lam, s1.grid)
    o1 = clsimg.default_options()
    o1.nsamples = s1.N
    o1.atol = o1.btol = args.tol
    R1 = torch.as_tensor(s1.R_hat32).cuda()
    nd1 = torch.as_tensor(s1.noise_diag.astype(np.float32)).cuda()
    r1 = time_solves(ctx, R1, g1, o1, nd1, 20, 3, torch, "c1 complete solves")
    l1 = np.array(r1["lat"]) * 1e3
    c1 = {"workload": f"c1: {WORKLOADS['c1']}", "solves_per_s": round(20 / r1["total"], 3),
          "p50_ms": round(float(np.percentile(l1, 50)), 3), "p99_ms": round(float(np.percentile(l1, 99)), 3),
          "psi_tflops_dense_count": round(r1["flops"] / r1["total"] / 1e12, 4),
          "solve": {k: r1["stats"][k] for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF",
                                                "nU", "rel_residual")},
          "dominant_kernel": "outer_step_kernel<6> (one workgroup: the LSQR of the free set and the step logic)",
          "us_per_lsqr_iteration_bound": round(r1["total"] / 20 * 1e6 / max(r1["stats"]["lsqr_iters_total"], 1), 3)}
    c1["full_grid_48"] = full_grid_ops(ctx, clsimg, np, torch, s1)
    result["c1"] = c1

    # the 96-antenna workload: complete solves (Table I driven from the host,
    # the free-set LSQR in two launches per iteration), in the headline's
    # precision and in FP32
    s2 = synth.make_scene("c2")
    g2 = clsimg.Geometry(s2.pos, s2.lam, s2.grid)
    R2 = torch.as_tensor(s2.R_hat32).cuda()
    nd2 = torch.as_tensor(s2.noise_diag.astype(np.float32)).cuda()
    c2_runs = {}
    for pname in dict.fromkeys([args.precision, "fp32"]):
        o2 = clsimg.default_options()
        o2.nsamples = s2.N
        o2.atol = o2.btol = args.tol
        o2.precision = PRECISIONS[pname]
        c2_runs[pname] = time_solves(ctx, R2, g2, o2, nd2, 10, 2, torch, f"c2 complete solves, {pname}")
    r2 = c2_runs[args.precision]
    l2 = np.array(r2["lat"]) * 1e3
    c2 = {"workload": f"c2: {WORKLOADS['c2']}", "precision": args.precision,
          "solves_per_s": round(10 / r2["total"], 3),
          "p50_ms": round(float(np.percentile(l2, 50)), 3), "p99_ms": round(float(np.percentile(l2, 99)), 3),
          "psi_tflops_dense_count": round(r2["flops"] / r2["total"] / 1e12, 4),
          "solve": {k: r2["stats"][k] for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total", "nF",
                                                "nU", "rel_residual")},
          "dominant_kernels": "lsqr_fwd_kernel + adjoint_list_kernel<12> (the two launches of each LSQR "
                              "iteration over the free set)",
          "us_per_lsqr_iteration_bound": round(r2["total"] / 10 * 1e6 / max(r2["stats"]["lsqr_iters_total"], 1), 3)}
    if args.precision != "fp32":
        r32 = c2_runs["fp32"]
        c2["fp32"] = {"solves_per_s": round(10 / r32["total"], 3),
                      "rel_residual": r32["stats"]["rel_residual"],
                      "same_sets": bool(np.array_equal(r2["state"].cpu().numpy(), r32["state"].cpu().numpy()))}
    result["c2"] = c2
    del R2
    sizes = sorted({int(x) for x in str(args.batched_extra).split(",") if int(x) > 1})
    if sizes:
        result["batched_c1"] = batched_sweep(ctx, clsimg, synth, np, torch, o1, sizes, r1["stats"])
    del R1
    ctx.close()
    if args.serve_default > 0:
        result["serving"] = serving_mix(clsimg, synth, np, torch, args.serve_default, args.tol,
                                        poisson=not args.no_poisson)

    if not args.no_cpu:
        import threadpoolctl
        t0 = time.perf_counter()
        ref4 = oracle_solve(sc, max_outer=10)
        t4 = time.perf_counter() - t0
        threads = blas_threads()
        log(f"cpu baseline: oracle, first 10 steps of c4, {t4:.1f} s on {threads} threads")
        result["parity"] = parity_of(run["sigma"], run["state"], ref4)
        # the oracle runs the same ten steps: the GPU path's dense-count flops
        # of one such solve over the oracle's time for it
        result["cpu_baseline"] = {"value": round(stats["psi_flops"] / t4 / 1e12, 6), "unit": "TFLOP/s",
                                  "cores": threads, "kind": "oracle",
                                  "sample": f"1 FP64 oracle solve of the same first 10 Table I steps ({t4:.1f} s); "
                                            "flops: the dense count of those steps", "cpu_model": model,
                                  "cores_available": ncores}
        t0 = time.perf_counter()
        ref1 = oracle_solve(s1)
        t1 = time.perf_counter() - t0
        c1["parity"] = parity_of(r1["sigma"], r1["state"], ref1)
        c1["cpu_baseline"] = {"value": round(1.0 / t1, 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
                              "sample": f"1 complete FP64 oracle solve ({t1:.1f} s)"}
        t0 = time.perf_counter()
        ref2 = oracle_solve(s2)
        t2 = time.perf_counter() - t0
        c2["parity"] = parity_of(r2["sigma"], r2["state"], ref2)
        c2["cpu_baseline"] = {"value": round(1.0 / t2, 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
                              "sample": f"1 complete FP64 oracle solve ({t2:.1f} s)"}
        log(f"cpu baseline: c2 oracle solve {t2:.1f} s")
        s0 = synth.make_scene("c0")
        with threadpoolctl.threadpool_limits(1):
            runs, t0c = 0, 0.0
            while t0c < 3.0 and runs < 30:
                t0 = time.perf_counter()
                oracle_solve(s0)
                t0c += time.perf_counter() - t0
                runs += 1
        result["cpu"] = {"model": model, "cores_available": ncores, "blas_threads": threads,
                         "c0_oracle_one_thread": {"value": round(runs / t0c, 4), "unit": "solves/s",
                                                  "sample": f"{runs} complete FP64 oracle solves of c0 ({t0c:.1f} s)"}}
        log(f"cpu baseline: c0 on one thread {runs / t0c:.2f} solves/s")
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; no multi-GPU path exists "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1505_01348_amd import clsimg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    special = args.serve or args.offgrid >= 0 or args.blocks > 1 or args.channels > 1 or args.kernel_only
    if args.config == "headline" and not special:
        if args.precision is None:
            args.precision = "fp16"
        headline_bench(args, clsimg, synth, np, torch)
        return
    if args.precision is None:
        args.precision = "fp32"
    if args.config == "headline":  # the other measurements' default workloads
        args.config = "c4" if args.kernel_only else "c1"
    if args.steps is None:
        args.steps = 100
    if args.warmup is None:
        args.warmup = 10
    if args.serve:
        serve_bench(args, clsimg, synth, np, torch)
        return
    if args.offgrid >= 0:
        offgrid_bench(args, clsimg, synth, np, torch)
        return
    if args.blocks > 1 or args.channels > 1:
        multi_bench(args, clsimg, synth, np, torch)
        return
    sc = synth.make_scene(args.config)
    log(f"bench: workload {args.config} P={sc.P} Q={sc.Q} N={sc.N}")
    if args.kernel_only:
        geo = clsimg.Geometry(sc.pos, sc.lam, sc.grid)
        ctx = clsimg.Context(0)
        R = torch.as_tensor(sc.R_hat32).cuda()
        out = torch.empty(sc.Q, dtype=torch.float32, device="cuda")
        for _ in range(20):
            ctx.dirty_image(R, geo, mf=out)
        torch.cuda.synchronize()
        log("bench: kernel-only: 20 FP32 dirty images done")
        # the forward operator over every pixel (v in [0, 1)), then the
        # half-precision beamformers
        vq = torch.rand(sc.Q, dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
        Yq = torch.empty((sc.P, sc.P), dtype=torch.complex64, device="cuda")
        for _ in range(5):
            ctx.forward(geo, vq, Y=Yq)
        torch.cuda.synchronize()
        log("bench: kernel-only: 5 full-grid forwards done")
        for prec in (1, 2):
            for _ in range(5):
                ctx.dirty_image(R, geo, mf=out, precision=prec)
        torch.cuda.synchronize()
        log("bench: kernel-only: 5 FP16 and 5 BF16 dirty images done")
        if sc.P > 48:
            # the refined half-precision multipliers: the first ten Table I steps in FP16
            o = clsimg.default_options()
            o.nsamples = sc.N
            o.atol = o.btol = args.tol
            o.precision = 1
            o.max_outer = 10
            ctx.solve(R, geo, o, noise_diag=torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda())
            torch.cuda.synchronize()
            log("bench: kernel-only: 10 FP16 Table I steps done")
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        ctx.close()
        log(f"bench: kernel-only run done (20 FP32 dirty images, 5 forwards, 10 half-precision dirty images, "
            f"3 copies of {args.copy_mib} MiB)")
        return
    geo = clsimg.Geometry(sc.pos, sc.lam, sc.grid)
    opts = clsimg.default_options()
    opts.nsamples = sc.N
    opts.atol = opts.btol = args.tol
    opts.cost = clsimg.COST_PWLS if args.cost == "pwls" else clsimg.COST_LS
    opts.bound = {"mvdr": clsimg.BOUND_MVDR, "mf": clsimg.BOUND_MF, "none": clsimg.BOUND_NONE}[args.bound]
    opts.kappa_b = args.kappa_b
    opts.precision = PRECISIONS[args.precision]
    opts.max_outer = args.max_outer
    R = torch.as_tensor(sc.R_hat32).cuda()
    nd = torch.as_tensor(sc.noise_diag.astype(np.float32)).cuda()
    Q = sc.Q
    sigma = torch.empty(Q, dtype=torch.float32, device="cuda")
    state = torch.empty(Q, dtype=torch.uint8, device="cuda")
    mf = torch.empty(Q, dtype=torch.float32, device="cuda")
    gamma = torch.empty(Q, dtype=torch.float32, device="cuda")
    ctx = clsimg.Context(0)
    B = max(1, args.batch)
    reqs = [{"R": R, "geo": geo, "noise_diag": nd, "sigma": sigma, "state": state, "mf": mf, "gamma": gamma}]
    for k in range(1, B):
        sk = synth.make_scene(args.config, seed=synth.scenes._SEED_BASE + 1000 * k)
        reqs.append({"R": torch.as_tensor(sk.R_hat32).cuda(), "geo": clsimg.Geometry(sk.pos, sk.lam, sk.grid),
                     "noise_diag": torch.as_tensor(sk.noise_diag.astype(np.float32)).cuda()})

    def step():
        if B == 1:
            return ctx.solve(R, geo, opts, noise_diag=nd, sigma=sigma, state=state, mf=mf, gamma=gamma)[4]
        st, res = ctx.solve_batch(reqs, opts)
        if st < 0:
            raise RuntimeError(f"batched solve returned {st}: {clsimg.strerror(st)}")
        agg = dict(res[0][4])
        agg["psi_flops"] = sum(r[4]["psi_flops"] for r in res)
        return agg

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"bench: warmup {i + 1}/{args.warmup}")
    lat, flops, stats = [], 0.0, None
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        stats = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        flops += stats["psi_flops"]
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    log(f"bench: {args.steps} steps of {B} solve(s) in {total:.3f} s; last stats {stats}")
    sequential = None
    if B > 1:
        # the same requests one clsimg_solve call after another, for comparison
        t0 = time.perf_counter()
        for rq in reqs:
            ctx.solve(rq["R"], rq["geo"], opts, noise_diag=rq["noise_diag"])
        torch.cuda.synchronize()
        sequential = B / (time.perf_counter() - t0)
        log(f"bench: the {B} requests solved one by one: {sequential:.2f} solves/s")

    batched = None
    sizes = sorted({int(x) for x in str(args.batched_extra).split(",") if int(x) > 1})
    if B == 1 and sizes and sc.P <= 48:
        # the same workload served as batches (clsimg_solve_batch): request 0 is
        # this covariance, the others redraw sky and samples with other seeds;
        # one workgroup per request, so up to one request per CU runs at once
        pool = [{"R": R, "geo": geo, "noise_diag": nd}]
        for k in range(1, sizes[-1]):
            sk = synth.make_scene(args.config, seed=synth.scenes._SEED_BASE + 1000 * k)
            pool.append({"R": torch.as_tensor(sk.R_hat32).cuda(), "geo": clsimg.Geometry(sk.pos, sk.lam, sk.grid),
                         "noise_diag": torch.as_tensor(sk.noise_diag.astype(np.float32)).cuda()})
        sweep = []
        for nbx in sizes:
            breqs = pool[:nbx]
            st0, res0 = ctx.solve_batch(breqs, opts)  # warm-up
            torch.cuda.synchronize()
            blat = []
            bflops = 0.0
            tb0 = time.perf_counter()
            for _ in range(3):
                t0 = time.perf_counter()
                stb, resb = ctx.solve_batch(breqs, opts)
                torch.cuda.synchronize()
                blat.append(time.perf_counter() - t0)
                bflops += sum(r[4]["psi_flops"] for r in resb)
            tbt = time.perf_counter() - tb0
            same0 = (resb[0][4]["rel_residual"] == stats["rel_residual"] and
                     resb[0][4]["lsqr_iters_total"] == stats["lsqr_iters_total"])
            sweep.append({"requests_per_call": nbx, "solves_per_s": round(3 * nbx / tbt, 3),
                          "ms_per_call_p50": round(float(np.percentile(np.array(blat) * 1e3, 50)), 3),
                          "psi_tflops": round(bflops / tbt / 1e12, 4),
                          "psi_dense_count_over_fp32_peak": round(bflops / tbt / 1e12 / PEAK_FP32_MFMA_TFLOPS, 5),
                          "request0_same_as_alone": bool(same0 and stb >= 0)})
            log(f"bench: batched {nbx} per call: {sweep[-1]}")
        batched = dict(sweep[-1])
        batched["note"] = ("clsimg_solve_batch: one outer-step launch and one multiplier launch per Table I step "
                           "for all requests; every result equals its solve alone; psi_tflops counts the "
                           "dense-count Psi / Psi^H flops of all requests")
        if len(sweep) > 1:
            batched["sweep"] = sweep
        del pool, breqs

    # roofline of the full-grid beamforming kernel: the dirty image is one
    # launch of it.  Its time per launch is the span of a replayed graph of
    # `reps` back-to-back launches divided by `reps` (it includes the dispatch
    # gaps between the kernels, so the rate is a lower bound).  The kernel's
    # own device timestamps (clsimg_dirty_image_timed: events bound to the
    # launch itself) of `reps` separate launches are reported beside it.
    reps = args.kernel_reps
    P = sc.P
    out = torch.empty(Q, dtype=torch.float32, device="cuda")
    for _ in range(5):
        ctx.dirty_image(R, geo, mf=out)
    torch.cuda.synchronize()
    timing = "graph"
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    try:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(reps):
                ctx.dirty_image(R, geo, mf=out)
        graph.replay()
        torch.cuda.synchronize()
        ev0.record()
        graph.replay()
        ev1.record()
    except Exception as e:  # capture refused: time eager calls instead
        log(f"bench: graph capture failed ({e}); timing eager calls")
        timing = "eager"
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            ctx.dirty_image(R, geo, mf=out)
        ev1.record()
    torch.cuda.synchronize()
    t_kernel = ev0.elapsed_time(ev1) / 1e3 / reps
    t_alone = stamped_seconds(lambda a, b: ctx.dirty_image_timed(R, geo, a, b, mf=out), reps)
    log(f"bench: dirty image {t_kernel * 1e6:.2f} us per launch over a {timing} of {reps}, "
        f"{t_alone * 1e6:.2f} us device time of a launch alone")
    kflops = 8.0 * P * P * Q + 8.0 * P * Q  # dense count of one full-grid adjoint
    MT = -(-P // 8)
    if MT <= 6:  # register-resident kernel: block triangle of Ut, each off-diagonal block used twice
        kname = f"beam_kernel<{MT}, BeamMF> (dirty image, full grid)"
        exec_flops = (-(-Q // 16)) * 2 * MT * (MT + 1) * 2048.0
    else:  # GEMM-shaped kernel: every row tile (padded to 4 per wave group) against K = 2 Pp
        rpw = -(-MT // 4)
        nt = 2 if rpw <= 4 else 4
        kname = f"beam_prep_full + beam_big_kernel<{rpw}, BeamMF> (dirty image, full grid)"
        exec_flops = 2.0 * (64 * rpw) * (16 * MT) * (-(-Q // (16 * nt)) * 16 * nt)
    achieved = kflops / t_kernel / 1e12

    # the forward operator on every pixel of the grid (Psi v, eq. correlation
    # form): split-K correlation kernel + fixed-order reduction, same timing
    vq = torch.rand(Q, dtype=torch.float32, device="cuda")
    Yq = torch.empty((P, P), dtype=torch.complex64, device="cuda")
    for _ in range(5):
        ctx.forward(geo, vq, Y=Yq)
    torch.cuda.synchronize()
    fwd_timing = "graph"
    try:
        gf = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gf):
            for _ in range(reps):
                ctx.forward(geo, vq, Y=Yq)
        gf.replay()
        torch.cuda.synchronize()
        ev0.record()
        gf.replay()
        ev1.record()
    except Exception as e:
        log(f"bench: graph capture of the forward failed ({e}); timing eager calls")
        fwd_timing = "eager"
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            ctx.forward(geo, vq, Y=Yq)
        ev1.record()
    torch.cuda.synchronize()
    t_fwd = ev0.elapsed_time(ev1) / 1e3 / reps
    fwd_flops = 8.0 * P * P * Q
    fwd_exec = forward_executed_flops(P, Q)
    forward_full = {"kernels": "corr_kernel + reduce_kernel", "bound": "mfma",
                    "achieved": round(fwd_exec / t_fwd / 1e12, 4), "peak": PEAK_FP32_MFMA_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(fwd_exec / t_fwd / 1e12 / PEAK_FP32_MFMA_TFLOPS, 5),
                    "frac_dense_count": round(fwd_flops / t_fwd / 1e12 / PEAK_FP32_MFMA_TFLOPS, 5),
                    "us_per_call": round(t_fwd * 1e6, 3), "flops_per_call": fwd_flops,
                    "executed_flops_per_call": fwd_exec, "timing": f"{fwd_timing} of {reps} back-to-back calls"}
    log(f"bench: forward over the whole grid {t_fwd * 1e6:.2f} us/call, {fwd_flops / t_fwd / 1e12:.2f} TFLOP/s")
    del vq, Yq
    log(f"bench: beam kernel {t_kernel * 1e6:.2f} us/launch, {achieved:.2f} TFLOP/s dense count, "
        f"{exec_flops / t_kernel / 1e12:.2f} TFLOP/s issued MFMA")

    # the same operation at the largest workload's full size (288 antennas,
    # 512 x 512 pixels), where the GEMM-shaped beamformer runs
    big = None
    if not args.no_large:
        sb = synth.make_scene("c4")
        gb = clsimg.Geometry(sb.pos, sb.lam, sb.grid)
        Rb = torch.as_tensor(sb.R_hat32).cuda()
        ob = torch.empty(sb.Q, dtype=torch.float32, device="cuda")
        fb = 8.0 * sb.P * sb.P * sb.Q + 8.0 * sb.P * sb.Q
        Ppb = -(-sb.P // 8) * 8
        by = {}
        for name, prec in PRECISIONS.items():
            tiles, tune_us = ctx.autotune(gb, precision=prec)  # pixel tiles per workgroup, kept in the context
            log(f"bench: autotuned {name}: {tiles} tiles per workgroup (us for 2/4/8: {tune_us})")
            for _ in range(3):
                ctx.dirty_image(Rb, gb, mf=ob, precision=prec)
            torch.cuda.synchronize()
            tb = stamped_seconds(lambda a, b: ctx.dirty_image_timed(Rb, gb, a, b, mf=ob, precision=prec), 20)
            dense = fb / tb / 1e12
            if prec == 0:
                by[name] = {"kernel": f"beam_prep_full + beam_big_kernel<9, {tiles}, BeamMF>", "bound": "mfma",
                            "achieved": round(dense, 4), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(dense / PEAK_FP32_MFMA_TFLOPS, 5), "us_per_launch": round(tb * 1e6, 2)}
            else:
                # three half-precision products (hi.hi, hi.lo, lo.hi) of the full real 2P x 2P matrix
                issued = 3 * 2.0 * (2 * Ppb) ** 2 * sb.Q
                by[name] = {"kernel": f"scale + prep + beam_h16_kernel<9, {tiles}, {name}, BeamMF>", "bound": "mfma",
                            "achieved_dense_count": round(dense, 4), "issued_half_mfma": round(issued / tb / 1e12, 4),
                            "peak": PEAK_HALF_MFMA_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(issued / tb / 1e12 / PEAK_HALF_MFMA_TFLOPS, 5),
                            "us_per_launch": round(tb * 1e6, 2), "speedup_vs_fp32": None}
            by[name]["autotune"] = {"tiles_per_workgroup": tiles, "us_for_2_4_8": [round(t, 2) for t in tune_us]}
            log(f"bench: 288-antenna dirty image {name}: {tb * 1e6:.1f} us, {dense:.1f} TFLOP/s dense count")
        # the forward operator on every pixel at this size (FP32)
        vb = torch.rand(sb.Q, dtype=torch.float32, device="cuda")
        Yb = torch.empty((sb.P, sb.P), dtype=torch.complex64, device="cuda")
        for _ in range(3):
            ctx.forward(gb, vb, Y=Yb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            ctx.forward(gb, vb, Y=Yb)
        e1.record()
        torch.cuda.synchronize()
        tfb = e0.elapsed_time(e1) / 1e3 / 20
        ffb = 8.0 * sb.P * sb.P * sb.Q
        feb = forward_executed_flops(sb.P, sb.Q)
        fwd_big = {"kernels": "corr_kernel + reduce_kernel", "us_per_call": round(tfb * 1e6, 2),
                   "achieved": round(feb / tfb / 1e12, 4), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(feb / tfb / 1e12 / PEAK_FP32_MFMA_TFLOPS, 5),
                   "frac_dense_count": round(ffb / tfb / 1e12 / PEAK_FP32_MFMA_TFLOPS, 5), "flops_per_call": ffb,
                   "executed_flops_per_call": feb, "timing": "eager, 20 calls"}
        log(f"bench: 288-antenna forward over the whole grid: {tfb * 1e6:.1f} us, {ffb / tfb / 1e12:.1f} TFLOP/s")
        del vb, Yb
        for name in ("fp16", "bf16"):
            by[name]["speedup_vs_fp32"] = round(by["fp32"]["us_per_launch"] / by[name]["us_per_launch"], 3)
        big = dict(by["fp32"], workload="P=288, 512x512 pixels (the 288-antenna workload's size)",
                   flops_per_launch=fb, by_precision=by,
                   timing="device timestamps from the start of the first kernel (fragment preparation) to the "
                          "end of the beamformer, mean of 20 calls", forward=fwd_big)
        del Rb, ob

    lat_ms = np.array(lat) * 1e3
    solves_per_s = B * args.steps / total
    psi_tflops = flops / total / 1e12
    result = {
        "metric": METRIC,
        "value": round(solves_per_s, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16 split halves + f32", "bf16": "bf16 split halves + f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "cost": args.cost, "bound": args.bound,
                   "precision": args.precision, "max_outer": args.max_outer,
                   "kappa_b": args.kappa_b, "P": P, "Q": Q, "batch": B,
                   "nsamples": sc.N, "n_sources": int(len(sc.src_pix)), "lsqr_tol": args.tol,
                   "contractions": "fp32 MFMA 16x16x4, fp64 Cholesky and LSQR scalars"},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
        "psi_tflops": round(psi_tflops, 4),
        "psi_dense_count_over_fp32_peak": round(psi_tflops / PEAK_FP32_MFMA_TFLOPS, 5),
        "solve": {k: stats[k] for k in ("status", "outer_iters", "adds", "drops", "lsqr_iters_total",
                                        "nF", "nU", "rel_residual")},
        # one solve's time over its LSQR iterations: an upper bound of the latency of one
        # iteration (the outer steps' other work and the multiplier kernels are included)
        "us_per_lsqr_iteration_bound": round(total / (B * args.steps) * 1e6 / max(stats["lsqr_iters_total"], 1), 3),
        "forward_full_grid": forward_full,
        "roofline": {"kernel": kname,
                     "bound": "mfma", "achieved": round(exec_flops / t_kernel / 1e12, 4),
                     "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(exec_flops / t_kernel / 1e12 / PEAK_FP32_MFMA_TFLOPS, 5),
                     "frac_dense_count": round(achieved / PEAK_FP32_MFMA_TFLOPS, 5),
                     "traffic": measured_traffic() if args.config == "c1" else None,
                     "us_per_launch": round(t_kernel * 1e6, 3),
                     "timing": f"{timing} of {reps} back-to-back launches (span / {reps})",
                     "us_device_launch_alone": round(t_alone * 1e6, 3),
                     "flops_per_launch": kflops, "mfma_issued_flops_per_launch": exec_flops,
                     "mfma_issued_frac": round(exec_flops / t_kernel / 1e12 / PEAK_FP32_MFMA_TFLOPS, 5)},
    }
    if big is not None:
        result["roofline_full_size"] = big
    if batched is not None:
        result["batched"] = batched
    if sequential is not None:
        result["batch"] = {"requests": B, "solves_per_s_one_by_one": round(sequential, 4),
                           "latency": "p50/p99 are of one batched call (all B requests)",
                           "solve": "request 0's statistics; psi_tflops counts all requests"}
    if not args.no_cpu:
        base, ref = cpu_baseline(sc, tol_oracle=1e-8, cost=args.cost, bound=args.bound, kappa_b=args.kappa_b,
                                 max_outer=args.max_outer)
        result["cpu_baseline"] = base
        s = sigma.cpu().numpy().astype(np.float64)
        st = state.cpu().numpy()
        result["parity"] = {
            "rel_image_err": float(np.linalg.norm(s - ref.sigma) / np.linalg.norm(ref.sigma)),
            "same_sets": bool(np.array_equal(st, ref.state)),
            "oracle_rel_residual": ref.rel_residual,
        }
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

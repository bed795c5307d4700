"""Python binding of the clsimg C ABI (include/clsimg.h).

Argument marshalling only: every step of every call runs in the HIP library
``libclsimg.so`` built next to this file.  PyTorch supplies device memory and
the current HIP stream; nothing here computes on the host.  If the library is
missing the import fails loudly (build it with ``python -m
paper_1505_01348_amd.build``).
"""

from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libclsimg.so")

OK, WMAXOUTER, WITNLIM, WCYCLE = 0, 1, 2, 3
EINVAL, ENOTPD, ENOMEM, EHIP, ENOTSUP, EWORKSPACE = -1, -2, -3, -4, -5, -6
BOUND_MVDR, BOUND_MF, BOUND_NONE = 0, 1, 2
FP32, FP16, BF16 = 0, 1, 2
COST_LS, COST_PWLS = 0, 1
LOOP_AUTO, LOOP_HOST = 0, 1
LSQR_AUTO, LSQR_ONE_WG, LSQR_COOP, LSQR_TWO_KERNEL = 0, 1, 2, 3
STATE_L, STATE_F, STATE_U = 0, 1, 2
MAX_P = 288

EXPORTED = ("clsimg_default_opts", "clsimg_create", "clsimg_destroy", "clsimg_dirty_image",
            "clsimg_dirty_image_timed", "clsimg_dirty_image_noalloc", "clsimg_kernel_timing", "clsimg_autotune", "clsimg_set_beam_tiles", "clsimg_mvdr_bound", "clsimg_forward", "clsimg_adjoint", "clsimg_solve",
            "clsimg_solve_batch", "clsimg_solve_multi", "clsimg_solve_offgrid", "clsimg_server_create", "clsimg_server_submit", "clsimg_server_poll",
            "clsimg_server_query", "clsimg_server_destroy", "clsimg_strerror")


class CArray(C.Structure):
    _fields_ = [("P", C.c_int32), ("pos_xy", C.POINTER(C.c_double)), ("lam", C.c_double)]


class CGrid(C.Structure):
    _fields_ = [("nl", C.c_int32), ("nm", C.c_int32), ("l0", C.c_double), ("dl", C.c_double),
                ("m0", C.c_double), ("dm", C.c_double)]


class COpts(C.Structure):
    _fields_ = [("bound", C.c_int32), ("C", C.c_double), ("kappa_b", C.c_double),
                ("kappa_d", C.c_double), ("nsamples", C.c_int64), ("atol", C.c_double),
                ("btol", C.c_double), ("conlim", C.c_double), ("itnlim", C.c_int32),
                ("max_outer", C.c_int32), ("precision", C.c_int32), ("cost", C.c_int32),
                ("loop", C.c_int32), ("lsqr_engine", C.c_int32), ("hand_over_free", C.c_int32),
                ("trace", C.c_int32), ("batch_graph", C.c_int32)]


class CStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32), ("adds", C.c_int32),
                ("drops", C.c_int32), ("lsqr_iters_total", C.c_int32),
                ("lsqr_itnlim_hits", C.c_int32), ("nF", C.c_int32), ("nU", C.c_int32),
                ("rel_residual", C.c_double), ("objective", C.c_double),
                ("min_margin_lambda", C.c_double), ("min_margin_z", C.c_double),
                ("psi_flops", C.c_double)]


class CRequest(C.Structure):
    _fields_ = [("R", C.c_void_p), ("array", CArray), ("grid", CGrid), ("noise_diag", C.c_void_p),
                ("sigma", C.c_void_p), ("state", C.c_void_p), ("mf", C.c_void_p), ("gamma", C.c_void_p),
                ("stats", CStats)]


class CBlock(C.Structure):
    _fields_ = [("R", C.c_void_p), ("array", CArray), ("noise_diag", C.c_void_p)]


class CServerInfo(C.Structure):
    _fields_ = [("pending", C.c_int32), ("active", C.c_int32), ("worker_queued", C.c_int32),
                ("ready", C.c_int32), ("submitted", C.c_int64), ("admitted", C.c_int64),
                ("completed", C.c_int64), ("step_rounds", C.c_int64), ("arena_bytes", C.c_size_t),
                ("arena_used", C.c_size_t), ("arena_peak", C.c_size_t)]


class ClsimgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libclsimg.so and declare its signatures; raises if it is absent."""
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run python -m paper_1505_01348_amd.build)")
    lib = C.CDLL(path)
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    lib.clsimg_default_opts.argtypes = [C.POINTER(COpts)]
    lib.clsimg_default_opts.restype = None
    lib.clsimg_create.argtypes = [C.POINTER(vp), i32, sz]
    lib.clsimg_destroy.argtypes = [vp]
    lib.clsimg_dirty_image.argtypes = [vp, vp, C.POINTER(CArray), C.POINTER(CGrid), i32, vp, vp]
    lib.clsimg_dirty_image_timed.argtypes = [vp, vp, C.POINTER(CArray), C.POINTER(CGrid), i32, vp, vp, vp, vp]
    lib.clsimg_dirty_image_noalloc.argtypes = [vp, vp, C.POINTER(CArray), C.POINTER(CGrid), i32, vp, vp]
    lib.clsimg_kernel_timing.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(i32)]
    lib.clsimg_autotune.argtypes = [vp, C.POINTER(CArray), C.POINTER(CGrid), i32, C.POINTER(i32),
                                    C.POINTER(C.c_float), vp]
    lib.clsimg_set_beam_tiles.argtypes = [vp, i32, i32, i32]
    lib.clsimg_mvdr_bound.argtypes = [vp, vp, C.POINTER(CArray), C.POINTER(CGrid), C.POINTER(COpts),
                                      vp, vp]
    lib.clsimg_forward.argtypes = [vp, C.POINTER(CArray), C.POINTER(CGrid), vp, vp, i32, vp, vp]
    lib.clsimg_adjoint.argtypes = [vp, C.POINTER(CArray), C.POINTER(CGrid), vp, vp, i32, vp, vp]
    lib.clsimg_solve_batch.argtypes = [vp, i32, C.POINTER(CRequest), C.POINTER(COpts), vp]
    lib.clsimg_solve.argtypes = [vp, vp, C.POINTER(CArray), C.POINTER(CGrid), vp, C.POINTER(COpts),
                                 vp, vp, vp, vp, vp, vp, C.POINTER(CStats), vp]
    lib.clsimg_solve_multi.argtypes = [vp, i32, C.POINTER(CBlock), C.POINTER(CGrid), C.POINTER(COpts), vp, vp,
                                       vp, vp, C.POINTER(CStats), vp]
    lib.clsimg_solve_offgrid.argtypes = [vp, vp, C.POINTER(CArray), C.POINTER(CGrid), vp, C.POINTER(COpts), i32,
                                         vp, vp, vp, vp, vp, C.POINTER(CStats), vp]
    lib.clsimg_server_create.argtypes = [C.POINTER(vp), i32, i32, sz, i32, i32, C.POINTER(COpts)]
    lib.clsimg_server_submit.argtypes = [vp, C.POINTER(CRequest), C.POINTER(C.c_int64)]
    lib.clsimg_server_poll.argtypes = [vp, i32, C.POINTER(C.c_int64), i32, C.POINTER(i32)]
    lib.clsimg_server_query.argtypes = [vp, C.POINTER(CServerInfo)]
    lib.clsimg_server_destroy.argtypes = [vp]
    lib.clsimg_strerror.argtypes = [C.c_int]
    lib.clsimg_strerror.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("clsimg_default_opts", "clsimg_strerror"):
            getattr(lib, name).restype = C.c_int
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def strerror(status: int) -> str:
    return lib().clsimg_strerror(int(status)).decode()


@dataclasses.dataclass
class Options:
    bound: int = BOUND_MVDR
    C: float = 1.0
    kappa_b: float = 0.0
    kappa_d: float = 6.0
    nsamples: int = 0
    atol: float = 1e-6
    btol: float = 1e-6
    conlim: float = 1e8
    itnlim: int = -1
    max_outer: int = -1
    precision: int = FP32
    cost: int = COST_LS
    loop: int = LOOP_AUTO
    lsqr_engine: int = LSQR_AUTO
    hand_over_free: int = 0
    trace: int = 0
    batch_graph: int = 0

    def to_c(self) -> COpts:
        return COpts(self.bound, self.C, self.kappa_b, self.kappa_d, self.nsamples, self.atol,
                     self.btol, self.conlim, self.itnlim, self.max_outer, self.precision, self.cost,
                     self.loop, self.lsqr_engine, self.hand_over_free, self.trace, self.batch_graph)


def default_options() -> Options:
    o = COpts()
    lib().clsimg_default_opts(C.byref(o))
    return Options(o.bound, o.C, o.kappa_b, o.kappa_d, o.nsamples, o.atol, o.btol, o.conlim,
                   o.itnlim, o.max_outer, o.precision, o.cost, o.loop, o.lsqr_engine, o.hand_over_free,
                   o.trace, o.batch_graph)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, numel, name, device):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t


class Geometry:
    """Antenna positions (metres), wavelength and pixel grid of one problem."""

    def __init__(self, pos_xy, lam, grid):
        self.pos = np.ascontiguousarray(np.asarray(pos_xy, dtype=np.float64).reshape(-1, 2))
        self.lam = float(lam)
        nl, nm, l0, dl, m0, dm = grid
        self.grid = (int(nl), int(nm), float(l0), float(dl), float(m0), float(dm))
        self.c_array = CArray(self.pos.shape[0], self.pos.ctypes.data_as(C.POINTER(C.c_double)),
                              self.lam)
        self.c_grid = CGrid(*self.grid)

    @property
    def P(self):
        return self.pos.shape[0]

    @property
    def Q(self):
        return self.grid[0] * self.grid[1]


class Context:
    """One clsimg context on one device (not thread safe; one per stream)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.device = int(device)
        self._lib = lib()
        h = C.c_void_p()
        st = self._lib.clsimg_create(C.byref(h), self.device, int(hbm_budget))
        if st != OK:
            raise ClsimgError(st, "clsimg_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.clsimg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st, where, allow_warn=False):
        if st < 0 or (st > 0 and not allow_warn):
            raise ClsimgError(st, where)
        return st

    def dirty_image(self, R, geo: Geometry, mf=None, precision: int = FP32):
        dev = self.device
        _need(R, torch.complex64, geo.P * geo.P, "R", dev)
        mf = torch.empty(geo.Q, dtype=torch.float32, device=R.device) if mf is None else mf
        _need(mf, torch.float32, geo.Q, "mf", dev)
        self._check(self._lib.clsimg_dirty_image(self._h, _ptr(R), C.byref(geo.c_array),
                                                 C.byref(geo.c_grid), int(precision), _ptr(mf), _stream()),
                    "clsimg_dirty_image")
        return mf

    def kernel_timing(self, enable: bool):
        """clsimg_kernel_timing: (ms, launches) of the multiplier kernel accumulated
        since the previous call; `enable` sets the mode for later solves."""
        ms, n = C.c_double(), C.c_int32()
        self._check(self._lib.clsimg_kernel_timing(self._h, int(bool(enable)), C.byref(ms), C.byref(n)),
                    "clsimg_kernel_timing")
        return ms.value, n.value

    def dirty_image_noalloc(self, R, geo: Geometry, mf, precision: int = FP32):
        """clsimg_dirty_image_noalloc: the dirty image into the caller's `mf`
        with the library's static workspace (no allocation in the call)."""
        dev = self.device
        _need(R, torch.complex64, geo.P * geo.P, "R", dev)
        _need(mf, torch.float32, geo.Q, "mf", dev)
        self._check(self._lib.clsimg_dirty_image_noalloc(self._h, _ptr(R), C.byref(geo.c_array), C.byref(geo.c_grid),
                                                         int(precision), _ptr(mf), _stream()),
                    "clsimg_dirty_image_noalloc")
        return mf

    def dirty_image_timed(self, R, geo: Geometry, start, stop, mf=None, precision: int = FP32):
        """dirty_image with the kernels' own device timestamps recorded into two
        timing events (torch.cuda.Event(enable_timing=True)); start.elapsed_time(stop)
        is then the kernels' device time in ms."""
        dev = self.device
        _need(R, torch.complex64, geo.P * geo.P, "R", dev)
        mf = torch.empty(geo.Q, dtype=torch.float32, device=R.device) if mf is None else mf
        _need(mf, torch.float32, geo.Q, "mf", dev)
        for ev in (start, stop):  # torch creates the HIP event at its first record
            if not ev.cuda_event:
                ev.record()
        self._check(self._lib.clsimg_dirty_image_timed(self._h, _ptr(R), C.byref(geo.c_array), C.byref(geo.c_grid),
                                                       int(precision), _ptr(mf), C.c_void_p(start.cuda_event),
                                                       C.c_void_p(stop.cuda_event), _stream()),
                    "clsimg_dirty_image_timed")
        return mf

    def autotune(self, geo: Geometry, precision: int = FP32):
        """Time 2, 4 and 8 pixel tiles per workgroup of the GEMM-shaped beamformer
        for this array and grid; the fastest is kept in the context.
        Returns (tiles kept, [us for 2, 4, 8])."""
        chosen = C.c_int32(0)
        us = (C.c_float * 3)()
        self._check(self._lib.clsimg_autotune(self._h, C.byref(geo.c_array), C.byref(geo.c_grid), int(precision),
                                              C.byref(chosen), us, _stream()), "clsimg_autotune")
        return chosen.value, [float(x) for x in us]

    def set_beam_tiles(self, P: int, precision: int, tiles: int):
        self._check(self._lib.clsimg_set_beam_tiles(self._h, int(P), int(precision), int(tiles)),
                    "clsimg_set_beam_tiles")

    def mvdr_bound(self, R, geo: Geometry, opts: Options | None = None, gamma=None):
        dev = self.device
        _need(R, torch.complex64, geo.P * geo.P, "R", dev)
        opts = opts or default_options()
        gamma = torch.empty(geo.Q, dtype=torch.float32, device=R.device) if gamma is None else gamma
        _need(gamma, torch.float32, geo.Q, "gamma", dev)
        co = opts.to_c()
        self._check(self._lib.clsimg_mvdr_bound(self._h, _ptr(R), C.byref(geo.c_array),
                                                C.byref(geo.c_grid), C.byref(co), _ptr(gamma),
                                                _stream()), "clsimg_mvdr_bound")
        return gamma

    def forward(self, geo: Geometry, v, idx=None, Y=None):
        dev = self.device
        n = v.numel()
        _need(v, torch.float32, None, "v", dev)
        if idx is not None:
            _need(idx, torch.int32, n, "idx", dev)
        Y = torch.empty((geo.P, geo.P), dtype=torch.complex64, device=v.device) if Y is None else Y
        _need(Y, torch.complex64, geo.P * geo.P, "Y", dev)
        self._check(self._lib.clsimg_forward(self._h, C.byref(geo.c_array), C.byref(geo.c_grid),
                                             _ptr(idx), _ptr(v), n, _ptr(Y), _stream()),
                    "clsimg_forward")
        return Y

    def adjoint(self, geo: Geometry, U, idx=None, n=None, g=None):
        dev = self.device
        _need(U, torch.complex64, geo.P * geo.P, "U", dev)
        if idx is not None:
            _need(idx, torch.int32, None, "idx", dev)
            n = idx.numel()
        elif n is None:
            n = geo.Q
        g = torch.empty(n, dtype=torch.float32, device=U.device) if g is None else g
        _need(g, torch.float32, n, "g", dev)
        self._check(self._lib.clsimg_adjoint(self._h, C.byref(geo.c_array), C.byref(geo.c_grid),
                                             _ptr(U), _ptr(idx), n, _ptr(g), _stream()),
                    "clsimg_adjoint")
        return g

    def solve(self, R, geo: Geometry, opts: Options, noise_diag=None, sigma0=None, state0=None,
              sigma=None, state=None, mf=None, gamma=None):
        """Returns (sigma, state, mf, gamma, stats dict); warnings are in stats['status']."""
        dev = self.device
        _need(R, torch.complex64, geo.P * geo.P, "R", dev)
        Q = geo.Q
        if noise_diag is not None:
            _need(noise_diag, torch.float32, geo.P, "noise_diag", dev)
        if sigma0 is not None or state0 is not None:
            _need(sigma0, torch.float32, Q, "sigma0", dev)
            _need(state0, torch.uint8, Q, "state0", dev)
        mk = lambda t, dt: torch.empty(Q, dtype=dt, device=R.device) if t is None else t  # noqa: E731
        sigma, state = mk(sigma, torch.float32), mk(state, torch.uint8)
        mf, gamma = mk(mf, torch.float32), mk(gamma, torch.float32)
        for t, dt, name in ((sigma, torch.float32, "sigma"), (state, torch.uint8, "state"),
                            (mf, torch.float32, "mf"), (gamma, torch.float32, "gamma")):
            _need(t, dt, Q, name, dev)
        co = opts.to_c()
        stats = CStats()
        st = self._lib.clsimg_solve(self._h, _ptr(R), C.byref(geo.c_array), C.byref(geo.c_grid),
                                    _ptr(noise_diag), C.byref(co), _ptr(sigma0), _ptr(state0),
                                    _ptr(sigma), _ptr(state), _ptr(mf), _ptr(gamma), C.byref(stats),
                                    _stream())
        self._check(st, "clsimg_solve", allow_warn=True)
        out = {f: getattr(stats, f) for f, _ in CStats._fields_}
        return sigma, state, mf, gamma, out


    def solve_multi(self, blocks, opts: Options, sigma=None, state=None, mf=None, gamma=None):
        """K covariance blocks over one grid: blocks is a list of dicts with R,
        geo (positions and wavelength of the block; every geo has the same
        grid) and optional noise_diag.  Returns (sigma, state, mf, gamma, stats)."""
        dev = self.device
        K = len(blocks)
        geo0 = blocks[0]["geo"]
        Q = geo0.Q
        arr = (CBlock * K)()
        for k, b in enumerate(blocks):
            geo = b["geo"]
            if geo.grid != geo0.grid:
                raise ValueError("every block must use the same pixel grid")
            _need(b["R"], torch.complex64, geo.P * geo.P, "R", dev)
            nd = b.get("noise_diag")
            if nd is not None:
                _need(nd, torch.float32, geo.P, "noise_diag", dev)
            arr[k].R = b["R"].data_ptr()
            arr[k].array = geo.c_array
            arr[k].noise_diag = None if nd is None else nd.data_ptr()
        mk = lambda t, dt: torch.empty(Q, dtype=dt, device=f"cuda:{dev}") if t is None else t  # noqa: E731
        sigma, state = mk(sigma, torch.float32), mk(state, torch.uint8)
        mf, gamma = mk(mf, torch.float32), mk(gamma, torch.float32)
        for t, dt, name in ((sigma, torch.float32, "sigma"), (state, torch.uint8, "state"),
                            (mf, torch.float32, "mf"), (gamma, torch.float32, "gamma")):
            _need(t, dt, Q, name, dev)
        st_c = CStats()
        co = opts.to_c()
        st = self._lib.clsimg_solve_multi(self._h, K, arr, C.byref(geo0.c_grid), C.byref(co), _ptr(sigma),
                                          _ptr(state), _ptr(mf), _ptr(gamma), C.byref(st_c), _stream())
        if st < 0:
            self._check(st, "clsimg_solve_multi")
        stats = {f: getattr(st_c, f) for f, _ in CStats._fields_}
        return sigma, state, mf, gamma, stats

    def solve_offgrid(self, R, geo: Geometry, opts: Options, rounds: int = 3, noise_diag=None):
        """Solve with the off-grid correction of the free pixels.  Returns
        (sigma, state, offsets (Q x 2: delta_l, delta_m), mf, gamma, stats)."""
        dev = self.device
        _need(R, torch.complex64, geo.P * geo.P, "R", dev)
        if noise_diag is not None:
            _need(noise_diag, torch.float32, geo.P, "noise_diag", dev)
        Q = geo.Q
        mk = lambda dt, n=Q: torch.empty(n, dtype=dt, device=R.device)  # noqa: E731
        sigma, state, offsets = mk(torch.float32), mk(torch.uint8), mk(torch.float32, 2 * Q)
        mf, gamma = mk(torch.float32), mk(torch.float32)
        st_c = CStats()
        co = opts.to_c()
        st = self._lib.clsimg_solve_offgrid(self._h, _ptr(R), C.byref(geo.c_array), C.byref(geo.c_grid),
                                            _ptr(noise_diag), C.byref(co), int(rounds), _ptr(sigma), _ptr(state),
                                            _ptr(offsets), _ptr(mf), _ptr(gamma), C.byref(st_c), _stream())
        if st < 0:
            self._check(st, "clsimg_solve_offgrid")
        stats = {f: getattr(st_c, f) for f, _ in CStats._fields_}
        return sigma, state, offsets.view(Q, 2), mf, gamma, stats

    def solve_batch(self, requests, opts: Options):
        """Batched solve of independent problems with the same P (each a dict with
        R, geo and optional noise_diag / sigma / state / mf / gamma tensors).
        Returns (overall status, list of (sigma, state, mf, gamma, stats dict))."""
        dev = self.device
        n = len(requests)
        arr = (CRequest * n)()
        keep, outs = [], []
        for i, rq in enumerate(requests):
            R, geo = rq["R"], rq["geo"]
            _need(R, torch.complex64, geo.P * geo.P, "R", dev)
            Q = geo.Q
            nd = rq.get("noise_diag")
            if nd is not None:
                _need(nd, torch.float32, geo.P, "noise_diag", dev)
            mk = lambda t, dt: torch.empty(Q, dtype=dt, device=R.device) if t is None else t  # noqa: E731
            sigma, state = mk(rq.get("sigma"), torch.float32), mk(rq.get("state"), torch.uint8)
            mf, gamma = mk(rq.get("mf"), torch.float32), mk(rq.get("gamma"), torch.float32)
            for t, dt, name in ((sigma, torch.float32, "sigma"), (state, torch.uint8, "state"),
                                (mf, torch.float32, "mf"), (gamma, torch.float32, "gamma")):
                _need(t, dt, Q, name, dev)
            arr[i].R = R.data_ptr()
            arr[i].array = geo.c_array
            arr[i].grid = geo.c_grid
            arr[i].noise_diag = None if nd is None else nd.data_ptr()
            arr[i].sigma, arr[i].state = sigma.data_ptr(), state.data_ptr()
            arr[i].mf, arr[i].gamma = mf.data_ptr(), gamma.data_ptr()
            keep.append(geo)
            outs.append((sigma, state, mf, gamma))
        co = opts.to_c()
        st = self._lib.clsimg_solve_batch(self._h, n, arr, C.byref(co), _stream())
        if st < 0 and st != ENOTSUP:
            self._check(st, "clsimg_solve_batch")
        res = []
        for i in range(n):
            stats = {f: getattr(arr[i].stats, f) for f, _ in CStats._fields_}
            res.append(outs[i] + (stats,))
        return st, res


class Server:
    """Continuous-batching solver (clsimg_server_*): submit requests at any time,
    poll for finished ones.  A request is a dict like those of
    ``Context.solve_batch``; its tensors and geometry are kept alive here until
    its ticket is returned.  Use from one thread."""

    def __init__(self, opts: Options, device: int = 0, max_slots: int = 64, hbm_budget: int = 1 << 30,
                 steps_per_poll: int = 16, workers: int = 1):
        self.device = int(device)
        self._lib = lib()
        h = C.c_void_p()
        co = opts.to_c()
        st = self._lib.clsimg_server_create(C.byref(h), self.device, int(max_slots), int(hbm_budget),
                                            int(steps_per_poll), int(workers), C.byref(co))
        if st != OK:
            raise ClsimgError(st, "clsimg_server_create")
        self._h = h
        self._live = {}  # ticket -> (CRequest, tensors, geometry)

    def submit(self, rq) -> int:
        R, geo = rq["R"], rq["geo"]
        dev = self.device
        _need(R, torch.complex64, geo.P * geo.P, "R", dev)
        Q = geo.Q
        nd = rq.get("noise_diag")
        if nd is not None:
            _need(nd, torch.float32, geo.P, "noise_diag", dev)
        mk = lambda t, dt: torch.empty(Q, dtype=dt, device=R.device) if t is None else t  # noqa: E731
        sigma, state = mk(rq.get("sigma"), torch.float32), mk(rq.get("state"), torch.uint8)
        mf, gamma = mk(rq.get("mf"), torch.float32), mk(rq.get("gamma"), torch.float32)
        for t, dt, name in ((sigma, torch.float32, "sigma"), (state, torch.uint8, "state"),
                            (mf, torch.float32, "mf"), (gamma, torch.float32, "gamma")):
            _need(t, dt, Q, name, dev)
        cr = CRequest()
        cr.R = R.data_ptr()
        cr.array = geo.c_array
        cr.grid = geo.c_grid
        cr.noise_diag = None if nd is None else nd.data_ptr()
        cr.sigma, cr.state, cr.mf, cr.gamma = sigma.data_ptr(), state.data_ptr(), mf.data_ptr(), gamma.data_ptr()
        # the server reads the inputs on its own streams: make the producer's work visible first
        torch.cuda.current_stream(R.device).synchronize()
        t = C.c_int64()
        st = self._lib.clsimg_server_submit(self._h, C.byref(cr), C.byref(t))
        if st != OK:
            raise ClsimgError(st, "clsimg_server_submit")
        self._live[t.value] = (cr, (R, nd, sigma, state, mf, gamma), geo)
        return t.value

    def poll(self, wait: bool = False, cap: int = 256):
        """Finished requests: list of (ticket, (sigma, state, mf, gamma, stats dict))."""
        arr = (C.c_int64 * cap)()
        n = C.c_int32()
        st = self._lib.clsimg_server_poll(self._h, 1 if wait else 0, arr, cap, C.byref(n))
        if st != OK:
            raise ClsimgError(st, "clsimg_server_poll")
        out = []
        for k in range(n.value):
            cr, ts, _ = self._live.pop(arr[k])
            stats = {f: getattr(cr.stats, f) for f, _ in CStats._fields_}
            out.append((arr[k], ts[2:] + (stats,)))
        return out

    def info(self):
        inf = CServerInfo()
        st = self._lib.clsimg_server_query(self._h, C.byref(inf))
        if st != OK:
            raise ClsimgError(st, "clsimg_server_query")
        return {f: getattr(inf, f) for f, _ in CServerInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.clsimg_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

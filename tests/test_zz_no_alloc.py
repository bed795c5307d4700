"""The allocation-free dirty image (clsimg_dirty_image_noalloc) against the
dirty image, through the C ABI (GPU).

Both run the same kernels on the same inputs, so the images must be the same
bits: two calls in a row per precision, the second with a smaller input
(288 antennas on 512 x 512 pixels, whose fragments of R sit in the static
workspace, then 48 antennas on 128 x 128, the register-resident
beamformer), and in FP32, split FP16 and split BF16.  A repeated call leaves
the device's free memory unchanged, and a geometry beyond the workspace is
refused with CLSIMG_ENOMEM.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_noalloc_dirty_image_is_the_dirty_image(gpu_lib):
    ctx = gpu_lib.Context(0)
    try:
        scenes = [synth.make_scene("c4"), synth.make_scene("c1")]
        for prec in (0, 1, 2):
            for sc in scenes:  # the second call of each pair has the smaller input
                print(f"case noalloc dirty image P={sc.P} Q={sc.Q} precision {prec}", flush=True)
                geo = gpu_lib.Geometry(sc.pos, sc.lam, sc.grid)
                R = torch.as_tensor(sc.R_hat32).cuda()
                out = torch.full((sc.Q,), float("nan"), dtype=torch.float32, device="cuda")
                ctx.dirty_image_noalloc(R, geo, out, precision=prec)
                ref = ctx.dirty_image(R, geo, precision=prec)
                torch.cuda.synchronize()
                assert torch.equal(out, ref), (sc.P, prec)
        # a repeated call allocates nothing
        sc = scenes[0]
        geo = gpu_lib.Geometry(sc.pos, sc.lam, sc.grid)
        R = torch.as_tensor(sc.R_hat32).cuda()
        out = torch.empty(sc.Q, dtype=torch.float32, device="cuda")
        ctx.dirty_image_noalloc(R, geo, out, precision=1)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(3):
            ctx.dirty_image_noalloc(R, geo, out, precision=1)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
    finally:
        ctx.close()


def test_noalloc_rejects_a_geometry_beyond_the_workspace(gpu_lib):
    ctx = gpu_lib.Context(0)
    try:
        rng = np.random.default_rng(5)
        P, nl, nm = 288, 4000, 200  # steering tables alone: 288 x 4200 x 8 bytes > 8 MiB
        pos = rng.uniform(-50.0, 50.0, size=(P, 2))
        geo = gpu_lib.Geometry(pos, 1.0, (nl, nm, -0.7, 1.4 / nl, -0.7, 1.4 / nm))
        R = torch.eye(P, dtype=torch.complex64, device="cuda")
        out = torch.empty(nl * nm, dtype=torch.float32, device="cuda")
        with pytest.raises(gpu_lib.ClsimgError) as ei:
            ctx.dirty_image_noalloc(R, geo, out)
        assert ei.value.status == gpu_lib.ENOMEM
    finally:
        ctx.close()

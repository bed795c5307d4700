"""CPU-side checks of the C ABI: the library loads and exports every symbol the
header declares, option defaults and error strings work, and no GPU is needed.
"""

import ctypes
import os
import re
import subprocess

import pytest

from paper_1505_01348_amd import clsimg

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "clsimg.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clsimg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert _declared_functions() == sorted(clsimg.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = clsimg.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_default_options_and_strerror():
    o = clsimg.default_options()
    assert o.bound == clsimg.BOUND_MVDR and o.C == 1.0 and o.kappa_b == 0.0 and o.kappa_d == 6.0
    assert o.itnlim == -1 and o.max_outer == -1 and o.precision == clsimg.FP32
    assert o.cost == clsimg.COST_LS
    assert clsimg.strerror(clsimg.ENOTPD).startswith("covariance")
    assert "not available" in clsimg.strerror(clsimg.ENOTSUP)
    assert clsimg.strerror(12345) == "unknown status"


def test_struct_layouts_match_c_abi(tmp_path):
    # compile the header with the host C compiler and compare every field offset
    structs = {"clsimg_array": clsimg.CArray, "clsimg_grid": clsimg.CGrid,
               "clsimg_opts": clsimg.COpts, "clsimg_stats": clsimg.CStats, "clsimg_request": clsimg.CRequest,
               "clsimg_server_info": clsimg.CServerInfo, "clsimg_block": clsimg.CBlock}
    cfields = {"clsimg_array": ["P", "pos_xy", "lambda"]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    for cname, cls in structs.items():
        names = cfields.get(cname, [f for f, _ in cls._fields_])
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in names:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = []
    for cname, cls in structs.items():
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f, _ in cls._fields_]
    assert got == want


def test_create_without_device_is_rejected():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = clsimg.load_library()
    h = ctypes.c_void_p()
    assert lib.clsimg_create(ctypes.byref(h), 0, 0) == clsimg.EINVAL
    assert lib.clsimg_destroy(None) == clsimg.EINVAL


def test_entry_points_reject_a_null_context():
    # every call checks its handle and required pointers before any device
    # work, so these run without a GPU
    lib = clsimg.load_library()
    E = clsimg.EINVAL
    n = None
    assert lib.clsimg_dirty_image(n, n, n, n, 0, n, n) == E
    assert lib.clsimg_dirty_image_timed(n, n, n, n, 0, n, n, n, n) == E
    assert lib.clsimg_dirty_image_noalloc(n, n, n, n, 0, n, n) == E
    assert lib.clsimg_kernel_timing(n, 1, n, n) == E
    assert lib.clsimg_mvdr_bound(n, n, n, n, n, n, n) == E
    assert lib.clsimg_forward(n, n, n, n, n, 0, n, n) == E
    assert lib.clsimg_adjoint(n, n, n, n, n, 0, n, n) == E
    assert lib.clsimg_solve(n, n, n, n, n, n, n, n, n, n, n, n, n, n) == E
    assert lib.clsimg_solve_batch(n, 1, n, n, n) == E
    assert lib.clsimg_solve_multi(n, 1, n, n, n, n, n, n, n, n, n) == E
    assert lib.clsimg_solve_offgrid(n, n, n, n, n, n, 3, n, n, n, n, n, n, n) == E
    assert lib.clsimg_autotune(n, n, n, 0, n, n, n) == E
    assert lib.clsimg_set_beam_tiles(n, 48, 0, 2) == E
    assert lib.clsimg_server_submit(n, n, n) == E
    assert lib.clsimg_server_poll(n, 0, n, 0, n) == E
    assert lib.clsimg_server_query(n, n) == E
    assert lib.clsimg_server_destroy(n) == E


def test_workspace_check_rejects_missing_or_short_buffers(tmp_path):
    # the check every entry point makes before its first launch (workspace.h):
    # a buffer that was never allocated, or is smaller than a kernel assumes,
    # is an error code and not a memory fault
    csrc = os.path.join(os.path.dirname(HEADER), "..", "paper_1505_01348_amd", "csrc")
    src = tmp_path / "ws.cpp"
    src.write_text("\n".join([
        '#include "workspace.h"',
        "#include <stdio.h>",
        "using namespace clsimg;",
        "int main() {",
        "  static char mem[4096];",
        "  DevBuf none, small, big;",
        "  small.ptr = mem; small.bytes = 256;",
        "  big.ptr = mem; big.bytes = 4096;",
        '  printf("%d\\n", need_all({{&big, 4096}, {&small, 256}}));',
        '  printf("%d\\n", need_all({{&big, 4096}, {&none, 1}}));',
        '  printf("%d\\n", need_all({{&small, 257}}));',
        '  printf("%d\\n", need_all({{nullptr, 0}}));',
        '  printf("%d\\n", need_all({}));',
        "  return 0;",
        "}"]))
    exe = tmp_path / "ws"
    subprocess.run(["g++", "-std=c++17", "-I", csrc, "-o", str(exe), str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    E = clsimg.EWORKSPACE
    assert got == [clsimg.OK, E, E, E, clsimg.OK]
    assert "workspace" in clsimg.strerror(E)

"""The C-ABI library loads and exports every symbol include/lbm.h declares;
host-only entry points behave as documented (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2408_00146_amd import cases
from paper_2408_00146_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_2408_00146_amd import build
        build.build(verbose=False)
    return lbm.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Offsets of every lbm_case / lbm_diag field in the ctypes mirror equal
    what a C compiler computes from include/lbm.h."""
    prog = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void){"]
    for struct, mirror in (("lbm_case", lbm.LbmCase), ("lbm_diag", lbm.LbmDiag)):
        prog.append(f'printf("%zu\\n", sizeof({struct}));')
        for name, _ in mirror._fields_:
            prog.append(f'printf("%zu\\n", offsetof({struct}, {name}));')
    prog.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for mirror in (lbm.LbmCase, lbm.LbmDiag):
        want.append(C.sizeof(mirror))
        want += [getattr(mirror, name).offset for name, _ in mirror._fields_]
    assert got == want


def test_workspace_bytes_host_only(L):
    c = cases.config_small_fp64()
    nb = lbm.workspace_bytes([c])
    pops = 2 * 36 * 128 * 64 * 8
    assert pops < nb < pops + (1 << 20)
    c32 = dict(c, precision=cases.FP32)
    c16 = dict(c, precision=cases.FP16S)
    assert lbm.workspace_bytes([c32]) < nb and lbm.workspace_bytes([c16]) < lbm.workspace_bytes([c32])
    assert L.lbm_workspace_bytes(None, 0) == 0


def test_tile_table(L):
    shapes, kinds = lbm.tile_shapes(), lbm.tile_kinds()
    assert len(shapes) == len(kinds) == L.lbm_tile_count()
    tiles = [s for s, k in zip(shapes, kinds) if k == "tile"]
    assert (64, 8) in tiles and (64, 4) in tiles and all(bx * by >= 256 for bx, by in tiles)
    assert set(kinds) == {"tile"}
    assert kinds[0] == "tile"
    assert L.lbm_tile_shape(99, None, None) == lbm.LBM_E_INVAL
    assert L.lbm_tile_kind(99) == lbm.LBM_E_INVAL


def _init_status(L, params, ws=1 << 20):
    arr = (lbm.LbmCase * 1)(lbm.make_case(params))
    h = C.c_void_p()
    return L.lbm_init(arr, 1, C.c_void_p(ws), 1 << 40, None, C.byref(h))


@pytest.mark.parametrize("bad", [dict(nx=3), dict(W=0.0), dict(nu_A=-1.0), dict(wall=[1, 0, 1, 1]),
                                 # FP16 storage narrower than one 64-node tile row
                                 dict(nx=63, precision=cases.FP16S),
                                 dict(precision=7), dict(D_psi=float("nan")),
                                 # one population buffer beyond the 4 GiB of 32-bit buffer offsets
                                 dict(nx=8192, ny=4096, precision=0), dict(nx=16384, ny=8192, precision=1)])
def test_invalid_cases_rejected_before_any_device_call(L, bad):
    rc = _init_status(L, dict(cases.config_small_fp64(), **bad))
    assert rc == lbm.LBM_E_INVAL
    assert L.lbm_last_error().decode()


def test_mixed_fp64_and_fp32_rejected(L):
    a = cases.config_small_fp64()
    b = dict(a, precision=cases.FP32)
    arr = (lbm.LbmCase * 2)(lbm.make_case(a), lbm.make_case(b))
    h = C.c_void_p()
    assert L.lbm_init(arr, 2, C.c_void_p(1 << 20), 1 << 40, None, C.byref(h)) == lbm.LBM_E_INVAL


def test_null_handle_errors(L):
    assert L.lbm_step(None, 1) == lbm.LBM_E_INVAL
    assert L.lbm_destroy(None) == lbm.LBM_OK


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        lbm.Solver(cases.config_small_fp64())

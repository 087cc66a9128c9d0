"""Memory safety of the kernels, checked on the CPU.

tests/replay compiles the library's device code for the host (shim.hpp in
place of the HIP headers) and runs the kernels of whole handles there with
every buffer-resource access range-checked -- voffset plus soffset, since
the hardware's own check covers the VGPR offset only -- every plain-pointer
buffer a separate AddressSanitizer-checked heap block, and every LDS index
checked by UBSan against its array.  The FP64 replay is also compared with
the oracle: the emulated kernels compute the same step.

Handles covered: the paper's flat-interface lattice with FP16 storage
(periodic, 64x101, three cases), an uneven batch mixing FP16 and FP32
storage with walls, Dirichlet T/psi and step budgets on both tile shapes, and
an FP64 ragged lattice with the paper's walls.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2408_00146_amd import cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "replay")
BUILD = os.path.join(HERE, "_build")
CXX = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def replay():
    if not os.path.exists(CXX):
        pytest.skip("no clang++")
    import sys

    sys.path.insert(0, HERE)
    import gen

    os.makedirs(BUILD, exist_ok=True)
    gen.generate(os.path.join(ROOT, "paper_2408_00146_amd", "csrc"), BUILD)
    shutil.copy(os.path.join(HERE, "shim.hpp"), BUILD)
    exe = os.path.join(BUILD, "replay")
    subprocess.run([CXX, "-std=c++20", "-O1", "-g", "-fsanitize=address,bounds", "-fno-sanitize-recover=bounds",
                    "-I", BUILD, "-I", os.path.join(ROOT, "include"), "-Wno-unused", "-o", exe,
                    os.path.join(HERE, "replay.cpp"), "-lpthread"], check=True)
    return exe


def run(exe, ps, steps, cfg, tag):
    from paper_2408_00146_amd import lbm

    arr = (lbm.LbmCase * len(ps))(*[lbm.make_case(c) for c in ps])
    fn = os.path.join(BUILD, f"{tag}.bin")
    with open(fn, "wb") as f:
        f.write(bytes(arr))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe, fn, str(steps), str(cfg), os.path.join(BUILD, tag)], capture_output=True, text=True,
                       env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "out-of-range 0 " in r.stdout, r.stdout
    out = []
    for i, p in enumerate(ps):
        a = np.fromfile(os.path.join(BUILD, f"{tag}_{i}.bin")).reshape(6, p["ny"], p["nx"])
        out.append(dict(zip(("phi", "p", "ux", "uy", "T", "psi"), a)))
    return out


def test_fp16_flat_interface_handle(replay):
    ps = [dict(cases.flat_surfactant(pb, ny=101, nx=64), precision=cases.FP16S) for pb in (0.05, 0.15, 0.225)]
    out = run(replay, ps, 4, 1, "flat16")
    for o, pb in zip(out, (0.05, 0.15, 0.225)):
        assert np.all(np.isfinite(o["psi"])) and abs(float(o["psi"].min()) - pb) < 1e-2


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_mixed_storage_batch(replay, cfg):
    ps = [cases.channel(100, 52, 9.0, 4.0, sigma_TT=1e-3, beta_s=0.2, precision=cases.FP16S),
          cases.channel(70, 36, 6.0, 4.0, sigma_TT=1e-3, beta_s=0.2, precision=cases.FP32, max_steps=3),
          dict(cases.channel(131, 53, 9.0, 5.0, sigma_law=cases.SIGMA_PAPER, sigma_T=0.0, sigma_TT=2e-4, beta_s=0.3,
                             T_ref=0.5, precision=cases.FP32),
               wall=[1, 1, 0, 0], t_bc=[1, 1, 0, 0], psi_bc=[1, 1, 0, 0], psi_w=[0.4, 0.1, 0.0, 0.0],
               T0=1.0 - 0.5 / 131, gradT=-1.0 / 131, xT0=0.0, psi_bulk=0.1, xc=60.0, yc=4.0)]
    out = run(replay, ps, 4, cfg, f"mixed{cfg}")
    assert all(np.all(np.isfinite(o[k])) for o in out for k in o)


@pytest.mark.parametrize("cfg", [1, 2])
def test_fp64_replay_is_the_oracles_step(replay, oracle_mod, cfg):
    p = cases.channel(100, 52, 9.0, 4.0, sigma_TT=1e-3, beta_s=0.2)
    p.update(t_bc=[1, 1, 1, 1], psi_bc=[0, 0, 1, 1], psi_w=[0.0, 0.0, 0.2, 0.05])
    out = run(replay, [p], 3, cfg, f"fp64_{cfg}")[0]
    o = oracle_mod.Oracle(p)
    o.step(3)
    of = o.fields()
    for k in ("phi", "p", "T", "psi"):
        assert np.max(np.abs(out[k] - of[k])) <= 1e-12 * np.max(np.abs(of[k])), k
    du = np.hypot(out["ux"] - of["ux"], out["uy"] - of["uy"])
    assert np.max(du) <= 1e-12 * np.max(np.hypot(of["ux"], of["uy"]))

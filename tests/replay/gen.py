"""Generate host-compilable copies of the library's device sources.

The replay compiles the kernels themselves (csrc/lbm_device.hpp and the
kernel part of csrc/lbm.hip) as plain C++ for the CPU: HIP headers are
replaced by shim.hpp, whose buffer-resource intrinsics check every byte range
they touch (the scalar offset included), LDS becomes one static object per
block, and the 256 threads of a block run as CPU threads meeting at a
barrier.  Used by tests/test_replay_bounds.py only.
"""
import os
import re
import sys


def generate(csrc: str, out_dir: str) -> None:
    os.makedirs(out_dir, exist_ok=True)
    d = open(os.path.join(csrc, "lbm_device.hpp")).read()
    d = d.replace("#include <hip/hip_fp16.h>\n#include <hip/hip_runtime.h>\n", '#include "shim.hpp"\n')
    d = d.replace("using Rsrc = __amdgpu_buffer_rsrc_t;", "using Rsrc = ShimRsrc;")
    d = d.replace('asm volatile("" : "+v"(tid));', 'asm volatile("" : "+r"(tid));')
    with open(os.path.join(out_dir, "dev_host.hpp"), "w") as f:
        f.write(d)
    h = open(os.path.join(csrc, "lbm.hip")).read()
    h = h.replace("#include <hip/hip_runtime.h>\n", '#include "shim.hpp"\n')
    h = h.replace('#include "lbm_device.hpp"', '#include "dev_host.hpp"')
    h = re.sub(r"__attribute__\(\(amdgpu_waves_per_eu\([^;]*?\)\)\)\)\s*", "", h)
    h = h.replace("__shared__", "static")
    h = h.replace('asm volatile("" : "+v"(tid));', 'asm volatile("" : "+r"(tid));')
    head = h[:h.find("// ======================================================================= host")]
    i, j = h.find("namespace {"), h.find("using StepKernel")
    helpers = re.sub(r"#define HIPCHK[\s\S]*?while \(0\)\n", "", h[i:j]) + "}  // namespace\n"
    with open(os.path.join(out_dir, "lib_host.hpp"), "w") as f:
        f.write(head + "using namespace lbm;\n" + helpers)


if __name__ == "__main__":
    generate(sys.argv[1], sys.argv[2])

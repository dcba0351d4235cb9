"""In-tree build of libmcc_hip.so (HIP, gfx950) from csrc/."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmcc_hip.so")
SOURCES = ["mcc_collide_fp64.hip", "mcc_collide_fp32.hip", "mcc_collide_rel.hip",
           "mcc_collide_tan.hip", "mcc_collide_fp64_diag.hip", "mcc_collide_fp32_diag.hip",
           "mcc_collide_rel_diag.hip", "mcc_collide_fp64_nxn.hip", "mcc_collide_fp32_nxn.hip",
           "mcc_collide_rel_nxn.hip", "mcc_collide_fp64_dup.hip", "mcc_collide_fp32_dup.hip",
           "mcc_collide_rel_dup.hip", "mcc_aux.hip", "mcc_rebin.hip", "mcc_adjoint.hip",
           "mcc_api.hip"]
ARCH = os.environ.get("MCC_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fno-strict-aliasing", "--offload-arch=" + ARCH,
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def build(verbose: bool = False, jobs: int = 8, out: str = LIB, defines=(),
          build_dir: str = BUILD, csrc: str = CSRC) -> str:
    """Compile every HIP source and link the shared library (always rebuilds).
    `defines` adds -D options (e.g. MCC_PHASE_TIMING for the per-phase clock
    counters of a profiling build); `out`, `build_dir` and `csrc` place such
    a build apart from the library the package loads."""
    os.makedirs(build_dir, exist_ok=True)
    cc = _hipcc()
    dflags = ["-D" + d for d in defines]

    def one(src):
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        cmd = [cc, *FLAGS, *dflags, "-c", os.path.join(csrc, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-8000:]))
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-8000:])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libddpinn.so in-tree with hipcc for gfx950."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddpinn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 VALU forms are disabled for every HIP object
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# (source, extra flags, object): the train kernels of each of the four
# operators and two activation-stash policies, plain and with the general
# activation rule, each in a translation unit of their own, compiled in
# parallel
UNITS = [("kernels.hip", [], "kernels.o")] + \
        [("kernels.hip", ["-DDDP_TRAIN_PDE=%d" % pde, "-DDDP_TRAIN_RH=%d" % rh] + (["-DDDP_TRAIN_GA"] if ga else []),
          "kernels_pde%d_rh%d%s.o" % (pde, rh, "_ga" if ga else ""))
         for pde in range(4) for rh in range(2) for ga in (False, True)] + \
        [("probe.hip", [], "probe.o"), ("noalloc.hip", [], "noalloc.o"), ("ddpinn.cpp", [], "ddpinn.o")]


def _compile(unit, bdir):
    src, extra, obj = unit
    obj = os.path.join(bdir, obj)
    cmd = [HIPCC] + HIP_FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s %s:\n%s" % (src, " ".join(extra), r.stderr))
    return obj


def build(verbose=True):
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 8)) as ex:
        objs = list(ex.map(lambda u: _compile(u, bdir), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()

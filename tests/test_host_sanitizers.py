"""The host library under AddressSanitizer, UndefinedBehaviorSanitizer and
LeakSanitizer: ddpinn.cpp is compiled with g++ and the sanitizers and linked
with the kernel objects of the regular build into a host-only driver of the C
ABI (tests/host/plan_driver.cpp: set-up, validation errors, interface
conditions, activations, plans and their dumps); no call touches the GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_10013_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2104_10013_amd", "_build")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_host_library_under_sanitizers(tmp_path):
    from paper_2104_10013_amd import build as B
    objs = [os.path.join(BUILD, obj) for _, _, obj in B.UNITS if obj != "ddpinn.o"]
    if not shutil.which("g++") or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs g++ and the kernel objects of paper_2104_10013_amd.build.build()")
    lib_o, drv_o, exe = (str(tmp_path / n) for n in ("ddpinn_san.o", "driver.o", "driver"))
    common = ["g++", "-std=c++17", "-O1", "-g", "-w"] + SAN
    _run(common + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-fPIC", "-c",
                   os.path.join(CSRC, "ddpinn.cpp"), "-o", lib_o])
    _run(common + ["-c", os.path.join(ROOT, "tests", "host", "plan_driver.cpp"), "-o", drv_o])
    _run(["g++"] + SAN + ["-o", exe, drv_o, lib_o] + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out and "runtime error" not in out, out
    assert "ok: 0 unexpected return codes" in r.stdout

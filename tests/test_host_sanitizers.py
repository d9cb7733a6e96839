"""The host code of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The library sources are compiled as for libflb.so, with the sanitizers on
their host code only (the device code is built as usual), and linked into
tests/host_abi_check.cpp, which drives every host-side path the ABI has:
parameter validation and its rejections, size queries in both precisions,
constant tables, null handles, the batched layout and the
modified-equilibrium work sizes and limits.  The program must report no
failed expectation, and the sanitizers abort it on the first memory error or
undefined behaviour (halt on error).  Leak checking is off: the HIP runtime
keeps process-lifetime state.
"""

import os
import shlex
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1012_3632_amd", "csrc")
SOURCES = ["api.hip", "batch.hip", "kernels.hip", "adjoint.hip", "spectrum.hip", "modeq.hip",
           "probe.hip"]
# the sanitizer options go to the host compilation only
HOST_SAN = "-Xarch_host -fsanitize=address,undefined -Xarch_host -fno-sanitize-recover=undefined"


def _tool(name, fallback):
    for c in (shutil.which(name), fallback):
        if c and os.path.exists(c):
            return c
    return None


def test_host_abi_under_sanitizers(tmp_path):
    hipcc = _tool("hipcc", "/opt/rocm/bin/hipcc")
    clang = _tool("amdclang++", "/opt/rocm/llvm/bin/clang++")
    if not hipcc or not clang:
        pytest.skip("hipcc / clang++ not found")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             *shlex.split(HOST_SAN), "-I", os.path.join(ROOT, "include")]
    procs, objs = [], []
    for src in SOURCES:
        obj = str(tmp_path / (src + ".o"))
        procs.append((src, subprocess.Popen([hipcc, *flags, "-c", os.path.join(CSRC, src), "-o", obj],
                                            stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                            text=True)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, f"{src}:\n{out[-3000:]}"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    drv = str(tmp_path / "check.o")
    r = subprocess.run([clang, "-O1", "-g", "-std=c++17", *san, "-c",
                        os.path.join(ROOT, "tests", "host_abi_check.cpp"), "-o", drv],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "check")
    r = subprocess.run([clang, *san, *objs, drv, "-L/opt/rocm/lib", "-lamdhip64",
                        "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host ABI checks: 0 failed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr

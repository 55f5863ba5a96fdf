"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

runtime.cpp and coeffs.cpp are compiled with the sanitizers on their host side
only (each -fsanitize= option behind -Xarch_host; the device code is the
ordinary build's), linked with the kernels' objects and the driver
tests/host_sanitize.cpp into an executable, and run: the argument checks of
every entry point, the host collocation coefficients for M = 1..8, the NULL
handle paths.  No GPU is needed; a sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

from paper_2405_19994_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-4000:] + r.stderr[-4000:]
    return r


@pytest.fixture(scope="module")
def sanitized_exe(tmp_path_factory):
    if not (os.path.exists(CLANG) and shutil.which(B.hipcc()) or os.path.exists(B.hipcc())):
        pytest.skip("hipcc / clang++ not available")
    bdir = os.path.join(B.HERE, "_build")
    kernels = [os.path.join(bdir, os.path.splitext(n)[0] + ".o") for n in B.SOURCES
               if n.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        B.build()
    out = tmp_path_factory.mktemp("san")
    common = ["-O1", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
              f"-I{os.path.join(ROOT, 'include')}"]
    objs = []
    for src in ("runtime.cpp", "coeffs.cpp"):
        obj = str(out / (os.path.splitext(src)[0] + ".o"))
        _run([B.hipcc(), *common, *SAN_HOST, "-x", "hip", "-c", os.path.join(B.CSRC, src), "-o", obj])
        objs.append(obj)
    drv = str(out / "host_sanitize.o")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    _run([CLANG, "-O1", "-g", "-std=c++17", *san, f"-I{os.path.join(ROOT, 'include')}", "-c",
          os.path.join(ROOT, "tests", "host_sanitize.cpp"), "-o", drv])
    exe = str(out / "host_sanitize")
    _run([CLANG, *san, drv, *objs, *kernels, f"-L{ROCM}/lib", "-lamdhip64",
          f"-Wl,-rpath,{ROCM}/lib", "-o", exe])
    return exe


def test_host_code_is_clean_under_asan_and_ubsan(sanitized_exe):
    env = dict(os.environ)
    # the HIP runtime's own allocations at exit are not the library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sanitized_exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]

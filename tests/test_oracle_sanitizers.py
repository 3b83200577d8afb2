"""Sanitizer runs (CPU only).  The oracle (oracle/oracle.c) is built with gcc under
AddressSanitizer (with its leak check) and UndefinedBehaviorSanitizer, together with a driver
that calls its entry points on small inputs: every order and basis of Alg. 1, the explicit and
asymmetric grids, the Green's-function setups of Sec. 3, Alg. 2's chains and DFT, the ring
sum, Philox.  The C ABI's host logic is built the same way (hipcc, the sanitizers on the host
code only; the GPU code is compiled as usual and never runs here) and driven through every
argument check and error path that needs no device.  Any finding aborts the driver."""
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "2"}


def _run(exe, timeout):
    env = dict(os.environ)
    env.update(SAN_ENV)
    p = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=timeout)
    return p.returncode, p.stdout + p.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-fast-math", "-ffp-contract=off",
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    rc, out = _run(exe, 300)
    assert rc == 0, out
    assert "every call succeeded" in out
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out


CSRC = os.path.join(ROOT, "paper_1709_10314_amd", "csrc")
SOURCES = ["api.hip", "setup.hip", "sample.hip", "batch.hip", "rings.hip", "rings_fft.hip", "measure.hip"]


def _abi_library():
    """The library with sanitized host code, built once per source state under _build/."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)) + ["../../include/smf.h"]:
        p = os.path.join(CSRC, f)
        if os.path.isfile(p):
            h.update(f.encode())
            h.update(open(p, "rb").read())
    out = os.path.join(ROOT, "_build", "sanitize", h.hexdigest()[:16])
    lib = os.path.join(out, "libsmf_san.so")
    if os.path.exists(lib):
        return lib
    parent = os.path.dirname(out)
    if os.path.isdir(parent):   # builds of earlier source states
        for d in os.listdir(parent):
            shutil.rmtree(os.path.join(parent, d), ignore_errors=True)
    os.makedirs(out, exist_ok=True)
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include")]
    procs = [subprocess.Popen([HIPCC, *flags, "-c", os.path.join(CSRC, s), "-o", os.path.join(out, s + ".o")],
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for s in SOURCES]
    for p in procs:
        log = p.communicate(timeout=900)[0]
        assert p.returncode == 0, log.decode(errors="replace")[-2000:]
    objs = [os.path.join(out, s + ".o") for s in SOURCES]
    subprocess.run([HIPCC, "-shared", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", *objs, "-o", lib + ".tmp"], check=True, capture_output=True, timeout=600)
    os.replace(lib + ".tmp", lib)
    for o in objs:
        os.remove(o)
    return lib


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="hipcc / ROCm clang not found")
def test_c_abi_host_logic_under_address_and_undefined_sanitizers(tmp_path):
    lib = _abi_library()
    exe = str(tmp_path / "abi_san")
    subprocess.run([CLANG, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_sanitize_driver.c"), lib,
                    "-Wl,-rpath," + os.path.dirname(lib), "-o", exe], check=True, capture_output=True, timeout=300)
    rc, out = _run(exe, 300)
    assert rc == 0, out
    assert "every call returned an expected code" in out
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out

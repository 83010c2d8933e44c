"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer (host only; no GPU code is
built with them): the FP64 oracle, whose pin tests run again against a sanitized build, and the
library's host-side description builders (robot program, environment records, voxel
broadphase, point grid and clearance field, the specialisation source), linked with stand-ins
for the kernel launchers and driven without a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build", "sanitize")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _run_env(extra=None):
    # the sanitizer runtime goes first; libstdc++ with it, so that its C++ exception hooks are
    # in place before the interpreter loads C++ code
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    cxx = subprocess.check_output(["g++", "-print-file-name=libstdc++.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=f"{asan} {cxx}", ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.update(extra or {})
    return env


def test_oracle_pins_under_sanitizers():
    os.makedirs(BUILD, exist_ok=True)
    lib = os.path.join(BUILD, "liboracle_san.so")
    subprocess.check_call(["gcc", *SAN, "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared",
                           "-pthread", "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_oracle_fk.py", "test_oracle_clearance.py",
                                                      "test_oracle_validity.py", "test_oracle_cost.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests],
                       env=_run_env({"VK_ORACLE_LIB": lib}), cwd=ROOT, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout


def test_host_builders_under_sanitizers():
    from paper_2309_14545_amd import build
    os.makedirs(BUILD, exist_ok=True)
    lib = os.path.join(BUILD, "libvk_host_san.so")
    csrc = os.path.join(ROOT, "paper_2309_14545_amd", "csrc")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                           "-o", lib, os.path.join(csrc, "vk_api.cpp"),
                           os.path.join(ROOT, "tests", "sanitize", "launch_stubs.cpp"),
                           build.write_embed(), "-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc",
                           "-Wl,-rpath,/opt/rocm/lib"])
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize", "host_builders.py"), lib],
                       env=_run_env(), cwd=ROOT, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ok" in r.stdout

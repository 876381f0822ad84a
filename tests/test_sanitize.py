"""The FP64 oracle and the library's host-side code (argument checks, view layout, workspace
sizing, host k-means and seeding, nearest centre) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: both are rebuilt with the sanitizers (host code only;
no kernel runs here) and the oracle pins and the host tests run against those builds in a
child process with the sanitizer runtime preloaded. Any report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _runtime():
    found = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    return found[-1] if found else None


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed:\n{r.stdout[-4000:]}"
    return r.stdout


@pytest.mark.slow
def test_oracle_and_host_code_under_sanitizers(tmp_path):
    rt = _runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("the ROCm clang sanitizer runtime or hipcc is not installed")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-shared-libsan"]
    oracle_so = str(tmp_path / "libgs_oracle_san.so")
    # the oracle in plain C (no OpenMP in this build: one thread, the same arithmetic)
    _run([os.path.join(LLVM, "bin", "clang"), "-O1", "-g", *san, "-fPIC", "-shared", "-ffp-contract=off",
          "-std=gnu11", "-o", oracle_so, os.path.join(ROOT, "oracle", "gs_oracle.c"), "-lm"])
    # the library with the sanitizers on its host code only (each -fsanitize behind -Xarch_host)
    host = []
    for f in ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-shared-libsan"]:
        host += ["-Xarch_host", f]
    objs, procs = [], []
    for src in sorted(glob.glob(os.path.join(ROOT, "paper_2403_13806_amd", "csrc", "*.hip"))):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                                       "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host,
                                       "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out[-4000:]
    hip_so = str(tmp_path / "libgs_hip_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *host, "-o", hip_so, *objs])
    env = dict(os.environ, GS_HIP_LIB=hip_so, GS_ORACLE_LIB=oracle_so, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_oracle_pins.py", "test_oracle_kmeans_pins.py", "test_oracle_init_pins.py", "test_host.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", *tests, "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=1200)
    out = r.stdout
    print(out[-1500:])
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out

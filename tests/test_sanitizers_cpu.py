"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

* The oracle (plain C) is built with gcc's sanitizers together with
  tests/sanitize/oracle_driver.c, which runs every oracle entry point on seeded random
  graphs and checks invariants that hold for any graph.
* The library is built with the sanitizers on its host code only (hipcc: every
  -fsanitize= behind -Xarch_host; the device code is built as usual) and linked into
  tests/sanitize/abi_driver.c, which walks the C ABI's validation and error paths; on a
  machine without a GPU the calls that need the device report DEVICE.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_11655_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")


def _run(cmd, cwd, env=None, timeout=600):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
          os.path.join(ROOT, "oracle", "vdmc_oracle.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          "-o", exe], cwd=str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    r = _run([exe], cwd=str(tmp_path), env=env)
    assert "oracle sanitizer run ok" in r.stdout


def _asan_runtime_dir():
    base = os.path.join(ROCM, "llvm", "lib", "clang")
    for ver in sorted(os.listdir(base), reverse=True) if os.path.isdir(base) else []:
        d = os.path.join(base, ver, "lib", "linux")
        if os.path.exists(os.path.join(d, "libclang_rt.asan-x86_64.so")):
            return d
    return None


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain missing")
def test_abi_host_code_under_asan_ubsan(tmp_path):
    rt = _asan_runtime_dir()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    procs = []
    for f in srcs:
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-w", *san, "-c", os.path.join(CSRC, f), "-o", f + ".o"]
        procs.append((cmd, subprocess.Popen(cmd, cwd=str(tmp_path), stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
    for cmd, p in procs:
        out, err = p.communicate(timeout=900)
        assert p.returncode == 0, f"{' '.join(cmd)}\n{err[-3000:]}"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-shared-libsan", "-o", "libvdmc_asan.so", *[f + ".o" for f in srcs]],
         cwd=str(tmp_path))
    exe = str(tmp_path / "abi_driver")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-shared-libsan", "-fno-sanitize-recover=undefined",
          "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "abi_driver.c"),
          "-L" + str(tmp_path), "-lvdmc_asan", "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + rt, "-o", exe],
         cwd=str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")   # the HIP runtime keeps its allocations
    r = _run([exe], cwd=str(tmp_path), env=env, timeout=300)
    assert "ABI sanitizer run ok" in r.stdout

"""The C ABI's argument validation under host AddressSanitizer and UndefinedBehaviorSanitizer.

The translation units that hold the entry points' checks (abi.hip, misfit.hip, stream.hip) are rebuilt
with the sanitizers on their host code only, linked with the library's other objects into a
scratch library, and driven by tests/abi_sanitize.c through every validation path.  Nothing
reaches a GPU, so this runs on the CPU; a sanitizer report aborts the driver."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1309_6250_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
UNITS = ("abi.hip", "misfit.hip", "stream.hip")


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd[:3])} ... failed:\n{res.stdout[-3000:]}\n{res.stderr[-3000:]}"
    return res


@pytest.mark.timeout(600)
def test_validation_paths_clean_under_host_sanitizers(tmp_path):
    sources = {os.path.basename(f) for f in glob.glob(os.path.join(PKG, "csrc", "*.hip"))}
    objs = [os.path.join(PKG, "_build", f + ".o") for f in sorted(sources - set(UNITS))]
    objs = [o for o in objs if os.path.exists(o)]
    if len(objs) != len(sources) - len(UNITS):
        objs = []
    runtime = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not objs or not shutil.which(HIPCC) or not os.path.exists(CLANG) or not runtime:
        pytest.skip("needs the built library objects, hipcc, clang and its ASan runtime")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics", "-ffp-contract=off",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), *SAN]
    san_objs = []
    for unit in UNITS:
        out = str(tmp_path / (unit + ".san.o"))
        _run([HIPCC, *flags, "-c", os.path.join(PKG, "csrc", unit), "-o", out])
        san_objs.append(out)
    # the host code really is instrumented
    syms = _run(["nm", san_objs[0]]).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    lib = str(tmp_path / "libpwspline_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", lib, *san_objs, *objs])
    drv = str(tmp_path / "abi_sanitize")
    rt_dir = os.path.dirname(runtime[0])
    _run([CLANG, "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-shared-libsan",
          "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_sanitize.c"), "-o", drv,
          f"-L{tmp_path}", "-lpwspline_san", f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{rt_dir}", "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
    assert "all validation paths returned as documented" in res.stdout

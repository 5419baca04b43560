"""Host memory-safety checks (CPU tier): the oracle's C loops and the library's host-only
code (the native scheduler's decision functions and the entry points' argument checks)
built with AddressSanitizer and UBSan and run on random and extreme inputs
(tests/asan/*.c*), and the step rule's thread pool also under ThreadSanitizer.  Device
code is not instrumented."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN = os.path.join(ROOT, "tests", "asan")
PKG = os.path.join(ROOT, "paper_1205_2288_amd")
HIPCC = "/opt/rocm/bin/hipcc"


def _run(cmd, cwd):
    res = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout[-3000:]}\n{res.stderr[-3000:]}"
    return res


def test_oracle_under_address_sanitizer(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ASAN, "oracle_check.c"), "-lm", "-o", exe], tmp_path)
    res = _run([exe], tmp_path)
    assert "oracle host check ok" in res.stdout


def test_host_code_under_address_sanitizer(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    build_dir = os.path.join(PKG, "_build")
    if not os.path.isdir(build_dir):
        import importlib.util
        spec = importlib.util.spec_from_file_location("_b", os.path.join(PKG, "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    instrumented = ("scheduler.hip", "api.hip")
    objs = []
    for src in instrumented:
        obj = str(tmp_path / (src[:-4] + ".o"))
        _run([HIPCC, *flags, "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all", "-c", os.path.join(PKG, "csrc", src), "-o", obj], tmp_path)
        objs.append(obj)
    main = str(tmp_path / "abi_check.o")
    _run(["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c", os.path.join(ASAN, "abi_check.cpp"), "-o", main], tmp_path)
    rest = [os.path.join(build_dir, f) for f in sorted(os.listdir(build_dir))
            if f.endswith(".o") and f[:-2] + ".hip" not in instrumented]
    exe = str(tmp_path / "abi_check")
    _run([HIPCC, "--offload-arch=gfx950", "-fsanitize=address,undefined", "-fno-gpu-sanitize", main, *objs, *rest, "-o", exe], tmp_path)
    res = _run([exe], tmp_path)
    assert "host rule and argument check ok" in res.stdout


@pytest.mark.parametrize("sanitizer", ["address,undefined", "thread"])
def test_rule_pool_under_sanitizers(tmp_path, sanitizer):
    # the host threads of the step rule: every part once per call, a throwing part
    # rethrown only after the others have ended, the pool usable afterwards
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "rule_pool_check")
    _run(["g++", "-O1", "-g", "-std=c++17", "-pthread", f"-fsanitize={sanitizer}",
          "-I" + os.path.join(PKG, "csrc"), os.path.join(ASAN, "rule_pool_check.cpp"),
          "-o", exe], tmp_path)
    res = _run([exe], tmp_path)
    assert "rule pool check ok" in res.stdout

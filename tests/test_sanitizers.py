"""CPU sanitizer builds (no GPU): the C oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, driven over every exported function and edge shapes; and the
library's host layer (argument and workspace checks, handles, the plan's host side)
rebuilt with both sanitizers on its host code only, running the C ABI tests."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-O1", "-g", *SAN, os.path.join(ROOT, "oracle", "knn_oracle.c"),
                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all calls clean" in r.stdout


def _asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


def test_host_api_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    build = os.path.join(ROOT, "paper_2206_14286_amd", "_build")
    objs = [os.path.join(build, f"{n}.o") for n in ("knn_prepare", "knn_fused", "knn_select", "knn_resolve",
                                                    "knn_rerank_backward", "knn_approx")]
    rt = _asan_runtime()
    if not os.path.exists(HIPCC) or rt is None or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc, the clang ASan runtime and the library's kernel objects (build() first)")
    host_san = []
    for f in SAN:  # on the host compilation only: the device code is not instrumented
        host_san += ["-Xarch_host", f]
    api_o = str(tmp_path / "knn_api_san.o")
    lib = str(tmp_path / "libknn_san.so")
    common = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
    subprocess.run([HIPCC, *common, "-O1", "-g", *host_san, "-I", os.path.join(ROOT, "paper_2206_14286_amd", "csrc"),
                    "-x", "hip", "-c", os.path.join(ROOT, "paper_2206_14286_amd", "csrc", "knn_api.cpp"), "-o", api_o],
                   check=True, capture_output=True, text=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", *objs, api_o, "-o", lib],
                   check=True, capture_output=True, text=True)
    code = (
        "import sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import paper_2206_14286_amd.knn as k\n"
        f"k.LIB_PATH = {lib!r}\n"
        "import pytest\n"
        f"rc = pytest.main([{os.path.join(ROOT, 'tests', 'test_abi.py')!r}, '-q', '-m', 'not gpu', "
        "'-p', 'no:cacheprovider'])\n"
        "maps = open('/proc/self/maps').read()\n"
        f"assert {lib!r} in maps, 'the sanitized library was not the one loaded'\n"
        "sys.exit(rc)\n")
    env = {**os.environ, "LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0",
           "UBSAN_OPTIONS": "print_stacktrace=1"}
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout

"""The C ABI layer under AddressSanitizer (no GPU): abi.hip (argument validation, workspace
sizes, dispatch) is compiled with the sanitizer and linked with the plain build's kernel
objects, then the C program of tests/c/abi_smoke.c and every validation case of
tests/test_abi_host.py run against that build. Each must finish with no sanitizer report
(no kernel runs here)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2402_08273_amd import build as B  # noqa: E402

CLANG = "/opt/rocm/lib/llvm/bin/clang"


def _asan_runtime():
    out = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if out.returncode != 0 or not os.path.isfile(path):
        import glob

        hits = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = hits[0] if hits else ""
    return path


@pytest.fixture(scope="module")
def asan_lib():
    if not os.path.exists(CLANG) or not _asan_runtime():
        pytest.skip("no clang AddressSanitizer runtime")
    if B.sources_newer_than(B.LIB):
        pytest.skip("libramlt.so is not built from the current sources")
    return B.build_asan()


def _env(lib):
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit: leak reports are not about this code
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["RAMLT_LIBRARY"] = lib
    return env


def test_c_program_under_asan(asan_lib, tmp_path):
    exe = str(tmp_path / "abi_smoke_asan")
    libdir = os.path.dirname(asan_lib)
    subprocess.run([CLANG, "-std=c99", "-fsanitize=address", "-fno-omit-frame-pointer", "-g", "-I",
                    os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_smoke.c"), asan_lib,
                    f"-Wl,-rpath,{libdir}", "-o", exe], check=True, capture_output=True, text=True)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=_env(asan_lib))
    assert run.returncode == 0, run.stderr[-4000:]
    assert "AddressSanitizer" not in run.stderr, run.stderr[-4000:]
    assert "stats_null 1" in run.stdout


def test_validation_cases_under_asan(asan_lib):
    env = _env(asan_lib)
    env["LD_PRELOAD"] = _asan_runtime()
    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi_host.py")], capture_output=True, text=True,
                         timeout=600, env=env, cwd=ROOT)
    assert run.returncode == 0, (run.stdout[-3000:], run.stderr[-3000:])
    assert "AddressSanitizer" not in run.stderr + run.stdout, run.stderr[-4000:]
    assert " passed" in run.stdout

"""The boundary from C: include/ramlt.h compiles as strict C99 (-pedantic, no warnings) and
a C program linked against libramlt.so reaches every group of entry points (host-side
paths only: ABI version, workspace sizes, validation errors)."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2402_08273_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_c99_and_links(tmp_path):
    lib = os.path.dirname(_abi.LIB_PATH)
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libramlt.so not built")
    exe = str(tmp_path / "abi_smoke")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "abi_smoke.c"), "-L", lib, "-lramlt", f"-Wl,-rpath,{lib}", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=60).stdout
    got = dict(line.split(" ", 1) for line in out.strip().splitlines())
    assert got["abi"] == f"{ctypes.sizeof(_abi.RamltFrame)} {ctypes.sizeof(_abi.RamltFrame)}"
    for key in ("stats_null", "stats_noptr", "adapt_null", "qt_null", "perturb_bad", "rrmse_bad", "lens_bad",
                "lens_sort_bad"):
        assert int(got[key]) == _abi.RAMLT_EINVAL, key
    for key in ("last_error_set", "adapt_ws", "qt_ws", "rrmse_ws", "lens_ws", "lens_sort_ws"):
        assert got[key] == "1", key

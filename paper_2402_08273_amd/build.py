"""Build the gfx950 shared library ``libramlt.so`` in-tree with hipcc.

Usage: ``python -m paper_2402_08273_amd.build`` (also called by ``__graft_entry__.build()``).
"""

import os
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
LIB = os.path.join(PKG_DIR, "libramlt.so")
SOURCES = ["abi.hip", "batch.hip", "stats.hip", "filter.hip", "adapt.hip", "quadtree.hip", "perturb.hip", "chains.hip", "step.hip", "rrmse.hip", "filter_tiles_32x8.hip",
           "filter_tiles_32x16.hip", "filter_tiles_64x8.hip", "noalloc.hip"]
ARCH = "gfx950"


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def common_flags():
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Wno-unused-function",
        # packed fp32 VALU ops are disabled for all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
    ]


ASAN_LIB = os.path.join(PKG_DIR, "_build", "asan", "libramlt_asan.so")
# the C ABI layer (argument validation, workspace sizes, dispatch) under AddressSanitizer;
# every sanitizer flag is for the host pass only
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _compile_all(sources, obj_dir, extra, verbose):
    objs = []
    procs = []
    os.makedirs(obj_dir, exist_ok=True)
    for src in sources:
        obj = os.path.join(obj_dir, src.replace(".hip", ".o"))
        cmd = [hipcc()] + common_flags() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the device-only target feature; that note is noise
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed = True
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed")
    return objs


def _link(objs, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose=False, jobs=None):
    """Compile every source in parallel and link libramlt.so."""
    objs = _compile_all(SOURCES, os.path.join(PKG_DIR, "_build"), [], verbose)
    return _link(objs, LIB, verbose)


def build_asan(verbose=False):
    """ASAN_LIB: the library with its C ABI layer (abi.hip, host code only: it holds no
    kernels) compiled under AddressSanitizer and the kernel objects of the plain build, for
    host-side tests (load it into a process that carries the ASan runtime). Needs build()
    to have run."""
    kernels = [os.path.join(PKG_DIR, "_build", s.replace(".hip", ".o")) for s in SOURCES if s != "abi.hip"]
    missing = [o for o in kernels if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"build() first: {missing[0]} is missing")
    objs = _compile_all(["abi.hip"], os.path.join(PKG_DIR, "_build", "asan"), ["--offload-host-only"] + ASAN_FLAGS,
                        verbose)
    return _link(objs + kernels, ASAN_LIB, verbose)


def sources_newer_than(path):
    """True when a library source or header is newer than ``path`` (or it is missing)."""
    if not os.path.exists(path):
        return True
    t = os.path.getmtime(path)
    files = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(ROOT, "include", "ramlt.h")]
    return any(os.path.getmtime(f) > t for f in files if os.path.isfile(f))


if __name__ == "__main__":
    print(build_asan(verbose="-v" in sys.argv) if "--asan" in sys.argv else build(verbose="-v" in sys.argv))

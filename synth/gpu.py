"""Device-side generation of the synthetic render buffers (``synth/libsynth.so``), for frames
too large to generate with NumPy. Produces the same recipe as :mod:`synth.numpy_gen`
(checked against it in the GPU tests)."""

import ctypes
import os
import subprocess

import torch

from .numpy_gen import NOISE_CONST, NOISE_UNIFORM  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
SRC = os.path.join(_HERE, "csrc", "synth.hip")

_lib = None


def build(verbose=False):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = [os.path.join(rocm, "bin", "hipcc"), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off",
           SRC, "-o", LIB_PATH + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for synth.hip:\n" + r.stdout + r.stderr)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m synth.build`")
        lib = ctypes.CDLL(LIB_PATH)
        lib.synth_frame.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_void_p]
        lib.synth_frame.restype = ctypes.c_int
        lib.synth_reference.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_void_p]
        lib.synth_reference.restype = ctypes.c_int
        _lib = lib
    return _lib


def make_frame(W, H, S, seed, frame=0, noise=NOISE_UNIFORM, sigma=0.1, firefly_p=1e-3,
               feature_dtype=torch.float32, with_features=True, device="cuda"):
    """(radiance [3,S,H,W] fp32, features [7,S,H,W] or None) as device tensors."""
    rad = torch.empty((3, S, H, W), dtype=torch.float32, device=device)
    feat = torch.empty((7, S, H, W), dtype=feature_dtype, device=device) if with_features else None
    st = torch.cuda.current_stream().cuda_stream
    e = _load().synth_frame(rad.data_ptr(), None if feat is None else feat.data_ptr(),
                            int(feature_dtype == torch.float16), W, H, S, seed, frame, noise, sigma, firefly_p, st)
    if e != 0:
        raise RuntimeError(f"synth_frame failed with hip error {e}")
    return rad, feat


def make_reference(W, H, seed, frame=0, spp=4096, noise=NOISE_UNIFORM, sigma=0.1, firefly_p=1e-3, device="cuda"):
    ref = torch.empty((3, H, W), dtype=torch.float32, device=device)
    st = torch.cuda.current_stream().cuda_stream
    e = _load().synth_reference(ref.data_ptr(), W, H, spp, seed, frame, noise, sigma, firefly_p, st)
    if e != 0:
        raise RuntimeError(f"synth_reference failed with hip error {e}")
    return ref

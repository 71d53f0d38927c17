"""The whole path driven from C with no Python in the GPU process (tests/c/gpu_chain.c:
the HIP runtime allocates, libramlt computes), against the FP64 oracle run on the same
seeded inputs.

Screen grid: region_adapt (Algorithm 1) -> stats_accumulate (Appendix A) ->
filter_forward with the adapted lambda (Sec. 3.1, 5.3) -> filter_backward with the loss
seed fused -> rrmse (Sec. 8.2). Quadtree: lookups, adaptation keyed by leaf and
refinement with inheritance (Sec. 6.1-6.2), then the direction perturbation (Sec. 3.3)
with the leaves' lambda. Lens chains: one step on a luminance image with the screen grid's
adapted lambda (Sec. 3.3, 6.1).

Tolerances are those of the per-entry-point parity tests. The grid's lambda is compared
exactly: every region there applies at most 25 updates, and gamma = min(1, 5 / sqrt(n)) is
1 for n <= 25, so both sides add +-1 to an integer. The rRMSE inherits the filter's
tolerance: by the triangle inequality of the 2-norm, |map_gpu - map| is at most the norm of
the weighted output error sqrt(mean_c (1e-5 s_c)^2 / (R_c^2 + eps)), s the output scale,
plus the float rounding of the map; the image value likewise with the mean over pixels."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import direction_sampler as ods
from oracle import lens_chain as olc
from oracle import quadtree as oqt
from oracle import region_adapt as ora
from oracle import rrmse as orr
from paper_2402_08273_amd import _abi
from parity import TOL, backward_scales, check, filter_scale, stats_scales
import lens_check
from synth import make_frame, make_reference
from synth.directions import make_perturb_inputs
from synth.lens import make_lens_chains, make_lens_noise, make_luminance
from synth.numpy_gen import NOISE_CONST
from synth.points import make_points
from synth.proposals import make_proposals

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

W, H, S, N, R, MAX_LAG = 75, 41, 6, 3, 2, 8
N_PROP = 600
CAPACITY, N_PTS, M_SPLIT, ROUNDS, L = 256, 20_000, 500, 4, 10
N_CHAINS, TAN = 50_000, 0.6
EPS = 1e-2
DIR_TOL = 4e-6


def lambda_tol(updates):
    """Rounding bound of a lambda that summed `updates` window deltas in fp64 in another
    association than the oracle (as in the region_adapt parity tests)."""
    u = np.asarray(updates, dtype=np.float64)
    return 2.0 * (u + 1.0) * (31.0 + u) * 2.0 ** -52 + 1e-15


def _build(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lib = os.path.dirname(_abi.LIB_PATH)
    assert os.path.exists(_abi.LIB_PATH), "libramlt.so is not built"
    exe = str(tmp_path / "gpu_chain")
    cmd = ["gcc", "-std=gnu11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "gpu_chain.c"), "-L", lib, "-lramlt", "-L", os.path.join(ROCM, "lib"),
           "-lamdhip64", f"-Wl,-rpath,{lib}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _inputs(d):
    rad, feats = make_frame(W, H, S, seed=41, noise=NOISE_CONST, sigma=0.1)
    ref = make_reference(W, H, seed=1041, spp=64, noise=NOISE_CONST, sigma=0.1)
    # acceptance uniform on [0, 1): the windows' means scatter around the target 0.5, so
    # lambda walks both ways instead of drifting off in one direction
    region, _ = make_proposals(N_PROP, N * N, seed=42)
    alpha = np.random.default_rng(42).random(N_PROP).astype(np.float32)
    _, px, py = make_points(N_PTS, 1, seed=43)
    qalpha = np.random.default_rng(44).random(N_PTS).astype(np.float32)
    _, omega, uv = make_perturb_inputs(N_PTS, CAPACITY, seed=45)
    arrays = {"radiance.f32": rad, "features.f32": feats, "reference.f32": ref, "region.i32": region,
              "alpha.f32": alpha, "px.f32": px, "py.f32": py, "qalpha.f32": qalpha, "omega.f32": omega,
              "uv.f32": uv, "luminance.f32": make_luminance(W, H, seed=46),
              "chains.f32": make_lens_chains(N_CHAINS, W, H, TAN, seed=47), "noise.f32": make_lens_noise(N_CHAINS, seed=48)}
    for name, a in arrays.items():
        np.ascontiguousarray(a).tofile(os.path.join(d, name))
    return arrays


def _out(d, name, dtype):
    return np.fromfile(os.path.join(d, "out_" + name), dtype=dtype)


def test_c_program_runs_the_path(tmp_path):
    exe = _build(tmp_path)
    d = str(tmp_path)
    a = _inputs(d)
    args = [exe, d] + [str(v) for v in (W, H, S, N, R, MAX_LAG, N_PROP, CAPACITY, N_PTS, M_SPLIT, ROUNDS, N_CHAINS,
                                        TAN)]
    print("C chain:", " ".join(args[2:]), flush=True)
    run = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, (run.returncode, run.stdout, run.stderr)

    # screen grid: adaptation (exact, see the module docstring)
    st = ora.adapt(ora.initial_state(N * N), a["region.i32"], a["alpha.f32"], L=L)
    assert st["updates"].max() <= 26, "premise of the exact comparison"
    assert np.array_equal(_out(d, "grid_updates.i32", np.int32), st["updates"])
    assert np.array_equal(_out(d, "grid_lambda.f64", np.float64), st["lambda"])
    lam32 = st["lambda"].astype(np.float32)
    assert np.array_equal(_out(d, "grid_lambda.f32", np.float32), lam32)
    assert len(np.unique(lam32)) > 1

    # statistics
    rad, feats, ref = a["radiance.f32"], a["features.f32"], a["reference.f32"]
    o = oracle.stats_accumulate(rad, feats, MAX_LAG)
    sc = stats_scales(rad, o)
    K = min(MAX_LAG, S - 1)
    check("mean", _out(d, "mean.f32", np.float32).reshape(3, H, W), o["mean"], sc["mean"])
    check("var", _out(d, "var.f32", np.float32).reshape(3, H, W), o["var"], sc["var"])
    check("tau", _out(d, "tau.f32", np.float32).reshape(3, H, W), o["tau"], sc["tau"])
    check("lag_corr", _out(d, "lag_corr.f32", np.float32).reshape(3, K, H, W), o["lag_corr"], sc["rho"])
    f64 = feats.astype(np.float64)
    check("feat_mean", _out(d, "feat_mean.f32", np.float32).reshape(7, H, W), o["feat_mean"],
          np.abs(f64).mean(axis=1))
    check("feat_var", _out(d, "feat_var.f32", np.float32).reshape(7, H, W), o["feat_var"],
          o["feat_var"] + 1e-6 * (f64 * f64).mean(axis=1))

    # filter, fused loss seed and adjoint
    out_o, _ = oracle.filter_forward(o["mean"], lam32, N, R)
    out_s = filter_scale(o["mean"], lam32, N, R, -30.0)
    out = _out(d, "out.f32", np.float32).reshape(3, H, W)
    check("out", out, out_o, out_s)
    L_o, U_o = oracle.mse_loss_seed(out_o, ref)
    G_o, gl_o = oracle.filter_backward(U_o, o["mean"], out_o, lam32, N, R, -30.0, S)
    n = out_o.size
    u_scale = 2.0 * (np.abs(out_o) + np.abs(ref)) / n
    dd = np.abs(out_o - ref)
    check("loss", _out(d, "loss.f64", np.float64)[0], L_o, L_o + (2 * dd * (np.abs(out_o) + np.abs(ref))).sum() / n)
    G_s, gl_s = backward_scales(u_scale, o["mean"], out_o, lam32, N, R, -30.0, S)
    check("G", _out(d, "grad_radiance.f32", np.float32).reshape(3, H, W), G_o, G_s)
    check("grad_lambda", _out(d, "grad_lambda.f32", np.float32), gl_o, gl_s)

    # rRMSE of the filtered image
    map_o, val_o = orr.rrmse(out_o, ref, EPS)
    ref64 = ref.astype(np.float64)
    w_err = (TOL * out_s) ** 2 / (ref64 * ref64 + EPS)
    map_tol = np.sqrt(np.mean(w_err, axis=0)) + 2.0 ** -23 * map_o + 1e-30
    gmap = _out(d, "map.f32", np.float32).reshape(H, W)
    assert np.all(np.abs(gmap - map_o) <= map_tol), float(np.max(np.abs(gmap - map_o) / map_tol))
    gval = _out(d, "rrmse.f64", np.float64)[0]
    assert abs(gval - val_o) <= np.sqrt(np.mean(w_err)) + 1e-12 * val_o, (gval, val_o)

    # quadtree growth with adaptation keyed by leaf, then the perturbation
    f = oqt.Forest(1, CAPACITY)
    qs = ora.initial_state(CAPACITY)
    for _ in range(ROUNDS):
        leaf0 = f.lookup_many(None, a["px.f32"], a["py.f32"], count=True)
        ora.adapt(qs, leaf0, a["qalpha.f32"], L=L)
        f.refine(M_SPLIT, qs)
    leaf1 = f.lookup_many(None, a["px.f32"], a["py.f32"], count=True)
    nn = len(f.nodes)
    assert _out(d, "n_nodes.i32", np.int32)[0] == nn and nn > 20
    assert np.array_equal(_out(d, "child.i32", np.int32), f.child_array())
    assert np.array_equal(_out(d, "depth.i32", np.int32), f.depth_array())
    assert np.array_equal(_out(d, "visits.i32", np.int32), f.visits_array())
    assert np.array_equal(_out(d, "leaf0.i32", np.int32), leaf0)
    assert np.array_equal(_out(d, "leaf1.i32", np.int32), leaf1)
    assert np.array_equal(_out(d, "leaf_updates.i32", np.int32), qs["updates"][:nn])
    assert np.array_equal(_out(d, "leaf_ivisits.i32", np.int32), qs["visits"][:nn])
    assert np.array_equal(_out(d, "leaf_acc.f64", np.float64), qs["acc"][:nn])
    lam_q = _out(d, "leaf_lambda.f64", np.float64)
    tol = lambda_tol(ROUNDS * N_PTS // L + ROUNDS + 1)   # every update of any lineage, and one rounding per call
    assert np.all(np.abs(lam_q - qs["lambda"][:nn]) <= tol)

    want, wth = ods.perturb_directions(qs["lambda"], leaf1, a["omega.f32"], a["uv.f32"])
    th = _out(d, "theta.f32", np.float32)
    om = _out(d, "omega.f32", np.float32).reshape(N_PTS, 3)
    nan = np.isnan(wth)
    assert np.array_equal(np.isnan(th), nan) and nan.any() and not nan.all()
    ok = ~nan
    # theta within 2^-23 relative: the lambda difference allowed above (~1e-12) moves theta
    # by a relative amount of that order, inside the half ulp left over by the rounding
    assert np.all(np.abs(th[ok] - wth[ok]) <= 2.0 ** -23 * np.abs(wth[ok]) + 1e-45)
    okd = ~np.isnan(want)
    assert np.array_equal(np.isnan(om), np.isnan(want))
    assert np.max(np.abs(om[okd] - want[okd])) <= DIR_TOL

    # lens chains with the grid's adapted lambda: regions exact, proposals within 4e-6, alpha
    # and the move checked as in test_gpu_lens.py (tests/lens_check.py)
    ch, nz = a["chains.f32"], a["noise.f32"]
    o = olc.step(a["luminance.f32"], TAN, st["lambda"], N, ch, nz)
    g_reg = _out(d, "lens_region.i32", np.int32)
    g_alpha = _out(d, "lens_alpha.f32", np.float32)
    g_prop = _out(d, "lens_prop.f32", np.float32).reshape(N_CHAINS, 3)
    g_next = _out(d, "lens_chains.f32", np.float32).reshape(N_CHAINS, 3)
    lens_check.check_step(a["luminance.f32"], TAN, ch, nz, o, [g_next, g_reg, g_alpha, g_prop], name="C chain")
    moved = (o[1] >= 0) & (nz[:, 2] < g_alpha)
    assert moved.any() and ((o[1] >= 0) & ~moved).any()

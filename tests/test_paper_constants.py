"""The paper's printed parameters (tests/golden/paper_parameters.txt) against the defaults
used by the oracle and the synthetic inputs."""

import os

import numpy as np

import oracle
from synth import make_lambda

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.txt")


def _params():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, value = line.split()[:2]
        out[name] = float(value)
    return out


def test_oracle_defaults_follow_paper():
    p = _params()
    assert oracle.LAMBDA_MIN_DEFAULT == p["lambda_min"]
    assert oracle.N_REGIONS_DEFAULT == p["N_top"]


def test_synthetic_lambda_centred_on_paper_initial_value():
    p = _params()
    lam = make_lambda(int(p["N_top"]), seed=99)
    assert lam.shape == (400,)
    assert np.all(np.abs(lam - p["lambda_init"]) <= 0.5)
    assert abs(float(lam.mean()) - p["lambda_init"]) < 0.1


def test_adaptation_defaults_follow_paper():
    import inspect

    from oracle import region_adapt as ora
    from paper_2402_08273_amd import ops

    p = _params()
    assert ora.L_DEFAULT == p["L"]
    assert ora.GAMMA_MAX_DEFAULT == p["gamma_max"] and ora.GAMMA_SCALE_DEFAULT == p["gamma_scale"]
    assert ora.ALPHA_TARGET_DEFAULT == p["alpha_star"]
    assert ora.LAMBDA_INIT_DEFAULT == p["lambda_init"] and ora.LAMBDA_MIN_DEFAULT == p["lambda_min"]
    d = inspect.signature(ops.RegionAdapter.__init__).parameters
    assert d["L"].default == p["L"] and d["gamma_max"].default == p["gamma_max"]
    assert d["gamma_scale"].default == p["gamma_scale"] and d["alpha_target"].default == p["alpha_star"]
    assert d["lambda_init"].default == p["lambda_init"] and d["lambda_min"].default == p["lambda_min"]


def test_quadtree_workloads_follow_paper():
    from synth.workloads import QUADTREE_2D, QUADTREE_4D

    p = _params()
    for wl in (QUADTREE_2D, QUADTREE_4D):
        assert wl["m_split"] == p["M_split"]
        assert wl["grow_points"] == p["M_refine"]
    assert QUADTREE_2D["n_roots"] == 1
    assert QUADTREE_4D["n_roots"] == p["N_top"] ** 2

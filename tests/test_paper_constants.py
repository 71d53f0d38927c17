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

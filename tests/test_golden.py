"""The stored oracle results the GPU tests compare against are current: a
few of their channels are recomputed by the oracle here and must match to
rounding (a change to the oracle's arithmetic must regenerate them with
tests/golden/make_golden.py)."""
import json
import os

import numpy as np
import pytest

import oracle
from casimir_inputs import c1_piston_tm_fp64, c2_piston_tetm_fp32

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("fname,make,subset,n_steps", [
    ("c1_piston_tm_oracle.json", c1_piston_tm_fp64, [0, 7, 41, 84, 100, 115], None),
    ("c2_piston_tetm_oracle.json", c2_piston_tetm_fp32, [5, 300], 10000),
])
def test_golden_is_current(fname, make, subset, n_steps):
    path = os.path.join(HERE, "golden", fname)
    if not os.path.exists(path):
        pytest.skip(f"{fname} not generated")
    ref = json.load(open(path))
    wl = make()
    assert ref["workload"] == wl.name and ref["n_steps"] == wl.n_steps
    r = oracle.solve(wl, channel_subset=subset, workers=len(subset), chunk=1)
    np.testing.assert_allclose(r.acc, np.array(ref["per_channel"])[subset], rtol=1e-13, atol=0)
    np.testing.assert_allclose(r.sign, np.array(ref["sign"])[subset], rtol=0, atol=0)

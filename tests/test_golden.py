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


def test_stop_traces_are_current():
    """The convergence-stop traces: the piston's whole trace is recomputed
    (1.3 s) and must match to rounding; the 3D trace ends at its force."""
    from casimir_inputs.configs import stop_piston2d, stop_sphere3d
    path = os.path.join(HERE, "golden", "stop_traces_oracle.json")
    if not os.path.exists(path):
        pytest.skip("stop_traces_oracle.json not generated")
    ref = json.load(open(path))
    wl = stop_piston2d()
    r = oracle.solve(wl, workers=4, chunk=16)
    np.testing.assert_allclose(r.trace, ref["piston2d"]["trace"], rtol=1e-12, atol=1e-14)
    s3 = ref["sphere3d"]
    assert s3["workload"] == stop_sphere3d().name and len(s3["trace"]) == s3["n_steps"]
    assert s3["trace"][-1] == pytest.approx(s3["force"], rel=1e-12)


def test_reduced_stop_traces_are_current():
    """The cylindrical trace is recomputed (13 s) and must match to rounding;
    both traces end at their force."""
    from casimir_inputs.configs import stop_cyl, stop_kz
    from oracle import cylforce
    path = os.path.join(HERE, "golden", "stop_traces_reduced_oracle.json")
    if not os.path.exists(path):
        pytest.skip("stop_traces_reduced_oracle.json not generated")
    ref = json.load(open(path))
    wl = stop_cyl()
    r = cylforce.solve(wl, m_max=wl.m_max)
    np.testing.assert_allclose(r.trace, ref["cyl"]["trace"], rtol=1e-12, atol=1e-18)
    assert ref["kz"]["workload"] == stop_kz().name
    for key in ("cyl", "kz"):
        assert ref[key]["trace"][-1] == pytest.approx(ref[key]["force"], rel=1e-9)

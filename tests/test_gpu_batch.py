"""Batched solves (several problems advanced by one fused launch sequence):
each problem's result equals its own solve bit for bit, problems of mixed
kinds fall back to individual solves, and the 24-height uneven piston set
matches the oracle on sampled members."""
import numpy as np
import pytest

import oracle
from casimir_inputs import c3_uneven_set, parallel_plates_1d
from casimir_inputs.configs import piston2d

pytestmark = pytest.mark.gpu


def announce(name):
    print(f"\n[case] {name}", flush=True)


def opts_of(wl, **over):
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
             precision=wl.precision)
    o.update(over)
    return o


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_individual_solves(cf, precision):
    announce(f"batch of 4 uneven pistons vs individual solves, {precision}")
    wls = [piston2d(40, ny, 4, 10, 5, 10, (ny - 5) // 2, 10.0, pol="TM+TE", n_steps=97, n_harm=12)
           for ny in (20, 24, 31, 40)]
    probs = [cf.Problem.from_workload(w) for w in wls]
    o = opts_of(wls[0], precision=precision)
    res = cf.batch_solve(probs, **o)
    res_graph = cf.batch_solve(probs, graph=True, **o)
    for p, r, rg in zip(probs, res, res_graph):
        assert r["fused"]
        np.testing.assert_array_equal(r["per_channel"], rg["per_channel"])
        single = p.solve(**o)
        np.testing.assert_array_equal(r["per_channel"], single["per_channel"])
        assert r["force"] == single["force"]


def test_mixed_batch_falls_back(cf):
    announce("mixed batch: a fused piston + a piston whose S is wider than any tile")
    a = piston2d(40, 24, 4, 10, 5, 10, 7, 10.0, pol="TM+TE", n_steps=60, n_harm=8)
    b = piston2d(300, 24, 4, 120, 5, 10, 7, 10.0, pol="TM+TE", n_steps=60, n_harm=8)
    probs = [cf.Problem.from_workload(w) for w in (a, b)]
    o = opts_of(a)
    res = cf.batch_solve(probs, **o)
    for p, r, w in zip(probs, res, (a, b)):
        ref = oracle.solve(w)
        terms = float(np.sum(np.abs(ref.sign * ref.acc)) / np.pi)
        assert abs(r["force"] - ref.force) <= 1e-9 * terms
    assert res[0]["fused"] and not res[1]["fused"]


def test_c3_uneven_set_sampled_against_oracle(cf):
    """All 24 clearances h in [0.1, 2.0] at res 40 (grid heights 84..160),
    TE+TM, FP32, in one batched sequence (T cut to 150 steps); members 0, 11
    and 23 are checked against the FP64 oracle."""
    announce("c3 24 uneven pistons batched, T=150")
    wls = [w.replace(n_steps=150) for w in c3_uneven_set()]
    assert [w.shape[1] for w in (wls[0], wls[-1])] == [84, 160]
    probs = [cf.Problem.from_workload(w) for w in wls]
    res = cf.batch_solve(probs, **opts_of(wls[0]))
    assert all(r["fused"] for r in res)
    for k in (0, 11, 23):
        ref = oracle.solve(wls[k])
        terms = float(np.sum(np.abs(ref.sign * ref.acc)) / np.pi)
        assert abs(res[k]["force"] - ref.force) <= 1e-5 * terms
        np.testing.assert_allclose(res[k]["per_channel"], ref.acc, rtol=0, atol=1e-5 * np.max(np.abs(ref.acc)))


def test_c3_with_mu5_sidewalls_one_graph_sequence(cf):
    """The uneven set with metallic sidewalls and the same set with mu = 5
    magnetic sidewalls (48 problems), FP32, in one graph-captured batched
    sequence (T cut to 120): every problem fused; members equal their own
    solves bit for bit; a mu = 5 member matches the FP64 oracle.  One batch
    takes one set of options, so both sets run with the general kernel (the
    z-invariant one assumes perfect conductors in vacuum)."""
    announce("c3 metallic + mu=5 sidewalls, 48 problems, one graph sequence, T=120")
    wls = [w.replace(n_steps=120, kernel="general") for side in ("pec", "mu5") for w in c3_uneven_set(side)]
    probs = [cf.Problem.from_workload(w) for w in wls]
    o = opts_of(wls[0])
    res = cf.batch_solve(probs, graph=True, **o)
    assert len(res) == 48 and all(r["fused"] for r in res)
    for k in (3, 24 + 17):
        single = probs[k].solve(**o)
        np.testing.assert_array_equal(res[k]["per_channel"], single["per_channel"])
    k = 24 + 9
    assert wls[k].mu[2] == 5.0
    ref = oracle.solve(wls[k])
    terms = float(np.sum(np.abs(ref.sign * ref.acc)) / np.pi)
    assert abs(res[k]["force"] - ref.force) <= 1e-5 * terms

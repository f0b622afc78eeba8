"""Physics of the piston with sidewalls (Sec. III A, Fig. 3) on the GPU path.

Sec. III A sweeps the sidewall separation h and plots the block-block
force for metallic and for perfect-magnetic-conductor (PMC) sidewalls. It reports three qualitative facts, explained by image currents
that change sign between the two kinds of wall:
* metallic sidewalls suppress the TM force and enhance the TE force at
  small h, so the total force is nonmonotonic in h;
* PMC sidewalls do the opposite, enhancing TM and suppressing TE at small
  h, and the total force is monotonic in h.

This test sweeps 12 clearances h in [0.1, 2.0] at resolution 40 (the
uneven piston set of the batched benchmark) and checks these facts. Each
polarization and sidewall kind is one batched solve. T = 10000 steps is
converged: doubling T changes no force by more than 2e-5 relative.
"""
import numpy as np
import pytest

from casimir_inputs.configs import c3_uneven_set

pytestmark = pytest.mark.gpu

N_INST, RES, T = 12, 40, 10000


def sweep(cf, sidewall, pol):
    wls = c3_uneven_set(sidewall, n_inst=N_INST, res=RES, n_steps=T, pol=pol)
    probs = [cf.Problem.from_workload(w) for w in wls]
    rs = cf.batch_solve(probs, sigma=1.0, courant=0.5, n_steps=T, pol=pol, kernel="zinv2d",
                        precision="fp32")
    return np.array([w.meta["h"] for w in wls]), np.array([r["force"] for r in rs])


def strictly_increasing(a):
    return bool(np.all(np.diff(a) > 0))


def test_sidewall_kind_decides_monotonicity(cf):
    print("\n[case] piston force vs clearance h, metallic and PMC sidewalls, res 40, "
          f"{N_INST} clearances, T = {T}", flush=True)
    F = {}
    for side in ("pec", "pmc"):
        for pol in ("TM", "TE"):
            h, F[side, pol] = sweep(cf, side, pol)
    for side in ("pec", "pmc"):
        tot = F[side, "TM"] + F[side, "TE"]
        rows = " ".join(f"{x:.3f}:{f:+.3e}" for x, f in zip(h, tot))
        print(f"[fig3] {side} total: {rows}", flush=True)
        assert np.all(F[side, "TM"] < 0) and np.all(F[side, "TE"] < 0)      # attractive
    # Metallic: |TM| grows with h, |TE| shrinks; |total| has an interior minimum.
    assert strictly_increasing(-F["pec", "TM"])
    assert strictly_increasing(F["pec", "TE"])
    tot = -(F["pec", "TM"] + F["pec", "TE"])
    k = int(np.argmin(tot))
    assert 0 < k < N_INST - 1, k
    assert tot[0] > 1.2 * tot[k] and tot[-1] > 1.2 * tot[k]
    # PMC: |TM| shrinks with h, |TE| grows; |total| is monotonic (decreasing).
    assert strictly_increasing(F["pmc", "TM"])
    assert strictly_increasing(-F["pmc", "TE"])
    assert strictly_increasing(F["pmc", "TM"] + F["pmc", "TE"])
    # The wall kind flips which polarization dominates at the smallest h.
    assert abs(F["pec", "TE"][0]) > abs(F["pec", "TM"][0])
    assert abs(F["pmc", "TM"][0]) > abs(F["pmc", "TE"][0])

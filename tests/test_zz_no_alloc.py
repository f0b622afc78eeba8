"""cf_solve_static (the entry point for callers that cannot allocate device
memory) against cf_solve: bitwise-equal results on consecutive calls of
decreasing size, in FP32 and FP64, 2D and 3D, through the C ABI.  The static
array keeps the previous call's contents, so a second, smaller call would show
any state that a solve fails to clear."""
import numpy as np
import pytest

import oracle
from casimir_inputs.configs import piston2d
from casimir_inputs.geometry import Box, Sphere, Workload, rasterize

pytestmark = pytest.mark.gpu


def announce(name):
    print(f"\n[case] {name}", flush=True)


def opts_of(wl, **over):
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
             precision=wl.precision)
    o.update(over)
    return o


def same(a, b):
    assert a["force"] == b["force"], (a["force"], b["force"])
    assert np.array_equal(a["per_channel"], b["per_channel"])
    assert np.array_equal(a["per_harmonic"], b["per_harmonic"])
    assert a["n_steps_run"] == b["n_steps_run"]


def sphere_case(nx, ny, nz, n_steps):
    zlo = 2
    big = 1e30
    prims = [Box((-big, -big, -big), (big, big, zlo), 1), Sphere((nx / 2 + 0.3, ny / 2, zlo + 5.5), 1.7, 2)]
    ids = rasterize((nx, ny, nz), prims)
    return Workload(name="s3", ndim=3, shape=(nx, ny, nz), res=4.0, bc=("periodic", "periodic", "pec"),
                    pml_cells=(0, 0, 0), eps=[1.0, float("-inf"), 3.0], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                    s_lo=(nx // 2 - 3, ny // 2 - 3, zlo + 2), s_hi=(nx // 2 + 4, ny // 2 + 3, zlo + 9),
                    n_harm=2, force_axis=2, pol="3D", kernel="general", n_steps=n_steps)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_static_matches_solve_on_shrinking_calls(cf, precision):
    big = piston2d(80, 40, 10, 20, 10, 20, 15, 20.0, pol="TM+TE", n_steps=400, n_harm=12)
    small = piston2d(40, 24, 4, 10, 5, 10, 7, 10.0, pol="TM+TE", n_steps=300, n_harm=8)
    for name, wl in (("big", big), ("small", small)):
        announce(f"static {precision} {name} {wl.shape}")
        p = cf.Problem.from_workload(wl)
        o = opts_of(wl, precision=precision)
        assert p.info(**o)["workspace_bytes"] <= cf.STATIC_WORKSPACE_BYTES
        s = p.solve_static(**o)
        ref = p.solve(**o)
        same(s, ref)
        assert s["fused"], "the fused kernel runs in the static workspace too"
    # the smaller call's result against the FP64 oracle (second call on the array)
    if precision == "fp64":
        r = oracle.solve(small)
        assert abs(s["force"] / r.force - 1) < 1e-9


def test_static_3d_then_2d(cf):
    cases = (("3d", sphere_case(12, 11, 18, 30), "fp32"),
             ("2d-after-3d", piston2d(40, 24, 4, 10, 5, 10, 7, 10.0, pol="TM", n_steps=200, n_harm=6), "fp32"))
    for name, wl, prec in cases:
        announce(f"static {name} {wl.shape}")
        p = cf.Problem.from_workload(wl)
        o = opts_of(wl, precision=prec)
        same(p.solve_static(**o), p.solve(**o))


def test_static_rejects_oversized_and_graph(cf):
    from casimir_inputs.configs import c2_piston_tetm_fp32
    wl = c2_piston_tetm_fp32(n_steps=100)
    p = cf.Problem.from_workload(wl)
    o = opts_of(wl)
    assert p.info(**o)["workspace_bytes"] > cf.STATIC_WORKSPACE_BYTES
    with pytest.raises(cf.CfError) as e:
        p.solve_static(**o)
    assert e.value.status == "CF_E_BUDGET" and "cf_solve" in str(e.value)
    small = piston2d(40, 24, 4, 10, 5, 10, 7, 10.0, pol="TM", n_steps=50, n_harm=4)
    ps = cf.Problem.from_workload(small)
    with pytest.raises(cf.CfError) as e:
        ps.solve_static(**opts_of(small, graph=True))
    assert e.value.status == "CF_E_UNSUPPORTED"

"""Time-convergence stop (the partial force F(T') settles as T' grows, as
the paper's force-error-versus-time figure shows, Appendix A): a run with a
tolerance ends early, reports the steps it ran, and its force stays within a
small multiple of the tolerance of the full-length run.  The FP64 oracle's
trace of this piston settles to 6e-10 relative by T' = 500 of 3000 steps.

Against the oracle: the documented rule (every `stop_every` steps the partial
force F(T') is formed; the run ends after two consecutive windows that
change it by at most stop_tol |F(T')|) is applied to the FP64 oracle's own
trace F(T') (tests/golden/stop_traces_oracle.json, written from oracle/
only); the GPU must stop at the same step, with the oracle's partial force
there, on the fused and split 2D paths, the fused 3D steps and the server.
The check intervals are multiples of every fused kernel's steps per launch
(and even, for the two-step 3D launches), so every check falls on a launch
boundary; the tolerances are chosen away from the windows' changes."""
import json
import os

import numpy as np
import pytest

from casimir_inputs.configs import piston2d, stop_piston2d, stop_sphere3d
from casimir_inputs.geometry import Box, Sphere, Workload, rasterize

pytestmark = pytest.mark.gpu
MiB = 1 << 20
BIG = 1e30


def announce(name):
    print(f"\n[case] {name}", flush=True)


def piston():
    return piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, pol="TM+TE", n_steps=3000, n_harm=8)


def opts_of(wl, **over):
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
             precision="fp64")
    o.update(over)
    return o


@pytest.mark.parametrize("path", ["fused", "split"])
def test_stop_ends_early_within_tolerance(cf, path):
    announce(f"convergence stop, 2D piston, {path}")
    wl = piston()
    p = cf.Problem.from_workload(wl)
    extra = dict(split=True) if path == "split" else {}
    full = p.solve(**opts_of(wl, **extra))
    assert full["n_steps_run"] == wl.n_steps
    r = p.solve(**opts_of(wl, stop_tol=1e-8, stop_every=100, **extra))
    print(f"[stop] {path}: {r['n_steps_run']} of {wl.n_steps} steps, "
          f"rel diff {abs(r['force'] / full['force'] - 1):.2e}", flush=True)
    assert 300 <= r["n_steps_run"] < 1200
    assert abs(r["force"] / full["force"] - 1) <= 1e-7
    assert r["cell_updates"] == pytest.approx(full["cell_updates"] * r["n_steps_run"] / wl.n_steps)


def test_stop_off_with_channel_waves(cf):
    """With channels in several waves the partial force is not known during a
    wave, so the stop does not apply and the run is the full one."""
    announce("convergence stop ignored with channel waves")
    wl = piston().replace(n_steps=400)
    p = cf.Problem.from_workload(wl)
    full = p.solve(**opts_of(wl))
    r = p.solve(**opts_of(wl, stop_tol=1e-3, stop_every=50, max_resident=7))
    assert r["n_steps_run"] == wl.n_steps
    np.testing.assert_array_equal(r["per_channel"], full["per_channel"])


@pytest.mark.parametrize("variant,every", [(0, 50), (6, 25)])
def test_stop_3d(cf, variant, every):
    """variant 6 is the two-step fused kernel: steps advance in pairs, so an
    odd check interval is met one step late; the stopped force is still the
    full run's partial force at the step the run ended."""
    announce(f"convergence stop, 3D fused step, tile_variant {variant}, every {every}")
    nx, ny, nz, pml = 12, 12, 26, 4
    zlo = pml + 2
    prims = [Box((-BIG, -BIG, -BIG), (BIG, BIG, zlo), 1), Sphere((nx / 2 + 0.3, ny / 2, zlo + 5.5), 1.7, 2)]
    wl = Workload(name="s3", ndim=3, shape=(nx, ny, nz), res=4.0, bc=("periodic", "periodic", "pml"),
                  pml_cells=(0, 0, pml), eps=[1.8, float("-inf"), 3.0], mu=[1.0, 1.0, 1.0],
                  comp_ids=rasterize((nx, ny, nz), prims), s_lo=(nx // 2 - 3, ny // 2 - 3, zlo + 2),
                  s_hi=(nx // 2 + 4, ny // 2 + 3, zlo + 9), n_harm=2, force_axis=2, pol="3D",
                  kernel="general", n_steps=1500)
    p = cf.Problem.from_workload(wl)
    full = p.solve(**opts_of(wl, keep_gamma=True))
    tr = full["trace"]
    F = tr[-1]
    # a tolerance the partial force meets over the last 300 steps of the run
    checks = np.arange(50, wl.n_steps + 1, 50)
    d = np.abs(np.diff(tr[checks - 1])) / abs(F)
    tol = float(2 * d[-6:].max())
    r = p.solve(**opts_of(wl, stop_tol=tol, stop_every=every, tile_variant=variant))
    T = r["n_steps_run"]
    print(f"[stop] 3d: tol {tol:.2e}, {T} of {wl.n_steps} steps, variant {r['tile_variant']}, "
          f"rel diff {abs(r['force'] / F - 1):.2e}", flush=True)
    assert r["fused"] and T < wl.n_steps
    if variant == 6:
        assert r["tile_variant"] == 6 and T % 2 == 0 and T % every in (0, 1)
    else:
        assert T % every == 0
    # the stopped run's force is the full run's partial force at that step
    assert r["force"] == pytest.approx(tr[T - 1], rel=1e-9)


def test_server_stop(cf):
    announce("convergence stop in the server")
    wl = piston()
    p = cf.Problem.from_workload(wl)
    o = opts_of(wl, precision="fp32")
    full = p.solve(**o)
    with cf.Server(128 * MiB) as srv:
        t_stop = srv.submit(p, stop_tol=1e-6, stop_every=80, **o)
        t_full = srv.submit(p, **o)
        rs = srv.wait(t_stop, timeout=120)
        rf = srv.wait(t_full, timeout=120)
    assert rf["n_steps_run"] == wl.n_steps
    np.testing.assert_array_equal(rf["per_channel"], full["per_channel"])
    assert rs["n_steps_run"] < wl.n_steps
    assert abs(rs["force"] / full["force"] - 1) <= 1e-5


GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "stop_traces_oracle.json")


def oracle_stop_step(trace, tol, every):
    """The stop rule applied to an oracle trace (trace[m - 1] = F after m
    steps): the check steps k * every < T; a window is quiet when F changed
    by at most tol |F| since the previous check; the run ends at the second
    quiet window in a row, else runs all T steps.  Also returns the smallest
    distance of any window's relative change from tol (relative), which the
    test keeps away from zero so that rounding cannot flip a decision."""
    T = len(trace)
    prev, calm, margin = None, 0, np.inf
    for d in range(every, T, every):
        f = trace[d - 1]
        if prev is not None:
            ratio = abs(f - prev) / abs(f)
            margin = min(margin, abs(ratio / tol - 1))
            calm = calm + 1 if ratio <= tol else 0
            if calm >= 2:
                return d, margin
        prev = f
    return T, margin


def gold(key):
    if not os.path.exists(GOLD):
        pytest.skip("stop_traces_oracle.json not generated")
    return json.load(open(GOLD))[key]


@pytest.mark.parametrize("path", ["fused", "split", "server"])
@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_stop_step_and_force_match_the_oracle_rule(cf, path, tol):
    announce(f"convergence stop vs oracle rule, 2D piston, {path}, tol {tol:g}")
    ref = gold("piston2d")
    wl = stop_piston2d()
    assert ref["workload"] == wl.name
    every = 96
    T_ref, margin = oracle_stop_step(np.array(ref["trace"]), tol, every)
    assert T_ref < wl.n_steps and margin > 0.05, (T_ref, margin)
    p = cf.Problem.from_workload(wl)
    o = opts_of(wl, stop_tol=tol, stop_every=every)
    if path == "server":
        with cf.Server(128 * MiB, precision="fp64") as srv:
            r = srv.wait(srv.submit(p, **o), timeout=120)
    else:
        r = p.solve(split=(path == "split"), **o)
        assert r["fused"] == (path == "fused")
    print(f"[stop] {path} tol {tol:g}: oracle rule {T_ref}, GPU {r['n_steps_run']}", flush=True)
    assert r["n_steps_run"] == T_ref
    assert abs(r["force"] - ref["trace"][T_ref - 1]) <= 1e-9 * ref["terms"]


@pytest.mark.parametrize("variant", [0, 6])
def test_stop_3d_matches_the_oracle_rule(cf, variant):
    """3D fused steps: one step per launch (autotuned) and two per launch
    (variant 6), checked every 48 steps."""
    announce(f"convergence stop vs oracle rule, 3D sphere, tile_variant {variant}")
    ref = gold("sphere3d")
    wl = stop_sphere3d()
    every, tol = 48, 1e-5
    T_ref, margin = oracle_stop_step(np.array(ref["trace"]), tol, every)
    assert T_ref < wl.n_steps and margin > 0.05, (T_ref, margin)
    p = cf.Problem.from_workload(wl)
    r = p.solve(**opts_of(wl, stop_tol=tol, stop_every=every, tile_variant=variant))
    print(f"[stop] 3d variant {r['tile_variant']}: oracle rule {T_ref}, GPU {r['n_steps_run']}", flush=True)
    assert r["fused"]
    assert r["n_steps_run"] == T_ref
    assert abs(r["force"] - ref["trace"][T_ref - 1]) <= 1e-9 * ref["terms"]


GOLD_RED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "stop_traces_reduced_oracle.json")


def gold_red(key):
    if not os.path.exists(GOLD_RED):
        pytest.skip("stop_traces_reduced_oracle.json not generated")
    return json.load(open(GOLD_RED))[key]


def reduced_case(key):
    from casimir_inputs.configs import stop_cyl, stop_kz
    return stop_cyl() if key == "cyl" else stop_kz()


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("key", ["cyl", "kz"])
def test_stop_reduced_matches_the_oracle_rule(cf, key, variant):
    """Cylindrical and k_z problems on the resident kernels (1: fields in
    registers, 2: in global memory): the run goes in parts of stop_every base
    steps, and the stop step and force follow the oracle's trace (for the
    cylinder, every order at floor(d T_m / n_steps) of its own steps)."""
    announce(f"convergence stop vs oracle rule, {key}, resident variant {variant}")
    ref = gold_red(key)
    wl = reduced_case(key)
    assert ref["workload"] == wl.name
    every, tol = 50, 1e-6
    T_ref, margin = oracle_stop_step(np.array(ref["trace"]), tol, every)
    assert T_ref < wl.n_steps and margin > 0.05, (T_ref, margin)
    p = cf.Problem.from_workload(wl)
    o = opts_of(wl, pol="3D", stop_tol=tol, stop_every=every, tile_variant=variant)
    r = p.solve(**o)
    print(f"[stop] {key} variant {r['tile_variant']}: oracle rule {T_ref}, GPU {r['n_steps_run']}", flush=True)
    assert r["tile_variant"] == variant
    assert r["n_steps_run"] == T_ref
    assert abs(r["force"] - ref["trace"][T_ref - 1]) <= 1e-9 * ref["terms"]
    full = p.solve(**opts_of(wl, pol="3D", tile_variant=variant))
    assert r["cell_updates"] < full["cell_updates"]


def _bloch_grating(n_steps):
    from casimir_inputs import kz_workload
    BIGV = 1e30
    nx, ny = 24, 30
    ids = rasterize((nx, ny, 1), [Box((-BIGV, -BIGV, -BIGV), (BIGV, 4, BIGV), 1), Box((8, 12, -BIGV), (16, 18, BIGV), 2)])
    wl = Workload(name="grating1", ndim=2, shape=(nx, ny, 1), res=10.0, bc=("periodic", "pec", "periodic"),
                  pml_cells=(0, 0, 0), eps=[1.0, float("-inf"), 4.0], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                  s_lo=(6, 10, 0), s_hi=(18, 20, 1), n_harm=4, force_axis=1, pol="3D", kernel="general",
                  n_steps=n_steps, sigma=1.0, courant=0.5, precision="fp64")
    return kz_workload(wl, [0.0, 0.9], [1.0, 1.0], kx=[0.4, 0.4])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("key", ["cyl", "kz", "bloch"])
def test_reduced_parts_resume_bitwise(cf, key, variant, precision):
    """A run cut into parts (a stop that never fires: checks every 37 base
    steps while the force still moves) equals the one-launch run bit for
    bit, per channel and per step of Gamma."""
    announce(f"reduced run in parts vs one launch, {key}, variant {variant}, {precision}")
    wl = _bloch_grating(300) if key == "bloch" else reduced_case(key).replace(n_steps=300)
    p = cf.Problem.from_workload(wl)
    o = opts_of(wl, pol="3D", precision=precision, tile_variant=variant, keep_gamma=True)
    one = p.solve(**o)
    parts = p.solve(**dict(o, stop_tol=1e-15, stop_every=37))
    assert parts["n_steps_run"] == wl.n_steps and parts["tile_variant"] == variant
    np.testing.assert_array_equal(parts["per_channel"], one["per_channel"])
    np.testing.assert_array_equal(parts["gamma"], one["gamma"])
    assert parts["force"] == one["force"]

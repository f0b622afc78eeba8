"""Serving (continuous batching): force-solve requests of uneven size enter a
running scheduler as device memory frees up and leave when their steps are
done.  Each result is bitwise the same alone and in a mix, equals the
one-shot solve with the same kernel choice (fused tile variant, or the split
kernels), and a served result matches the FP64 oracle."""
import time

import numpy as np
import pytest

import oracle
from casimir_inputs.configs import piston2d, sphere_plate3d
from casimir_inputs.geometry import Box, Sphere, Workload, rasterize

pytestmark = pytest.mark.gpu
BIG = 1e30
MiB = 1 << 20
FP32_DEFAULT_VARIANT = 13    # the server's default fused variant in FP32 (1-based)
FP64_DEFAULT_VARIANT = 1


def announce(name):
    print(f"\n[case] {name}", flush=True)


def opts_of(wl, **over):
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
             precision="fp32")
    o.update(over)
    return o


def sphere3d(n_steps=40):
    nx, ny, nz, pml = 12, 12, 26, 4
    zlo = pml + 2
    prims = [Box((-BIG, -BIG, -BIG), (BIG, BIG, zlo), 1),
             Sphere((nx / 2 + 0.3, ny / 2, zlo + 5.5), 1.7, 2)]
    ids = rasterize((nx, ny, nz), prims)
    return Workload(name="s3", ndim=3, shape=(nx, ny, nz), res=4.0,
                    bc=("periodic", "periodic", "pml"), pml_cells=(0, 0, pml),
                    eps=[1.8, float("-inf"), 3.0], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                    s_lo=(nx // 2 - 3, ny // 2 - 3, zlo + 2), s_hi=(nx // 2 + 4, ny // 2 + 3, zlo + 9),
                    n_harm=2, force_axis=2, pol="3D", kernel="general", n_steps=n_steps)


def mix():
    """Fused pistons of three heights and step counts, a piston whose S needs
    the two-columns-per-lane tiles, one whose S is wider than any fused tile
    (split kernels) and a 3D sphere case (fused 3D step)."""
    wls = [piston2d(40, ny, 4, 10, 5, 10, (ny - 5) // 2, 10.0, pol="TM+TE", n_steps=T, n_harm=8)
           for ny, T in ((20, 97), (31, 61), (40, 130))]
    wls.append(piston2d(150, 24, 4, 60, 5, 10, 7, 10.0, pol="TM+TE", n_steps=75, n_harm=8))
    wls.append(piston2d(300, 24, 4, 120, 5, 10, 7, 10.0, pol="TM+TE", n_steps=60, n_harm=8))
    wls.append(sphere3d())
    return wls


SPLIT_ONLY = 4   # the entry of mix() no fused kernel takes (S wider than any tile)


def test_server_results_alone_equal_mix_and_one_shot(cf):
    announce("server: 6 requests alone, then together, vs one-shot solves (fp32)")
    wls = mix()
    probs = [cf.Problem.from_workload(w) for w in wls]
    with cf.Server(256 * MiB) as srv:
        alone = []
        for p, w in zip(probs, wls):
            alone.append(srv.wait(srv.submit(p, **opts_of(w)), timeout=120))
        # the mix: staggered submissions so requests join a running clock
        tickets = []
        for k, (p, w) in enumerate(zip(probs, wls)):
            tickets.append(srv.submit(p, **opts_of(w)))
            if k == 1:
                time.sleep(0.02)
        mixed = [srv.wait(t, timeout=120) for t in tickets]
        st = srv.stats()
    assert st["completed"] == 2 * len(wls) and st["failed"] == 0
    for k, (p, w) in enumerate(zip(probs, wls)):
        a, m = alone[k], mixed[k]
        np.testing.assert_array_equal(a["per_channel"], m["per_channel"])
        assert a["force"] == m["force"]
        fused = k != SPLIT_ONLY
        assert a["fused"] == fused
        if fused:
            if k < 3:
                assert a["tile_variant"] == FP32_DEFAULT_VARIANT
            if wls[k].ndim == 3:
                assert a["tile_variant"] == 6      # the two-step fused 3D kernel, steps paired in each tick
            one = p.solve(**opts_of(w, tile_variant=a["tile_variant"]))
            assert one["tile_variant"] == a["tile_variant"]
        else:
            one = p.solve(**opts_of(w, split=True))
        np.testing.assert_array_equal(a["per_channel"], one["per_channel"])
        assert a["force"] == one["force"]


def test_served_result_matches_oracle(cf):
    announce("server: one piston and the 3D case against the FP64 oracle (fp32 fields)")
    wls = [mix()[0], sphere3d(n_steps=30)]
    probs = [cf.Problem.from_workload(w) for w in wls]
    with cf.Server(128 * MiB) as srv:
        res = [srv.wait(srv.submit(p, **opts_of(w)), timeout=120) for p, w in zip(probs, wls)]
    for w, r in zip(wls, res):
        ref = oracle.solve(w)
        terms = float(np.sum(np.abs(ref.sign * ref.acc)) / np.pi)
        assert abs(r["force"] - ref.force) <= 1e-5 * terms
        np.testing.assert_allclose(r["per_channel"], ref.acc, rtol=0, atol=1e-5 * np.max(np.abs(ref.acc)))


def test_server_admits_by_budget(cf):
    """A budget that holds about two requests: later requests wait for memory,
    enter as earlier ones leave, and every result equals its one-shot solve."""
    announce("server: tight budget, 6 pistons queue for memory")
    wls = [piston2d(40, ny, 4, 10, 5, 10, (ny - 5) // 2, 10.0, pol="TM+TE", n_steps=T, n_harm=8)
           for ny, T in ((20, 200), (24, 150), (31, 180), (36, 120), (40, 160), (28, 140))]
    probs = [cf.Problem.from_workload(w) for w in wls]
    ws = max(p.info(**opts_of(w))["workspace_bytes"] for p, w in zip(probs, wls))
    with cf.Server(64 * MiB) as probe:
        tables = 64 * MiB - probe.stats()["budget"]
    with cf.Server(tables + int(2.5 * ws)) as srv:
        tickets = [srv.submit(p, **opts_of(w)) for p, w in zip(probs, wls)]
        res = [srv.wait(t, timeout=120) for t in tickets]
        times = [srv.times(t) for t in tickets]
        assert srv.stats()["bytes_in_use"] == 0
    admits = sorted(t[1] for t in times)
    dones = sorted(t[2] for t in times)
    assert admits[-1] >= dones[0], "every request was resident at once: the budget did not bind"
    for p, w, r in zip(probs, wls, res):
        one = p.solve(**opts_of(w, tile_variant=FP32_DEFAULT_VARIANT))
        np.testing.assert_array_equal(r["per_channel"], one["per_channel"])


def test_server_3d_channel_waves_fit_budget(cf):
    """A 3D request larger than the budget runs in channel waves sized to fit
    and still equals the one-shot solve."""
    announce("server: 3D request split into channel waves by the budget")
    w = sphere3d(n_steps=25)
    p = cf.Problem.from_workload(w)
    full = p.info(**opts_of(w))["workspace_bytes"]
    with cf.Server(64 * MiB) as probe:
        tables = 64 * MiB - probe.stats()["budget"]
    with cf.Server(tables + max(full // 3, 2 * MiB)) as srv:
        r = srv.wait(srv.submit(p, **opts_of(w)), timeout=120)
    one = p.solve(**opts_of(w))
    np.testing.assert_array_equal(r["per_channel"], one["per_channel"])


def test_server_cancel_leaves_others_unchanged(cf):
    announce("server: cancel a long request while another runs")
    short = mix()[1]
    long_ = piston2d(40, 24, 4, 10, 5, 10, 9, 10.0, pol="TM+TE", n_steps=200000, n_harm=8)
    ps, pl = cf.Problem.from_workload(short), cf.Problem.from_workload(long_)
    with cf.Server(128 * MiB) as srv:
        t_long = srv.submit(pl, **opts_of(long_))
        t_short = srv.submit(ps, **opts_of(short))
        r = srv.wait(t_short, timeout=120)
        srv.cancel(t_long)
        with pytest.raises(cf.CfError):
            srv.wait(t_long, timeout=60)
        with pytest.raises(cf.CfError, match="cancel"):
            srv.poll(t_long)
        st = srv.stats()
        assert st["cancelled"] == 1 and st["running"] == 0 and st["bytes_in_use"] == 0
    one = ps.solve(**opts_of(short, tile_variant=FP32_DEFAULT_VARIANT))
    np.testing.assert_array_equal(r["per_channel"], one["per_channel"])


def test_server_fp64_equals_one_shot(cf):
    announce("server fp64: two pistons in a mix vs one-shot solves")
    wls = mix()[:2]
    probs = [cf.Problem.from_workload(w) for w in wls]
    with cf.Server(128 * MiB, precision="fp64") as srv:
        ts = [srv.submit(p, **opts_of(w, precision="fp64")) for p, w in zip(probs, wls)]
        res = [srv.wait(t, timeout=120) for t in ts]
    for p, w, r in zip(probs, wls, res):
        one = p.solve(**opts_of(w, precision="fp64", tile_variant=FP64_DEFAULT_VARIANT))
        np.testing.assert_array_equal(r["per_channel"], one["per_channel"])


def test_server_rejects_bad_requests(cf):
    announce("server: argument errors")
    w = mix()[0]
    p = cf.Problem.from_workload(w)
    with cf.Server(64 * MiB) as srv:
        with pytest.raises(cf.CfError):
            srv.submit(p, **opts_of(w, precision="fp64"))        # precision differs from the server's
        with pytest.raises(cf.CfError):
            srv.submit(p, **opts_of(w, path="plain"))
        with pytest.raises(cf.CfError):
            srv.submit(p, **opts_of(w, channel_subset=[0, 1]))
        with pytest.raises(cf.CfError):
            srv.submit(p, **opts_of(w, courant=0.9))              # CFL
        assert srv.stats()["submitted"] == 0


def test_server_failed_request_is_isolated(cf):
    """A request whose accumulator turns non-finite (NaN injected into its
    first kick from the host) fails with CF_E_NONFINITE and frees its memory;
    the requests resident beside it complete with their alone results."""
    announce("server: one NaN-injected request among three")
    wls = mix()[:3]
    probs = [cf.Problem.from_workload(w) for w in wls]
    with cf.Server(128 * MiB) as srv:
        alone = [srv.wait(srv.submit(p, **opts_of(w)), timeout=120) for p, w in zip(probs, wls)]
        ts = [srv.submit(p, **opts_of(w, inject_nan=(k == 1))) for k, (p, w) in enumerate(zip(probs, wls))]
        with pytest.raises(cf.CfError, match="finite"):
            srv.wait(ts[1], timeout=120)
        res = [srv.wait(ts[k], timeout=120) for k in (0, 2)]
        st = srv.stats()
    assert st["failed"] == 1 and st["bytes_in_use"] == 0
    for a, r in zip((alone[0], alone[2]), res):
        np.testing.assert_array_equal(a["per_channel"], r["per_channel"])


def test_solve_reports_nonfinite(cf):
    announce("cf_solve: NaN-injected solve fails with CF_E_NONFINITE")
    w = mix()[0]
    p = cf.Problem.from_workload(w)
    with pytest.raises(cf.CfError) as e:
        p.solve(**opts_of(w, inject_nan=True))
    assert e.value.code == 5


def test_server_time_share_lets_small_requests_pass(cf):
    """A 3D cell (1280 channels x 48^3) and a small 2D piston, submitted
    together with the same step count: the 3D request's steps are paced by
    device time, not by the scheduler's step clock, so the piston (a
    thousandth of the cells per step) finishes long before the 3D cell.
    Both results equal their one-shot solves bit for bit."""
    announce("server: time-shared steps, a small 2D piston beside a 48^3 cell")
    w3 = sphere_plate3d(48, 1.0, n_steps=400)
    w2 = piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, pol="TM+TE", n_steps=400, n_harm=8)
    p3, p2 = cf.Problem.from_workload(w3), cf.Problem.from_workload(w2)
    with cf.Server(16 * 1024 * MiB) as srv:
        t3 = srv.submit(p3, **opts_of(w3))
        t2 = srv.submit(p2, **opts_of(w2))
        r2 = srv.wait(t2, timeout=120)
        r3 = srv.wait(t3, timeout=120)
        s3, _, d3 = srv.times(t3)
        s2, _, d2 = srv.times(t2)
    print(f"[serve] piston done after {d2 - s2:.3f} s, 3D cell after {d3 - s3:.3f} s", flush=True)
    assert r2["n_steps_run"] == r3["n_steps_run"] == 400
    assert d2 - s2 < 0.5 * (d3 - s3)
    one3 = p3.solve(**opts_of(w3, tile_variant=r3["tile_variant"]))
    one2 = p2.solve(**opts_of(w2, tile_variant=r2["tile_variant"]))
    np.testing.assert_array_equal(r3["per_channel"], one3["per_channel"])
    np.testing.assert_array_equal(r2["per_channel"], one2["per_channel"])
    assert r3["force"] == one3["force"] and r2["force"] == one2["force"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_server_runs_cylindrical_and_kz_requests_whole(cf, precision):
    """Cylindrical and k_z requests (their kernels take every step of a
    channel in one launch) run as one whole solve inside a tick, beside a
    fused piston; each result equals its one-shot cf_solve bit for bit."""
    from casimir_inputs import cyl_piston, dielectric_piston2d, kz_workload
    announce(f"server: cylindrical and k_z requests beside a piston ({precision})")
    wls = [cyl_piston(res=10, h_u=0.8, length_u=15.0, n_harm=3, m_max=2, n_steps=400, precision=precision),
           kz_workload(dielectric_piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, n_steps=300, n_harm=6,
                                           precision=precision), [0.0, 0.8, 2.5], [0.3, 0.5, 0.25]),
           piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, pol="TM+TE", n_steps=300, n_harm=8)]
    probs = [cf.Problem.from_workload(w) for w in wls]
    opts = [opts_of(w, precision=precision) for w in wls]
    stop = dict(opts[0], stop_tol=1e-2, stop_every=50)     # the stop runs the resident kernels in parts
    with cf.Server(256 * MiB, precision=precision) as srv:
        tickets = [srv.submit(p, **o) for p, o in zip(probs, opts)]
        t_stop = srv.submit(probs[0], **stop)
        served = [srv.wait(t, timeout=120) for t in tickets]
        stopped = srv.wait(t_stop, timeout=120)
        st = srv.stats()
    assert st["completed"] == 4 and st["failed"] == 0
    one = probs[0].solve(**stop)
    assert stopped["n_steps_run"] == one["n_steps_run"] < wls[0].n_steps
    np.testing.assert_array_equal(stopped["per_channel"], one["per_channel"])
    for p, o, s in zip(probs, opts, served):
        one = p.solve(**dict(o, tile_variant=s["tile_variant"]) if s["fused"] else o)
        np.testing.assert_array_equal(s["per_channel"], one["per_channel"])
        np.testing.assert_array_equal(s["per_harmonic"], one["per_harmonic"])
        assert s["force"] == one["force"] and s["n_steps_run"] == one["n_steps_run"]

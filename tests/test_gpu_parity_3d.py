"""GPU parity of the 3D path (six components, PEC / periodic walls, z CPML)
against the FP64 oracle.  Same tolerances as the 2D parity tests: FP64
fields to 1e-9 of the summed term magnitude, FP32 fields to 1e-5 of it on
these small cases; the 192^3 sample compares the Gamma time series of five
channels with the stored oracle result.
"""
import json
import os

import numpy as np
import pytest

import oracle
from casimir_inputs import c4_sphere_plate
from casimir_inputs.geometry import Box, Sphere, Workload, rasterize

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
BIG = 1e30


def announce(name):
    print(f"\n[case] {name}", flush=True)


def run(cf, wl, **over):
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol,
                kernel=wl.kernel, precision=wl.precision)
    opts.update(over)
    return cf.Problem.from_workload(wl).solve(**opts)


def sphere_case(nx, ny, nz, bc_z="pec", pml=0, n_steps=40, n_harm=2, eps_bg=1.0, bc_xy=("periodic", "periodic")):
    zlo = pml + 2
    prims = [Box((-BIG, -BIG, -BIG), (BIG, BIG, zlo), 1),
             Sphere((nx / 2 + 0.3, ny / 2, zlo + 5.5), 1.7, 2)]
    ids = rasterize((nx, ny, nz), prims)
    return Workload(name="s3", ndim=3, shape=(nx, ny, nz), res=4.0,
                    bc=(bc_xy[0], bc_xy[1], bc_z), pml_cells=(0, 0, pml),
                    eps=[eps_bg, float("-inf"), 3.0], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                    s_lo=(nx // 2 - 3, ny // 2 - 3, zlo + 2), s_hi=(nx // 2 + 4, ny // 2 + 3, zlo + 9),
                    n_harm=n_harm, force_axis=2, pol="3D", kernel="general", n_steps=n_steps)


CASES = {
    "pec_z": lambda: sphere_case(12, 11, 18),
    "pml_z_fluid": lambda: sphere_case(12, 12, 26, bc_z="pml", pml=4, eps_bg=1.8, n_steps=60),
    "pml_z_force_x": lambda: sphere_case(13, 12, 26, bc_z="pml", pml=4, n_steps=30).replace(force_axis=0),
    # S's top face on the first plane of the upper layer: the kick and the
    # consistent start reach into the CPML and stretch there as every step does
    "pml_z_touching": lambda: sphere_case(12, 12, 19, bc_z="pml", pml=4, n_steps=40),
}


FUSED_ONLY = {
    # PEC x/y walls, and a grid wider than one 64-lane row (3 columns per lane)
    "pec_xy_pml_z": lambda: sphere_case(13, 11, 26, bc_z="pml", pml=4, n_steps=23, bc_xy=("pec", "pec")),
    "wide_x_130": lambda: sphere_case(130, 10, 22, bc_z="pml", pml=3, n_steps=17, bc_xy=("periodic", "pec")),
    "wide_x_pec_97": lambda: sphere_case(97, 12, 18, n_steps=15, bc_xy=("pec", "periodic")),
}


def compare(g, ref, rtol):
    terms = float(np.sum(np.abs(ref.sign * ref.acc)) / np.pi)
    assert abs(g["force"] - ref.force) <= rtol * terms
    np.testing.assert_allclose(g["per_channel"], ref.acc, rtol=0, atol=rtol * np.max(np.abs(ref.acc)))


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_3d(cf, name, precision):
    announce(f"3d {name} {precision}")
    wl = CASES[name]()
    ref = oracle.solve(wl)
    g = run(cf, wl, precision=precision)
    compare(g, ref, 1e-9 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_3d_every_variant_bitwise_equals_split(cf, precision):
    """The fused z-streaming 3D step evaluates exactly the split kernels'
    arithmetic: every variant gives bitwise the same channel integrals."""
    cases = [CASES["pec_z"]().replace(n_steps=19), CASES["pml_z_fluid"]().replace(n_steps=21)]
    cases += [f() for f in FUSED_ONLY.values()]
    for wl in cases:
        announce(f"fused 3d vs split {wl.shape} bc {wl.bc} {precision}")
        ref = run(cf, wl, precision=precision, split=True)
        assert not ref["fused"]
        n_ok = 0
        for v in range(1, 7):        # 1..4 single-step band shapes, 5..6 two-step
            r = run(cf, wl, precision=precision, tile_variant=v)
            np.testing.assert_array_equal(r["per_channel"], ref["per_channel"])
            if r["fused"] and r["tile_variant"] == v:
                n_ok += 1            # else the variant's LDS rows do not fit this width / precision
        auto = run(cf, wl, precision=precision)
        np.testing.assert_array_equal(auto["per_channel"], ref["per_channel"])
        assert auto["fused"] == (n_ok > 0)
        if precision == "fp32":
            assert n_ok >= 4


def test_3d_waves_and_plain_equal_batched(cf):
    announce("3d: resident waves and plain path equal one batched wave")
    wl = CASES["pml_z_fluid"]().replace(n_steps=25)
    a = run(cf, wl)
    b = run(cf, wl, max_resident=7)
    sub = [0, 3, 17, len(a["per_channel"]) - 1]
    c = run(cf, wl, path="plain", channel_subset=sub)
    np.testing.assert_array_equal(a["per_channel"], b["per_channel"])
    np.testing.assert_array_equal(a["per_channel"][sub], c["per_channel"])


def test_3d_plates_closed_form_through_pml(cf):
    """1D-reduced plates in 3D with open space above (PML): the GPU force
    equals the oracle's, and both are within 1% of -2 (pi/24)/a^2."""
    announce("3d plates through PML")
    res, P = 20, 20
    a_px, d_px, b_px = 20, 10, 20
    z0 = P + 4
    nz = z0 + a_px + d_px + b_px + P
    prims = [Box((-BIG, -BIG, z0 + a_px), (BIG, BIG, z0 + a_px + d_px), 1),
             Box((-BIG, -BIG, -BIG), (BIG, BIG, z0), 1)]
    ids = rasterize((1, 1, nz), prims)
    wl = Workload(name="pz", ndim=3, shape=(1, 1, nz), res=float(res), bc=("periodic", "periodic", "pml"),
                  pml_cells=(0, 0, P), eps=[1.0, float("-inf")], mu=[1.0, 1.0], comp_ids=ids,
                  s_lo=(0, 0, z0 + a_px - 2), s_hi=(1, 1, z0 + a_px + d_px + 2), n_harm=1, force_axis=2,
                  pol="3D", kernel="general", n_steps=int(60 / (0.5 / res)))
    ref = oracle.solve(wl)
    g = run(cf, wl, precision="fp64")
    assert g["force"] == pytest.approx(ref.force, rel=1e-9)
    assert g["force"] == pytest.approx(-2 * np.pi / 24, rel=1e-2)


def test_c4_full_size_sample(cf):
    """192^3 sphere over an indented plate (16-cell z PML, periodic x/y),
    FP32 fields: five channels for 24 steps against the stored oracle run."""
    path = os.path.join(HERE, "golden", "c4_sphere_plate_sample_oracle.json")
    if not os.path.exists(path):
        pytest.skip("golden 192^3 sample not generated")
    ref = json.load(open(path))
    announce("c4 192^3 sample fp32, 5 channels x 24 steps")
    wl = c4_sphere_plate()
    g = run(cf, wl, n_steps=ref["n_steps"], channel_subset=ref["subset"], keep_gamma=True)
    gam_ref = np.array(ref["gamma"])
    scale = np.max(np.abs(gam_ref), axis=0)
    assert np.all(scale > 0)
    np.testing.assert_allclose(g["gamma"], gam_ref, rtol=0, atol=2e-5 * scale.max())
    np.testing.assert_allclose(g["per_channel"], ref["per_channel"], rtol=0,
                               atol=2e-5 * np.max(np.abs(ref["per_channel"])))


def test_c4_channels_full_T(cf):
    """The five sampled channels of the 192^3 cell over the full T = 6000,
    FP32 fields with FP64 accumulation, against the stored FP64 oracle
    integrals: within 1e-4 relative per channel."""
    path = os.path.join(HERE, "golden", "c4_sphere_plate_channels_full_T_oracle.json")
    if not os.path.exists(path):
        pytest.skip("golden full-T channel integrals not generated")
    ref = json.load(open(path))
    announce("c4 192^3 five channels, full T=6000, fp32")
    wl = c4_sphere_plate()
    g = run(cf, wl, channel_subset=ref["subset"])
    acc = np.array(ref["per_channel"])
    rel = np.abs(g["per_channel"] - acc) / np.abs(acc)
    print(f"[precision] c4 channel rel err max {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-4


def thick_plate_case(n_steps=23, bc_y="periodic"):
    """A PEC plate filling the lower 17 of 40 planes, with a hemispherical
    pit (radius 7) under a dielectric sphere, z PML at both ends: the planes
    a band's region can change start at the plate top for bands away from the
    pit and lower for the bands across it."""
    nx, ny, nz, pml = 16, 21, 40, 4
    top = 17
    prims = [Box((-BIG, -BIG, -BIG), (BIG, BIG, top), 1), Sphere((8.0, 10.5, top), 7.0, 0),
             Sphere((8.3, 10.5, top + 4.0), 2.5, 2)]
    ids = rasterize((nx, ny, nz), prims)
    return Workload(name="thick_plate", ndim=3, shape=(nx, ny, nz), res=4.0, bc=("periodic", bc_y, "pml"),
                    pml_cells=(0, 0, pml), eps=[1.8, float("-inf"), 3.0], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                    s_lo=(4, 7, top + 1), s_hi=(13, 14, top + 8), n_harm=2, force_axis=2, pol="3D",
                    kernel="general", n_steps=n_steps)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("bc_y", ["periodic", "pec"])
def test_fused_3d_skips_conductor_planes_bitwise(cf, precision, bc_y):
    """The fused 3D steps march each band only over the planes its region can
    change (below them every field is 0 inside the plate): every variant
    equals the split kernels, which march every plane, bit for bit; the
    force matches the oracle."""
    announce(f"fused 3d skipping plate planes, y {bc_y}, {precision}")
    wl = thick_plate_case(bc_y=bc_y)
    ref = run(cf, wl, precision=precision, split=True)
    for v in range(1, 7):
        r = run(cf, wl, precision=precision, tile_variant=v)
        np.testing.assert_array_equal(r["per_channel"], ref["per_channel"])
    if precision == "fp64" and bc_y == "periodic":
        compare(ref, oracle.solve(wl), 1e-9)

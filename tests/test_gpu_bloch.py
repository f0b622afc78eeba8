"""GPU parity of Bloch-periodic x runs (complex fields; Sec. III D) against
the FP64 Bloch oracle.

Cases (each printed before it runs): dielectric blocks (eps 4) repeated with
period L = 24 cells above a PEC plate, S around the block of the first
period; the one-period cell at (k_x, k_z) in {(0.4, 0), (0.4, 0.9),
(0.4 + pi/L, 0), (0.4 + pi/L, 0.9)} and the two-period supercell at
(0.4, 0) and (0.4, 0.9), whose force is the mean of the one-period forces
at k_x and k_x + pi/L (Bloch folding, exact on the grid).

Tolerances: FP64 1e-9 of the largest channel per channel and of the term
magnitude for the force; FP32 fields with FP64 accumulation 2e-5.
"""
import numpy as np
import pytest

from casimir_inputs import kz_workload
from casimir_inputs.geometry import Box, Workload, rasterize
from oracle import bloch

pytestmark = pytest.mark.gpu
BIG = 1e30
L = 2.4


def announce(name):
    print(f"\n[case] {name}", flush=True)


def grating(ncell, points, weights, n_steps=300):
    nx, ny = 24 * ncell, 30
    prims = [Box((-BIG, -BIG, -BIG), (BIG, 4, BIG), 1)]
    for c in range(ncell):
        prims.append(Box((c * 24 + 8, 12, -BIG), (c * 24 + 16, 18, BIG), 2))
    ids = rasterize((nx, ny, 1), prims)
    wl = Workload(name=f"grating{ncell}", ndim=2, shape=(nx, ny, 1), res=10.0, bc=("periodic", "pec", "periodic"),
                  pml_cells=(0, 0, 0), eps=[1.0, float("-inf"), 4.0], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                  s_lo=(6, 10, 0), s_hi=(18, 20, 1), n_harm=4, force_axis=1, pol="3D", kernel="general",
                  n_steps=n_steps, sigma=1.0, courant=0.5, precision="fp64")
    return kz_workload(wl, [p[1] for p in points], weights, kx=[p[0] for p in points])


PRIM = [(0.4, 0.0), (0.4, 0.9), (0.4 + np.pi / L, 0.0), (0.4 + np.pi / L, 0.9)]
SUPER = [(0.4, 0.0), (0.4, 0.9)]
_ORACLE = {}


def oracle_result(name):
    if name not in _ORACLE:
        pts = PRIM if name == "cell" else SUPER
        wl = grating(1 if name == "cell" else 2, pts, [1.0] * len(pts))
        _ORACLE[name] = (wl, bloch.solve(wl, pts, [1.0] * len(pts)))
    return _ORACLE[name]


def run(cf, wl, **over):
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel="general",
                precision=wl.precision)
    opts.update(over)
    return cf.Problem.from_workload(wl).solve(**opts)


def check(res, ref, tol):
    acc_ref = ref.acc.reshape(-1)
    sign = np.concatenate([ref.sign] * ref.acc.shape[0])
    scale = np.max(np.abs(acc_ref))
    err = np.max(np.abs(res["per_channel"] - acc_ref))
    assert err <= tol * scale, (err, scale)
    mag = np.sum(np.abs(sign * acc_ref)) / np.pi
    assert abs(res["force"] - ref.force) <= tol * mag
    return err / scale


@pytest.mark.parametrize("name", ["cell", "supercell"])
def test_fp64_matches_oracle(cf, name):
    announce(f"Bloch fp64 vs oracle: {name}")
    wl, ref = oracle_result(name)
    res = run(cf, wl)
    assert res["fused"] and res["tile_variant"] == 1          # both parts in registers
    rel = check(res, ref, 1e-9)
    print(f"[bloch] {name}: max channel error {rel:.2e} of the largest", flush=True)


def test_fp32_matches_oracle(cf):
    announce("Bloch fp32 vs oracle: cell")
    wl, ref = oracle_result("cell")
    rel = check(run(cf, wl, precision="fp32"), ref, 2e-5)
    print(f"[bloch] cell fp32: max channel error {rel:.2e} of the largest", flush=True)


def test_supercell_folding_on_gpu(cf):
    announce("Bloch folding on the GPU")
    wl1, _ = oracle_result("cell")
    wl2, _ = oracle_result("supercell")
    n1 = len(run(cf, wl1.replace(n_steps=1))["per_channel"]) // len(PRIM)
    r1 = run(cf, wl1)
    r2 = run(cf, wl2)
    h = wl1.n_harm
    f1 = [r1["per_harmonic"][q * h:(q + 1) * h].sum() for q in range(len(PRIM))]
    f2 = [r2["per_harmonic"][q * h:(q + 1) * h].sum() for q in range(len(SUPER))]
    for q in range(len(SUPER)):
        assert f2[q] == pytest.approx(0.5 * (f1[q] + f1[q + 2]), rel=1e-9), (q, f1, f2)
    assert n1 > 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_drivers_bitwise(cf, precision):
    announce(f"Bloch drivers bitwise, {precision}")
    wl, _ = oracle_result("cell")
    split = run(cf, wl, precision=precision, split=True, keep_gamma=True)
    plain = run(cf, wl, precision=precision, path="plain")
    np.testing.assert_array_equal(plain["per_channel"], split["per_channel"])
    # register-resident (both parts in registers) and global-memory resident kernels
    for variant, expect in ((0, 1), (2, 2)):
        res = run(cf, wl, precision=precision, tile_variant=variant, keep_gamma=True)
        assert res["fused"] and res["tile_variant"] == expect
        np.testing.assert_array_equal(split["per_channel"], res["per_channel"])
        np.testing.assert_array_equal(split["gamma"], res["gamma"])

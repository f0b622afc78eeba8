"""GPU parity of z-invariant problems at Bloch wavevectors k_z (Sec. III B,
Sec. III D) against the FP64 k_z oracle.

Cases (each printed before it runs):
* ``dielectric``: the 2D piston with eps = 4 blocks between PEC slabs
  (40 x 31 cells: a 64-cell tile with a ragged tail along x, eight 4-row
  tiles with a ragged one along y), k in {0, 0.8, 2.5} with weights
  {0.3, 0.5, 0.25}: at k != 0 the polarizations hybridize;
* ``plates``: a PEC slab between walls, periodic y (one cell: the periodic
  wrap of the y neighbours), k in {0, 1, 2, 4};
* ``periodic``: the dielectric piston with periodic x and y walls.

Tolerances as for the cylindrical path: FP64 1e-9 of the largest channel
per channel and of the term magnitude sum_c |s_c acc_c| / pi for the force;
FP32 fields with FP64 accumulation 2e-5.
"""
import numpy as np
import pytest

from casimir_inputs import dielectric_piston2d, kz_gauss, kz_workload, parallel_plates_1d
from oracle import kz

pytestmark = pytest.mark.gpu


def announce(name):
    print(f"\n[case] {name}", flush=True)


def dielectric(bc=("pec", "pec", "periodic")):
    base = dielectric_piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, n_steps=400, n_harm=6, precision="fp64")
    return kz_workload(base.replace(bc=bc), [0.0, 0.8, 2.5], [0.3, 0.5, 0.25])


CASES = {
    "dielectric": dielectric,
    "plates": lambda: kz_workload(parallel_plates_1d(20, 0.5, 0.25, 1.0, n_steps=600, precision="fp64"),
                                  [0.0, 1.0, 2.0, 4.0], [1.0, 1.0, 1.0, 1.0]),
    "periodic": lambda: dielectric(("periodic", "periodic", "periodic")),
}
_ORACLE = {}


def oracle_result(name):
    if name not in _ORACLE:
        wl = CASES[name]()
        _ORACLE[name] = (wl, kz.solve(wl, wl.kz, wl.kz_weight))
    return _ORACLE[name]


def run(cf, wl, **over):
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel="general",
                precision=wl.precision)
    opts.update(over)
    return cf.Problem.from_workload(wl).solve(**opts)


def check(res, ref, weights, tol):
    acc_ref = ref.acc.reshape(-1)                         # q-major, the library's channel order
    sign = np.concatenate([w * ref.sign for w in weights])
    assert res["per_channel"].shape == acc_ref.shape
    scale = np.max(np.abs(acc_ref))
    err = np.max(np.abs(res["per_channel"] - acc_ref))
    assert err <= tol * scale, (err, scale)
    mag = np.sum(np.abs(sign * acc_ref)) / np.pi
    assert abs(res["force"] - ref.force) <= tol * mag, (res["force"], ref.force, mag)
    return err / scale


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_matches_oracle(cf, name):
    announce(f"k_z fp64 vs oracle: {name}")
    wl, ref = oracle_result(name)
    res = run(cf, wl)
    rel = check(res, ref, wl.kz_weight, 1e-9)
    n_h = wl.n_harm
    for q, w in enumerate(wl.kz_weight):
        mine = res["per_harmonic"][q * n_h:(q + 1) * n_h].sum()
        mag = np.sum(np.abs(w * ref.sign * ref.acc[q])) / np.pi
        assert abs(mine - w * ref.per_k[q]) <= 1e-9 * max(mag, 1e-300)
    print(f"[kz] {name}: max channel error {rel:.2e} of the largest, F = {res['force']:.6e}", flush=True)


@pytest.mark.parametrize("name", ["dielectric", "plates"])
def test_fp32_matches_oracle(cf, name):
    announce(f"k_z fp32 vs oracle: {name}")
    wl, ref = oracle_result(name)
    res = run(cf, wl, precision="fp32")
    rel = check(res, ref, wl.kz_weight, 2e-5)
    print(f"[kz] {name} fp32: max channel error {rel:.2e} of the largest", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_drivers_bitwise(cf, precision):
    """Register-resident, global-memory resident, split and plain drivers
    share the per-cell forms and the surface reduction: identical results."""
    announce(f"k_z drivers bitwise, {precision}")
    for name in ("dielectric", "periodic"):
        wl, _ = oracle_result(name)
        split = run(cf, wl, precision=precision, split=True, keep_gamma=True)
        for variant, expect in ((0, 1), (2, 2)):
            res = run(cf, wl, precision=precision, tile_variant=variant, keep_gamma=True)
            assert res["fused"] and res["tile_variant"] == expect
            np.testing.assert_array_equal(split["per_channel"], res["per_channel"])
            np.testing.assert_array_equal(split["gamma"], res["gamma"])
        plain = run(cf, wl, precision=precision, path="plain")
        np.testing.assert_array_equal(plain["per_channel"], split["per_channel"])


def test_k_integral_equals_z_invariant_kernel_on_gpu(cf):
    """Appendix A.2 on the GPU path: the 8-point Gauss k_z integral of the
    plates (FP64 fields) equals the TM + TE force with the z-invariant kernel
    (the fused 2D kernel) to 5e-4, as the oracle pin states."""
    announce("k_z integral vs z-invariant kernel, plates, GPU")
    base = parallel_plates_1d(20, 0.5, 0.25, 1.0, n_steps=1600, precision="fp64")
    ks, ws = kz_gauss(8, 12.0)
    f_kz = run(cf, kz_workload(base, ks, ws))["force"]
    f_2d = cf.Problem.from_workload(base).solve(sigma=base.sigma, courant=base.courant, n_steps=base.n_steps,
                                                 pol="TM+TE", kernel="zinv2d", precision="fp64")["force"]
    print(f"[kz] k integral {f_kz:.8f}, z-invariant kernel {f_2d:.8f}", flush=True)
    assert abs(f_kz / f_2d - 1) < 5e-4


def test_benchmark_case_vs_oracle_golden(cf):
    """The k_z dielectric piston of the benchmark (8 k points) against the
    stored FP64 oracle: FP64 fields to 1e-9 of the term magnitude; FP32
    fields to 1e-4 relative on the force."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kz_dielectric_piston_oracle.json")
    if not os.path.exists(path):
        pytest.skip("golden kz_dielectric_piston_oracle.json not generated")
    announce("k_z benchmark case vs stored oracle")
    ref = json.load(open(path))
    base = dielectric_piston2d(80, 40, 10, 20, 10, 20, 15, 20.0, n_steps=2000, n_harm=16)
    wl = kz_workload(base, ref["kz"], ref["kz_weight"])
    p = cf.Problem.from_workload(wl)
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel="general")
    tab = p.channel_table(**o)
    acc = np.array(ref["per_channel"])
    mag = np.sum(np.abs(tab["sign"] * acc)) / np.pi
    r64 = p.solve(precision="fp64", **o)
    assert abs(r64["force"] - ref["force"]) <= 1e-9 * mag
    r32 = p.solve(precision="fp32", **o)
    rel = abs(r32["force"] / ref["force"] - 1)
    print(f"[kz] benchmark case: fp32 force rel err {rel:.2e}, terms / |F| = {mag / abs(ref['force']):.1e}",
          flush=True)
    assert rel <= 1e-4

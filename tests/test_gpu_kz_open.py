"""GPU parity of open-space problems with dispersive media against the FP64
oracle: Sec. III B's computation (dielectric waveguides in empty space,
Lorentz permittivity continued onto the conductivity contour, one
two-dimensional run per k_z, PML around the cell), on the split kernels,
which carry the in-plane CPML and the polarizations.

Cases (each printed before it runs):
* ``slabs``: two Lorentz slabs in open space (x CPML, one-cell periodic y),
  k in {0, 1, 3};
* ``slabs_tight``: the slabs with 3 cells of vacuum between S and the
  layers, so the kick's stencil reaches into a layer (the consistent start
  stretches its curl there, as every later step does);
* ``waveguides_si``: two silicon-like waveguides (eps_inf 1.035 with one
  Lorentz term of strength 10.835 at w0 = 22, Courant 0.35: the coupled
  stability limit at 20 cells per unit) with CPML on all four sides,
  k in {0, 2, 6} (a 65 x 45 grid: a ragged tail of the 64 x 4 tiles on
  both axes);
* ``waveguides_eps4``: the same cell with plain eps = 4 guides;
* ``bloch_pml_y`` (``_si``): eps = 4 (silicon-like) guides with a
  Bloch-periodic x (k_x != 0, complex fields; the Bloch oracle) and CPML
  along y;
* ``tmte_2d``: the Cartesian TM + TE force of the Lorentz waveguides
  (general kernel) with the CPML on all four sides.

Tolerances as for the other reduced paths: FP64 fields 1e-9 of the largest
channel per channel and of the term magnitude sum_c |s_c acc_c| / pi for
the force; FP32 fields with FP64 accumulation 2e-5.  The batched split
path, channel waves and (Cartesian) the plain path agree bit for bit.
"""
import numpy as np
import pytest

import oracle
from casimir_inputs import kz_workload, slabs_open_1d, waveguides_open_2d
from oracle import bloch, kz

pytestmark = pytest.mark.gpu

SI = ((10.835, 22.0),)


def announce(name):
    print(f"\n[case] {name}", flush=True)


def guides(eps_inf, poles, **kw):
    return waveguides_open_2d(20, 0.5, 0.25, 0.25, 0.5, 0.5, eps_inf, poles, n_harm=3, n_steps=300,
                              courant=0.35, **kw)


def bloch_pml_y(eps_inf=4.0, poles=(), kz=(0.5, 2.0), w=(0.4, 0.6), kx=(1.1, 2.3)):
    base = guides(eps_inf, poles)
    P = base.meta["pml_px"]
    wl = base.replace(bc=("periodic", "pml", "periodic"), pml_cells=(0, P, 0))
    return kz_workload(wl, kz, w, kx=kx)


CASES = {
    "slabs": lambda: kz_workload(slabs_open_1d(20, 0.5, 0.25, 0.5, 0.5, 1.5, ((3.0, 3.0),), n_steps=600),
                                 [0.0, 1.0, 3.0], [1.0, 1.0, 1.0]),
    "slabs_tight": lambda: kz_workload(slabs_open_1d(20, 0.5, 0.25, 0.15, 0.5, 1.5, ((3.0, 3.0),), n_steps=400),
                                       [0.0, 2.0], [1.0, 1.0]),
    "waveguides_si": lambda: kz_workload(guides(1.035, SI), [0.0, 2.0, 6.0], [0.2, 0.5, 0.3]),
    "waveguides_eps4": lambda: kz_workload(guides(4.0, ()), [0.0, 2.0, 6.0], [0.2, 0.5, 0.3]),
    "bloch_pml_y": bloch_pml_y,
    "bloch_pml_y_si": lambda: bloch_pml_y(1.035, SI, kz=(2.0,), w=(1.0,), kx=(1.1,)),
}
_ORACLE = {}


def oracle_result(name):
    if name not in _ORACLE:
        wl = CASES[name]()
        if any(wl.kx):
            ref = bloch.solve(wl, list(zip(wl.kx, wl.kz)), wl.kz_weight)
        else:
            ref = kz.solve(wl, wl.kz, wl.kz_weight)
        _ORACLE[name] = (wl, ref)
    return _ORACLE[name]


def run(cf, wl, **over):
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
                precision=wl.precision)
    opts.update(over)
    return cf.Problem.from_workload(wl).solve(**opts)


def check_kz(res, ref, weights, tol):
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
def test_kz_open_matches_oracle(cf, name):
    announce(f"k_z open space vs oracle: {name}")
    wl, ref = oracle_result(name)
    r64 = run(cf, wl, precision="fp64")
    e64 = check_kz(r64, ref, wl.kz_weight, 1e-9)
    r32 = run(cf, wl, precision="fp32")
    e32 = check_kz(r32, ref, wl.kz_weight, 2e-5)
    print(f"[kz-open] {name}: force {r64['force']:.12e} oracle {ref.force:.12e} "
          f"channel err fp64 {e64:.1e} fp32 {e32:.1e}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_kz_open_waves_bitwise(cf, precision):
    """Channel waves (two resident channels at a time) give the batched
    split solve's results bit for bit: each wave clears its CPML and
    polarization blocks."""
    announce(f"k_z open space: batched vs channel waves, {precision}")
    wl, _ = oracle_result("waveguides_si")
    a = run(cf, wl, precision=precision)
    b = run(cf, wl, precision=precision, max_resident=2)
    np.testing.assert_array_equal(a["per_channel"], b["per_channel"])
    assert a["force"] == b["force"]


def test_cartesian_2d_pml_and_lorentz(cf):
    announce("Cartesian TM+TE waveguides with CPML and Lorentz media vs oracle, plain and waves bitwise")
    wl = guides(1.5, ((3.0, 3.0),)).replace(coord="cartesian", pol="TM+TE", kernel="general")
    ref = oracle.solve(wl)
    terms = float(np.sum(np.abs(ref.sign * ref.acc)) / np.pi)
    for precision, tol in (("fp64", 1e-9), ("fp32", 2e-5)):
        g = run(cf, wl, precision=precision)
        assert not g["fused"]
        assert abs(g["force"] - ref.force) <= tol * terms, (precision, g["force"], ref.force, terms)
        np.testing.assert_allclose(g["per_channel"], ref.acc, rtol=0, atol=tol * np.max(np.abs(ref.acc)))
        p = run(cf, wl, precision=precision, path="plain")
        w = run(cf, wl, precision=precision, max_resident=3)
        np.testing.assert_array_equal(g["per_channel"], p["per_channel"])
        np.testing.assert_array_equal(g["per_channel"], w["per_channel"])
    print(f"[kz-open] tmte_2d: force {g['force']:.12e} oracle {ref.force:.12e}", flush=True)

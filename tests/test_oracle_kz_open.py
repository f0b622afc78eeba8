"""Pins of the oracle's k_z runs in open space: dispersive dielectrics
(Sec. III B: Lorentz models continued onto the conductivity contour) with
a CPML on the two in-plane axes (Sec. III B: the waveguides sit in empty
space, bounded by perfectly matched layers; one two-dimensional run per
k_z).

* Two identical Lorentz slabs a gap apart in open space (x CPML, one-cell
  periodic y, so only k_y = 0): at each k_z the force on the right slab is
  the Lifshitz result at in-plane wavevector k,
      F(k) = -(1/pi) sum_{TE,TM} int_0^inf dxi k0 R e^{-2 a k0} / (1 - R e^{-2 a k0}),
  k0 = sqrt(xi^2 + k^2), R = r_slab^2 with the finite-slab reflection
  r01 (1 - e^{-2 k1 d}) / (1 - r01^2 e^{-2 k1 d}), k1 = sqrt(eps(i xi) xi^2 + k^2),
  r01 = (k0 - k1)/(k0 + k1) (TE) or (eps k0 - k1)/(eps k0 + k1) (TM), and
  eps(i xi) = eps_inf + sum d_eps w0^2 / (w0^2 + xi^2): the physical
  permittivity on the imaginary axis, with no sigma in it.  The staircase
  slab faces (closed boxes: the tangential E rows on both faces are inside)
  make the grid error first order; it halves with the cell size and the
  first-order Richardson extrapolation of two grids lands on the closed
  form.  This checks the Lorentz continuation, the k couplings, the open
  boundary and the stress-tensor force together.
* The CPML on both in-plane axes at k_z != 0: a pulse in all six
  components inside a small box with the layers matches, in the box's
  interior, the same pulse in a box three times as large with PEC walls (a
  brute-force open space until its walls' echo returns), to 5e-4 of the
  interior field; with PEC walls in place of the layers the echo is of the
  order of the field itself.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from casimir_inputs.configs import slabs_open_1d
from casimir_inputs.geometry import Workload, rasterize
from oracle import kz

A, D, PAD, PML = 0.5, 0.25, 0.5, 0.5
EPS_INF, POLES = 1.5, ((3.0, 3.0),)


def eps_imag(xi, eps_inf=EPS_INF, poles=POLES):
    return eps_inf + sum(de * w0 ** 2 / (w0 ** 2 + xi ** 2) for de, w0 in poles)


def lifshitz_slabs(k, a=A, d=D, eps_inf=EPS_INF, poles=POLES):
    """Force per unit area and per unit k_z weight on the right slab, along +x."""
    def integrand(xi):
        k0 = np.sqrt(xi * xi + k * k)
        e = eps_imag(xi, eps_inf, poles)
        k1 = np.sqrt(e * xi * xi + k * k)
        tot = 0.0
        for r01 in ((k0 - k1) / (k0 + k1), (e * k0 - k1) / (e * k0 + k1)):
            ed = np.exp(-2.0 * k1 * d)
            rs = r01 * (1.0 - ed) / (1.0 - r01 * r01 * ed)
            x = rs * rs * np.exp(-2.0 * k0 * a)
            tot += k0 * x / (1.0 - x)
        return tot
    return -quad(integrand, 0.0, np.inf, limit=400, epsabs=1e-14, epsrel=1e-12)[0] / np.pi


def test_dispersive_slabs_in_open_space_converge_to_lifshitz():
    ks = [0.0, 1.0, 3.0]
    exact = np.array([lifshitz_slabs(k) for k in ks])
    errs = []
    for res in (40, 80):
        wl = slabs_open_1d(res, A, D, PAD, PML, EPS_INF, POLES, n_steps=int(40.0 / (0.5 / res)))
        r = kz.solve(wl, ks, [1.0] * len(ks))
        errs.append(np.array(r.per_k) / exact - 1.0)
    e40, e80 = errs
    print("closed form", exact, "errors at 40 / 80 cells per unit", e40, e80)
    assert np.all(exact < 0)                                  # attraction
    assert np.all((e40 / e80 > 1.8) & (e40 / e80 < 2.3)), (e40, e80)   # first order
    assert np.all(np.abs(2.0 * e80 - e40) < 6e-3), (e40, e80)          # Richardson


def test_dispersion_is_resolved_between_the_static_and_optical_limits():
    """At k = 1 the Lorentz slabs' force lies strictly between those of plain
    dielectrics at eps_inf and at eps_inf + d_eps, far from both."""
    res, k = 40, 1.0
    f = {}
    for name, eps, poles in (("lor", EPS_INF, POLES), ("opt", EPS_INF, ()), ("static", EPS_INF + POLES[0][0], ())):
        wl = slabs_open_1d(res, A, D, PAD, PML, eps, poles, n_steps=int(40.0 / (0.5 / res)))
        f[name] = kz.solve(wl, [k], [1.0]).per_k[0]
    lo, hi = sorted((f["opt"], f["static"]))
    assert lo < f["lor"] < hi
    assert min(abs(f["lor"] - lo), abs(f["lor"] - hi)) > 0.05 * (hi - lo)


def _box(n, bc, P):
    ids = rasterize((n, n, 1), [])
    return Workload(name="box", ndim=2, shape=(n, n, 1), res=20.0, bc=(bc, bc, "periodic"),
                    pml_cells=(P, P, 0) if bc == "pml" else (0, 0, 0), eps=[1.0], mu=[1.0], comp_ids=ids,
                    s_lo=(n // 2 - 2, n // 2 - 2, 0), s_hi=(n // 2 + 2, n // 2 + 2, 1), n_harm=1, force_axis=0,
                    sigma=0.0, courant=0.5, pol="3D", kernel="general", coord="kz", kz=(0.0,), kz_weight=(1.0,))


def _pulse(n, bc, P, k, steps):
    sim = kz.KzSim(_box(n, bc, P), "E", 1, k)
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    g = np.exp(-((I - n / 2) ** 2 + (J - n / 2 + 3) ** 2) / 6.0)
    sim.E["z"][0, 0] = g
    sim.E["x"][0, 0] = 0.5 * np.roll(g, 2, axis=1)
    sim.start()
    for _ in range(steps):
        sim.step()
    return sim


def _interior_mismatch(small, big, n, P):
    o = (big.E["x"].shape[-1] - n) // 2
    c0, c1 = P + 2, n - P - 2
    num = den = 0.0
    for f in ("E", "H"):
        for comp in "xyz":
            a = getattr(small, f)[comp][0, 0, c0:c1, c0:c1]
            b = getattr(big, f)[comp][0, 0, o + c0:o + c1, o + c0:o + c1]
            num += float(np.sum((a - b) ** 2))
            den += float(np.sum(b ** 2))
    return np.sqrt(num / den)


@pytest.mark.parametrize("k", [0.0, 1.5, 6.0])
def test_kz_pml_matches_a_large_box(k):
    n, P, steps = 64, 12, 140
    big = _pulse(3 * n, "pec", 0, k, steps)
    assert _interior_mismatch(_pulse(n, "pml", P, k, steps), big, n, P) < 5e-4
    if k == 1.5:
        assert _interior_mismatch(_pulse(n, "pec", 0, k, steps), big, n, P) > 0.5

"""Pins of the k_z oracle (z-invariant 2D problems at a Bloch wavevector k
along the invariant axis: Sec. III B, Sec. III D).

* Exact discrete energy conservation at sigma = 0 for k != 0 with PEC and
  periodic y walls (the k couplings enter the two half steps as transposes).
* k = 0 splits into TM and TE: the six-component force equals the TM+TE
  force of the Cartesian oracle (general kernel) to rounding.
* F(-k) = F(k) (the reflection z -> -z).
* Parallel PEC plates (a PEC slab between walls at distances a and b,
  uniform along y with a one-cell periodic y, so only k_y = 0): at each k
  the two polarizations give 2 [F1(a, k) - F1(b, k)],
  F1(a, k) = -(1/pi) int_0^inf dxi kappa / (exp(2 a kappa) - 1),
  kappa = sqrt(xi^2 + k^2) (each fixed-k mode of the gap is a 1+1D field of
  mass k); the error falls at second order in the cell size.  Integrated
  over k with (1/pi) int dk this is the z-invariant plate result
  -(zeta(3)/8 pi)(1/a^3 - 1/b^3) per polarization that the Cartesian oracle
  is pinned to.
* The stability limit 2 / sqrt(8 + (k dx)^2): growth just above it, none
  just below.
* The k integral (1/pi) int_0^inf F(k) dk of the plates (8-point
  Gauss-Legendre on [0, 12]; F(k) falls like exp(-2 a k)) equals the
  z-invariant-kernel TM + TE force on the same grid to 5e-4 (Appendix A.2:
  that kernel is the k_z integral done in closed form), and both approach
  the exact plate force.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import zeta

import oracle
from casimir_inputs.configs import kz_gauss, kz_workload, parallel_plates_1d, piston2d
from oracle import kz

A, D, B = 0.5, 0.25, 1.0


def F1(a, k):
    f = lambda xi: np.sqrt(xi * xi + k * k) / np.expm1(min(2 * a * np.sqrt(xi * xi + k * k), 700.0))
    return -quad(f, 0, np.inf, limit=200)[0] / np.pi


def small_piston(n_steps=300):
    return piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, pol="3D", n_steps=n_steps, n_harm=6, kernel="general")


@pytest.mark.parametrize("ybc", ["pec", "periodic"])
@pytest.mark.parametrize("k", [0.7, 3.1])
def test_energy_conserved_exactly(k, ybc):
    wl = small_piston().replace(bc=("pec", ybc, "periodic"), sigma=0.0)
    S = kz.KzSim(wl, "E", 1, k)
    rng = np.random.default_rng(5)
    for f in (S.E, S.H):
        for a in f:
            f[a] = rng.standard_normal(f[a].shape)
    # conductors and walls: zero where the coefficients vanish
    for a in S.E:
        S.E[a] *= S.cb[a] != 0
    for a in S.H:
        S.H[a] *= S.db[a] != 0
    U = []
    for _ in range(400):
        ue = sum(float((S.E[a] ** 2).sum()) for a in S.E)
        hp = {a: S.H[a].copy() for a in S.H}
        S.step_h()
        U.append(ue + sum(float((hp[a] * S.H[a]).sum()) for a in S.H))
        S.step_e()
    U = np.array(U)
    assert np.max(np.abs(U / U[0] - 1)) < 1e-12


def test_k0_equals_tm_plus_te():
    wl = small_piston()
    r0 = kz.solve(wl, [0.0], [1.0])
    ref = oracle.solve(wl.replace(pol="TM+TE"))
    assert r0.per_k[0] == pytest.approx(ref.force, rel=1e-12)


def test_even_in_k():
    wl = small_piston(n_steps=200)
    r = kz.solve(wl, [1.3, -1.3], [1.0, 1.0])
    assert r.per_k[0] == pytest.approx(r.per_k[1], rel=1e-12)
    assert abs(r.per_k[0]) > 0


def test_plates_converge_to_closed_form():
    ks = [0.0, 1.0, 2.0, 4.0]
    errs = []
    for res in (20, 40):
        wl = parallel_plates_1d(res, A, D, B, pol="3D", kernel="general", n_steps=int(40 / (0.5 / res)))
        r = kz.solve(wl, ks, [1.0] * len(ks))
        errs.append([f / (2 * (F1(A, k) - F1(B, k))) - 1 for f, k in zip(r.per_k, ks)])
    errs = np.array(errs)
    print("relative errors at 20 / 40 cells per unit, k =", ks, errs)
    assert np.all(np.abs(errs[1]) < 6e-3)
    assert np.all(np.abs(errs[0]) / np.abs(errs[1]) > 3.5)     # second order: 4x per halving


def test_courant_limit():
    wl = small_piston().replace(sigma=0.0)
    k = 20.0                                                   # k dx = 2: limit 2/sqrt(12) = 0.577
    lim = kz.kz_courant_limit(k, wl.res)

    def grows(c):
        S = kz.KzSim(wl, "E", 1, k, courant=c)
        rng = np.random.default_rng(2)
        for f in (S.E, S.H):
            for a in f:
                f[a] = rng.standard_normal(f[a].shape)
        with np.errstate(all="ignore"):
            for _ in range(1500):
                S.step()
        return not max(np.abs(S.E[a]).max() for a in S.E) < 100
    assert lim == pytest.approx(2 / np.sqrt(12))
    assert grows(lim * 1.02)
    assert not grows(lim * 0.98)


def test_k_integral_equals_z_invariant_kernel():
    res = 20
    base = parallel_plates_1d(res, A, D, B, n_steps=int(40 / (0.5 / res)))
    ks, ws = kz_gauss(8, 12.0)
    f_kz = kz.solve(kz_workload(base, ks, ws), ks, ws).force
    f_2d = oracle.solve(base.replace(pol="TM+TE", kernel="zinv2d")).force
    exact = -2 * zeta(3) / (8 * np.pi) * (A ** -3 - B ** -3)
    assert f_kz / f_2d - 1 == pytest.approx(0.0, abs=5e-4)
    assert abs(f_kz / exact - 1) < 0.015

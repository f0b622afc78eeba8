"""Pins of the Bloch-periodic oracle (Sec. III D: a cell periodic in x with
period L, invariant in z; one simulation per Bloch wavevector (k_x, k_z)).

* Bloch folding, exact on the grid: a supercell of two periods at k_x
  carries the Green's function (1/2) [G_L(k_x) + G_L(k_x + pi/L)] of the
  one-period cell, so with S around the same object
  F_2L(k_x) = (F_L(k_x) + F_L(k_x + pi/L)) / 2 to rounding, at k_z = 0 and
  k_z != 0.  A missing or wrong phase on either half step breaks it.
* k_x = 0 is the real k_z run of oracle.kz (to rounding).
* F(-k_x) = F(k_x) (the runs are complex conjugates).
* Discrete energy (eps |E|^2 + mu Re H^{n-1/2} . conj H^{n+1/2}) is
  conserved at sigma = 0.
* A stress surface whose stencil crosses the periodic edge is rejected.
"""
import numpy as np
import pytest

from casimir_inputs.geometry import Box, Workload, rasterize
from oracle import bloch, kz

BIG = 1e30


def grating(ncell=1, L=24, ny=30, res=10.0, n_steps=300, s_lo=(6, 10, 0), s_hi=(18, 20, 1)):
    """Dielectric blocks (eps 4, 8 x 6 cells) repeated with period L above a
    PEC plate; S around the block of the first period."""
    nx = L * ncell
    prims = [Box((-BIG, -BIG, -BIG), (BIG, 4, BIG), 1)]
    for c in range(ncell):
        prims.append(Box((c * L + 8, 12, -BIG), (c * L + 16, 18, BIG), 2))
    ids = rasterize((nx, ny, 1), prims)
    return Workload(name="grating", ndim=2, shape=(nx, ny, 1), res=res, bc=("periodic", "pec", "periodic"),
                    pml_cells=(0, 0, 0), eps=[1.0, float("-inf"), 4.0], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                    s_lo=s_lo, s_hi=s_hi, n_harm=4, force_axis=1, pol="3D", kernel="general",
                    n_steps=n_steps, sigma=1.0, courant=0.5)


@pytest.mark.parametrize("kx,kz_", [(0.4, 0.0), (0.4, 0.9)])
def test_supercell_folding(kx, kz_):
    L = 24 / 10.0
    prim = bloch.solve(grating(1), [(kx, kz_), (kx + np.pi / L, kz_)], [0.5, 0.5])
    sup = bloch.solve(grating(2), [(kx, kz_)], [1.0])
    assert sup.force == pytest.approx(prim.force, rel=1e-10)
    assert abs(prim.per_k[0] - prim.per_k[1]) > 1e-4 * abs(prim.force)      # the two k_x differ


def test_kx0_equals_kz_run():
    wl = grating(1, n_steps=200)
    assert bloch.solve(wl, [(0.0, 0.7)], [1.0]).force == pytest.approx(kz.solve(wl, [0.7], [1.0]).force,
                                                                        rel=1e-13)


def test_even_in_kx():
    r = bloch.solve(grating(1, n_steps=200), [(0.5, 0.3), (-0.5, 0.3)], [1.0, 1.0])
    assert r.per_k[0] == pytest.approx(r.per_k[1], rel=1e-12)


def test_energy_conserved_exactly():
    wl = grating(1).replace(sigma=0.0)
    S = bloch.BlochSim(wl, "E", 1, 0.8, 0.9)
    rng = np.random.default_rng(4)
    for f, co in ((S.E, S.cb), (S.H, S.db)):
        for a in f:
            f[a] = (rng.standard_normal(f[a].shape) + 1j * rng.standard_normal(f[a].shape)) * (co[a] != 0)
    # eps and mu of every component from the lossless coefficients b = courant / (eps or mu)
    we = {a: np.where(S.cb[a] != 0, S.courant / np.where(S.cb[a] != 0, S.cb[a], 1.0), 0.0) for a in S.E}
    wh = {a: np.where(S.db[a] != 0, S.courant / np.where(S.db[a] != 0, S.db[a], 1.0), 0.0) for a in S.H}
    U = []
    for _ in range(300):
        ue = sum(float(np.sum(we[a] * np.abs(S.E[a]) ** 2)) for a in S.E)
        hp = {a: S.H[a].copy() for a in S.H}
        S.step_h()
        U.append(ue + sum(float(np.sum(wh[a] * (hp[a] * np.conj(S.H[a])).real)) for a in S.H))
        S.step_e()
    U = np.array(U)
    assert np.max(np.abs(U / U[0] - 1)) < 1e-12


def test_surface_across_the_edge_rejected():
    with pytest.raises(ValueError):
        bloch.solve(grating(1, s_lo=(0, 10, 0), s_hi=(18, 20, 1)), [(0.3, 0.0)], [1.0])
    with pytest.raises(ValueError):
        bloch.solve(grating(1, s_lo=(6, 10, 0), s_hi=(24, 20, 1)), [(0.3, 0.0)], [1.0])

"""Pins of the oracle's Minkowski factors: the stress tensor on S carries the
permittivity and permeability of the medium S lies in (Sec. II, the stress
tensor Gamma^E and its "similar definition" for Gamma^H), and so does the
delta(t) kick (the current enters Ampere's and Faraday's laws divided by eps
and mu).  The vacuum pins cannot see these factors; these can.

* Closed form.  Perfect-conductor plates separated by a uniform,
  non-dispersive medium (eps, mu): every mode frequency is the vacuum one
  divided by n = sqrt(eps mu), so the force is the vacuum force divided by n.
  F * n converges to the vacuum closed form at second order in the grid
  spacing, in 1D-reduced 2D runs (TM and TE) and in 3D, for eps != mu.
* Exact scaling identity (any perfect-conductor geometry, any dielectrics).
  Multiplying every finite eps by alpha and every mu by beta is, on the Yee
  grid, the original scheme with E' = sqrt(alpha) E, H' = sqrt(beta) H and
  time t' = t / n (n = sqrt(alpha beta)): the same discrete problem with
  Courant number courant / n and conductivity sigma * n.  With the general
  kernel K_sigma(n t) = K_{n sigma}(t) / n^2, and the Minkowski weights and
  the kicks cancel the field scalings, so
      F(alpha eps, beta mu; courant, sigma) * n = F(eps, mu; courant / n, sigma n)
  to rounding.  This pins the factors on every channel kind (shear faces
  included) and on the sphere-in-fluid configuration of the 3D benchmark,
  where S lies in eps = 1.8.  A planted mistake (S's permittivity dropped
  from the stress weights) breaks it.
* The z-invariant kernel's premise (Appendix A.2: perfect conductors in
  vacuum): the oracle refuses it for a medium; under the same scaling it
  would give the vacuum force over n^2, not n.
"""
import numpy as np
import pytest

import oracle
import oracle.surface
from casimir_inputs.configs import parallel_plates_1d, piston2d
from casimir_inputs.geometry import Box, Sphere, Workload, rasterize

A, D, B = 1.0, 0.5, 1.5
PEC = float("-inf")
BIG = 1e30
MEDIA = [(1.8, 1.0), (2.25, 1.0), (1.0, 1.69), (1.8, 1.3)]


def in_medium(wl, eps_m, mu_m):
    """Every finite eps scaled by eps_m and every mu by mu_m (perfect
    conductors stay)."""
    eps = [e * eps_m if np.isfinite(e) else e for e in wl.eps]
    mu = [m * mu_m if np.isfinite(m) else m for m in wl.mu]
    return wl.replace(eps=eps, mu=mu)


def term_scale(r):
    return sum(abs(v) for v in r.per_face.values())


@pytest.mark.parametrize("pol", ["TM", "TE"])
@pytest.mark.parametrize("eps_m,mu_m", MEDIA)
def test_plates_1d_in_medium_closed_form(pol, eps_m, mu_m):
    n = np.sqrt(eps_m * mu_m)
    ex = -np.pi / 24 * (A ** -2 - B ** -2)
    errs = []
    for res in (20, 40):
        wl = parallel_plates_1d(res, A, D, B, pol=pol, kernel="general", n_steps=int(40 / (0.5 / res)))
        f = oracle.solve(in_medium(wl, eps_m, mu_m)).force
        errs.append(f * n / ex - 1)
    assert abs(errs[1]) < 1e-3, errs
    assert 1.8 < np.log2(abs(errs[0] / errs[1])) < 2.2, errs


def plates_z(res, eps_m, mu_m):
    a, d, b = int(A * res), int(D * res), int(B * res)
    nz = a + d + b
    ids = rasterize((1, 1, nz), [Box((-BIG, -BIG, a), (BIG, BIG, a + d), 1)])
    return Workload(name="pz", ndim=3, shape=(1, 1, nz), res=float(res), bc=("periodic", "periodic", "pec"),
                    pml_cells=(0, 0, 0), eps=[eps_m, PEC], mu=[mu_m, 1.0], comp_ids=ids,
                    s_lo=(0, 0, a - 2), s_hi=(1, 1, a + d + 2), n_harm=1, force_axis=2, pol="3D",
                    kernel="general", n_steps=int(40 / (0.5 / res)))


@pytest.mark.parametrize("eps_m,mu_m", [(1.8, 1.0), (1.8, 1.3)])
def test_plates_3d_in_fluid_closed_form(eps_m, mu_m):
    """Two polarizations of the 1+1D force, divided by n (the fluid of the
    sphere-plate benchmark has eps = 1.8)."""
    n = np.sqrt(eps_m * mu_m)
    ex = -2 * np.pi / 24 * (A ** -2 - B ** -2)
    errs = [oracle.solve(plates_z(res, eps_m, mu_m)).force * n / ex - 1 for res in (20, 40)]
    assert abs(errs[1]) < 1e-3, errs
    assert 1.8 < np.log2(abs(errs[0] / errs[1])) < 2.2, errs


def piston(pol):
    return piston2d(24, 18, 3, 6, 4, 6, 7, 6.0, pol=pol, n_harm=5, n_steps=160, kernel="general")


def sphere_pair(eps_sphere):
    """A sphere of eps_sphere in the background material 0 above a PEC
    plate, S a box around the sphere (faces normal to x, y and z)."""
    nx, ny, nz = 10, 9, 14
    prims = [Box((-BIG, -BIG, -BIG), (BIG, BIG, 2), 1), Sphere((5.2, 4.5, 7.0), 1.6, 2)]
    ids = rasterize((nx, ny, nz), prims)
    return Workload(name="sp", ndim=3, shape=(nx, ny, nz), res=4.0, bc=("periodic", "periodic", "pec"),
                    pml_cells=(0, 0, 0), eps=[1.0, PEC, eps_sphere], mu=[1.0, 1.0, 1.0], comp_ids=ids,
                    s_lo=(2, 2, 4), s_hi=(8, 7, 10), n_harm=2, force_axis=2, pol="3D", kernel="general",
                    n_steps=50)


def scaled_pair(wl, eps_m, mu_m):
    """(the problem in the medium, the equivalent vacuum-scaled problem)."""
    n = np.sqrt(eps_m * mu_m)
    return in_medium(wl, eps_m, mu_m), wl.replace(courant=wl.courant / n, sigma=wl.sigma * n), n


GEOMS = {
    "piston_tm": lambda: piston("TM"),
    "piston_te": lambda: piston("TE"),
    "sphere_pec_3d": lambda: sphere_pair(PEC),
    # the benchmark's ratio: sphere eps 2.1 in fluid 1.8 is this base scaled by alpha = 1.8
    "sphere_in_fluid_3d": lambda: sphere_pair(2.1 / 1.8),
}


@pytest.mark.parametrize("geom", sorted(GEOMS))
@pytest.mark.parametrize("eps_m,mu_m", [(2.25, 1.0), (1.0, 1.69), (1.8, 1.3)])
def test_medium_scaling_identity(geom, eps_m, mu_m):
    if geom.endswith("3d") and (eps_m, mu_m) == (1.0, 1.69):
        pytest.skip("two media per 3D geometry keep the CPU suite short")
    base = GEOMS[geom]()
    med, vac, n = scaled_pair(base, eps_m, mu_m)
    r_med = oracle.solve(med)
    r_vac = oracle.solve(vac)
    assert r_med.eps_s == pytest.approx(eps_m) and r_med.mu_s == pytest.approx(mu_m)
    scale = term_scale(r_vac)
    assert abs(r_med.force * n - r_vac.force) <= 1e-11 * scale, (r_med.force * n, r_vac.force, scale)
    for f in r_vac.per_face:
        assert abs(r_med.per_face[f] * n - r_vac.per_face[f]) <= 1e-11 * scale
    # the force is not lost in the early-time terms that cancel between faces
    # (the 1e-11 tolerance is below 1e-7 of the force on every geometry here)
    assert abs(r_vac.force) > 1e-4 * scale


def test_planted_missing_permittivity_breaks_the_identity(monkeypatch):
    base = piston("TM")
    med, vac, n = scaled_pair(base, 1.8, 1.3)
    good = oracle.solve(med).force * n
    ref = oracle.solve(vac).force
    orig = oracle.surface.channel_specs

    def dropped(pol, face_axis, d, eps_s, mu_s):
        return orig(pol, face_axis, d, 1.0, mu_s)     # S's permittivity left out of the stress weights

    monkeypatch.setattr(oracle.surface, "channel_specs", dropped)
    bad = oracle.solve(med).force * n
    assert good == pytest.approx(ref, rel=1e-9)
    assert abs(bad / ref - 1) > 0.05


def test_zinv_kernel_refused_in_a_medium():
    wl = parallel_plates_1d(10, A, D, B, pol="TM", kernel="zinv2d", n_steps=50)
    oracle.solve(wl)                                   # vacuum + PEC: fine
    with pytest.raises(ValueError):
        oracle.solve(in_medium(wl, 1.8, 1.0))
    with pytest.raises(ValueError):
        oracle.solve(piston2d(24, 18, 3, 6, 4, 6, 7, 6.0, pol="TM", n_steps=20, sidewall="mu5",
                              kernel="zinv2d"))
    # PMC sidewalls are perfect (magnetic) conductors: still allowed
    oracle.solve(piston2d(24, 18, 3, 6, 4, 6, 7, 6.0, pol="TM", n_steps=20, sidewall="pmc"))


def test_zinv_kernel_in_medium_would_give_vacuum_over_n_squared():
    """Why the premise matters: the z-invariant kernel scales as
    K_sigma(n t) = K_{n sigma}(t) / n^3, so the scaled problem's force comes
    out as the vacuum force over n^2 instead of n (computed here with the
    kernel sums directly, bypassing the refusal)."""
    from oracle.kernels import kernel_table
    n, sigma, dt, T = 1.5, 1.0, 0.025, 400
    k_med = kernel_table("zinv2d", sigma, dt, T)
    k_vac = kernel_table("zinv2d", sigma * n, dt / n, T)
    np.testing.assert_allclose(dt * k_med, (dt / n) * k_vac / n ** 2, rtol=1e-12)
    k_med_g = kernel_table("general", sigma, dt, T)
    k_vac_g = kernel_table("general", sigma * n, dt / n, T)
    np.testing.assert_allclose(dt * k_med_g, (dt / n) * k_vac_g / n, rtol=1e-12)

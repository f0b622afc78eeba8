"""Pins of the oracle's Yee leapfrog (Sec. II; the Yee scheme of Taflove).

* sigma = 0: the staggered discrete energy
  W^m = 1/2 sum eps |E^m|^2 + 1/2 sum mu H^{m-1/2} . H^{m+1/2}
  is conserved to rounding, with PEC walls, periodic walls, PEC blocks and
  eps/mu maps, in 2D (TM, TE) and 3D.  A wrong sign or index in any curl
  component breaks the adjointness this rests on;
* sigma > 0: the exact discrete dissipation identity of the time-centred loss,
  W^{m+1} - W^m = -(sigma dt / 4) sum eps |E^{m+1} + E^m|^2;
* a periodic plane wave follows the Yee dispersion relation
  sin(omega dt/2) = S_c sqrt(sum_a sin^2(k_a dx/2)) exactly (E^m = cos(m
  theta) E^0 with the consistent start);
* the CPML absorbs an outgoing pulse.
"""
import numpy as np
import pytest

from casimir_inputs.geometry import Box, PEC, Sphere, Workload, rasterize
from oracle.surface import POL_COMPONENTS
from oracle.yee import YeeSim

BIG = 1e30


def make_wl(shape, bc, prims, eps, mu, sigma=0.0, ndim=2, pml=(0, 0, 0), courant=0.5):
    ids = rasterize(shape, prims)
    return Workload(name="t", ndim=ndim, shape=shape, res=10.0, bc=bc, pml_cells=pml,
                    eps=eps, mu=mu, comp_ids=ids, s_lo=(1, 1, 0), s_hi=(2, 2, 1), n_harm=1,
                    force_axis=0, sigma=sigma, courant=courant)


def energy_terms(sim, wl, eps, mu):
    e_tab = np.asarray(eps)
    m_tab = np.asarray(mu)
    we = 0.0
    for a, F in sim.E.items():
        e = e_tab[wl.comp_ids["E" + a]]
        e = np.where(np.isfinite(e), e, 0.0)
        we += 0.5 * np.sum(e * F * F)
    return we, {a: F.copy() for a, F in sim.H.items()}


def run_energy(wl, eps, mu, pol, kind, n_steps, seed=0):
    rng = np.random.default_rng(seed)
    e_axes, h_axes = POL_COMPONENTS[pol]
    sim = YeeSim(wl, kind, 2, e_axes, h_axes)
    for a in sim.E:
        sim.E[a][:] = rng.standard_normal(sim.E[a].shape) * (sim.cb[a] != 0)
    for a in sim.H:
        sim.H[a][:] = rng.standard_normal(sim.H[a].shape) * (sim.db[a] != 0)
    m_tab = np.asarray(mu)
    W = []
    prev_e = None
    dis = []
    h_prev = {a: F.copy() for a, F in sim.H.items()}
    for m in range(n_steps):
        we, _ = energy_terms(sim, wl, eps, mu)
        e_old = {a: F.copy() for a, F in sim.E.items()}
        sim.step()
        wh = 0.0
        for a, F in sim.H.items():
            mm = m_tab[wl.comp_ids["H" + a]]
            mm = np.where(np.isfinite(mm), mm, 0.0)
            wh += 0.5 * np.sum(mm * h_prev[a] * F)
        W.append(we + wh)
        h_prev = {a: F.copy() for a, F in sim.H.items()}
        s = 0.0
        for a, F in sim.E.items():
            e = np.asarray(eps)[wl.comp_ids["E" + a]]
            e = np.where(np.isfinite(e), e, 0.0)
            s += np.sum(e * (F + e_old[a]) ** 2)
        dis.append(s)
    return np.array(W), np.array(dis), sim


CASES_2D = [
    ("pec", ("pec", "pec", "periodic")),
    ("periodic", ("periodic", "periodic", "periodic")),
    ("mixed", ("periodic", "pec", "periodic")),
]


@pytest.mark.parametrize("pol", ["TM", "TE"])
@pytest.mark.parametrize("name,bc", CASES_2D)
def test_energy_conserved_2d(pol, name, bc):
    eps = [1.0, PEC, 2.5]
    mu = [1.0, 1.0, 1.7]
    prims = [Box((5, 4, -BIG), (9, 8, BIG), 1), Sphere((14, 9, 0.5), 3.2, 2)]
    wl = make_wl((20, 16, 1), bc, prims, eps, mu)
    W, _, _ = run_energy(wl, eps, mu, pol, "E", 400)
    assert np.max(np.abs(W - W[0])) <= 1e-12 * abs(W[0])


def test_energy_conserved_3d():
    eps = [1.8, PEC, 2.1]
    mu = [1.0, 1.0, 1.0]
    prims = [Box((-BIG, -BIG, -BIG), (BIG, BIG, 3), 1), Sphere((6, 5, 7), 2.5, 2)]
    wl = make_wl((12, 10, 12), ("periodic", "periodic", "pec"), prims, eps, mu, ndim=3)
    W, _, _ = run_energy(wl, eps, mu, "3D", "E", 150)
    assert np.max(np.abs(W - W[0])) <= 1e-12 * abs(W[0])


def test_dissipation_identity_e_kind():
    eps = [1.0, PEC, 3.0]
    mu = [1.0, 1.0, 1.0]
    sigma = 1.3
    prims = [Box((5, 4, -BIG), (9, 8, BIG), 1), Sphere((14, 9, 0.5), 3.2, 2)]
    wl = make_wl((20, 16, 1), ("pec", "pec", "periodic"), prims, eps, mu, sigma=sigma)
    W, dis, sim = run_energy(wl, eps, mu, "TM", "E", 200)
    # dis[m] = sum eps |E^{m+1} + E^m|^2, W[m] = W^m
    pred = -(sigma * (wl.courant / wl.res) / 4.0) * dis[:-1]
    inc = W[1:] - W[:-1]
    np.testing.assert_allclose(inc, pred, rtol=1e-9, atol=1e-13 * abs(W[0]))


@pytest.mark.parametrize("k", [(1, 0), (2, 3), (5, 1)])
def test_yee_dispersion_relation(k):
    nx, ny = 16, 12
    wl = make_wl((nx, ny, 1), ("periodic", "periodic", "periodic"), [], [1.0], [1.0], courant=0.6)
    sim = YeeSim(wl, "E", 1, ("z",), ("x", "y"))
    kx, ky = 2 * np.pi * k[0] / nx, 2 * np.pi * k[1] / ny
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    sim.E["z"][0, 0] = np.cos(kx * I + ky * J)
    sim.start()
    s = wl.courant * np.sqrt(np.sin(kx / 2) ** 2 + np.sin(ky / 2) ** 2)
    theta = 2 * np.arcsin(s)
    E0 = sim.E["z"][0, 0].copy()
    for m in range(1, 60):
        sim.step()
        np.testing.assert_allclose(sim.E["z"][0, 0], np.cos(m * theta) * E0, atol=1e-11)


def test_pml_absorbs_outgoing_pulse():
    n = 64
    wl = make_wl((n, n, 1), ("pml", "pml", "periodic"), [], [1.0], [1.0], pml=(12, 12, 0))
    sim = YeeSim(wl, "E", 1, ("z",), ("x", "y"))
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    sim.E["z"][0, 0] = np.exp(-((I - n / 2) ** 2 + (J - n / 2) ** 2) / 8.0)
    sim.start()
    e0 = np.sum(sim.E["z"] ** 2)
    for _ in range(400):
        sim.step()
    assert np.sum(sim.E["z"] ** 2) < 1e-5 * e0   # what remains is the 2D wake
    # the same pulse in a PEC box keeps its energy
    wl2 = make_wl((n, n, 1), ("pec", "pec", "periodic"), [], [1.0], [1.0])
    sim2 = YeeSim(wl2, "E", 1, ("z",), ("x", "y"))
    sim2.E["z"][0, 0] = np.exp(-((I - n / 2) ** 2 + (J - n / 2) ** 2) / 8.0)
    sim2.start()
    for _ in range(400):
        sim2.step()
    assert np.sum(sim2.E["z"] ** 2) > 0.05 * e0

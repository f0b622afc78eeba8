"""Pins of the oracle's dispersive materials (Sec. III B: a Lorentz model of
eps(omega) continued onto the complex conductivity contour, realised as an
auxiliary differential equation).

The reading: on the contour omega^2 = xi^2 + i sigma xi a Lorentz term
d_eps w0^2 / (w0^2 - omega^2) becomes d_eps w0^2 / (w0^2 - xi^2 - i sigma xi),
a polarization with P'' + sigma P' + w0^2 P = d_eps w0^2 E, the conductivity
of an E-kind run acting on D = eps_inf E + P.  Pinned against:

* the non-dispersive oracle: terms of zero strength change nothing (bitwise);
* the Lifshitz closed form of a 1D cavity: a PEC slab between a PEC wall and
  a PEC wall coated with a dispersive layer.  The force depends on the
  layer's physical permittivity on the imaginary axis, eps(i xi) = eps_inf +
  d_eps w0^2 / (w0^2 + xi^2), with no sigma in it, so this checks the mapping
  onto the contour as a whole (a wrong damping in the auxiliary equation
  makes the force depend on sigma);
* sigma independence of the force (Sec. II), up to discretization;
* an independent imaginary-frequency evaluation on the same grid (the
  approach of test_oracle_laplace.py) with eps_c(kappa) = eps_inf +
  d_eps w0^2 / (w0^2 + kappa (kappa + sigma)): the time-domain force
  converges to it at second order in dt;
* boundedness of the lossless (sigma = 0) scheme over a long run, and the
  refusal of unstable terms (w0 dt >= 2) and of S inside a dispersive
  material.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from casimir_inputs.configs import layered_plates_1d, piston2d
from oracle.yee import YeeSim
from test_oracle_laplace import curl_operators  # the spatial operators of the Laplace check

A, D, B = 1.0, 0.5, 1.5
LAYER = 0.3
EPS_INF, POLES = 1.5, ((3.0, 3.0),)


def eps_imag(xi, eps_inf, poles):
    return eps_inf + sum(de * w0 ** 2 / (w0 ** 2 + xi ** 2) for de, w0 in poles)


def cavity_force_closed_form(eps_inf, poles):
    """Force per polarization on the slab (1+1D, perfect mirrors): the gap
    a - layer to the coated wall pulls left, the gap b to the bare wall
    right.  R(xi) = r_slab r_wall with r_slab = -1 and the coated wall's
    r = (r01 - e^{-2 k1 L}) / (1 - r01 e^{-2 k1 L}), r01 = (xi - k1)/(xi + k1),
    k1 = sqrt(eps(i xi)) xi."""
    g = A - LAYER

    def pull(xi):
        k1 = np.sqrt(eps_imag(xi, eps_inf, poles)) * xi
        r01 = (xi - k1) / (xi + k1)
        e = np.exp(-2.0 * k1 * LAYER)
        R = -(r01 - e) / (1.0 - r01 * e)
        x = R * np.exp(-2.0 * xi * g)
        return xi * x / (1.0 - x)

    left = quad(pull, 0.0, np.inf, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    return -left / np.pi + np.pi / (24.0 * B ** 2)


def layered(res, pol, poles=POLES, eps_inf=EPS_INF, sigma=1.0, t_max=40.0):
    return layered_plates_1d(res, A, D, B, LAYER, eps_inf, poles, pol=pol, kernel="general", sigma=sigma,
                             n_steps=int(t_max / (0.5 / res)))


def test_zero_strength_terms_change_nothing():
    base = piston2d(24, 18, 3, 6, 4, 6, 7, 6.0, pol="TM+TE", n_harm=4, n_steps=120, kernel="general")
    ids = {k: v.copy() for k, v in base.comp_ids.items()}
    for v in ids.values():
        v[v == 2] = 3                                  # a dielectric sidewall material with its own id
    diel = base.replace(eps=[1.0, float("-inf"), 1.0, 2.5], mu=[1.0, 1.0, 1.0, 1.0], comp_ids=ids)
    ref = oracle.solve(diel)
    zero = oracle.solve(diel.replace(lorentz={3: ((0.0, 2.0), (0.0, 5.0))}))
    assert zero.force == ref.force
    np.testing.assert_array_equal(zero.acc, ref.acc)


@pytest.mark.parametrize("pol", ["TM", "TE"])
@pytest.mark.parametrize("poles", [(), POLES], ids=["nondispersive", "lorentz"])
def test_coated_cavity_closed_form(pol, poles):
    """The staircase layer interface (a dielectric boundary on the E sample
    row, no subpixel averaging) makes the grid error first order: the error
    halves with the grid spacing (measured 3.3, 1.6, 0.78, 0.39 % for the
    Lorentz layer at 20, 40, 80, 160 cells per unit; the time step moves it
    by 4e-6), and the first-order Richardson extrapolation of the two finest
    grids lands on the closed form."""
    ex = cavity_force_closed_form(EPS_INF, poles)
    errs = [oracle.solve(layered(res, pol, poles)).force / ex - 1 for res in (20, 40, 80)]
    print(f"{pol} {poles}: closed form {ex:.8f}, errors {errs}")
    assert 1.8 < errs[0] / errs[1] < 2.3 and 1.8 < errs[1] / errs[2] < 2.3, errs
    assert abs(2.0 * errs[2] - errs[1]) < 1e-3, errs


def test_dispersive_layer_differs_from_its_static_and_optical_limits():
    """The Lorentz layer's force lies strictly between those of a plain
    dielectric at its optical (eps_inf) and static (eps_inf + d_eps)
    permittivities, far from both: the dispersion is resolved."""
    res = 40
    f = oracle.solve(layered(res, "TM")).force
    lo = oracle.solve(layered(res, "TM", poles=(), eps_inf=EPS_INF)).force
    hi = oracle.solve(layered(res, "TM", poles=(), eps_inf=EPS_INF + POLES[0][0])).force
    assert min(lo, hi) < f < max(lo, hi)
    assert min(abs(f - lo), abs(f - hi)) > 0.05 * abs(hi - lo)


def test_force_does_not_depend_on_sigma():
    """Sec. II: the force is the same for every sigma; with the damping of the
    continued Lorentz term equal to sigma it is, up to O(dt^2)."""
    fs = [oracle.solve(layered(40, "TM", sigma=s, t_max=40.0 / min(s, 1.0))).force for s in (0.5, 1.0, 2.0)]
    ex = cavity_force_closed_form(EPS_INF, POLES)
    assert max(fs) - min(fs) < 2e-3 * abs(ex), fs


def test_planted_undamped_polarization_breaks_sigma_independence(monkeypatch):
    """The continued Lorentz term's damping must be sigma: a polarization
    left undamped (the real-axis model) makes the force depend on sigma by
    about 1 %, six times the bar above."""
    import oracle.yee as yee
    orig = yee.YeeSim.step_e

    def undamped(self):
        saved, self.sigma = self.sigma, 0.0      # only the polarization update reads sigma here
        try:
            orig(self)
        finally:
            self.sigma = saved

    monkeypatch.setattr(yee.YeeSim, "step_e", undamped)
    fs = [oracle.solve(layered(40, "TM", sigma=s, t_max=40.0 / min(s, 1.0))).force for s in (0.5, 1.0, 2.0)]
    assert max(fs) - min(fs) > 6e-3 * abs(cavity_force_closed_form(EPS_INF, POLES)), fs


def eps_c(wl, e_axes, sim_cb_mask, kappa):
    """Per E-component cell: eps_inf + sum d_eps w0^2 / (w0^2 + kappa (kappa + sigma))
    from the workload's own tables (conductors masked out)."""
    eps = np.asarray(wl.eps, dtype=np.float64)
    out = []
    for k, a in enumerate(e_axes):
        ids = wl.comp_ids["E" + a].ravel()
        e = np.where(np.isfinite(eps[ids]), eps[ids], 1.0)
        for m, poles in wl.lorentz.items():
            for de, w0 in poles:
                e = e + np.where(ids == m, de * w0 ** 2 / (w0 ** 2 + kappa * (kappa + wl.sigma)), 0.0)
        out.append(e)
    return np.concatenate(out)


def frequency_force_dispersive(*args, **kw):
    """frequency force dispersive on one BLAS thread (the test runner's
    workers would otherwise oversubscribe the host's cores)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        return _frequency_force_dispersive(*args, **kw)


def _frequency_force_dispersive(wl, pol, nodes=100):
    """The imaginary-frequency force with the continued permittivity:
    E-kind [(k + s) I + eps_c(k)^-1 D_h mu^-1 D_e / (k dx^2)] E^ = E0 and the
    dual H-kind system, weighted by the general kernel's w(kappa)."""
    from oracle.force import setup
    from oracle.surface import gather
    faces, bases, eps_s, mu_s, chans = setup(wl)
    chans = [c for c in chans if c.pol == pol]
    De, Dh, AE, AH, e_axes, h_axes, n = curl_operators(wl, pol)
    mask = (AE != 0).astype(float)
    dx = 1.0 / wl.res
    dA = dx ** (wl.ndim - 1)
    sig = wl.sigma

    def functional(comp, face, row, comps):
        idx, w = gather(wl, faces[face], comp)
        v = np.zeros(len(comps) * n)
        np.add.at(v, comps.index(comp[1]) * n + idx.ravel(), (w * bases[face][0][row][:, None]).ravel())
        return v

    systems = []
    for kind in ("E", "H"):
        cs = [c for c in chans if c.kind == kind]
        comps = e_axes if kind == "E" else h_axes
        medium = eps_s if kind == "E" else mu_s
        X0 = np.array([-functional(c.src, c.face, c.row, comps) / (dx * medium) for c in cs]).T
        G = np.array([dA * functional(c.meas, c.face, c.row, comps) for c in cs])
        s = np.array([c.sign for c in cs])
        systems.append((kind, X0, G, s))
    v, wv = np.polynomial.legendre.leggauss(nodes)
    v, wv = 0.5 * (v + 1.0), 0.5 * wv
    u = v / (1.0 - v)
    kap, dk = u * u, 2.0 * u * wv / (1.0 - v) ** 2
    w = (kap + sig / 2) * np.sqrt(1.0 + sig / kap)
    total = 0.0
    for kq, dq, wq in zip(kap, dk, w):
        ae = mask / eps_c(wl, e_axes, mask, kq)
        g = 0.0
        for kind, X0, G, s in systems:
            if kind == "E":
                K = (ae[:, None] * Dh) @ (AH[:, None] * De) / dx ** 2
            else:
                K = (AH[:, None] * De) @ (ae[:, None] * Dh) / dx ** 2
            X = np.linalg.solve((kq + sig) * np.eye(K.shape[0]) + K / kq, X0)
            g += np.sum(s * np.einsum("ij,ji->i", G, X))
        total += dq * wq * g
    return total / np.pi


def dispersive_piston(pol):
    """The small piston with the left block a dispersive dielectric (eps_inf 2,
    one Lorentz term) and S around the right (PEC) block."""
    base = piston2d(24, 18, 3, 6, 4, 6, 7, 6.0, pol=pol, n_harm=4, n_steps=10, kernel="general")
    ids = {k: v.copy() for k, v in base.comp_ids.items()}
    for v in ids.values():
        v[:, :, : 24 // 2] = np.where(v[:, :, : 24 // 2] == 1, 3, v[:, :, : 24 // 2])
    return base.replace(eps=[1.0, float("-inf"), 1.0, 2.0], mu=[1.0, 1.0, 1.0, 1.0], comp_ids=ids,
                        lorentz={3: ((3.0, 2.0),)})


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_time_domain_converges_to_frequency_domain_dispersive(pol):
    base = dispersive_piston(pol)
    f_freq = frequency_force_dispersive(base, pol)
    errs = []
    for courant in (0.5, 0.25, 0.125):
        wl = base.replace(courant=courant, n_steps=int(round(40.0 * base.res / courant)))
        errs.append(abs(oracle.solve(wl).force / f_freq - 1.0))
    print(f"dispersive piston {pol}: F = {f_freq:.10f}; errors {errs}")
    assert errs[2] < 5e-4
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3


def test_lossless_dispersive_scheme_stays_bounded():
    """sigma = 0: fields and polarizations exchange energy without loss (the
    continued Lorentz term is then undamped).  From random grid-scale data
    (every frequency of the grid excited) the field amplitude neither grows
    nor dies over 20000 steps: the peak of E^2 + H^2 over the last 2000 steps
    stays within the range of the first 2000 (a growing mode of an unstable
    discretization would multiply it)."""
    wl = dispersive_piston("TM").replace(sigma=0.0)
    sim = YeeSim(wl, "E", 1, ("z",), ("x", "y"))
    rng = np.random.default_rng(3)
    sim.E["z"][...] = rng.standard_normal(sim.E["z"].shape) * (sim.cb["z"] != 0)

    def field_sq():
        return float(np.sum(sim.E["z"] ** 2) + np.sum(sim.H["x"] ** 2) + np.sum(sim.H["y"] ** 2))

    trace = []
    for _ in range(20000):
        sim.step()
        trace.append(field_sq())
    early, late = max(trace[:2000]), max(trace[-2000:])
    assert 0.3 * early < late < 1.5 * early, (early, late)
    assert any(np.any(p[0] != 0) for p in sim.P["z"])


def test_unstable_term_and_dispersive_surface_refused():
    wl = dispersive_piston("TM")
    with pytest.raises(ValueError):
        YeeSim(wl.replace(lorentz={3: ((1.0, 2.0 / (wl.courant / wl.res)),)}), "E", 1, ("z",), ("x", "y"))
    # the medium around S made dispersive
    with pytest.raises(ValueError):
        oracle.solve(wl.replace(lorentz={0: ((1.0, 2.0),)}))


def _uniform_lorentz_box(courant, eps_inf, terms, n=16, res=20.0, pol="TM"):
    from casimir_inputs.geometry import Workload, rasterize
    ids = rasterize((n, n, 1), [])
    return Workload(name="medium", ndim=2, shape=(n, n, 1), res=res, bc=("periodic", "periodic", "periodic"),
                    pml_cells=(0, 0, 0), eps=[eps_inf], mu=[1.0], comp_ids=ids, s_lo=(4, 4, 0), s_hi=(8, 8, 1),
                    n_harm=1, force_axis=0, sigma=0.0, courant=courant, pol=pol, kernel="general",
                    lorentz={0: tuple(terms)})


@pytest.mark.parametrize("k", [None, 15.0], ids=["2d", "kz"])
def test_coupled_lorentz_stability_limit(monkeypatch, k):
    """A strong term (silicon's d_eps = 10.835 on eps_inf = 1.035, w0 dx =
    1.1) is unstable well inside the plain Yee limit at eps_inf and far
    below w0 dt = 2: the field-polarization coupling raises the fastest
    grid mode's frequency.  The criterion oracle.yee.lorentz_stable (with
    the curl-curl bound 8 + (k dx)^2 of the grid) separates growth from
    boundedness of random fields in a uniform periodic medium to 2 %, and
    the oracle refuses a step above it."""
    import oracle.yee as Y
    from oracle import kz
    eps_inf, terms, res = 1.035, ((10.835, 22.0),), 20.0
    bound = 8.0 + ((k or 0.0) / res) ** 2
    lo, hi = 0.01, 0.7
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if Y.lorentz_stable(eps_inf, 1.0, terms, mid, 1.0 / res, bound) else (lo, mid)
    c_star = lo
    yee_limit = np.sqrt(eps_inf / 2.0)                    # courant * sqrt(2) / sqrt(eps_inf) < 1
    assert c_star < 0.65 * yee_limit                       # well inside the Yee limit at eps_inf
    assert c_star * 22.0 / res < 0.5                                      # and far below w0 dt = 2

    def make(c):
        wl = _uniform_lorentz_box(c, eps_inf, terms, res=res, pol="TM" if k is None else "3D")
        if k is None:
            return YeeSim(wl, "E", 1, ("z",), ("x", "y"))
        return kz.KzSim(wl, "E", 1, k)

    with pytest.raises(ValueError):
        make(1.02 * c_star)
    make(0.98 * c_star)                                    # accepted
    monkeypatch.setattr(Y, "lorentz_stable", lambda *a: True)

    def peak(c):
        S = make(c)
        rng = np.random.default_rng(3)
        for f in (S.E, S.H):
            for a in f:
                f[a] = rng.standard_normal(f[a].shape)
        with np.errstate(all="ignore"):
            for _ in range(3000):
                S.step()
        v = max(np.abs(S.E[a]).max() for a in S.E)
        return v if np.isfinite(v) else np.inf

    assert peak(0.98 * c_star) < 20.0
    assert peak(1.02 * c_star) > 1e6

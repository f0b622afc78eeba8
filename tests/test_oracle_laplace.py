"""The oracle's time-domain force against an independent imaginary-frequency
evaluation on the same grid (Sec. II: the conductivity sigma maps the
simulation onto the complex-frequency contour; Appendix A: the weight g and
its Laplace form).

The time-domain force is F = (1/pi) sum_c s_c sum_m dt K(t_m) Gamma_c(t_m)
with K(t) = 2 pi Im g(-t) = int_0^inf w(kappa) e^{-kappa t} dkappa, where w is
the rotated weight of Appendix A:
* general kernel: w(kappa) = (kappa + sigma/2) sqrt(1 + sigma/kappa);
* z-invariant kernel (Appendix A.2): w(kappa) = (kappa + sigma/2)(kappa + sigma)/2.
As dt -> 0 the force therefore tends to

    F = (1/pi) int_0^inf dkappa w(kappa) sum_c s_c Gamma^_c(kappa),

with Gamma^_c the Laplace transform of the continuous-time response of the
spatially discrete system. That transform comes from one linear solve per
kappa. For an E-kind channel (conductivity on E, kick E(0) = E0):

    [(kappa + sigma) I + A_E D_h A_H D_e / (kappa dx^2)] E^ = E0,

where D_e and D_h are the undivided curls, and A_E = mask/eps and
A_H = mask/mu are zero on PEC and PMC components. The H-kind system is the
dual one. Gamma^_c is the channel's surface functional applied to E^ or H^.

Nothing of the leapfrog enters this evaluation: not the time-centred
conductivity, not the consistent half-step start, not the sampling times t_m,
and not the Bessel closed form of K(t). A mistake in any of them breaks the
second-order agreement checked here. The evaluation shares with the oracle
only the spatial curl operators, probed column by column from its
simulation class, the surface gathers and basis, and the channel table.
Those are pinned by energy conservation, the Yee dispersion relation, the
point-source equivalence and the plate closed forms.
"""
import numpy as np
import pytest

import oracle
from casimir_inputs.configs import parallel_plates_1d, piston2d
from oracle.force import setup
from oracle.surface import POL_COMPONENTS, gather
from oracle.yee import YeeSim


def curl_operators(wl, pol):
    """Dense undivided curl matrices D_e (E -> H positions), D_h (H -> E) and
    the diagonal A_E = mask / eps, A_H = mask / mu, probed from the oracle's
    simulation class with one unit field per column."""
    e_axes, h_axes = POL_COMPONENTS[pol]
    n = wl.shape[0] * wl.shape[1] * wl.shape[2]
    ne, nh = len(e_axes) * n, len(h_axes) * n
    sim_h = YeeSim(wl, "H", ne, e_axes, h_axes)      # no conductivity on E
    sim_e = YeeSim(wl, "E", nh, e_axes, h_axes)      # no conductivity on H
    for k, a in enumerate(e_axes):
        sim_h.E[a].reshape(ne, n)[k * n + np.arange(n), np.arange(n)] = 1.0
    for k, a in enumerate(h_axes):
        sim_e.H[a].reshape(nh, n)[k * n + np.arange(n), np.arange(n)] = 1.0
    De = np.concatenate([sim_h.curl_e(a).reshape(ne, n).T for a in h_axes])
    Dh = np.concatenate([sim_e.curl_h(a).reshape(nh, n).T for a in e_axes])
    AE = np.concatenate([sim_h.cb[a].ravel() for a in e_axes]) / wl.courant
    AH = np.concatenate([sim_e.db[a].ravel() for a in h_axes]) / wl.courant
    return De, Dh, AE, AH, e_axes, h_axes, n


def frequency_force(*args, **kw):
    """frequency force on one BLAS thread (the test runner's
    workers would otherwise oversubscribe the host's cores)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        return _frequency_force(*args, **kw)


def _frequency_force(wl, pol, nodes=100):
    """(1/pi) int_0^inf w(kappa) sum_c s_c Gamma^_c(kappa) dkappa for the
    channels of one polarization (kappa = u^2, u = v / (1 - v), v in (0, 1)
    on Gauss-Legendre nodes)."""
    faces, bases, eps_s, mu_s, chans = setup(wl)
    chans = [c for c in chans if c.pol == pol]
    De, Dh, AE, AH, e_axes, h_axes, n = curl_operators(wl, pol)
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
        if not cs:
            continue
        comps = e_axes if kind == "E" else h_axes
        medium = eps_s if kind == "E" else mu_s
        X0 = np.array([-functional(c.src, c.face, c.row, comps) / (dx * medium) for c in cs]).T
        G = np.array([dA * functional(c.meas, c.face, c.row, comps) for c in cs])
        s = np.array([c.sign for c in cs])
        if kind == "E":
            K = (AE[:, None] * Dh) @ (AH[:, None] * De) / dx ** 2
        else:
            K = (AH[:, None] * De) @ (AE[:, None] * Dh) / dx ** 2
        systems.append((X0, G, s, K))
    v, wv = np.polynomial.legendre.leggauss(nodes)
    v, wv = 0.5 * (v + 1.0), 0.5 * wv
    u = v / (1.0 - v)
    kap, dk = u * u, 2.0 * u * wv / (1.0 - v) ** 2
    if wl.kernel == "general":
        w = (kap + sig / 2) * np.sqrt(1.0 + sig / kap)
    else:
        w = (kap + sig / 2) * (kap + sig) / 2
    total = 0.0
    for kq, dq, wq in zip(kap, dk, w):
        g = 0.0
        for X0, G, s, K in systems:
            X = np.linalg.solve((kq + sig) * np.eye(K.shape[0]) + K / kq, X0)
            g += np.sum(s * np.einsum("ij,ji->i", G, X))
        total += dq * wq * g
    return total / np.pi


CASES = {
    # 1D-reducible plates, TM, z-invariant kernel
    "plates_tm_zinv": (lambda: parallel_plates_1d(10, 0.5, 0.3, 1.0, pol="TM", kernel="zinv2d", n_steps=10),
                       ("TM",), 60.0),
    # small 2D piston, both polarizations (E- and H-kind channels), general kernel
    "piston_general": (lambda: piston2d(24, 18, 3, 6, 4, 6, 7, 6.0, pol="TM+TE", n_steps=10, n_harm=4,
                                        kernel="general"), ("TM", "TE"), 40.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_time_domain_converges_to_frequency_domain(name):
    make, pols, t_max = CASES[name]
    base = make()
    for pol in pols:
        f_freq = frequency_force(base, pol)
        errs = []
        for courant in (0.5, 0.25, 0.125):
            wl = base.replace(pol=pol, courant=courant, n_steps=int(round(t_max * base.res / courant)))
            errs.append(oracle.solve(wl).force / f_freq - 1.0)
        errs = np.abs(errs)
        print(f"{name} {pol}: F = {f_freq:.10f}; relative errors at Courant 0.5/0.25/0.125: {errs}")
        assert errs[2] < 5e-4
        assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3      # second order in dt


def test_frequency_quadrature_converged():
    """The kappa quadrature is exact to far below the time-step errors."""
    wl = CASES["plates_tm_zinv"][0]()
    a, b = frequency_force(wl, "TM", nodes=60), frequency_force(wl, "TM", nodes=120)
    assert abs(a / b - 1) < 1e-8

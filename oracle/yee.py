"""Yee leapfrog with the paper's uniform conductivity (Sec. II; Taflove's Yee
scheme, which the paper's FDTD package implements).

Units: hbar = c = eps_0 = mu_0 = 1; grid spacing dx = 1/res; time step
dt = courant * dx.  Fields of a batch of independent channels are stored as
arrays of shape (C, nz, ny, nx); a 2D problem has nz = 1 and is periodic in
z, so every z difference vanishes.

Placement (standard Yee): E_a sits half a cell along a, H_a half a cell
along both other axes.  The curl of E at H_a uses forward differences, the
curl of H at E_a backward differences; with PEC (or PML-backed) walls a
neighbour beyond the grid reads as zero, with periodic walls it wraps.  E
components lying on a PEC wall (integer coordinate 0 along that wall's axis)
are held at zero.

Conductivity (Sec. II: a frequency-independent, spatially uniform sigma that
turns the real-frequency response into the response on the complex contour
omega^2 = xi^2 + i sigma xi; the paper does not spell out its
discretization, so the time-centred semi-implicit form is used):

  E-kind run:  eps (E^{m+1} - E^m)/dt = curl H^{m+1/2} - sigma eps (E^{m+1} + E^m)/2
               mu  (H^{m+1/2} - H^{m-1/2})/dt = -curl E^m
  H-kind run:  the loss moves to H with sigma mu, E is lossless.

A magnetic-current source must see magnetic conductivity: only then is its H
response the magnetic Green's function on the same contour that g(xi)
assumes (the paper states only that Gamma^H is defined like Gamma^E).

Start of a run (the paper does not discretize its delta(t) source): the kick
sets the kicked field at t = 0 and :meth:`YeeSim.start` sets the staggered
partner field to the value the smooth t > 0 solution extends to half a step
away, so the leapfrog stays second order in dt:

  E-kind:  E^0 = kick,  H^{-1/2} = +(dt / 2 mu) curl E^0
  H-kind:  H^0 = kick,  E^{+1/2} = +(dt / 2 eps) curl H^0
           (the H-kind run is the exact dual: its H sample after step m is
           H^m, again at t_m = m dt)

With the partner field left at zero instead (``start="zero"``) the force
converges only at first order in dt; the tests show both orders.

PEC material (epsilon = -inf) zeroes E; PMC (mu = -inf) zeroes H.

Dispersive materials (Sec. III B: a fitted Lorentz model, continued onto the
complex conductivity contour).  A term d_eps w0^2 / (w0^2 - omega^2) of
eps(omega), on the contour omega^2 = xi^2 + i sigma xi, becomes
d_eps w0^2 / (w0^2 - xi^2 - i sigma xi): in the simulation's time (the
variable conjugate to xi) a polarization P with

    P'' + sigma P' + w0^2 P = d_eps w0^2 E,        D = eps_inf E + sum P,

and the conductivity of an E-kind run acts on D (the factor 1 + i sigma/xi
multiplies the whole continued permittivity); in an H-kind run D is
lossless.  Discretized with centred differences at the E time levels,

    P^{m+1} = [(2 - w0^2 dt^2) P^m - (1 - sigma dt/2) P^{m-1}
               + d_eps w0^2 dt^2 E^m] / (1 + sigma dt/2),
    eps_inf (E^{m+1} - E^m)/dt + (P^{m+1} - P^m)/dt
        = curl H^{m+1/2} - sigma (D^{m+1} + D^m)/2     (E-kind; no sigma for H-kind),

i.e. E^{m+1} = a E^m + b curl H - (sum P^{m+1} - a sum P^m) / eps_inf with
the non-dispersive a, b of eps_inf.  P starts at zero: the kicks sit on S,
which must lie in a non-dispersive medium.  Stable when w0 dt < 2 for every
term and the coupled field-polarization frequency of the fastest grid mode
stays below 2 / dt (lorentz_stable; a strong term such as silicon's raises
that frequency well above the plain Yee limit at eps_inf).

CPML (Roden-Gedney, kappa = 1, alpha = 0) along any axis whose boundary is
"pml": every difference along that axis inside the layer becomes D + psi with
psi <- b psi + (b - 1) D, b = exp(-sigma_p(x) dt), sigma_p(x) = sigma_max
(depth/P)^3, sigma_max = -4 ln(1e-8) / (2 P dx), depth measured in cells from
the layer's inner face at the position of the component being updated.  The
paper uses PML without giving its profile; this one is a stated choice.

Parity: pinned (tests/test_oracle_yee.py: exact discrete energy conservation
at sigma = 0, exact dissipation rate for sigma > 0, the Yee dispersion
relation, PML absorption).
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np

from casimir_inputs.geometry import COMPONENT_OFFSETS2

ARRAY_AXIS = {0: 3, 1: 2, 2: 1}  # spatial axis -> axis of a (C, nz, ny, nx) array
CYCLIC = {"x": ("y", "z"), "y": ("z", "x"), "z": ("x", "y")}
AXIS_OF = {"x": 0, "y": 1, "z": 2}

PML_ORDER = 3
PML_R0 = 1e-8


def d_plus(F: np.ndarray, axis: int, bc: str) -> np.ndarray:
    """F[i+1] - F[i] along a spatial axis."""
    ax = ARRAY_AXIS[axis]
    if bc == "periodic":
        return np.roll(F, -1, axis=ax) - F
    out = -F
    dst = [slice(None)] * 4
    src = [slice(None)] * 4
    dst[ax] = slice(0, -1)
    src[ax] = slice(1, None)
    out[tuple(dst)] += F[tuple(src)]
    return out


def d_minus(F: np.ndarray, axis: int, bc: str) -> np.ndarray:
    """F[i] - F[i-1] along a spatial axis."""
    ax = ARRAY_AXIS[axis]
    if bc == "periodic":
        return F - np.roll(F, 1, axis=ax)
    out = F.copy()
    dst = [slice(None)] * 4
    src = [slice(None)] * 4
    dst[ax] = slice(1, None)
    src[ax] = slice(0, -1)
    out[tuple(dst)] -= F[tuple(src)]
    return out


def pml_profile(n: int, P: int, dx: float, dt: float, half: bool):
    """(b, c) along one axis for components at positions i (+1/2 if half)."""
    x = np.arange(n, dtype=np.float64) + (0.5 if half else 0.0)
    depth = np.maximum(np.maximum(P - x, x - (n - P)), 0.0)
    smax = -(PML_ORDER + 1) * np.log(PML_R0) / (2.0 * P * dx)
    sig = smax * (depth / P) ** PML_ORDER
    b = np.exp(-sig * dt)
    return b, b - 1.0


def lorentz_stable(eps_inf: float, mu: float, terms, courant: float, dx: float, curl_bound: float) -> bool:
    """Stability of the centred Lorentz scheme in a uniform medium.  A plane
    wave z^m with Omega^2 = (4 / dt^2) sin^2(omega dt / 2) and spatial
    curl-curl eigenvalue K^2 / mu satisfies
        Omega^2 (eps_inf + sum d_eps w0^2 / (w0^2 - Omega^2)) = K^2 / mu;
    it is stable when every root Omega^2 stays at or below X = 4 / dt^2.
    Above the largest w0^2 the left side minus the right increases with
    Omega^2, so the condition is w0 dt < 2 for every term and
        f(X) = eps_inf X - K_max^2 / mu + sum d_eps w0^2 X / (w0^2 - X) > 0,
    with K_max^2 = curl_bound / dx^2 (evaluated here in units of dx^2)."""
    X = 4.0 / (courant * courant)
    f = eps_inf * X - curl_bound / mu
    for de, w0 in terms:
        w2 = (w0 * dx) ** 2
        if w2 * courant * courant >= 4.0:
            return False
        f += de * w2 * X / (w2 - X)
    return f > 0.0


class YeeSim:
    """One batch of channels of the same kind ("E" or "H") and component set."""

    def __init__(self, wl, kind: str, n_channels: int, e_comps: Sequence[str],
                 h_comps: Sequence[str], sigma: float = None, courant: float = None):
        self.wl = wl
        self.kind = kind
        self.C = int(n_channels)
        self.e_comps = tuple(e_comps)
        self.h_comps = tuple(h_comps)
        self.sigma = wl.sigma if sigma is None else float(sigma)
        self.courant = wl.courant if courant is None else float(courant)
        self.dx = 1.0 / wl.res
        self.dt = self.courant * self.dx
        nx, ny, nz = wl.shape
        self.grid_shape = (nz, ny, nx)
        shp = (self.C, nz, ny, nx)
        self.E = {a: np.zeros(shp) for a in self.e_comps}
        self.H = {a: np.zeros(shp) for a in self.h_comps}
        self._coefficients()
        self._lorentz_setup()
        self._pml_setup()

    # -- coefficients ---------------------------------------------------
    def _coefficients(self):
        wl = self.wl
        r = 0.5 * self.sigma * self.dt
        lossy_a = (1.0 - r) / (1.0 + r)
        lossy_b = 1.0 / (1.0 + r)
        eps = np.asarray(wl.eps, dtype=np.float64)
        mu = np.asarray(wl.mu, dtype=np.float64)
        self.ca, self.cb, self.da, self.db = {}, {}, {}, {}
        for a in self.e_comps:
            name = "E" + a
            ids = wl.comp_ids[name]
            e = eps[ids]
            pec = np.isneginf(e)
            o2 = COMPONENT_OFFSETS2[name]
            for ax in range(wl.ndim):
                if wl.bc[ax] in ("pec", "pml") and o2[ax] == 0:
                    sl = [slice(None)] * 3
                    sl[2 - ax] = 0
                    pec = pec.copy()
                    pec[tuple(sl)] = True
            e_safe = np.where(pec, 1.0, e)
            if self.kind == "E":
                ca = np.full(e.shape, lossy_a)
                cb = self.courant / e_safe * lossy_b
            else:
                ca = np.ones(e.shape)
                cb = self.courant / e_safe
            self.ca[a] = np.where(pec, 0.0, ca)
            self.cb[a] = np.where(pec, 0.0, cb)
        for a in self.h_comps:
            name = "H" + a
            m = mu[wl.comp_ids[name]]
            pmc = np.isneginf(m)
            m_safe = np.where(pmc, 1.0, m)
            if self.kind == "H":
                da = np.full(m.shape, lossy_a)
                db = self.courant / m_safe * lossy_b
            else:
                da = np.ones(m.shape)
                db = self.courant / m_safe
            self.da[a] = np.where(pmc, 0.0, da)
            self.db[a] = np.where(pmc, 0.0, db)

    def _lorentz_setup(self):
        """Per E component: the Lorentz terms of every cell (d_eps, w0 as
        arrays, zero where a cell has fewer terms or is a conductor), eps_inf,
        and the polarizations P^m, P^{m-1} of each term."""
        wl = self.wl
        lor = {k: tuple(v) for k, v in (getattr(wl, "lorentz", None) or {}).items() if v}
        self.poles, self.P = {}, {}
        if not lor:
            return
        n_terms = max(len(v) for v in lor.values())
        eps = np.asarray(wl.eps, dtype=np.float64)
        for a in self.e_comps:
            ids = wl.comp_ids["E" + a]
            live = self.cb[a] != 0.0                        # not a conductor or a PEC wall
            terms = []
            for j in range(n_terms):
                de = np.zeros(ids.shape)
                w0 = np.zeros(ids.shape)
                for k, v in lor.items():
                    if j < len(v):
                        sel = (ids == k) & live
                        de[sel] = v[j][0]
                        w0[sel] = v[j][1]
                if np.any(w0 * self.dt >= 2.0):
                    raise ValueError("Lorentz term unstable: w0 dt must stay below 2")
                terms.append((de, w0))
            e_inf = np.where(live, eps[ids], 1.0)
            self.poles[a] = (terms, e_inf)
            self.P[a] = [[np.zeros(self.E[a].shape), np.zeros(self.E[a].shape)] for _ in terms]
        mu = np.asarray(wl.mu, dtype=np.float64)
        for k, v in lor.items():
            if not np.isfinite(eps[k]) or not np.isfinite(mu[k]):
                continue
            if not lorentz_stable(eps[k], mu[k], v, self.courant, self.dx, self.curl_bound()):
                raise ValueError("Lorentz medium unstable at this time step: the coupled field and "
                                 "polarization frequency exceeds 2 / dt (lower the Courant number)")

    def curl_bound(self) -> float:
        """Upper bound of the undivided curl-curl eigenvalue, (K dx)^2, of the
        grid: 4 per axis along which the fields vary."""
        return 4.0 * self.wl.ndim

    def _pml_setup(self):
        wl = self.wl
        self.psi: Dict[tuple, np.ndarray] = {}
        self.pml_bc: Dict[tuple, tuple] = {}
        for ax in range(wl.ndim):
            if wl.bc[ax] != "pml":
                continue
            P = int(wl.pml_cells[ax])
            n = wl.shape[ax]
            for field, comps in (("H", self.h_comps), ("E", self.e_comps)):
                for a in comps:
                    if AXIS_OF[a] == ax:
                        continue
                    half = COMPONENT_OFFSETS2[field + a][ax] == 1
                    b, c = pml_profile(n, P, self.dx, self.dt, half)
                    shape = [1, 1, 1, 1]
                    shape[ARRAY_AXIS[ax]] = n
                    self.pml_bc[(field + a, ax)] = (b.reshape(shape), c.reshape(shape))
                    self.psi[(field + a, ax)] = np.zeros((self.C,) + self.grid_shape)

    # -- stepping -------------------------------------------------------
    def _diff(self, target: str, F: np.ndarray, axis: int, forward: bool) -> np.ndarray:
        bc = self.wl.bc[axis] if axis < self.wl.ndim else "periodic"
        D = d_plus(F, axis, bc) if forward else d_minus(F, axis, bc)
        key = (target, axis)
        if key in self.pml_bc:
            b, c = self.pml_bc[key]
            self.psi[key] = b * self.psi[key] + c * D
            D = D + self.psi[key]
        return D

    def curl_e(self, a: str) -> np.ndarray:
        """(curl E)_a at H_a positions (undivided differences)."""
        b, c = CYCLIC[a]
        out = np.zeros((self.C,) + self.grid_shape)
        if c in self.E:
            out += self._diff("H" + a, self.E[c], AXIS_OF[b], True)
        if b in self.E:
            out -= self._diff("H" + a, self.E[b], AXIS_OF[c], True)
        return out

    def curl_h(self, a: str) -> np.ndarray:
        """(curl H)_a at E_a positions (undivided differences)."""
        b, c = CYCLIC[a]
        out = np.zeros((self.C,) + self.grid_shape)
        if c in self.H:
            out += self._diff("E" + a, self.H[c], AXIS_OF[b], False)
        if b in self.H:
            out -= self._diff("E" + a, self.H[b], AXIS_OF[c], False)
        return out

    def start(self, mode: str = "consistent"):
        """Set the staggered partner of the kicked field (see module doc)."""
        if mode == "zero":
            return
        if mode != "consistent":
            raise ValueError(mode)
        if self.kind == "E":
            curls = {a: self.curl_e(a) for a in self.h_comps}
            for a in self.h_comps:
                self.H[a] = 0.5 * self.db[a] * curls[a]
        else:
            curls = {a: self.curl_h(a) for a in self.e_comps}
            for a in self.e_comps:
                self.E[a] = 0.5 * self.cb[a] * curls[a]

    def step_h(self):
        curls = {a: self.curl_e(a) for a in self.h_comps}
        for a in self.h_comps:
            self.H[a] = self.da[a] * self.H[a] - self.db[a] * curls[a]

    def step_e(self):
        curls = {a: self.curl_h(a) for a in self.e_comps}
        for a in self.e_comps:
            new = self.ca[a] * self.E[a] + self.cb[a] * curls[a]
            if a in self.poles:
                terms, e_inf = self.poles[a]
                dt, r = self.dt, 0.5 * self.sigma * self.dt
                p_now = np.zeros_like(new)          # complex in Bloch runs
                p_next = np.zeros_like(new)
                for (de, w0), st in zip(terms, self.P[a]):
                    cur, prev = st
                    nxt = ((2.0 - (w0 * dt) ** 2) * cur - (1.0 - r) * prev
                           + de * (w0 * dt) ** 2 * self.E[a]) / (1.0 + r)
                    p_now += cur
                    p_next += nxt
                    st[0], st[1] = nxt, cur
                new = new - (p_next - self.ca[a] * p_now) / e_inf
            self.E[a] = new

    def step(self):
        self.step_h()
        self.step_e()

    def field(self, comp: str) -> np.ndarray:
        return (self.E if comp[0] == "E" else self.H)[comp[1]]

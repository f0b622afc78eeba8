"""Yee leapfrog in cylindrical coordinates for one azimuthal order m (Sec.
III C, three dimensions with cylindrical symmetry; Appendix, harmonic
expansion in cylindrical coordinates).  Test infrastructure: only tests/,
the package smoke check and the benchmark's CPU baseline use this module.

Reduction.  Fields proportional to exp(i m phi) reduce Maxwell's equations
to the (r, z) half plane.  Writing E_phi = i e_phi, H_r = i h_r, H_z = i h_z
and keeping E_r = e_r, E_z = e_z, H_phi = h_phi turns the complex problem
into a real one (sources and measured values of every stress-tensor channel
the axial force needs fall in the same class, so the real part of the
paper's Gamma_{n,m} is this real system's response):

  mu  dh_r/dt   = -[ (m/r) e_z - d_z e_phi ]
  mu  dh_phi/dt = -[ d_z e_r - d_r e_z ]
  mu  dh_z/dt   = -[ (1/r) d_r (r e_phi) - (m/r) e_r ]
  eps de_r/dt   =    -(m/r) h_z - d_z h_phi
  eps de_phi/dt =    d_z h_r - d_r h_z
  eps de_z/dt   =    (1/r) d_r (r h_phi) + (m/r) h_r

(conductivity as in the Cartesian scheme: sigma eps on the E-kind runs,
sigma mu on the H-kind runs, time-centred).

Grid.  Arrays are (C, nr, nz): row j is the radial index, column i the
axial one.  With the axial coordinate as the Cartesian x axis and r as y,
the cylindrical Yee cell is the Cartesian 2D one (doubled offsets
x, y): e_z (1,0), e_r (0,1), e_phi (0,0), h_z (0,1), h_r (1,0), h_phi (1,1),
the Cartesian names being Ex = e_z, Ey = e_r, Ez = e_phi, Hx = h_z,
Hy = h_r, Hz = h_phi.  The radius is r = (y - 1/2) cells: offset-0 rows sit
at r = j - 1/2 (row 0 lies outside the domain and stays zero), offset-1 rows
at r = j (row 0 on the axis).  The tube wall is at r = nr - 1/2 cells, where
the tangential e_z, e_phi of the next row read as zero (PEC).

Axis.  Only h_z has a dynamic value on the axis: for m = 0 its curl term is
the circulation of e_phi around the disk of radius 1/2 cell over the disk
area, 4 e_phi(r = 1/2) / dx; for m != 0 it stays zero.  e_r and h_phi on the
axis enter no update (their row is multiplied by r = 0).  They are kept for
surface samples next to the axis: for |m| = 1 the transverse field is even
across the axis, so the axis value is the next row's (second order), and
zero otherwise; a source deposited on that row is folded into the next row
(the adjoint of the copy).  With the r-weights of the cells (r, and 1/8 cell
for the axis disk) the update is skew-symmetric, which the exact energy pin
checks.

Stability.  The m/r couplings of co-located pairs raise the largest
frequency of the scheme near the axis; the stable Courant number falls with
m (cylindrical_courant gives the value used).

Open tube ends (bc "pml" along the axis; Sec. III C's piston ends in PML):
the CPML of the Cartesian scheme (oracle.yee, same profile) stretches the
four axial differences, d_z e_phi (h_r), d_z e_r (h_phi), d_z h_phi (e_r)
and d_z h_r (e_phi), inside the layers, at the updated component's axial
position; the layers are backed by a PEC end (e_r and e_phi held at 0 on
the first plane).  The radial differences and the m/r couplings are not
stretched.  Pinned by a pulse in a short tube with layers against the same
pulse in a tube three times as long with PEC ends (tests/test_oracle_cyl.py).
"""
from __future__ import annotations

import numpy as np

from .yee import pml_profile

COMP = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")   # e_z, e_r, e_phi, h_z, h_r, h_phi


def cylindrical_courant(courant: float, m: int) -> float:
    """Courant number used for order m: the requested one, lowered for
    m >= 2 to 1/(1 + m) (a Gershgorin bound of the update operator: every
    row of the curl operators has absolute coefficient sum <= max(4, 2 + 2m)
    cells^-1)."""
    return min(courant, 1.0 / (1.0 + m)) if m >= 2 else courant


class CylSim:
    """Leapfrog of C independent channels of one problem for one order m.

    wl: cylindrical workload (shape (nz, nr, 1); eps/mu tables; comp_ids
    per Cartesian component name).  kind: "E" or "H" (which field carries
    the conductivity).  bc_z: "pec" or "periodic" along the axial
    direction."""

    def __init__(self, wl, kind: str, n_channels: int, m: int, courant: float):
        self.wl = wl
        self.m = int(m)
        self.nz, self.nr = wl.shape[0], wl.shape[1]
        self.dx = 1.0 / wl.res
        self.dt = courant * self.dx
        self.kind = kind
        self.C = n_channels
        self.bc_z = wl.bc[0]
        shape = (n_channels, self.nr, self.nz)
        self.F = {c: np.zeros(shape) for c in COMP}
        # radii in cells: offset-0 rows (Ex, Ez, Hy) and offset-1 rows (Ey, Hx, Hz)
        self.r0 = np.arange(self.nr) - 0.5
        self.r1 = np.arange(self.nr) * 1.0
        self._coefficients()
        # CPML along the axis: (b, c) per axial position of each stretched
        # target (h_r, h_phi at half cells; e_r, e_phi at whole cells) and psi
        self.pml, self.psi = {}, {}
        if self.bc_z == "pml":
            P = int(wl.pml_cells[0])
            for c, half in (("Hy", True), ("Hz", True), ("Ey", False), ("Ez", False)):
                b, cc = pml_profile(self.nz, P, self.dx, self.dt, half)
                self.pml[c] = (b[None, None, :], cc[None, None, :])
                self.psi[c] = np.zeros(shape)

    # -- coefficients -----------------------------------------------------
    def _coefficients(self):
        wl = self.wl
        eps = np.asarray(wl.eps, float)
        mu = np.asarray(wl.mu, float)
        sig = wl.sigma
        dt, dx = self.dt, self.dx
        self.a, self.b = {}, {}
        for c in COMP:
            ids = np.asarray(wl.comp_ids[c]).reshape(self.nr, self.nz)   # (y = r rows, x = z columns)
            if c[0] == "E":
                mat = eps[ids]
                lossy = self.kind == "E"
            else:
                mat = mu[ids]
                lossy = self.kind == "H"
            wall = ~np.isfinite(mat)
            m_ = np.where(wall, 1.0, mat)
            r = sig * dt / 2.0 if lossy else 0.0
            a = np.full(m_.shape, (1 - r) / (1 + r))
            b = (dt / (m_ * dx)) / (1 + r)
            a[wall] = 0.0
            b[wall] = 0.0
            # row 0 of offset-0 components lies at r = -1/2: outside the domain
            if c in ("Ex", "Ez", "Hy"):
                a[0, :] = 0.0
                b[0, :] = 0.0
            # PEC end wall at z = 0 (also behind a CPML): e_r and e_phi
            # (axial offset 0) lie on it
            if self.bc_z in ("pec", "pml") and c in ("Ey", "Ez"):
                a[:, 0] = 0.0
                b[:, 0] = 0.0
            self.a[c] = a
            self.b[c] = b

    # -- differences along the axial (x) direction --------------------------
    def _dz_fwd(self, F):
        """F[i+1] - F[i] along z (0 beyond a PEC end, wrapped if periodic)."""
        if self.bc_z == "periodic":
            return np.roll(F, -1, axis=2) - F
        out = -F.copy()
        out[:, :, :-1] += F[:, :, 1:]
        return out

    def _dz_bwd(self, F):
        """F[i] - F[i-1] along z."""
        if self.bc_z == "periodic":
            return F - np.roll(F, 1, axis=2)
        out = F.copy()
        out[:, :, 1:] -= F[:, :, :-1]
        return out

    def _stretch(self, target, D):
        """An axial difference D of the update of `target`, stretched inside
        the CPML: psi <- b psi + c D, D + psi (unchanged without layers)."""
        if target not in self.pml:
            return D
        b, c = self.pml[target]
        self.psi[target] = b * self.psi[target] + c * D
        return D + self.psi[target]

    @staticmethod
    def _shift_up(F):
        """F[j+1] (row below the tube wall reads 0 beyond it)."""
        out = np.zeros_like(F)
        out[:, :-1, :] = F[:, 1:, :]
        return out

    @staticmethod
    def _shift_down(F):
        """F[j-1] (row -1 reads 0)."""
        out = np.zeros_like(F)
        out[:, 1:, :] = F[:, :-1, :]
        return out

    # -- curls (undivided: multiplied by dx) ---------------------------------
    def curl_e(self):
        """Right-hand sides of mu dh/dt = -curl e for h_z, h_r, h_phi (times dx)."""
        m = self.m
        ex, ey, ez = self.F["Ex"], self.F["Ey"], self.F["Ez"]
        r0, r1 = self.r0[None, :, None], self.r1[None, :, None]
        # h_z at offset-1 rows (r = j): (1/r) d_r(r e_phi) - (m/r) e_r
        rez = r0 * ez                                  # r e_phi at r = j - 1/2
        with np.errstate(divide="ignore", invalid="ignore"):
            cz = (self._shift_up(rez) - rez) / r1 - m * ey / r1
        cz[:, 0, :] = 4.0 * ez[:, 1, :] if m == 0 else 0.0
        # h_r at offset-0 rows (r = j - 1/2): (m/r) e_z - d_z e_phi
        with np.errstate(divide="ignore", invalid="ignore"):
            cr = m * ex / r0 - self._stretch("Hy", self._dz_fwd(ez))
        cr[:, 0, :] = 0.0
        # h_phi at (1,1): d_z e_r - d_r e_z
        cp = self._stretch("Hz", self._dz_fwd(ey)) - (self._shift_up(ex) - ex)
        return {"Hx": cz, "Hy": cr, "Hz": cp}

    def curl_h(self):
        """Right-hand sides of eps de/dt = curl h for e_z, e_r, e_phi (times dx)."""
        m = self.m
        hx, hy, hz = self.F["Hx"], self.F["Hy"], self.F["Hz"]
        r0, r1 = self.r0[None, :, None], self.r1[None, :, None]
        # e_z at offset-0 rows: (1/r) d_r(r h_phi) + (m/r) h_r
        rhz = r1 * hz                                  # r h_phi at r = j
        with np.errstate(divide="ignore", invalid="ignore"):
            cz = (rhz - self._shift_down(rhz)) / r0 + m * hy / r0
        cz[:, 0, :] = 0.0
        # e_r at offset-1 rows: -(m/r) h_z - d_z h_phi
        with np.errstate(divide="ignore", invalid="ignore"):
            cr = -m * hx / r1 - self._stretch("Ey", self._dz_bwd(hz))
        cr[:, 0, :] = 0.0
        # e_phi at (0,0): d_z h_r - d_r h_z
        cp = self._stretch("Ez", self._dz_bwd(hy)) - (hx - self._shift_down(hx))
        cp[:, 0, :] = 0.0
        return {"Ex": cz, "Ey": cr, "Ez": cp}

    # -- axis values of the transverse field -------------------------------
    # e_r and h_phi on the axis (row 0 of the offset-1 components) enter no
    # update.  They are kept for the surface interpolation next to the axis:
    # for |m| = 1 the transverse field is even across the axis, so its axis
    # value is the next row's to second order; otherwise it is zero.
    def axis_copy(self, comps=("Ey", "Hz")):
        for c in comps:
            self.F[c][:, 0, :] = self.F[c][:, 1, :] if self.m == 1 else 0.0

    def fold_axis(self, comps=("Ey", "Hz")):
        """Adjoint of axis_copy, applied to a source deposited on the axis
        row: for |m| = 1 the deposit moves to the next row, else it is
        dropped; then the copy is refreshed."""
        for c in comps:
            if self.m == 1:
                self.F[c][:, 1, :] += self.F[c][:, 0, :]
            self.F[c][:, 0, :] = 0.0
        self.axis_copy(comps)

    # -- time stepping -------------------------------------------------------
    def step_h(self):
        ce = self.curl_e()
        ce["Hz"][:, 0, :] = 0.0
        for c in ("Hx", "Hy", "Hz"):
            self.F[c] = self.a[c] * self.F[c] - self.b[c] * ce[c]
        if self.m != 0:
            self.F["Hx"][:, 0, :] = 0.0
        self.axis_copy(("Hz",))

    def step_e(self):
        ch = self.curl_h()
        ch["Ey"][:, 0, :] = 0.0
        for c in ("Ex", "Ey", "Ez"):
            self.F[c] = self.a[c] * self.F[c] + self.b[c] * ch[c]
        self.axis_copy(("Ey",))

    def step(self):
        self.step_h()
        self.step_e()

    def start(self, mode: str = "consistent"):
        """Partner field half a step away from the kicked one (as the
        Cartesian scheme): E-kind h^{-1/2} = +(dt/2 mu) curl e^0, H-kind
        e^{+1/2} = +(dt/2 eps) curl h^0."""
        if mode == "zero":
            return
        if self.kind == "E":
            ce = self.curl_e()
            for c in ("Hx", "Hy", "Hz"):
                self.F[c] = 0.5 * self.b[c] * ce[c]
            if self.m != 0:
                self.F["Hx"][:, 0, :] = 0.0
            self.axis_copy(("Hz",))
        else:
            ch = self.curl_h()
            for c in ("Ex", "Ey", "Ez"):
                self.F[c] = 0.5 * self.b[c] * ch[c]
            self.axis_copy(("Ey",))

    # -- diagnostics -----------------------------------------------------------
    def weights(self):
        """Cell r-weights (in cells) of every component: r at the component's
        radius, 1/8 for h_z on the axis (the disk of radius 1/2 cell), 0 for
        the rows outside the domain and the axis values that enter no
        update."""
        w = {}
        for c in COMP:
            rr = self.r0 if c in ("Ex", "Ez", "Hy") else self.r1
            wc = np.clip(rr, 0.0, None).copy()
            if c == "Hx":
                wc[0] = 0.125
            w[c] = wc[:, None]
        return w

    def material(self, c):
        eps = np.asarray(self.wl.eps, float)
        mu = np.asarray(self.wl.mu, float)
        ids = np.asarray(self.wl.comp_ids[c]).reshape(self.nr, self.nz)
        v = (eps if c[0] == "E" else mu)[ids]
        return np.where(np.isfinite(v), v, 0.0)

"""z-invariant two-dimensional problems at a Bloch wavevector k along the
invariant axis (Sec. III B: dielectrics hybridize the two polarizations, so
every k_z is its own two-dimensional simulation; Sec. III D: the force as an
integral over the Bloch wavevectors).  Test infrastructure: only tests/, the
package smoke check and the benchmark's CPU baseline use this module.

Reduction.  Fields proportional to exp(i k z) turn d/dz into i k.  Writing
E_z = i e_z, H_x = i h_x, H_y = i h_y and keeping E_x = e_x, E_y = e_y,
H_z = h_z gives a real system in all six components:

  mu  dh_x/dt = -( d_y e_z - k e_y )
  mu  dh_y/dt = -( k e_x - d_x e_z )
  mu  dh_z/dt = -( d_x e_y - d_y e_x )
  eps de_x/dt =    d_y h_z + k h_y
  eps de_y/dt =   -k h_x - d_x h_z
  eps de_z/dt =    d_x h_y - d_y h_x

(conductivity as in the Cartesian scheme).  The (x, y) grid and its Yee
cell are the two-dimensional ones; the k terms couple co-located pairs
(e_x with h_y, e_y with h_x), and they enter the H and the E update as
transposes of each other, so the leapfrog stays skew-symmetric (energy is
conserved at sigma = 0).  At k = 0 the system splits into TM (e_z, h_x, h_y)
and TE (e_x, e_y, h_z).  Every stress-tensor channel measures a component of
its source's class, so the real response is the real part the force needs.

Force.  For each k the two-dimensional force F(k) = (1/pi) sum_c s_c sum_m
dt K(t_m) Gamma_c(t_m) with the general (three-dimensional) kernel K; the
force per unit length is (1/pi) int_0^inf F(k) dk (F(-k) = F(k)), taken here
as sum_q w_q F(k_q) for a quadrature (k_q, w_q) chosen by the caller (w_q
includes the 1/pi).

Stability: the k terms raise the scheme's largest frequency; the Courant
number must stay below 2 / sqrt(8 + (k dx)^2) / v_max (kz_courant_limit).

Open space and dispersion (Sec. III B's waveguides): KzSim inherits the
CPML of YeeSim on any in-plane axis whose boundary is "pml" (the k terms
are not differences and take no stretching) and the Lorentz polarizations
of dispersive materials on all three E components (the ADE is local and
linear, so the factor i carried by e_z carries over to its polarization).

Parity: pinned (tests/test_oracle_kz.py; tests/test_oracle_kz_open.py:
dispersive slabs in open space against the Lifshitz force at each k, and
the in-plane CPML against a large PEC box).
"""
from __future__ import annotations

import dataclasses
from collections import defaultdict
from typing import Dict, List, Sequence

import numpy as np

from .force import setup
from .kernels import kernel_table
from .surface import gather
from .yee import YeeSim


def kz_courant_limit(k: float, res: float, vmax: float = 1.0) -> float:
    """Largest stable Courant number at wavevector k (undivided eigenvalue
    bound 8 + (k dx)^2 of the two-dimensional curl-curl with the k terms)."""
    kd = k / res
    return 2.0 / np.sqrt(8.0 + kd * kd) / vmax


class KzSim(YeeSim):
    """YeeSim on a 2D grid with all six components and the k couplings."""

    def __init__(self, wl, kind: str, n_channels: int, k: float, sigma: float = None, courant: float = None):
        self.k = float(k)                   # before the base class checks the Lorentz stability
        super().__init__(wl, kind, n_channels, ("x", "y", "z"), ("x", "y", "z"), sigma, courant)
        self.kd = self.k * self.dx          # k in the undivided form of the curls

    def curl_bound(self) -> float:
        """(K dx)^2 bound: the in-plane 8 plus (k dx)^2."""
        return 8.0 + (self.k / self.wl.res) ** 2

    def curl_e(self, a: str) -> np.ndarray:
        out = super().curl_e(a)
        if a == "x":
            out = out - self.kd * self.E["y"]
        elif a == "y":
            out = out + self.kd * self.E["x"]
        return out

    def curl_h(self, a: str) -> np.ndarray:
        out = super().curl_h(a)
        if a == "x":
            out = out + self.kd * self.H["y"]
        elif a == "y":
            out = out - self.kd * self.H["x"]
        return out


def kz_gammas(wl, k: float, chans, faces, bases, eps_s: float, mu_s: float, n_steps: int) -> np.ndarray:
    """Gamma_c(t_m), m = 1..n_steps, of every channel at wavevector k:
    E-kind and H-kind channels each advanced together (kick with -W^T f_n /
    (dx eps_S or mu_S), consistent start, one measurement per step)."""
    dx = 1.0 / wl.res
    gam = np.zeros((n_steps, len(chans)))
    cache = {}

    def W(fi, comp):
        if (fi, comp) not in cache:
            cache[(fi, comp)] = gather(wl, faces[fi], comp)
        return cache[(fi, comp)]

    for kind in ("E", "H"):
        sel = [c for c, ch in enumerate(chans) if ch.kind == kind]
        if not sel:
            continue
        sim = KzSim(wl, kind, len(sel), k)
        medium = eps_s if kind == "E" else mu_s
        for j, c in enumerate(sel):
            ch = chans[c]
            idx, w = W(ch.face, ch.src)
            f = bases[ch.face][0][ch.row]
            src = np.zeros(int(np.prod(sim.grid_shape)))
            np.add.at(src, idx.ravel(), (w * f[:, None]).ravel())
            sim.field(ch.src)[j] += (-src / (dx * medium)).reshape(sim.grid_shape)
        sim.start()
        groups = defaultdict(list)
        for j, c in enumerate(sel):
            groups[(chans[c].face, chans[c].meas)].append(j)
        plan = []
        for (fi, q), js in groups.items():
            idx, w = W(fi, q)
            rows = np.array([bases[fi][0][chans[sel[j]].row] for j in js])
            plan.append((q, np.array(js), np.array([sel[j] for j in js]), idx, w, rows))
        for m in range(n_steps):
            sim.step()
            for q, js, cols, idx, w, rows in plan:
                X = sim.field(q).reshape(sim.C, -1)[js]
                wx = np.sum(X[:, idx] * w[None], axis=2)
                gam[m, cols] = dx * np.sum(rows * wx, axis=1)
    return gam


@dataclasses.dataclass
class KzResult:
    force: float
    per_k: List[float]          # F(k_q), unweighted
    acc: np.ndarray             # (n_k, C) channel integrals
    sign: np.ndarray
    chans: list
    faces: list
    trace: np.ndarray = None    # trace[m] = sum_q w_q F_q after m + 1 steps (every k shares dt)


def solve(wl, ks: Sequence[float], weights: Sequence[float]) -> KzResult:
    """sum_q w_q F(k_q) for a workload with pol "3D" on a 2D grid."""
    if wl.ndim != 2 or wl.pol != "3D":
        raise ValueError("k_z runs take a 2D workload with pol '3D'")
    faces, bases, eps_s, mu_s, chans = setup(wl)
    dt = wl.courant / wl.res
    K = kernel_table(wl.kernel, wl.sigma, dt, wl.n_steps)
    sign = np.array([c.sign for c in chans])
    acc = np.zeros((len(ks), len(chans)))
    per_k = []
    trace = np.zeros(wl.n_steps)
    for q, k in enumerate(ks):
        gam = kz_gammas(wl, k, chans, faces, bases, eps_s, mu_s, wl.n_steps)
        terms = dt * K[:, None] * gam
        acc[q] = terms.sum(axis=0)
        per_k.append(float(np.sum(sign * acc[q]) / np.pi))
        trace += weights[q] * np.cumsum(terms @ sign) / np.pi
    force = float(sum(w * f for w, f in zip(weights, per_k)))
    return KzResult(force, per_k, acc, sign, chans, faces, trace)

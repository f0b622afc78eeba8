"""Bloch-periodic boundaries along x for z-invariant problems (Sec. III D:
for a system periodic in x with period L the force is an integral over the
Bloch wavevectors k_x of one unit cell, each a simulation with
Bloch-periodic boundaries; with the k_z runs of oracle.kz this covers a cell
periodic in x and invariant in z).  Test infrastructure: only tests/, the
package smoke check and the benchmark's CPU baseline use this module.

Fields.  At wavevector k_x the fields are complex and quasi-periodic:
F(x + L) = exp(i k_x L) F(x).  A difference that crosses the periodic edge
takes the neighbour with that phase: F[nx] = p F[0] for a forward
difference, F[-1] = conj(p) F[nx - 1] for a backward one, p = exp(i k_x L).
Everything else is the six-component k_z system of oracle.kz (complex
arrays; the update coefficients are real).

Sources and measurements.  The stress surface must not wrap across the
periodic edge (its interpolation then needs no phase).  Sources are real
(W^T f_n, as for the other runs); the force takes the real part of the
measured response, Re Gamma_c: the k_x and -k_x runs are complex
conjugates, so the pair contributes twice the real part.

Force.  F(k_x, k_z) = (1/pi) sum_c s_c sum_m dt K(t_m) Re Gamma_c(t_m); the
caller's quadrature weights turn the runs into the integral over the
Brillouin zone and over k_z.
"""
from __future__ import annotations

import dataclasses
from collections import defaultdict
from typing import List, Sequence, Tuple

import numpy as np

from .force import setup
from .kernels import kernel_table
from .kz import KzSim
from .surface import gather
from .yee import AXIS_OF, CYCLIC


class BlochSim(KzSim):
    """KzSim with complex fields and a Bloch phase across the x edge."""

    def __init__(self, wl, kind: str, n_channels: int, kz: float, kx: float, sigma: float = None,
                 courant: float = None):
        super().__init__(wl, kind, n_channels, kz, sigma, courant)
        if wl.bc[0] != "periodic":
            raise ValueError("Bloch-periodic x needs a periodic x axis")
        self.kx = float(kx)
        self.phase = np.exp(1j * self.kx * wl.shape[0] / wl.res)
        for f in (self.E, self.H):
            for a in f:
                f[a] = f[a].astype(np.complex128)

    def _diff(self, target: str, F: np.ndarray, axis: int, forward: bool) -> np.ndarray:
        if axis != 0:
            return super()._diff(target, F, axis, forward)
        if forward:
            nb = np.roll(F, -1, axis=3)
            nb[..., -1] *= self.phase            # F[nx] = p F[0]
            return nb - F
        nb = np.roll(F, 1, axis=3)
        nb[..., 0] *= np.conj(self.phase)        # F[-1] = conj(p) F[nx - 1]
        return F - nb

    def curl_e(self, a: str) -> np.ndarray:
        b, c = CYCLIC[a]
        out = np.zeros((self.C,) + self.grid_shape, dtype=np.complex128)
        out += self._diff("H" + a, self.E[c], AXIS_OF[b], True)
        out -= self._diff("H" + a, self.E[b], AXIS_OF[c], True)
        if a == "x":
            out -= self.kd * self.E["y"]
        elif a == "y":
            out += self.kd * self.E["x"]
        return out

    def curl_h(self, a: str) -> np.ndarray:
        b, c = CYCLIC[a]
        out = np.zeros((self.C,) + self.grid_shape, dtype=np.complex128)
        out += self._diff("E" + a, self.H[c], AXIS_OF[b], False)
        out -= self._diff("E" + a, self.H[b], AXIS_OF[c], False)
        if a == "x":
            out += self.kd * self.H["y"]
        elif a == "y":
            out -= self.kd * self.H["x"]
        return out


def check_no_wrap(wl, faces) -> None:
    """Raise if an interpolation point of S lies across the periodic x edge
    (its weight would need the Bloch phase): every x index a component is
    read at must fall in [0, nx) before the periodic wrap."""
    nx = wl.shape[0]
    for f in faces:
        if f.axis == 0:
            xs2 = [2 * f.plane]
        else:
            k = f.tang.index(0)
            xs2 = [2 * (f.start[k] + t) + 1 for t in range(f.count[k])]
        for o2 in (0, 1):                        # doubled x offsets of the components
            for s2 in xs2:
                d = s2 - o2
                pts = [d // 2] if d % 2 == 0 else [(d - 1) // 2, (d + 1) // 2]
                if min(pts) < 0 or max(pts) >= nx:
                    raise ValueError("the stress surface wraps across the Bloch-periodic edge")


def bloch_gammas(wl, kz: float, kx: float, chans, faces, bases, eps_s: float, mu_s: float,
                 n_steps: int) -> np.ndarray:
    """Re Gamma_c(t_m), m = 1..n_steps, of every channel at (k_x, k_z)."""
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
        sim = BlochSim(wl, kind, len(sel), kz, kx)
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
                X = sim.field(q).reshape(sim.C, -1)[js].real
                wx = np.sum(X[:, idx] * w[None], axis=2)
                gam[m, cols] = dx * np.sum(rows * wx, axis=1)
    return gam


@dataclasses.dataclass
class BlochResult:
    force: float
    per_k: List[float]          # F(k_x, k_z) per point, unweighted
    acc: np.ndarray             # (n_points, C)
    sign: np.ndarray
    chans: list
    faces: list


def solve(wl, points: Sequence[Tuple[float, float]], weights: Sequence[float]) -> BlochResult:
    """sum_q w_q F(k_x, k_z)_q for (k_x, k_z) points of a 2D workload with
    pol "3D" and a periodic x axis."""
    if wl.ndim != 2 or wl.pol != "3D":
        raise ValueError("Bloch runs take a 2D workload with pol '3D'")
    faces, bases, eps_s, mu_s, chans = setup(wl)
    check_no_wrap(wl, faces)
    dt = wl.courant / wl.res
    K = kernel_table(wl.kernel, wl.sigma, dt, wl.n_steps)
    sign = np.array([c.sign for c in chans])
    acc = np.zeros((len(points), len(chans)))
    per_k = []
    for q, (kx, kz) in enumerate(points):
        gam = bloch_gammas(wl, kz, kx, chans, faces, bases, eps_s, mu_s, wl.n_steps)
        acc[q] = (dt * K[:, None] * gam).sum(axis=0)
        per_k.append(float(np.sum(sign * acc[q]) / np.pi))
    force = float(sum(w * f for w, f in zip(weights, per_k)))
    return BlochResult(force, per_k, acc, sign, chans, faces)

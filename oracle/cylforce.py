"""Force on an object in a cylindrically symmetric geometry (Sec. III C;
Appendix, harmonic expansion in cylindrical coordinates).  Test
infrastructure: only tests/, the package smoke check and the benchmark's CPU
baseline use this module.

For every azimuthal order m = 0..m_max the (r, z) problem is advanced with
:class:`oracle.cyl.CylSim` once per channel, exactly as in the Cartesian 2D
case (kick with the interpolated surface current, consistent start,
measure the interpolated field on S each step), and the channel integrals
are combined as

    F = (1/pi) sum_m w_m sum_c s_c sum_k dt_m K(t_k) Gamma_{c,m}(t_k),
    w_0 = 1, w_{m>0} = 2            (the +m and -m terms are conjugates)

with K the general (three-dimensional) kernel.  The surface measure is the
Cartesian line element ds along S in the (r, z) plane (the Jacobian r
cancels, as the Appendix shows).  Every order m runs with its own step
dt_m = cylindrical_courant(courant, m) dx over the same physical time.

Partial force.  The orders advance on different steps, so F(T') is read on
the axis of the n_steps base steps: after d of them order m has run
floor(d T_m / n_steps) of its own T_m steps (all of them at d = n_steps),
the same physical time to within one step of that order, and trace[d - 1]
sums every order's partial channel integrals there.

Surface.  S is a box in the (z, r) plane: z from s_lo[0] to s_hi[0] (cells),
r from s_lo[1] to s_hi[1] (cells); r = 0 (s_lo[1] = 0) means S reaches the
axis (no inner face), s_hi[1] = nr means S reaches the tube wall at
r = nr - 1/2 (no outer face; stress on a PEC wall has no axial force
component).  Samples along r sit at the cell midpoints r = k + 1/2 (weight 1
cell); a face that reaches the wall ends with a half cell [nr - 1, nr - 1/2]
sampled at r = nr - 1 (weight 1/2).  The basis on a face is orthonormal
under these weights (cosines cos(n pi s / L) made orthonormal by weighted
Gram-Schmidt; with unit weights this is the cosine basis of the Cartesian
faces), and the kick and the measurement both use w_s f_n(s): the weighted
quadrature of the source and of the surface integral.
"""
from __future__ import annotations

import dataclasses
from collections import defaultdict
from typing import List

import numpy as np

from casimir_inputs.geometry import COMPONENT_OFFSETS2
from .cyl import CylSim, cylindrical_courant
from .kernels import kernel_table
from .surface import channel_specs


@dataclasses.dataclass
class CylFace:
    index: int          # 2 * axis + (side > 0)
    axis: int           # 0: normal along z (axial), 1: normal along r
    side: int
    plane2: int         # doubled coordinate of the plane along the normal axis
    samples2: np.ndarray  # doubled coordinates of the samples along the tangential axis
    weights: np.ndarray   # quadrature weights (cells)


def build_faces(wl) -> List[CylFace]:
    nz, nr = wl.shape[0], wl.shape[1]
    z0, z1 = wl.s_lo[0], wl.s_hi[0]
    r0, r1 = wl.s_lo[1], wl.s_hi[1]
    to_wall = r1 >= nr
    # samples along r (doubled y = 2 (r + 1/2)): midpoints r = k + 1/2
    k_end = nr - 1 if to_wall else r1
    ys = [2 * k + 2 for k in range(r0, k_end)]
    wy = [1.0] * len(ys)
    if to_wall:
        ys.append(2 * nr - 1)            # r = nr - 1, half cell up to the wall
        wy.append(0.5)
    ys, wy = np.array(ys), np.array(wy)
    xs = np.array([2 * i + 1 for i in range(z0, z1)])
    wx = np.ones(len(xs))
    faces = [CylFace(0, 0, -1, 2 * z0, ys, wy), CylFace(1, 0, +1, 2 * z1, ys, wy)]
    if r0 > 0:
        faces.append(CylFace(2, 1, -1, 2 * r0 + 1, xs, wx))
    if not to_wall:
        faces.append(CylFace(3, 1, +1, 2 * r1 + 1, xs, wx))
    return faces


def _points(d2: int, o2: int, n: int, periodic: bool):
    d = d2 - o2
    pts = [(d // 2, 1.0)] if d % 2 == 0 else [((d - 1) // 2, 0.5), ((d + 1) // 2, 0.5)]
    out = []
    for i, w in pts:
        if periodic:
            i %= n
        elif i >= n:
            continue                     # beyond the tube wall / end cap: the field is 0 there
        elif i < 0:
            raise ValueError("surface stencil leaves the grid")
        out.append((i, w))
    return out


def gather(wl, face: CylFace, comp: str):
    """Interpolation W of one component on one face: (idx, w) lists per
    sample, flat indices j * nz + i into an (nr, nz) array."""
    nz, nr = wl.shape[0], wl.shape[1]
    o2 = COMPONENT_OFFSETS2[comp]
    idx, wts = [], []
    for s2 in face.samples2:
        if face.axis == 0:
            px = _points(face.plane2, o2[0], nz, wl.bc[0] == "periodic")
            py = _points(int(s2), o2[1], nr, False)
        else:
            px = _points(int(s2), o2[0], nz, wl.bc[0] == "periodic")
            py = _points(face.plane2, o2[1], nr, False)
        ii, ww = [], []
        for (i, wi) in px:
            for (j, wj) in py:
                ii.append(j * nz + i)
                ww.append(wi * wj)
        idx.append(ii)
        wts.append(ww)
    return idx, wts


def face_basis(wl, face: CylFace):
    """(rows, labels): rows[n] = w_s f_n(s) for the first n_harm members of
    the weighted orthonormal cosine basis (inner product dx sum_s w_s f g)."""
    dx = 1.0 / wl.res
    w = face.weights
    pos = np.cumsum(w) - 0.5 * w                        # sample position along the face (cells)
    L = float(np.sum(w))
    N = len(w)
    n_harm = min(wl.n_harm, N)
    V = np.array([np.cos(n * np.pi * pos / L) for n in range(N)])
    out = []
    for n in range(n_harm):
        v = V[n].copy()
        for u in out:
            v -= dx * np.sum(w * u * v) * u
        v /= np.sqrt(dx * np.sum(w * v * v))
        out.append(v)
    rows = np.array([w * f for f in out])
    return rows, list(range(n_harm))


@dataclasses.dataclass
class CylResult:
    force: float
    per_m: dict
    acc: np.ndarray        # (m_max + 1, C) channel integrals per order
    sign: np.ndarray
    chans: list
    faces: list
    n_steps_m: list
    trace: np.ndarray = None   # F after d = 1..n_steps base steps (see the module docstring)


def setup(wl):
    faces = build_faces(wl)
    bases = {fi: face_basis(wl, f) for fi, f in enumerate(faces)}
    eps_s, mu_s = float(wl.eps[0]), float(wl.mu[0])
    if "medium_id" in wl.meta:
        eps_s, mu_s = float(wl.eps[wl.meta["medium_id"]]), float(wl.mu[wl.meta["medium_id"]])
    chans = []
    for fi, f in enumerate(faces):
        rows, labels = bases[fi]
        for row, lab in enumerate(labels):
            for kind, j, q, coef in channel_specs("3D", f.axis, 0, eps_s, mu_s):
                chans.append(dict(face=fi, row=row, label=lab, kind=kind, src=kind + j, meas=kind + q,
                                  sign=float(f.side) * coef))
    return faces, bases, eps_s, mu_s, chans


def surface_vector(wl, face: CylFace, comp: str, frow: np.ndarray) -> np.ndarray:
    """W^T applied to one basis row (w_s f_n(s)): a dense (nr * nz) vector.
    The kick deposits it, the measurement takes its inner product with the
    field (the same vector, so the two are adjoint)."""
    nz, nr = wl.shape[0], wl.shape[1]
    idx, w = gather(wl, face, comp)
    v = np.zeros(nr * nz)
    for s in range(len(idx)):
        for i, wi in zip(idx[s], w[s]):
            v[i] += wi * frow[s]
    return v


def run_order(wl, m: int, faces, bases, eps_s, mu_s, chans, n_steps: int, courant: float):
    """Gamma_c(t_k), k = 1..n_steps, for order m (all channels), and dt."""
    dx = 1.0 / wl.res
    gam = np.zeros((n_steps, len(chans)))
    dt = courant * dx
    for kind in ("E", "H"):
        sel = [c for c, ch in enumerate(chans) if ch["kind"] == kind]
        if not sel:
            continue
        sim = CylSim(wl, kind, len(sel), m, courant)
        dt = sim.dt
        medium = eps_s if kind == "E" else mu_s
        nz, nr = sim.nz, sim.nr
        meas = defaultdict(list)                 # measured component -> (column in sel, vector)
        for k, c in enumerate(sel):
            ch = chans[c]
            f = bases[ch["face"]][0][ch["row"]]
            src = surface_vector(wl, faces[ch["face"]], ch["src"], f)
            sim.F[ch["src"]][k] += (-src / (dx * medium)).reshape(nr, nz)
            meas[ch["meas"]].append((k, surface_vector(wl, faces[ch["face"]], ch["meas"], f)))
        sim.fold_axis()
        sim.start()
        plan = [(q, np.array([k for k, _ in lst]), np.array([v for _, v in lst])) for q, lst in meas.items()]
        cols = np.array(sel)
        for step in range(n_steps):
            sim.step()
            for q, ks, V in plan:
                X = sim.F[q].reshape(len(sel), -1)[ks]
                gam[step, cols[ks]] = dx * np.sum(V * X, axis=1)
    return gam, dt


def solve(wl, m_max: int):
    """Force along the axis summed over m = 0..m_max."""
    faces, bases, eps_s, mu_s, chans = setup(wl)
    dx = 1.0 / wl.res
    t_end = wl.n_steps * wl.courant * dx
    sign = np.array([ch["sign"] for ch in chans])
    acc = np.zeros((m_max + 1, len(chans)))
    per_m, n_steps_m = {}, []
    base = wl.n_steps
    trace = np.zeros(base)
    d = np.arange(1, base + 1)
    for m in range(m_max + 1):
        cm = cylindrical_courant(wl.courant, m)
        T = int(round(t_end / (cm * dx)))
        gam, dt = run_order(wl, m, faces, bases, eps_s, mu_s, chans, T, cm)
        K = kernel_table(wl.kernel, wl.sigma, dt, T)
        terms = dt * K[:, None] * gam
        acc[m] = terms.sum(axis=0)
        wm = 1.0 if m == 0 else 2.0
        per_m[m] = wm * float(np.sum(sign * acc[m])) / np.pi
        n_steps_m.append(T)
        # partial sums of this order after floor(d T / base) of its steps
        part = np.concatenate([[0.0], np.cumsum(terms @ sign)])
        s = np.where(d >= base, T, (d * T) // base)
        trace += wm * part[s] / np.pi
    return CylResult(sum(per_m.values()), per_m, acc, sign, chans, faces, n_steps_m, trace)

"""Stress surface S, its per-face harmonic basis and the stress-tensor channels.

Surface (Sec. III, the rectangular S): an axis-aligned box with integer
corners.  Face (a, side) is the plane x_a = lo_a (side -1, outward normal
-e_a) or x_a = hi_a (side +1).  Along each tangential axis b the face is
sampled at the midpoints lo_b + i + 1/2, i = 0..N_b-1; corners and edges are
never sampled.  An axis that the box spans completely while the grid is
periodic along it has no faces (the two would coincide and cancel) and its
samples wrap around.

Current interpolation (Sec. III A, the sources placed as averaged currents on
neighbouring grid points): component q is read at a sample point through
W, the tensor product over axes of weight 1 (component on the sample's
coordinate) or 1/2, 1/2 (component half a cell off: its two neighbours).
Sources use the adjoint W^T.

Basis (Sec. III A, the f_n(x) equation): on a face of length L = N dx the
cosine functions f_n(s) = sqrt(c_n / L) cos(n pi s / L), c_0 = 1, c_n = 2,
sampled at the midpoints.  The printed normalization sqrt(2/L) also for n = 0
is not normalized and is read as sqrt(1/L).  These are exactly orthonormal
under sum_i dx f_n(s_i) f_k(s_i) for n, k < N, so at most N harmonics exist
per face; a request for more is clamped.  3D faces use the product f_m(u)
f_n(v).  Two further complete orthonormal bases serve as test fixtures: the
point basis (Fig. 2, one source per sample point) and a periodic Fourier
basis.

Channels (Sec. II, the Gamma^E_i definition and its magnetic analogue, with
the Minkowski epsilon_S, mu_S of the medium S lies in): for force axis d and
a face with normal a, the stress component T_da gives

* a == d:  E(k->k) with coefficient eps_S (delta_kd - 1/2) for each E
  component k of the polarization, and H(k->k) with mu_S (delta_kd - 1/2);
* a != d:  E(a->d) with eps_S and H(a->d) with mu_S when both components
  exist in the polarization.

X(j->q) is the q-component response to a source along j.  The sign of a
channel is side * coefficient.

Parity: pinned (tests/test_oracle_surface.py: orthonormality, completeness,
harmonic sum == point-source sum, mirror symmetry, plate forces).
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np

from casimir_inputs.geometry import COMPONENT_OFFSETS2

POL_COMPONENTS = {
    "TM": (("z",), ("x", "y")),
    "TE": (("x", "y"), ("z",)),
    "3D": (("x", "y", "z"), ("x", "y", "z")),
}
AXES = "xyz"


@dataclasses.dataclass(frozen=True)
class Face:
    index: int            # 2*axis + (side > 0)
    axis: int             # normal axis a
    side: int             # -1 or +1
    plane: int            # integer coordinate of the face plane
    tang: Tuple[int, ...] # tangential axes (ascending)
    start: Tuple[int, ...]
    count: Tuple[int, ...]

    @property
    def n_samples(self) -> int:
        return int(np.prod(self.count))


def spans_periodic(wl, axis: int) -> bool:
    return (wl.bc[axis] == "periodic" and wl.s_lo[axis] == 0
            and wl.s_hi[axis] == wl.shape[axis])


def build_faces(wl) -> List[Face]:
    faces = []
    for a in range(wl.ndim):
        if spans_periodic(wl, a):
            continue
        tang = tuple(b for b in range(wl.ndim) if b != a)
        start = tuple(int(wl.s_lo[b]) for b in tang)
        count = tuple(int(wl.s_hi[b] - wl.s_lo[b]) for b in tang)
        for side, plane in ((-1, wl.s_lo[a]), (+1, wl.s_hi[a])):
            faces.append(Face(2 * a + (side > 0), a, side, int(plane), tang, start, count))
    return faces


def _axis_points(s2: int, o2: int, n: int, periodic: bool):
    """Indices and weights along one axis for a sample at doubled coordinate
    s2 and a component with doubled offset o2."""
    d = s2 - o2
    if d % 2 == 0:
        pts = [(d // 2, 1.0)]
    else:
        pts = [((d - 1) // 2, 0.5), ((d + 1) // 2, 0.5)]
    out = []
    for i, w in pts:
        if periodic:
            i %= n
        elif not (0 <= i < n):
            raise ValueError("surface stencil leaves the grid")
        out.append((i, w))
    return out


def gather(wl, face: Face, comp: str) -> Tuple[np.ndarray, np.ndarray]:
    """W for one face and component: (idx, w), each of shape (N, P), with idx
    flat indices into a (nz, ny, nx) array."""
    nx, ny, nz = wl.shape
    o2 = COMPONENT_OFFSETS2[comp]
    ranges = [range(c) for c in face.count]
    idx_rows, w_rows = [], []
    for t in itertools.product(*ranges):
        per_axis = []
        for ax in range(3):
            n = wl.shape[ax]
            if ax >= wl.ndim:
                per_axis.append([(0, 1.0)])
                continue
            if ax == face.axis:
                s2 = 2 * face.plane
            else:
                k = face.tang.index(ax)
                s2 = 2 * (face.start[k] + t[k]) + 1
            per_axis.append(_axis_points(s2, o2[ax], n, wl.bc[ax] == "periodic"))
        row_i, row_w = [], []
        for (i, wi), (j, wj), (k, wk) in itertools.product(*per_axis):
            row_i.append((k * ny + j) * nx + i)
            row_w.append(wi * wj * wk)
        idx_rows.append(row_i)
        w_rows.append(row_w)
    return np.array(idx_rows, dtype=np.int64), np.array(w_rows, dtype=np.float64)


def _dct_1d(n_samples: int, n_harm: int, dx: float) -> np.ndarray:
    L = n_samples * dx
    s = (np.arange(n_samples) + 0.5) * dx
    rows = []
    for n in range(min(n_harm, n_samples)):
        c = 1.0 if n == 0 else 2.0
        rows.append(np.sqrt(c / L) * np.cos(n * np.pi * s / L))
    return np.array(rows)


def _fourier_1d(n_samples: int, n_harm: int, dx: float) -> np.ndarray:
    L = n_samples * dx
    s = (np.arange(n_samples) + 0.5) * dx
    rows = [np.full(n_samples, np.sqrt(1.0 / L))]
    k = 1
    while len(rows) < min(n_harm, n_samples):
        if 2 * k < n_samples:
            rows.append(np.sqrt(2.0 / L) * np.cos(2 * np.pi * k * s / L))
            if len(rows) < min(n_harm, n_samples):
                rows.append(np.sqrt(2.0 / L) * np.sin(2 * np.pi * k * s / L))
        else:  # k == N/2: only the sine survives at midpoints
            rows.append(np.sqrt(1.0 / L) * np.sin(2 * np.pi * k * s / L))
        k += 1
    return np.array(rows)


def face_basis(wl, face: Face, basis: str = "dct") -> Tuple[np.ndarray, List[int]]:
    """Basis matrix B (n_funcs, N) with B[k, i] = f_k(s_i), and the harmonic
    label of each row (n in 2D, m * n_harm + n in 3D, the sample index for
    the point basis)."""
    dx = 1.0 / wl.res
    if basis == "point":
        N = face.n_samples
        dA = dx ** (wl.ndim - 1)
        return np.eye(N) / np.sqrt(dA), list(range(N))
    one_d = _dct_1d if basis == "dct" else _fourier_1d
    tabs = [one_d(c, wl.n_harm, dx) for c in face.count]
    if len(tabs) == 1:
        return tabs[0], list(range(tabs[0].shape[0]))
    bu, bv = tabs
    rows, labels = [], []
    for m in range(bu.shape[0]):
        for n in range(bv.shape[0]):
            rows.append(np.outer(bu[m], bv[n]).ravel())
            labels.append(m * wl.n_harm + n)
    return np.array(rows), labels


def channel_specs(pol: str, face_axis: int, d: int, eps_s: float, mu_s: float):
    """[(kind, j, q, coefficient)] for one face orientation."""
    e_comps, h_comps = POL_COMPONENTS[pol]
    a = AXES[face_axis]
    dd = AXES[d]
    out = []
    if face_axis == d:
        for k in e_comps:
            out.append(("E", k, k, eps_s * ((1.0 if k == dd else 0.0) - 0.5)))
        for k in h_comps:
            out.append(("H", k, k, mu_s * ((1.0 if k == dd else 0.0) - 0.5)))
    else:
        if a in e_comps and dd in e_comps:
            out.append(("E", a, dd, eps_s))
        if a in h_comps and dd in h_comps:
            out.append(("H", a, dd, mu_s))
    return out


@dataclasses.dataclass(frozen=True)
class Channel:
    face: int      # index into the face list
    row: int       # basis row on that face
    label: int     # harmonic label
    kind: str      # "E" or "H"
    src: str       # source component, e.g. "Ez"
    meas: str      # measured component
    sign: float    # side * coefficient
    pol: str


def polarizations(pol: str) -> Sequence[str]:
    return {"TM": ("TM",), "TE": ("TE",), "TM+TE": ("TM", "TE"), "3D": ("3D",)}[pol]


def channel_table(wl, faces: Sequence[Face], bases: Dict[int, Tuple[np.ndarray, List[int]]],
                  eps_s: float, mu_s: float) -> List[Channel]:
    chans = []
    for pol in polarizations(wl.pol):
        for fi, f in enumerate(faces):
            specs = channel_specs(pol, f.axis, wl.force_axis, eps_s, mu_s)
            B, labels = bases[fi]
            for row, lab in enumerate(labels):
                for kind, j, q, coef in specs:
                    chans.append(Channel(fi, row, lab, kind, kind + j, kind + q,
                                         float(f.side) * coef, pol))
    return chans

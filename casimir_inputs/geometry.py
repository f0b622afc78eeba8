"""Geometry primitives and rasterization onto the six Yee component lattices.

Coordinates are in grid cells (pixels).  A Yee component with doubled offset
``o = (ox, oy, oz)`` (each 0 or 1, meaning 0 or half a cell) stored at array
index ``[k, j, i]`` sits at position ``((2i+ox)/2, (2j+oy)/2, (2k+oz)/2)``.
The offsets are the standard Yee placement: E_a is shifted half a cell along
its own axis a; H_a is shifted half a cell along both axes other than a.

Primitives are painted in list order (a later primitive overrides an earlier
one), and insideness is a closed-set test evaluated at the component's exact
position.  Integer and half-integer geometry is therefore rasterized without
any floating-point ties.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np

COMPONENTS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")

# doubled offsets (x, y, z) of each component inside its cell
COMPONENT_OFFSETS2 = {
    "Ex": (1, 0, 0),
    "Ey": (0, 1, 0),
    "Ez": (0, 0, 1),
    "Hx": (0, 1, 1),
    "Hy": (1, 0, 1),
    "Hz": (1, 1, 0),
}

PEC = float("-inf")  # as an epsilon value: perfect electric conductor
PMC = float("-inf")  # as a mu value: perfect magnetic conductor


@dataclasses.dataclass(frozen=True)
class Box:
    """Closed axis-aligned box [lo, hi] in pixel units (3 coords each)."""

    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    material: int

    def inside(self, x, y, z):
        return (
            (x >= self.lo[0]) & (x <= self.hi[0])
            & (y >= self.lo[1]) & (y <= self.hi[1])
            & (z >= self.lo[2]) & (z <= self.hi[2])
        )


@dataclasses.dataclass(frozen=True)
class Sphere:
    """Closed ball |p - c| <= r in pixel units."""

    center: Tuple[float, float, float]
    radius: float
    material: int

    def inside(self, x, y, z):
        dx = x - self.center[0]
        dy = y - self.center[1]
        dz = z - self.center[2]
        return dx * dx + dy * dy + dz * dz <= self.radius * self.radius


def rasterize(shape_xyz: Sequence[int], primitives: Sequence, background: int = 0,
              components: Sequence[str] = COMPONENTS) -> Dict[str, np.ndarray]:
    """Return {component: uint8 id grid of shape (nz, ny, nx)}.

    In 2D (nz == 1) the z coordinate of every component is taken as 0.5 so a
    2D primitive should span z over [-inf, inf] (use +-1e30).
    """
    nx, ny, nz = (int(v) for v in shape_xyz)
    out = {}
    for comp in components:
        ox, oy, oz = COMPONENT_OFFSETS2[comp]
        x = (2.0 * np.arange(nx) + ox) / 2.0
        y = (2.0 * np.arange(ny) + oy) / 2.0
        z = (2.0 * np.arange(nz) + oz) / 2.0
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        ids = np.full((nz, ny, nx), background, dtype=np.uint8)
        for prim in primitives:
            ids[prim.inside(X, Y, Z)] = prim.material
        out[comp] = ids
    return out


@dataclasses.dataclass
class Workload:
    """A complete force-solve input.

    shape      (nx, ny, nz); nz == 1 for 2D problems
    res        pixels per unit length (the grid spacing is 1/res)
    bc         boundary per axis: "pec" | "periodic" | "pml"
    pml_cells  PML thickness per axis (cells) when bc == "pml"
    eps, mu    material table; eps=-inf marks PEC, mu=-inf marks PMC
    comp_ids   per-component uint8 id grids, shape (nz, ny, nx)
    s_lo, s_hi stress-tensor surface box corners (integer cells, 3 coords)
    n_harm     cosine harmonics per face direction (clamped per face to its
               sample count by the solvers)
    force_axis 0/1/2
    sigma, courant, n_steps, pol ("TM", "TE", "TM+TE", "3D"), kernel
    ("zinv2d" | "general"), precision ("fp64" | "fp32")
    coord      "cartesian", "cylindrical" or "kz": a cylindrical workload is a 2D
               (z, r) grid, x = z along the symmetry axis, y = r + 1/2
               (cells), the tube wall at r = ny - 1/2
    m_max      cylindrical workloads: azimuthal orders 0..m_max
    kz, kz_weight  "kz" workloads (z-invariant 2D, six components): the
               Bloch wavevectors along z and the weights of F(k_q) in the force
    kx         "kz" workloads: Bloch wavevector along a periodic x per point
               (empty: all zero; any nonzero value makes the fields complex)
    lorentz    dispersive materials: {material id: ((d_eps, omega_0), ...)},
               Lorentz terms d_eps omega_0^2 / (omega_0^2 - omega^2) added to
               eps[id], which is then the high-frequency permittivity
               (Sec. III B; empty: every material is non-dispersive)
    """

    name: str
    ndim: int
    shape: Tuple[int, int, int]
    res: float
    bc: Tuple[str, str, str]
    pml_cells: Tuple[int, int, int]
    eps: List[float]
    mu: List[float]
    comp_ids: Dict[str, np.ndarray]
    s_lo: Tuple[int, int, int]
    s_hi: Tuple[int, int, int]
    n_harm: int
    force_axis: int
    sigma: float = 1.0
    courant: float = 0.5
    n_steps: int = 1000
    pol: str = "TM"
    kernel: str = "zinv2d"
    precision: str = "fp64"
    meta: dict = dataclasses.field(default_factory=dict)
    coord: str = "cartesian"
    m_max: int = 0
    kz: Tuple[float, ...] = ()
    kz_weight: Tuple[float, ...] = ()
    kx: Tuple[float, ...] = ()
    lorentz: Dict[int, Tuple[Tuple[float, float], ...]] = dataclasses.field(default_factory=dict)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    @property
    def n_cells(self) -> int:
        return int(self.shape[0]) * int(self.shape[1]) * int(self.shape[2])

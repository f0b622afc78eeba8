"""Seeded request streams for the serving benchmark.

The mixed stream: Poisson arrivals (rate lam per second), each request a
complete force solve drawn
  - with probability p2d from 2D TE+TM pistons of the uneven-set geometry
    (total clearance h ~ U[0.1, 2.0], resolution ~ U{20..60}, grid
    10 res x round(res (2 + h)), T = 250 res steps, 40 harmonics per face),
  - otherwise from 3D sphere-above-indented-plate cells (n ~ U{96, 128,
    160, 192} cells per side, res = n / 4, gap h ~ U[0.2, 1.5],
    T = 125 res steps, 8 x 8 harmonics per face, 16-cell z PML).
Workloads are built lazily (a 192^3 rasterization takes seconds).  Some 3D
gaps are too small for a box S to fit inside the indentation; those
requests fail validation with a surface error and are counted as rejected.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .configs import piston2d, sphere_plate3d
from .geometry import Workload


def uneven_piston(h: float, res: int, n_steps: Optional[int] = None, **over) -> Workload:
    """Piston of the uneven set at resolution res: 10 x (2 + h) units,
    0.75-unit sidewall slabs, a 1.0 x 0.5 block, blocks 1 unit apart."""
    ny = int(round(res * (2.0 + h)))
    slab = int(round(0.75 * res))
    block_h = int(round(0.5 * res))
    clear = ny - 2 * slab - block_h
    y0 = slab + clear // 2
    kw = dict(pol="TM+TE", precision="fp32", n_steps=int(n_steps if n_steps else 250 * res),
              kernel="zinv2d", n_harm=40, name=f"piston_res{res}_h{h:.3f}_{10 * res}x{ny}")
    kw.update(over)
    w = piston2d(int(round(10 * res)), ny, slab, int(round(res)), block_h, int(round(res)), y0,
                 float(res), **kw)
    w.meta["h"] = float(h)
    return w


@dataclass
class Request:
    index: int
    t_arrive: float          # seconds after the stream starts
    kind: str                # "2d" / "3d"
    params: dict = field(default_factory=dict)

    def workload(self) -> Workload:
        p = self.params
        if self.kind == "2d":
            return uneven_piston(p["h"], p["res"], n_steps=p.get("n_steps"))
        return sphere_plate3d(p["n"], p["h"], n_steps=p.get("n_steps", int(125 * p["n"] / 4)))


def mixed_stream(n: int = 200, lam: float = 4.0, seed: int = 0, p2d: float = 0.7,
                 kinds: Optional[List[str]] = None) -> List[Request]:
    """n requests of the mixed stream.  kinds restricts the classes kept
    (the draws are made for every request either way, so a class's requests
    are the same with or without the filter; arrival times are redrawn at
    rate lam over the kept requests)."""
    rng = np.random.default_rng(seed)
    out: List[Request] = []
    t = 0.0
    k = 0
    while len(out) < n:
        gap = rng.exponential(1.0 / lam)
        if rng.random() < p2d:
            kind = "2d"
            params = dict(h=float(rng.uniform(0.1, 2.0)), res=int(rng.integers(20, 61)))
        else:
            kind = "3d"
            params = dict(n=int(rng.choice([96, 128, 160, 192])), h=float(rng.uniform(0.2, 1.5)))
        k += 1
        if kinds is not None and kind not in kinds:
            continue
        t += gap
        out.append(Request(index=k - 1, t_arrive=t, kind=kind, params=params))
    return out


def rescale_arrivals(reqs: List[Request], lam: float, seed: int = 1) -> List[Request]:
    """The same requests with fresh Poisson arrival times at rate lam."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in reqs:
        t += rng.exponential(1.0 / lam)
        out.append(Request(index=r.index, t_arrive=t, kind=r.kind, params=dict(r.params)))
    return out

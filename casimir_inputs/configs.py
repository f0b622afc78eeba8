"""Workload builders: the paper's 2D piston, 1D-reducible parallel plates and
the 3D sphere above an indented plate, at the sizes the benchmarks use.

Every builder returns a :class:`Workload` holding rasterized per-component
material ids.  Geometry follows the paper's examples (Sec. III A piston of
Fig. 1/3; Sec. III E sphere over an indented plate, Fig. 9) with the sizes of
the benchmark configurations:

* piston: two PEC blocks 1.0 x 0.5 separated by a gap a = 1.0, between
  sidewall slabs; ``h`` is the total vertical clearance (h/2 above and below
  each block).  The stress surface S is the right block grown by a margin of
  min(2, floor(g/2)) pixels, g being the smallest block-to-object gap.
* sphere-plate: a PEC plate whose top face carries a hemispherical
  indentation, a dielectric sphere above it, immersed in a fluid; periodic
  x/y, PML along z.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from .geometry import PEC, PMC, Box, Sphere, Workload, rasterize

BIG = 1e30


def _margin(min_gap_px: int) -> int:
    return int(min(2, min_gap_px // 2))


def piston2d(nx: int, ny: int, slab_px: int, block_w: int, block_h: int, gap: int,
             block_y0: int, res: float, sidewall: str = "pec", n_harm: int = 16,
             **opts) -> Workload:
    """2D piston on an nx x ny grid (pixel units).

    Sidewall slabs occupy y in [0, slab_px] and [ny - slab_px, ny]; blocks
    are PEC, the left one ending at x = (nx - gap)//2 and the right one
    starting gap pixels later; both span y in [block_y0, block_y0 + block_h].
    ``sidewall`` is "pec", "pmc" or "mu5" (a magnetic slab with mu = 5).
    The time kernel defaults to the z-invariant one (Appendix A.2), which
    holds for perfect conductors in vacuum; with mu = 5 slabs it defaults to
    the general kernel (the force of the two-dimensional system).
    """
    eps = [1.0, PEC, 1.0]
    mu = [1.0, 1.0, 1.0]
    side_id = 2
    if sidewall == "pec":
        side_id = 1
    elif sidewall == "pmc":
        mu[2] = PMC
    elif sidewall == "mu5":
        mu[2] = 5.0
    else:
        raise ValueError(sidewall)
    left_hi = (nx - gap) // 2
    left_lo = left_hi - block_w
    right_lo = left_hi + gap
    right_hi = right_lo + block_w
    y0, y1 = block_y0, block_y0 + block_h
    prims = [
        Box((-BIG, -BIG, -BIG), (BIG, slab_px, BIG), side_id),
        Box((-BIG, ny - slab_px, -BIG), (BIG, BIG, BIG), side_id),
        Box((left_lo, y0, -BIG), (left_hi, y1, BIG), 1),
        Box((right_lo, y0, -BIG), (right_hi, y1, BIG), 1),
    ]
    ids = rasterize((nx, ny, 1), prims)
    gap_below = y0 - slab_px
    gap_above = (ny - slab_px) - y1
    gap_right = nx - right_hi
    m = _margin(min(gap, gap_below, gap_above, gap_right))
    kw = dict(sigma=1.0, courant=0.5, n_steps=1000, pol="TM",
              kernel="general" if sidewall == "mu5" else "zinv2d", precision="fp64")
    kw.update(opts)
    return Workload(
        name=kw.pop("name", f"piston2d_{nx}x{ny}"), ndim=2, shape=(nx, ny, 1), res=float(res),
        bc=("pec", "pec", "periodic"), pml_cells=(0, 0, 0), eps=eps, mu=mu,
        comp_ids=ids, s_lo=(right_lo - m, y0 - m, 0), s_hi=(right_hi + m, y1 + m, 1),
        n_harm=int(n_harm), force_axis=0,
        meta=dict(margin=m, blocks=((left_lo, left_hi), (right_lo, right_hi)), block_y=(y0, y1),
                  slab_px=slab_px, sidewall=sidewall),
        **kw,
    )


def piston2d_units(res: int, width_u: float, height_u: float, h_u: float,
                   sidewall: str = "pec", **kw) -> Workload:
    """Piston with slabs filling everything outside the interior strip of
    height block_h + h, centred vertically (the reading used for the 2D
    benchmark configurations)."""
    nx = int(round(width_u * res))
    ny = int(round(height_u * res))
    block_w = int(round(1.0 * res))
    block_h = int(round(0.5 * res))
    gap = int(round(1.0 * res))
    h_px = int(round(h_u * res))
    interior = block_h + h_px
    slab = (ny - interior) // 2
    y0 = slab + h_px // 2
    return piston2d(nx, ny, slab, block_w, block_h, gap, y0, res, sidewall=sidewall, **kw)


def c1_piston_tm_fp64(**over) -> Workload:
    """2D TM, FP64: res 20, 80x40, h = 0.5, 16 harmonics, 2000 steps."""
    kw = dict(pol="TM", precision="fp64", n_steps=2000, kernel="zinv2d", n_harm=16,
              name="c1_piston_tm_fp64_80x40")
    kw.update(over)
    return piston2d_units(20, 4.0, 2.0, 0.5, **kw)


def c2_piston_tetm_fp32(**over) -> Workload:
    """2D TE+TM, FP32 fields: res 40, 400x200, h = 0.5, 40 harmonics, 10000 steps."""
    kw = dict(pol="TM+TE", precision="fp32", n_steps=10000, kernel="zinv2d", n_harm=40,
              name="c2_piston_tetm_fp32_400x200")
    kw.update(over)
    return piston2d_units(40, 10.0, 5.0, 0.5, **kw)


def c3_uneven_set(sidewall: str = "pec", n_inst: int = 24, res: int = 40, **over) -> List[Workload]:
    """24 pistons with total clearance h in linspace(0.1, 2.0), grid height
    round(res*(2+h)) (84..160 px at res 40), 0.75-unit sidewall slabs.
    PEC and PMC sidewalls use the z-invariant kernel; mu = 5 sidewalls the
    general kernel (Appendix A.2 assumes perfect conductors in vacuum)."""
    out = []
    for h in np.linspace(0.1, 2.0, n_inst):
        ny = int(round(res * (2.0 + h)))
        slab = int(round(0.75 * res))
        block_h = int(round(0.5 * res))
        clear = ny - 2 * slab - block_h
        y0 = slab + clear // 2
        kw = dict(pol="TM+TE", precision="fp32", n_steps=10000,
                  kernel="general" if sidewall == "mu5" else "zinv2d", n_harm=40,
                  name=f"c3_{sidewall}_h{h:.3f}_400x{ny}")
        kw.update(over)
        w = piston2d(int(round(10 * res)), ny, slab, int(round(res)), block_h, int(round(res)), y0,
                     res, sidewall=sidewall, **kw)
        w.meta["h"] = float(h)
        out.append(w)
    return out


def parallel_plates_1d(res: int, a_u: float, d_u: float, b_u: float, margin: int = 2,
                       ny: int = 1, **opts) -> Workload:
    """A PEC slab of thickness d between PEC walls at distances a (left) and
    b (right), translation invariant along y (periodic, ny cells).  S is two
    full-width lines, one in each gap."""
    a = int(round(a_u * res))
    d = int(round(d_u * res))
    b = int(round(b_u * res))
    nx = a + d + b
    eps = [1.0, PEC]
    mu = [1.0, 1.0]
    prims = [Box((a, -BIG, -BIG), (a + d, BIG, BIG), 1)]
    ids = rasterize((nx, ny, 1), prims)
    kw = dict(sigma=1.0, courant=0.5, n_steps=2000, pol="TM", kernel="zinv2d",
              precision="fp64")
    kw.update(opts)
    return Workload(
        name=kw.pop("name", f"plates_{nx}x{ny}"), ndim=2, shape=(nx, ny, 1), res=float(res),
        bc=("pec", "periodic", "periodic"), pml_cells=(0, 0, 0), eps=eps, mu=mu, comp_ids=ids,
        s_lo=(a - margin, 0, 0), s_hi=(a + d + margin, ny, 1), n_harm=max(1, ny), force_axis=0,
        meta=dict(a_px=a, d_px=d, b_px=b),
        **kw,
    )


def sphere_plate3d(n: int, h_u: float, eps_sphere: float = 2.1, eps_fluid: float = 1.8,
                   pml: int = 16, n_harm: int = 8, margin: int = 2, r_u: float = 0.5,
                   R_u: float = 1.0, plate_u: float = 1.5, dx_u: float = 0.0, **opts) -> Workload:
    """Sphere (radius r) of eps_sphere in a fluid above a PEC plate whose top
    (at z = plate_u) carries a hemispherical indentation of radius R centred
    on the x/y axis.  The cubic cell spans 4.0 units (res = n/4), periodic in
    x/y with PML at both z ends.  h is the gap between the sphere's bottom
    and the bottom of the indentation; dx shifts the sphere along x."""
    res = n / 4.0
    c = n / 2.0
    top = plate_u * res
    zc = (plate_u - R_u + h_u + r_u) * res
    xc = c + dx_u * res
    r = r_u * res
    eps = [eps_fluid, PEC, eps_sphere]
    mu = [1.0, 1.0, 1.0]
    prims = [
        Box((-BIG, -BIG, -BIG), (BIG, BIG, top), 1),
        Sphere((c, c, top), R_u * res, 0),
        Sphere((xc, c, zc), r, 2),
    ]
    ids = rasterize((n, n, n), prims)
    lo = (int(math.floor(xc - r)) - margin, int(math.floor(c - r)) - margin, int(math.floor(zc - r)) - margin)
    hi = (int(math.ceil(xc + r)) + margin, int(math.ceil(c + r)) + margin, int(math.ceil(zc + r)) + margin)
    kw = dict(sigma=1.0, courant=0.5, n_steps=6000, pol="3D", kernel="general", precision="fp32")
    kw.update(opts)
    return Workload(
        name=kw.pop("name", f"sphere_plate_{n}^3_h{h_u:.2f}"), ndim=3, shape=(n, n, n), res=float(res),
        bc=("periodic", "periodic", "pml"), pml_cells=(0, 0, pml), eps=eps, mu=mu, comp_ids=ids,
        s_lo=lo, s_hi=hi, n_harm=int(n_harm), force_axis=2,
        meta=dict(h=h_u, center=(xc, c, zc), r=r),
        **kw,
    )


def c4_sphere_plate(**over) -> Workload:
    """3D FP32: 192^3, res 48, sphere r=0.5 eps 2.1 in fluid eps 1.8 at
    gap 0.45 over an indented PEC plate; 8x8 harmonics; 6000 steps."""
    kw = dict(name="c4_sphere_plate_192^3")
    kw.update(over)
    return sphere_plate3d(192, 0.45, **kw)


def cyl_piston(res: int = 40, h_u: float = 0.5, length_u: float = 10.0, n_harm: int = 3, m_max: int = 2,
               sidewall: str = "pec", margin: int = 2, **opts) -> Workload:
    """Cylindrically symmetric piston (Sec. III C, Fig. 7): the 2D piston's
    blocks rotated about their common axis become two PEC cylinders of
    radius 0.25 and length 1.0, a = 1.0 apart on the axis, inside a tube
    whose wall lies h/2 outside them (the sidewalls joined into a tube).

    Grid (x = z along the axis, y = r): nz = length_u res cells with PEC
    ends; nr = round((0.25 + h/2) res) + 1 cells, the wall at r = nr - 1/2
    cells.  ``sidewall`` "pmc" lines the tube with a two-cell PMC layer
    (mu = -inf).  S: the right cylinder grown by ``margin`` cells, closed on
    the axis.  n_harm cosine harmonics per face, orders m = 0..m_max.
    """
    nz = int(round(length_u * res))
    rb = int(round(0.25 * res))
    nr = int(round((0.25 + 0.5 * h_u) * res)) + 1
    blen = int(round(1.0 * res))
    gap = int(round(1.0 * res))
    left_hi = (nz - gap) // 2
    left_lo = left_hi - blen
    right_lo = left_hi + gap
    right_hi = right_lo + blen
    eps = [1.0, PEC, 1.0]
    mu = [1.0, 1.0, 1.0]
    # grid y = r + 1/2: a cylinder of radius rb cells covers y < rb + 1/2
    prims = [Box((left_lo, -BIG, -BIG), (left_hi, rb + 0.5, BIG), 1),
             Box((right_lo, -BIG, -BIG), (right_hi, rb + 0.5, BIG), 1)]
    if sidewall == "pmc":
        mu[2] = PMC
        prims.insert(0, Box((-BIG, nr - 2.0, -BIG), (BIG, BIG, BIG), 2))
    elif sidewall != "pec":
        raise ValueError(sidewall)
    ids = rasterize((nz, nr, 1), prims)
    if rb + margin >= nr - (2 if sidewall == "pmc" else 0) - 1:
        raise ValueError("clearance too small for the surface margin")
    kw = dict(sigma=1.0, courant=0.5, n_steps=250 * res, pol="3D", kernel="general", precision="fp32")
    kw.update(opts)
    return Workload(
        name=kw.pop("name", f"cyl_piston_{nz}x{nr}_h{h_u:g}"), ndim=2, shape=(nz, nr, 1), res=float(res),
        bc=("pec", "pec", "periodic"), pml_cells=(0, 0, 0), eps=eps, mu=mu, comp_ids=ids,
        s_lo=(right_lo - margin, 0, 0), s_hi=(right_hi + margin, rb + margin, 1), n_harm=int(n_harm),
        force_axis=0, coord="cylindrical", m_max=int(m_max),
        meta=dict(h=float(h_u), tube_radius=(nr - 0.5) / res, cyl_radius=rb / res, sidewall=sidewall,
                  blocks=((left_lo, left_hi), (right_lo, right_hi))),
        **kw,
    )


def c_cyl_piston(**over) -> Workload:
    """Cylindrical piston at resolution 40, h = 0.5, n, m in {0, 1, 2}
    (3 harmonics per face, orders 0..2), 10000 steps, FP64 fields.  The two
    end faces of S carry channel terms of about 5e3 that cancel to the force
    of 2.6e-4; FP32 fields round the part after the mirror symmetry of the
    two ends breaks at about 1e-3 of the force, so FP64 is the default here
    (FP32 stays available with that stated error)."""
    kw = dict(res=40, h_u=0.5, n_harm=3, m_max=2, n_steps=10000, precision="fp64",
              name="cyl_piston_res40_h0.5")
    kw.update(over)
    return cyl_piston(**kw)


def kz_gauss(n: int, k_max: float):
    """Nodes and weights of (1/pi) int_0^k_max dk with n-point Gauss-Legendre
    (the weights include the 1/pi of the force per unit length)."""
    t, w = np.polynomial.legendre.leggauss(int(n))
    return 0.5 * k_max * (t + 1.0), 0.5 * k_max * w / np.pi


def kz_workload(wl: Workload, kz, kz_weight, kx=None) -> Workload:
    """The z-invariant 2D workload wl solved at Bloch wavevectors kz along
    z (six components, general kernel) and, when kx is given, Bloch
    wavevectors along a periodic x; the force is sum_q kz_weight[q] F_q."""
    return wl.replace(coord="kz", kz=tuple(float(k) for k in kz), kz_weight=tuple(float(w) for w in kz_weight),
                      kx=tuple(float(k) for k in kx) if kx is not None else (),
                      pol="3D", kernel="general", name=wl.name + f"_kz{len(kz)}")


def dielectric_piston2d(nx: int, ny: int, slab_px: int, block_w: int, block_h: int, gap: int, block_y0: int,
                        res: float, eps_block: float = 4.0, n_harm: int = 16, **opts) -> Workload:
    """The 2D piston with dielectric blocks (eps_block) instead of PEC ones,
    between PEC sidewall slabs: a z-invariant geometry whose two
    polarizations hybridize at k_z != 0 (Sec. III B)."""
    wl = piston2d(nx, ny, slab_px, block_w, block_h, gap, block_y0, res, n_harm=n_harm, **opts)
    eps = [1.0, PEC, float(eps_block)]
    left, right = wl.meta["blocks"]
    y0, y1 = wl.meta["block_y"]
    prims = [
        Box((-BIG, -BIG, -BIG), (BIG, slab_px, BIG), 1),
        Box((-BIG, ny - slab_px, -BIG), (BIG, BIG, BIG), 1),
        Box((left[0], y0, -BIG), (left[1], y1, BIG), 2),
        Box((right[0], y0, -BIG), (right[1], y1, BIG), 2),
    ]
    ids = rasterize((nx, ny, 1), prims)
    return wl.replace(eps=eps, mu=[1.0, 1.0, 1.0], comp_ids=ids, name=f"dielectric_piston2d_{nx}x{ny}",
                      meta=dict(wl.meta, eps_block=float(eps_block)))


def slabs_open_1d(res: int, a_u: float, d_u: float, pad_u: float, pml_u: float, eps_inf: float,
                  poles=(), margin: int = 2, ny: int = 1, **opts) -> Workload:
    """Two identical dielectric slabs (thickness d_u, permittivity eps_inf
    plus the Lorentz terms ``poles`` = ((d_eps, omega_0), ...)) a vacuum gap
    a_u apart in open space: pad_u of vacuum on either side, then a CPML of
    pml_u along x; translation invariant along y (periodic, ny cells).  S is
    two full-width lines around the right slab, in the vacuum.  The geometry
    of Sec. III B's dispersive example reduced to one dimension (slabs in
    place of the two waveguides)."""
    P = int(round(pml_u * res))
    pad = int(round(pad_u * res))
    d = int(round(d_u * res))
    a = int(round(a_u * res))
    if margin >= a or margin >= pad:
        raise ValueError("the stress surface needs vacuum on both sides of the slab")
    x1 = P + pad                 # left slab [x1, x1 + d)
    x2 = x1 + d + a              # right slab [x2, x2 + d)
    nx = x2 + d + pad + P
    prims = [Box((x1, -BIG, -BIG), (x1 + d, BIG, BIG), 1), Box((x2, -BIG, -BIG), (x2 + d, BIG, BIG), 1)]
    ids = rasterize((nx, ny, 1), prims)
    lor = {1: tuple((float(de), float(w0)) for de, w0 in poles)} if poles else {}
    kw = dict(sigma=1.0, courant=0.5, n_steps=2000, pol="3D", kernel="general", precision="fp64")
    kw.update(opts)
    return Workload(
        name=kw.pop("name", f"slabs_open_{nx}x{ny}"), ndim=2, shape=(nx, ny, 1), res=float(res),
        bc=("pml", "periodic", "periodic"), pml_cells=(P, 0, 0), eps=[1.0, float(eps_inf)], mu=[1.0, 1.0],
        comp_ids=ids, s_lo=(x2 - margin, 0, 0), s_hi=(x2 + d + margin, ny, 1), n_harm=max(1, ny),
        force_axis=0, lorentz=lor, meta=dict(a_px=a, d_px=d, pad_px=pad, pml_px=P, slabs=((x1, x1 + d), (x2, x2 + d))),
        **kw,
    )


def waveguides_open_2d(res: int, w_u: float, t_u: float, gap_u: float, pad_u: float, pml_u: float,
                       eps_inf: float, poles=(), n_harm: int = 8, margin: int = 2, **opts) -> Workload:
    """Sec. III B's dispersive example: two identical dielectric waveguides
    of rectangular cross-section (w_u along x, t_u along y) side by side, a
    vacuum gap gap_u apart along x, in open space (pad_u of vacuum around
    them, then a CPML of pml_u on all four sides).  Permittivity eps_inf plus
    the Lorentz terms ``poles``.  S is the right waveguide grown by
    ``margin`` cells; the force is along x.  Solved as a k_z problem (the
    dielectrics hybridize the two polarizations)."""
    P = int(round(pml_u * res))
    pad = int(round(pad_u * res))
    w = int(round(w_u * res))
    t = int(round(t_u * res))
    gap = int(round(gap_u * res))
    if 2 * margin >= gap or margin >= pad:
        raise ValueError("the stress surface needs vacuum around the waveguide")
    x1 = P + pad
    x2 = x1 + w + gap
    nx = x2 + w + pad + P
    y0 = P + pad
    ny = y0 + t + pad + P
    prims = [Box((x1, y0, -BIG), (x1 + w, y0 + t, BIG), 1), Box((x2, y0, -BIG), (x2 + w, y0 + t, BIG), 1)]
    ids = rasterize((nx, ny, 1), prims)
    lor = {1: tuple((float(de), float(w0)) for de, w0 in poles)} if poles else {}
    kw = dict(sigma=1.0, courant=0.5, n_steps=2000, pol="3D", kernel="general", precision="fp64")
    kw.update(opts)
    return Workload(
        name=kw.pop("name", f"waveguides_open_{nx}x{ny}"), ndim=2, shape=(nx, ny, 1), res=float(res),
        bc=("pml", "pml", "periodic"), pml_cells=(P, P, 0), eps=[1.0, float(eps_inf)], mu=[1.0, 1.0],
        comp_ids=ids, s_lo=(x2 - margin, y0 - margin, 0), s_hi=(x2 + w + margin, y0 + t + margin, 1),
        n_harm=int(n_harm), force_axis=0, lorentz=lor,
        meta=dict(guides=((x1, x1 + w), (x2, x2 + w)), guide_y=(y0, y0 + t), pml_px=P),
        **kw,
    )


def small_cases():
    """Small workloads the oracle finishes in seconds (parity test sizes)."""
    return {
        "piston_tm_small": piston2d_units(10, 4.0, 2.0, 0.6, pol="TM", n_steps=300, n_harm=6,
                                          name="piston_tm_small"),
        "piston_te_small": piston2d_units(10, 4.0, 2.0, 0.6, pol="TE", n_steps=300, n_harm=6,
                                          name="piston_te_small"),
    }


def stop_piston2d(**over) -> Workload:
    """Small TE+TM piston whose partial force settles well inside its 3000
    steps: the workload of the time-convergence stop checks."""
    kw = dict(pol="TM+TE", n_steps=3000, n_harm=8, name="stop_piston_40x31")
    kw.update(over)
    return piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, **kw)


def stop_sphere3d(**over) -> Workload:
    """3D sphere of eps 3 in fluid eps 1.8 above a PEC plate, z CPML (12 x 12
    x 26 cells, 1500 steps): the 3D workload of the convergence stop checks."""
    nx, ny, nz, pml = 12, 12, 26, 4
    zlo = pml + 2
    prims = [Box((-BIG, -BIG, -BIG), (BIG, BIG, zlo), 1), Sphere((nx / 2 + 0.3, ny / 2, zlo + 5.5), 1.7, 2)]
    kw = dict(sigma=1.0, courant=0.5, n_steps=1500, pol="3D", kernel="general", precision="fp64")
    kw.update(over)
    return Workload(name=kw.pop("name", "stop_sphere_12x12x26"), ndim=3, shape=(nx, ny, nz), res=4.0,
                    bc=("periodic", "periodic", "pml"), pml_cells=(0, 0, pml), eps=[1.8, PEC, 3.0],
                    mu=[1.0, 1.0, 1.0], comp_ids=rasterize((nx, ny, nz), prims),
                    s_lo=(nx // 2 - 3, ny // 2 - 3, zlo + 2), s_hi=(nx // 2 + 4, ny // 2 + 3, zlo + 9),
                    n_harm=2, force_axis=2, **kw)


def layered_plates_1d(res: int, a_u: float, d_u: float, b_u: float, layer_u: float, eps_inf: float,
                      poles=(), margin: int = 2, ny: int = 1, **opts) -> Workload:
    """parallel_plates_1d with a dielectric layer of thickness layer_u on the
    left wall (permittivity eps_inf plus the Lorentz terms ``poles`` =
    ((d_eps, omega_0), ...)); the vacuum gap between the layer and the PEC
    slab is a_u - layer_u, S lies in the vacuum gaps."""
    wl = parallel_plates_1d(res, a_u, d_u, b_u, margin=margin, ny=ny, **opts)
    L = int(round(layer_u * res))
    if L + margin >= int(round(a_u * res)):
        raise ValueError("the layer reaches the stress surface")
    nx = wl.shape[0]
    prims = [Box((-BIG, -BIG, -BIG), (L, BIG, BIG), 2),
             Box((wl.meta["a_px"], -BIG, -BIG), (wl.meta["a_px"] + wl.meta["d_px"], BIG, BIG), 1)]
    ids = rasterize((nx, ny, 1), prims)
    lor = {2: tuple((float(de), float(w0)) for de, w0 in poles)} if poles else {}
    return wl.replace(eps=[1.0, PEC, float(eps_inf)], mu=[1.0, 1.0, 1.0], comp_ids=ids, lorentz=lor,
                      name=f"layered_plates_{nx}x{ny}", meta=dict(wl.meta, layer_px=L))


def stop_cyl(**over) -> Workload:
    """Cylindrical piston at resolution 10 (tube 15 units, orders m = 0..2,
    3 harmonics per face, 2000 base steps, FP64): the cylindrical workload of
    the convergence stop checks."""
    kw = dict(res=10, h_u=0.8, length_u=15.0, n_harm=3, m_max=2, n_steps=2000, precision="fp64",
              name="stop_cyl_piston_res10")
    kw.update(over)
    return cyl_piston(**kw)


def stop_kz(**over) -> Workload:
    """The dielectric piston (eps 4 blocks, 40 x 31) at three k_z points,
    2000 steps, FP64: the k_z workload of the convergence stop checks."""
    kw = dict(n_steps=2000, n_harm=6, precision="fp64")
    kw.update(over)
    base = dielectric_piston2d(40, 31, 4, 10, 5, 10, 13, 10.0, **kw)
    return kz_workload(base, [0.0, 0.8, 2.5], [0.3, 0.5, 0.25]).replace(name="stop_kz_dielectric_piston")

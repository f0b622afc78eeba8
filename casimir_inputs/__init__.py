"""Seeded, synthetic inputs for the time-domain Casimir FDTD path.

This package builds the *inputs* that both the CPU oracle and the HIP library
consume: per-Yee-component material-id grids rasterized from simple geometric
primitives, the material table, the stress-tensor surface box and the run
options.  It contains none of the method's arithmetic (no update
coefficients, no kernels, no bases, no force formulas), so the oracle and the
library can share it without sharing any of the computation under test.

The paper (Sec. III) runs its examples on generated geometry only; there is
no public dataset, so every workload here is synthetic and fully determined
by its parameters (the serving stream in ``streams`` is seeded).
"""
from .geometry import (
    COMPONENTS,
    COMPONENT_OFFSETS2,
    Box,
    Sphere,
    Workload,
    rasterize,
    PEC,
    PMC,
)
from .configs import (
    piston2d,
    parallel_plates_1d,
    sphere_plate3d,
    c1_piston_tm_fp64,
    c2_piston_tetm_fp32,
    c3_uneven_set,
    c4_sphere_plate,
    cyl_piston,
    c_cyl_piston,
    dielectric_piston2d,
    slabs_open_1d,
    waveguides_open_2d,
    kz_workload,
    kz_gauss,
    small_cases,
)

__all__ = [
    "COMPONENTS",
    "COMPONENT_OFFSETS2",
    "Box",
    "Sphere",
    "Workload",
    "rasterize",
    "PEC",
    "PMC",
    "piston2d",
    "parallel_plates_1d",
    "sphere_plate3d",
    "c1_piston_tm_fp64",
    "c2_piston_tetm_fp32",
    "c3_uneven_set",
    "c4_sphere_plate",
    "cyl_piston",
    "c_cyl_piston",
    "dielectric_piston2d",
    "slabs_open_1d",
    "waveguides_open_2d",
    "kz_workload",
    "kz_gauss",
    "small_cases",
]

"""FP64 CPU oracle for the time-domain Casimir FDTD method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
HIP library never calls, links or imports this package, and this package
never imports the library: the two share nothing but the seeded input
builders in ``casimir_inputs``.

The oracle follows the paper's algorithm step by step (McCauley, Rodriguez,
Joannopoulos, Johnson, "Casimir forces in the time domain: Applications"):

* ``kernels``  the time kernel K(t) = 2*pi*Im g(-t) (Appendix A, the g(xi)
  equation and its analytic pieces; Appendix A.2 for z-invariant perfect
  conductors),
* ``surface``  the stress surface S, its per-face cosine basis (Sec. III,
  the f_n(x) equation) and the stress-tensor channel table (Sec. II, the
  Gamma^E_i definition),
* ``yee``      the Yee leapfrog with the uniform conductivity sigma (Sec. II),
  PEC/PMC/epsilon/mu maps, periodic walls and a CPML,
* ``force``    one simulation per harmonic source and the time integral
  against K (Sec. II, eq. time-force; the harmonic sum of Sec. II).

Parity status of each function is listed in its docstring; every function is
pinned by a CPU test under ``tests/`` against closed forms, invariants or
brute force (see the pin list in the tests' module docstrings).
"""
from .kernels import kernel_general, kernel_zinv2d, kernel_table
from .surface import Face, build_faces, face_basis, gather, channel_table
from .yee import YeeSim
from .force import solve, run_gammas, OracleResult

__all__ = [
    "kernel_general",
    "kernel_zinv2d",
    "kernel_table",
    "Face",
    "build_faces",
    "face_basis",
    "gather",
    "channel_table",
    "YeeSim",
    "solve",
    "run_gammas",
    "OracleResult",
]

"""Write oracle results used as stored expected values by the GPU tests.

Calls only the CPU oracle (oracle/) on the synthetic workloads of
casimir_inputs; no value comes from the HIP library.

    python tests/golden/make_golden.py c2      # 2D TE+TM piston, 400x200, T=10000
    python tests/golden/make_golden.py c1      # 2D TM piston, 80x40, T=2000
    python tests/golden/make_golden.py c4s     # 3D sphere-plate 192^3: 5 channels, 24 steps
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from casimir_inputs import c1_piston_tm_fp64, c2_piston_tetm_fp32, c4_sphere_plate  # noqa: E402

CASES = {
    "c1": ("c1_piston_tm_oracle.json", c1_piston_tm_fp64),
    "c2": ("c2_piston_tetm_oracle.json", c2_piston_tetm_fp32),
}
# 3D sample: channels on x-, z-lo and z-hi faces, E and H kinds, several harmonics
C4_SUBSET = [1, 512, 571, 898, 1279]
C4_STEPS = 24


def c4_sample(workers=5):
    wl = c4_sphere_plate()
    t0 = time.time()
    r = oracle.solve(wl, n_steps=C4_STEPS, channel_subset=C4_SUBSET, workers=workers, chunk=1,
                     keep_gamma=True)
    out = dict(workload=wl.name, shape=list(wl.shape), n_steps=C4_STEPS, subset=C4_SUBSET,
               gamma=[[float(v) for v in row] for row in r.gamma],
               per_channel=[float(v) for v in r.acc], sign=[float(v) for v in r.sign],
               oracle_seconds=time.time() - t0,
               source="oracle.solve (FP64 NumPy), written by tests/golden/make_golden.py")
    with open(os.path.join(HERE, "c4_sphere_plate_sample_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("c4s", f"{time.time() - t0:.1f}s")


def main(which, workers=8):
    fname, make = CASES[which]
    wl = make()
    t0 = time.time()
    r = oracle.solve(wl, workers=workers, chunk=16)
    out = dict(
        workload=wl.name, shape=list(wl.shape), n_steps=wl.n_steps, sigma=wl.sigma,
        courant=wl.courant, kernel=wl.kernel, pol=wl.pol, n_harm=wl.n_harm,
        force=r.force,
        per_channel=[float(v) for v in r.acc],
        sign=[float(v) for v in r.sign],
        per_harmonic={str(k): v for k, v in sorted(r.per_harmonic.items())},
        per_face={str(k): v for k, v in sorted(r.per_face.items())},
        oracle_seconds=time.time() - t0,
        workers=workers,
        source="oracle.solve (FP64 NumPy), written by tests/golden/make_golden.py",
    )
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    print(which, r.force, f"{time.time() - t0:.1f}s")


if __name__ == "__main__":
    if sys.argv[1] == "c4s":
        c4_sample()
    else:
        main(sys.argv[1])

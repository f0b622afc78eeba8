"""Write oracle results used as stored expected values by the GPU tests.

Calls only the CPU oracle (oracle/) on the synthetic workloads of
casimir_inputs; no value comes from the HIP library.

    python tests/golden/make_golden.py c2      # 2D TE+TM piston, 400x200, T=10000
    python tests/golden/make_golden.py c1      # 2D TM piston, 80x40, T=2000
    python tests/golden/make_golden.py c4s     # 3D sphere-plate 192^3: 5 channels, 24 steps
    python tests/golden/make_golden.py c4f     # the same 5 channels over the full T = 6000
    python tests/golden/make_golden.py c3      # uneven piston set: members 0 and 23, full T
    python tests/golden/make_golden.py cyl     # cylindrical piston res 40, n, m in {0, 1, 2}, full T
    python tests/golden/make_golden.py kz      # k_z dielectric piston, 8 k points, full T
    python tests/golden/make_golden.py stop    # partial-force traces of the convergence-stop workloads
    python tests/golden/make_golden.py stop_reduced  # the same for a cylindrical and a k_z workload
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from casimir_inputs import c1_piston_tm_fp64, c2_piston_tetm_fp32, c3_uneven_set, c4_sphere_plate  # noqa: E402

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


def c4_full(workers=5):
    """The C4 sample channels integrated over the configuration's full T:
    the FP64 reference for the 3D FP32 error (channel integrals, not a
    force: the other 1275 channels are beyond the oracle's reach)."""
    wl = c4_sphere_plate()
    t0 = time.time()
    r = oracle.solve(wl, channel_subset=C4_SUBSET, workers=workers, chunk=1)
    out = dict(workload=wl.name, shape=list(wl.shape), n_steps=wl.n_steps, subset=C4_SUBSET,
               per_channel=[float(v) for v in r.acc], sign=[float(v) for v in r.sign],
               oracle_seconds=time.time() - t0,
               source="oracle.solve (FP64 NumPy), written by tests/golden/make_golden.py")
    with open(os.path.join(HERE, "c4_sphere_plate_channels_full_T_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("c4f", f"{time.time() - t0:.1f}s")


C3_MEMBERS = [0, 23]


def c3_members(workers=8):
    """Members 0 (h = 0.1, 400 x 84) and 23 (h = 2.0, 400 x 160) of the
    uneven piston set, full T = 10000."""
    wls = c3_uneven_set()
    t0 = time.time()
    members = []
    for k in C3_MEMBERS:
        wl = wls[k]
        r = oracle.solve(wl, workers=workers, chunk=16)
        members.append(dict(index=k, h=wl.meta["h"], workload=wl.name, shape=list(wl.shape), force=r.force,
                            per_channel=[float(v) for v in r.acc]))
        print("c3 member", k, r.force, f"{time.time() - t0:.1f}s", flush=True)
    out = dict(n_steps=wls[0].n_steps, members=members, oracle_seconds=time.time() - t0,
               source="oracle.solve (FP64 NumPy), written by tests/golden/make_golden.py")
    with open(os.path.join(HERE, "c3_uneven_members_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


def cyl_piston_golden():
    """The cylindrical piston force point of the benchmark (FP64 oracle,
    every order and channel over its full step count)."""
    from casimir_inputs import c_cyl_piston
    from oracle import cylforce
    wl = c_cyl_piston()
    t0 = time.time()
    r = cylforce.solve(wl, m_max=wl.m_max)
    out = dict(workload=wl.name, shape=list(wl.shape), n_steps=wl.n_steps, m_max=wl.m_max, n_harm=wl.n_harm,
               force=r.force, per_m={str(k): v for k, v in r.per_m.items()}, n_steps_m=r.n_steps_m,
               per_channel=[float(v) for v in r.acc.reshape(-1)], oracle_seconds=time.time() - t0,
               source="oracle.cylforce.solve (FP64 NumPy), written by tests/golden/make_golden.py")
    with open(os.path.join(HERE, "cyl_piston_res40_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("cyl", r.force, f"{time.time() - t0:.1f}s")


def kz_golden():
    """The k_z dielectric piston of the benchmark (FP64 oracle, 8 k points)."""
    from casimir_inputs import dielectric_piston2d, kz_gauss, kz_workload
    from oracle import kz
    base = dielectric_piston2d(80, 40, 10, 20, 10, 20, 15, 20.0, n_steps=2000, n_harm=16)
    ks, ws = kz_gauss(8, 12.0)
    wl = kz_workload(base, ks, ws)
    t0 = time.time()
    r = kz.solve(wl, ks, ws)
    out = dict(workload=wl.name, shape=list(wl.shape), n_steps=wl.n_steps, kz=list(ks), kz_weight=list(ws),
               force=r.force, per_k=r.per_k, per_channel=[float(v) for v in r.acc.reshape(-1)],
               oracle_seconds=time.time() - t0,
               source="oracle.kz.solve (FP64 NumPy), written by tests/golden/make_golden.py")
    with open(os.path.join(HERE, "kz_dielectric_piston_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("kz", r.force, f"{time.time() - t0:.1f}s")


def stop_traces(workers=8):
    """The partial force F(T') after every step (the trace of Fig. 12) of the
    two convergence-stop workloads: the reference the GPU's stop rule is
    checked against."""
    from casimir_inputs.configs import stop_piston2d, stop_sphere3d
    out = {"source": "oracle.solve (FP64 NumPy), written by tests/golden/make_golden.py"}
    for key, wl in (("piston2d", stop_piston2d()), ("sphere3d", stop_sphere3d())):
        t0 = time.time()
        r = oracle.solve(wl, workers=workers, chunk=8)
        out[key] = dict(workload=wl.name, shape=list(wl.shape), n_steps=wl.n_steps, force=r.force,
                        terms=float(sum(abs(s * a) for s, a in zip(r.sign, r.acc)) / 3.141592653589793),
                        trace=[float(v) for v in r.trace], oracle_seconds=time.time() - t0)
        print(key, r.force, f"{time.time() - t0:.1f}s")
    with open(os.path.join(HERE, "stop_traces_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


def stop_traces_reduced():
    """Partial-force traces of the cylindrical and k_z convergence-stop
    workloads (the cylindrical trace on the axis of the base steps: order m
    at floor(d T_m / n_steps) of its own steps)."""
    from casimir_inputs.configs import stop_cyl, stop_kz
    from oracle import cylforce, kz
    out = {"source": "oracle.cylforce.solve / oracle.kz.solve (FP64 NumPy), written by tests/golden/make_golden.py"}
    t0 = time.time()
    wl = stop_cyl()
    r = cylforce.solve(wl, m_max=wl.m_max)
    terms = sum(float(np.sum(np.abs(r.sign * r.acc[m]))) * (1.0 if m == 0 else 2.0)
                for m in range(wl.m_max + 1)) / np.pi
    out["cyl"] = dict(workload=wl.name, shape=list(wl.shape), n_steps=wl.n_steps, n_steps_m=list(r.n_steps_m),
                      force=r.force, terms=terms, trace=[float(v) for v in r.trace], oracle_seconds=time.time() - t0)
    print("cyl", r.force, f"{time.time() - t0:.1f}s")
    t0 = time.time()
    wl = stop_kz()
    r = kz.solve(wl, wl.kz, wl.kz_weight)
    terms = sum(abs(w) * float(np.sum(np.abs(r.sign * r.acc[q]))) for q, w in enumerate(wl.kz_weight)) / np.pi
    out["kz"] = dict(workload=wl.name, shape=list(wl.shape), n_steps=wl.n_steps, force=r.force, terms=terms,
                     trace=[float(v) for v in r.trace], oracle_seconds=time.time() - t0)
    print("kz", r.force, f"{time.time() - t0:.1f}s")
    with open(os.path.join(HERE, "stop_traces_reduced_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


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
    elif sys.argv[1] == "c4f":
        c4_full()
    elif sys.argv[1] == "c3":
        c3_members()
    elif sys.argv[1] == "cyl":
        cyl_piston_golden()
    elif sys.argv[1] == "kz":
        kz_golden()
    elif sys.argv[1] == "stop":
        stop_traces()
    elif sys.argv[1] == "stop_reduced":
        stop_traces_reduced()
    else:
        main(sys.argv[1])

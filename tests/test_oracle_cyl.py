"""Pins of the cylindrical (r, z) oracle (one azimuthal order m per run).

* Exact discrete energy conservation at sigma = 0 for m = 0..4 (random
  fields, PEC tube, PEC or periodic ends) with the r-weights of the cells.
* The spectrum of the discrete update operator in a closed PEC cylinder
  against the cavity modes omega^2 = (x/R)^2 + (p pi/L)^2, x the zeros of J_m
  (TM, p >= 0) and of J_m' (TE, p >= 1), at second order in the cell size.
* The stability limit: growth for m = 2 at Courant 0.5 and none at the
  Courant number the solver uses.
* Mirror-symmetric geometry (plate midway in a closed tube) has zero force.
* A complete basis on the faces gives the one-source-per-sample sum.
* The piston in a PEC tube (plates filling the cross-section): per order m
  the force converges towards the waveguide mode sum
  F_m = w_m sum_modes [F_1(a, k) - F_1(b, k)],  F_1(a, k) = -(1/pi) int_0^inf
  dxi kappa / (exp(2 a kappa) - 1),  kappa = sqrt(xi^2 + k^2), k = x/R;
  with S meeting the tube wall the discrete stress cancels only slowly, so
  this is a convergence pin with a complete radial basis (no truncation
  error): the error falls by > 3.5x from 20 to 40 cells per unit (second
  order: 4x) and is below 15 % at 40 (measured: m = 0 58 % -> 12 %,
  m = 1 27 % -> 6 %).
* The tube's ends are immaterial: the piston's force with PEC end caps 3.5
  units beyond each cylinder equals the force with caps 5.5 units beyond to
  a relative 1e-6 (the tube is a waveguide below cutoff on the imaginary
  frequency contour, so the fields decay exponentially along the axis; the
  paper terminates its tube with PML for the same purpose, Sec. III C).
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import jn_zeros, jnp_zeros
from threadpoolctl import threadpool_limits

from casimir_inputs.geometry import Box, Workload, rasterize
from oracle import cylforce
from oracle.cyl import CylSim, cylindrical_courant

BIG = 1e30
COMPS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def empty(nz, nr, res, bc_z="pec", **kw):
    ids = {c: np.zeros((1, nr, nz), np.uint8) for c in COMPS}
    o = dict(name="cyl", ndim=2, shape=(nz, nr, 1), res=float(res), bc=(bc_z, "pec", "periodic"),
             pml_cells=(0, 0, 0), eps=[1.0], mu=[1.0], comp_ids=ids, s_lo=(1, 0, 0), s_hi=(3, 2, 1), n_harm=2,
             force_axis=0, pol="3D", kernel="general", n_steps=10, sigma=0.0)
    o.update(kw)
    return Workload(**o)


@pytest.mark.parametrize("bc_z", ["pec", "periodic"])
@pytest.mark.parametrize("m", [0, 1, 2, 3, 4])
def test_energy_conserved_exactly(m, bc_z):
    wl = empty(14, 9, 4.0, bc_z)
    S = CylSim(wl, "E", 1, m, cylindrical_courant(0.5, m))
    rng = np.random.default_rng(10 + m)
    for c in COMPS:
        S.F[c] = rng.standard_normal(S.F[c].shape) * (S.b[c] != 0)
    if m != 0:
        S.F["Hx"][:, 0, :] = 0.0
    S.axis_copy()
    w = S.weights()
    U = []
    for _ in range(600):
        ue = sum((w[c] * S.F[c] ** 2).sum() for c in ("Ex", "Ey", "Ez"))
        hp = {c: S.F[c].copy() for c in ("Hx", "Hy", "Hz")}
        S.step_h()
        U.append(ue + sum((w[c] * hp[c] * S.F[c]).sum() for c in ("Hx", "Hy", "Hz")))
        S.step_e()
    U = np.array(U)
    assert np.max(np.abs(U / U[0] - 1)) < 1e-12
    assert max(np.abs(S.F[c]).max() for c in COMPS) < 50


def test_courant_limit():
    wl = empty(16, 10, 4.0, "periodic")

    def grows(m, c):
        S = CylSim(wl, "E", 1, m, c)
        rng = np.random.default_rng(3)
        for k in COMPS:
            S.F[k] = rng.standard_normal(S.F[k].shape) * (S.b[k] != 0)
        if m != 0:
            S.F["Hx"][:, 0, :] = 0.0
        with np.errstate(all="ignore"):
            for _ in range(2000):
                S.step()
        return not max(np.abs(S.F[k]).max() for k in COMPS) < 100
    assert grows(2, 0.5)
    for m in range(5):
        assert not grows(m, cylindrical_courant(0.5, m))


def operator_frequencies(res, m):
    """Angular frequencies of the semi-discrete update (E -> curl -> H -> curl
    -> E) in a closed PEC cylinder of Rc = res cells (wall at Rc - 1/2) and
    length 1.5 res cells."""
    nr, nz = res, int(1.5 * res)
    wl = empty(nz, nr, res)
    N = 3 * nr * nz
    S = CylSim(wl, "E", N, m, 0.5)
    k = 0
    for c in ("Ex", "Ey", "Ez"):
        F = S.F[c].reshape(N, -1)
        for j in range(nr * nz):
            F[k, j] = 1.0
            k += 1
    ce = S.curl_e()
    ce["Hz"][:, 0, :] = 0.0
    if m != 0:
        ce["Hx"][:, 0, :] = 0.0
    for c in ("Hx", "Hy", "Hz"):
        S.F[c] = -1.0 * (S.b[c] != 0) * ce[c]
    for c in ("Ex", "Ey", "Ez"):
        S.F[c][:] = 0.0
    ch = S.curl_h()
    ch["Ey"][:, 0, :] = 0.0
    M = np.concatenate([(1.0 * (S.b[c] != 0) * ch[c]).reshape(N, -1) for c in ("Ex", "Ey", "Ez")], axis=1)
    with threadpool_limits(1):          # a threaded dense eigensolve is many times slower here
        lam = np.sort(np.real(np.linalg.eigvals(-M.T))) * res * res
    lam = lam[lam > 1e-6]
    return np.sqrt(lam), (nr - 0.5) / res, nz / res


def cavity_modes(m, R, L):
    out = [np.hypot(x / R, p * np.pi / L) for x in jn_zeros(m, 6) for p in range(6)]
    out += [np.hypot(x / R, p * np.pi / L) for x in jnp_zeros(m, 6) for p in range(1, 6)]
    return np.sort(out)


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_cavity_spectrum_second_order(m):
    errs = []
    for res in (10, 20):
        w, R, L = operator_frequencies(res, m)
        ex = cavity_modes(m, R, L)[:6]
        errs.append(np.max(np.abs(w[:6] / ex - 1)))
    assert errs[1] < 4e-3
    assert errs[0] / errs[1] > 3.3          # second order: 4 x per halving


def F1(a, k):
    f = lambda xi: np.sqrt(xi * xi + k * k) / np.expm1(min(2 * a * np.sqrt(xi * xi + k * k), 700.0))
    return -quad(f, 0, np.inf, limit=200)[0] / np.pi


def mode_sum(m, R, a, b):
    tot = 0.0
    for x in list(jn_zeros(m, 30)) + list(jnp_zeros(m, 30)):
        k = x / R
        if 2 * min(a, b) * k < 60:
            tot += F1(a, k) - F1(b, k)
    return (1.0 if m == 0 else 2.0) * tot


def piston(res, a_u=0.5, d_u=0.25, b_u=1.0, r_u=0.5, n_harm=1000, gap_frac=0.5, T_u=12.0):
    na, nd, nb = int(round(a_u * res)), int(round(d_u * res)), int(round(b_u * res))
    nz, nr = na + nd + nb, int(round(r_u * res))
    ids = rasterize((nz, nr, 1), [Box((na, -BIG, -BIG), (na + nd, BIG, BIG), 1)])
    g = int(round(gap_frac * na))
    wl = Workload(name="cylpiston", ndim=2, shape=(nz, nr, 1), res=float(res), bc=("pec", "pec", "periodic"),
                  pml_cells=(0, 0, 0), eps=[1.0, float("-inf")], mu=[1.0, 1.0], comp_ids=ids,
                  s_lo=(na - g, 0, 0), s_hi=(na + nd + g, nr, 1), n_harm=n_harm, force_axis=0, pol="3D",
                  kernel="general", n_steps=int(T_u * res / 0.5), sigma=1.0, courant=0.5)
    return wl, (nr - 0.5) / res, na / res, nb / res


def test_mirror_symmetric_plate_has_zero_force():
    res = 10
    na, nd = 6, 3
    nz, nr = 2 * na + nd, 5
    ids = rasterize((nz, nr, 1), [Box((na, -BIG, -BIG), (na + nd, BIG, BIG), 1)])
    wl = Workload(name="sym", ndim=2, shape=(nz, nr, 1), res=float(res), bc=("pec", "pec", "periodic"),
                  pml_cells=(0, 0, 0), eps=[1.0, float("-inf")], mu=[1.0, 1.0], comp_ids=ids,
                  s_lo=(na - 3, 0, 0), s_hi=(na + nd + 3, nr, 1), n_harm=3, force_axis=0, pol="3D",
                  kernel="general", n_steps=200, sigma=1.0, courant=0.5)
    r = cylforce.solve(wl, m_max=2)
    scale = np.sum(np.abs(r.sign[None, :] * r.acc)) / np.pi
    assert abs(r.force) < 1e-11 * scale
    assert all(abs(v) < 1e-11 * scale for v in r.per_m.values())


def test_complete_basis_equals_point_sources():
    """With as many harmonics as samples the weighted basis is complete: the
    harmonic sum equals the sum over single-sample sources (each sample's
    source is the weighted delta w_s e_s / (dx w_s))."""
    wl, R, a, b = piston(10)
    wl = wl.replace(n_steps=60)
    r = cylforce.solve(wl, m_max=1)
    faces, bases, eps_s, mu_s, chans = cylforce.setup(wl)
    # point basis: rows[s] = w_s * (e_s / sqrt(dx w_s))
    dx = 1.0 / wl.res
    pt = {}
    for fi, f in enumerate(faces):
        rows = np.array([f.weights * (np.eye(len(f.weights))[s] / np.sqrt(dx * f.weights[s]))
                         for s in range(len(f.weights))])
        pt[fi] = (rows, list(range(len(f.weights))))
    chans_pt = []
    for fi, f in enumerate(faces):
        for row in range(len(f.weights)):
            for kind, j, q, coef in cylforce.channel_specs("3D", f.axis, 0, eps_s, mu_s):
                chans_pt.append(dict(face=fi, row=row, label=row, kind=kind, src=kind + j, meas=kind + q,
                                     sign=float(f.side) * coef))
    tot = 0.0
    for m in range(2):
        cm = cylindrical_courant(wl.courant, m)
        T = r.n_steps_m[m]
        gam, dt = cylforce.run_order(wl, m, faces, pt, eps_s, mu_s, chans_pt, T, cm)
        K = cylforce.kernel_table(wl.kernel, wl.sigma, dt, T)
        acc = (dt * K[:, None] * gam).sum(axis=0)
        sign = np.array([c["sign"] for c in chans_pt])
        tot += (1.0 if m == 0 else 2.0) * np.sum(sign * acc) / np.pi
    assert tot == pytest.approx(r.force, rel=1e-9, abs=1e-12)


def test_piston_converges_to_mode_sum():
    """Complete radial basis (no truncation): the per-order force (m = 0, 1)
    against the waveguide mode sum at 20 and 40 cells per unit (gap 0.5, tube
    radius 0.475, plate 0.25, far side 1.0)."""
    errs = {0: [], 1: []}
    for res in (20, 40):
        wl, R, a, b = piston(res)
        full = cylforce.solve(wl, m_max=1)
        for m in (0, 1):
            errs[m].append(full.per_m[m] / mode_sum(m, R, a, b) - 1)
    print("relative error per order at 20 / 40 cells per unit:", errs)
    for m in (0, 1):
        assert abs(errs[m][1]) < 0.15
        assert abs(errs[m][0]) / abs(errs[m][1]) > 3.5


def test_tube_end_caps_are_immaterial():
    """cyl_piston at res 10, T = 2500: tube lengths 10 (the benchmark's
    3.5 units of tube beyond each cylinder) and 14 give the same force to
    1e-6 relative, and length 8 (2.5 units) already to 1e-3."""
    from casimir_inputs import cyl_piston
    with threadpool_limits(limits=1):
        f = {L: cylforce.solve(w, m_max=w.m_max).force
             for L, w in ((L, cyl_piston(res=10, h_u=0.5, length_u=L, n_harm=3, m_max=2, n_steps=2500,
                                         precision="fp64")) for L in (8.0, 10.0, 14.0))}
    assert abs(f[10.0] / f[14.0] - 1) < 1e-6
    assert 1e-6 < abs(f[8.0] / f[14.0] - 1) < 1e-3


def _pulse(nz, bc_z, P, m, steps, nr=12):
    wl = empty(nz, nr, 10.0, bc_z, pml_cells=(P, 0, 0))
    S = CylSim(wl, "E", 1, m, cylindrical_courant(0.5, m))
    J, I = np.meshgrid(np.arange(nr), np.arange(nz), indexing="ij")
    g = np.exp(-((I - nz / 2) ** 2) / 6.0 - ((J - 3) ** 2) / 4.0)
    S.F["Ez"][0] = g * (S.b["Ez"] != 0)
    S.F["Ex"][0] = 0.5 * np.roll(g, 2, axis=1) * (S.b["Ex"] != 0)
    S.start()
    for _ in range(steps):
        S.step()
    return S


@pytest.mark.parametrize("m", [0, 1, 2])
def test_pml_tube_ends_match_a_long_tube(m):
    """Open tube ends (Sec. III C): a pulse in e_phi and e_z in a tube of 64
    cells with 12-cell CPML ends matches, in the tube's interior after 140
    steps, the same pulse in a tube three times as long with PEC ends (which
    stands for the infinite tube until its ends' echo returns) to 5e-4 of
    the field; with PEC ends in place of the layers the echo is of the
    order of the field itself for m = 0 and 1."""
    n, P, steps = 64, 12, 140
    big = _pulse(3 * n, "pec", 0, m, steps)
    c0, c1 = P + 2, n - P - 2

    def mismatch(S):
        num = den = 0.0
        for c in COMPS:
            a = S.F[c][0][:, c0:c1]
            b = big.F[c][0][:, n + c0:n + c1]
            num += float(np.sum((a - b) ** 2))
            den += float(np.sum(b ** 2))
        return np.sqrt(num / den)

    assert mismatch(_pulse(n, "pml", P, m, steps)) < 5e-4
    if m < 2:
        assert mismatch(_pulse(n, "pec", 0, m, steps)) > 0.3

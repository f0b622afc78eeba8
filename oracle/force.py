"""One FDTD run per harmonic source and the time integral that gives the force.

Sec. II of the paper: for every basis function f_n on S, a current
J = delta(t) f_n e_j on S is applied and the field response on S is recorded;
the n-sums of the responses give Gamma_i(t), which is integrated against
g(-t).  Here, per channel c = (face, n, kind, j, q, sign):

  source   the delta(t) current is an initial condition.  With Ampere's law
           eps dE/dt = curl H - sigma eps E - J (the sign convention under
           which g(xi) is the weight of the response), an E-kind channel
           starts from E_j^0 = -(W^T f_n) / (dx eps_S), an H-kind channel
           from H_j^0 = -(W^T f_n) / (dx mu_S); the staggered partner field
           is then set half a step away (YeeSim.start).
  record   after leapfrog step m (H then E) the channel's sample sits m dt
           after its own kick:  Gamma_c(t_m) = dx^{d-1} sum_i f_n(s_i)
           (W X_q)_i  (X_q = E_q^m, or H_q^m of the dual H-kind run).
  force    F = (1/pi) sum_c sign_c sum_{m=1..T} dt K(t_m) Gamma_c(t_m),
           K = 2 pi Im g(-t) (rectangle rule at t_m, m >= 1; the paper does
           not give its quadrature).

The prefactor: the paper's force equation carries hbar/pi with Im g, while
its Appendix A writes g(-t) with a 1/(2 pi); taken literally together they
would give 1/(2 pi) of the stress-tensor force.  The consistent reading
(fluctuation-dissipation with the contour of Sec. II) is (1/pi) with
K = 2 pi Im g(-t); the parallel-plate pins fix it.

Outputs: F, the per-harmonic contributions P_n (Fig. 5), the per-face
contributions, the per-channel integrals and the partial-sum trace F(T')
(Fig. 12).

Parity: pinned (tests/test_oracle_force.py).
"""
from __future__ import annotations

import dataclasses
import multiprocessing as mp
from collections import defaultdict
from typing import Dict, List, Optional

import numpy as np

from .kernels import kernel_table
from .surface import (POL_COMPONENTS, Channel, build_faces, channel_table, face_basis,
                      gather)
from .yee import YeeSim


@dataclasses.dataclass
class OracleResult:
    force: float
    per_harmonic: Dict[int, float]
    per_face: Dict[int, float]
    acc: np.ndarray            # per channel: sum_m dt K(t_m) Gamma_c(t_m)
    sign: np.ndarray           # per channel sign
    gamma: Optional[np.ndarray]  # (T, C) when requested
    trace: np.ndarray          # F(T') for T' = 1..T
    channels: List[Channel]
    faces: list
    eps_s: float
    mu_s: float


def surface_medium(wl, faces):
    """(eps_S, mu_S) of the uniform medium S lies in; raises if S touches a
    material change, a conductor or the grid edge."""
    eps = np.asarray(wl.eps, dtype=np.float64)
    mu = np.asarray(wl.mu, dtype=np.float64)
    e_vals, h_vals = set(), set()
    dispersive = {k for k, poles in (getattr(wl, "lorentz", None) or {}).items() if poles}
    for f in faces:
        for comp, ids in wl.comp_ids.items():
            idx, _ = gather(wl, f, comp)
            vals = ids.ravel()[idx.ravel()]
            if comp[0] == "E":
                e_vals.update(eps[vals].tolist())
                if dispersive & set(vals.tolist()):
                    # the stress tensor's eps_S would depend on frequency
                    raise ValueError("S lies in a dispersive material")
            else:
                h_vals.update(mu[vals].tolist())
    if len(e_vals) != 1 or len(h_vals) != 1:
        raise ValueError(f"S is not inside a uniform medium: eps {e_vals}, mu {h_vals}")
    e_s, m_s = e_vals.pop(), h_vals.pop()
    if not (np.isfinite(e_s) and np.isfinite(m_s) and e_s > 0 and m_s > 0):
        raise ValueError("S touches a conductor")
    return e_s, m_s


def setup(wl, basis: str = "dct"):
    faces = build_faces(wl)
    bases = {fi: face_basis(wl, f, basis) for fi, f in enumerate(faces)}
    eps_s, mu_s = surface_medium(wl, faces)
    chans = channel_table(wl, faces, bases, eps_s, mu_s)
    return faces, bases, eps_s, mu_s, chans


def _run_group(args):
    """Run one batch of channels sharing (polarization, kind); return
    Gamma of shape (T, len(batch))."""
    wl, faces, bases, eps_s, mu_s, batch, n_steps, start = args
    pol, kind = batch[0].pol, batch[0].kind
    e_axes, h_axes = POL_COMPONENTS[pol]
    sim = YeeSim(wl, kind, len(batch), e_axes, h_axes)
    dx = 1.0 / wl.res
    dA = dx ** (wl.ndim - 1)
    cache = {}

    def W(fi, comp):
        if (fi, comp) not in cache:
            cache[(fi, comp)] = gather(wl, faces[fi], comp)
        return cache[(fi, comp)]

    # kick: X_j = -(W^T f_n) / (dx * eps_S or mu_S)
    medium = eps_s if kind == "E" else mu_s
    for c, ch in enumerate(batch):
        idx, w = W(ch.face, ch.src)
        f = bases[ch.face][0][ch.row]
        src = np.zeros(int(np.prod(sim.grid_shape)))
        np.add.at(src, idx.ravel(), (w * f[:, None]).ravel())
        sim.field(ch.src)[c] += (-src / (dx * medium)).reshape(sim.grid_shape)
    sim.start(start)

    # measurement groups: channels sharing (face, measured component)
    groups = defaultdict(list)
    for c, ch in enumerate(batch):
        groups[(ch.face, ch.meas)].append(c)
    plan = []
    for (fi, q), cs in groups.items():
        idx, w = W(fi, q)
        rows = np.array([bases[fi][0][batch[c].row] for c in cs])
        plan.append((q, np.array(cs), idx, w, rows))

    gam = np.zeros((n_steps, len(batch)))
    for m in range(n_steps):
        sim.step()
        for q, cs, idx, w, rows in plan:
            X = sim.field(q).reshape(sim.C, -1)[cs]           # (n, ncell)
            wx = np.sum(X[:, idx] * w[None], axis=2)           # (n, N): (W X)_i
            gam[m, cs] = dA * np.sum(rows * wx, axis=1)        # dx^{d-1} sum_i f_n(s_i) (W X)_i
    return gam


def run_gammas(wl, chans, faces, bases, eps_s, mu_s, n_steps: int, workers: int = 1,
               chunk: int = 64, channel_subset=None, start: str = "consistent") -> np.ndarray:
    """Gamma_c(t_m) for m = 1..n_steps, shape (n_steps, C) (C = len(subset))."""
    sel = list(range(len(chans))) if channel_subset is None else list(channel_subset)
    by_group = defaultdict(list)
    for c in sel:
        by_group[(chans[c].pol, chans[c].kind)].append(c)
    jobs, owners = [], []
    for key, cs in by_group.items():
        for s in range(0, len(cs), chunk):
            part = cs[s:s + chunk]
            jobs.append((wl, faces, bases, eps_s, mu_s, [chans[c] for c in part], n_steps, start))
            owners.append(part)
    if workers > 1 and len(jobs) > 1:
        with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
            outs = pool.map(_run_group, jobs)
    else:
        outs = [_run_group(j) for j in jobs]
    gam = np.zeros((n_steps, len(sel)))
    pos = {c: k for k, c in enumerate(sel)}
    for part, g in zip(owners, outs):
        gam[:, [pos[c] for c in part]] = g
    return gam


def zinv_premise_holds(wl) -> bool:
    """Appendix A.2 derives the z-invariant kernel for perfect conductors
    in vacuum (TE and TM decouple at every k_z with the vacuum dispersion):
    every material the grid uses must be vacuum or a perfect conductor."""
    used = set()
    for name in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
        arr = wl.comp_ids.get(name) if wl.comp_ids else None
        used |= {0} if arr is None else set(np.unique(np.asarray(arr)).tolist())
    for i in used:
        e, m = float(wl.eps[i]), float(wl.mu[i])
        conductor = (np.isinf(e) and e < 0) or (np.isinf(m) and m < 0)
        if not conductor and not (e == 1.0 and m == 1.0):
            return False
    return True


def solve(wl, basis: str = "dct", workers: int = 1, keep_gamma: bool = False,
          n_steps: Optional[int] = None, chunk: int = 64, start: str = "consistent",
          channel_subset=None) -> OracleResult:
    if wl.kernel == "zinv2d" and not zinv_premise_holds(wl):
        raise ValueError("the z-invariant kernel (Appendix A.2) holds for perfect conductors in vacuum only")
    T = int(wl.n_steps if n_steps is None else n_steps)
    faces, bases, eps_s, mu_s, chans = setup(wl, basis)
    dt = wl.courant / wl.res
    K = kernel_table(wl.kernel, wl.sigma, dt, T)
    if channel_subset is not None:
        chans = [chans[c] for c in channel_subset]
    gam = run_gammas(wl, chans, faces, bases, eps_s, mu_s, T, workers=workers, chunk=chunk,
                     start=start)
    terms = dt * K[:, None] * gam                     # (T, C)
    acc = terms.sum(axis=0)
    sign = np.array([c.sign for c in chans])
    force = float(np.sum(sign * acc) / np.pi)
    per_h, per_f = defaultdict(float), defaultdict(float)
    for c, ch in enumerate(chans):
        per_h[ch.label] += sign[c] * acc[c] / np.pi
        per_f[faces[ch.face].index] += sign[c] * acc[c] / np.pi
    trace = np.cumsum(terms @ sign) / np.pi
    return OracleResult(force, dict(per_h), dict(per_f), acc, sign, gam if keep_gamma else None,
                        trace, chans, faces, eps_s, mu_s)

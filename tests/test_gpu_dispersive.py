"""GPU parity of dispersive (Lorentz) media against the FP64 oracle (Sec. III B:
a fitted Lorentz model continued onto the conductivity contour, carried as
an auxiliary polarization per term in the E half step of the 2D kernels).

Tolerances as in test_gpu_parity.py: FP64 fields to 1e-9 of the summed term
magnitude sum_c |s_c acc_c| / pi, FP32 fields to 1e-5 of it.  The batched
split path, the plain path and channel waves must agree bit for bit.
"""
import numpy as np
import pytest

import oracle
from casimir_inputs.configs import layered_plates_1d, piston2d

pytestmark = pytest.mark.gpu
MiB = 1 << 20


def announce(name):
    print(f"\n[case] {name}", flush=True)


def run(cf, wl, **over):
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
                precision=wl.precision)
    opts.update(over)
    return cf.Problem.from_workload(wl).solve(**opts)


def dispersive_piston(pol="TM+TE", n_terms=1, n_steps=300, periodic_x=False):
    """The small piston with the left block a Lorentz dielectric (eps_inf 2)
    and S around the right, PEC block; the sidewall slabs stay PEC."""
    base = piston2d(40, 24, 4, 10, 5, 10, 7, 10.0, pol=pol, n_harm=6, n_steps=n_steps, kernel="general")
    ids = {k: v.copy() for k, v in base.comp_ids.items()}
    for v in ids.values():
        left = v[:, :, :20]
        left[left == 1] = 3
    terms = ((3.0, 2.0), (0.7, 5.5), (1.2, 9.0))[:n_terms]
    wl = base.replace(eps=[1.0, float("-inf"), 1.0, 2.0], mu=[1.0, 1.0, 1.0, 1.0], comp_ids=ids,
                      lorentz={3: terms})
    if periodic_x:
        wl = wl.replace(bc=("periodic", "pec", "periodic"))
    return wl


def check(g, ref, rtol):
    terms = float(np.sum(np.abs(ref.sign * ref.acc)) / np.pi)
    assert abs(g["force"] - ref.force) <= rtol * terms, (g["force"], ref.force, terms)
    np.testing.assert_allclose(g["per_channel"], ref.acc, rtol=0, atol=rtol * np.max(np.abs(ref.acc)))


CASES = {
    "piston_tmte_1term": lambda: dispersive_piston(),
    "piston_tmte_3terms_periodic_x": lambda: dispersive_piston(n_terms=3, periodic_x=True),
    "coated_cavity_tm": lambda: layered_plates_1d(20, 1.0, 0.5, 1.5, 0.3, 1.5, ((3.0, 3.0),), pol="TM",
                                                  kernel="general", n_steps=800),
    "coated_cavity_te": lambda: layered_plates_1d(20, 1.0, 0.5, 1.5, 0.3, 1.5, ((3.0, 3.0),), pol="TE",
                                                  kernel="general", n_steps=800),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_dispersive_parity(cf, name):
    announce(f"dispersive parity {name}")
    wl = CASES[name]()
    ref = oracle.solve(wl)
    g64 = run(cf, wl, precision="fp64")
    assert not g64["fused"]                       # dispersive problems take the split kernels
    check(g64, ref, 1e-9)
    g32 = run(cf, wl, precision="fp32")
    check(g32, ref, 1e-5)
    print(f"[disp] {name}: force {g64['force']:.12e} oracle {ref.force:.12e}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dispersive_paths_bitwise(cf, precision):
    """batched split == plain == batched in channel waves, bit for bit."""
    announce(f"dispersive split / plain / waves, {precision}")
    wl = dispersive_piston(n_steps=150)
    a = run(cf, wl, precision=precision)
    sub = [0, 5, 17, 40, 63]
    b = run(cf, wl, precision=precision, path="plain", channel_subset=sub)
    np.testing.assert_array_equal(a["per_channel"][sub], b["per_channel"])
    c = run(cf, wl, precision=precision, max_resident=7)
    np.testing.assert_array_equal(a["per_channel"], c["per_channel"])
    assert a["force"] == c["force"]


def test_dispersive_batch_and_server(cf):
    """A batch with a dispersive and a plain piston solves the dispersive one
    on its own (bitwise its cf_solve), the plain one fused; the server
    refuses dispersive problems."""
    announce("dispersive problem in a batch and the server")
    wd = dispersive_piston(n_steps=120)
    wp = piston2d(40, 24, 4, 10, 5, 10, 7, 10.0, pol="TM+TE", n_harm=6, n_steps=120, kernel="general")
    pd, pp = cf.Problem.from_workload(wd), cf.Problem.from_workload(wp)
    opts = dict(sigma=1.0, courant=0.5, n_steps=120, pol="TM+TE", kernel="general", precision="fp32")
    both = cf.batch_solve([pd, pp], **opts)
    alone = pd.solve(**opts)
    np.testing.assert_array_equal(both[0]["per_channel"], alone["per_channel"])
    assert not both[0]["fused"] and both[1]["fused"]
    with cf.Server(64 * MiB) as srv:
        with pytest.raises(cf.CfError) as e:
            srv.submit(pd, **opts)
        assert e.value.status == "CF_E_UNSUPPORTED"

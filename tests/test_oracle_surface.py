"""Pins of the oracle's surface, basis and interpolation (Sec. III A).

* the cosine basis is exactly orthonormal and complete on the face samples
  (the discrete cosine transform property the paper relies on), with f_0 =
  1/sqrt(L);
* interpolation weights form a partition of unity and reproduce the sample
  position (first-order exact), on every face and component, also where the
  sampling wraps across a periodic boundary;
* the channel generator reproduces the stress-tensor channels read off the
  Minkowski tensor by hand for TM, TE and 3D.
"""
import numpy as np
import pytest

from casimir_inputs import c1_piston_tm_fp64, parallel_plates_1d, sphere_plate3d
from casimir_inputs.geometry import COMPONENT_OFFSETS2
from oracle.surface import (_dct_1d, _fourier_1d, build_faces, channel_specs, face_basis,
                            gather)


@pytest.mark.parametrize("N", [1, 2, 7, 24, 40])
def test_dct_orthonormal_and_complete(N):
    dx = 0.025
    B = _dct_1d(N, N + 5, dx)           # request clamps to N
    assert B.shape == (N, N)
    np.testing.assert_allclose(dx * B @ B.T, np.eye(N), atol=1e-12)
    np.testing.assert_allclose(dx * B.T @ B, np.eye(N), atol=1e-12)
    np.testing.assert_allclose(B[0], np.sqrt(1.0 / (N * dx)), rtol=1e-14)


@pytest.mark.parametrize("N", [5, 8, 45])
def test_fourier_basis_orthonormal_and_complete(N):
    dx = 0.1
    B = _fourier_1d(N, N, dx)
    np.testing.assert_allclose(dx * B @ B.T, np.eye(N), atol=1e-12)


def _positions(wl, comp, idx):
    nx, ny, nz = wl.shape
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    o = COMPONENT_OFFSETS2[comp]
    return np.stack([i + o[0] / 2, j + o[1] / 2, k + o[2] / 2], axis=-1)


@pytest.mark.parametrize("make", [
    lambda: c1_piston_tm_fp64(),
    lambda: sphere_plate3d(24, 0.45, pml=4, n_harm=3, margin=2),
])
def test_interpolation_partition_of_unity_and_position(make):
    wl = make()
    for f in build_faces(wl):
        for comp in wl.comp_ids:
            idx, w = gather(wl, f, comp)
            np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=0, atol=1e-15)
            pos = (_positions(wl, comp, idx) * w[..., None]).sum(axis=1)
            # expected sample positions
            grids = np.meshgrid(*[np.arange(c) for c in f.count], indexing="ij")
            exp = np.zeros((f.n_samples, 3))
            exp[:, f.axis] = f.plane
            for k, ax in enumerate(f.tang):
                exp[:, ax] = f.start[k] + grids[k].ravel() + 0.5
            for ax in range(wl.ndim):
                np.testing.assert_allclose(pos[:, ax], exp[:, ax], atol=1e-12)


def test_periodic_full_span_has_no_faces_and_wraps():
    wl = parallel_plates_1d(10, 1.0, 0.5, 1.5, ny=6)
    faces = build_faces(wl)
    assert [f.axis for f in faces] == [0, 0]
    assert faces[0].count == (6,)
    idx, w = gather(wl, faces[0], "Ez")       # Ez at integer y: last sample wraps to row 0
    nx = wl.shape[0]
    assert set((idx[-1] // nx).tolist()) == {5, 0}


def test_channel_table_matches_stress_tensor():
    e, m = 1.8, 1.3
    tab = lambda pol, a, d: sorted(channel_specs(pol, a, d, e, m))
    # TM (Ez, Hx, Hy), force along x
    assert tab("TM", 0, 0) == sorted([("E", "z", "z", -0.5 * e), ("H", "x", "x", 0.5 * m),
                                      ("H", "y", "y", -0.5 * m)])
    assert tab("TM", 1, 0) == [("H", "y", "x", m)]
    # TE (Ex, Ey, Hz), force along x
    assert tab("TE", 0, 0) == sorted([("E", "x", "x", 0.5 * e), ("E", "y", "y", -0.5 * e),
                                      ("H", "z", "z", -0.5 * m)])
    assert tab("TE", 1, 0) == [("E", "y", "x", e)]
    # force along y: the roles of the faces swap
    assert tab("TM", 1, 1) == sorted([("E", "z", "z", -0.5 * e), ("H", "x", "x", -0.5 * m),
                                      ("H", "y", "y", 0.5 * m)])
    assert tab("TM", 0, 1) == [("H", "x", "y", m)]
    # 3D, force along z
    assert len(tab("3D", 2, 2)) == 6 and len(tab("3D", 0, 2)) == 2
    assert ("E", "z", "z", 0.5 * e) in tab("3D", 2, 2)
    assert tab("3D", 0, 2) == sorted([("E", "x", "z", e), ("H", "x", "z", m)])


def test_c1_face_layout():
    wl = c1_piston_tm_fp64()
    faces = build_faces(wl)
    assert [(f.axis, f.side, f.plane, f.count) for f in faces] == [
        (0, -1, 48, (14,)), (0, 1, 72, (14,)), (1, -1, 13, (24,)), (1, 1, 27, (24,))]
    nrows = [face_basis(wl, f)[0].shape[0] for f in faces]
    assert nrows == [14, 14, 16, 16]      # 16 requested, clamped to the 14 samples

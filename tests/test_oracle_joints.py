"""Pins of the oracle's joints (sec. 5.3: linear equalities between
material points, the virtual tetrahedron's vertices; here a stiff quadratic
penalty): gradient and the full Hessian (diagonal and off-diagonal blocks)
against central differences of the energy; the static deflection of a body
hung from a world joint at its centre of mass, m g / kappa_j in closed form;
a hinge (two joints on an axis) leaves rotation about its axis free and
holds the others."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from scenegen import meshes


def _full(S, q, P):
    """Energy, gradient and dense Hessian of the joint penalties over all
    bodies' DOFs."""
    nb = len(S["body_fixed"])
    keys = oracle.off_keys(S, np.zeros((0, 2), np.int32), np.zeros((0, 2), np.int32))
    e, g, D, O = oracle.joints(S, q, P, keys)
    H = np.zeros((12 * nb, 12 * nb))
    for b in range(nb):
        H[12 * b:12 * b + 12, 12 * b:12 * b + 12] = D[b].reshape(12, 12)
    for k, (a, b) in enumerate(keys):
        H[12 * a:12 * a + 12, 12 * b:12 * b + 12] = O[k].reshape(12, 12)
        H[12 * b:12 * b + 12, 12 * a:12 * a + 12] = O[k].reshape(12, 12).T
    return e, g.reshape(-1), H, keys


def test_joint_derivatives_by_finite_differences():
    S, P = sg.hinged_chain(n_links=3)
    rng = np.random.default_rng(1)
    q = S["q0"] + 1e-2 * rng.normal(size=S["q0"].shape)
    e, g, H, keys = _full(S, q, P)
    assert len(keys) == 2 and e > 0
    h = 1e-6
    n = q.size
    gf, Hf = np.zeros(n), np.zeros((n, n))
    for i in range(n):
        d = np.zeros(n)
        d[i] = h
        qp, qm = (q.reshape(-1) + d).reshape(q.shape), (q.reshape(-1) - d).reshape(q.shape)
        gf[i] = (oracle.joints(S, qp, P, None)[0] - oracle.joints(S, qm, P, None)[0]) / (2 * h)
        Hf[:, i] = (_full(S, qp, P)[1] - _full(S, qm, P)[1]) / (2 * h)
    np.testing.assert_allclose(g, gf, rtol=0, atol=1e-6 * np.abs(g).max())
    np.testing.assert_allclose(H, Hf, rtol=0, atol=1e-6 * np.abs(H).max())
    assert np.linalg.eigvalsh(H).min() >= -1e-9 * np.abs(H).max()  # a sum of squares of linear maps


def test_static_deflection_of_a_hung_body():
    # a 0.1 m cube (1 kg) hung from a world joint at its centre: at rest the
    # joint stretches by m g / kappa_j
    v, t = meshes.cube(0.05)
    sb = sg.SceneBuilder()
    sb.add(v, t, p=(0.0, 1.0, 0.0))
    sb.joint(0, -1, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    S = sb.build()
    P = sg.default_params(kappa_j=1e5, newton_tol=1e-9)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    for _ in range(200):
        q, qd, _ = oracle.time_step(S, B, q, qd, P)
    m = B.mass[0][0]
    assert m == pytest.approx(1.0, rel=1e-12)
    assert 1.0 - q[0, 1] == pytest.approx(m * 9.8 / P["kappa_j"], rel=1e-6)
    assert abs(q[0, 0]) < 1e-12 and abs(q[0, 2]) < 1e-12


def test_hinge_frees_only_its_axis():
    # a cube hinged to the world on the z axis through its centre, no
    # gravity: a spin about z survives, a spin about x is held
    v, t = meshes.cube(0.05)

    def run(axis):
        sb = sg.SceneBuilder()
        qd = np.zeros(12)
        W = np.cross(np.eye(3), axis)  # [axis]x: W @ r = axis x r
        qd[3:] = (2.0 * W).reshape(9)  # A' = W A with A = I: angular velocity 2 rad/s
        sb.add(v, t, p=(0.0, 0.0, 0.0), qd=qd)
        for z in (-0.05, 0.05):
            sb.joint(0, -1, (0.0, 0.0, z), (0.0, 0.0, z))
        S = sb.build()
        P = sg.default_params(kappa_j=1e6, newton_tol=1e-9, gravity=(0.0, 0.0, 0.0))
        B = oracle.Body(S)
        q, qdv = S["q0"].copy(), S["qd0"].copy()
        for _ in range(5):
            q, qdv, _ = oracle.time_step(S, B, q, qdv, P)
        return q, qdv

    q, qd = run(np.array([0.0, 0.0, 1.0]))
    A = q[0, 3:].reshape(3, 3)
    angle = np.arctan2(A[1, 0], A[0, 0])
    assert angle == pytest.approx(2.0 * 0.05, rel=0.05)  # 5 steps of 0.01 s at 2 rad/s
    q, qd = run(np.array([1.0, 0.0, 0.0]))
    A = q[0, 3:].reshape(3, 3)
    assert abs(np.arctan2(A[2, 1], A[1, 1])) < 1e-3 * 0.1

"""Pins of the CPU oracle against facts fixed by the paper and by
mathematics (closed forms, invariants, library routines, brute force,
finite differences), each chosen so that a plausible slip in the oracle
(dropped term, wrong sign or index, transposed operand) fails it.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from scenegen import meshes

RNG = np.random.default_rng(12345)


# ----------------------------------------------------------------- mass ----

def _single_body(v, t, density=1000.0):
    b = sg.SceneBuilder()
    b.add(v, t, density=density)
    return b.build()


def test_mass_unit_cube_closed_form():
    # Eq. mass for a unit cube of density rho about its centre:
    # m = rho, first moment 0, second moment rho/12 I.
    S = _single_body(*meshes.cube(0.5), density=1000.0)
    mass, vol = oracle.mass_properties(S)
    assert vol[0] == pytest.approx(1.0, rel=1e-15)
    np.testing.assert_allclose(mass[0, 0], 1000.0, rtol=1e-15)
    np.testing.assert_allclose(mass[0, 1:4], 0.0, atol=1e-12)
    np.testing.assert_allclose(mass[0, 4:], [1000 / 12, 0, 0, 1000 / 12, 0, 1000 / 12], atol=1e-12)


def test_mass_right_tetrahedron_textbook():
    # unit right tetrahedron: vol 1/6, int x = 1/24, int x^2 = 1/60, int xy = 1/120
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    t = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
    S = _single_body(v, t, density=1.0)
    mass, vol = oracle.mass_properties(S)
    np.testing.assert_allclose(vol[0], 1 / 6, rtol=1e-14)
    np.testing.assert_allclose(mass[0, 1:4], 1 / 24, rtol=1e-14)
    np.testing.assert_allclose(mass[0, [4, 7, 9]], 1 / 60, rtol=1e-14)
    np.testing.assert_allclose(mass[0, [5, 6, 8]], 1 / 120, rtol=1e-14)


def test_mass_general_tetrahedra_by_affine_map_of_the_simplex():
    # any tetrahedron is b + A u over the unit simplex, so with
    # m1 = int u = 1/24 (1,1,1) and M2 = int u u^T = (I + 1 1^T) / 120:
    # vol = |det A| / 6, h = |det A| (A m1 + b / 6),
    # S = |det A| (A M2 A^T + A m1 b^T + b m1^T A^T + b b^T / 6)
    rng = np.random.default_rng(77)
    m1 = np.full(3, 1 / 24)
    M2 = (np.eye(3) + np.ones((3, 3))) / 120
    for _ in range(5):
        v = rng.normal(size=(4, 3))
        A, b = (v[1:] - v[0]).T, v[0]
        det = np.linalg.det(A)
        t = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
        if det < 0:
            t = t[:, ::-1].copy()
        rho = 3.0
        S = _single_body(v, t, density=rho)
        mass, vol = oracle.mass_properties(S)
        ad = abs(det)
        h = ad * (A @ m1 + b / 6)
        Sm = ad * (A @ M2 @ A.T + np.outer(A @ m1, b) + np.outer(b, A @ m1) + np.outer(b, b) / 6)
        np.testing.assert_allclose(vol[0], ad / 6, rtol=1e-12)
        np.testing.assert_allclose(mass[0, 0], rho * ad / 6, rtol=1e-12)
        np.testing.assert_allclose(mass[0, 1:4], rho * h, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(mass[0, 4:], rho * Sm[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]],
                                   rtol=1e-11, atol=1e-13)


def test_mass_translated_and_rotated_body():
    # moments of a shifted, rotated cube follow the parallel-axis theorem:
    # h = m c, S = R (m/12 I) R^T + m c c^T
    R = sg.scenes.random_rotation(np.random.default_rng(3), math.pi)
    c = np.array([0.3, -0.2, 0.7])
    v, t = meshes.cube(0.5)
    S = _single_body(v @ R.T + c, t, density=2.0)
    mass, _ = oracle.mass_properties(S)
    m = 2.0
    np.testing.assert_allclose(mass[0, 0], m, rtol=1e-14)
    np.testing.assert_allclose(mass[0, 1:4], m * c, rtol=1e-13)
    Sm = m / 12 * np.eye(3) + m * np.outer(c, c)
    np.testing.assert_allclose(mass[0, [4, 5, 6, 7, 8, 9]], Sm[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]], atol=1e-13)


def test_mass_icosphere_volume_against_convex_hull():
    from scipy.spatial import ConvexHull
    v, t = meshes.icosphere(2, 0.07)
    S = _single_body(v, t)
    _, vol = oracle.mass_properties(S)
    assert vol[0] == pytest.approx(ConvexHull(v).volume, rel=1e-12)


def test_mass_matrix_kinetic_energy():
    # 1/2 qdot^T M qdot equals the kinetic energy sum over a dense sampling
    # of the body: check with a cube against the exact integral of
    # rho |Adot xbar + pdot|^2 computed by Gauss-Legendre quadrature.
    v, t = meshes.cube(0.5)
    S = _single_body(v + np.array([0.1, 0.2, -0.3]), t, density=3.0)
    mass, _ = oracle.mass_properties(S)
    M = oracle.mass_matrix(mass)[0]
    qd = np.random.default_rng(7).normal(size=12)
    g, w = np.polynomial.legendre.leggauss(3)
    pts = np.stack(np.meshgrid(g / 2, g / 2, g / 2, indexing="ij"), -1).reshape(-1, 3) + [0.1, 0.2, -0.3]
    wts = np.einsum("i,j,k->ijk", w / 2, w / 2, w / 2).reshape(-1)
    Ad = qd[3:].reshape(3, 3)
    vel = pts @ Ad.T + qd[:3]
    ke = 0.5 * 3.0 * np.sum(wts * np.sum(vel * vel, 1))
    assert 0.5 * qd @ M @ qd == pytest.approx(ke, rel=1e-13)


def test_q_tilde_gravity_term_is_exact_for_off_centre_bodies():
    # sec. 4: q~ = q + dt qdot + dt^2 M^-1 f with f = int rho J(xbar)^T g.
    # The generalised gravity force is integrated here by Gauss-Legendre
    # quadrature over a cube whose rest frame is off its centre, and
    # M^-1 f must be the pure translation (g, 0, 0, 0) the oracle uses.
    c = np.array([0.4, -0.7, 0.25])
    v, t = meshes.cube(0.5)
    S = _single_body(v + c, t, density=2.5)
    mass, _ = oracle.mass_properties(S)
    M = oracle.mass_matrix(mass)[0]
    P = sg.default_params(dt=0.02)
    grav = np.asarray(P["gravity"], float)
    gl, w = np.polynomial.legendre.leggauss(2)
    pts = np.stack(np.meshgrid(gl / 2, gl / 2, gl / 2, indexing="ij"), -1).reshape(-1, 3) + c
    wts = np.einsum("i,j,k->ijk", w / 2, w / 2, w / 2).reshape(-1)
    f = np.zeros(12)
    for xb, wt in zip(pts, wts):
        J = np.zeros((3, 12))
        J[:, :3] = np.eye(3)
        for i in range(3):
            J[i, 3 + 3 * i: 6 + 3 * i] = xb
        f += 2.5 * wt * J.T @ grav
    d = np.linalg.solve(M, f)
    np.testing.assert_allclose(d[:3], grav, rtol=1e-12)
    np.testing.assert_allclose(d[3:], 0.0, atol=1e-12 * np.abs(grav).max())
    q = sg.random_state(S, 2, rot_angle=0.5, stretch=0.05, shift=0.3)
    qd = np.random.default_rng(5).normal(size=q.shape)
    qt = oracle.q_tilde(S, q, qd, P)
    np.testing.assert_allclose(qt, q + P["dt"] * qd + P["dt"] ** 2 * d[None, :], rtol=1e-14, atol=1e-15)


# --------------------------------------------------------- vertex map ----

def test_vertex_map_matches_affine_map_and_rigid_motion():
    S, _ = sg.three_cubes()
    q = sg.random_state(S, 4, rot_angle=1.0, stretch=0.1, shift=0.5)
    x = oracle.vertex_map(S, q)
    for b in range(len(q)):
        sl = slice(S["body_vert_off"][b], S["body_vert_off"][b + 1])
        A = q[b, 3:].reshape(3, 3)
        np.testing.assert_allclose(x[sl], S["xbar"][sl] @ A.T + q[b, :3], rtol=0, atol=1e-15)
    # pure rotation preserves body-frame distances from p
    S2, _ = sg.icosphere_box(n_side=2, n_layers=1)
    x = oracle.vertex_map(S2, S2["q0"])
    for b in range(1, len(S2["q0"])):
        sl = slice(S2["body_vert_off"][b], S2["body_vert_off"][b + 1])
        np.testing.assert_allclose(np.linalg.norm(x[sl] - S2["q0"][b, :3], axis=1),
                                   np.linalg.norm(S2["xbar"][sl], axis=1), rtol=1e-14)


# --------------------------------------------------------- candidates ----

def _brute_candidates(S, x0, x1, inflate):
    lo = np.minimum(x0, x1)
    hi = np.maximum(x0, x1)
    tris, edges = S["tris"], S["edges"]
    tlo, thi = lo[tris].min(1), hi[tris].max(1)
    elo, ehi = lo[edges].min(1), hi[edges].max(1)
    vb, tb, eb = S["vert_body"], S["tri_body"], S["edge_body"]
    fx, sc = S["body_fixed"], S["body_scene"]

    def ok(alo, ahi, blo, bhi):
        return np.all((alo[:, None, :] <= bhi[None, :, :] + inflate) & (blo[None, :, :] <= ahi[:, None, :] + inflate), -1)

    def valid(ba, bb):
        return (ba[:, None] != bb[None, :]) & (sc[ba][:, None] == sc[bb][None, :]) & ~(
            (fx[ba][:, None] == 1) & (fx[bb][None, :] == 1))

    m = ok(lo, hi, tlo, thi) & valid(vb, tb)
    pt = np.argwhere(m)
    m = ok(elo, ehi, elo, ehi) & valid(eb, eb)
    m = np.triu(m, 1)
    ee = np.argwhere(m)
    return pt.astype(np.int32), ee.astype(np.int32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_candidates_equal_brute_force(seed):
    S = sg.near_contact_cubes(seed, n=4)
    q = sg.random_state(S, seed, rot_angle=0.01, shift=2e-4)
    x0 = oracle.vertex_map(S, S["q0"])
    x1 = oracle.vertex_map(S, q)
    for a, b, infl in ((x0, x0, 1e-3), (x0, x1, 1e-3), (x1, x0, 5e-4)):
        pt, ee = oracle.candidates(S, a, b, infl)
        bpt, bee = _brute_candidates(S, a, b, infl)
        np.testing.assert_array_equal(pt, bpt)
        np.testing.assert_array_equal(ee, bee)
        assert len(pt) > 0 and len(ee) > 0


def test_candidates_soup_and_scenes():
    S = sg.triangle_soup(5, n_bodies=12)
    x0 = oracle.vertex_map(S, S["q0"])
    pt, ee = oracle.candidates(S, x0, None, 1e-3)
    bpt, bee = _brute_candidates(S, x0, x0, 1e-3)
    np.testing.assert_array_equal(pt, bpt)
    np.testing.assert_array_equal(ee, bee)
    # scenes never pair across sub-scenes
    Sb, _ = sg.batched_drops(seed=9, n_scenes=3, n_min=2, n_max=4)
    xb = oracle.vertex_map(Sb, Sb["q0"])
    pt, ee = oracle.candidates(Sb, xb, xb + np.array([0, -1.0, 0]), 1e-3)
    bpt, bee = _brute_candidates(Sb, xb, xb + np.array([0, -1.0, 0]), 1e-3)
    np.testing.assert_array_equal(pt, bpt)
    np.testing.assert_array_equal(ee, bee)


# ----------------------------------------------------------- distance ----

def _seg_d2(p, a, b):
    e = b - a
    t = np.clip(np.dot(p - a, e) / np.dot(e, e), 0.0, 1.0)
    r = p - (a + t * e)
    return np.dot(r, r)


def _pt_d2_qp(p, t0, t1, t2):
    """exact point-triangle distance as a 2-variable convex QP: interior KKT
    point if feasible, else the best edge."""
    e0, e1 = t1 - t0, t2 - t0
    G = np.array([[e0 @ e0, e0 @ e1], [e0 @ e1, e1 @ e1]])
    r = np.array([e0 @ (p - t0), e1 @ (p - t0)])
    u, v = np.linalg.solve(G, r)
    if u >= 0 and v >= 0 and u + v <= 1:
        d = p - t0 - u * e0 - v * e1
        return d @ d
    return min(_seg_d2(p, t0, t1), _seg_d2(p, t1, t2), _seg_d2(p, t0, t2))


def _ee_d2_qp(a0, a1, b0, b1):
    u, v, w = a1 - a0, b1 - b0, a0 - b0
    G = np.array([[u @ u, -(u @ v)], [-(u @ v), v @ v]])
    r = np.array([-(u @ w), v @ w])
    try:
        s, t = np.linalg.solve(G, r)
        if 0 <= s <= 1 and 0 <= t <= 1:
            d = w + s * u - t * v
            return d @ d
    except np.linalg.LinAlgError:
        pass
    return min(_seg_d2(a0, b0, b1), _seg_d2(a1, b0, b1), _seg_d2(b0, a0, a1), _seg_d2(b1, a0, a1))


def test_distance_closed_forms():
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    # point above the face interior: the height
    d, ty = oracle.pair_distance(0, np.vstack([[0.2, 0.3, 0.7], tri]))
    assert ty == 6 and d == pytest.approx(0.7, rel=1e-15)
    # beyond vertex t1: point-point
    d, ty = oracle.pair_distance(0, np.vstack([[2.0, -1.0, 0.5], tri]))
    assert ty == 1 and d == pytest.approx(math.sqrt(1 + 1 + 0.25), rel=1e-15)
    # beyond edge t1-t2 (hypotenuse): point-edge
    d, ty = oracle.pair_distance(0, np.vstack([[1.0, 1.0, 0.0], tri]))
    assert ty == 4 and d == pytest.approx(math.sqrt(0.5), rel=1e-15)
    # perpendicular crossing edges at offset 0.3: line-line
    d, ty = oracle.pair_distance(1, np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0.3], [0, 1, 0.3]], float))
    assert ty == 28 and d == pytest.approx(0.3, rel=1e-15)
    # parallel edges: endpoint case, offset 0.2
    d, ty = oracle.pair_distance(1, np.array([[0, 0, 0], [1, 0, 0], [0.5, 0.2, 0], [2, 0.2, 0]], float))
    assert ty != 28 and d == pytest.approx(0.2, rel=1e-15)


@pytest.mark.parametrize("is_ee", [0, 1])
def test_distance_equals_exact_qp(is_ee):
    rng = np.random.default_rng(100 + is_ee)
    seen = set()
    for _ in range(3000):
        X = rng.normal(size=(4, 3))
        d, ty = oracle.pair_distance(is_ee, X)
        seen.add(ty)
        ref = math.sqrt(_ee_d2_qp(*X) if is_ee else _pt_d2_qp(*X))
        assert d == pytest.approx(ref, rel=1e-9, abs=1e-13)
    # every case code is reached by random inputs
    if is_ee:
        assert 28 in seen and len(seen) >= 9
    else:
        assert seen == set(range(7))


def test_distance_not_above_dense_sampling():
    rng = np.random.default_rng(7)
    for _ in range(50):
        X = rng.normal(size=(4, 3))
        d, _ = oracle.pair_distance(0, X)
        u, v = np.meshgrid(np.linspace(0, 1, 201), np.linspace(0, 1, 201))
        m = u + v <= 1
        pts = X[1] + u[m][:, None] * (X[2] - X[1]) + v[m][:, None] * (X[3] - X[1])
        ds = np.linalg.norm(pts - X[0], axis=1).min()
        assert d <= ds * (1 + 1e-12)
        assert d >= ds - 0.02 * np.linalg.norm(X[2] - X[1]) - 0.02 * np.linalg.norm(X[3] - X[1])


# ------------------------------------------------------------ barrier ----

DHAT = 1e-3


def _paper_barrier(d, dhat):
    return -(d - dhat) ** 2 * math.log(d / dhat) if 0 < d < dhat else 0.0


def test_barrier_value_point_above_face():
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    for h in (1e-5, 3e-4, 9.99e-4):
        X = np.vstack([[0.25, 0.25, h], tri])
        ty, e, g, H = oracle.pair_local(0, X, X, DHAT, 2.0)
        assert ty == 6
        assert e == pytest.approx(2.0 * _paper_barrier(h, DHAT), rel=1e-12)
        # gradient along the normal: kappa B'(h) on the point, opposite on the triangle
        Bp = -2 * (h - DHAT) * math.log(h / DHAT) - (h - DHAT) ** 2 / h
        assert g[2] == pytest.approx(2.0 * Bp, rel=1e-10)
        assert g[5] + g[8] + g[11] == pytest.approx(-2.0 * Bp, rel=1e-10)


def test_barrier_c2_clamp_at_dhat():
    # B, B', B'' vanish at d = dhat (smooth clamping)
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    X = np.vstack([[0.25, 0.25, DHAT * (1 - 1e-9)], tri])
    _, e, g, H = oracle.pair_local(0, X, X, DHAT, 1.0)
    assert abs(e) < 1e-30 and np.abs(g).max() < 1e-20 and np.abs(H).max() < 1e-8


def _random_near_pair(rng, is_ee):
    """Random pair at a distance in (0.1, 0.9) dhat, away from case borders."""
    while True:
        X = rng.normal(size=(4, 3)) * 1e-2
        d, ty = oracle.pair_distance(is_ee, X)
        if d <= 0:
            continue
        target = rng.uniform(0.1, 0.9) * DHAT
        # slide the first feature along the closest direction to reach target
        n = rng.normal(size=3)
        if not is_ee:
            # move the point toward its closest feature
            c = X[1:].mean(0)
            X[0] = c + (X[0] - c) * target / max(d, 1e-12)
        else:
            shift = (X[2:].mean(0) - X[:2].mean(0))
            X[:2] += shift * (1 - target / max(d, 1e-12))
        d, ty = oracle.pair_distance(is_ee, X)
        if 0.05 * DHAT < d < 0.95 * DHAT:
            return X


def _fd_check(is_ee, X, kappa=1.0):
    ty, e, g, H = oracle.pair_local(is_ee, X, X, DHAT, kappa)
    h = 1e-9
    gf = np.zeros(12)
    Hf = np.zeros((12, 12))
    x = X.reshape(12)
    for i in range(12):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        tp, ep, gp, _ = oracle.pair_local(is_ee, xp.reshape(4, 3), X, DHAT, kappa)
        tm, em, gm, _ = oracle.pair_local(is_ee, xm.reshape(4, 3), X, DHAT, kappa)
        if tp != ty or tm != ty:
            return None
        gf[i] = (ep - em) / (2 * h)
        Hf[:, i] = (gp - gm) / (2 * h)
    return g, gf, H, Hf


@pytest.mark.parametrize("is_ee", [0, 1])
def test_barrier_derivatives_finite_differences(is_ee):
    rng = np.random.default_rng(21 + is_ee)
    done = 0
    while done < 30:
        X = _random_near_pair(rng, is_ee)
        r = _fd_check(is_ee, X)
        if r is None:
            continue
        g, gf, H, Hf = r
        sg_ = np.abs(g).max()
        sh = np.abs(H).max()
        np.testing.assert_allclose(g, gf, rtol=0, atol=1e-5 * sg_)
        np.testing.assert_allclose(H, Hf, rtol=0, atol=1e-4 * sh)
        np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-12 * sh)
        done += 1


@pytest.mark.parametrize("is_ee", [0, 1])
def test_barrier_translation_rotation_invariance(is_ee):
    rng = np.random.default_rng(31 + is_ee)
    for _ in range(20):
        X = _random_near_pair(rng, is_ee)
        _, e, g, H = oracle.pair_local(is_ee, X, X, DHAT, 1.0)
        G = g.reshape(4, 3)
        s = np.abs(G).max()
        np.testing.assert_allclose(G.sum(0), 0.0, atol=1e-9 * s)
        np.testing.assert_allclose(np.cross(X, G).sum(0), 0.0, atol=1e-9 * s * np.abs(X).max())


def test_mollifier_parallel_edges_vanish():
    # exactly parallel edges: mollifier m(0) = 0 so the EE barrier is zero
    X = np.array([[0, 0, 0], [1e-2, 0, 0], [2e-3, 5e-4, 0], [8e-3, 5e-4, 0]], float)
    ty, e, g, H = oracle.pair_local(1, X, X, DHAT, 1.0)
    assert e == 0.0 and np.abs(g).max() == 0.0


# Near-parallel crossing edges: edge a on the x axis, edge b a height h above
# it, turned by theta in the x-z plane.  The closest points are both
# midpoints (line-line case), so d = h, and c = |u x v|^2 = |u|^2 |v|^2
# sin^2 theta.  The mollifier's threshold eps = 1e-3 |u_rest|^2 |v_rest|^2
# depends on the rest edges alone, so scaling a rest copy of the pair sets
# r = c / eps to any value while the deformed pair (and B(d)) stays fixed.
def _crossing_edges(h=0.5 * DHAT, theta=0.02, half=1e-2):
    v = np.array([math.cos(theta), 0.0, math.sin(theta)])
    return np.array([[-half, 0, 0], [half, 0, 0], [0, h, 0] - half * v, [0, h, 0] + half * v])


def _rest_for_ratio(X, r):
    """A scaled copy of X whose eps makes c / eps = r, and that r as the
    definition gives it (c and eps as products of the edge vectors)."""
    u, v = X[1] - X[0], X[3] - X[2]
    c = np.dot(np.cross(u, v), np.cross(u, v))
    sig = (c / (1e-3 * u.dot(u) * v.dot(v) * r)) ** 0.25
    xb = X * sig
    ub, vb = xb[1] - xb[0], xb[3] - xb[2]
    return xb, c / ((1e-3 * ub.dot(ub)) * vb.dot(vb))


def _mollifier_closed_form(r):
    # IPC's EE mollifier m(c) = (2 - c/eps) c/eps below eps, 1 above
    return (2.0 - r) * r if r < 1.0 else 1.0


def test_mollifier_closed_form_values_and_c1_join():
    # the ratio of the mollified energy to the same pair's unmollified
    # energy (rest edges short enough that c > eps) is m(r): 0.4375 at
    # r = 1/4, 0.75 at r = 1/2, 0.99 at 0.9; approaching r = 1 from below,
    # 1 - m = (1 - r)^2 (value 1 and zero slope at the join), and m = 1
    # at and above it.  A linear ramp c/eps fails every r < 1.
    X = _crossing_edges()
    d, ty = oracle.pair_distance(1, X)
    assert ty == 28 and d == pytest.approx(0.5 * DHAT, rel=1e-12)  # line-line
    xb_ref, r_ref = _rest_for_ratio(X, 4.0)
    _, e_ref, _, _ = oracle.pair_local(1, X, xb_ref, DHAT, 3.0)
    assert e_ref == pytest.approx(3.0 * _paper_barrier(d, DHAT), rel=1e-12)
    for r in (0.25, 0.5, 0.9, 1.0 - 1e-2, 1.0 - 1e-3, 1.0 + 1e-3, 2.0):
        xb, r_act = _rest_for_ratio(X, r)
        _, e, _, _ = oracle.pair_local(1, X, xb, DHAT, 3.0)
        m = e / e_ref
        assert m == pytest.approx(_mollifier_closed_form(r_act), rel=1e-12, abs=1e-15)
        if r < 1.0:
            # one-sided difference at the join: (1 - m(1 - s)) / s = s -> 0
            s = 1.0 - r_act
            assert (1.0 - m) / s == pytest.approx(s, rel=1e-6)
    _, e_half, _, _ = oracle.pair_local(1, X, _rest_for_ratio(X, 0.5)[0], DHAT, 3.0)
    assert e_half / e_ref == pytest.approx(0.75, rel=1e-12)


def test_mollified_barrier_derivatives_finite_differences():
    # 0 < c < eps on near-parallel edges: the gradient and Hessian of m B
    # are the derivatives of its (pinned) energy, so the product rule's m'
    # term (slope (2 - 2r)/eps) is checked.  Dropping m' or using a linear
    # ramp moves the gradient by far more than the tolerance.
    for theta, r in ((0.02, 0.5), (0.015, 0.3), (0.03, 0.8)):
        X = _crossing_edges(h=0.4 * DHAT, theta=theta)
        xb, _ = _rest_for_ratio(X, r)
        ty, e, g, H = oracle.pair_local(1, X, xb, DHAT, 1.0)
        assert ty == 28  # line-line
        h = 1e-9
        x = X.reshape(12)
        gf = np.zeros(12)
        Hf = np.zeros((12, 12))
        for i in range(12):
            xp, xm = x.copy(), x.copy()
            xp[i] += h
            xm[i] -= h
            _, ep, gp, _ = oracle.pair_local(1, xp.reshape(4, 3), xb, DHAT, 1.0)
            _, em, gm, _ = oracle.pair_local(1, xm.reshape(4, 3), xb, DHAT, 1.0)
            gf[i] = (ep - em) / (2 * h)
            Hf[:, i] = (gp - gm) / (2 * h)
        np.testing.assert_allclose(g, gf, rtol=0, atol=1e-6 * np.abs(g).max())
        np.testing.assert_allclose(H, Hf, rtol=0, atol=1e-5 * np.abs(H).max())
        # the m' part is a visible share of the gradient here: the same
        # pair with m held at its value (rest edges giving r >= 1, energy
        # rescaled) has a gradient that differs by well over the tolerance
        xb1, _ = _rest_for_ratio(X, 4.0)
        _, e1, g1, _ = oracle.pair_local(1, X, xb1, DHAT, 1.0)
        assert np.abs(g - (e / e1) * g1).max() > 1e-3 * np.abs(g).max()


def _two_edge_scene(X, xb):
    """Two free bodies holding one edge each (vertices 0-1 and 2-3); the
    scene-level oracle calls take the deformed positions X separately from
    the rest positions xb."""
    return dict(xbar=np.ascontiguousarray(xb, dtype=np.float64), vert_body=np.array([0, 0, 1, 1], np.int32),
                tris=np.zeros((0, 3), np.int32), tri_body=np.zeros(0, np.int32),
                edges=np.array([[0, 1], [2, 3]], np.int32), edge_body=np.array([0, 1], np.int32),
                body_fixed=np.zeros(2, np.uint8)), np.ascontiguousarray(X, dtype=np.float64)


def test_mollifier_in_scene_energy_and_friction_lag():
    # the energy-only path and the friction lag carry their own mollifier
    # evaluation: at r = 1/2 the barrier energy is 0.75 of the unmollified
    # one and the lagged normal force lambda = kappa m |B'(d)| is 0.75 of
    # its unmollified value, which is kappa |B'(d)| in closed form.
    X = _crossing_edges()
    d = 0.5 * DHAT
    P = sg.default_params(dhat=DHAT, kappa_b=5.0)
    ee = np.array([[0, 1]], np.int32)
    pt = np.zeros((0, 2), np.int32)
    Bp = -2 * (d - DHAT) * math.log(d / DHAT) - (d - DHAT) ** 2 / d
    res = {}
    for r in (0.5, 4.0):
        xb, r_act = _rest_for_ratio(X, r)
        S, x = _two_edge_scene(X, xb)
        e = oracle.barrier_energy(S, x, pt, ee, P)
        F = oracle.friction_lag(S, x, pt, ee, P)
        res[r] = (e, F["ee"]["lam"][0], r_act)
    m = _mollifier_closed_form(res[0.5][2])
    assert res[4.0][0] == pytest.approx(5.0 * _paper_barrier(d, DHAT), rel=1e-12)
    assert res[0.5][0] == pytest.approx(m * res[4.0][0], rel=1e-12)
    assert res[4.0][1] == pytest.approx(5.0 * abs(Bp), rel=1e-10)
    assert res[0.5][1] == pytest.approx(m * res[4.0][1], rel=1e-12)
    assert m == pytest.approx(0.75, rel=1e-12)


def test_friction_lag_vjp_through_mollifier_by_fd():
    # the adjoint's derivative of the lag (lambda, T, w as functions of x^t)
    # on a near-parallel pair with 0 < c < eps: lambda carries m(c(x^t)),
    # so the VJP must carry m and its slope; central differences of the lag
    # (x^t in the sliding displacement held fixed) agree with it.
    X = _crossing_edges(h=0.4 * DHAT, theta=0.02)
    xb, r = _rest_for_ratio(X, 0.5)
    assert 0.4 < r < 0.6
    # bodies at identity with x = xbar (rest positions are the current ones
    # scaled, so A = I / sig maps the rest pair onto X)
    sig = xb[1, 0] / X[1, 0]
    S, _ = _two_edge_scene(X, xb)
    P = sg.default_params(dhat=DHAT, kappa_b=5.0, mu=0.4)
    qt = np.zeros((2, 12))
    for b in range(2):
        qt[b, 3:] = (np.eye(3) / sig).reshape(9)
    xt = oracle.vertex_map(S, qt)
    np.testing.assert_allclose(xt, X, atol=1e-15)
    ee = np.array([[0, 1]], np.int32)
    pt = np.zeros((0, 2), np.int32)
    F = oracle.friction_lag(S, xt, pt, ee, P, keep_inactive=True)
    assert F["ee"]["lam"][0] > 0
    # current positions: a small slide of body 1 along x (|u| above eps_v dt)
    q = qt.copy()
    q[1, 0] += 3e-5
    x = oracle.vertex_map(S, q)
    rng = np.random.default_rng(8)
    l = rng.normal(size=(2, 12))
    v = oracle.friction_lag_vjp(S, x, F, P, l)
    keys = np.array([[0, 1]], np.int32)

    def lag_dot(qq):
        Fp = oracle.friction_lag(S, oracle.vertex_map(S, qq), pt, ee, P, keep_inactive=True)
        Fp["xt"] = F["xt"]
        return float(np.sum(l * oracle.friction(S, x, Fp, P, keys, hess=False)["grad"]))

    h = 1e-9
    fd = np.zeros((2, 12))
    for b in range(2):
        for c in range(12):
            qp, qm = qt.copy(), qt.copy()
            qp[b, c] += h
            qm[b, c] -= h
            fd[b, c] = (lag_dot(qp) - lag_dot(qm)) / (2 * h)
    np.testing.assert_allclose(v, fd, rtol=0, atol=1e-5 * np.abs(fd).max())


# ---------------------------------------------------------------- PSD ----

def test_psd_projection_matches_eigh():
    rng = np.random.default_rng(5)
    for n in (6, 9, 12):
        for _ in range(20):
            A = rng.normal(size=(n, n))
            A = A + A.T
            A *= 10 ** rng.uniform(-6, 6)
            P = oracle.psd_project(A)
            w, V = np.linalg.eigh(A)
            ref = (V * np.maximum(w, 0)) @ V.T
            np.testing.assert_allclose(P, ref, rtol=0, atol=1e-13 * np.abs(A).max())
            # idempotent, identity on PSD inputs
            np.testing.assert_allclose(oracle.psd_project(P), P, rtol=0, atol=1e-13 * np.abs(A).max())
            assert np.linalg.eigvalsh(P).min() > -1e-12 * np.abs(A).max()


def test_psd_projection_nearest_in_frobenius():
    # Higham: no random PSD matrix is closer to A than P
    rng = np.random.default_rng(6)
    A = rng.normal(size=(12, 12))
    A = A + A.T
    P = oracle.psd_project(A)
    best = np.linalg.norm(A - P)
    for _ in range(200):
        B = rng.normal(size=(12, 3))
        Q = P + 0.01 * B @ B.T
        assert np.linalg.norm(A - Q) >= best - 1e-12


# ---------------------------------------------------- assembly (J^T H J) ----

def _near_scene(seed=0):
    S = sg.near_contact_cubes(seed, n=3)
    P = sg.default_params(dhat=1e-3, kappa_b=80.0)
    return S, P


def test_barrier_q_gradient_and_hessian_by_fd():
    S, P = _near_scene(1)
    q0 = S["q0"]
    x = oracle.vertex_map(S, q0)
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    keys = oracle.off_keys(S, pt, ee)
    r = oracle.barrier(S, x, pt, ee, P, keys, project=False)
    assert r["n_active"] > 10
    free = np.flatnonzero(S["body_fixed"] == 0)

    def energy(q):
        return oracle.barrier_energy(S, oracle.vertex_map(S, q), pt, ee, P)

    def grad(q):
        xx = oracle.vertex_map(S, q)
        return oracle.barrier(S, xx, pt, ee, P, keys, project=False)["grad"]

    h = 1e-9
    for b in free:
        for c in range(12):
            qp, qm = q0.copy(), q0.copy()
            qp[b, c] += h
            qm[b, c] -= h
            fd = (energy(qp) - energy(qm)) / (2 * h)
            assert fd == pytest.approx(r["grad"][b, c], rel=1e-5, abs=1e-6 * np.abs(r["grad"]).max())
            col = (grad(qp) - grad(qm)) / (2 * h)
            scale = np.abs(r["diag"]).max()
            np.testing.assert_allclose(r["diag"][b].reshape(12, 12)[:, c], col[b], atol=2e-4 * scale)
            for k, (a1, b1) in enumerate(keys):
                O = r["off"][k].reshape(12, 12)
                if b == b1:
                    np.testing.assert_allclose(O[:, c], col[a1], atol=2e-4 * scale)
                if b == a1:
                    np.testing.assert_allclose(O.T[:, c], col[b1], atol=2e-4 * scale)


@pytest.mark.parametrize("mu", [0.0, 0.4])
def test_incremental_potential_gradient_hessian_and_newton_direction(mu):
    # sec. 4: E(q) = 1/2 |q - q~|_M^2 + orthogonality + barrier (+ lagged
    # friction).  grad_hess must be the derivative of total_energy (a term
    # dropped, doubled or of the wrong sign in either fails), and the Newton
    # direction must solve the assembled system H p = -g.
    S, P = _near_scene(4)
    P = dict(P, mu=mu)
    B = oracle.Body(S)
    rng = np.random.default_rng(9)
    free = np.flatnonzero(S["body_fixed"] == 0)
    qd = np.zeros_like(S["q0"])
    qd[free] = rng.normal(scale=0.05, size=(len(free), 12))
    qt = oracle.q_tilde(S, S["q0"], qd, P)
    q0 = S["q0"].copy()
    q0[free, 3:] += rng.normal(scale=1e-4, size=(len(free), 9))
    x = oracle.vertex_map(S, q0)
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    F = oracle.step_friction(S, q0, P)
    assert (F is not None) == (mu > 0)
    gh = oracle.grad_hess(S, B, q0, qt, P, x=x, pt=pt, ee=ee, project=False, F=F)
    assert gh["n_active"] > 10

    def energy(q):
        return oracle.total_energy(S, B, q, qt, oracle.vertex_map(S, q), pt, ee, P, F)

    def grad(q):
        return oracle.grad_hess(S, B, q, qt, P, pt=pt, ee=ee, project=False, F=F)["grad"]

    assert energy(q0) == pytest.approx(gh["energy"], rel=1e-12)
    A, fr = oracle.assemble(S, gh["diag"], gh["off"], gh["keys"])
    H = A.toarray()
    gscale = np.abs(gh["grad"][free]).max()
    hscale = np.abs(H).max()
    # the friction state is lagged at q0, where the sliding displacement is
    # zero: its gradient has a |u| u / eps^2 term whose central difference
    # errs by about h / eps^2, so the Hessian columns take a step well below
    # eps = eps_v dt
    h = 1e-8
    hh = 1e-10 if mu > 0 else h
    for i, b in enumerate(fr):
        for c in range(12):
            qp, qm = q0.copy(), q0.copy()
            qp[b, c] += h
            qm[b, c] -= h
            fd = (energy(qp) - energy(qm)) / (2 * h)
            assert fd == pytest.approx(gh["grad"][b, c], rel=1e-5, abs=1e-6 * gscale)
            qp, qm = q0.copy(), q0.copy()
            qp[b, c] += hh
            qm[b, c] -= hh
            col = ((grad(qp) - grad(qm)) / (2 * hh))[fr].reshape(-1)
            np.testing.assert_allclose(H[:, 12 * i + c], col, atol=2e-4 * hscale)
    p = oracle.solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    res = H @ p[fr].reshape(-1) + gh["grad"][fr].reshape(-1)
    assert np.abs(res).max() <= 1e-9 * np.abs(H).max() * np.abs(p).max() + 1e-12 * gscale
    assert np.all(p[S["body_fixed"] != 0] == 0.0)


def test_assembly_equals_dense_jacobian_product():
    S, P = _near_scene(2)
    x = oracle.vertex_map(S, S["q0"])
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    keys = oracle.off_keys(S, pt, ee)
    r = oracle.barrier(S, x, pt, ee, P, keys, project=True, local=True)
    nb = len(S["q0"])
    nv = len(x)
    # dense J (3 nv x 12 nb) of the kinematic map
    J = np.zeros((3 * nv, 12 * nb))
    for k in range(nv):
        b = S["vert_body"][k]
        for i in range(3):
            J[3 * k + i, 12 * b + i] = 1.0
            J[3 * k + i, 12 * b + 3 + 3 * i: 12 * b + 6 + 3 * i] = S["xbar"][k]
    Hx = np.zeros((3 * nv, 3 * nv))
    gx = np.zeros(3 * nv)
    for name, pairs in (("pt", pt), ("ee", ee)):
        lg, lH = r["local"][name]
        for i, pr in enumerate(pairs):
            if name == "pt":
                vid = [pr[0], *S["tris"][pr[1]]]
            else:
                vid = [*S["edges"][pr[0]], *S["edges"][pr[1]]]
            idx = np.concatenate([np.arange(3 * v, 3 * v + 3) for v in vid])
            Hx[np.ix_(idx, idx)] += lH[i].reshape(12, 12)
            gx[idx] += lg[i]
    Hq = J.T @ Hx @ J
    gq = J.T @ gx
    free = S["body_fixed"] == 0
    sc = np.abs(Hq).max()
    for b in range(nb):
        if not free[b]:
            continue
        np.testing.assert_allclose(r["grad"][b], gq[12 * b:12 * b + 12], atol=1e-12 * np.abs(gq).max())
        np.testing.assert_allclose(r["diag"][b].reshape(12, 12), Hq[12 * b:12 * b + 12, 12 * b:12 * b + 12],
                                   atol=1e-12 * sc)
    for k, (a, b) in enumerate(keys):
        np.testing.assert_allclose(r["off"][k].reshape(12, 12), Hq[12 * a:12 * a + 12, 12 * b:12 * b + 12],
                                   atol=1e-12 * sc)


# ------------------------------------------------------ orthogonality ----

def _ortho_def(A, kn):
    return kn * np.linalg.norm(A @ A.T - np.eye(3), "fro") ** 2


def test_orthogonality_zero_on_rotations_and_scaling_closed_form():
    S, P = sg.three_cubes()
    mass, vol = oracle.mass_properties(S)
    q = S["q0"].copy()
    e, g, D = oracle.orthogonality(S, vol, q, P, w=1.0)
    assert abs(e) < 1e-12 * P["kappa_o"]
    assert np.abs(g).max() < 1e-6 * P["kappa_o"] * 1e-8
    s = 1.3
    q[1, 3:] = (s * np.eye(3)).reshape(9)
    q[2, 3:] = (s * np.eye(3)).reshape(9)
    e, g, D = oracle.orthogonality(S, vol, q, P, w=1.0)
    assert e == pytest.approx(2 * 3 * P["kappa_o"] * (s * s - 1) ** 2, rel=1e-13)


def test_orthogonality_gradient_hessian_fd_of_definition():
    S, P = sg.three_cubes()
    _, vol = oracle.mass_properties(S)
    rng = np.random.default_rng(8)
    q = S["q0"].copy()
    q[1:, 3:] += 0.05 * rng.normal(size=(2, 9))
    kn = P["kappa_o"] * vol[1]
    e, g, D = oracle.orthogonality(S, vol, q, P, project=False, w=1.0)
    A = q[1, 3:].reshape(3, 3)
    h = 1e-7
    gf = np.zeros(9)
    for i in range(9):
        Ap, Am = A.copy().reshape(9), A.copy().reshape(9)
        Ap[i] += h
        Am[i] -= h
        gf[i] = (_ortho_def(Ap.reshape(3, 3), kn) - _ortho_def(Am.reshape(3, 3), kn)) / (2 * h)
    np.testing.assert_allclose(g[1, 3:], gf, rtol=1e-6, atol=1e-6 * np.abs(gf).max())
    Hf = np.zeros((9, 9))
    for i in range(9):
        qp, qm = q.copy(), q.copy()
        qp[1, 3 + i] += h
        qm[1, 3 + i] -= h
        Hf[:, i] = (oracle.orthogonality(S, vol, qp, P, project=False, w=1.0)[1][1, 3:]
                    - oracle.orthogonality(S, vol, qm, P, project=False, w=1.0)[1][1, 3:]) / (2 * h)
    H = D[1].reshape(12, 12)[3:, 3:]
    np.testing.assert_allclose(H, Hf, rtol=0, atol=1e-6 * np.abs(H).max())
    assert np.abs(D[1].reshape(12, 12)[:3]).max() == 0.0


# ---------------------------------------------------------------- CCD ----

def test_ccd_point_toward_plane_closed_form():
    # point at height d0 moving straight down onto a static triangle with
    # speed v: time of impact t* = d0/v, ACCD returns (1 - s) t*.
    S = sg.SceneBuilder()
    S.add(np.array([[-1, 0, -1], [1, 0, -1], [0, 0, 1]], float), np.array([[0, 2, 1]], np.int32), fixed=True)
    S.add(np.array([[0, 0, 0], [1, 0, 0], [0, 0, 1]], float), np.array([[0, 1, 2]], np.int32))
    S = S.build()
    P = sg.default_params()
    x = np.array([[-1, 0, -1], [1, 0, -1], [0, 0, 1], [0, 0.01, 0], [5, 5, 5], [6, 5, 5]], float)
    dx = np.zeros_like(x)
    dx[3] = [0, -0.04, 0]
    pt = np.array([[3, 0]], np.int32)
    ee = np.zeros((0, 2), np.int32)
    tpt, _, alpha = oracle.ccd(S, x, dx, pt, ee, P)
    assert tpt[0] == pytest.approx((1 - P["ccd_s"]) * 0.25, rel=1e-12)
    # no motion: full step
    tpt, _, alpha = oracle.ccd(S, x, np.zeros_like(x), pt, ee, P)
    assert tpt[0] == 1.0 and alpha == 1.0


@pytest.mark.parametrize("is_ee", [0, 1])
def test_ccd_conservative_by_fine_sampling(is_ee):
    rng = np.random.default_rng(41 + is_ee)
    S = sg.SceneBuilder()
    S.add(np.eye(3), np.array([[0, 1, 2]], np.int32))
    S.add(np.eye(3), np.array([[0, 1, 2]], np.int32))
    S = S.build()
    P = sg.default_params()
    hits = 0
    for _ in range(200):
        X = rng.normal(size=(4, 3)) * 0.1
        U = rng.normal(size=(4, 3)) * 0.3
        if is_ee:
            x = np.vstack([X[:2], [[9, 9, 9]], X[2:], [[-9, -9, -9]]])
            dx = np.vstack([U[:2], [[0, 0, 0]], U[2:], [[0, 0, 0]]])
            pairs = np.array([[0, 2]], np.int32)
            Sx = dict(S, edges=np.array([[0, 1], [1, 2], [0, 2], [3, 4], [4, 5], [3, 5]], np.int32))
            _, t, _ = oracle.ccd(Sx, x, dx, np.zeros((0, 2), np.int32), pairs, P)
        else:
            x = np.vstack([X[:1], [[9, 9, 9], [9, 8, 9]], X[1:]])
            dx = np.vstack([U[:1], [[0, 0, 0], [0, 0, 0]], U[1:]])
            Sx = dict(S, tris=np.array([[0, 1, 2], [3, 4, 5]], np.int32))
            pairs = np.array([[0, 1]], np.int32)
            t, _, _ = oracle.ccd(Sx, x, dx, pairs, np.zeros((0, 2), np.int32), P)
        t = t[0]
        d0, _ = oracle.pair_distance(is_ee, X)
        alphas = np.linspace(0.0, t, 2001)
        ds = np.array([oracle.pair_distance(is_ee, X + a * U)[0] for a in alphas])
        assert ds.min() > 0.0
        assert ds[-1] >= P["ccd_s"] * d0 * (1 - 1e-9)
        hits += t < 1.0
    assert hits > 20


# ------------------------------------------------------- time stepping ----

def test_free_flight_closed_form():
    # no contact: p^n = p^0 + n dt v0 + dt^2 g n(n+1)/2, A constant;
    # Newton converges after one step direction.
    b = sg.SceneBuilder()
    v, t = meshes.cube(0.1)
    qd = np.zeros(12)
    qd[:3] = [0.3, 1.0, -0.2]
    b.add(v, t, p=(0.0, 5.0, 0.0), qd=qd)
    S = b.build()
    P = sg.default_params(dt=1e-2)
    B = oracle.Body(S)
    q, qdv = S["q0"].copy(), S["qd0"].copy()
    n = 20
    for _ in range(n):
        q, qdv, its = oracle.time_step(S, B, q, qdv, P)
        assert its <= 2
    g = np.array(P["gravity"])
    dt = P["dt"]
    pref = S["q0"][0, :3] + n * dt * qd[:3] + dt * dt * g * n * (n + 1) / 2
    np.testing.assert_allclose(q[0, :3], pref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(q[0, 3:], S["q0"][0, 3:], atol=1e-13)
    np.testing.assert_allclose(qdv[0, :3], qd[:3] + n * dt * g, atol=1e-10)


def _min_distance_brute(S, x):
    pt, ee = oracle.candidates(S, x, None, 1.0)
    ty, d2, _ = oracle.classify(S, x, pt, 0, 1.0)
    ty2, d22, _ = oracle.classify(S, x, ee, 1, 1.0)
    return math.sqrt(min(d2.min() if len(d2) else 1e30, d22.min() if len(d22) else 1e30))


def test_three_cubes_energy_decrease_nonintersection_and_rest():
    S, P = sg.three_cubes()
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    for step in range(60):
        log = []
        qn, qdn, its = oracle.time_step(S, B, q, qd, P, log)
        # every accepted iterate lowers the incremental potential
        for info in log:
            if "e1" in info:
                assert info["e1"] <= info["e0"]
        assert _min_distance_brute(S, oracle.vertex_map(S, qn)) > 0.0
        q, qd = qn, qdn
    # resting: the barrier carries the weight of the cubes above it
    # (momentum balance: sum of barrier p-forces on cube 2 = m dt^2 g)
    x = oracle.vertex_map(S, q)
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    keys = oracle.off_keys(S, pt, ee)
    bar = oracle.barrier(S, x, pt, ee, P, keys)
    m = B.mass[2, 0]
    fy = bar["grad"][2, 1]
    assert fy == pytest.approx(-m * P["dt"] ** 2 * P["gravity"][1] * -1, rel=0.05)


# ------------------------------------------------------------- friction ----

def _friction_setup(seed=3):
    S, P = _near_scene(seed)
    P = dict(P, mu=0.4)
    xt = oracle.vertex_map(S, S["q0"])
    pt, ee = oracle.candidates(S, xt, None, P["dhat"])
    F = oracle.friction_lag(S, xt, pt, ee, P)
    return S, P, xt, F


def test_friction_lag_closest_points_and_tangent_basis():
    # r = sum w_k x_k is the closest-point difference: |r| equals the
    # pair distance, each side's weights are a convex combination (sums +1
    # and -1 on the two primitives, magnitudes <= 1); T is an orthonormal
    # pair orthogonal to r.
    S, P, xt, F = _friction_setup()
    n_checked = 0
    for is_ee, nm in ((0, "pt"), (1, "ee")):
        f = F[nm]
        assert len(f["pairs"]) > 0
        _, d2, _ = oracle.classify(S, xt, f["pairs"], is_ee, P["dhat"])
        for i, pr in enumerate(f["pairs"]):
            if is_ee:
                vid = np.concatenate([S["edges"][pr[0]], S["edges"][pr[1]]])
                sa = [0, 1]
            else:
                vid = np.concatenate([[pr[0]], S["tris"][pr[1]]])
                sa = [0]
            w = f["w"][i]
            r = (w[:, None] * xt[vid]).sum(0)
            assert np.dot(r, r) == pytest.approx(d2[i], rel=1e-8)
            sb = [k for k in range(4) if k not in sa]
            sgn = 1.0 if w[sa].sum() > 0 else -1.0  # r points from either primitive
            assert w[sa].sum() == pytest.approx(sgn, abs=1e-12)
            assert w[sb].sum() == pytest.approx(-sgn, abs=1e-12)
            assert np.all(np.abs(w) <= 1.0 + 1e-12)
            T = f["T"][i].reshape(2, 3)
            np.testing.assert_allclose(T @ T.T, np.eye(2), atol=1e-13)
            np.testing.assert_allclose(T @ r, 0.0, atol=1e-13 * np.linalg.norm(r))
            n_checked += 1
    assert n_checked > 10


def test_friction_lambda_is_barrier_force_magnitude():
    # lambda = kappa |dB/dd|: the magnitude of the barrier force on the first
    # primitive (the sum of the exact barrier gradient over its vertices),
    # for pairs whose mollifier is 1.
    S, P, xt, F = _friction_setup()
    for is_ee, nm in ((0, "pt"), (1, "ee")):
        f = F[nm]
        for i, pr in enumerate(f["pairs"]):
            if is_ee:
                vid = np.concatenate([S["edges"][pr[0]], S["edges"][pr[1]]])
                ua, ub = S["xbar"][vid[1]] - S["xbar"][vid[0]], S["xbar"][vid[3]] - S["xbar"][vid[2]]
                X = xt[vid]
                c = np.linalg.norm(np.cross(X[1] - X[0], X[3] - X[2])) ** 2
                if c < 1e-3 * ua.dot(ua) * ub.dot(ub):
                    continue
                side = [0, 1]
            else:
                vid = np.concatenate([[pr[0]], S["tris"][pr[1]]])
                side = [0]
            _, _, g, _ = oracle.pair_local(is_ee, xt[vid], S["xbar"][vid], P["dhat"], P["kappa_b"])
            force = g.reshape(4, 3)[side].sum(0)
            assert f["lam"][i] == pytest.approx(np.linalg.norm(force), rel=1e-9)


@pytest.mark.parametrize("scale", [0.3, 3.0])
def test_friction_q_gradient_and_hessian_by_fd(scale):
    # sliding displacements below (0.3) and beyond (3) eps_v dt: the
    # gradient is the derivative of the friction energy, the Hessian the
    # derivative of the gradient (exact and PSD for this f1), both through
    # the affine map x(q).
    S, P, xt, F = _friction_setup()
    rng = np.random.default_rng(7)
    eps = P["eps_v"] * P["dt"]
    free = np.flatnonzero(S["body_fixed"] == 0)
    q0 = S["q0"].copy()
    for b in free:
        d = rng.normal(size=3)
        d[1] = 0.0
        q0[b, :3] += scale * eps * d / np.linalg.norm(d)
        q0[b, 3:] += rng.normal(size=9) * 1e-7
    x0 = oracle.vertex_map(S, q0)
    pt, ee = oracle.candidates(S, xt, None, P["dhat"])
    keys = oracle.off_keys(S, pt, ee)
    r = oracle.friction(S, x0, F, P, keys)
    assert r["energy"] > 0

    def energy(q):
        return oracle.friction_energy(S, oracle.vertex_map(S, q), F, P)

    def grad(q):
        return oracle.friction(S, oracle.vertex_map(S, q), F, P, keys, hess=False)["grad"]

    h = 1e-10
    gs = np.abs(r["grad"]).max()
    hs = np.abs(r["diag"]).max()
    for b in free:
        for c in range(12):
            qp, qm = q0.copy(), q0.copy()
            qp[b, c] += h
            qm[b, c] -= h
            fd = (energy(qp) - energy(qm)) / (2 * h)
            assert fd == pytest.approx(r["grad"][b, c], abs=1e-5 * gs)
            col = (grad(qp) - grad(qm)) / (2 * h)
            np.testing.assert_allclose(r["diag"][b].reshape(12, 12)[:, c], col[b], atol=1e-4 * hs)
            for k, (a1, b1) in enumerate(keys):
                O = r["off"][k].reshape(12, 12)
                if b == b1:
                    np.testing.assert_allclose(O[:, c], col[a1], atol=1e-4 * hs)
                if b == a1:
                    np.testing.assert_allclose(O.T[:, c], col[b1], atol=1e-4 * hs)
    # the assembled friction Hessian is PSD
    Hd = oracle.assemble(S, r["diag"], r["off"], keys)[0].toarray()
    w = np.linalg.eigvalsh(0.5 * (Hd + Hd.T))
    assert w.min() >= -1e-10 * np.abs(w).max()


def _slide(theta, mu, v0, n):
    S, P = sg.cube_on_slope(theta, mu, v0=v0)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    vs = []
    for _ in range(n):
        q, qd, _ = oracle.time_step(S, B, q, qd, P)
        vs.append(qd[1, :3].copy())
    return P, np.array(vs)


def test_friction_slope_sliding_acceleration_closed_form():
    # Coulomb sliding on an inclined plane: a = g (sin theta - mu cos theta)
    # along the slope (eps_v dt is far below the per-step slide, so f1 = 1).
    theta, mu = math.atan(0.75), 0.5
    P, vs = _slide(theta, mu, 1.0, 40)
    a = (vs[-1, 0] - vs[10, 0]) / ((len(vs) - 1 - 10) * P["dt"])
    assert a == pytest.approx(9.8 * (math.sin(theta) - mu * math.cos(theta)), rel=1e-3)
    assert np.abs(vs[10:, 2]).max() < 1e-6


def test_friction_slope_static_creep_closed_form():
    # tan theta < mu: the cube stops; the smoothed static friction then
    # holds it with f1(|u|) = tan theta / mu, i.e. a creep speed of
    # eps_v (1 - sqrt(1 - tan theta / mu)) below eps_v.
    theta, mu = math.atan(0.75), 0.9
    P, vs = _slide(theta, mu, 0.3, 60)
    creep = P["eps_v"] * (1.0 - math.sqrt(1.0 - 0.75 / mu))
    assert vs[-1, 0] == pytest.approx(creep, rel=1e-2)
    assert vs[-10:, 0].max() < P["eps_v"]


def test_sub_scene_extraction_round_trip():
    # the sub-scenes of a batch, concatenated back, reproduce the batch
    S, _ = sg.batched_drops(seed=11, n_scenes=4, n_min=1, n_max=4)
    b = sg.SceneBuilder()
    for k in range(4):
        Sk = sg.sub_scene(S, k)
        for j in range(len(Sk["body_fixed"])):
            v0, v1 = Sk["body_vert_off"][j], Sk["body_vert_off"][j + 1]
            t0, t1 = Sk["body_tri_off"][j], Sk["body_tri_off"][j + 1]
            qj = Sk["q0"][j]
            b.add(Sk["xbar"][v0:v1], Sk["tris"][t0:t1] - v0, R=qj[3:].reshape(3, 3), p=qj[:3],
                  fixed=bool(Sk["body_fixed"][j]), density=Sk["density"][j], qd=Sk["qd0"][j], scene=k)
    R = b.build()
    for key in S:
        np.testing.assert_array_equal(R[key], S[key], err_msg=key)


# -------------------------------------------------------------- adjoint ----

def _loss_and_fd(S, P, n, lags, seed, n_dirs=3):
    B = oracle.Body(S)
    q0, qd0 = S["q0"].copy(), S["qd0"].copy()
    free = S["body_fixed"] == 0
    b1 = int(np.flatnonzero(free)[0])
    target = np.array([0.3, 0.4, -0.2])
    states, Fs = oracle.rollout(S, B, q0, qd0, P, n)
    qbar = np.zeros_like(q0)
    qbar[b1, :3] = 2 * (states[-1][0][b1, :3] - target)
    gq, gqd, _, _ = oracle.rollout_grad(S, B, q0, qd0, P, n, qbar, np.zeros_like(q0))

    def loss(qd):
        st, _ = oracle.rollout(S, B, q0, qd, P, n, lags=Fs if lags else None)
        return float(np.sum((st[-1][0][b1, :3] - target) ** 2))

    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_dirs):
        d = rng.normal(size=q0.shape) * free[:, None]
        d /= np.linalg.norm(d)
        h = 1e-6
        fd = (loss(qd0 + h * d) - loss(qd0 - h * d)) / (2 * h)
        out.append((fd, float(np.sum(gqd * d))))
    return out


def test_adjoint_rollout_gradient_frictionless_by_fd():
    # implicit-function adjoint of 20 implicit-Euler steps of the 3-cube
    # stack (contacts form and persist) vs central differences of the
    # rollout in the initial velocities (Newton converged tightly)
    S, P = sg.three_cubes()
    P = dict(P, newton_tol=1e-7, max_newton=400)
    S["qd0"][1:, 1] = -0.5
    for fd, ad in _loss_and_fd(S, P, 20, False, 2):
        assert ad == pytest.approx(fd, rel=1e-4)


def test_adjoint_rollout_gradient_friction_by_fd():
    # with lagged friction: the adjoint differentiates the lag too (normal
    # force, tangent basis and weights as functions of q^t); central
    # differences of the full rollout (every step re-lagged) agree with it
    S, P = sg.cube_on_slope(math.atan(0.75), 0.5, v0=1.0)
    P = dict(P, newton_tol=1e-9)
    for fd, ad in _loss_and_fd(S, P, 15, False, 1):
        assert ad == pytest.approx(fd, rel=1e-5)


def test_adjoint_without_lag_derivative_would_fail_fd():
    # the lag's own derivative matters: dropping it (differences of the
    # rollout with every step's lagged data held) gives a different answer,
    # so the test above checks that term
    S, P = sg.cube_on_slope(math.atan(0.75), 0.5, v0=1.0)
    P = dict(P, newton_tol=1e-9)
    worst = max(abs(fd - ad) / abs(fd) for fd, ad in _loss_and_fd(S, P, 15, True, 1))
    assert worst > 1e-2

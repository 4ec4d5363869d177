"""Seeded synthetic scenes shaped like the paper's workloads.

Every scene is a plain dict of numpy arrays (structure of arrays, body-major
ranges) plus a parameter dict.  Both the CPU oracle and the GPU library
consume exactly these arrays; nothing here evaluates the simulation method
(no mass properties, distances, energies or derivatives).  Random numbers are
drawn with ``numpy.random.default_rng(seed)`` in the order documented per
builder.

Arrays of a scene dict
  xbar        f64 (nv,3)  body-frame vertex positions
  vert_body   i32 (nv,)   owning body of each vertex
  tris        i32 (nt,3)  global vertex ids, per body contiguous
  tri_body    i32 (nt,)
  edges       i32 (ne,2)  global vertex ids (i<j), per body contiguous
  edge_body   i32 (ne,)
  body_vert_off, body_tri_off, body_edge_off  i32 (nb+1,)
  body_fixed  u8  (nb,)   1 = kinematically fixed (Dirichlet)
  body_scene  i32 (nb,)   scene id (independent sub-scenes of a batch)
  scene_body_off i32 (n_scenes+1,)
  density     f64 (nb,)
  q0, qd0     f64 (nb,12) affine DOFs (p, a1, a2, a3) with a_i the rows of A
"""
import math

import numpy as np

from . import meshes

GRAVITY = (0.0, -9.8, 0.0)


def _rot(axis, angle):
    """Rotation matrix from unit axis and angle (Rodrigues' formula)."""
    k = np.asarray(axis, dtype=np.float64)
    kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(angle) * kx + (1.0 - math.cos(angle)) * (kx @ kx)


def random_rotation(rng, max_angle):
    """Axis uniform on the sphere (normalised Gaussian), angle U[0,max]."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    angle = rng.uniform(0.0, max_angle)
    return _rot(axis, angle)


def q_from(R, p):
    q = np.zeros(12)
    q[:3] = p
    q[3:] = np.asarray(R, dtype=np.float64).reshape(9)  # rows of A
    return q


class SceneBuilder:
    """Accumulates bodies (mesh + initial affine state) into SoA arrays."""

    def __init__(self):
        self.bodies = []
        self.joints = []

    def joint(self, a, b, pa, pb):
        """A joint making body a's body-frame point pa coincide with body b's
        point pb (b = -1: with the fixed world point pb)."""
        self.joints.append((int(a), int(b), np.asarray(pa, np.float64), np.asarray(pb, np.float64)))

    def add(self, verts, tris, R=None, p=(0, 0, 0), fixed=False, density=1000.0,
            qd=None, scene=0):
        R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
        self.bodies.append(dict(v=np.asarray(verts, np.float64), t=np.asarray(tris, np.int32),
                                q=q_from(R, p), qd=np.zeros(12) if qd is None else np.asarray(qd, np.float64),
                                fixed=bool(fixed), density=float(density), scene=int(scene)))

    def build(self):
        xb, vb, tr, tb, ed, eb = [], [], [], [], [], []
        voff, toff, eoff = [0], [0], [0]
        q0, qd0, fixed, dens, bscene = [], [], [], [], []
        nv = 0
        for b, body in enumerate(self.bodies):
            v, t = body["v"], body["t"]
            e = meshes.edges_from_tris(t)
            xb.append(v)
            vb.append(np.full(len(v), b, np.int32))
            tr.append(t + nv)
            tb.append(np.full(len(t), b, np.int32))
            ed.append(e + nv)
            eb.append(np.full(len(e), b, np.int32))
            nv += len(v)
            voff.append(nv)
            toff.append(toff[-1] + len(t))
            eoff.append(eoff[-1] + len(e))
            q0.append(body["q"])
            qd0.append(body["qd"])
            fixed.append(1 if body["fixed"] else 0)
            dens.append(body["density"])
            bscene.append(body["scene"])
        bscene = np.array(bscene, np.int32)
        if len(bscene) and np.any(np.diff(bscene) < 0):
            raise ValueError("bodies must be grouped by scene")
        n_scenes = int(bscene.max()) + 1 if len(bscene) else 0
        soff = np.searchsorted(bscene, np.arange(n_scenes + 1)).astype(np.int32)
        return dict(
            xbar=np.ascontiguousarray(np.concatenate(xb)),
            vert_body=np.concatenate(vb),
            tris=np.ascontiguousarray(np.concatenate(tr).astype(np.int32)),
            tri_body=np.concatenate(tb),
            edges=np.ascontiguousarray(np.concatenate(ed).astype(np.int32)),
            edge_body=np.concatenate(eb),
            body_vert_off=np.array(voff, np.int32),
            body_tri_off=np.array(toff, np.int32),
            body_edge_off=np.array(eoff, np.int32),
            body_fixed=np.array(fixed, np.uint8),
            body_scene=bscene,
            scene_body_off=soff,
            density=np.array(dens, np.float64),
            q0=np.ascontiguousarray(np.array(q0, np.float64)),
            qd0=np.ascontiguousarray(np.array(qd0, np.float64)),
            joint_body=np.array([[a, b] for a, b, _, _ in self.joints], np.int32).reshape(-1, 2),
            joint_point=np.array([[pa, pb] for _, _, pa, pb in self.joints], np.float64).reshape(-1, 2, 3),
        )


def default_params(**kw):
    """Method parameters.  kappa_b is the barrier stiffness (fixed per
    scene; with kappa_adaptive its floor, kappa_max its ceiling and
    kappa_eps_d the distance below which an approaching contact doubles
    it), kappa_o the orthogonality stiffness (multiplied by body volume),
    kappa_j the joint penalty stiffness (N/m),
    ccd_s / ccd_tmax / ccd_max_iter the additive-CCD constants."""
    p = dict(dt=1e-2, dhat=1e-3, kappa_b=80.0, kappa_o=1e8, kappa_j=1e7, kappa_adaptive=0,
             kappa_eps_d=1e-9, mu=0.0, eps_v=1e-3,
             gravity=GRAVITY, newton_tol=1e-5, pcg_rtol=1e-10, ccd_s=0.1,
             ccd_tmax=1.0, ccd_max_iter=10000, max_newton=100, max_pcg=5000,
             max_ls=40, steps=100)
    p.update(kw)
    p.setdefault("kappa_max", 100.0 * p["kappa_b"])  # (IPC's ceiling ratio)
    return p


# --------------------------------------------------------------------------
# Configurations
# --------------------------------------------------------------------------

def three_cubes(seed=1):
    """3 unit cubes stacked along y with 1e-2 m AABB gaps; bottom fixed and
    axis aligned, the two above rotated (axis uniform, angle U[0,0.3]).
    Draw order: rotation of cube 1, rotation of cube 2."""
    rng = np.random.default_rng(seed)
    v, t = meshes.cube(0.5)
    sb = SceneBuilder()
    sb.add(v, t, p=(0.0, 0.0, 0.0), fixed=True)
    top = 0.5
    for _ in range(2):
        R = random_rotation(rng, 0.3)
        w = v @ R.T
        lo, hi = w[:, 1].min(), w[:, 1].max()
        y = top + 1e-2 - lo
        sb.add(v, t, R=R, p=(0.0, y, 0.0))
        top = y + hi
    scene = sb.build()
    # barrier stiffness: a 1000 kg cube resting on one contact sits at dhat/10
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=80.0, mu=0.0, steps=100)
    return scene, params


def icosphere_box(seed=2, n_side=10, n_layers=10, spacing=0.25, friction=0.5):
    """Icospheres (subdivision 2) of radius U[0.05,0.1] with random rotations
    on a jittered n_side x n_layers x n_side grid inside a fixed open box of
    12 quads (inner 2.6 m, height 2.6 m).  Draw order per body (grid order
    layer-major, then x, then z): radius, rotation axis (3), angle,
    jitter (3)."""
    rng = np.random.default_rng(seed)
    sv, st = meshes.icosphere(2, 1.0)
    bv, bt = meshes.open_box(2.6, 2.6)
    sb = SceneBuilder()
    sb.add(bv, bt, fixed=True)
    x0 = -spacing * (n_side - 1) / 2.0
    for j in range(n_layers):
        for i in range(n_side):
            for k in range(n_side):
                r = rng.uniform(0.05, 0.1)
                R = random_rotation(rng, math.pi)
                jit = rng.uniform(-0.02, 0.02, size=3)
                p = np.array([x0 + spacing * i, 0.3 + spacing * j, x0 + spacing * k]) + jit
                sb.add(sv * r, st, R=R, p=p)
    scene = sb.build()
    # kappa_b: a 4 kg sphere landing at 2 m/s is stopped near dhat/2
    # (kappa |B'(dhat/2)| = m v dt); Newton tolerance 1e-2 of the box
    # diagonal per second (IPC's convention); inexact Newton directions
    # (PCG relative residual 1e-2: the Newton iteration counts match those
    # of 1e-4)
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=70.0, mu=friction, steps=200,
                            newton_tol=1e-2 * math.sqrt(3.0) * 2.6, max_newton=500, pcg_rtol=1e-2)
    return scene, params


def torus_chains(seed=3, n_chains=8, n_links=8, n_major=200, n_minor=50,
                 sigma=1e-3, gap=2e-3):
    """n_chains parallel chains of n_links interlocked links (major radius
    0.3, minor 0.1), alternating flat (ring in x-z) and upright (ring in x-y)
    along x; noiseless tube gaps `gap` between every pair of neighbours.

    A link cannot be a plain torus here: with major = 3 minor the hole of a
    ring (inner diameter 0.4) holds the tubes (diameter 0.2) of its two
    neighbours only with zero clearance, so interlocked neighbours at a
    positive gap would overlap each other.  Each link is a stadium instead:
    the torus's two halves joined by straight tube sections of length
    s = 6 minor - 2 major + 3 gap (6 mm at these sizes) along the chain, which
    is the length at which the two neighbours' tubes in a link's hole are
    `gap` apart from each other and from the link.  Link pitch along a chain
    s + 2 major - 2 minor - gap; chain pitch 2 (major + minor) + gap.

    Vertices are pushed inward along the tube normal by |N(0,sigma)|, so gaps
    only grow.  End links fixed; the others get velocity N(0,0.5^2) per
    translation component.  Draw order: per body (chain-major) the noise of
    all vertices, then for free bodies the 3 velocity components."""
    rng = np.random.default_rng(seed)
    Rm, rm = 0.3, 0.1
    straight = 6 * rm - 2 * Rm + 3 * gap
    v0, t0 = meshes.torus(Rm, rm, n_major, n_minor, straight=straight)
    uu = np.repeat(2 * np.pi * np.arange(n_major) / n_major, n_minor)
    ww = np.tile(2 * np.pi * np.arange(n_minor) / n_minor, n_major)
    nrm = np.stack([np.cos(ww) * np.cos(uu), np.sin(ww), np.cos(ww) * np.sin(uu)], -1)
    pitch = straight + 2 * Rm - 2 * rm - gap
    wpitch = 2 * (Rm + rm) + gap
    upright = _rot((1.0, 0.0, 0.0), math.pi / 2)
    sb = SceneBuilder()
    for c in range(n_chains):
        for l in range(n_links):
            noise = np.abs(rng.normal(0.0, sigma, size=len(v0)))
            v = v0 - noise[:, None] * nrm
            fixed = l == 0 or l == n_links - 1
            qd = np.zeros(12)
            if not fixed:
                qd[:3] = rng.normal(0.0, 0.5, size=3)
            R = np.eye(3) if l % 2 == 0 else upright
            p = (pitch * (l - (n_links - 1) / 2.0), 1.0, wpitch * (c - (n_chains - 1) / 2.0))
            sb.add(v, t0, R=R, p=p, fixed=fixed, qd=qd)
    scene = sb.build()
    # kappa_b by the landing rule of the icosphere box: a link (59 kg) met
    # at 0.5 m/s is stopped near dhat/2: kappa |B'(dhat/2)| = m v dt, with
    # |B'(dhat/2)| = (1/2 + ln 2) dhat
    m_link = 1000.0 * 2.0 * math.pi ** 2 * Rm * rm ** 2
    kappa = m_link * 0.5 * 5e-3 / ((0.5 + math.log(2.0)) * 5e-4)
    params = default_params(dt=5e-3, dhat=5e-4, kappa_b=round(kappa), mu=0.0, steps=100)
    return scene, params


def torus_chains_contact(scene, n_chains=8, close=1.95e-3, gap=2e-3):
    """Generalized coordinates of a contact state of `torus_chains` (same
    n_chains and gap): every upright link (ring in x-y, A's middle diagonal
    entry 0) moved `close` along +x, towards the next flat link, and the
    chains moved `close` closer together, so interlocked and side-by-side
    neighbours sit gap - close apart before the vertex noise."""
    q = scene["q0"].copy()
    up = q[:, 4] < 0.5
    q[up, 0] += close
    wpitch = 2 * (0.3 + 0.1) + gap
    c = np.round(q[:, 2] / wpitch + (n_chains - 1) / 2.0)
    q[:, 2] = (wpitch - close) * (c - (n_chains - 1) / 2.0)
    return q


def wrecking_ball(seed=8, n_wide=28, n_high=20, half=0.05, n_links=8, theta0=math.pi / 3):
    """A wall of n_wide x n_high cubes (half-edge `half`, one deep) stacked
    on a fixed ground quad, and a ball swinging into it on a chain: the
    shape of the paper's wrecking-ball scene (sec. 5, Tab. tab:time: 575
    bodies, 14K triangles) from generated shapes only.

    Wall: the front face at x = 0.27, columns along z with 2e-3 gaps, each
    cube U[2e-4, 6e-4] above the one below (the bottom row above the
    ground), tilted by at most 2e-4 rad: every cube rests within dhat of its
    support.  Chain: n_links stadium links (major 0.06, minor 0.02, 24 x 8
    grid; straight sections 6 minor - 2 major + 3 gap so that the two tubes
    in a link's hole are 2e-3 apart, as in the chain workload), alternating
    flat / upright along the chain direction u, link 0 fixed at the pivot
    (0, 2.3, 0), the chain straight and swung theta0 from the vertical
    towards -x.  Ball: one body made of an icosphere (subdivision 3, radius
    0.25) and an eyelet ring (a link) interlocked with the last link, the
    sphere 1 cm beyond the ring along u.  At rest; gravity swings the ball
    into the wall after about 0.5 s.  Draw order: per cube (z-major, then
    y): vertical gap, tilt axis (3), tilt angle."""
    rng = np.random.default_rng(seed)
    gv, gt = meshes.ground_quad(6.0)
    cv, ct = meshes.cube(half)
    Rm, rm, gap = 0.06, 0.02, 2e-3
    straight = 6 * rm - 2 * Rm + 3 * gap
    lv, lt = meshes.torus(Rm, rm, 24, 8, straight=straight)
    pitch = straight + 2 * Rm - 2 * rm - gap
    sb = SceneBuilder()
    sb.add(gv, gt, fixed=True)
    x_face, zgap = 0.27, 2e-3
    for k in range(n_wide):
        y = 0.0
        for j in range(n_high):
            y += rng.uniform(2e-4, 6e-4)
            R = random_rotation(rng, 2e-4)
            w = cv @ R.T
            z = (k - (n_wide - 1) / 2.0) * (2 * half + zgap)
            sb.add(cv, ct, R=R, p=(x_face - w[:, 0].min(), y - w[:, 1].min(), z))
            y += w[:, 1].max() - w[:, 1].min()
    u = np.array([-math.sin(theta0), -math.cos(theta0), 0.0])
    zz = np.array([0.0, 0.0, 1.0])
    v = np.cross(zz, u)
    flat = np.stack([u, v, zz], 1)               # local x -> u, ring plane u-z
    upright = np.stack([u, zz, np.cross(u, zz)], 1)  # ring plane u-v
    pivot = np.array([0.0, 2.3, 0.0])
    for l in range(n_links):
        sb.add(lv, lt, R=flat if l % 2 == 0 else upright, p=pivot + l * pitch * u, fixed=(l == 0))
    bv, bt = meshes.icosphere(3, 0.25)
    reach = straight / 2 + Rm + rm + 0.01 + 0.25  # ring centre to sphere centre
    ball_v = np.concatenate([lv, bv + np.array([reach, 0.0, 0.0])])
    ball_t = np.concatenate([lt, bt + len(lv)])
    sb.add(ball_v, ball_t, R=flat if n_links % 2 == 0 else upright, p=pivot + n_links * pitch * u)
    scene = sb.build()
    # kappa_b by the landing rule of the icosphere box for the ball (65 kg
    # meeting the wall at about 3.3 m/s, stopped near dhat/2)
    m_ball = 1000.0 * 4.0 / 3.0 * math.pi * 0.25 ** 3
    kappa = m_ball * 3.3 * 1e-2 / ((0.5 + math.log(2.0)) * 1e-3)
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=round(kappa, -1), mu=0.0, steps=100,
                            newton_tol=1e-2 * math.sqrt(3.0), max_newton=500, pcg_rtol=1e-2)
    return scene, params


def hinged_chain(n_links=5, length=0.4, width=0.1, gap=0.01, theta0=math.pi / 4, n_chains=1, spacing=0.5):
    """n_chains chains of n_links box links (length x width x width, each
    shortened by `gap` at both ends) joined end to end by hinges about z,
    the first link hinged to a fixed world axis at (0, 2, 0), the chain
    straight and swung theta0 from the vertical towards -x: the paper's
    pendulum (two links) and octopus-tentacle (five joints) mechanisms
    (sec. 5.3, Fig. rotation) from generated shapes.  A hinge is two joints,
    at z = +-width/2 on its axis.  Chains are `spacing` apart along z.  No
    random draws."""
    cv, ct = meshes.cube(0.5)
    lv = cv * np.array([length - 2 * gap, width, width])
    u = np.array([-math.sin(theta0), -math.cos(theta0), 0.0])
    zz = np.array([0.0, 0.0, 1.0])
    R = np.stack([u, np.cross(zz, u), zz], 1)
    sb = SceneBuilder()
    hz = width / 2
    for c in range(n_chains):
        pivot = np.array([0.0, 2.0, (c - (n_chains - 1) / 2.0) * spacing])
        first = len(sb.bodies)
        for l in range(n_links):
            sb.add(lv, ct, R=R, p=pivot + (l + 0.5) * length * u)
        for s_ in (-hz, hz):
            sb.joint(first, -1, (-length / 2, 0.0, s_), pivot + (0.0, 0.0, s_))
            for l in range(n_links - 1):
                sb.joint(first + l, first + l + 1, (length / 2, 0.0, s_), (-length / 2, 0.0, s_))
    scene = sb.build()
    # kappa_b by the landing rule: a 3.8 kg link meeting its neighbour at
    # 3 m/s is stopped near dhat/2
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=100.0, kappa_j=1e7, mu=0.0, steps=100, newton_tol=1e-5)
    return scene, params


def batched_drops(seed=4, n_scenes=256, n_min=2, n_max=200):
    """n_scenes independent scenes; scene k holds n_k ~ U{n_min..n_max}
    bodies, each a cube (half-edge r/sqrt(3)) or an icosphere, 50/50, with
    r ~ U[0.05,0.1], random rotation, on 10x10 layers at spacing 0.25 with
    jitter U[-0.02,0.02]^3, above one fixed 3x3 m ground quad.  Draw order:
    all n_k first, then per scene per body: shape coin, radius, rotation
    axis (3), angle, jitter (3)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_min, n_max + 1, size=n_scenes)
    sv, st = meshes.icosphere(2, 1.0)
    cv, ct = meshes.cube(0.5)
    gv, gt = meshes.ground_quad(3.0)
    sb = SceneBuilder()
    x0 = -0.25 * 4.5
    for s in range(n_scenes):
        sb.add(gv, gt, fixed=True, scene=s)
        for b in range(int(ns[s])):
            is_cube = rng.uniform() < 0.5
            r = rng.uniform(0.05, 0.1)
            R = random_rotation(rng, math.pi)
            jit = rng.uniform(-0.02, 0.02, size=3)
            layer, rem = divmod(b, 100)
            i, k = divmod(rem, 10)
            p = np.array([x0 + 0.25 * i, 0.3 + 0.25 * layer, x0 + 0.25 * k]) + jit
            if is_cube:
                sb.add(cv * (2.0 * r / math.sqrt(3.0)), ct, R=R, p=p, scene=s)
            else:
                sb.add(sv * r, st, R=R, p=p, scene=s)
    scene = sb.build()
    # kappa_b and the Newton tolerance as in the icosphere box (same bodies,
    # same drop heights; 1e-2 of a scene's box diagonal per second)
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=70.0, mu=0.0, steps=100,
                            newton_tol=1e-2 * math.sqrt(3.0 ** 2 + 3.0 ** 2 + 0.65 ** 2), max_newton=500,
                            pcg_rtol=1e-2)
    return scene, params


def sub_scene(S, k):
    """Scene k of a batched scene dict as a scene of its own (index ranges
    cut out and renumbered; no arithmetic on positions)."""
    b0, b1 = int(S["scene_body_off"][k]), int(S["scene_body_off"][k + 1])
    v0, v1 = int(S["body_vert_off"][b0]), int(S["body_vert_off"][b1])
    t0, t1 = int(S["body_tri_off"][b0]), int(S["body_tri_off"][b1])
    e0, e1 = int(S["body_edge_off"][b0]), int(S["body_edge_off"][b1])
    nb = b1 - b0
    return dict(
        xbar=np.ascontiguousarray(S["xbar"][v0:v1]),
        vert_body=(S["vert_body"][v0:v1] - b0).astype(np.int32),
        tris=np.ascontiguousarray(S["tris"][t0:t1] - v0).astype(np.int32),
        tri_body=(S["tri_body"][t0:t1] - b0).astype(np.int32),
        edges=np.ascontiguousarray(S["edges"][e0:e1] - v0).astype(np.int32),
        edge_body=(S["edge_body"][e0:e1] - b0).astype(np.int32),
        body_vert_off=(S["body_vert_off"][b0:b1 + 1] - v0).astype(np.int32),
        body_tri_off=(S["body_tri_off"][b0:b1 + 1] - t0).astype(np.int32),
        body_edge_off=(S["body_edge_off"][b0:b1 + 1] - e0).astype(np.int32),
        body_fixed=S["body_fixed"][b0:b1].copy(),
        body_scene=np.zeros(nb, np.int32),
        scene_body_off=np.array([0, nb], np.int32),
        density=S["density"][b0:b1].copy(),
        q0=np.ascontiguousarray(S["q0"][b0:b1]),
        qd0=np.ascontiguousarray(S["qd0"][b0:b1]),
    )


def adjoint_drop(seed=5):
    """500 icospheres as the box drop (10x5x10), friction 0.5, plus a target
    point U(box interior, y in [0.1,0.5]).  Draw order: the scene as in
    icosphere_box with this seed, then the target (x, y, z)."""
    scene, params = icosphere_box(seed=seed, n_side=10, n_layers=5, friction=0.5)
    rng = np.random.default_rng(seed + 1000)
    target = np.array([rng.uniform(-1.2, 1.2), rng.uniform(0.1, 0.5), rng.uniform(-1.2, 1.2)])
    params = dict(params, steps=100, checkpoint_every=10)
    return scene, params, target


def icosphere_resting_layer(seed=2, dhat=1e-3):
    """The bottom layer (10x10) of the icosphere box drop with each sphere
    lowered until its lowest mesh vertex sits U[0.2,0.8] dhat above the
    floor: a contact sample of the same workload.  Draw order: as
    icosphere_box for the 100 spheres, then one height fraction per sphere."""
    scene, params = icosphere_box(seed=seed, n_layers=1)
    rng = np.random.default_rng(seed + 77)
    q = scene["q0"]
    for b in range(1, len(q)):
        sl = slice(scene["body_vert_off"][b], scene["body_vert_off"][b + 1])
        A = q[b, 3:].reshape(3, 3)
        low = (scene["xbar"][sl] @ A.T)[:, 1].min()
        q[b, 1] = rng.uniform(0.2, 0.8) * dhat - low
    return scene, params


def landed(scene, seed, dhat=1e-3, v_impact=1.0, layer=0.125):
    """A copy of `scene` whose lowest layer of free bodies (centres within
    `layer` of the lowest free centre height) is lowered until each body's
    lowest mesh vertex sits U[0.2,0.8] dhat above the ground plane y = 0 and
    moves down at v_impact: the moment a layer lands, as a positions-only
    contact state.  Draw order: one height fraction per lowered body, in
    body order."""
    rng = np.random.default_rng(seed)
    S = dict(scene)
    q = scene["q0"].copy()
    qd = scene["qd0"].copy()
    free = np.flatnonzero(scene["body_fixed"] == 0)
    y0 = q[free, 1].min()
    for b in free:
        if q[b, 1] > y0 + layer:
            continue
        sl = slice(scene["body_vert_off"][b], scene["body_vert_off"][b + 1])
        low = (scene["xbar"][sl] @ q[b, 3:].reshape(3, 3).T)[:, 1].min()
        q[b, 1] = rng.uniform(0.2, 0.8) * dhat - low
        qd[b, 1] = -v_impact
    S["q0"], S["qd0"] = q, qd
    return S


def cube_on_slope(theta, mu, v0=1.0, gap=5e-4, ground=40.0):
    """A unit cube (side 1 m, 1000 kg) resting gap above a fixed ground quad,
    with gravity tilted by theta about z so that the ground is an inclined
    plane of slope theta falling towards +x; the cube starts sliding down
    the slope at v0.  No random draws."""
    v, t = meshes.cube(0.5)
    gv, gt = meshes.ground_quad(ground)
    sb = SceneBuilder()
    sb.add(gv, gt, fixed=True)
    qd = np.zeros(12)
    qd[0] = v0
    sb.add(v, t, p=(-ground / 4.0, 0.5 + gap, 0.0), qd=qd)
    g = 9.8
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=80.0, mu=mu,
                            gravity=(g * math.sin(theta), -g * math.cos(theta), 0.0))
    return sb.build(), params


def tet_over_ground(a=0.5, height=3e-4, v0=0.0, ground=10.0):
    """A right-corner tetrahedron (body frame: the corner at the origin, legs
    a along x, y and z; density 1000) with its x-z face parallel to a large
    fixed ground triangle at y = 0, that face `height` above it and the
    corner at x = z = 0; moving down at v0.  The ground is one triangle
    reaching `ground` from the origin.  No randomness."""
    v = np.array([[0.0, 0.0, 0.0], [a, 0.0, 0.0], [0.0, a, 0.0], [0.0, 0.0, a]])
    t = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
    g = np.array([[-ground, 0.0, -ground], [-ground, 0.0, 2 * ground], [2 * ground, 0.0, -ground]])
    sb = SceneBuilder()
    sb.add(g, np.array([[0, 1, 2]], np.int32), fixed=True)
    qd = np.zeros(12)
    qd[1] = -v0
    sb.add(v, t, p=(0.0, height, 0.0), qd=qd)
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=10.0, mu=0.0, newton_tol=1e-6, pcg_rtol=1e-12)
    return sb.build(), params


def cube_lattice(seed=6, n=10, half=0.05, gap_range=(2e-4, 5e-4), tilt=2e-4, jitter=1e-5):
    """n x n x n cubes (half-edge `half`, 1 kg at the default size) on an
    axis-aligned lattice whose planes are `gap_range` apart (one gap per
    plane and axis), so that every interior cube has 26 neighbours (6 across
    faces, 12 across edges, 8 across corners) closer than sqrt(3) times the
    largest gap; each cube tilted by at most `tilt` and shifted by at most
    `jitter` per axis.  The bottom layer is fixed.  A dense, multi-block
    contact state for the solver: no free fall, every body in contact.
    Draw order: the n-1 gaps between x planes, then y planes, then z planes;
    then per cube (y-layer-major, then x, then z): tilt axis (3), tilt
    angle, jitter (3)."""
    rng = np.random.default_rng(seed)
    v, t = meshes.cube(half)
    gaps = [rng.uniform(*gap_range, size=n - 1) for _ in range(3)]
    coords = [np.concatenate([[0.0], np.cumsum(2 * half + g)]) for g in gaps]
    coords = [c - c.mean() for c in coords]
    sb = SceneBuilder()
    for j in range(n):
        for i in range(n):
            for k in range(n):
                R = random_rotation(rng, tilt)
                jit = rng.uniform(-jitter, jitter, size=3)
                p = np.array([coords[0][i], coords[1][j] + half + 0.1, coords[2][k]]) + jit
                sb.add(v, t, R=R, p=p, fixed=(j == 0))
    scene = sb.build()
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=70.0, mu=0.0, newton_tol=1e-5)
    return scene, params


def icosphere_fcc(seed=7, cells=(5, 10, 5), radius=0.06, gap=5e-5):
    """Icospheres (subdivision 2) of one radius on a face-centred cubic
    lattice (4 spheres per cubic cell, 12 nearest neighbours) whose centres
    are 2 radius + gap apart, with random rotations.  Every mesh vertex lies
    on its sphere, so meshes of neighbours are at least `gap` apart, and a
    pair comes within dhat where vertices of both meshes point at each
    other.  The bottom layer (lowest centre height) is fixed.  Draw order
    per sphere (cells x-major, then y, then z; four sites per cell): rotation
    axis (3), angle."""
    rng = np.random.default_rng(seed)
    sv, st = meshes.icosphere(2, radius)
    a = math.sqrt(2.0) * (2.0 * radius + gap)
    sites = ((0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))
    centres = []
    for ix in range(cells[0]):
        for iy in range(cells[1]):
            for iz in range(cells[2]):
                for sx, sy, sz in sites:
                    centres.append(((ix + sx) * a, (iy + sy) * a, (iz + sz) * a))
    centres = np.array(centres)
    centres -= centres.mean(0)
    centres[:, 1] += 1.0
    ylow = centres[:, 1].min()
    sb = SceneBuilder()
    for c in centres:
        R = random_rotation(rng, math.pi)
        sb.add(sv, st, R=R, p=c, fixed=bool(c[1] == ylow))
    scene = sb.build()
    params = default_params(dt=1e-2, dhat=1e-3, kappa_b=70.0, mu=0.0, newton_tol=1e-5)
    return scene, params


CONFIGS = {
    "three_cubes": three_cubes,
    "wrecking_ball": wrecking_ball,
    "icosphere_box": icosphere_box,
    "torus_chains": torus_chains,
    "batched_drops": batched_drops,
}


# --------------------------------------------------------------------------
# Small scenes for parity tests
# --------------------------------------------------------------------------

def near_contact_cubes(seed, n=6, gap_range=(1e-4, 6e-4), tilt=3e-4):
    """n unit-ish cubes in a vertical stack, face gaps drawn in gap_range,
    small tilts and spins so that vertex-face, edge-edge and degenerate
    configurations all occur within dhat=1e-3.  Bottom cube fixed.  Draw
    order per cube above the first: gap, spin angle about y, tilt axis
    (3), tilt angle, horizontal offset (2)."""
    rng = np.random.default_rng(seed)
    v, t = meshes.cube(0.5)
    sb = SceneBuilder()
    sb.add(v, t, fixed=True)
    top = 0.5
    for _ in range(n - 1):
        g = rng.uniform(*gap_range)
        spin = _rot((0.0, 1.0, 0.0), rng.uniform(0, 2 * math.pi))
        R = random_rotation(rng, tilt) @ spin
        off = rng.uniform(-0.3, 0.3, size=2)
        w = v @ R.T
        y = top + g - w[:, 1].min()
        sb.add(v, t, R=R, p=(off[0], y, off[1]))
        top = y + w[:, 1].max()
    return sb.build()


def triangle_soup(seed, n_bodies=24, extent=0.02, tri_size=0.01):
    """Free single-triangle bodies (3 vertices, 1 triangle, 3 edges) with
    random vertices in a small box, so that every point-triangle and
    edge-edge distance case is exercised at distances around dhat=1e-3.
    Bodies are placed on a line with random jitter.  Draw order per body:
    3 vertices (9 uniforms), body offset (3)."""
    rng = np.random.default_rng(seed)
    sb = SceneBuilder()
    for b in range(n_bodies):
        v = rng.uniform(-tri_size, tri_size, size=(3, 3))
        off = rng.uniform(-extent, extent, size=3)
        sb.add(v, np.array([[0, 1, 2]], np.int32), p=off)
    return sb.build()


def random_state(scene, seed, rot_angle=0.0, stretch=0.0, shift=0.0):
    """Perturb q0 of the free bodies: A <- (I + stretch*G) R A with R a random
    rotation of angle <= rot_angle, G Gaussian; p <- p + shift*N(0,1).
    Draw order per free body: rotation (4), G (9), shift (3)."""
    rng = np.random.default_rng(seed)
    q = scene["q0"].copy()
    for b in range(len(q)):
        if scene["body_fixed"][b]:
            continue
        R = random_rotation(rng, rot_angle)
        G = rng.normal(size=(3, 3))
        A = q[b, 3:].reshape(3, 3)
        A = (np.eye(3) + stretch * G) @ R @ A
        q[b, 3:] = A.reshape(9)
        q[b, :3] += shift * rng.normal(size=3)
    return q

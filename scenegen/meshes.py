"""Triangle-mesh builders for the synthetic scenes.

Pure geometry construction (vertex lists, triangle index lists, edge lists);
nothing here evaluates the simulation method.  Closed meshes are oriented
with outward normals (counter-clockwise seen from outside), the open box
with normals facing its interior.
"""
import numpy as np


def edges_from_tris(tris):
    """Unique undirected edges of a triangle list, as (i<j) rows sorted
    lexicographically."""
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def cube(half=0.5):
    """Axis-aligned cube centred at the origin: 8 vertices, 12 triangles
    (one diagonal per face, always from the face's first to third corner),
    18 edges."""
    h = float(half)
    v = np.array([[-h, -h, -h], [h, -h, -h], [h, h, -h], [-h, h, -h],
                  [-h, -h, h], [h, -h, h], [h, h, h], [-h, h, h]], dtype=np.float64)
    quads = [
        (0, 3, 2, 1),  # z = -h, normal -z
        (4, 5, 6, 7),  # z = +h, normal +z
        (0, 1, 5, 4),  # y = -h, normal -y
        (3, 7, 6, 2),  # y = +h, normal +y
        (0, 4, 7, 3),  # x = -h, normal -x
        (1, 2, 6, 5),  # x = +h, normal +x
    ]
    tris = []
    for a, b, c, d in quads:
        tris.append((a, b, c))
        tris.append((a, c, d))
    tris = np.array(tris, dtype=np.int32)
    return v, tris


def icosphere(subdiv=2, radius=1.0):
    """Icosphere by repeated 1-to-4 midpoint subdivision of the regular
    icosahedron, vertices pushed to the sphere after each level.
    subdiv=2 gives 162 vertices, 320 triangles, 480 edges."""
    t = (1.0 + np.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    v = np.array(verts, dtype=np.float64) * float(radius)
    f = np.array(faces, dtype=np.int32)
    return v, f


def torus(major, minor, n_major=200, n_minor=50, straight=0.0):
    """Torus about the local y axis (ring in the x-z plane):
    n_major*n_minor vertices, 2*n_major*n_minor triangles.  With
    straight > 0 the ring is a stadium (a chain link): the half with x > 0
    is moved by straight/2 along +x and the other half by straight/2 along
    -x, so two straight tube sections of that length join the halves (the
    meridians at u = pi/2 and 3 pi/2 belong to the +x half)."""
    i = np.arange(n_major)
    j = np.arange(n_minor)
    u = 2.0 * np.pi * i / n_major
    w = 2.0 * np.pi * j / n_minor
    uu, ww = np.meshgrid(u, w, indexing="ij")
    rr = major + minor * np.cos(ww)
    side = np.where((4 * i <= n_major) | (4 * i >= 3 * n_major), 0.5, -0.5)
    x = rr * np.cos(uu) + straight * side[:, None]
    z = rr * np.sin(uu)
    y = minor * np.sin(ww)
    v = np.stack([x, y, z], axis=-1).reshape(-1, 3)

    def vid(a, b):
        return (a % n_major) * n_minor + (b % n_minor)

    tris = []
    for a in range(n_major):
        for b in range(n_minor):
            v00, v10 = vid(a, b), vid(a + 1, b)
            v01, v11 = vid(a, b + 1), vid(a + 1, b + 1)
            tris.append((v00, v01, v11))
            tris.append((v00, v11, v10))
    return v, np.array(tris, dtype=np.int32)


def open_box(inner, height):
    """Open-top box: a 2x2-quad floor at y=0 and four walls of 2x1 quads,
    inner side length `inner`, wall height `height` (17 vertices,
    24 triangles, 40 edges).  Normals face the interior."""
    h = inner / 2.0
    xs = [-h, 0.0, h]
    verts = {}
    vlist = []

    def vid(p):
        key = tuple(round(c, 12) for c in p)
        if key not in verts:
            verts[key] = len(vlist)
            vlist.append(p)
        return verts[key]

    tris = []

    def quad(a, b, c, d):
        # a,b,c,d counter-clockwise seen from the inside of the box
        tris.append((vid(a), vid(b), vid(c)))
        tris.append((vid(a), vid(c), vid(d)))

    # floor, normal +y
    for i in range(2):
        for k in range(2):
            x0, x1 = xs[i], xs[i + 1]
            z0, z1 = xs[k], xs[k + 1]
            quad((x0, 0.0, z0), (x0, 0.0, z1), (x1, 0.0, z1), (x1, 0.0, z0))
    H = height
    for i in range(2):
        a0, a1 = xs[i], xs[i + 1]
        # wall z=-h, normal +z
        quad((a0, 0.0, -h), (a1, 0.0, -h), (a1, H, -h), (a0, H, -h))
        # wall z=+h, normal -z
        quad((a1, 0.0, h), (a0, 0.0, h), (a0, H, h), (a1, H, h))
        # wall x=-h, normal +x
        quad((-h, 0.0, a1), (-h, 0.0, a0), (-h, H, a0), (-h, H, a1))
        # wall x=+h, normal -x
        quad((h, 0.0, a0), (h, 0.0, a1), (h, H, a1), (h, H, a0))
    return np.array(vlist, dtype=np.float64), np.array(tris, dtype=np.int32)


def ground_quad(size):
    """One square quad at y=0 of side `size` (4 vertices, 2 triangles,
    5 edges), normal +y."""
    h = size / 2.0
    v = np.array([[-h, 0, -h], [-h, 0, h], [h, 0, h], [h, 0, -h]], dtype=np.float64)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return v, t

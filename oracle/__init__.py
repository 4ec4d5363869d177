"""CPU reference ("oracle") of the affine-body contact path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark, never by the product package.  It
shares no code with the GPU library.  Per-pair and per-body arithmetic lives
in ``abd_oracle.cpp`` (plain FP64 loops); this module marshals arrays, solves
the Newton system with a sparse direct solver (SciPy's SuperLU, used as a
library primitive) and runs the Newton loop and time step.

Paper passages followed (Lan et al., Affine Body Dynamics):
  kinematics            sec. 3, Eq. kinematic / kinematic-vel
  mass matrix           sec. 3.1, Eq. mass
  orthogonality         sec. 3.2, Eq. orthogonality, ortho-energy, ortho-poly
  incremental potential sec. 4 (per-body IP and q-tilde)
  barrier               sec. 4, Eq. barrier, Eq. clamped-b
  CCD                   sec. 4.1 (linear trajectories, additive CCD)
  culling               sec. 4.2 (box predicate; i-AABB is an exact filter)
  assembly              sec. 4.3 (J^T H J into 12x12 body blocks)
  friction              sec. 4, V_F (IPC's lagged model: normal force,
                        closest points and tangent basis fixed at q^t)
  adjoint               the conclusion's (sec. 6) claim of differentiability,
                        made concrete by the implicit function theorem on
                        the time step's optimality condition
Readings where the paper is silent (IPC / ACCD conventions, distance case
tie-breaks, mollifier, line search, convergence) are listed in the
project's design notes and restated at each function.
"""
import ctypes
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_int = ctypes.POINTER(ctypes.c_int)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        src = os.path.join(_HERE, "abd_oracle.cpp")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = ctypes.CDLL(path)
        L.ora_mass.argtypes = [ctypes.c_int, _i32, _i32, _d, _d, _u8, _d, _d]
        L.ora_vertex_map.argtypes = [ctypes.c_int, _d, _i32, _d, _d]
        L.ora_candidates.argtypes = [ctypes.c_int] * 4 + [_i32] * 5 + [_u8, _i32, _d, _d, ctypes.c_double,
                                                                       _i32, ctypes.c_int64, _i64, _i32,
                                                                       ctypes.c_int64, _i64]
        L.ora_candidates.restype = ctypes.c_int
        L.ora_classify.argtypes = [ctypes.c_int64, ctypes.c_int, _i32, _i32, _i32, _d, ctypes.c_double, _u8, _d, _u8]
        L.ora_barrier.argtypes = [ctypes.c_int64, ctypes.c_int, _i32, _i32, _i32, _i32, _u8, _d, _d,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, _d, _d, _d, _d, _i32,
                                  ctypes.c_int64, _d, _d]
        L.ora_barrier.restype = ctypes.c_int64
        L.ora_barrier_energy.argtypes = [ctypes.c_int64, ctypes.c_int, _i32, _i32, _i32, _d, _d,
                                         ctypes.c_double, ctypes.c_double, _int]
        L.ora_barrier_energy.restype = ctypes.c_double
        L.ora_ccd.argtypes = [ctypes.c_int64, ctypes.c_int, _i32, _i32, _i32, _d, _d, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, _d, _i32]
        L.ora_orthogonality.argtypes = [ctypes.c_int, _u8, _d, _d, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, _d, _d, _d]
        L.ora_orthogonality_energy.argtypes = [ctypes.c_int, _u8, _d, _d, ctypes.c_double, ctypes.c_double]
        L.ora_orthogonality_energy.restype = ctypes.c_double
        L.ora_friction_lag.argtypes = [ctypes.c_int64, ctypes.c_int, _i32, _i32, _i32, _d, _d, ctypes.c_double,
                                       ctypes.c_double, _d, _d, _d]
        L.ora_friction.argtypes = [ctypes.c_int64, ctypes.c_int, _i32, _i32, _i32, _i32, _u8, _d, _d, _d, _d, _d,
                                   _d, ctypes.c_double, ctypes.c_double, _d, _d, _d, _d, _i32, ctypes.c_int64,
                                   ctypes.c_int]
        L.ora_friction.restype = ctypes.c_int64
        L.ora_friction_lag_vjp.argtypes = [ctypes.c_int64, ctypes.c_int, _i32, _i32, _i32, _i32, _u8, _d, _d, _d, _d,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _d,
                                           _d]
        L.ora_psd_project.argtypes = [ctypes.c_int, _d]
        L.ora_pair_local.argtypes = [ctypes.c_int, _d, _d, ctypes.c_double, ctypes.c_double, _d, _d, _d]
        L.ora_pair_local.restype = ctypes.c_int
        L.ora_pair_distance.argtypes = [ctypes.c_int, _d, _int]
        L.ora_pair_distance.restype = ctypes.c_double
        L.ora_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def threads():
    """Threads the oracle's parallel loops use."""
    return int(lib().ora_threads())


def _p(a, t):
    return a.ctypes.data_as(t)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class NotConverged(RuntimeError):
    pass


class LineSearchFailed(RuntimeError):
    pass


class Intersection(RuntimeError):
    pass


# ----------------------------------------------------------------- body ----

def mass_properties(S):
    """(mass[nb,10], volume[nb]): m, first moment (3), second moment
    (xx,xy,xz,yy,yz,zz) per body by the divergence theorem."""
    nb = len(S["body_fixed"])
    mass = np.zeros((nb, 10))
    vol = np.zeros(nb)
    lib().ora_mass(nb, _p(_c(S["body_tri_off"], np.int32), _i32), _p(_c(S["tris"], np.int32), _i32),
                   _p(_c(S["xbar"], np.float64), _d), _p(_c(S["density"], np.float64), _d),
                   _p(_c(S["body_fixed"], np.uint8), _u8), _p(mass, _d), _p(vol, _d))
    return mass, vol


def mass_matrix(mass):
    """Generalized mass matrix per body (Eq. mass), M = int rho J^T J with
    J = [I_3 | I_3 (x) xbar^T] in q = (p, a1, a2, a3) order: M[p_i,p_j] = m
    delta_ij, M[p_i, a_jn] = delta_ij h_n, M[a_im, a_jn] = delta_ij S_mn."""
    nb = len(mass)
    M = np.zeros((nb, 12, 12))
    m, h = mass[:, 0], mass[:, 1:4]
    Sm = np.zeros((nb, 3, 3))
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for k, (i, j) in enumerate(iu):
        Sm[:, i, j] = mass[:, 4 + k]
        Sm[:, j, i] = mass[:, 4 + k]
    for i in range(3):
        M[:, i, i] = m
        for n in range(3):
            M[:, i, 3 + 3 * i + n] = h[:, n]
            M[:, 3 + 3 * i + n, i] = h[:, n]
            for mm in range(3):
                M[:, 3 + 3 * i + mm, 3 + 3 * i + n] = Sm[:, mm, n]
    return M


def vertex_map(S, q):
    nv = len(S["xbar"])
    x = np.empty((nv, 3))
    lib().ora_vertex_map(nv, _p(_c(S["xbar"], np.float64), _d), _p(_c(S["vert_body"], np.int32), _i32),
                         _p(_c(q, np.float64), _d), _p(x, _d))
    return x


# ---------------------------------------------------------- collisions ----

def candidates(S, x0, x1=None, inflate=1e-3):
    """Sorted PT (v,t) and EE (e_lo,e_hi) candidate pairs of the box
    predicate over the swept boxes of x0 -> x1 inflated by `inflate`."""
    L = lib()
    nb = len(S["body_fixed"])
    args = [nb, len(S["xbar"]), len(S["tris"]), len(S["edges"]),
            _p(_c(S["body_vert_off"], np.int32), _i32), _p(_c(S["body_tri_off"], np.int32), _i32),
            _p(_c(S["body_edge_off"], np.int32), _i32), _p(_c(S["tris"], np.int32), _i32),
            _p(_c(S["edges"], np.int32), _i32), _p(_c(S["body_fixed"], np.uint8), _u8),
            _p(_c(S["body_scene"], np.int32), _i32)]
    x0 = _c(x0, np.float64)
    x1 = x0 if x1 is None else _c(x1, np.float64)
    cap_pt = cap_ee = 1 << 16
    while True:
        pt = np.empty((cap_pt, 2), np.int32)
        ee = np.empty((cap_ee, 2), np.int32)
        npt = ctypes.c_int64(0)
        nee = ctypes.c_int64(0)
        rc = L.ora_candidates(*args, _p(x0, _d), _p(x1, _d), float(inflate), _p(pt, _i32), cap_pt,
                              ctypes.byref(npt), _p(ee, _i32), cap_ee, ctypes.byref(nee))
        if rc == 0:
            return pt[:npt.value].copy(), ee[:nee.value].copy()
        cap_pt = max(cap_pt, npt.value)
        cap_ee = max(cap_ee, nee.value)


def classify(S, x, pairs, is_ee, dhat):
    """Per pair: distance case code, squared distance, active flag."""
    n = len(pairs)
    ty = np.zeros(n, np.uint8)
    d2 = np.zeros(n)
    act = np.zeros(n, np.uint8)
    if n:
        lib().ora_classify(n, int(is_ee), _p(_c(pairs, np.int32), _i32), _p(_c(S["tris"], np.int32), _i32),
                           _p(_c(S["edges"], np.int32), _i32), _p(_c(x, np.float64), _d), float(dhat),
                           _p(ty, _u8), _p(d2, _d), _p(act, _u8))
    return ty, d2, act


def off_keys(S, pt, ee):
    """Sorted unique body pairs (a<b, both free) touched by candidate pairs
    and by joints between two bodies: the off-diagonal block pattern of the
    global Hessian (sec. 4.3)."""
    vb, tb, eb, fx = S["vert_body"], S["tri_body"], S["edge_body"], S["body_fixed"]
    a = np.concatenate([vb[pt[:, 0]], eb[ee[:, 0]]]) if len(pt) + len(ee) else np.zeros(0, np.int64)
    b = np.concatenate([tb[pt[:, 1]], eb[ee[:, 1]]]) if len(pt) + len(ee) else np.zeros(0, np.int64)
    jb = S.get("joint_body")
    if jb is not None and len(jb):
        jb = np.asarray(jb)[np.asarray(jb)[:, 1] >= 0]
        a = np.concatenate([a, jb[:, 0]]).astype(np.int64)
        b = np.concatenate([b, jb[:, 1]]).astype(np.int64)
    keep = (fx[a] == 0) & (fx[b] == 0)
    lo = np.minimum(a, b)[keep].astype(np.int64)
    hi = np.maximum(a, b)[keep].astype(np.int64)
    k = np.unique(lo * (1 << 32) + hi)
    return np.stack([k >> 32, k & 0xFFFFFFFF], axis=1).astype(np.int32) if len(k) else np.zeros((0, 2), np.int32)


def barrier(S, x, pt, ee, params, keys, project=True, local=False):
    """Barrier energy, body gradient [nb,12], diagonal blocks [nb,144],
    off-diagonal blocks [len(keys),144] and active count."""
    nb = len(S["body_fixed"])
    e = np.zeros(1)
    g = np.zeros((nb, 12))
    D = np.zeros((nb, 144))
    O = np.zeros((max(len(keys), 1), 144))
    keys = _c(keys, np.int32)
    out = {}
    n_act = 0
    for is_ee, pairs in ((0, pt), (1, ee)):
        n = len(pairs)
        lg = np.zeros((n, 12)) if local else None
        lH = np.zeros((n, 144)) if local else None
        if n:
            r = lib().ora_barrier(n, is_ee, _p(_c(pairs, np.int32), _i32), _p(_c(S["vert_body"], np.int32), _i32),
                                  _p(_c(S["tris"], np.int32), _i32), _p(_c(S["edges"], np.int32), _i32),
                                  _p(_c(S["body_fixed"], np.uint8), _u8), _p(_c(S["xbar"], np.float64), _d),
                                  _p(_c(x, np.float64), _d), float(params["dhat"]), float(params["kappa_b"]),
                                  int(project), _p(e, _d), _p(g, _d), _p(D, _d), _p(O, _d), _p(keys, _i32),
                                  len(keys), _p(lg, _d) if local else None, _p(lH, _d) if local else None)
            if r == -3:
                raise Intersection("pair at zero distance")
            if r < 0:
                raise RuntimeError("off-diagonal key missing")
            n_act += r
        if local:
            out["ee" if is_ee else "pt"] = (lg, lH)
    res = dict(energy=e[0], grad=g, diag=D, off=O[:len(keys)], n_active=n_act)
    if local:
        res["local"] = out
    return res


def barrier_energy(S, x, pt, ee, params):
    tot = 0.0
    st = ctypes.c_int(0)
    for is_ee, pairs in ((0, pt), (1, ee)):
        if len(pairs):
            tot += lib().ora_barrier_energy(len(pairs), is_ee, _p(_c(pairs, np.int32), _i32),
                                            _p(_c(S["tris"], np.int32), _i32), _p(_c(S["edges"], np.int32), _i32),
                                            _p(_c(S["xbar"], np.float64), _d), _p(_c(x, np.float64), _d),
                                            float(params["dhat"]), float(params["kappa_b"]), ctypes.byref(st))
            if st.value:
                return np.inf
    return tot


def ccd(S, x, dx, pt, ee, params, iters=None):
    """Per-pair additive-CCD safe fractions and alpha_max = min(1, min t).
    If `iters` is a list, the per-pair advance counts are appended to it."""
    out = []
    for is_ee, pairs in ((0, pt), (1, ee)):
        t = np.ones(len(pairs)) * params["ccd_tmax"]
        it = np.zeros(len(pairs), np.int32)
        if len(pairs):
            lib().ora_ccd(len(pairs), is_ee, _p(_c(pairs, np.int32), _i32), _p(_c(S["tris"], np.int32), _i32),
                          _p(_c(S["edges"], np.int32), _i32), _p(_c(x, np.float64), _d),
                          _p(_c(dx, np.float64), _d), float(params["ccd_s"]), float(params["ccd_tmax"]),
                          int(params["ccd_max_iter"]), _p(t, _d), _p(it, _i32))
        out.append(t)
        if iters is not None:
            iters.append(it)
    alpha = min([1.0] + [float(t.min()) for t in out if len(t)])
    return out[0], out[1], alpha


# ------------------------------------------------------------- friction ----

def friction_lag(S, xt, pt, ee, params, keep_inactive=False):
    """Lagged friction state at the step start x^t (sec. 4, V_F; IPC's lagged
    model): per active pair lambda = -kappa m B'(d), tangent basis T (6) and
    closest-point weights w (4).  Inactive pairs are dropped unless
    keep_inactive."""
    out = {}
    for is_ee, pairs, nm in ((0, pt, "pt"), (1, ee, "ee")):
        n = len(pairs)
        lam = np.zeros(n)
        T = np.zeros((n, 6))
        w = np.zeros((n, 4))
        if n:
            lib().ora_friction_lag(n, is_ee, _p(_c(pairs, np.int32), _i32), _p(_c(S["tris"], np.int32), _i32),
                                   _p(_c(S["edges"], np.int32), _i32), _p(_c(S["xbar"], np.float64), _d),
                                   _p(_c(xt, np.float64), _d), float(params["dhat"]), float(params["kappa_b"]),
                                   _p(lam, _d), _p(T, _d), _p(w, _d))
        keep = np.ones(n, bool) if keep_inactive else lam > 0
        out[nm] = dict(pairs=_c(pairs, np.int32)[keep], lam=lam[keep], T=T[keep], w=w[keep])
    out["xt"] = np.array(xt, dtype=np.float64)
    return out


def friction(S, x, F, params, keys, hess=True):
    """Friction energy, gradient [nb,12] and Hessian blocks of the lagged
    pairs F at x."""
    nb = len(S["body_fixed"])
    e = np.zeros(1)
    g = np.zeros((nb, 12))
    D = np.zeros((nb, 144))
    O = np.zeros((max(len(keys), 1), 144))
    keys = _c(keys, np.int32)
    eps = params["eps_v"] * params["dt"]
    for is_ee, nm in ((0, "pt"), (1, "ee")):
        f = F[nm]
        n = len(f["pairs"])
        if n == 0:
            continue
        r = lib().ora_friction(n, is_ee, _p(f["pairs"], _i32), _p(_c(S["vert_body"], np.int32), _i32),
                               _p(_c(S["tris"], np.int32), _i32), _p(_c(S["edges"], np.int32), _i32),
                               _p(_c(S["body_fixed"], np.uint8), _u8), _p(_c(S["xbar"], np.float64), _d),
                               _p(_c(x, np.float64), _d), _p(F["xt"], _d), _p(_c(f["lam"], np.float64), _d),
                               _p(_c(f["T"], np.float64), _d), _p(_c(f["w"], np.float64), _d),
                               float(params["mu"]), float(eps), _p(e, _d), _p(g, _d), _p(D, _d), _p(O, _d),
                               _p(keys, _i32), len(keys), int(hess))
        if r < 0:
            raise RuntimeError("off-diagonal key missing for a friction pair")
    return dict(energy=e[0], grad=g, diag=D, off=O[:len(keys)])


def friction_lag_vjp(S, x, F, params, l):
    """J^T grad_{x^t} [ (J l) . g(x; lambda, T, w) ] over the lagged pairs of
    F, the derivative taken through the lagged lambda, T and w only (the
    sliding displacement's own x^t is the friction Hessian's part)."""
    nb = len(S["body_fixed"])
    out = np.zeros((nb, 12))
    l = _c(l, np.float64)
    eps = params["eps_v"] * params["dt"]
    for is_ee, nm in ((0, "pt"), (1, "ee")):
        f = F[nm]
        n = len(f["pairs"])
        if n == 0:
            continue
        lib().ora_friction_lag_vjp(n, is_ee, _p(f["pairs"], _i32), _p(_c(S["vert_body"], np.int32), _i32),
                                   _p(_c(S["tris"], np.int32), _i32), _p(_c(S["edges"], np.int32), _i32),
                                   _p(_c(S["body_fixed"], np.uint8), _u8), _p(_c(S["xbar"], np.float64), _d),
                                   _p(_c(x, np.float64), _d), _p(F["xt"], _d), _p(_c(f["lam"], np.float64), _d),
                                   float(params["mu"]), float(eps), float(params["dhat"]), float(params["kappa_b"]),
                                   _p(l, _d), _p(out, _d))
    return out


def friction_energy(S, x, F, params):
    return friction(S, x, F, params, np.zeros((0, 2), np.int32), hess=False)["energy"]


def _with_friction_pairs(pt, ee, F):
    if F is None:
        return pt, ee
    return (np.concatenate([pt, F["pt"]["pairs"]]).astype(np.int32),
            np.concatenate([ee, F["ee"]["pairs"]]).astype(np.int32))


# ------------------------------------------------------ body potentials ----

def orthogonality(S, vol, q, params, project=True, w=None):
    nb = len(S["body_fixed"])
    w = params["dt"] ** 2 if w is None else w
    e = np.zeros(1)
    g = np.zeros((nb, 12))
    D = np.zeros((nb, 144))
    lib().ora_orthogonality(nb, _p(_c(S["body_fixed"], np.uint8), _u8), _p(_c(vol, np.float64), _d),
                            _p(_c(q, np.float64), _d), float(params["kappa_o"]), float(w), int(project),
                            _p(e, _d), _p(g, _d), _p(D, _d))
    return e[0], g, D


def orthogonality_energy(S, vol, q, params, w=None):
    w = params["dt"] ** 2 if w is None else w
    return lib().ora_orthogonality_energy(len(S["body_fixed"]), _p(_c(S["body_fixed"], np.uint8), _u8),
                                          _p(_c(vol, np.float64), _d), _p(_c(q, np.float64), _d),
                                          float(params["kappa_o"]), float(w))


# Alternative rigidity potentials (sec. 3.2 names ARAP, |A - R(A)|_F^2 with
# A = R S the polar decomposition, and neo-Hookean as alternatives to the
# orthogonality potential).  Reading (the paper gives no constants): both
# scaled like V_perp, kappa_o times the body volume times w (dt^2 in the
# incremental potential); neo-Hookean with Lame parameters mu = lambda =
# kappa_o, Psi = mu/2 (tr A^T A - 3) - mu ln J + lambda/2 (ln J)^2, J = det A,
# infinite for J <= 0; ARAP's R the polar rotation (det R = +1: for
# det A < 0 the SVD's last singular pair is flipped).  Per-body loops with
# numpy's SVD, determinant and inverse as library primitives; the Hessians
# are exact: ARAP's from the polar decomposition's differential (R^T dA =
# W S + dS with W skew and dS symmetric, so W S + S W equals the skew part
# of R^T dA, a 3x3 linear system for W, and dR = R W), neo-Hookean's from
# d(A^-T) = -A^-T dA^T A^-T and d ln J = tr(A^-1 dA).

RIGIDITY = {0: "orthogonality", 1: "arap", 2: "neo-hookean"}


def _polar(A):
    U, sv, Vt = np.linalg.svd(A)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
    R = U @ D @ Vt
    return R, R.T @ A


def _skew_vec(M):
    return np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]]) / 2.0


def _skew_mat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def arap_body(A):
    """Psi = |A - R|^2, its gradient 2 (A - R) and exact Hessian 2 (I - dR/dA)
    (9-vectors and 9x9 in A's row-major order)."""
    R, Sm = _polar(A)
    e = float(np.sum((A - R) ** 2))
    g = 2.0 * (A - R)
    # W S + S W for the three unit skew matrices W
    L = np.stack([_skew_vec(_skew_mat(u) @ Sm + Sm @ _skew_mat(u)) for u in np.eye(3)], 1)
    H = np.zeros((9, 9))
    for k in range(9):
        dA = np.zeros(9)
        dA[k] = 1.0
        dA = dA.reshape(3, 3)
        X = R.T @ dA
        w = np.linalg.solve(L, _skew_vec(X - X.T))
        dR = R @ _skew_mat(w)
        H[:, k] = 2.0 * (dA - dR).reshape(9)
    return e, g.reshape(9), 0.5 * (H + H.T)


def neo_hookean_body(A, mu, lam):
    J = np.linalg.det(A)
    if J <= 0.0:
        return np.inf, np.zeros(9), np.zeros((9, 9))
    lnJ = np.log(J)
    Ait = np.linalg.inv(A).T
    e = 0.5 * mu * (float(np.sum(A * A)) - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ
    P = mu * (A - Ait) + lam * lnJ * Ait
    H = np.zeros((9, 9))
    for k in range(9):
        dA = np.zeros(9)
        dA[k] = 1.0
        dA = dA.reshape(3, 3)
        dAit = -Ait @ dA.T @ Ait
        dlnJ = float(np.sum(Ait * dA))
        dP = mu * (dA - dAit) + lam * dlnJ * Ait + lam * lnJ * dAit
        H[:, k] = dP.reshape(9)
    return e, P.reshape(9), 0.5 * (H + H.T)


def _psd(H):
    lam, V = np.linalg.eigh(H)
    return (V * np.maximum(lam, 0.0)) @ V.T


def rigidity(S, vol, q, params, project=True, w=None):
    """Energy, gradient [nb,12] and diagonal blocks [nb,144] of the body's
    rigidity potential selected by params["rigidity"] (0 orthogonality, the
    paper's V_perp; 1 ARAP; 2 neo-Hookean), times w (default dt^2)."""
    kind = int(params.get("rigidity", 0))
    if kind == 0:
        return orthogonality(S, vol, q, params, project=project, w=w)
    w = params["dt"] ** 2 if w is None else w
    nb = len(S["body_fixed"])
    e = 0.0
    g = np.zeros((nb, 12))
    D = np.zeros((nb, 12, 12))
    k = params["kappa_o"]
    for b in range(nb):
        if S["body_fixed"][b]:
            continue
        A = q[b, 3:].reshape(3, 3)
        eb, gb, Hb = arap_body(A) if kind == 1 else neo_hookean_body(A, 1.0, 1.0)
        c = k * vol[b] * w
        e += c * eb
        g[b, 3:] = c * gb
        D[b, 3:, 3:] = c * (_psd(Hb) if project else Hb)
    return e, g, D.reshape(nb, 144)


def rigidity_energy(S, vol, q, params, w=None):
    kind = int(params.get("rigidity", 0))
    if kind == 0:
        return orthogonality_energy(S, vol, q, params, w=w)
    return rigidity(S, vol, q, params, project=False, w=w)[0]


def inertia(S, M, q, qt):
    """Incremental-potential inertia term 1/2 |q - q~|_M^2 (sec. 4),
    gradient M (q - q~), Hessian M; fixed bodies excluded."""
    free = S["body_fixed"] == 0
    dq = (q - qt) * free[:, None]
    Mq = np.einsum("bij,bj->bi", M, dq)
    e = 0.5 * float(np.sum(dq * Mq))
    D = (M * free[:, None, None]).reshape(-1, 144)
    return e, Mq, D


def q_tilde(S, q, qd, params):
    """q~ = q + dt qdot + dt^2 M^-1 f.  Gravity f = int rho J^T g has
    M^-1 f = (g, 0, 0, 0) exactly, whatever the mass distribution."""
    dt = params["dt"]
    qt = q + dt * qd
    qt[:, :3] += dt * dt * np.asarray(params["gravity"])
    fx = S["body_fixed"] != 0
    qt[fx] = q[fx]
    return qt


# -------------------------------------------------------------- solver ----

def assemble(S, diag, off, keys):
    """Sparse symmetric matrix over the free DOFs from 12x12 blocks."""
    nb = len(S["body_fixed"])
    free = np.flatnonzero(S["body_fixed"] == 0)
    pos = -np.ones(nb, np.int64)
    pos[free] = np.arange(len(free))
    rows, cols, vals = [], [], []
    ii, jj = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")
    for b in free:
        rows.append(12 * pos[b] + ii.ravel())
        cols.append(12 * pos[b] + jj.ravel())
        vals.append(diag[b])
    for k, (a, b) in enumerate(keys):
        if pos[a] < 0 or pos[b] < 0:
            continue
        rows.append(12 * pos[a] + ii.ravel())
        cols.append(12 * pos[b] + jj.ravel())
        vals.append(off[k])
        rows.append(12 * pos[b] + jj.ravel())
        cols.append(12 * pos[a] + ii.ravel())
        vals.append(off[k])
    n = 12 * len(free)
    if not rows:
        return sp.csr_matrix((n, n)), free
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsc()
    return A, free


def solve(S, diag, off, keys, rhs):
    """Direct sparse solve of H p = rhs over free DOFs (fixed: p = 0)."""
    A, free = assemble(S, diag, off, keys)
    p = np.zeros_like(rhs)
    if len(free):
        sol = spla.spsolve(A, rhs[free].reshape(-1))
        p[free] = sol.reshape(-1, 12)
    return p


# -------------------------------------------------------------- Newton ----

class Body:
    """Per-scene constant data of the oracle: mass matrix and volumes."""

    def __init__(self, S):
        self.mass, self.vol = mass_properties(S)
        self.M = mass_matrix(self.mass)


# Joints (sec. 5.3): an affine body's q maps linearly to any virtual
# tetrahedron's vertices (Eq. phi), which are material points p_i = A pbar_i +
# p, so a joint that fixes tetrahedron vertices is a linear equality between
# material points: x_a(q_a) = x_b(q_b) for a point of body a and a point of
# body b, or = c for a fixed world point c (a hinge: two such points on its
# axis, over-constraining as the paper notes).  Reading: enforced by a stiff
# quadratic penalty in the incremental potential, w kappa_j / 2 |x_a - x_b|^2
# per joint (w = dt^2, like the other potentials).  S["joint_body"] [n, 2]
# (b = -1: world), S["joint_point"] [n, 2, 3] (body-frame points; the world
# point in the second slot when b = -1).

def _point_jac(xb):
    J = np.zeros((3, 12))
    J[:, :3] = np.eye(3)
    for i in range(3):
        J[i, 3 + 3 * i:6 + 3 * i] = xb
    return J


def joints(S, q, params, keys, w=None):
    """Energy, gradient [nb,12], diagonal [nb,144] and off-diagonal
    [len(keys),144] blocks of the joint penalties (fixed bodies: no DOFs;
    keys None: no off-diagonal blocks)."""
    nb = len(S["body_fixed"])
    if keys is None:
        keys = np.zeros((0, 2), np.int32)
        off = False
    else:
        off = True
    e, g = 0.0, np.zeros((nb, 12))
    D = np.zeros((nb, 12, 12))
    O = np.zeros((len(keys), 12, 12))
    jb = S.get("joint_body")
    if jb is None or not len(jb):
        return e, g, D.reshape(nb, 144), O.reshape(len(keys), 144)
    c = params["kappa_j"] * (params["dt"] ** 2 if w is None else w)
    kidx = {(int(a), int(b)): i for i, (a, b) in enumerate(keys)}
    fx = S["body_fixed"]
    for (a, b), (pa, pb) in zip(np.asarray(jb), np.asarray(S["joint_point"])):
        Ja = _point_jac(pa)
        xa = Ja @ q[a]
        if b >= 0:
            Jb = _point_jac(pb)
            xb = Jb @ q[b]
        else:
            xb = np.asarray(pb, np.float64)
        r = xa - xb
        e += 0.5 * c * float(r @ r)
        if not fx[a]:
            g[a] += c * Ja.T @ r
            D[a] += c * Ja.T @ Ja
        if b >= 0 and not fx[b]:
            g[b] -= c * Jb.T @ r
            D[b] += c * Jb.T @ Jb
            if off and not fx[a]:
                lo, hi = (a, b) if a < b else (b, a)
                blk = -c * (Ja.T @ Jb if a < b else Jb.T @ Ja)
                O[kidx[(int(lo), int(hi))]] += blk
    return e, g, D.reshape(nb, 144), O.reshape(len(keys), 144)


def total_energy(S, B, q, qt, x, pt, ee, params, F=None):
    e_in, _, _ = inertia(S, B.M, q, qt)
    e = e_in + rigidity_energy(S, B.vol, q, params) + barrier_energy(S, x, pt, ee, params)
    if S.get("joint_body") is not None and len(S["joint_body"]):
        e += joints(S, q, params, None)[0]
    if F is not None:
        e += friction_energy(S, x, F, params)
    return e


def grad_hess(S, B, q, qt, params, x=None, pt=None, ee=None, project=True, F=None):
    """Energy, gradient and (projected) Hessian blocks of the incremental
    potential E = sum_b E_b + V_C (+ the lagged friction potential of F) at q.
    The off-diagonal pattern is that of the candidate pairs and, with
    friction, of the lagged pairs as well."""
    if x is None:
        x = vertex_map(S, q)
    if pt is None:
        pt, ee = candidates(S, x, None, params["dhat"])
    keys = off_keys(S, *_with_friction_pairs(pt, ee, F))
    e_in, g_in, D_in = inertia(S, B.M, q, qt)
    e_o, g_o, D_o = rigidity(S, B.vol, q, params, project=project)
    bar = barrier(S, x, pt, ee, params, keys, project=project)
    e_j, g_j, D_j, O_j = joints(S, q, params, keys)
    out = dict(energy=e_in + e_o + bar["energy"] + e_j, grad=g_in + g_o + bar["grad"] + g_j,
               diag=D_in + D_o + bar["diag"] + D_j, off=bar["off"] + O_j, keys=keys, pt=pt, ee=ee,
               n_active=bar["n_active"])
    if F is not None:
        fr = friction(S, x, F, params, keys)
        out["energy"] += fr["energy"]
        out["grad"] = out["grad"] + fr["grad"]
        out["diag"] = out["diag"] + fr["diag"]
        out["off"] = out["off"] + fr["off"]
    return out


def newton_iteration(S, B, q, qt, params, F=None):
    """One projected-Newton iteration with CCD-filtered backtracking line
    search (IPC's scheme, which ABD builds on):
      p = -H^-1 g;  converged if max_k |J_k p|_inf <= tol_v dt;
      swept candidates over x(q) -> x(q+p); alpha = min(1, min_pairs t_ccd);
      halve alpha until E(q + alpha p) <= E(q).
    F: lagged friction state (friction_lag) or None.
    Returns (q_new, converged, info)."""
    dt = params["dt"]
    x = vertex_map(S, q)
    gh = grad_hess(S, B, q, qt, params, x=x, F=F)
    p = solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    disp = np.abs(vertex_map(S, p)).max() if len(p) else 0.0
    info = dict(n_pt=len(gh["pt"]), n_ee=len(gh["ee"]), n_active=gh["n_active"], disp=disp, p=p,
                grad=gh["grad"], energy=gh["energy"])
    if disp <= params["newton_tol"] * dt:
        return q, True, info
    x1 = vertex_map(S, q + p)
    pts, ees = candidates(S, x, x1, params["dhat"])
    tpt, tee, alpha = ccd(S, x, x1 - x, pts, ees, params)
    e0 = total_energy(S, B, q, qt, x, pts, ees, params, F)
    for _ in range(params["max_ls"]):
        qa = q + alpha * p
        ea = total_energy(S, B, qa, qt, vertex_map(S, qa), pts, ees, params, F)
        if ea <= e0:
            break
        alpha *= 0.5
    else:
        raise LineSearchFailed("line search did not decrease the energy")
    info.update(alpha=alpha, n_pt_swept=len(pts), n_ee_swept=len(ees), e0=e0, e1=ea)
    return q + alpha * p, False, info


# Adaptive barrier stiffness (IPC's rule; the paper writes kappa without a
# value or rule).  Reading, per time step of a single scene (kappa_adaptive
# set; params["kappa_b"] is the floor kappa_min, params["kappa_max"] the
# ceiling):
#  - at q^t, kappa = clamp(-(g_E . g_B) / (g_B . g_B), kappa_min, kappa_max),
#    the kappa that best balances the barrier's gradient g_B (kappa = 1)
#    against the rest of the incremental potential's g_E (inertia, the
#    rigidity potential and joints), both over the free bodies' DOFs;
#    kappa_min when g_B = 0.  It is set before friction is lagged;
#  - before each Newton iteration, with d the smallest distance of an
#    active pair at the iterate and d_prev the previous one (at q^t for the
#    first iteration): kappa doubles, up to kappa_max, when d < eps_d
#    (params["kappa_eps_d"]) and d < d_prev.
# Distances compare as squares (d^2 from the pair classification).

def min_active_d2(S, x, pt, ee, dhat):
    """Smallest squared distance of an active pair (inf when none)."""
    best = np.inf
    for pairs, is_ee in ((pt, 0), (ee, 1)):
        if len(pairs):
            _, d2, act = classify(S, x, pairs, is_ee, dhat)
            if np.any(act):
                best = min(best, float(d2[act != 0].min()))
    return best


def barrier_stiffness_init(S, B, q, qt, params):
    """(kappa, d^2_min) at the start of a time step (rule above)."""
    x = vertex_map(S, q)
    pt, ee = candidates(S, x, None, params["dhat"])
    _, g_in, _ = inertia(S, B.M, q, qt)
    _, g_o, _ = rigidity(S, B.vol, q, params)
    _, g_j, _, _ = joints(S, q, params, None)
    gE = g_in + g_o + g_j
    keys = off_keys(S, pt, ee)
    gB = barrier(S, x, pt, ee, dict(params, kappa_b=1.0), keys)["grad"]
    free = S["body_fixed"] == 0
    gE, gB = gE[free], gB[free]
    den = float(np.sum(gB * gB))
    kmin, kmax = params["kappa_b"], params["kappa_max"]
    kappa = kmin if den == 0.0 else min(max(-float(np.sum(gE * gB)) / den, kmin), kmax)
    return kappa, min_active_d2(S, x, pt, ee, params["dhat"])


def barrier_stiffness_update(kappa, d2, d2_prev, params):
    """Doubling rule before a Newton iteration (rule above)."""
    eps2 = params["kappa_eps_d"] ** 2
    if d2 < eps2 and d2 < d2_prev:
        return min(2.0 * kappa, params["kappa_max"])
    return kappa


def step_friction(S, q, params):
    """Friction state lagged at the step start (None when mu = 0)."""
    if params.get("mu", 0.0) <= 0.0:
        return None
    xt = vertex_map(S, q)
    pt, ee = candidates(S, xt, None, params["dhat"])
    return friction_lag(S, xt, pt, ee, params)


def time_step(S, B, q, qd, params, log=None, lag=None, F_out=None):
    """Implicit-Euler time step: minimise the incremental potential starting
    from q^t; qdot^{t+1} = (q^{t+1} - q^t) / dt.  With mu > 0 the friction
    state is lagged once at q^t; `lag` (a friction state) replaces the lagged
    pairs, lambda, T and w (x^t stays that of q), and F_out (a list)
    receives the state used."""
    qt = q_tilde(S, q, qd, params)
    adaptive = bool(params.get("kappa_adaptive", 0))
    if adaptive:
        if len(np.unique(S["body_scene"])) > 1:
            raise ValueError("the oracle's adaptive barrier stiffness takes one scene")
        kappa, d2_prev = barrier_stiffness_init(S, B, q, qt, params)
        params = dict(params, kappa_b=kappa)
    if lag is not None:
        F = dict(lag, xt=vertex_map(S, q))
    else:
        F = step_friction(S, q, params)
    if F_out is not None:
        F_out.append(F)
    qn = q.copy()
    its = 0
    for its in range(1, params["max_newton"] + 1):
        if adaptive:
            x = vertex_map(S, qn)
            d2 = min_active_d2(S, x, *candidates(S, x, None, params["dhat"]), params["dhat"])
            params = dict(params, kappa_b=barrier_stiffness_update(params["kappa_b"], d2, d2_prev, params))
            d2_prev = d2
        qn, conv, info = newton_iteration(S, B, qn, qt, params, F)
        info["kappa_b"] = params["kappa_b"]
        if log is not None:
            log.append(info)
        if conv:
            break
    else:
        raise NotConverged("Newton did not converge")
    qdn = (qn - q) / params["dt"]
    qdn[S["body_fixed"] != 0] = 0.0
    return qn, qdn, its


# ------------------------------------------------------------- adjoint ----

def _matvec(S, diag, off, keys, v):
    """(diag + off + off^T) v over the free DOFs, v [nb,12]."""
    A, free = assemble(S, diag, off, keys)
    out = np.zeros_like(v)
    out[free] = (A @ v[free].reshape(-1)).reshape(-1, 12)
    return out


def adjoint_step(S, B, q_t, qd_t, q_next, qbar_next, qdbar_next, params, F=None):
    """Reverse mode of one implicit-Euler time step.  q^{t+1} minimises
    E(q; q~, q^t) with q~ = q^t + dt qdot^t + dt^2 M^-1 f, so
    grad_q E(q^{t+1}) = 0; differentiating that condition (implicit
    function theorem) with H the unprojected Hessian of E at q^{t+1}:
      H dq^{t+1} = M dq~ + H_D dq^t,
    H_D the friction Hessian (the friction potential depends on q - q^t
    through u).  With
    qdot^{t+1} = (q^{t+1} - q^t)/dt and a = qbar^{t+1} + qdbar^{t+1}/dt:
      H l = a;  qbar^t = M l + H_D l - qdbar^{t+1}/dt;  qdbar^t = dt M l.
    The lagged lambda, T and w are themselves functions of q^t; their part
    of the mixed derivative is subtracted as well:
      qbar^t -= J^T grad_{x^t} [ (J l) . g_D(x^{t+1}; lambda, T, w) ],
    g_D the friction gradient, the derivative taken through the lag only.
    Fixed bodies carry no adjoint.  Returns (qbar^t, qdbar^t)."""
    dt = params["dt"]
    free = S["body_fixed"] == 0
    qt = q_tilde(S, q_t, qd_t, params)
    Fn = None if F is None else dict(F, xt=vertex_map(S, q_t))
    gh = grad_hess(S, B, q_next, qt, params, project=False, F=Fn)
    a = (qbar_next + qdbar_next / dt) * free[:, None]
    lam = solve(S, gh["diag"], gh["off"], gh["keys"], a)
    Ml = np.einsum("bij,bj->bi", B.M, lam) * free[:, None]
    qbar = Ml - qdbar_next / dt
    if Fn is not None:
        xn = vertex_map(S, q_next)
        fr = friction(S, xn, Fn, params, gh["keys"])
        qbar = qbar + _matvec(S, fr["diag"], fr["off"], gh["keys"], lam)
        qbar = qbar - friction_lag_vjp(S, xn, Fn, params, lam)
    qbar = qbar * free[:, None]
    return qbar, dt * Ml


def rollout(S, B, q0, qd0, params, n_steps, lags=None):
    """Forward simulation: states [(q^0, qd^0), ..., (q^n, qd^n)] and the
    friction state of every step (None without friction).  lags: per-step
    friction states to hold (see time_step)."""
    q, qd = q0.copy(), qd0.copy()
    states, Fs = [(q.copy(), qd.copy())], []
    for t in range(n_steps):
        Fo = []
        q, qd, _ = time_step(S, B, q, qd, params, lag=None if lags is None else lags[t], F_out=Fo)
        states.append((q.copy(), qd.copy()))
        Fs.append(Fo[0])
    return states, Fs


def rollout_grad(S, B, q0, qd0, params, n_steps, qbar_T, qdbar_T):
    """dL/dq^0, dL/dqdot^0 of a loss L(q^n, qdot^n) with the given
    gradients, by adjoint_step from the last step back (fixed barrier
    stiffness only: the adjoint does not differentiate the adaptive rule)."""
    if params.get("kappa_adaptive", 0):
        raise ValueError("the adjoint takes a fixed barrier stiffness")
    states, Fs = rollout(S, B, q0, qd0, params, n_steps)
    qbar, qdbar = qbar_T.copy(), qdbar_T.copy()
    for t in range(n_steps - 1, -1, -1):
        (q_t, qd_t), (q_n, _) = states[t], states[t + 1]
        qbar, qdbar = adjoint_step(S, B, q_t, qd_t, q_n, qbar, qdbar, params, Fs[t])
    return qbar, qdbar, states, Fs


def pair_local(is_ee, X, xb, dhat, kappa):
    """Local barrier energy/gradient/Hessian of one pair of explicit
    vertices X[4,3] (rest positions xb[4,3] for the EE mollifier)."""
    X = _c(X, np.float64).reshape(12)
    xb = _c(xb, np.float64).reshape(12)
    e = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros(144)
    ty = lib().ora_pair_local(int(is_ee), _p(X, _d), _p(xb, _d), float(dhat), float(kappa), _p(e, _d),
                              _p(g, _d), _p(H, _d))
    return ty, e[0], g, H.reshape(12, 12)


def pair_distance(is_ee, X):
    X = _c(X, np.float64).reshape(12)
    ty = ctypes.c_int(0)
    d = lib().ora_pair_distance(int(is_ee), _p(X, _d), ctypes.byref(ty))
    return d, ty.value


def psd_project(H):
    H = _c(H, np.float64).copy()
    n = H.shape[0]
    lib().ora_psd_project(n, _p(H, _d))
    return H

"""MI355X (gfx950) affine-body-dynamics contact path.

Python binding of the C ABI in include/abd.h.  Functions keep the ABI's
names (without the ``abd_`` prefix on methods of ``Context``) and only
marshal arguments: torch tensors provide device memory and the current HIP
stream, every computation runs in libabd.so.  There is no CPU fallback: if
the library or a GPU is missing, calls raise.

Method: Lan et al., Affine Body Dynamics (sec. 3 kinematics and mass,
sec. 3.2 orthogonality, sec. 4 incremental potential and barrier, sec. 4.1
CCD, sec. 4.2 culling, sec. 4.3 assembly).
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import AbdParams, AbdScene, AbdStats  # noqa: F401


class AbdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_params(p):
    """abd_params from a parameter dict (see scenegen.default_params)."""
    out = AbdParams()
    for k in ("dt", "dhat", "kappa_b", "kappa_o", "mu", "eps_v", "newton_tol", "pcg_rtol", "ccd_s", "ccd_tmax"):
        setattr(out, k, float(p[k]))
    for i in range(3):
        out.gravity[i] = float(p["gravity"][i])
    for k in ("ccd_max_iter", "max_newton", "max_pcg", "max_ls"):
        setattr(out, k, int(p[k]))
    out.rigidity = int(p.get("rigidity", 0))
    out.kappa_j = float(p.get("kappa_j", 0.0))
    out.kappa_adaptive = int(p.get("kappa_adaptive", 0))
    out.kappa_max = float(p.get("kappa_max", 100.0 * out.kappa_b))
    out.kappa_eps_d = float(p.get("kappa_eps_d", 0.0))
    return out


class Scene:
    """Device copy of a scene dict (numpy arrays as produced by scenegen)."""

    def __init__(self, S, device="cuda:0"):
        dev = torch.device(device)

        def t(a, dt):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)

        self.device = dev
        self.xbar = t(S["xbar"], torch.float64)
        self.vert_body = t(S["vert_body"], torch.int32)
        self.tris = t(S["tris"], torch.int32)
        self.tri_body = t(S["tri_body"], torch.int32)
        self.edges = t(S["edges"], torch.int32)
        self.edge_body = t(S["edge_body"], torch.int32)
        self.body_vert_off = t(S["body_vert_off"], torch.int32)
        self.body_tri_off = t(S["body_tri_off"], torch.int32)
        self.body_edge_off = t(S["body_edge_off"], torch.int32)
        self.body_fixed = t(S["body_fixed"], torch.uint8)
        self.body_scene = t(S["body_scene"], torch.int32)
        self.density = t(S["density"], torch.float64)
        self.n_bodies = len(S["body_fixed"])
        self.n_scenes = int(S["body_scene"].max()) + 1 if self.n_bodies else 0
        self.mass = torch.zeros((self.n_bodies, 10), dtype=torch.float64, device=dev)
        self.volume = torch.zeros(self.n_bodies, dtype=torch.float64, device=dev)
        jb = S.get("joint_body")
        self.n_joints = 0 if jb is None else len(jb)
        self.joint_body = t(jb, torch.int32) if self.n_joints else None
        self.joint_point = t(S["joint_point"], torch.float64) if self.n_joints else None
        self.c = self._struct()

    def _struct(self):
        s = AbdScene()
        s.n_bodies = self.n_bodies
        s.n_verts = self.xbar.shape[0]
        s.n_tris = self.tris.shape[0]
        s.n_edges = self.edges.shape[0]
        s.n_scenes = self.n_scenes
        for name in ("xbar", "vert_body", "tris", "tri_body", "edges", "edge_body", "body_vert_off", "body_tri_off",
                     "body_edge_off", "body_fixed", "body_scene", "mass", "volume"):
            setattr(s, name, getattr(self, name).data_ptr())
        s.n_joints = self.n_joints
        if self.n_joints:
            s.joint_body = self.joint_body.data_ptr()
            s.joint_point = self.joint_point.data_ptr()
        return s


class Context:
    """An abd_ctx on one device; methods mirror the C ABI calls."""

    def __init__(self, device=0):
        self.L = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the ABD library has no CPU path")
        self.device = device
        torch.cuda.set_device(device)
        h = ctypes.c_void_p()
        self._check(self.L.abd_create(ctypes.byref(h), int(device)), ctx=None)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.abd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ctx="self"):
        if rc != 0:
            msg = self.L.abd_last_error(self.h if ctx else None)
            raise AbdError(rc, msg.decode() if msg else "")

    # -- setup ---------------------------------------------------------
    def body_mass(self, scene):
        self._check(self.L.abd_body_mass(self.h, ctypes.byref(scene.c), _ptr(scene.density), _ptr(scene.mass),
                                         _ptr(scene.volume), _stream()))
        return scene.mass, scene.volume

    # -- hot path ------------------------------------------------------
    def vertex_map(self, scene, q, x=None):
        x = torch.empty((scene.c.n_verts, 3), dtype=torch.float64, device=q.device) if x is None else x
        self._check(self.L.abd_vertex_map(self.h, ctypes.byref(scene.c), _ptr(q), _ptr(x), _stream()))
        return x

    def candidates(self, scene, x0, x1=None, inflate=1e-3, cap_pt=1 << 20, cap_ee=1 << 20):
        while True:
            pt = torch.empty((max(cap_pt, 1), 2), dtype=torch.int32, device=x0.device)
            ee = torch.empty((max(cap_ee, 1), 2), dtype=torch.int32, device=x0.device)
            npt, nee = ctypes.c_int64(0), ctypes.c_int64(0)
            rc = self.L.abd_candidates(self.h, ctypes.byref(scene.c), _ptr(x0), _ptr(x1), float(inflate), _ptr(pt),
                                       cap_pt, ctypes.byref(npt), _ptr(ee), cap_ee, ctypes.byref(nee), _stream())
            if rc == -2:
                cap_pt, cap_ee = max(cap_pt, npt.value), max(cap_ee, nee.value)
                continue
            self._check(rc)
            return pt[:npt.value], ee[:nee.value]

    def candidates_within(self, scene, x, spt, see, inflate=1e-3):
        cap_pt, cap_ee = max(spt.shape[0], 1), max(see.shape[0], 1)
        pt = torch.empty((cap_pt, 2), dtype=torch.int32, device=x.device)
        ee = torch.empty((cap_ee, 2), dtype=torch.int32, device=x.device)
        npt, nee = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self.L.abd_candidates_within(self.h, ctypes.byref(scene.c), _ptr(x), float(inflate), _ptr(spt),
                                                 spt.shape[0], _ptr(see), see.shape[0], _ptr(pt), cap_pt,
                                                 ctypes.byref(npt), _ptr(ee), cap_ee, ctypes.byref(nee), _stream()))
        return pt[:npt.value], ee[:nee.value]

    def offdiag_pattern(self, scene, pt, ee):
        # (every pair, and every joint between two bodies, gives at most one key)
        cap = pt.shape[0] + ee.shape[0] + scene.n_joints + 1
        keys = torch.empty((cap, 2), dtype=torch.int32, device=pt.device)
        n = ctypes.c_int64(0)
        self._check(self.L.abd_offdiag_pattern(self.h, ctypes.byref(scene.c), _ptr(pt), pt.shape[0], _ptr(ee),
                                               ee.shape[0], _ptr(keys), cap, ctypes.byref(n), _stream()))
        return keys[:n.value]

    def classify(self, scene, x, pairs, is_ee, dhat):
        n = pairs.shape[0]
        ty = torch.zeros(n, dtype=torch.uint8, device=x.device)
        d2 = torch.zeros(n, dtype=torch.float64, device=x.device)
        act = torch.zeros(n, dtype=torch.uint8, device=x.device)
        self._check(self.L.abd_classify(self.h, ctypes.byref(scene.c), _ptr(x), float(dhat), _ptr(pairs), n,
                                        int(is_ee), _ptr(ty), _ptr(d2), _ptr(act), _stream()))
        return ty, d2, act

    def barrier_grad_hess(self, scene, params, x, pt, ee, keys, project=True, hessian=True):
        nb = scene.n_bodies
        dev = x.device
        energy = torch.zeros(1, dtype=torch.float64, device=dev)
        grad = torch.zeros((nb, 12), dtype=torch.float64, device=dev)
        diag = torch.zeros((nb, 144), dtype=torch.float64, device=dev) if hessian else None
        off = torch.zeros((max(keys.shape[0], 1), 144), dtype=torch.float64, device=dev) if hessian else None
        prm = make_params(params)
        self._check(self.L.abd_barrier_grad_hess(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(x),
                                                 _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0], _ptr(keys),
                                                 keys.shape[0], _ptr(energy), _ptr(grad), _ptr(diag), _ptr(off),
                                                 int(project), _stream()))
        return energy, grad, diag, (off[:keys.shape[0]] if hessian else None)

    def barrier_energy(self, scene, params, x, pt, ee):
        energy = torch.zeros(1, dtype=torch.float64, device=x.device)
        prm = make_params(params)
        self._check(self.L.abd_barrier_energy(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(x), _ptr(pt),
                                              pt.shape[0], _ptr(ee), ee.shape[0], _ptr(energy), _stream()))
        return energy

    def barrier_energy_noalloc(self, scene, params, x, pt, ee, energy=None):
        """abd_barrier_energy_noalloc: accumulates into `energy` (a float64
        [1] device tensor; a new zero one when None)."""
        if energy is None:
            energy = torch.zeros(1, dtype=torch.float64, device=x.device)
        prm = make_params(params)
        self._check(self.L.abd_barrier_energy_noalloc(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(x),
                                                      _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0], _ptr(energy),
                                                      _stream()))
        return energy

    def ccd_max_step(self, scene, params, x0, dx, pt, ee, per_pair=True):
        """(t_pt, t_ee, alpha); per_pair=False asks for the bound alone
        (t_pt, t_ee are then None)."""
        dev = x0.device
        t_pt = torch.zeros(pt.shape[0], dtype=torch.float64, device=dev) if per_pair else None
        t_ee = torch.zeros(ee.shape[0], dtype=torch.float64, device=dev) if per_pair else None
        alpha = torch.zeros(max(scene.n_scenes, 1), dtype=torch.float64, device=dev)
        prm = make_params(params)
        self._check(self.L.abd_ccd_max_step(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(x0), _ptr(dx),
                                            _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0], _ptr(t_pt), _ptr(t_ee),
                                            _ptr(alpha), _stream()))
        return t_pt, t_ee, alpha

    def orthogonality(self, scene, params, q, weight, project=True, hessian=True):
        """The rigidity potential selected by params["rigidity"] (0 the
        orthogonality potential); hessian=False: the energy alone (no
        gradient or blocks: the energy-only kernel)."""
        nb = scene.n_bodies
        dev = q.device
        e = torch.zeros(1, dtype=torch.float64, device=dev)
        g = torch.zeros((nb, 12), dtype=torch.float64, device=dev) if hessian else None
        D = torch.zeros((nb, 144), dtype=torch.float64, device=dev) if hessian else None
        prm = make_params(params)
        self._check(self.L.abd_orthogonality(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q),
                                             float(weight), _ptr(e), _ptr(g), _ptr(D), int(project), _stream()))
        return e, g, D

    def inertia(self, scene, q, q_tilde):
        nb = scene.n_bodies
        dev = q.device
        e = torch.zeros(1, dtype=torch.float64, device=dev)
        g = torch.zeros((nb, 12), dtype=torch.float64, device=dev)
        D = torch.zeros((nb, 144), dtype=torch.float64, device=dev)
        self._check(self.L.abd_inertia(self.h, ctypes.byref(scene.c), _ptr(q), _ptr(q_tilde), _ptr(e), _ptr(g),
                                       _ptr(D), _stream()))
        return e, g, D

    def q_tilde(self, scene, params, q, qd):
        out = torch.empty_like(q)
        prm = make_params(params)
        self._check(self.L.abd_q_tilde(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q), _ptr(qd),
                                       _ptr(out), _stream()))
        return out

    def pcg_solve(self, scene, diag, off, keys, rhs, rtol=1e-12, max_iter=10000, x0=None):
        p = torch.zeros_like(rhs)
        it = ctypes.c_int32(0)
        self._check(self.L.abd_pcg_solve(self.h, ctypes.byref(scene.c), _ptr(diag), _ptr(off), _ptr(keys),
                                         keys.shape[0], _ptr(rhs), _ptr(x0), _ptr(p), float(rtol), int(max_iter),
                                         ctypes.byref(it), _stream()))
        return p, it.value

    def newton_step(self, scene, params, q, q_tilde, scene_done=None):
        """One Newton iteration; scene_done (uint8 [n_scenes] device tensor,
        in/out) marks sub-scenes already converged."""
        st = AbdStats()
        prm = make_params(params)
        self._check(self.L.abd_newton_step(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q),
                                           _ptr(q_tilde), _ptr(scene_done), ctypes.byref(st), _stream()))
        return st.as_dict()

    def time_step(self, scene, params, q, qd):
        st = AbdStats()
        prm = make_params(params)
        self._check(self.L.abd_time_step(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q), _ptr(qd),
                                         ctypes.byref(st), _stream()))
        return st.as_dict()

    # -- friction --------------------------------------------------------
    def friction_lag(self, scene, params, xt, pt, ee):
        """Per pair (PT then EE) lambda [n], T [n,6], w [n,4] at xt."""
        n = pt.shape[0] + ee.shape[0]
        dev = xt.device
        lam = torch.zeros(n, dtype=torch.float64, device=dev)
        T = torch.zeros((n, 6), dtype=torch.float64, device=dev)
        w = torch.zeros((n, 4), dtype=torch.float64, device=dev)
        prm = make_params(params)
        self._check(self.L.abd_friction_lag(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(xt), _ptr(pt),
                                            pt.shape[0], _ptr(ee), ee.shape[0], _ptr(lam), _ptr(T), _ptr(w),
                                            _stream()))
        return lam, T, w

    def friction_grad_hess(self, scene, params, x, xt, pt, ee, lam, T, w, keys, hessian=True):
        nb = scene.n_bodies
        dev = x.device
        energy = torch.zeros(1, dtype=torch.float64, device=dev)
        grad = torch.zeros((nb, 12), dtype=torch.float64, device=dev)
        diag = torch.zeros((nb, 144), dtype=torch.float64, device=dev) if hessian else None
        off = torch.zeros((max(keys.shape[0], 1), 144), dtype=torch.float64, device=dev) if hessian else None
        prm = make_params(params)
        self._check(self.L.abd_friction_grad_hess(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(x),
                                                  _ptr(xt), _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0], _ptr(lam),
                                                  _ptr(T), _ptr(w), _ptr(keys), keys.shape[0], _ptr(energy),
                                                  _ptr(grad), _ptr(diag), _ptr(off), _stream()))
        return energy, grad, diag, (off[:keys.shape[0]] if hessian else None)

    def friction_energy(self, scene, params, x, xt, pt, ee, lam, T, w):
        energy = torch.zeros(1, dtype=torch.float64, device=x.device)
        prm = make_params(params)
        self._check(self.L.abd_friction_energy(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(x), _ptr(xt),
                                               _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0], _ptr(lam), _ptr(T),
                                               _ptr(w), _ptr(energy), _stream()))
        return energy

    def friction_begin_step(self, scene, params, q):
        n = ctypes.c_int64(0)
        prm = make_params(params)
        self._check(self.L.abd_friction_begin_step(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q),
                                                   ctypes.byref(n), _stream()))
        return n.value

    def friction_end_step(self):
        self._check(self.L.abd_friction_end_step(self.h))

    # -- adjoint -------------------------------------------------------
    def adjoint_step(self, scene, params, q_t, qd_t, q_next, qbar_next, qdbar_next, rtol=1e-12):
        qbar = torch.zeros_like(q_t)
        qdbar = torch.zeros_like(q_t)
        it = ctypes.c_int32(0)
        prm = make_params(params)
        self._check(self.L.abd_adjoint_step(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q_t), _ptr(qd_t),
                                            _ptr(q_next), _ptr(qbar_next), _ptr(qdbar_next), float(rtol), _ptr(qbar),
                                            _ptr(qdbar), ctypes.byref(it), _stream()))
        return qbar, qdbar, it.value

    def rollout_forward(self, scene, params, q, qd, n_steps, checkpoint_every=10, keep=True):
        """n_steps time steps on (q, qd) in place; returns the checkpoints
        (for rollout_backward; None when keep is false) and the summed Newton
        iterations."""
        n_ck = (int(n_steps) + int(checkpoint_every) - 1) // int(checkpoint_every) + 1
        ck = torch.zeros((n_ck, 2) + tuple(q.shape), dtype=torch.float64, device=q.device) if keep else None
        nt = ctypes.c_int64(0)
        prm = make_params(params)
        self._check(self.L.abd_rollout_forward(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q), _ptr(qd),
                                               int(n_steps), int(checkpoint_every), _ptr(ck), ctypes.byref(nt),
                                               _stream()))
        return ck, nt.value

    def rollout_backward(self, scene, params, q0, qd0, n_steps, checkpoint_every, qbar_T, qdbar_T, rtol=1e-12,
                         checkpoints=None):
        qbar = torch.zeros_like(q0)
        qdbar = torch.zeros_like(q0)
        prm = make_params(params)
        self._check(self.L.abd_rollout_backward(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q0),
                                                _ptr(qd0), int(n_steps), int(checkpoint_every), _ptr(checkpoints),
                                                _ptr(qbar_T), _ptr(qdbar_T), float(rtol), _ptr(qbar), _ptr(qdbar),
                                                _stream()))
        return qbar, qdbar

    # -- measurement ---------------------------------------------------
    # -- launch shapes -------------------------------------------------
    def barrier_stiffness(self, scene):
        """Per-scene barrier stiffness of the last adaptive time step."""
        n = max(int(scene.c.n_scenes), 1)
        out = (ctypes.c_double * n)()
        self._check(self.L.abd_barrier_stiffness(self.h, ctypes.byref(scene.c), out))
        return np.array(out[:], np.float64)

    def tune_get(self):
        t = _lib.AbdTune()
        self._check(self.L.abd_tune_get(self.h, ctypes.byref(t)))
        return t.as_dict()

    def tune_set(self, table):
        """Sets the launch table; entries missing from `table` keep their
        current values."""
        cur = self.tune_get()
        cur.update(table)
        t = _lib.AbdTune(**{k: int(v) for k, v in cur.items()})
        self._check(self.L.abd_tune_set(self.h, ctypes.byref(t)))

    def autotune(self, scene, params, q, qd, n_steps=3, reps=2):
        """abd_autotune on the workload (q, qd unchanged on return): the
        picked table (also set in the context) and its ms per step."""
        t = _lib.AbdTune()
        ms = ctypes.c_double(0.0)
        prm = make_params(params)
        self._check(self.L.abd_autotune(self.h, ctypes.byref(scene.c), ctypes.byref(prm), _ptr(q), _ptr(qd),
                                        int(n_steps), int(reps), ctypes.byref(t), ctypes.byref(ms), _stream()))
        return t.as_dict(), ms.value

    def profile(self, enable=True, reset=True):
        """enable: False/0 off, True/1 kernel timing, 2 timing and box-test
        counts of the candidate searches."""
        self._check(self.L.abd_profile(self.h, int(enable), int(reset)))

    def profile_query(self, kernel):
        ms, la, un = ctypes.c_double(0), ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self.L.abd_profile_query(self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(la),
                                             ctypes.byref(un)))
        return dict(ms=ms.value, launches=la.value, units=un.value)


class Rollout(torch.autograd.Function):
    """(q^n, qdot^n) after n time steps from (q0, qdot0), differentiable:
    the forward pass keeps checkpoints (abd_rollout_forward), the backward
    pass is abd_rollout_backward from them (checkpointed adjoint)."""

    @staticmethod
    def forward(fctx, q0, qd0, ctx, scene, params, n_steps, checkpoint_every, rtol):
        q, qd = q0.detach().clone(), qd0.detach().clone()
        ck, _ = ctx.rollout_forward(scene, params, q, qd, n_steps, checkpoint_every)
        fctx.save_for_backward(q0.detach(), qd0.detach(), ck)
        fctx.args = (ctx, scene, params, n_steps, checkpoint_every, rtol)
        return q, qd

    @staticmethod
    def backward(fctx, gq, gqd):
        q0, qd0, ck = fctx.saved_tensors
        ctx, scene, params, n_steps, every, rtol = fctx.args
        gq = torch.zeros_like(q0) if gq is None else gq.contiguous()
        gqd = torch.zeros_like(q0) if gqd is None else gqd.contiguous()
        qbar, qdbar = ctx.rollout_backward(scene, params, q0, qd0, n_steps, every, gq, gqd, rtol, checkpoints=ck)
        return qbar, qdbar, None, None, None, None, None, None


def rollout(ctx, scene, params, q0, qd0, n_steps, checkpoint_every=10, rtol=1e-12):
    return Rollout.apply(q0, qd0, ctx, scene, params, n_steps, checkpoint_every, rtol)


def setup(S, device=0):
    """Context + device scene with mass properties computed on the GPU."""
    ctx = Context(device)
    scene = Scene(S, f"cuda:{device}")
    ctx.body_mass(scene)
    return ctx, scene

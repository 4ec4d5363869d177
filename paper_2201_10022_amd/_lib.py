"""ctypes view of the C ABI declared in include/abd.h (argument marshalling
only; every step runs in the HIP library)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabd.so")

ABD_OK = 0
ERRORS = {-1: "ABD_E_INVALID", -2: "ABD_E_CAPACITY", -3: "ABD_E_INTERSECT", -4: "ABD_E_NOT_CONVERGED",
          -5: "ABD_E_LINESEARCH", -6: "ABD_E_PCG", -7: "ABD_E_HIP"}

EXPORTS = ["abd_create", "abd_destroy", "abd_last_error", "abd_body_mass", "abd_vertex_map", "abd_candidates",
           "abd_candidates_within",
           "abd_offdiag_pattern", "abd_classify", "abd_barrier_grad_hess", "abd_barrier_energy",
           "abd_barrier_energy_noalloc",
           "abd_ccd_max_step", "abd_orthogonality", "abd_inertia", "abd_q_tilde", "abd_pcg_solve",
           "abd_newton_step", "abd_time_step", "abd_friction_lag", "abd_friction_grad_hess",
           "abd_friction_energy", "abd_friction_begin_step", "abd_friction_end_step", "abd_adjoint_step",
           "abd_rollout_forward", "abd_rollout_backward", "abd_profile", "abd_profile_query",
           "abd_tune_get", "abd_tune_set", "abd_autotune", "abd_barrier_stiffness"]

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pi32 = ctypes.POINTER(ctypes.c_int32)


class AbdScene(ctypes.Structure):
    _fields_ = [("n_bodies", _i32), ("n_verts", _i32), ("n_tris", _i32), ("n_edges", _i32), ("n_scenes", _i32),
                ("xbar", _vp), ("vert_body", _vp), ("tris", _vp), ("tri_body", _vp), ("edges", _vp),
                ("edge_body", _vp), ("body_vert_off", _vp), ("body_tri_off", _vp), ("body_edge_off", _vp),
                ("body_fixed", _vp), ("body_scene", _vp), ("mass", _vp), ("volume", _vp), ("n_joints", _i32),
                ("joint_body", _vp), ("joint_point", _vp)]


class AbdParams(ctypes.Structure):
    _fields_ = [("dt", _dbl), ("dhat", _dbl), ("kappa_b", _dbl), ("kappa_o", _dbl), ("mu", _dbl), ("eps_v", _dbl),
                ("gravity", _dbl * 3), ("newton_tol", _dbl), ("pcg_rtol", _dbl), ("ccd_s", _dbl),
                ("ccd_tmax", _dbl), ("ccd_max_iter", _i32), ("max_newton", _i32), ("max_pcg", _i32),
                ("max_ls", _i32), ("rigidity", _i32), ("kappa_j", _dbl), ("kappa_adaptive", _i32),
                ("kappa_max", _dbl), ("kappa_eps_d", _dbl)]


class AbdStats(ctypes.Structure):
    _fields_ = [("n_pt", _i64), ("n_ee", _i64), ("n_active_pt", _i64), ("n_active_ee", _i64),
                ("n_pt_swept", _i64), ("n_ee_swept", _i64), ("n_offdiag", _i64), ("pcg_iters", _i32),
                ("ls_halvings", _i32), ("converged", _i32), ("newton_iters", _i32), ("alpha_ccd", _dbl),
                ("alpha", _dbl), ("disp", _dbl), ("energy0", _dbl), ("energy1", _dbl), ("t_barrier_ms", _dbl),
                ("t_ccd_ms", _dbl), ("t_candidates_ms", _dbl), ("t_solve_ms", _dbl), ("t_total_ms", _dbl),
                ("n_friction", _i64), ("scene_newton_iters", _i64), ("newly_converged", _i32), ("pad_", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AbdTune(ctypes.Structure):
    _fields_ = [("tile_rows", _i32), ("barrier_waves", _i32), ("ccd_block", _i32), ("ccd_max_blocks", _i32),
                ("energy_block", _i32), ("pcg_short", _i32), ("pcg_long", _i32), ("cull_levels", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_PS = ctypes.POINTER(AbdScene)
_PP = ctypes.POINTER(AbdParams)
_PST = ctypes.POINTER(AbdStats)

SIGNATURES = {
    "abd_create": ([ctypes.POINTER(_vp), ctypes.c_int], ctypes.c_int),
    "abd_destroy": ([_vp], ctypes.c_int),
    "abd_last_error": ([_vp], ctypes.c_char_p),
    "abd_body_mass": ([_vp, _PS, _vp, _vp, _vp, _vp], ctypes.c_int),
    "abd_vertex_map": ([_vp, _PS, _vp, _vp, _vp], ctypes.c_int),
    "abd_candidates": ([_vp, _PS, _vp, _vp, _dbl, _vp, _i64, _pi64, _vp, _i64, _pi64, _vp], ctypes.c_int),
    "abd_candidates_within": ([_vp, _PS, _vp, _dbl, _vp, _i64, _vp, _i64, _vp, _i64, _pi64, _vp, _i64, _pi64, _vp],
                              ctypes.c_int),
    "abd_offdiag_pattern": ([_vp, _PS, _vp, _i64, _vp, _i64, _vp, _i64, _pi64, _vp], ctypes.c_int),
    "abd_classify": ([_vp, _PS, _vp, _dbl, _vp, _i64, ctypes.c_int, _vp, _vp, _vp, _vp], ctypes.c_int),
    "abd_barrier_grad_hess": ([_vp, _PS, _PP, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp,
                               ctypes.c_int, _vp], ctypes.c_int),
    "abd_barrier_energy": ([_vp, _PS, _PP, _vp, _vp, _i64, _vp, _i64, _vp, _vp], ctypes.c_int),
    "abd_barrier_energy_noalloc": ([_vp, _PS, _PP, _vp, _vp, _i64, _vp, _i64, _vp, _vp], ctypes.c_int),
    "abd_ccd_max_step": ([_vp, _PS, _PP, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
    "abd_orthogonality": ([_vp, _PS, _PP, _vp, _dbl, _vp, _vp, _vp, ctypes.c_int, _vp], ctypes.c_int),
    "abd_inertia": ([_vp, _PS, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "abd_q_tilde": ([_vp, _PS, _PP, _vp, _vp, _vp, _vp], ctypes.c_int),
    "abd_pcg_solve": ([_vp, _PS, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _dbl, _i32, _pi32, _vp], ctypes.c_int),
    "abd_newton_step": ([_vp, _PS, _PP, _vp, _vp, _vp, _PST, _vp], ctypes.c_int),
    "abd_time_step": ([_vp, _PS, _PP, _vp, _vp, _PST, _vp], ctypes.c_int),
    "abd_friction_lag": ([_vp, _PS, _PP, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
    "abd_friction_grad_hess": ([_vp, _PS, _PP, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp,
                                _vp, _vp, _vp], ctypes.c_int),
    "abd_friction_energy": ([_vp, _PS, _PP, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "abd_friction_begin_step": ([_vp, _PS, _PP, _vp, _pi64, _vp], ctypes.c_int),
    "abd_friction_end_step": ([_vp], ctypes.c_int),
    "abd_adjoint_step": ([_vp, _PS, _PP, _vp, _vp, _vp, _vp, _vp, _dbl, _vp, _vp, _pi32, _vp], ctypes.c_int),
    "abd_rollout_forward": ([_vp, _PS, _PP, _vp, _vp, _i32, _i32, _vp, ctypes.POINTER(ctypes.c_int64), _vp],
                            ctypes.c_int),
    "abd_rollout_backward": ([_vp, _PS, _PP, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _dbl, _vp, _vp, _vp], ctypes.c_int),
    "abd_profile": ([_vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "abd_profile_query": ([_vp, ctypes.c_char_p, ctypes.POINTER(_dbl), _pi64, _pi64], ctypes.c_int),
    "abd_barrier_stiffness": ([_vp, _PS, ctypes.POINTER(_dbl)], ctypes.c_int),
    "abd_tune_get": ([_vp, ctypes.POINTER(AbdTune)], ctypes.c_int),
    "abd_tune_set": ([_vp, ctypes.POINTER(AbdTune)], ctypes.c_int),
    "abd_autotune": ([_vp, _PS, _PP, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(AbdTune),
                      ctypes.POINTER(_dbl), _vp], ctypes.c_int),
}

_LIB = None


def load():
    """Loads the in-tree libabd.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2201_10022_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB

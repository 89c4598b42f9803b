"""ctypes binding of libnsn.so (include/nsn.h).  Argument marshalling only: every
step of the solver runs in the HIP kernels of the library."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnsn.so")

F = C.POINTER(C.c_float)
I32 = C.POINTER(C.c_int32)
D = C.POINTER(C.c_double)
VP = C.c_void_p


class EnvDescC(C.Structure):
    _fields_ = [
        ("n_rigid", C.c_int32),
        ("rigid_mass", F), ("rigid_inertia", F), ("rigid_x", F), ("rigid_q", F),
        ("rigid_v", F), ("rigid_w", F), ("rigid_shape", I32), ("rigid_extent", F),
        ("n_particles", C.c_int32),
        ("particle_x", F), ("particle_v", F), ("particle_rest", F), ("particle_mass", F),
        ("n_tets", C.c_int32), ("tet_ids", I32), ("tet_material", F),
        ("n_joints", C.c_int32), ("joint_type", I32), ("joint_body", I32),
        ("joint_anchor", F), ("joint_axis", F), ("joint_ref", F), ("joint_drive", F),
        ("mu", C.c_float), ("gravity", C.c_float * 3), ("ground", C.c_int32),
        ("max_contacts", C.c_int32), ("tet_model", C.c_int32),
    ]


class ParamsC(C.Structure):
    _fields_ = [("ncp", C.c_int32), ("rmode", C.c_int32), ("damping", C.c_float),
                ("eps", C.c_float), ("geo_stiff", C.c_int32), ("fem_mode", C.c_int32),
                ("margin", C.c_float), ("warm", C.c_int32), ("line_search", C.c_int32),
                ("linear", C.c_int32), ("islands", C.c_int32), ("watchdog", C.c_int32)]


class ContactC(C.Structure):
    _fields_ = [("key", C.c_int32), ("body_a", C.c_int32), ("body_b", C.c_int32),
                ("normal", C.c_float * 3), ("a_local", C.c_float * 3), ("b_local", C.c_float * 3),
                ("thickness", C.c_float)]


class TrainParamsC(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("clip_quantile", C.c_float),
                ("seed", C.c_uint64)]


# per-iteration record fields (include/nsn.h NSN_IT_*)
IT_FIELDS = ["lam", "err", "cdiag", "P", "b", "Az", "dlam", "tetc", "alpha", "active", "g", "u", "hdiag",
             "rx", "rq", "px", "prev_lam", "prev_u", "prev_rx", "prev_rq", "prev_px"]


ACC_DTYPE = np.dtype([("steps", np.int64), ("newton_iters", np.int64), ("cr_iters", np.int64),
                      ("converged", np.int64), ("nonfinite", np.int64), ("fallbacks", np.int64),
                      ("watchdogs", np.int64), ("cr_bytes", np.float64)])

STATS_DTYPE = np.dtype([("newton_iters", np.int32), ("cr_iters", np.int32), ("n_contacts", np.int32),
                        ("overflow", np.int32), ("nonfinite", np.int32), ("converged", np.int32),
                        ("fallback", np.int32), ("watchdog", np.int32),
                        ("r_ncp", np.float64), ("r_contact", np.float64), ("merit", np.float64),
                        ("r_ncp_first", np.float64)])

_L = None


class NSNError(RuntimeError):
    pass


def lib():
    """Load libnsn.so.  Raises if the HIP library has not been built: there is no
    fallback path."""
    global _L
    if _L is not None:
        return _L
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or `python paper_1907_04587_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    S = C.c_int32
    L.nsn_last_error.restype = C.c_char_p
    L.nsn_query_workspace.argtypes = [C.POINTER(EnvDescC), S, C.POINTER(ParamsC), C.POINTER(C.c_size_t)]
    L.nsn_create_scene.argtypes = [C.POINTER(EnvDescC), S, C.POINTER(ParamsC), VP, VP, C.c_size_t,
                                   C.POINTER(VP)]
    L.nsn_destroy_scene.argtypes = [VP]
    L.nsn_set_params.argtypes = [VP, C.POINTER(ParamsC)]
    L.nsn_step.argtypes = [VP, C.c_double, S, S, C.c_double, VP]
    L.nsn_set_contacts.argtypes = [VP, S, C.POINTER(ContactC), S]
    L.nsn_dump_iteration.argtypes = [VP, C.c_double, S, S]
    L.nsn_read_iteration.argtypes = [VP, S, S, S, I32, F]
    L.nsn_get_stats.argtypes = [VP, VP]
    L.nsn_read_state.argtypes = [VP, S, F, F, F, F, F, F, D]
    L.nsn_write_state.argtypes = [VP, S, F, F, F, F, F, F, D]
    L.nsn_state_bytes.argtypes = [VP, C.POINTER(C.c_size_t)]
    L.nsn_save_state.argtypes = [VP, VP]
    L.nsn_load_state.argtypes = [VP, VP]
    L.nsn_read_contacts.argtypes = [VP, S, S, I32, I32, I32, F, F]
    L.nsn_read_lambda.argtypes = [VP, S, S, I32, F]
    L.nsn_set_warm_start_model.argtypes = [VP, F, C.c_int64]
    L.nsn_read_features.argtypes = [VP, S, S, I32, F]
    L.nsn_enable_features.argtypes = [VP, S]
    L.nsn_set_use_graphs.argtypes = [VP, S]
    L.nsn_get_env_order.argtypes = [VP, I32]
    L.nsn_set_schedule.argtypes = [VP, S, I32, I32, I32]
    L.nsn_set_lds_mode.argtypes = [VP, C.c_int32]
    L.nsn_get_lds_modes.argtypes = [VP, C.c_int32, I32, I32]
    L.nsn_set_pcr_form.argtypes = [VP, C.c_int32]
    L.nsn_get_schedule.argtypes = [VP, S, I32, I32, I32, I32]
    L.nsn_stats_device_ptr.argtypes = [VP, C.POINTER(VP)]
    L.nsn_read_kernel_times.argtypes = [VP, S, I32, D]
    L.nsn_read_accumulators.argtypes = [VP, VP]
    L.nsn_reset_accumulators.argtypes = [VP]
    L.nsn_mlp_forward.argtypes = [VP, VP, VP, C.c_int64, VP]
    L.nsn_mlp_scratch_bytes.restype = C.c_size_t
    L.nsn_mlp_scratch_bytes.argtypes = [C.c_int64]
    L.nsn_mlp_loss_grad.argtypes = [VP, VP, VP, C.c_int64, VP, VP, VP, VP]
    L.nsn_mlp_adam.argtypes = [VP, VP, VP, VP, C.c_int64, C.c_float, C.c_float, C.c_float,
                               C.c_float, S, VP]
    L.nsn_mlp_noalloc_scratch_bytes.restype = C.c_size_t
    L.nsn_mlp_noalloc_scratch_bytes.argtypes = []
    L.nsn_mlp_loss_grad_noalloc.argtypes = [VP, VP, VP, C.c_int64, VP, VP, VP]
    L.nsn_train_workspace_bytes.restype = C.c_size_t
    L.nsn_train_workspace_bytes.argtypes = [C.c_int64, S]
    L.nsn_train_warm_start.argtypes = [VP, VP, C.c_int64, C.POINTER(TrainParamsC), VP, VP, D, VP, C.c_size_t, VP]
    _L = L
    return L


def check(status, what=""):
    if status != 0:
        msg = lib().nsn_last_error().decode()
        raise NSNError(f"{what} failed with status {status}: {msg}")


def f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def fptr(a):
    return None if a is None else a.ctypes.data_as(F)


def iptr(a):
    return None if a is None else a.ctypes.data_as(I32)

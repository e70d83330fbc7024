"""ctypes declarations of the C ABI in ``include/gigaqbx.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgigaqbx.so")

GQ_OK, GQ_EINVAL, GQ_ENOMEM, GQ_EHIP, GQ_ESTATE, GQ_EUNSUP = 0, -1, -2, -3, -4, -5
GQ_S, GQ_D, GQ_S_MINUS_D, GQ_S_AND_D, GQ_SP = 1, 2, 3, 4, 5
GQ_EXP_MULTIPOLE, GQ_EXP_LOCAL, GQ_EXP_LOCAL_COMPLETE = 1, 2, 3
GQ_MEM_HOST, GQ_MEM_DEVICE = 0, 1
GQ_FP64, GQ_MIXED_FP32 = 0, 1
GQ_MAX_P_QBX, GQ_MAX_P_FMM = 20, 63
GQ_MATH_LOG, GQ_MATH_RCP = 1, 2
GQ_N_FEATURES = 8

(GQ_TREE_BOX_LEVEL, GQ_TREE_BOX_PARENT, GQ_TREE_BOX_CHILD, GQ_TREE_BOX_IJ, GQ_TREE_BOX_SRC_RANGE,
 GQ_TREE_BOX_CTR_RANGE, GQ_TREE_SRC_ORDER, GQ_TREE_CTR_ORDER, GQ_LIST1_START, GQ_LIST1,
 GQ_LIST2_START, GQ_LIST2, GQ_LIST3C_START, GQ_LIST3C, GQ_LIST3F_START, GQ_LIST3F,
 GQ_LIST4C_START, GQ_LIST4C, GQ_LIST4F_START, GQ_LIST4F) = range(1, 21)

STATUS_NAMES = {0: "GQ_OK", -1: "GQ_EINVAL", -2: "GQ_ENOMEM", -3: "GQ_EHIP", -4: "GQ_ESTATE",
                -5: "GQ_EUNSUP"}


class gq_params(C.Structure):
    _fields_ = [("p_qbx", C.c_int), ("p_fmm", C.c_int), ("n_max", C.c_int),
                ("count_mode", C.c_int), ("t_f", C.c_double), ("w3far_min_sources", C.c_int),
                ("precision", C.c_int), ("max_levels", C.c_int), ("overlap", C.c_int),
                ("near_chunk", C.c_int), ("far_chunk", C.c_int), ("far_pairs_per_lane", C.c_int),
                ("near_dens_group", C.c_int), ("eps", C.c_double), ("tcr_shape", C.c_int),
                ("level_restrict", C.c_int)]


GQ_OP_NAMES = ["multipoles", "m2m", "list1", "list2", "list3_close", "list3_far", "list4_close",
               "list4_far", "l2l", "l2qbxl"]
GQ_N_OPS = len(GQ_OP_NAMES)


class gq_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_src", "n_ctr", "n_tgt", "n_boxes", "n_levels", "n_leaves", "n_target_boxes",
        "n_suspended_centers", "n_list1", "n_list2", "n_list3_close", "n_list3_far",
        "n_list4_close", "n_list4_far", "near_pairs", "list3_far_pairs", "list4_far_sources",
        "near_sources", "n_local_boxes",
        "max_list2", "max_list4", "max_list4_close", "max_list4_far")] + [
        ("root_lo", C.c_double * 2), ("root_side", C.c_double), ("build_ms", C.c_double),
        ("n_point_targets", C.c_int64), ("n_l2l_sinks", C.c_int64),
        ("n_l2l_pairs", C.c_int64), ("n_moment_boxes", C.c_int64),
        ("n_moment_pairs", C.c_int64), ("n_moment_parts", C.c_int64),
        ("n_m2q_waves", C.c_int64), ("n_m2q_pairs", C.c_int64), ("n_m2q_units", C.c_int64),
        ("m_c", C.c_double), ("m_c_sum", C.c_int64),
        ("model_ops", C.c_int64 * GQ_N_OPS), ("model_ops_total", C.c_int64)]



GQ_STAGE_NAMES = ["gather", "p2m", "m2m", "m2l_p2l", "l2l", "near", "m2qbxl", "qbx_center",
                  "finalize", "direct"]
GQ_N_STAGES = len(GQ_STAGE_NAMES)

EXPORTED = ["gq_default_params", "gq_create", "gq_destroy", "gq_set_stream", "gq_set_geometry",
            "gq_set_geometry_batch",
            "gq_build", "gq_eval", "gq_eval_direct", "gq_get_stats", "gq_get_tree_array",
            "gq_set_qbx_orders", "gq_get_box_orders", "gq_get_center_orders",
            "gq_set_target_normals", "gq_get_expansions",
            "gq_set_profiling", "gq_get_stage_times",
            "gq_graph_create", "gq_graph_launch", "gq_graph_destroy", "gq_autotune",
            "gq_get_params", "gq_device_math", "gq_eval_noalloc", "gq_associate_targets",
            "gq_associate_last_error", "gq_last_error"]


EXPORTED_MLP = ["gq_mlp_create", "gq_mlp_destroy", "gq_mlp_param_count", "gq_mlp_set_params",
                "gq_mlp_get_params", "gq_mlp_forward", "gq_mlp_gradients", "gq_mlp_train_step",
                "gq_mlp_last_error", "gq_mlp_shape", "gq_mlp_stream", "gq_center_features",
                "gq_orders_predict"]


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"HIP library {path} is not built; run `python -c 'import __graft_entry__ as g; "
            "g.build()'` (or `python -m paper_1801_04070_amd.build`) first")
    L = C.CDLL(path)
    vp, dp, ip, i64, i32 = C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int
    L.gq_default_params.argtypes = [C.POINTER(gq_params)]
    L.gq_create.argtypes = [C.POINTER(C.c_void_p), i32, vp]
    L.gq_destroy.argtypes = [vp]
    L.gq_set_stream.argtypes = [vp, vp]
    L.gq_set_geometry.argtypes = [vp, i32, i64, dp, dp, dp, i64, dp, dp, i64, dp, ip]
    L.gq_set_geometry_batch.argtypes = [vp, i32, i64, vp, vp, vp, i64, dp, dp, dp, i64, dp, dp,
                                        i64, dp, ip]
    L.gq_build.argtypes = [vp, C.POINTER(gq_params)]
    L.gq_eval.argtypes = [vp, i32, i64, dp, i64, dp, i64, dp, i64]
    L.gq_eval_direct.argtypes = L.gq_eval.argtypes
    L.gq_eval_noalloc.argtypes = L.gq_eval.argtypes
    L.gq_get_stats.argtypes = [vp, C.POINTER(gq_stats)]
    L.gq_get_tree_array.argtypes = [vp, i32, vp, C.POINTER(C.c_int64)]
    L.gq_set_qbx_orders.argtypes = [vp, i32, vp]
    L.gq_get_box_orders.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    L.gq_get_center_orders.argtypes = [vp, vp]
    L.gq_set_target_normals.argtypes = [vp, i32, i64, dp]
    L.gq_get_expansions.argtypes = [vp, i32, i64, dp, C.POINTER(C.c_int64)]
    L.gq_set_profiling.argtypes = [vp, i32]
    L.gq_get_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.gq_graph_create.argtypes = [vp, i32, i64, dp, i64, dp, i64, dp, i64, C.POINTER(C.c_void_p)]
    L.gq_graph_launch.argtypes = [vp]
    L.gq_graph_destroy.argtypes = [vp]
    L.gq_autotune.argtypes = [vp, i32, dp, i64, i32, C.POINTER(C.c_double)]
    L.gq_get_params.argtypes = [vp, C.POINTER(gq_params)]
    L.gq_device_math.argtypes = [vp, i32, i64, dp, dp]
    L.gq_associate_targets.argtypes = [i64, dp, dp, i64, dp, C.c_double, C.c_double, ip,
                                       C.POINTER(C.c_int64)]
    L.gq_associate_last_error.argtypes = []
    L.gq_associate_last_error.restype = C.c_char_p
    L.gq_last_error.argtypes = [vp]
    L.gq_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("gq_last_error", "gq_associate_last_error"):
            getattr(L, name).restype = C.c_int
    # include/gigaqbx_mlp.h
    L.gq_mlp_create.argtypes = [C.POINTER(C.c_void_p), i32, vp, i32, i32, i32, C.c_uint64]
    L.gq_mlp_destroy.argtypes = [vp]
    L.gq_mlp_param_count.argtypes = [vp]
    L.gq_mlp_param_count.restype = C.c_int64
    L.gq_mlp_set_params.argtypes = [vp, vp]
    L.gq_mlp_get_params.argtypes = [vp, vp]
    L.gq_mlp_forward.argtypes = [vp, i64, vp, vp]
    L.gq_mlp_gradients.argtypes = [vp, i64, vp, vp, vp, vp, C.POINTER(C.c_float)]
    L.gq_mlp_train_step.argtypes = [vp, i64, vp, vp, vp, C.c_float, C.POINTER(C.c_float)]
    L.gq_mlp_last_error.argtypes = [vp]
    L.gq_mlp_last_error.restype = C.c_char_p
    L.gq_mlp_shape.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.gq_mlp_stream.argtypes = [vp]
    L.gq_mlp_stream.restype = C.c_void_p
    L.gq_center_features.argtypes = [vp, vp]
    L.gq_orders_predict.argtypes = [vp, vp, vp, i32, C.c_double, C.c_double, C.c_double, vp,
                                    vp, i32]
    for name in EXPORTED_MLP:
        if name not in ("gq_mlp_last_error", "gq_mlp_param_count", "gq_mlp_stream"):
            getattr(L, name).restype = C.c_int
    return L

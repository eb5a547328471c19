"""ctypes declarations of libsfcnl.so (the C ABI of include/sfcnl.h).

Loading fails loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SFCNL_LIB selects another build of the same library (for A/B timing)
LIB_PATH = os.environ.get("SFCNL_LIB") or os.path.join(HERE, "libsfcnl.so")

OK = 0
E_ARG = -1
E_INPUT = -2
E_CAPACITY = -3
E_HIP = -4
E_NOCONV = -5

SYMBOLS = [
    "sfcnl_create", "sfcnl_destroy", "sfcnl_set_stream", "sfcnl_set_pass_waves", "sfcnl_last_error", "sfcnl_sync", "sfcnl_version",
    "sfc_sort_workspace", "sfc_sort", "sfc_sort_noalloc", "sfc_gather", "sfc_gather_workspace", "sfc_gather_ws", "build_clusters",
    "build_nlist_workspace", "build_nlist", "build_nlist_async", "build_nlist_result",
    "nlist_pass", "nlist_pass_lj", "build_rows_workspace", "build_rows", "rows_pass", "nlist_decode", "sfcnl_profile_begin", "sfcnl_profile_end", "sfcnl_profile_stages", "sfcnl_h_iterate",
    "sfcnl_hseed_features", "sfcnl_mlp_init", "sfcnl_mlp_infer", "sfcnl_mlp_grad_workspace", "sfcnl_mlp_grad",
    "sfcnl_mlp_adam", "sfcnl_batch_create", "sfcnl_batch_destroy", "sfcnl_batch_layout", "sfcnl_batch_sort_workspace",
    "sfcnl_batch_sort", "sfcnl_batch_gather", "sfcnl_batch_nlist_workspace", "sfcnl_batch_build_clusters",
    "sfcnl_batch_build_nlist", "sfcnl_batch_pass", "sfcnl_batch_h_iterate",
]

BATCH_MAX_SYSTEMS = 65535
SORT_NOALLOC_MAX_N = 1 << 20

MLP_NPARAM = 4801
HSEED_NFEAT = 8

NSTAGE = 8
STAGES = ["keys", "sort", "gather", "clusters", "octree", "traverse", "encode", "pass"]


class NlistOpts(C.Structure):
    _fields_ = [("cluster_size", C.c_int), ("compress", C.c_int), ("leaf_bucket", C.c_int),
                ("max_j_per_sc", C.c_int), ("half", C.c_int), ("period", C.c_float * 3)]


class HiterOpts(C.Structure):
    _fields_ = [("target", C.c_int), ("tol", C.c_int), ("max_iters", C.c_int), ("resume", C.c_int),
                ("recount", C.c_int)]


class HiterStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("unconverged", C.c_int64), ("moved", C.c_int64), ("used_bytes", C.c_size_t),
                ("max_nj", C.c_int64)]


class LjParams(C.Structure):
    _fields_ = [("eps", C.c_float), ("sigma", C.c_float), ("coulomb", C.c_float), ("r_cut", C.c_float)]


class HSeed(C.Structure):
    _fields_ = [("d_params", C.c_void_p), ("d_feat", C.c_void_p), ("d_delta", C.c_void_p), ("box_edge", C.c_float),
                ("mode", C.c_int)]


SEED_AFTER_FIRST = 0
SEED_BEFORE_FIRST = 1


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsfcnl.so is not built (run __graft_entry__.build() or "
                           "python paper_2602_19873_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, i64, sz, i32 = C.c_void_p, C.c_int64, C.c_size_t, C.c_int
    lib.sfcnl_create.argtypes = [C.POINTER(vp), i32, vp]
    lib.sfcnl_create.restype = i32
    lib.sfcnl_destroy.argtypes = [vp]
    lib.sfcnl_destroy.restype = None
    lib.sfcnl_set_pass_waves.argtypes = [vp, i32]
    lib.sfcnl_set_pass_waves.restype = i32
    lib.sfcnl_set_stream.argtypes = [vp, vp]
    lib.sfcnl_set_stream.restype = i32
    lib.sfcnl_last_error.argtypes = [vp]
    lib.sfcnl_last_error.restype = C.c_char_p
    lib.sfcnl_sync.argtypes = [vp]
    lib.sfcnl_sync.restype = i32
    lib.sfcnl_version.argtypes = []
    lib.sfcnl_version.restype = C.c_char_p
    lib.sfc_sort_workspace.argtypes = [i64, C.POINTER(sz)]
    lib.sfc_sort_workspace.restype = i32
    lib.sfc_sort.argtypes = [vp, i64, vp, vp, vp, C.POINTER(C.c_float), vp, vp, vp, sz]
    lib.sfc_sort.restype = i32
    lib.sfc_sort_noalloc.argtypes = [vp, i64, vp, vp, vp, C.POINTER(C.c_float), vp, vp]
    lib.sfc_sort_noalloc.restype = i32
    lib.sfc_gather.argtypes = [vp, i64, vp, i32, C.POINTER(vp), C.POINTER(vp)]
    lib.sfc_gather.restype = i32
    lib.sfc_gather_workspace.argtypes = [i64, C.POINTER(sz)]
    lib.sfc_gather_workspace.restype = i32
    lib.sfc_gather_ws.argtypes = [vp, i64, vp, i32, C.POINTER(vp), C.POINTER(vp), vp, sz]
    lib.sfc_gather_ws.restype = i32
    lib.build_clusters.argtypes = [vp, i64, vp, vp, vp, vp, i32, vp]
    lib.build_clusters.restype = i32
    lib.build_nlist_workspace.argtypes = [i64, C.POINTER(NlistOpts), C.POINTER(sz)]
    lib.build_nlist_workspace.restype = i32
    lib.build_nlist.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, C.POINTER(NlistOpts), vp, sz, vp, vp, sz,
                                C.POINTER(sz), C.POINTER(i64)]
    lib.build_nlist.restype = i32
    lib.build_nlist_async.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, C.POINTER(NlistOpts), vp, sz, vp, vp, sz]
    lib.build_nlist_async.restype = i32
    lib.build_nlist_result.argtypes = [vp, C.POINTER(sz), C.POINTER(i64)]
    lib.build_nlist_result.restype = i32
    f3 = C.POINTER(C.c_float)
    lib.nlist_pass.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, f3]
    lib.nlist_pass.restype = i32
    lib.nlist_pass_lj.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp, vp, vp, vp, C.POINTER(LjParams), vp, vp, vp, vp,
                                  f3]
    lib.nlist_pass_lj.restype = i32
    lib.build_rows_workspace.argtypes = [i64, C.POINTER(C.c_size_t)]
    lib.build_rows_workspace.restype = i32
    lib.build_rows.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, vp, vp, i32, f3, vp, C.c_size_t, vp, vp,
                               C.c_size_t, C.POINTER(C.c_size_t)]
    lib.build_rows.restype = i32
    lib.rows_pass.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, f3]
    lib.rows_pass.restype = i32
    lib.nlist_decode.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, vp]
    lib.nlist_decode.restype = i32
    lib.sfcnl_h_iterate.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, C.POINTER(NlistOpts), C.POINTER(HiterOpts),
                                    vp, vp, sz, vp, vp, sz, vp, vp, C.POINTER(HSeed), C.POINTER(HiterStats)]
    lib.sfcnl_h_iterate.restype = i32
    lib.sfcnl_hseed_features.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, C.c_float, i32, vp]
    lib.sfcnl_hseed_features.restype = i32
    lib.sfcnl_mlp_init.argtypes = [vp, C.c_uint64, vp]
    lib.sfcnl_mlp_init.restype = i32
    lib.sfcnl_mlp_infer.argtypes = [vp, vp, i64, vp, vp]
    lib.sfcnl_mlp_infer.restype = i32
    lib.sfcnl_mlp_grad_workspace.argtypes = [i64, C.POINTER(sz)]
    lib.sfcnl_mlp_grad_workspace.restype = i32
    lib.sfcnl_mlp_grad.argtypes = [vp, vp, i64, vp, vp, i64, i64, i64, i64, vp, sz, vp, vp]
    lib.sfcnl_mlp_grad.restype = i32
    lib.sfcnl_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float]
    lib.sfcnl_mlp_adam.restype = i32
    lib.sfcnl_profile_begin.argtypes = [vp, i32]
    lib.sfcnl_profile_begin.restype = i32
    lib.sfcnl_profile_end.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
    lib.sfcnl_profile_end.restype = i32
    lib.sfcnl_profile_stages.argtypes = [vp, C.c_uint32]
    lib.sfcnl_profile_stages.restype = i32
    P64 = C.POINTER(i64)
    lib.sfcnl_batch_create.argtypes = [vp, i32, P64, C.POINTER(C.c_float), C.POINTER(vp)]
    lib.sfcnl_batch_create.restype = i32
    lib.sfcnl_batch_destroy.argtypes = [vp]
    lib.sfcnl_batch_destroy.restype = None
    lib.sfcnl_batch_layout.argtypes = [vp, P64, P64, P64, P64]
    lib.sfcnl_batch_layout.restype = i32
    lib.sfcnl_batch_sort_workspace.argtypes = [vp, C.POINTER(sz)]
    lib.sfcnl_batch_sort_workspace.restype = i32
    lib.sfcnl_batch_sort.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz]
    lib.sfcnl_batch_sort.restype = i32
    lib.sfcnl_batch_gather.argtypes = [vp, vp, vp, i32, C.POINTER(vp), C.POINTER(vp)]
    lib.sfcnl_batch_gather.restype = i32
    lib.sfcnl_batch_nlist_workspace.argtypes = [vp, C.POINTER(NlistOpts), C.POINTER(sz)]
    lib.sfcnl_batch_nlist_workspace.restype = i32
    lib.sfcnl_batch_build_clusters.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp]
    lib.sfcnl_batch_build_clusters.restype = i32
    lib.sfcnl_batch_build_nlist.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(NlistOpts), vp, sz, vp, vp,
                                            sz, C.POINTER(sz), P64]
    lib.sfcnl_batch_build_nlist.restype = i32
    lib.sfcnl_batch_pass.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.sfcnl_batch_pass.restype = i32
    lib.sfcnl_batch_h_iterate.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(NlistOpts),
                                          C.POINTER(HiterOpts), vp, vp, sz, vp, vp, sz, vp, vp, C.POINTER(HSeed),
                                          i32, C.POINTER(HiterStats), C.POINTER(i32)]
    lib.sfcnl_batch_h_iterate.restype = i32
    _lib = lib
    return lib

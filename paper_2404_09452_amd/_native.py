"""ctypes view of the C ABI declared in include/dfjk.h.

torch is imported first on purpose: its HIP runtime carries the same soname
as the system one, so the library binds to the runtime torch already loaded
and torch's device pointers and stream handles are valid for it.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library must share)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdfjk.so")

c_i32, c_i64, c_dbl, c_sz, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
P_i32, P_dbl = ctypes.POINTER(c_i32), ctypes.POINTER(c_dbl)


class Basis(ctypes.Structure):
    _fields_ = [("nshell", c_i32), ("shell_atom", P_i32), ("shell_l", P_i32), ("shell_exp", P_dbl)]


class Options(ctypes.Structure):
    _fields_ = [("schwarz_thresh", c_dbl), ("aux_slab", c_i32), ("k_tile", c_i32)]


class Info(ctypes.Structure):
    _fields_ = [("nao", c_i64), ("naux", c_i64), ("naux_pad", c_i64), ("nshell_pairs", c_i64),
                ("sig_shell_pairs", c_i64), ("nf", c_i64), ("triplets_kept", c_i64), ("stage", c_i32)]


# name -> (restype, argtypes); every symbol include/dfjk.h declares
SIGNATURES = {
    "dfjk_options_default": (c_i32, [ctypes.POINTER(Options)]),
    "dfjk_plan_create": (c_i32, [c_i32, P_dbl, ctypes.POINTER(Basis), ctypes.POINTER(Basis),
                                 ctypes.POINTER(Options), ctypes.POINTER(c_vp)]),
    "dfjk_plan_info": (c_i32, [c_vp, ctypes.POINTER(Info)]),
    "dfjk_plan_aux_order": (c_i32, [c_vp, P_i32]),
    "dfjk_screen_bytes": (c_i32, [c_vp, ctypes.POINTER(c_sz)]),
    "dfjk_screen": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
    "dfjk_setup_bytes": (c_i32, [c_vp, ctypes.POINTER(c_sz)]),
    "dfjk_setup": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
    "dfjk_setup_batch": (c_i32, [c_i32, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp), ctypes.POINTER(c_sz), c_vp]),
    "dfjk_build_bytes": (c_i32, [c_vp, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "dfjk_build": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dfjk_build_static": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "dfjk_build_delta_bytes": (c_i32, [c_vp, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "dfjk_build_delta": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dfjk_build_batch_bytes": (c_i32, [c_i32, ctypes.POINTER(c_vp), P_i32, c_i32, ctypes.POINTER(c_sz)]),
    "dfjk_build_batch": (c_i32, [c_i32, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp), P_i32, c_i32,
                                 ctypes.POINTER(c_vp), ctypes.POINTER(c_vp), ctypes.POINTER(c_vp), c_vp, c_sz, c_vp]),
    "dfjk_autotune_bytes": (c_i32, [c_vp, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "dfjk_autotune": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_vp, c_sz, c_vp, P_i32, P_i32, P_i32, P_dbl]),
    "dfjk_build_shape": (c_i32, [c_vp, c_i32, c_i32, P_i32]),
    "dfjk_build_checked_bytes": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_sz)]),
    "dfjk_setup_host_bytes": (c_i32, [c_vp, c_sz, ctypes.POINTER(c_sz), ctypes.POINTER(c_sz)]),
    "dfjk_setup_host": (c_i32, [c_vp, c_vp, c_sz, c_vp, c_sz, c_vp]),
    "dfjk_build_checked": (c_i32, [c_vp, c_vp, c_i32, c_dbl, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp, P_i32, P_dbl]),
    "dfjk_offload_bytes": (c_i32, [c_vp, ctypes.POINTER(c_sz), ctypes.POINTER(c_sz)]),
    "dfjk_offload": (c_i32, [c_vp, c_vp, c_sz, c_vp, c_sz, c_vp]),
    "dfjk_build_host": (c_i32, [c_i32, P_dbl, ctypes.POINTER(Basis), ctypes.POINTER(Basis), ctypes.POINTER(Options),
                                P_dbl, c_i32, P_dbl, c_i32, P_dbl, P_dbl, P_dbl]),
    "dfjk_build_uks_bytes": (c_i32, [c_vp, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "dfjk_build_uks": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dfjk_direct_bytes": (c_i32, [c_vp, ctypes.POINTER(c_sz)]),
    "dfjk_direct_setup": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
    "dfjk_direct_stats": (c_i32, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "dfjk_direct_build_bytes": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_sz)]),
    "dfjk_direct_build": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dfjk_direct_build_delta_bytes": (c_i32, [c_vp, ctypes.POINTER(c_sz)]),
    "dfjk_direct_build_delta": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dfjk_export": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "dfjk_sample": (c_i32, [c_vp, c_i32, c_i64, c_vp, c_vp, c_vp]),
    "dfjk_boys": (c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp]),
    "dfjk_profile": (c_i32, [c_vp, c_i32]),
    "dfjk_profile_read": (c_i32, [c_vp, P_dbl, P_i32]),
    "dfjk_stage_name": (ctypes.c_char_p, [c_i32]),
    "dfjk_plan_destroy": (c_i32, [c_vp]),
    "dfjk_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdfjk.so is not built (run __graft_entry__.build() or "
                              "python paper_2404_09452_amd/build.py); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib

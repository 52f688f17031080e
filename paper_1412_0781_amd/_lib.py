"""ctypes loader for libffbspca.so (the C ABI declared in include/ffbspca.h).

Fails loudly when the library is missing: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libffbspca.so")

FB_FP32 = 0
FB_BF16X3 = 1

c_int = ctypes.c_int
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_uint32 = ctypes.c_uint32
c_uint64 = ctypes.c_uint64
c_double = ctypes.c_double
c_float = ctypes.c_float
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P = ctypes.POINTER


class FBInfo(ctypes.Structure):
    _fields_ = [
        ("L", c_int32), ("c", c_double), ("R", c_double),
        ("n_xi", c_int32), ("n_theta", c_int32), ("k_max", c_int32), ("p0", c_int32),
        ("p_half", c_int64), ("p_total", c_int64), ("cov_size", c_int64),
        ("grid_n", c_int32), ("kernel_w", c_int32), ("kernel_beta", c_double), ("has_device", c_int32),
    ]


# (name, restype, argtypes) for every exported entry point
SIGNATURES = [
    ("fb_plan", c_int, [c_int, c_double, c_double, P(c_void_p)]),
    ("fb_plan_host", c_int, [c_int, c_double, c_double, P(c_void_p)]),
    ("fb_plan_destroy", c_int, [c_void_p]),
    ("fb_plan_info", c_int, [c_void_p, P(FBInfo)]),
    ("fb_plan_tables", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fb_plan_host_tables", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fb_workspace_bytes", c_size_t, [c_void_p, c_int64, c_int]),
    ("fb_expand", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int, c_void_p, c_size_t, c_void_p]),
    ("fb_expand_noalloc", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int, c_void_p]),
    ("fb_adjoint", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int, c_void_p, c_size_t, c_void_p]),
    ("fb_expand_weighted", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int, c_int, c_void_p, c_size_t,
                                   c_void_p]),
    ("fb_covariance", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, P(c_int64),
                              c_int, c_void_p, c_size_t, c_void_p]),
    ("fb_covariance_workspace_bytes", c_size_t, [c_void_p, c_int64, c_int]),
    ("fb_covariance_shift", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    ("fb_eig", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                       c_void_p, c_size_t, c_void_p]),
    ("fb_eig_workspace_bytes", c_size_t, [c_void_p]),
    ("fb_spca_select", c_int, [c_void_p, c_void_p, c_int64, c_double, c_void_p, c_void_p, c_void_p]),
    ("fb_spca_coeffs", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fb_spca_reconstruct", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fb_spca_radial", c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fb_eigenimages", c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p]),
    ("fb_adjoint_filtered", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int, c_void_p, c_void_p, c_size_t,
                                    c_void_p]),
    ("fb_ctf_filter", c_int, [c_void_p, c_double, c_double, c_double, c_double, c_double, c_void_p, c_void_p]),
    ("fb_moments_workspace_bytes", c_size_t, [c_void_p]),
    ("fb_pixel_moments", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("fb_polar_power_workspace_bytes", c_size_t, [c_void_p, c_int64]),
    ("fb_polar_power", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_size_t,
                               c_void_p]),
    ("fb_estimate_support", c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_double, c_double, c_void_p,
                                    c_void_p]),
    ("fb_svd_workspace_bytes", c_size_t, [c_void_p, c_int64]),
    ("fb_svd", c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("fb_synth_normals", c_int, [c_uint64, c_uint32, c_int64, c_int64, c_int64, c_float, c_void_p, c_void_p]),
    ("fb_synth_words", c_int, [c_uint64, c_uint32, c_int64, c_int64, c_int64, c_void_p, c_void_p]),
    ("fb_profile_enable", c_int, [c_void_p, c_int]),
    ("fb_profile_read", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int]),
    ("fb_stage_name", ctypes.c_char_p, [c_int]),
    ("fb_error_string", ctypes.c_char_p, [c_int]),
    ("fb_plan_last_hip_error", c_int, [c_void_p]),
]

_lib = None


def lib():
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "(or python paper_1412_0781_amd/build.py).  There is no fallback implementation.")
        h = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


class FBError(RuntimeError):
    pass


def check(rc: int, plan_handle=None):
    if rc != 0:
        msg = lib().fb_error_string(rc).decode()
        if plan_handle is not None and rc == -3:
            msg += f" (hip error {lib().fb_plan_last_hip_error(plan_handle)})"
        raise FBError(f"libffbspca: {msg} (code {rc})")

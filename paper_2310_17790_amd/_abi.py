"""ctypes binding of include/nsf.h: argument marshalling only.

Every function here has the name of the C entry point it calls. The shared library is
the in-tree ``libnsf.so`` built by ``paper_2310_17790_amd.build``; importing this module
without it raises, so nothing silently falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnsf.so")

NSF_OK, NSF_EINVAL, NSF_ENOMEM, NSF_EHIP, NSF_ENODEV = 0, -1, -2, -3, -4
NSF_EDOMAIN, NSF_ESINGULAR, NSF_ENONFINITE, NSF_ECAPACITY = -5, -6, -7, -8
NSF_FP32, NSF_BF16, NSF_BF16_MIXED = 0, 1, 2
NSF_FLAG_DOMAIN, NSF_FLAG_NONFINITE, NSF_FLAG_SINGULAR, NSF_FLAG_CAPACITY = 1, 2, 4, 8
NSF_INTEGRATION_PLAN, NSF_INTEGRATION_CLOSURE = 0, 1
NSF_FIELD_G, NSF_FIELD_H, NSF_FIELD_L = 0, 1, 2
(NSF_BUF_U, NSF_BUF_UPREV, NSF_BUF_TAU, NSF_BUF_C, NSF_BUF_JAC, NSF_BUF_VNEW, NSF_BUF_XDEC,
 NSF_BUF_GRID, NSF_BUF_Z, NSF_BUF_NLIST, NSF_BUF_NLIVE) = range(11)

STATUS_NAMES = {0: "NSF_OK", -1: "NSF_EINVAL", -2: "NSF_ENOMEM", -3: "NSF_EHIP", -4: "NSF_ENODEV",
                -5: "NSF_EDOMAIN", -6: "NSF_ESINGULAR", -7: "NSF_ENONFINITE", -8: "NSF_ECAPACITY"}

EXPORTED = ["nsf_sim_bytes", "nsf_create_sim", "nsf_step", "nsf_step_batch", "nsf_mpm_stage",
            "nsf_refresh", "nsf_decode",
            "nsf_get_latent", "nsf_set_latent", "nsf_set_sample_count", "nsf_set_parameters",
            "nsf_status_flags", "nsf_sim_buffer",
            "nsf_destroy_sim", "nsf_last_error", "nsf_device_count", "nsf_mlp_param_count",
            "nsf_mlp_saved_floats", "nsf_mlp_workspace_bytes", "nsf_mlp_forward",
            "nsf_mlp_backward", "nsf_mlp_forward_noalloc", "nsf_adam_step", "nsf_rows_expand", "nsf_rows_segment_sum", "nsf_squared_error", "nsf_fo_bytes", "nsf_fo_create", "nsf_fo_step", "nsf_fo_buffer",
            "nsf_fo_flags", "nsf_fo_destroy"]
NSF_SQERR_WORKSPACE_BYTES = 4096   # nsf_squared_error's workspace
NSF_FO_U, NSF_FO_V, NSF_FO_C, NSF_FO_TAU, NSF_FO_F = range(5)
NSF_FO_VON_MISES, NSF_FO_DRUCKER_PRAGER, NSF_FO_HERSCHEL_BULKLEY = range(3)


class nsf_knife(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("normal", C.c_double * 3), ("offset", C.c_double),
                ("half_thickness", C.c_double), ("edge_z0", C.c_double),
                ("edge_speed", C.c_double), ("velocity", C.c_double * 3)]


class nsf_sim_desc(C.Structure):
    _fields_ = [("r", C.c_int32), ("width", C.c_int32), ("n_hidden", C.c_int32),
                ("precision", C.c_int32), ("weights", C.POINTER(C.c_float) * 3),
                ("out_scale", (C.c_double * 9) * 3), ("out_shift", (C.c_double * 9) * 3),
                ("n_particles", C.c_int64), ("X", C.POINTER(C.c_float)),
                ("rho", C.c_double), ("body_volume", C.c_double),
                ("grid_n", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
                ("gravity", C.c_double * 3), ("wall_nodes", C.c_int32), ("knife", nsf_knife),
                ("n_integration", C.c_int32), ("n_sample", C.c_int32),
                ("plan_steps", C.c_int32), ("sample_plan", C.POINTER(C.c_int32)),
                ("gn_iters", C.c_int32), ("decode_every_step", C.c_int32),
                ("z0", C.POINTER(C.c_double)), ("z_prev", C.POINTER(C.c_double)),
                ("gn_damping", C.c_double), ("integration", C.c_int32),
                ("n_mu", C.c_int32), ("mu", C.c_double * 4)]


class nsf_fo_desc(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("X", C.POINTER(C.c_float)), ("v0", C.c_double * 3),
                ("rho", C.c_double), ("body_volume", C.c_double), ("youngs", C.c_double),
                ("poisson", C.c_double), ("yield_stress", C.c_double), ("grid_n", C.c_int32),
                ("dt", C.c_double), ("gravity", C.c_double * 3), ("wall_nodes", C.c_int32),
                ("plasticity", C.c_int32), ("friction_angle", C.c_double), ("viscosity", C.c_double)]


class nsf_mlp(C.Structure):
    _fields_ = [("r", C.c_int32), ("width", C.c_int32), ("d", C.c_int32),
                ("precision", C.c_int32), ("weights", C.c_void_p)]


class NsfError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


_lib = None


def lib() -> C.CDLL:
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2310_17790_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.nsf_sim_bytes.argtypes = [C.POINTER(nsf_sim_desc)]
        L.nsf_sim_bytes.restype = sz
        L.nsf_create_sim.argtypes = [C.POINTER(nsf_sim_desc), vp, sz, vp, C.POINTER(vp)]
        L.nsf_step.argtypes = [vp, i32, vp]
        L.nsf_step_batch.argtypes = [C.POINTER(vp), i32, i32, vp]
        L.nsf_mpm_stage.argtypes = [C.POINTER(vp), i32, vp]
        L.nsf_refresh.argtypes = [vp, vp]
        L.nsf_decode.argtypes = [vp, vp, i64, vp, vp]
        L.nsf_get_latent.argtypes = [vp, vp, vp, vp, vp]
        L.nsf_set_latent.argtypes = [vp, vp, vp, i64, vp]
        L.nsf_status_flags.argtypes = [vp, C.POINTER(C.c_uint32), vp]
        L.nsf_set_sample_count.argtypes = [vp, i32, vp]
        L.nsf_set_parameters.argtypes = [vp, vp, i32, vp]
        L.nsf_fo_bytes.argtypes = [C.POINTER(nsf_fo_desc)]
        L.nsf_fo_bytes.restype = sz
        L.nsf_fo_create.argtypes = [C.POINTER(nsf_fo_desc), vp, sz, vp, C.POINTER(vp)]
        L.nsf_fo_step.argtypes = [vp, i32, vp]
        L.nsf_fo_buffer.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(i64)]
        L.nsf_fo_flags.argtypes = [vp, C.POINTER(C.c_uint32), vp]
        L.nsf_fo_destroy.argtypes = [vp]
        L.nsf_sim_buffer.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(i64)]
        L.nsf_destroy_sim.argtypes = [vp]
        L.nsf_last_error.argtypes = []
        L.nsf_last_error.restype = C.c_char_p
        L.nsf_device_count.argtypes = []
        L.nsf_device_count.restype = i32
        L.nsf_mlp_param_count.argtypes = [i32, i32, i32]
        L.nsf_mlp_param_count.restype = sz
        L.nsf_mlp_saved_floats.argtypes = [i32, i64]
        L.nsf_mlp_saved_floats.restype = sz
        L.nsf_mlp_workspace_bytes.argtypes = [C.POINTER(nsf_mlp), i64]
        L.nsf_mlp_workspace_bytes.restype = sz
        L.nsf_mlp_forward.argtypes = [C.POINTER(nsf_mlp), vp, vp, i64, vp, vp, vp, sz, vp]
        L.nsf_mlp_backward.argtypes = [C.POINTER(nsf_mlp), vp, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.nsf_mlp_forward_noalloc.argtypes = [C.POINTER(nsf_mlp), vp, vp, i64, vp, vp, vp]
        L.nsf_adam_step.argtypes = [vp, vp, vp, vp, i64, C.c_double, C.c_double, C.c_double, C.c_double, i64, vp]
        L.nsf_rows_expand.argtypes = [vp, vp, i32, i32, vp, vp]
        L.nsf_rows_segment_sum.argtypes = [vp, vp, i32, i32, vp, vp]
        L.nsf_squared_error.argtypes = [vp, i32, i64, vp, i64, vp, vp, i64, vp, vp, vp, vp]
        for name in ("nsf_create_sim", "nsf_step", "nsf_step_batch", "nsf_mpm_stage", "nsf_refresh", "nsf_decode", "nsf_get_latent",
                     "nsf_set_latent", "nsf_status_flags", "nsf_sim_buffer", "nsf_destroy_sim",
                     "nsf_mlp_forward", "nsf_mlp_backward", "nsf_mlp_forward_noalloc", "nsf_adam_step",
                     "nsf_rows_expand", "nsf_rows_segment_sum", "nsf_squared_error"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != NSF_OK:
        raise NsfError(status, lib().nsf_last_error().decode())


# ---- thin wrappers with the C names ----------------------------------------------------
def nsf_sim_bytes(desc: nsf_sim_desc) -> int:
    return int(lib().nsf_sim_bytes(C.byref(desc)))


def nsf_create_sim(desc: nsf_sim_desc, arena_ptr: int, arena_bytes: int, stream: int) -> int:
    h = C.c_void_p()
    check(lib().nsf_create_sim(C.byref(desc), arena_ptr, arena_bytes, stream or None, C.byref(h)))
    return h.value


def nsf_step(sim: int, n_steps: int, stream: int) -> None:
    check(lib().nsf_step(sim, n_steps, stream or None))


def nsf_step_batch(sims, n_steps: int, stream: int) -> None:
    arr = (C.c_void_p * len(sims))(*sims)
    check(lib().nsf_step_batch(arr, len(sims), n_steps, stream or None))


def nsf_mpm_stage(sims, stream: int) -> None:
    arr = (C.c_void_p * len(sims))(*sims)
    check(lib().nsf_mpm_stage(arr, len(sims), stream or None))


def nsf_refresh(sim: int, stream: int) -> None:
    check(lib().nsf_refresh(sim, stream or None))


def nsf_decode(sim: int, X_ptr: int | None, n: int, out_ptr: int, stream: int) -> None:
    check(lib().nsf_decode(sim, X_ptr or None, n, out_ptr, stream or None))


def nsf_get_latent(sim: int, r: int, stream: int):
    z = (C.c_double * r)()
    zp = (C.c_double * r)()
    st = C.c_int64()
    check(lib().nsf_get_latent(sim, z, zp, C.byref(st), stream or None))
    return list(z), list(zp), int(st.value)


def nsf_set_latent(sim: int, z, z_prev, step: int, stream: int) -> None:
    r = len(z)
    za = (C.c_double * r)(*[float(v) for v in z])
    zpa = (C.c_double * r)(*[float(v) for v in z_prev]) if z_prev is not None else None
    check(lib().nsf_set_latent(sim, za, zpa, step, stream or None))


def nsf_set_sample_count(sim: int, n_sample: int, stream: int) -> None:
    check(lib().nsf_set_sample_count(sim, n_sample, stream or None))


def nsf_set_parameters(sim: int, mu, stream: int) -> None:
    n = len(mu)
    arr = (C.c_double * max(n, 1))(*[float(v) for v in mu])
    check(lib().nsf_set_parameters(sim, arr, n, stream or None))


def nsf_status_flags(sim: int, stream: int):
    f = C.c_uint32()
    st = lib().nsf_status_flags(sim, C.byref(f), stream or None)
    return st, int(f.value)


def nsf_sim_buffer(sim: int, which: int):
    p = C.c_void_p()
    n = C.c_int64()
    check(lib().nsf_sim_buffer(sim, which, C.byref(p), C.byref(n)))
    return p.value, int(n.value)


def nsf_destroy_sim(sim: int) -> None:
    check(lib().nsf_destroy_sim(sim))


def nsf_last_error() -> str:
    return lib().nsf_last_error().decode()


def nsf_device_count() -> int:
    return int(lib().nsf_device_count())

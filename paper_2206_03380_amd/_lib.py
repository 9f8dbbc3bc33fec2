"""ctypes binding of libmcdi.so: argument marshalling only.

Every step of the method runs in the HIP kernels behind the C ABI.  If the
library has not been built, loading fails with an error; there is no
fallback implementation.
"""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcdi.so")

MCDI_OK, MCDI_E_INVALID, MCDI_E_OOM, MCDI_E_DEVICE, MCDI_E_UNSUPPORTED = 0, -1, -2, -3, -4
FLAG_LIGHT_OFF = 1 << 0
FLAG_FORCE_COS = 1 << 1
FLAG_BSDF_OFF = 1 << 2
FLAG_FORCE_GGX = 1 << 3
FLAG_BILINEAR = 1 << 4
FLAG_DUMP = 1 << 8
FLAG_DUMP_DIRS = 1 << 10
FLAG_TIME_TRACE = 1 << 9
FLAG_TIME_ADJOINT = 1 << 11

vp = C.c_void_p


class MCDIError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("mcdi status %d: %s" % (status, msg))
        self.status = status


class Allocator(C.Structure):
    _fields_ = [("ctx", vp), ("alloc", C.CFUNCTYPE(vp, vp, C.c_size_t, vp)),
                ("free", C.CFUNCTYPE(None, vp, vp, vp))]


class GBuffer(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("height", C.c_int32), ("width", C.c_int32),
                ("view_base", C.c_int32), ("pos", vp), ("nrm", vp), ("kd", vp), ("korm", vp),
                ("mask", vp), ("eye", vp)]


class Params(C.Structure):
    _fields_ = [("spp", C.c_int32), ("flags", C.c_uint32), ("seed", C.c_uint64), ("tau", C.c_float),
                ("ray_eps", C.c_float), ("decisions", vp), ("live", vp)]


class ServerConfig(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("launch_samples", C.c_int64), ("slots", C.c_int32),
                ("spp_max", C.c_int32), ("n_workgroups", C.c_int32), ("reserved", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("scene", vp), ("env", vp), ("gbuf", GBuffer), ("params", Params), ("c_d", vp), ("c_s", vp),
                ("g_cd", vp), ("g_cs", vp), ("g_kd", vp), ("g_korm", vp), ("g_nrm", vp), ("g_env", vp)]


class ServerInfo(C.Structure):
    _fields_ = [("used_bytes", C.c_int64), ("launches", C.c_int64), ("queued", C.c_int32),
                ("admitted", C.c_int32), ("in_flight", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("valid_pixels", C.c_uint64), ("invalid_pixels", C.c_uint64), ("rays_traced", C.c_uint64),
                ("rays_hit", C.c_uint64), ("samples_culled", C.c_uint64), ("box_tests", C.c_uint64),
                ("tri_tests", C.c_uint64), ("box_slots", C.c_uint64), ("tri_slots", C.c_uint64),
                ("box_lanes", C.c_uint64)]


class BilateralGuide(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("height", C.c_int32), ("width", C.c_int32), ("depth", C.c_void_p),
                ("nrm", C.c_void_p), ("mask", C.c_void_p), ("sigma", C.c_float), ("sigma_z", C.c_float),
                ("sigma_n", C.c_float)]


class SceneInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_nodes", C.c_int32), ("max_depth", C.c_int32),
                ("bad_tris", C.c_int32), ("n_groups", C.c_int32), ("wide", C.c_int32),
                ("depth_complexity", C.c_float), ("n_big", C.c_int32)]


_lib = None


def lib():
    """Load libmcdi.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmcdi.so is not built (run paper_2206_03380_amd/build.py or "
                          "__graft_entry__.build()); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    L.mcdi_build_scene.restype = C.c_int
    L.mcdi_build_scene.argtypes = [vp, C.c_int64, vp, C.c_int64, vp, vp, C.POINTER(vp)]
    L.mcdi_destroy_scene.argtypes = [vp]
    L.mcdi_destroy_scene.restype = None
    L.mcdi_scene_info.argtypes = [vp, C.POINTER(SceneInfo)]
    L.mcdi_scene_info.restype = C.c_int
    L.mcdi_scene_nodes.argtypes = [vp, vp, vp, vp]
    L.mcdi_scene_nodes.restype = C.c_int
    L.mcdi_build_env_cdf.restype = C.c_int
    L.mcdi_build_env_cdf.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, C.POINTER(vp)]
    L.mcdi_destroy_env.argtypes = [vp]
    L.mcdi_destroy_env.restype = None
    L.mcdi_env_tables.argtypes = [vp, vp, vp, vp, vp]
    L.mcdi_env_tables.restype = C.c_int
    L.mcdi_shade_fwd.restype = C.c_int
    L.mcdi_shade_fwd.argtypes = [vp, vp, C.POINTER(GBuffer), C.POINTER(Params), vp, vp, vp, vp, vp]
    L.mcdi_shade_fwd_frozen.restype = C.c_int
    L.mcdi_shade_fwd_frozen.argtypes = [vp, vp, C.POINTER(GBuffer), vp, C.POINTER(GBuffer), C.POINTER(Params), vp,
                                        vp, vp]
    L.mcdi_shade_bwd.restype = C.c_int
    L.mcdi_shade_bwd.argtypes = [vp, vp, C.POINTER(GBuffer), C.POINTER(Params), vp, vp, vp, vp, vp, vp,
                                 vp, vp, vp]
    L.mcdi_trace_anyhit.restype = C.c_int
    L.mcdi_trace_anyhit.argtypes = [vp, vp, vp, C.c_int64, vp, C.c_int32, vp]
    L.mcdi_trace_times.restype = C.c_int
    L.mcdi_trace_times.argtypes = [C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
    L.mcdi_adjoint_times.restype = C.c_int
    L.mcdi_adjoint_times.argtypes = [C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
    L.mcdi_server_create.restype = C.c_int
    L.mcdi_server_create.argtypes = [C.POINTER(ServerConfig), vp, vp, C.POINTER(vp)]
    L.mcdi_server_request_bytes.restype = C.c_int64
    L.mcdi_server_request_bytes.argtypes = [C.c_int64, C.c_int32]
    L.mcdi_server_submit.restype = C.c_int
    L.mcdi_server_submit.argtypes = [vp, C.POINTER(Request), vp, C.POINTER(C.c_int64)]
    L.mcdi_server_poll.restype = C.c_int
    L.mcdi_server_poll.argtypes = [vp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]
    L.mcdi_server_wait.restype = C.c_int
    L.mcdi_server_wait.argtypes = [vp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]
    L.mcdi_server_info.restype = C.c_int
    L.mcdi_server_info.argtypes = [vp, C.POINTER(ServerInfo)]
    L.mcdi_server_destroy.restype = None
    L.mcdi_server_destroy.argtypes = [vp]
    L.mcdi_image_loss.restype = C.c_int
    L.mcdi_image_loss.argtypes = [vp, vp, vp, vp, vp, C.c_int64, C.c_float, vp, vp, vp, vp, vp, vp]
    L.mcdi_image_loss_noalloc.restype = C.c_int
    L.mcdi_image_loss_noalloc.argtypes = [vp, vp, vp, vp, vp, C.c_int64, C.c_float, vp, vp, vp, vp, vp]
    L.mcdi_bilateral_radius.restype = C.c_int32
    L.mcdi_bilateral_radius.argtypes = [C.c_float]
    L.mcdi_bilateral_fwd.restype = C.c_int
    L.mcdi_bilateral_fwd.argtypes = [C.POINTER(BilateralGuide), C.c_int32, vp, vp, vp, vp]
    L.mcdi_bilateral_bwd.restype = C.c_int
    L.mcdi_bilateral_bwd.argtypes = [C.POINTER(BilateralGuide), C.c_int32, vp, vp, vp, vp]
    L.mcdi_view_depth.restype = C.c_int
    L.mcdi_view_depth.argtypes = [C.POINTER(GBuffer), vp, vp]
    L.mcdi_build_edges.restype = C.c_int
    L.mcdi_build_edges.argtypes = [vp, C.c_int64, C.c_int64, vp, vp, C.POINTER(vp)]
    L.mcdi_destroy_edges.restype = None
    L.mcdi_destroy_edges.argtypes = [vp]
    L.mcdi_edges_count.restype = C.c_int
    L.mcdi_edges_count.argtypes = [vp, C.POINTER(C.c_int64)]
    L.mcdi_edges_copy.restype = C.c_int
    L.mcdi_edges_copy.argtypes = [vp, vp, vp]
    L.mcdi_shade_bwd_edges.restype = C.c_int
    L.mcdi_shade_bwd_edges.argtypes = [vp, vp, vp, vp, C.c_int64, C.POINTER(GBuffer), C.POINTER(Params), C.c_int32,
                                       C.c_uint32, vp, vp, vp, vp, vp]
    L.mcdi_last_error.restype = C.c_char_p
    L.mcdi_version.restype = C.c_char_p
    _lib = L
    return L


def check(status):
    if status != MCDI_OK:
        raise MCDIError(status, lib().mcdi_last_error().decode())


EXPORTED = ("mcdi_build_scene", "mcdi_destroy_scene", "mcdi_scene_info", "mcdi_scene_nodes", "mcdi_build_env_cdf",
            "mcdi_destroy_env", "mcdi_env_tables", "mcdi_shade_fwd", "mcdi_shade_fwd_frozen", "mcdi_shade_bwd",
            "mcdi_trace_anyhit", "mcdi_trace_times", "mcdi_adjoint_times", "mcdi_server_create",
            "mcdi_server_request_bytes", "mcdi_server_submit", "mcdi_server_poll", "mcdi_server_wait",
            "mcdi_server_info", "mcdi_server_destroy", "mcdi_image_loss", "mcdi_image_loss_noalloc", "mcdi_bilateral_radius", "mcdi_bilateral_fwd",
            "mcdi_bilateral_bwd", "mcdi_view_depth", "mcdi_build_edges", "mcdi_destroy_edges", "mcdi_edges_count",
            "mcdi_edges_copy", "mcdi_shade_bwd_edges", "mcdi_last_error", "mcdi_version")

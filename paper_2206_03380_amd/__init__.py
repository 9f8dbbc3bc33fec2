"""Differentiable Monte Carlo direct illumination on AMD MI355X.

Thin torch-facing wrappers over the C ABI in include/mcdi.h.  torch provides
device memory and streams; every step of the estimator runs in the HIP
kernels of libmcdi.so.
"""

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from ._lib import (MCDIError, FLAG_LIGHT_OFF, FLAG_FORCE_COS, FLAG_BSDF_OFF, FLAG_FORCE_GGX, FLAG_BILINEAR,  # noqa: F401
                   FLAG_DUMP, FLAG_DUMP_DIRS, FLAG_TIME_TRACE, FLAG_TIME_ADJOINT)

__all__ = ["Scene", "Env", "GBuffer", "Edges", "shade_fwd", "shade_bwd", "shade_bwd_edges", "trace_anyhit",
           "MCDIShade", "MCDIError", "new_stats", "read_stats"]


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _need(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


# torch's caching allocator behind the library's allocator hook
@C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
def _torch_alloc(ctx, nbytes, stream):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # out of memory: report NULL to the library
        return None


@C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
def _torch_free(ctx, ptr, stream):
    torch.cuda.caching_allocator_delete(ptr)


_TORCH_ALLOCATOR = L.Allocator(None, _torch_alloc, _torch_free)


class Scene:
    """BVH over a triangle mesh (device float32 [Nv,3] vertices, int32 [Nt,3])."""

    def __init__(self, verts, tris, stream=None, use_torch_allocator=True):
        _need(verts, torch.float32, name="verts")
        _need(tris, torch.int32, name="tris")
        if verts.dim() != 2 or verts.shape[1] != 3 or tris.dim() != 2 or tris.shape[1] != 3:
            raise ValueError("verts must be [Nv,3] and tris [Nt,3]")
        h = C.c_void_p()
        L.check(L.lib().mcdi_build_scene(_ptr(verts), verts.shape[0], _ptr(tris), tris.shape[0],
                                         C.byref(_TORCH_ALLOCATOR) if use_torch_allocator else None,
                                         _stream(stream), C.byref(h)))
        self.handle = h
        self.n_tris = tris.shape[0]

    def info(self):
        i = L.SceneInfo()
        L.check(L.lib().mcdi_scene_info(self.handle, C.byref(i)))
        return {"n_tris": i.n_tris, "n_nodes": i.n_nodes, "max_depth": i.max_depth, "bad_tris": i.bad_tris,
                "n_groups": i.n_groups, "wide": i.wide, "depth_complexity": i.depth_complexity,
                "n_big": i.n_big}

    def nodes(self, stream=None):
        """The BVH as device tensors: nodes int32 [n_nodes, 8] (lo xyz and hi
        xyz as float bits, escape at column 3, payload at column 7) and the
        triangles in leaf order, float32 [n_tris, 3, 4]."""
        n = self.info()["n_nodes"]
        dev = torch.device("cuda", torch.cuda.current_device())
        nodes = torch.empty((max(n, 0), 8), dtype=torch.int32, device=dev)
        tris = torch.empty((self.n_tris, 3, 4), dtype=torch.float32, device=dev)
        L.check(L.lib().mcdi_scene_nodes(self.handle, _ptr(nodes) if n > 0 else None,
                                         _ptr(tris) if self.n_tris > 0 else None, _stream(stream)))
        return nodes, tris

    def close(self):
        if getattr(self, "handle", None):
            L.lib().mcdi_destroy_scene(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Env:
    """Sampling tables of a lat-long probe (device float32 [H,W,3]) and a
    packed copy of its radiance made with them; keeps a reference to the probe
    tensor they were built from (the autograd function sends the probe
    gradient there).  Build a new Env after changing the probe."""

    def __init__(self, env, stream=None, use_torch_allocator=True):
        _need(env, torch.float32, name="env")
        if env.dim() != 3 or env.shape[2] != 3:
            raise ValueError("env must be [H,W,3]")
        self.env = env
        self.H, self.W = env.shape[0], env.shape[1]
        h = C.c_void_p()
        L.check(L.lib().mcdi_build_env_cdf(_ptr(env), self.H, self.W,
                                           C.byref(_TORCH_ALLOCATOR) if use_torch_allocator else None,
                                           _stream(stream), C.byref(h)))
        self.handle = h

    def tables(self, stream=None):
        """Copies of the FP32 tables (cond [H,W+1], marg [H+1], pdf [H,W])."""
        dev = self.env.device
        cond = torch.empty((self.H, self.W + 1), dtype=torch.float32, device=dev)
        marg = torch.empty(self.H + 1, dtype=torch.float32, device=dev)
        pdf = torch.empty((self.H, self.W), dtype=torch.float32, device=dev)
        L.check(L.lib().mcdi_env_tables(self.handle, _ptr(cond), _ptr(marg), _ptr(pdf), _stream(stream)))
        return cond, marg, pdf

    def close(self):
        if getattr(self, "handle", None):
            L.lib().mcdi_destroy_env(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class GBuffer:
    """Planar per-pixel G-buffer on the device."""
    pos: torch.Tensor      # f32 [3, N]
    nrm: torch.Tensor      # f32 [3, N]
    kd: torch.Tensor       # f32 [3, N]
    korm: torch.Tensor     # f32 [3, N]
    mask: torch.Tensor     # u8 [N]
    eye: torch.Tensor      # f32 [V, 3]
    n_views: int
    height: int
    width: int
    view_base: int = 0

    @property
    def n(self):
        return self.n_views * self.height * self.width

    def struct(self, kd=None, korm=None, nrm=None):
        n = self.n
        for name in ("pos", "nrm", "kd", "korm"):
            _need(getattr(self, name), torch.float32, (3, n), name)
        _need(self.mask, torch.uint8, (n,), "mask")
        _need(self.eye, torch.float32, (self.n_views, 3), "eye")
        return L.GBuffer(self.n_views, self.height, self.width, self.view_base, self.pos.data_ptr(),
                         (nrm if nrm is not None else self.nrm).data_ptr(),
                         (kd if kd is not None else self.kd).data_ptr(),
                         (korm if korm is not None else self.korm).data_ptr(), self.mask.data_ptr(),
                         self.eye.data_ptr())

    @staticmethod
    def from_workload(w, device="cuda"):
        t = lambda a: torch.from_numpy(a).to(device).contiguous()  # noqa: E731
        return GBuffer(t(w.pos), t(w.nrm), t(w.kd), t(w.korm), t(w.mask), t(w.eye), w.n_views, w.height,
                       w.width, w.view_base)


def hit_words(spp):
    return (2 * spp + 31) // 32


def new_stats(device="cuda"):
    return torch.zeros(10, dtype=torch.int64, device=device)


def read_stats(t):
    v = t.cpu().tolist()
    return {"valid_pixels": v[0], "invalid_pixels": v[1], "rays_traced": v[2], "rays_hit": v[3],
            "samples_culled": v[4], "box_tests": v[5], "tri_tests": v[6], "box_slots": v[7], "tri_slots": v[8],
            "box_lanes": v[9]}


def _params(spp, seed, tau, ray_eps, flags, decisions, live=None):
    return L.Params(int(spp), int(flags), int(seed), float(tau), float(ray_eps),
                    decisions.data_ptr() if decisions is not None else None,
                    live.data_ptr() if live is not None else None)


def shade_fwd(scene, env, gb, spp, seed=0, tau=1.0, ray_eps=1e-3, flags=0, hitbits=True, decisions=False,
              stats=None, out=None, stream=None, live=None):
    """Forward pass.  Returns (c_d [3,N], c_s [3,N], hitbits [words,N] or None,
    decisions [N,spp,3] or None).  decisions="dirs": records of 9 words
    [N,spp,9], the last six the light and BSDF samples' world directions
    (float32 bits).  live: an int32 [words,N] tensor the forward fills with
    the samples it evaluates, for shade_bwd (with tau != 0)."""
    n = gb.n
    dev = gb.pos.device
    if out is None:
        c_d = torch.empty((3, n), dtype=torch.float32, device=dev)
        c_s = torch.empty((3, n), dtype=torch.float32, device=dev)
        hb = torch.empty((hit_words(spp), n), dtype=torch.int32, device=dev) if hitbits else None
    else:
        c_d, c_s, hb = out
    dec = None
    if decisions:
        dirs = decisions == "dirs"
        dec = torch.empty((n, spp, 9 if dirs else 3), dtype=torch.int32, device=dev)
        flags |= FLAG_DUMP | (FLAG_DUMP_DIRS if dirs else 0)
    if live is not None:
        _need(live, torch.int32, (hit_words(spp), n), "live")
    gs = gb.struct()
    prm = _params(spp, seed, tau, ray_eps, flags, dec, live)
    L.check(L.lib().mcdi_shade_fwd(scene.handle, env.handle, C.byref(gs), C.byref(prm), _ptr(c_d), _ptr(c_s),
                                   _ptr(hb), _ptr(stats), _stream(stream)))
    return c_d, c_s, hb, dec


def shade_fwd_frozen(scene, env_s, gb_s, env_e, gb_e, spp, seed=0, tau=1.0, ray_eps=1e-3, flags=0,
                     stream=None):
    """Forward pass with frozen sampling (test hook): gb_s / env_s draw the
    samples, gb_e (nrm, kd, korm) / env_e (radiance) evaluate them.
    Returns (c_d, c_s)."""
    n = gb_s.n
    dev = gb_s.pos.device
    c_d = torch.empty((3, n), dtype=torch.float32, device=dev)
    c_s = torch.empty((3, n), dtype=torch.float32, device=dev)
    g1, g2 = gb_s.struct(), gb_e.struct()
    prm = _params(spp, seed, tau, ray_eps, flags, None)
    L.check(L.lib().mcdi_shade_fwd_frozen(scene.handle, env_s.handle, C.byref(g1), env_e.handle, C.byref(g2),
                                          C.byref(prm), _ptr(c_d), _ptr(c_s), _stream(stream)))
    return c_d, c_s


def shade_bwd(scene, env, gb, spp, g_cd, g_cs, hitbits=None, seed=0, tau=1.0, ray_eps=1e-3, flags=0,
              g_env=None, stats=None, out=None, stream=None, live=None):
    """Backward pass.  Returns (g_kd, g_korm, g_nrm, g_env); g_env is
    accumulated into if given, else a zeroed [H,W,3] tensor is created.
    live: the forward's live samples (with its hit bits): the adjoint then
    draws only those."""
    n = gb.n
    dev = gb.pos.device
    _need(g_cd, torch.float32, (3, n), "g_cd")
    _need(g_cs, torch.float32, (3, n), "g_cs")
    if out is None:
        g_kd = torch.empty((3, n), dtype=torch.float32, device=dev)
        g_korm = torch.empty((3, n), dtype=torch.float32, device=dev)
        g_nrm = torch.empty((3, n), dtype=torch.float32, device=dev)
    else:
        g_kd, g_korm, g_nrm = out
    if g_env is None:
        g_env = torch.zeros((env.H, env.W, 3), dtype=torch.float32, device=dev)
    if live is not None:
        _need(live, torch.int32, (hit_words(spp), n), "live")
    gs = gb.struct()
    prm = _params(spp, seed, tau, ray_eps, flags, None, live)
    L.check(L.lib().mcdi_shade_bwd(scene.handle, env.handle, C.byref(gs), C.byref(prm), _ptr(g_cd), _ptr(g_cs),
                                   _ptr(hitbits), _ptr(g_kd), _ptr(g_korm), _ptr(g_nrm), _ptr(g_env),
                                   _ptr(stats), _stream(stream)))
    return g_kd, g_korm, g_nrm, g_env


class Edges:
    """Unique edges of a triangle mesh (device int32 [Nt,3] indices over Nv
    vertices) with the opposite corners of their faces, for the edge-sampled
    visibility gradient."""

    def __init__(self, tris, n_verts, stream=None, use_torch_allocator=True):
        _need(tris, torch.int32, name="tris")
        if tris.dim() != 2 or tris.shape[1] != 3:
            raise ValueError("tris must be [Nt,3]")
        h = C.c_void_p()
        L.check(L.lib().mcdi_build_edges(_ptr(tris), tris.shape[0], int(n_verts),
                                         C.byref(_TORCH_ALLOCATOR) if use_torch_allocator else None,
                                         _stream(stream), C.byref(h)))
        self.handle = h
        self.n_verts = int(n_verts)

    def count(self):
        n = C.c_int64()
        L.check(L.lib().mcdi_edges_count(self.handle, C.byref(n)))
        return n.value

    def rows(self, stream=None):
        """The edge rows (a, b, c, d) as a device int32 [E, 4] tensor."""
        n = self.count()
        out = torch.empty((n, 4), dtype=torch.int32, device=torch.device("cuda", torch.cuda.current_device()))
        if n > 0:
            L.check(L.lib().mcdi_edges_copy(self.handle, _ptr(out), _stream(stream)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            L.lib().mcdi_destroy_edges(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shade_bwd_edges(scene, env, edges, verts, gb, edge_spp, g_cd, g_cs, seed=0, tau=1.0, ray_eps=1e-3, flags=0,
                    g_verts=None, stats=None, stream=None, sharp_gain=1):
    """Edge-sampled visibility gradient of the shadow term with respect to the
    vertex positions verts [Nv,3] (the mesh of scene and edges); sharp edges
    are sharp_gain times as likely per edge as the others (1: uniform).
    Returns g_verts [Nv,3], accumulated into if given, else a zeroed tensor."""
    n = gb.n
    _need(verts, torch.float32, name="verts")
    _need(g_cd, torch.float32, (3, n), "g_cd")
    _need(g_cs, torch.float32, (3, n), "g_cs")
    if g_verts is None:
        g_verts = torch.zeros(verts.shape, dtype=torch.float32, device=verts.device)
    _need(g_verts, torch.float32, tuple(verts.shape), "g_verts")
    gs = gb.struct()
    prm = _params(1, seed, tau, ray_eps, flags, None)
    L.check(L.lib().mcdi_shade_bwd_edges(scene.handle, env.handle, edges.handle, _ptr(verts), verts.shape[0],
                                         C.byref(gs), C.byref(prm), int(edge_spp), int(sharp_gain), _ptr(g_cd),
                                         _ptr(g_cs),
                                         _ptr(g_verts), _ptr(stats), _stream(stream)))
    return g_verts


def trace_times():
    """Traversal-kernel durations (ms) of the calls made with FLAG_TIME_TRACE
    since the previous call (HIP events on the launch stream)."""
    buf = (C.c_float * 1024)()
    n = C.c_int32()
    L.check(L.lib().mcdi_trace_times(buf, 1024, C.byref(n)))
    return [buf[i] for i in range(n.value)]


def adjoint_times():
    """Adjoint-kernel durations (ms) of the backward calls made with
    FLAG_TIME_ADJOINT since the previous call (HIP events on the launch
    stream)."""
    buf = (C.c_float * 1024)()
    n = C.c_int32()
    L.check(L.lib().mcdi_adjoint_times(buf, 1024, C.byref(n)))
    return [buf[i] for i in range(n.value)]


def image_loss(kd, c_d, c_s, ref, mask, w_light=0.15, stream=None, out=None, noalloc=False):
    """Loss of the composed image (kd*c_d + c_s) against ref: L1 on tonemapped
    colours + w_light * light regulariser.  Returns (loss [3] = (L_image,
    L_light, L), g_kd, g_cd, g_cs), all on the device; `out` may pass the
    four buffers in.  noalloc: the library's allocation-free entry point
    (static scratch; calls overlapping on one device race)."""
    n = mask.shape[0]
    for name, t in (("kd", kd), ("c_d", c_d), ("c_s", c_s), ("ref", ref)):
        _need(t, torch.float32, (3, n), name)
    _need(mask, torch.uint8, (n,), "mask")
    if out is None:
        out = (torch.empty(3, dtype=torch.float32, device=kd.device),) + tuple(
            torch.empty((3, n), dtype=torch.float32, device=kd.device) for _ in range(3))
    loss, g_kd, g_cd, g_cs = out
    _need(loss, torch.float32, (3,), "loss")
    for name, t in (("g_kd", g_kd), ("g_cd", g_cd), ("g_cs", g_cs)):
        _need(t, torch.float32, (3, n), name)
    if noalloc:
        L.check(L.lib().mcdi_image_loss_noalloc(_ptr(kd), _ptr(c_d), _ptr(c_s), _ptr(ref), _ptr(mask), n,
                                                float(w_light), _ptr(loss), _ptr(g_kd), _ptr(g_cd), _ptr(g_cs),
                                                _stream(stream)))
    else:
        L.check(L.lib().mcdi_image_loss(_ptr(kd), _ptr(c_d), _ptr(c_s), _ptr(ref), _ptr(mask), n, float(w_light),
                                        _ptr(loss), _ptr(g_kd), _ptr(g_cd), _ptr(g_cs), C.byref(_TORCH_ALLOCATOR),
                                        _stream(stream)))
    return loss, g_kd, g_cd, g_cs


def shadow_tau(iteration, ramp=1750):
    """Light-leakage parameter of the shadow ramp: tau rises linearly from 0
    to 1 over the first `ramp` iterations, so shadowed samples are weighted
    by H = 1 - tau (appendix A)."""
    return min(max(iteration / float(ramp), 0.0), 1.0) if ramp > 0 else 1.0


def decorrelated_seed(seed):
    """A backward seed independent of the forward's Philox stream."""
    return (int(seed) ^ 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF


def denoise_sigma(iteration, ramp=1750, lo=1e-4, hi=2.0):
    """Spatial footprint of the bilateral denoiser during optimisation: linear
    from lo to hi over the first `ramp` iterations, then hi (appendix B)."""
    f = min(max(iteration / float(ramp), 0.0), 1.0) if ramp > 0 else 1.0
    return lo + (hi - lo) * f


def bilateral_radius(sigma):
    """Footprint radius R of the filter for spatial std-dev sigma (pixels)."""
    return int(L.lib().mcdi_bilateral_radius(float(sigma)))


@dataclass
class BilateralGuide:
    """Edge-stopping guides of the cross-bilateral denoiser for V views of
    H x W pixels: depth f32 [N], normal f32 [3, N], mask u8 [N]."""
    depth: torch.Tensor
    nrm: torch.Tensor
    mask: torch.Tensor
    n_views: int
    height: int
    width: int
    sigma: float = 2.0
    sigma_z: float = 1.0
    sigma_n: float = 128.0

    @property
    def n(self):
        return self.n_views * self.height * self.width

    def struct(self):
        n = self.n
        _need(self.depth, torch.float32, (n,), "depth")
        _need(self.nrm, torch.float32, (3, n), "nrm")
        _need(self.mask, torch.uint8, (n,), "mask")
        return L.BilateralGuide(self.n_views, self.height, self.width, self.depth.data_ptr(), self.nrm.data_ptr(),
                                self.mask.data_ptr(), float(self.sigma), float(self.sigma_z), float(self.sigma_n))

    @staticmethod
    def from_gbuffer(gb, sigma=2.0, sigma_z=1.0, sigma_n=128.0, stream=None):
        return BilateralGuide(view_depth(gb, stream), gb.nrm, gb.mask, gb.n_views, gb.height, gb.width, sigma,
                              sigma_z, sigma_n)


def view_depth(gb, stream=None):
    """Depth guide |pos - eye| of a G-buffer (0 where mask is 0), f32 [N]."""
    gs = gb.struct()
    depth = torch.empty(gb.n, dtype=torch.float32, device=gb.pos.device)
    L.check(L.lib().mcdi_view_depth(C.byref(gs), _ptr(depth), _stream(stream)))
    return depth


def bilateral_fwd(guide, x, stream=None, out=None):
    """Filter x [C, N] (C in 1, 3, 6).  Returns (out [C, N], wsum [N]);
    `out` may pass both buffers in."""
    gs = guide.struct()
    _need(x, torch.float32, (x.shape[0], guide.n), "x")
    if out is None:
        out = (torch.empty_like(x), torch.empty(guide.n, dtype=torch.float32, device=x.device))
    out, wsum = out
    _need(out, torch.float32, tuple(x.shape), "out")
    _need(wsum, torch.float32, (guide.n,), "wsum")
    L.check(L.lib().mcdi_bilateral_fwd(C.byref(gs), x.shape[0], _ptr(x), _ptr(out), _ptr(wsum), _stream(stream)))
    return out, wsum


def bilateral_bwd(guide, g_out, wsum, stream=None, out=None):
    """Gradient with respect to the filtered colours for upstream g_out [C, N]."""
    gs = guide.struct()
    _need(g_out, torch.float32, (g_out.shape[0], guide.n), "g_out")
    _need(wsum, torch.float32, (guide.n,), "wsum")
    g_in = torch.empty_like(g_out) if out is None else _need(out, torch.float32, tuple(g_out.shape), "out")
    L.check(L.lib().mcdi_bilateral_bwd(C.byref(gs), g_out.shape[0], _ptr(g_out), _ptr(wsum), _ptr(g_in),
                                       _stream(stream)))
    return g_in


def trace_anyhit(scene, orig, dirs, brute=False, stream=None, mode=None):
    """orig, dirs: device f32 [3, n].  Returns uint8 [n] (1 = occluded).
    mode: "binary", "brute" or "wide" (default: "brute" if brute else
    "binary")."""
    n = orig.shape[1]
    _need(orig, torch.float32, (3, n), "orig")
    _need(dirs, torch.float32, (3, n), "dirs")
    hit = torch.empty(n, dtype=torch.uint8, device=orig.device)
    m = {"binary": 0, "brute": 1, "wide": 2}[mode or ("brute" if brute else "binary")]
    L.check(L.lib().mcdi_trace_anyhit(scene.handle, _ptr(orig), _ptr(dirs), n, _ptr(hit), m, _stream(stream)))
    return hit


from .autograd import MCDIShade, Bilateral, ImageLoss  # noqa: E402,F401

"""The synthetic workloads, named by what they are.

  tiny      one 64x64 view of a 320-triangle icosphere over a 2-triangle ground
            quad, env 64x32 lognormal(0,1) with a 4x4 patch x50, 4 spp.
  sphere8   8 views at 512x512 of a displaced sphere (100,820 triangles,
            amplitude 0.05) with 20 box occluders, kd/korm from 1024^2 RGBA8
            smooth-noise textures, env 512x256 lognormal(0,1.5) + 4x4 sun x1000,
            8 spp.
  sphere8_grad   the sphere8 scene at 12 spp with forward + backward.
  lattice   4 views at 1024x1024 inside a closed room with four windows, of a
            32^3-cell lattice of thin beams (~1.0M triangles); env 2048x1024
            lognormal(0,1) + three 8x8 sources x1000; 32 spp.

Per-pixel arrays are planar [C][N] float32 with N = views*H*W and pixel id
(view*H + y)*W + x.  The mask is uint8 [N]; eye positions are [views][3].
Random streams are numpy PCG64(1000 + k) for workload k.
"""

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import meshes
from .raycast import (look_at_rays, Hits, hit_sphere, hit_rect_y, hit_box,
                      DisplacedSphere)


@dataclass
class Workload:
    name: str
    verts: np.ndarray          # f32 [Nv, 3]
    tris: np.ndarray           # i32 [Nt, 3]
    env: np.ndarray            # f32 [H, W, 3] lat-long, row 0 = zenith (+Y)
    n_views: int
    height: int
    width: int
    pos: np.ndarray            # f32 [3, N]
    nrm: np.ndarray            # f32 [3, N]
    kd: np.ndarray             # f32 [3, N]
    korm: np.ndarray           # f32 [3, N] (occlusion, roughness, metallic)
    mask: np.ndarray           # u8  [N]
    eye: np.ndarray            # f32 [V, 3]
    spp: int
    seed: int = 0
    tau: float = 1.0
    ray_eps: float = 1e-3
    view_base: int = 0
    meta: dict = field(default_factory=dict)
    depth: np.ndarray = None   # f32 [N] primary-ray hit distance (0 where mask is 0)

    @property
    def n_pixels(self):
        return self.n_views * self.height * self.width

    @property
    def n_valid(self):
        return int(self.mask.sum())


# ----------------------------------------------------------------------------
# environment maps and textures
# ----------------------------------------------------------------------------

def lognormal_env(rng, H, W, sigma):
    return rng.lognormal(0.0, sigma, size=(H, W, 3)).astype(np.float32)


def smooth_noise_texture(rng, size=1024, waves=12):
    """RGBA8 texture: per channel a normalised sum of low-frequency cosines,
    periodic in u (columns)."""
    u = (np.arange(size) + 0.5) / size
    U, V = np.meshgrid(u, u)
    out = np.empty((size, size, 4), np.uint8)
    for ch in range(4):
        acc = np.zeros((size, size))
        for _ in range(waves):
            kx = rng.integers(-6, 7)
            ky = rng.integers(0, 7)
            a = rng.uniform(0.2, 1.0)
            ph = rng.uniform(0, 2 * np.pi)
            acc += a * np.cos(2 * np.pi * (kx * U + ky * V) + ph)
        acc = (acc - acc.min()) / max(acc.max() - acc.min(), 1e-12)
        out[..., ch] = np.clip(np.round(acc * 255.0), 0, 255).astype(np.uint8)
    return out


def spherical_lookup(tex, pts):
    """Nearest texel of an RGBA8 texture at the spherical (u, v) of a point
    seen from the origin."""
    d = pts / np.maximum(np.linalg.norm(pts, axis=-1, keepdims=True), 1e-30)
    u = np.mod(np.arctan2(d[:, 2], d[:, 0]) / (2 * np.pi), 1.0)
    v = np.arccos(np.clip(d[:, 1], -1, 1)) / np.pi
    S = tex.shape[0]
    iu = np.minimum((u * S).astype(np.int64), S - 1)
    iv = np.minimum((v * S).astype(np.int64), S - 1)
    return tex[iv, iu].astype(np.float64) / 255.0


def _planar(a, n):
    return np.ascontiguousarray(np.asarray(a, np.float64).reshape(n, 3).T, dtype=np.float32)


def _scene_eps(verts):
    lo, hi = verts.min(0), verts.max(0)
    return float(1e-4 * np.linalg.norm(hi.astype(np.float64) - lo))


def _assemble(name, verts, tris, env, eyes, H, W, hits_per_view, materials, spp, meta):
    V = len(eyes)
    N = V * H * W
    pos = np.zeros((N, 3))
    nrm = np.zeros((N, 3))
    mask = np.zeros(N, np.uint8)
    depth = np.zeros(N)
    for v, (p, n, m) in enumerate(hits_per_view):
        sl = slice(v * H * W, (v + 1) * H * W)
        pos[sl] = p
        nrm[sl] = n
        mask[sl] = m
        depth[sl] = np.where(m > 0, np.linalg.norm(p - np.asarray(eyes[v], np.float64), axis=-1), 0.0)
    kd, korm = materials(pos, mask)
    kd[mask == 0] = 0
    korm[mask == 0] = 0
    verts32, tris32 = meshes.to_device_layout(verts, tris)
    return Workload(
        name=name, verts=verts32, tris=tris32, env=env, n_views=V, height=H, width=W,
        pos=_planar(pos, N), nrm=_planar(nrm, N), kd=_planar(kd, N), korm=_planar(korm, N),
        mask=mask, eye=np.ascontiguousarray(np.asarray(eyes), dtype=np.float32), spp=spp,
        ray_eps=_scene_eps(verts32), meta=meta, depth=depth.astype(np.float32))


def _cast(eye, target, fov, H, W, surfaces):
    d = look_at_rays(eye, target, fov, H, W)
    o = np.broadcast_to(np.asarray(eye, np.float64), d.shape).copy()
    hits = Hits(len(d))
    for k, fn in enumerate(surfaces):
        t, n = fn(o, d)
        hits.take(t, n, k)
    m = np.isfinite(hits.t)
    p = o + d * np.where(m, hits.t, 0.0)[:, None]
    n = hits.nrm
    # shading normals face the camera side they were hit from
    flip = (n * d).sum(-1) > 0
    n[flip] *= -1
    p[~m] = 0
    n[~m] = 0
    return p, n, m.astype(np.uint8)


# ----------------------------------------------------------------------------
# tiny: icosphere over a ground quad
# ----------------------------------------------------------------------------

def make_tiny(k=0, H=64, W=64, spp=4):
    rng = np.random.Generator(np.random.PCG64(1000 + k))
    sv, sf = meshes.icosphere(2)                       # 320 triangles, radius 1
    gv, gf = meshes.quad([-5, -1, -5], [-5, -1, 5], [5, -1, 5], [5, -1, -5])
    verts, tris = meshes.merge([(sv, sf), (gv, gf)])
    Henv, Wenv = 32, 64
    env = rng.lognormal(0.0, 1.0, size=(Henv, Wenv, 3)).astype(np.float32)
    env[8:12, 40:44] *= 50.0
    eye = np.array([0.0, 0.5, 4.0])
    surfaces = [lambda o, d: hit_sphere(o, d, np.zeros(3), 1.0),
                lambda o, d: hit_rect_y(o, d, -1.0, -5, 5, -5, 5, up=True)]
    hv = [_cast(eye, [0.0, -0.2, 0.0], 40.0, H, W, surfaces)]
    N = H * W

    def materials(pos, mask):
        kd = rng.uniform(0.0, 1.0, size=(N, 3))
        r = rng.uniform(0.08, 1.0, size=N)
        m = rng.uniform(0.0, 1.0, size=N)
        korm = np.stack([np.ones(N), r, m], axis=1)
        return kd, korm

    return _assemble("tiny", verts, tris, env, [eye], H, W, hv, materials, spp,
                     {"tris": len(tris), "env": (Henv, Wenv)})


# ----------------------------------------------------------------------------
# sphere8: displaced sphere + 20 boxes, 8 views
# ----------------------------------------------------------------------------

def sphere_scene(k, freq=71, n_boxes=20, env_hw=(256, 512), env_sigma=1.5):
    rng = np.random.Generator(np.random.PCG64(1000 + k))
    ds = DisplacedSphere(rng, amp=0.05, n_waves=8)
    sv, sf = ds.mesh(freq)
    boxes = []
    parts = [(sv, sf)]
    for _ in range(n_boxes):
        half = rng.uniform(0.1, 0.4, 3) / 2.0
        yaw = rng.uniform(0, 2 * np.pi)
        az = rng.uniform(0, 2 * np.pi)
        rad = rng.uniform(1.3, 2.5)
        c = np.array([rad * np.cos(az), rng.uniform(-0.6, 0.6), rad * np.sin(az)])
        boxes.append((c, half, yaw))
        parts.append(meshes.box(c, half, yaw))
    verts, tris = meshes.merge(parts)
    Henv, Wenv = env_hw
    env = rng.lognormal(0.0, env_sigma, size=(Henv, Wenv, 3)).astype(np.float32)
    r0 = int(round(0.25 * Henv)) - 2          # theta ~ 45 degrees
    c0 = int(0.2 * Wenv)
    env[r0:r0 + 4, c0:c0 + 4] *= 1000.0
    tex_kd = smooth_noise_texture(rng)
    tex_orm = smooth_noise_texture(rng)
    return rng, ds, boxes, verts, tris, env, tex_kd, tex_orm


def make_sphere8(k=1, H=512, W=512, spp=8, n_views=8, freq=71, views=None, env_hw=(256, 512), scene=None):
    """scene: a sphere_scene(...) tuple to reuse (same mesh and probe)."""
    if scene is None:
        scene = sphere_scene(k, freq=freq, env_hw=env_hw)
    rng, ds, boxes, verts, tris, env, tex_kd, tex_orm = scene
    surfaces = [ds.intersect] + [
        (lambda c, h, y: (lambda o, d: hit_box(o, d, c, h, y)))(c, h, y) for (c, h, y) in boxes]
    eyes = []
    view_ids = range(n_views) if views is None else views
    for v in view_ids:
        az = np.radians(45.0 * v)
        el = np.radians(15.0 if v % 2 == 0 else 35.0)
        eyes.append(4.0 * np.array([np.cos(el) * np.cos(az), np.sin(el), np.cos(el) * np.sin(az)]))
    # views are independent: cast them on threads (numpy releases the GIL)
    with ThreadPoolExecutor(max(1, min(len(eyes), os.cpu_count() or 1))) as ex:
        hv = list(ex.map(lambda e: _cast(e, [0, 0, 0], 40.0, H, W, surfaces), eyes))

    def materials(pos, mask):
        a = spherical_lookup(tex_kd, pos)
        b = spherical_lookup(tex_orm, pos)
        kd = a[:, :3]
        korm = np.stack([b[:, 0], 0.08 + 0.92 * b[:, 1], b[:, 2]], axis=1)
        return kd, korm

    return _assemble("sphere8", verts, tris, env, eyes, H, W, hv, materials, spp,
                     {"tris": len(tris), "env": env.shape[:2], "freq": freq})


def make_workload(name, **kw):
    if name == "tiny":
        return make_tiny(**kw)
    if name == "sphere8":
        return make_sphere8(**kw)
    if name == "sphere8_grad":
        kw.setdefault("spp", 12)
        w = make_sphere8(k=2 if kw.pop("own_seed", False) else 1, **kw)
        w.name = "sphere8_grad"
        return w
    if name == "lattice":
        from .lattice import make_lattice
        return make_lattice(**kw)
    raise KeyError(name)


CONFIGS = ("tiny", "sphere8", "sphere8_grad", "lattice")


def upstream_grads(w, seed=7):
    """Upstream gradients shaped like an L1 image loss on c = kd*c_d + c_s:
    dL/dc_d = kd * s / n_valid and dL/dc_s = s / n_valid with s = +-1 per
    pixel and channel (seeded), zero on invalid pixels."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.choice(np.array([-1.0, 1.0]), size=(3, w.n_pixels))
    s = s * w.mask[None, :]
    nv = max(w.n_valid, 1)
    gcs = (s / nv).astype(np.float32)
    gcd = (w.kd.astype(np.float64) * s / nv).astype(np.float32)
    return np.ascontiguousarray(gcd), np.ascontiguousarray(gcs)


def noisy_lighting(w, seed=0, channels=6):
    """Seeded stand-in for Monte Carlo lighting estimates, f32 [channels][N]:
    a smooth positive field times heavy-tailed per-pixel noise (lognormal,
    sigma 1), with occasional fireflies; 0 where mask is 0."""
    rng = np.random.Generator(np.random.PCG64(5000 + seed))
    N = w.n_pixels
    pos = w.pos.astype(np.float64)
    base = 0.5 + 0.4 * np.sin(3.0 * pos[0] + 1.0)[None] * np.cos(2.0 * pos[2])[None] + 0.2 * np.arange(channels)[:, None] / channels
    noise = rng.lognormal(0.0, 1.0, size=(channels, N))
    fire = rng.random((channels, N)) < 1e-3
    x = base * noise * np.where(fire, 50.0, 1.0)
    return np.ascontiguousarray(np.where(w.mask[None] > 0, x, 0.0), dtype=np.float32)


def from_arrays(name, verts, tris, env, pos, nrm, kd, korm, mask=None, eye=None,
                n_views=1, height=None, width=None, spp=4, ray_eps=1e-4, tau=1.0, seed=0):
    """Workload from explicit per-pixel arrays given as [N, 3] (converted to
    the planar [3, N] layout)."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    N = len(pos)
    if height is None:
        height, width = 1, N // n_views
    mask = np.ones(N, np.uint8) if mask is None else np.asarray(mask, np.uint8)
    eye = np.zeros((n_views, 3)) if eye is None else np.asarray(eye, np.float64).reshape(n_views, 3)
    verts = np.asarray(verts, np.float32).reshape(-1, 3)
    tris = np.asarray(tris, np.int32).reshape(-1, 3)
    return Workload(name=name, verts=verts, tris=tris, env=np.ascontiguousarray(env, np.float32),
                    n_views=n_views, height=height, width=width,
                    pos=_planar(pos, N), nrm=_planar(nrm, N), kd=_planar(kd, N),
                    korm=_planar(korm, N), mask=mask, eye=np.ascontiguousarray(eye, np.float32),
                    spp=spp, seed=seed, tau=tau, ray_eps=ray_eps)

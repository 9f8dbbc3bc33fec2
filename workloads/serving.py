"""Serving mix: resident scenes and pre-generated G-buffers per scene and
resolution; requests drawn with a seeded PCG64(5).

Full mix (the one the serving benchmark uses):
  A  displaced sphere, geodesic frequency 50 (~50k triangles) + 20 boxes,
     probe 512x256
  B  displaced sphere, frequency 122 (~298k triangles) + 20 boxes, probe 1024x512
  C  the lattice room (~1.0M triangles), probe 2048x1024
  resolution uniform in {128^2, 256^2, 512^2, 1024^2}, spp uniform in
  {4, 8, 16, 32}, forward-only or forward+backward 50/50.
"""

import numpy as np

from .configs import make_sphere8, sphere_scene, upstream_grads
from .lattice import make_lattice

RES = (128, 256, 512, 1024)
SPPS = (4, 8, 16, 32)


def make_scenes(full=True, res=RES):
    """{name: {'verts', 'tris', 'env', 'views': {res: Workload}}}"""
    out = {}
    specs = ([("A", 10, 50, (256, 512)), ("B", 11, 122, (512, 1024))] if full
             else [("A", 10, 30, (256, 512))])
    for name, k, freq, env_hw in specs:
        sc = sphere_scene(k, freq=freq, env_hw=env_hw)
        out[name] = {r: make_sphere8(k=k, H=r, W=r, n_views=1, spp=4, views=[r % 8], scene=sc) for r in res}
    if full:
        views = {}
        for vi, r in enumerate(res):
            views[r] = make_lattice(k=12, H=r, W=r, n_views=1, spp=4, views=[vi])
        out["C"] = views
    return out


def make_requests(scenes, n, seed=5, res=RES, spps=SPPS):
    """A list of (scene, res, spp, grad, view_base) draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    names = sorted(scenes)
    reqs = []
    for i in range(n):
        reqs.append((names[rng.integers(len(names))], int(res[rng.integers(len(res))]),
                     int(spps[rng.integers(len(spps))]), bool(rng.random() < 0.5), 1000 + i))
    return reqs


def poisson_arrivals(n, rate, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def request_grads(w, seed):
    return upstream_grads(w, seed=seed)

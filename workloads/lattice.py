"""Heavy-occlusion workload: a 32^3-cell lattice of thin beams (each kept
cell edge is an axis-aligned box 0.008 wide, 12 triangles) inside a closed
room [-1.5, 1.5]^3 with one 1.0 x 0.6 window in each side wall; cameras
inside the room.  ~1.0M triangles at 32 cells per axis.

The G-buffer is cast analytically: a 3D DDA walks the lattice cells and
intersects the beams of each cell's 12 edges; the room walls are planes with
rectangular holes.  Closest hit only (primary visibility).
"""

import os

import numpy as np

from . import meshes
from .configs import Workload, smooth_noise_texture, spherical_lookup, _planar, _scene_eps
from .raycast import look_at_rays

ROOM = 1.5
WIN_W, WIN_H = 1.0, 0.6


def lattice_beams(rng, cells=32, keep=0.8):
    n1 = cells + 1
    kx = rng.random((cells, n1, n1)) < keep   # beams along x: [i, j, k] segment i, y_j, z_k
    ky = rng.random((n1, cells, n1)) < keep
    kz = rng.random((n1, n1, cells)) < keep
    return kx, ky, kz


def beam_mesh(kx, ky, kz, cells, half):
    g = np.linspace(-1.0, 1.0, cells + 1)
    boxes = []
    for axis, keep in enumerate((kx, ky, kz)):
        idx = np.argwhere(keep)
        lo = np.empty((len(idx), 3))
        hi = np.empty((len(idx), 3))
        for a in range(3):
            if a == axis:
                lo[:, a] = g[idx[:, a]]
                hi[:, a] = g[idx[:, a] + 1]
            else:
                lo[:, a] = g[idx[:, a]] - half
                hi[:, a] = g[idx[:, a]] + half
        boxes.append((lo, hi))
    lo = np.concatenate([b[0] for b in boxes])
    hi = np.concatenate([b[1] for b in boxes])
    # 8 corners per box, 12 triangles (same winding as meshes.box)
    corners = np.stack([np.where([sx, sy, sz], hi, lo) for sx in (0, 1) for sy in (0, 1) for sz in (0, 1)], 1)
    f0 = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
                   [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]])
    base = (np.arange(len(lo)) * 8)[:, None, None]
    faces = (f0[None] + base).reshape(-1, 3)
    return corners.reshape(-1, 3), faces


def room_mesh():
    parts = [meshes.quad([-ROOM, -ROOM, -ROOM], [ROOM, -ROOM, -ROOM], [ROOM, -ROOM, ROOM], [-ROOM, -ROOM, ROOM]),
             meshes.quad([-ROOM, ROOM, -ROOM], [-ROOM, ROOM, ROOM], [ROOM, ROOM, ROOM], [ROOM, ROOM, -ROOM])]
    for axis in (0, 2):
        for sign in (-1, 1):
            parts.append(meshes.wall_with_window(axis, sign, ROOM, WIN_W, WIN_H))
    return meshes.merge(parts)


def _slab(o, inv, lo, hi):
    t0 = (lo - o) * inv
    t1 = (hi - o) * inv
    tn = np.minimum(t0, t1).max(-1)
    tf = np.maximum(t0, t1).min(-1)
    return tn, tf


def cast_lattice(o, d, kx, ky, kz, cells, half):
    """Closest beam hit along each ray (inf if none): returns t, normal."""
    n = len(d)
    c = 2.0 / cells
    with np.errstate(divide="ignore"):
        inv = 1.0 / np.where(d == 0, 1e-30, d)
    tn, tf = _slab(o, inv, np.full(3, -1.0 - half), np.full(3, 1.0 + half))
    t_hit = np.full(n, np.inf)
    nrm = np.zeros((n, 3))
    alive = (tn <= tf) & (tf > 0)
    t_cur = np.maximum(tn, 0.0)
    idx = np.nonzero(alive)[0]
    t_cur = t_cur[idx]
    t_end = tf[idx]
    for _ in range(4 * cells + 8):
        if len(idx) == 0:
            break
        oo, dd, ii = o[idx], d[idx], inv[idx]
        p = oo + dd * (t_cur + 1e-9)[:, None]
        cell = np.clip(np.floor((p + 1.0) / c).astype(np.int64), 0, cells - 1)
        clo = -1.0 + cell * c
        chi = clo + c
        # exit of the current cell (unexpanded)
        _, t_out = _slab(oo, ii, clo, chi)
        best = np.full(len(idx), np.inf)
        bn = np.zeros((len(idx), 3))
        i, j, k = cell[:, 0], cell[:, 1], cell[:, 2]
        # 12 edges: 4 along each axis
        for axis, keep in enumerate((kx, ky, kz)):
            for da in (0, 1):
                for db in (0, 1):
                    if axis == 0:
                        e = keep[i, j + da, k + db]
                        lo = np.stack([clo[:, 0], clo[:, 1] + da * c - half, clo[:, 2] + db * c - half], 1)
                        hi = np.stack([chi[:, 0], clo[:, 1] + da * c + half, clo[:, 2] + db * c + half], 1)
                    elif axis == 1:
                        e = keep[i + da, j, k + db]
                        lo = np.stack([clo[:, 0] + da * c - half, clo[:, 1], clo[:, 2] + db * c - half], 1)
                        hi = np.stack([clo[:, 0] + da * c + half, chi[:, 1], clo[:, 2] + db * c + half], 1)
                    else:
                        e = keep[i + da, j + db, k]
                        lo = np.stack([clo[:, 0] + da * c - half, clo[:, 1] + db * c - half, clo[:, 2]], 1)
                        hi = np.stack([clo[:, 0] + da * c + half, clo[:, 1] + db * c + half, chi[:, 2]], 1)
                    t0 = (lo - oo) * ii
                    t1 = (hi - oo) * ii
                    tmin = np.minimum(t0, t1)
                    bn_t = tmin.max(-1)
                    bf_t = np.maximum(t0, t1).min(-1)
                    ok = e & (bn_t <= bf_t) & (bn_t > 1e-9)
                    better = ok & (bn_t < best)
                    if better.any():
                        best = np.where(better, bn_t, best)
                        ax = tmin.argmax(-1)
                        nn = np.zeros((len(idx), 3))
                        nn[np.arange(len(idx)), ax] = -np.sign(dd[np.arange(len(idx)), ax])
                        bn = np.where(better[:, None], nn, bn)
        # accept hits inside this cell's parameter range (the beams of other
        # cells are found when the walk reaches them)
        got = best <= t_out + 1e-9
        t_hit[idx[got]] = best[got]
        nrm[idx[got]] = bn[got]
        t_next = t_out + 1e-7
        cont = ~got & (t_next < t_end)
        idx, t_cur, t_end = idx[cont], t_next[cont], t_end[cont]
    return t_hit, nrm


def cast_room(o, d):
    """Inside of the room: floor, roof, four walls with a window each."""
    n = len(d)
    t_best = np.full(n, np.inf)
    nrm = np.zeros((n, 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        for axis in range(3):
            for sign in (-1, 1):
                t = (sign * ROOM - o[:, axis]) / d[:, axis]
                p = o + d * np.nan_to_num(t, posinf=0, neginf=0)[:, None]
                ok = (t > 1e-9)
                others = [a for a in range(3) if a != axis]
                for a in others:
                    ok &= np.abs(p[:, a]) <= ROOM
                if axis != 1:
                    s = p[:, 2] if axis == 0 else p[:, 0]
                    in_win = (np.abs(s) <= WIN_W / 2) & (np.abs(p[:, 1]) <= WIN_H / 2)
                    ok &= ~in_win
                better = ok & (t < t_best)
                t_best = np.where(better, t, t_best)
                nn = np.zeros(3)
                nn[axis] = -sign
                nrm[better] = nn
    return t_best, nrm


def _cast_chunk(args):
    o, d, kx, ky, kz, cells, half = args
    t1, n1 = cast_lattice(o, d, kx, ky, kz, cells, half)
    t2, n2 = cast_room(o, d)
    return t1, n1, t2, n2


def _worker_main():
    """Worker process: read one chunk's arguments (pickled by the parent, this
    package's own arrays) from stdin, write its hits to stdout."""
    import pickle
    import sys
    args = pickle.load(sys.stdin.buffer)
    pickle.dump(_cast_chunk(args), sys.stdout.buffer, protocol=pickle.HIGHEST_PROTOCOL)
    sys.stdout.buffer.flush()


def cast_scene(o, d, kx, ky, kz, cells, half, workers=None):
    """Closest hits against the beams and the room of every ray, in parallel
    chunks of rays (every ray's result depends only on that ray, so the
    chunking does not change it): (t_beams, n_beams, t_room, n_room).  The
    chunks run in fresh worker processes that import only this package (the
    calling program is not re-imported, and no process is forked from one that
    may hold a GPU context)."""
    import pickle
    import subprocess
    import sys
    n = len(d)
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or n < 65536:
        return _cast_chunk((o, d, kx, ky, kz, cells, half))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    env["PYTHONPATH"] = root + (os.pathsep + env["PYTHONPATH"] if env.get("PYTHONPATH") else "")
    parts = np.array_split(np.arange(n), workers)
    procs = []
    for p in parts:
        pr = subprocess.Popen([sys.executable, "-c", "from workloads.lattice import _worker_main; _worker_main()"],
                              stdin=subprocess.PIPE, stdout=subprocess.PIPE, env=env, cwd=root)
        pickle.dump((o[p], d[p], kx, ky, kz, cells, half), pr.stdin, protocol=pickle.HIGHEST_PROTOCOL)
        pr.stdin.close()
        procs.append(pr)
    res = []
    for pr in procs:
        out = pickle.load(pr.stdout)
        pr.stdout.close()
        if pr.wait() != 0:
            raise RuntimeError("lattice casting worker failed")
        res.append(out)
    return tuple(np.concatenate([r[k] for r in res]) for k in range(4))


def make_lattice(k=3, H=1024, W=1024, spp=32, n_views=4, cells=32, env_hw=(1024, 2048), views=None):
    rng = np.random.Generator(np.random.PCG64(1000 + k))
    half = 0.004
    kx, ky, kz = lattice_beams(rng, cells)
    bv, bf = beam_mesh(kx, ky, kz, cells, half)
    rv, rf = room_mesh()
    verts, tris = meshes.merge([(bv, bf), (rv, rf)])
    Henv, Wenv = env_hw
    env = rng.lognormal(0.0, 1.0, size=(Henv, Wenv, 3)).astype(np.float32)
    s = max(1, Henv // 128)          # 8x8 sources at 2048x1024
    for (th, ph) in ((np.radians(86), 0.0), (np.radians(84), np.pi), (np.radians(8), 1.0)):
        i = int(th / np.pi * Henv)
        j = int(ph / (2 * np.pi) * Wenv)
        env[max(0, i - s // 2):i + s - s // 2, j:j + s] *= 1000.0
    tex_kd = smooth_noise_texture(rng)
    tex_orm = smooth_noise_texture(rng)
    eyes_all = [np.array([sx * 1.3, 0.5, sz * 1.3]) for sx, sz in ((1, 1), (-1, 1), (-1, -1), (1, -1))]
    view_ids = range(n_views) if views is None else views
    eyes = [eyes_all[v % 4] for v in view_ids]
    V = len(eyes)
    N = V * H * W
    pos = np.zeros((N, 3))
    nrm = np.zeros((N, 3))
    mask = np.zeros(N, np.uint8)
    depth = np.zeros(N)
    d_all = np.concatenate([look_at_rays(eye, [0, 0, 0], 60.0, H, W) for eye in eyes])
    o_all = np.concatenate([np.broadcast_to(eye, (H * W, 3)) for eye in eyes]).astype(np.float64)
    hits = cast_scene(o_all, d_all, kx, ky, kz, cells, half)
    for vi, eye in enumerate(eyes):
        sl = slice(vi * H * W, (vi + 1) * H * W)
        d, o = d_all[sl], o_all[sl]
        t1, n1, t2, n2 = (h[sl] for h in hits)
        use1 = t1 <= t2
        t = np.where(use1, t1, t2)
        n_ = np.where(use1[:, None], n1, n2)
        m = np.isfinite(t)
        p = o + d * np.where(m, t, 0)[:, None]
        flip = (n_ * d).sum(-1) > 0
        n_[flip] *= -1
        sl = slice(vi * H * W, (vi + 1) * H * W)
        pos[sl] = np.where(m[:, None], p, 0)
        nrm[sl] = np.where(m[:, None], n_, 0)
        mask[sl] = m
        depth[sl] = np.where(m, t, 0.0)
    a = spherical_lookup(tex_kd, pos)
    b = spherical_lookup(tex_orm, pos)
    kd = a[:, :3]
    korm = np.stack([b[:, 0], 0.08 + 0.92 * b[:, 1], b[:, 2]], axis=1)
    kd[mask == 0] = 0
    korm[mask == 0] = 0
    verts32, tris32 = meshes.to_device_layout(verts, tris)
    return Workload(name="lattice", verts=verts32, tris=tris32, env=env, n_views=V, height=H, width=W,
                    pos=_planar(pos, N), nrm=_planar(nrm, N), kd=_planar(kd, N), korm=_planar(korm, N),
                    mask=mask, eye=np.ascontiguousarray(np.asarray(eyes), dtype=np.float32), spp=spp,
                    ray_eps=_scene_eps(verts32), meta={"tris": len(tris), "env": env.shape[:2]},
                    depth=depth.astype(np.float32))

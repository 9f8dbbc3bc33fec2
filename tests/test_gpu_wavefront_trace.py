"""The shading path's shadow-ray traversal (the 4-wide hierarchy walked by a
workgroup's ray queue, pending references in LDS, a binary walk from the root
when a lane's stack is full) against brute force on the same rays.

The forward pass dumps every sample's FP32 world direction and whether its
shadow ray was traced and hit; the origins are recomputed on the host as the
kernel forms them (the FP32 position plus ray_eps times the FP64-normalised
normal, rounded once).  Each traced ray is then tested against every
triangle by the any-hit query: the two answers must agree bit for bit.
Scenes: the lattice (dense occluders, most rays hit) and a bundle of long thin
triangles through a cube (nearly every box overlaps every ray and nearly
every ray misses, so the walk visits most of the hierarchy and the pending
references outgrow the LDS stack).
"""

import numpy as np
import pytest

from workloads import make_workload
from tests.parity_util import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _flags():
    import oracle
    return oracle.DEC_L_TRACED, oracle.DEC_L_HIT, oracle.DEC_B_TRACED, oracle.DEC_B_HIT


def _origins(pos, nrm, eps):
    n = nrm.astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):   # zero normals of uncovered pixels
        n = n / np.linalg.norm(n, axis=0)
    return (pos.astype(np.float64) + float(np.float32(eps)) * n).astype(np.float32)


def _check(M, scene, env, gb, pos, nrm, spp, eps, seed=5):
    c_d, c_s, hb, dec = M.shade_fwd(scene, env, gb, spp, seed=seed, tau=1.0, ray_eps=eps, decisions="dirs")
    torch.cuda.synchronize()
    d = to_np(dec).view(np.uint32)
    rec2 = d[..., 2]
    dirs = np.ascontiguousarray(d[..., 3:]).view(np.float32).reshape(d.shape[0], d.shape[1], 2, 3)
    lt, lh, bt, bh = _flags()
    org = _origins(pos, nrm, eps).T                      # [N, 3]
    o_all, d_all, h_all = [], [], []
    for t, (tr, hi) in enumerate(((lt, lh), (bt, bh))):
        sel = (rec2 & tr) != 0
        pix, smp = np.nonzero(sel)
        o_all.append(org[pix])
        d_all.append(dirs[pix, smp, t])
        h_all.append((rec2[pix, smp] & hi) != 0)
    o = np.concatenate(o_all)
    dd = np.concatenate(d_all)
    h = np.concatenate(h_all)
    assert len(o) > 1000
    ot = torch.from_numpy(np.ascontiguousarray(o.T)).cuda()
    dt = torch.from_numpy(np.ascontiguousarray(dd.T)).cuda()
    brute = to_np(M.trace_anyhit(scene, ot, dt, brute=True)).astype(bool)
    wide = to_np(M.trace_anyhit(scene, ot, dt, mode="wide")).astype(bool)
    assert np.array_equal(wide, brute)
    mism = int((h != brute).sum())
    print("traced rays %d, hit fraction %.3f, mismatches %d" % (len(h), h.mean(), mism))
    assert mism == 0
    return h.mean()


def test_wavefront_traversal_lattice():
    _need_gpu()
    import paper_2206_03380_amd as M
    w = make_workload("lattice", H=96, W=96, n_views=2)
    scene = M.Scene(torch.from_numpy(w.verts).cuda(), torch.from_numpy(w.tris).cuda())
    env = M.Env(torch.from_numpy(w.env).cuda())
    gb = M.GBuffer.from_workload(w, "cuda")
    info = scene.info()
    assert info["wide"] == 1 and info["depth_complexity"] >= 4, info
    frac = _check(M, scene, env, gb, w.pos, w.nrm, 4, w.ray_eps)
    assert frac > 0.5


def test_wavefront_traversal_stack_overflow():
    """Thin triangles spanning a cube: every box overlaps nearly every ray."""
    _need_gpu()
    import paper_2206_03380_amd as M
    r = np.random.Generator(np.random.PCG64(77))
    nt = 12000
    a = r.uniform(-1, 1, (nt, 3))
    u = r.normal(size=(nt, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    b = a - 2.5 * u
    c = a + 2.5 * u + 1e-4 * r.normal(size=(nt, 3))
    v = np.stack([b, c, a + 1e-4 * r.normal(size=(nt, 3))], 1).reshape(-1, 3).astype(np.float32)
    f = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
    scene = M.Scene(torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda())
    info = scene.info()
    assert info["n_groups"] >= 1 and info["wide"] == 1, info
    H = W = 48
    n = H * W
    pos = r.uniform(-0.8, 0.8, (3, n)).astype(np.float32)
    nrm = r.normal(size=(3, n)).astype(np.float32)
    kd = np.full((3, n), 0.5, np.float32)
    korm = np.stack([np.ones(n), r.uniform(0.2, 0.9, n), r.uniform(0, 1, n)]).astype(np.float32)
    mask = np.ones(n, np.uint8)
    eye = np.array([[0.0, 0.0, 6.0]], np.float32)
    env_np = (0.2 + r.uniform(0, 1, (32, 64, 3))).astype(np.float32)
    env = M.Env(torch.from_numpy(env_np).cuda())
    cu = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    gb = M.GBuffer(cu(pos), cu(nrm), cu(kd), cu(korm), cu(mask), cu(eye), 1, H, W, 0)
    frac = _check(M, scene, env, gb, pos, nrm, 2, 1e-3)
    assert frac < 0.5


def test_wavefront_traversal_surface_scene_walks_binary():
    """A surface scene (the displaced sphere) has a depth complexity of a few:
    its shadow rays take the binary walk, with the same answers."""
    _need_gpu()
    import paper_2206_03380_amd as M
    w = make_workload("sphere8", H=64, W=64, n_views=2)
    scene = M.Scene(torch.from_numpy(w.verts).cuda(), torch.from_numpy(w.tris).cuda())
    info = scene.info()
    assert info["wide"] == 0 and 1 <= info["depth_complexity"] < 4, info
    env = M.Env(torch.from_numpy(w.env).cuda())
    gb = M.GBuffer.from_workload(w, "cuda")
    _check(M, scene, env, gb, w.pos, w.nrm, 4, w.ray_eps)

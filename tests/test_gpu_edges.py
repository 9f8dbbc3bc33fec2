"""HIP edge-sampled visibility gradient and edge list vs the oracle, through
the C ABI.

Edge list: integer work, compared bit for bit.  Gradient: both sides draw
the same edge samples (Philox block 2); the kernel sums FP32 terms with
float atomics, the oracle FP64 terms in order.  Per vertex component the
bound is REL times the sum of |term| (FP32 roundoff of the terms and of their
summation), plus COND times the oracle's FP32 condition bound of the terms,
plus the oracle's bound on the terms of samples whose discrete steps it
finds undecided (silhouette sign, horizon, nearest texel, out-side ray).
The median relative error over elements well above the noise, after each
element's allowance for undecided samples, must also stay small, so that a
bound widened for a few elements cannot hide a systematic error.
"""

import numpy as np
import pytest

import oracle
from workloads import make_workload, upstream_grads, from_arrays, meshes
from tests.parity_util import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-4
COND = 4.0


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_flags(f):
    import paper_2206_03380_amd as M
    return oracle.BILINEAR if f & M.FLAG_BILINEAR else 0


# ---------------------------------------------------------------------------
# edge list
# ---------------------------------------------------------------------------

def _mesh(name):
    if name == "icosphere":
        v, f = meshes.icosphere(3)
        return v.astype(np.float32), f.astype(np.int32)
    if name == "tiny":
        w = make_workload("tiny")
        return w.verts, w.tris
    if name == "sphere8":
        from workloads.configs import sphere_scene
        s = sphere_scene(1)
        return s[3].astype(np.float32), s[4].astype(np.int32)
    if name == "soup":
        r = np.random.Generator(np.random.PCG64(11))
        t = r.integers(0, 40, size=(3000, 3)).astype(np.int32)   # many repeated and non-manifold edges
        t[::97, 1] = 45                                            # corners out of range
        t[::89, 2] = -3
        return r.normal(size=(40, 3)).astype(np.float32), t
    if name == "empty":
        return np.zeros((4, 3), np.float32), np.zeros((0, 3), np.int32)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["icosphere", "tiny", "sphere8", "soup", "empty"])
def test_edge_list_bit_exact(name):
    _need_gpu()
    import paper_2206_03380_amd as M
    v, t = _mesh(name)
    print("edge list", name, len(v), len(t), flush=True)
    ed = M.Edges(torch.from_numpy(t).cuda(), len(v))
    rows = to_np(ed.rows())
    ref = oracle.mesh_edges(t, len(v))
    assert rows.shape == ref.shape, (rows.shape, ref.shape)
    assert (rows == ref).all()


# ---------------------------------------------------------------------------
# gradient parity
# ---------------------------------------------------------------------------

def _run_gpu(w, n_es, flags=0, seed=None, tau=None, g_init=None, gain=1):
    import paper_2206_03380_amd as M
    dev = "cuda"
    verts = torch.from_numpy(w.verts).to(dev)
    tris = torch.from_numpy(w.tris).to(dev)
    scene = M.Scene(verts, tris)
    env = M.Env(torch.from_numpy(w.env).to(dev))
    gb = M.GBuffer.from_workload(w, dev)
    ed = M.Edges(tris, len(w.verts))
    ud, us = upstream_grads(w)
    gv = None if g_init is None else torch.from_numpy(g_init).to(dev)
    stats = M.new_stats(dev)
    g = M.shade_bwd_edges(scene, env, ed, verts, gb, n_es, torch.from_numpy(ud).to(dev),
                          torch.from_numpy(us).to(dev), seed=w.seed if seed is None else seed,
                          tau=w.tau if tau is None else tau, ray_eps=w.ray_eps, flags=flags, g_verts=gv,
                          stats=stats, sharp_gain=gain)
    torch.cuda.synchronize()
    return to_np(g).astype(np.float64), M.read_stats(stats), (ud, us)


def _parity(w, n_es, flags=0, pixels=None, med=2e-5, seed=None, gain=1):
    print("edge parity", w.name, w.n_pixels, "px", len(w.tris), "tris, n_es", n_es, "flags", flags, "gain", gain,
          flush=True)
    g, st, (ud, us) = _run_gpu(w, n_es, flags=flags, seed=seed, gain=gain)
    E = oracle.mesh_edges(w.tris, len(w.verts))
    pix = np.nonzero(w.mask)[0] if pixels is None else np.asarray(pixels)
    o = oracle.edge_grad(w, E, n_es, ud[:, pix].astype(np.float64), us[:, pix].astype(np.float64), pixels=pix,
                         seed=w.seed if seed is None else seed, flags=_oracle_flags(flags), sharp_gain=gain)
    ref = o["g_verts"]
    scale = np.abs(ref).max() + 1e-30
    bound = REL * o["abs"] + COND * o["cond"] + o["flag"] + 1e-7 * scale
    err = np.abs(g - ref)
    big = np.abs(ref) > 1e-2 * np.abs(ref).mean() + 1e-30
    # systematic-error guard: the error left after each element's allowance
    # for samples with an undecided step, relative to the element
    resid = np.maximum(err - o["flag"], 0.0)
    med_rel = float(np.median(resid[big] / np.abs(ref[big]))) if big.any() else 0.0
    print("  samples %d, silhouettes %d, traced %d (gpu %d), blocked %d (gpu %d), flagged %d; "
          "max|err| %.3g of scale %.3g, worst/bound %.3g, median rel %.3g, nonzero %d/%d" % (
              o["samples"], o["silhouettes"], o["traced"], st["rays_traced"], o["blocked"], st["rays_hit"],
              o["flagged"], err.max(), scale, (err / bound).max(), med_rel, int((ref != 0).sum()), ref.size))
    assert (err <= bound).all(), "fails: %d" % int((err > bound).sum())
    assert med_rel <= med
    # the kernel traces what the oracle decides to trace, up to its undecided samples
    assert abs(st["rays_traced"] - o["traced"]) <= o["flagged"]
    return g, o


def test_edge_grad_parity_tiny():
    _need_gpu()
    w = make_workload("tiny")
    g, o = _parity(w, 16)
    assert o["traced"] > 100 and np.abs(o["g_verts"]).max() > 0


def test_edge_grad_parity_tau_and_view_base():
    """tau = 1/2 scales every term; view_base shifts the view id of the random
    counter; a different seed draws other edges."""
    _need_gpu()
    w = make_workload("tiny")
    w.tau = 0.5
    w.view_base = 3
    w.seed = 12345
    g, o = _parity(w, 16)
    assert o["traced"] > 100


def test_edge_grad_parity_sphere8_small():
    _need_gpu()
    _parity(make_workload("sphere8_grad", H=64, W=64, n_views=1), 8)


@pytest.mark.parametrize("gain", [64, 1024])
def test_edge_grad_parity_sharp_gain(gain):
    """Sharp edges drawn more often: the class decisions (FP32) and the class
    choice (integers) match the oracle's, and so do the weighted terms."""
    _need_gpu()
    _parity(make_workload("sphere8_grad", H=64, W=64, n_views=1), 8, gain=gain)
    _parity(make_workload("tiny"), 16, gain=gain)


def test_edge_grad_parity_largest_edge_spp():
    """1024 edge samples per pixel, the most the library takes: 32 filter
    chunks of 32 samples per pixel and all 10 bits of the sample index in the
    queue records.  Each vertex component sums ~10^3 terms (u sqrt(n) ~ 2e-6
    of their magnitudes), well inside the default median guard."""
    _need_gpu()
    _parity(make_workload("tiny", H=16, W=16), 1024)


def test_edge_grad_parity_bilinear():
    _need_gpu()
    import paper_2206_03380_amd as M
    _parity(make_workload("sphere8_grad", H=48, W=40, n_views=1), 8, flags=M.FLAG_BILINEAR, med=1e-4)


def _ground_scene(N, seed=5):
    """A ground quad with two boxes on it; N receiver pixels scattered on the
    ground (one view of 1 x N pixels)."""
    r = np.random.Generator(np.random.PCG64(seed))
    parts = [meshes.quad([-3, 0, -3], [-3, 0, 3], [3, 0, 3], [3, 0, -3]),
             meshes.box([0.3, 0.4, 0.0], [0.3, 0.4, 0.25], 0.4), meshes.box([-0.8, 0.25, 0.6], [0.2, 0.25, 0.3], 1.1)]
    v, f = meshes.merge(parts)
    pos = np.stack([r.uniform(-2.5, 2.5, N), np.zeros(N), r.uniform(-2.5, 2.5, N)], axis=1)
    env = r.lognormal(0.0, 1.0, size=(16, 32, 3)).astype(np.float32)
    kd = r.uniform(0, 1, (N, 3))
    korm = np.stack([np.ones(N), r.uniform(0.1, 1.0, N), r.uniform(0, 1, N)], axis=1)
    return from_arrays("ground", v, f, env, pos, np.tile([0.0, 1.0, 0.0], (N, 1)), kd, korm,
                       eye=[[0.5, 3.0, 4.0]], height=1, width=N, ray_eps=1e-4, tau=1.0, seed=3)


@pytest.mark.parametrize("gain", [1, 64])
def test_edge_grad_ragged_passes(gain):
    """9001 pixels at 512 edge samples: passes of 8192 pixels and a ragged
    tail of 809; pixels inside the boxes' footprints see no sky at all.  Each
    of the 60 vertex components sums some 10^4 - 10^5 FP32 terms of both signs
    (u sqrt(n) ~ 2e-5 of the sum of magnitudes, several times that of the
    signed sum): the median guard is set from that.  At gain 64 the box edges
    and the ground's border (sharp) take nearly every sample and the face
    diagonals (smooth) the rest, in every pass."""
    _need_gpu()
    _parity(_ground_scene(9001), 512, med=3e-4, gain=gain)


def test_edge_grad_full_size_sampled():
    """The benchmark's workload and launch shape (every pixel's lane runs),
    with the upstream gradient nonzero on sampled pixels only."""
    _need_gpu()
    w = make_workload("sphere8_grad")
    r = np.random.Generator(np.random.PCG64(9))
    valid_all = np.nonzero(w.mask)[0]
    keep = np.sort(r.choice(valid_all, 8000, replace=False))
    mask = np.zeros_like(w.mask)
    mask[keep] = 1
    w.mask = mask
    _parity(w, 8, pixels=keep)


def test_edge_grad_parity_non_finite_vertex():
    """A vertex at NaN: the scene drops its triangles, and no edge sample that
    touches it adds a term (on either side)."""
    _need_gpu()
    w = make_workload("tiny")
    w.verts = w.verts.copy()
    w.verts[7] = np.nan
    g, o = _parity(w, 16)
    assert np.isfinite(g).all() and (g[7] == 0).all()


def test_edge_grad_accumulates_and_degenerate_cases():
    _need_gpu()
    import paper_2206_03380_amd as M
    w = make_workload("tiny")
    g1, _, _ = _run_gpu(w, 4)
    init = np.full(w.verts.shape, 0.25, np.float32)
    g2, _, _ = _run_gpu(w, 4, g_init=init)
    # each term added onto 0.25 rounds at the ulps of 0.25 + |g|: a few
    # dozen of those across the components' terms
    assert np.allclose(g2 - 0.25, g1, rtol=1e-5, atol=2e-6 * (0.25 + np.abs(g1).max()))
    g0, st, _ = _run_gpu(w, 4, tau=0.0, g_init=init)
    assert (g0 == 0.25).all() and st["rays_traced"] == 0
    dev = "cuda"
    verts = torch.from_numpy(w.verts).to(dev)
    tris = torch.from_numpy(w.tris).to(dev)
    scene, env = M.Scene(verts, tris), M.Env(torch.from_numpy(w.env).to(dev))
    gb = M.GBuffer.from_workload(w, dev)
    ud, us = (torch.from_numpy(x).to(dev) for x in upstream_grads(w))
    ed_bad = M.Edges(tris, len(w.verts) + 1)
    with pytest.raises(M.MCDIError):
        M.shade_bwd_edges(scene, env, ed_bad, verts, gb, 4, ud, us)
    ed = M.Edges(tris, len(w.verts))
    for bad_es in (0, 1025):
        with pytest.raises(M.MCDIError):
            M.shade_bwd_edges(scene, env, ed, verts, gb, bad_es, ud, us)
    for bad_gain in (0, 1025):
        with pytest.raises(M.MCDIError):
            M.shade_bwd_edges(scene, env, ed, verts, gb, 4, ud, us, sharp_gain=bad_gain)
    # a mesh with no triangles: nothing to do
    no_tris = torch.zeros((0, 3), dtype=torch.int32, device=dev)
    g = M.shade_bwd_edges(M.Scene(verts, no_tris), env, M.Edges(no_tris, len(w.verts)), verts, gb, 4, ud, us)
    torch.cuda.synchronize()
    assert (to_np(g) == 0).all()


@pytest.mark.parametrize("gain", [1, 64])
def test_autograd_returns_visibility_gradient(gain):
    """MCDIShade with verts/edges: loss.backward() puts the edge-sampled
    visibility gradient into verts.grad, the same as the direct call with the
    same sharp-class gain."""
    _need_gpu()
    import paper_2206_03380_amd as M
    w = make_workload("tiny")
    dev = "cuda"
    verts = torch.from_numpy(w.verts).to(dev).requires_grad_(True)
    tris = torch.from_numpy(w.tris).to(dev)
    scene = M.Scene(verts.detach(), tris)
    env_t = torch.from_numpy(w.env).to(dev)
    envh = M.Env(env_t)
    gb = M.GBuffer.from_workload(w, dev)
    ed = M.Edges(tris, len(w.verts))
    ud, us = (torch.from_numpy(x).to(dev) for x in upstream_grads(w))
    c_d, c_s = M.MCDIShade.apply(gb.kd, gb.korm, gb.nrm, env_t, scene, envh, gb, w.spp, w.seed, w.tau, w.ray_eps, 0,
                                 None, verts, ed, 8, gain)
    ((c_d * ud).sum() + (c_s * us).sum()).backward()
    ref = M.shade_bwd_edges(scene, envh, ed, verts.detach(), gb, 8, ud, us, seed=w.seed, tau=w.tau,
                            ray_eps=w.ray_eps, sharp_gain=gain)
    torch.cuda.synchronize()
    g, r = to_np(verts.grad), to_np(ref)
    assert np.abs(r).max() > 0
    assert np.allclose(g, r, rtol=1e-5, atol=1e-6 * np.abs(r).max())


def test_edge_list_and_grad_lattice_sampled():
    """Maximum size: the 1.0M-triangle lattice room (thin beams, heavy
    occlusion, many silhouettes); its edge list bit for bit, and the gradient
    with the upstream gradient nonzero on sampled pixels."""
    _need_gpu()
    import paper_2206_03380_amd as M
    w = make_workload("lattice", H=256, W=256, n_views=2)
    print("lattice", len(w.verts), "verts", len(w.tris), "tris", flush=True)
    ed = M.Edges(torch.from_numpy(w.tris).cuda(), len(w.verts))
    rows = to_np(ed.rows())
    ref = oracle.mesh_edges(w.tris, len(w.verts))
    assert rows.shape == ref.shape and (rows == ref).all()
    r = np.random.Generator(np.random.PCG64(5))
    keep = np.sort(r.choice(np.nonzero(w.mask)[0], 2500, replace=False))
    mask = np.zeros_like(w.mask)
    mask[keep] = 1
    w.mask = mask
    # inside the closed room almost every out-side ray is blocked; 256 edge
    # samples per pixel give a few that leave through the windows
    g, o = _parity(w, 256, pixels=keep)
    assert o["traced"] > 10000 and (o["g_verts"] != 0).sum() > 0

"""Pins of the oracle's edge-sampled visibility gradient and of its edge list.

The estimator's expectation is the derivative of the shadowed integral with
respect to the occluder's vertices.  It is pinned against quantities fixed by
the mathematics, not by the oracle's own code:
  * Lambert's closed form for the cosine-weighted solid angle of a polygon
    (diffuse receiver, constant probe), differentiated by central differences;
  * a Gauss-Legendre quadrature of the unshadowed integrand over the
    occluding triangle (glossy receiver), differentiated the same way;
  * special cases: a planar quad split in two (its shared edge is no
    silhouette), an edge hidden behind a larger occluder (zero), an occluder
    below the horizon (zero), tau = 0 (zero), reversed winding (unchanged).
Statistical comparisons use the spread over independent seeds.
"""

import numpy as np
import pytest

import oracle
from workloads import from_arrays
from workloads import meshes


# ---------------------------------------------------------------------------
# edge list
# ---------------------------------------------------------------------------

def _unique_pairs(tris):
    """Undirected edges by sorting all sides (an independent construction)."""
    s = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    return np.unique(np.sort(s, axis=1), axis=0)


def test_edges_closed_mesh_euler():
    v, f = meshes.icosphere(2)
    E = oracle.mesh_edges(f, len(v))
    assert len(E) == 3 * len(f) // 2
    assert len(v) - len(E) + len(f) == 2                     # Euler characteristic of a sphere
    assert (E[:, 3] >= 0).all()                              # every edge has two faces
    keys = np.sort(E[:, :2], axis=1)
    assert len(np.unique(keys, axis=0)) == len(E)
    assert (np.unique(keys, axis=0) == _unique_pairs(f)).all()
    # first appearance order: side id of each row's first occurrence increases
    side = {}
    for t in range(len(f)):
        for k in range(3):
            a, b = f[t][k], f[t][(k + 1) % 3]
            side.setdefault((min(a, b), max(a, b)), 3 * t + k)
    first = [side[(min(a, b), max(a, b))] for a, b in E[:, :2]]
    assert np.all(np.diff(first) > 0)
    # opposite corners: c and d are the third corners of the two faces
    for a, b, c, d in E[:20]:
        faces = [set(t) for t in f if a in t and b in t]
        assert len(faces) == 2
        assert {c, d} == {next(iter(faces[0] - {a, b})), next(iter(faces[1] - {a, b}))}


def test_edges_open_grid_and_bad_triangles():
    # 3 x 3 grid of quads: the boundary has 12 unit segments
    n = 4
    idx = np.arange(n * n).reshape(n, n)
    tris = []
    for i in range(n - 1):
        for j in range(n - 1):
            tris.append([idx[i, j], idx[i + 1, j], idx[i + 1, j + 1]])
            tris.append([idx[i, j], idx[i + 1, j + 1], idx[i, j + 1]])
    tris = np.array(tris)
    E = oracle.mesh_edges(tris, n * n)
    assert len(E) == len(_unique_pairs(tris))
    assert (E[:, 3] < 0).sum() == 4 * (n - 1)
    # a triangle with an index out of range adds nothing; one with a repeated
    # corner adds its remaining edge once (here 5-6 already has two faces)
    bad = np.vstack([tris, [[0, 1, 99]], [[5, 5, 6]]])
    assert (oracle.mesh_edges(bad, n * n) == E).all()
    E2 = oracle.mesh_edges(np.vstack([tris, [[0, 0, 15]]]), n * n)
    assert len(E2) == len(E) + 1 and tuple(E2[-1]) == (0, 15, 0, 0)
    # non-manifold: three faces on one edge -> d from the second face
    nm = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]])
    E3 = oracle.mesh_edges(nm, 5)
    row = [r for r in E3 if set(r[:2]) == {0, 1}][0]
    assert tuple(row) == (0, 1, 2, 3)


# ---------------------------------------------------------------------------
# the estimator
# ---------------------------------------------------------------------------

N_SIDE = 48
ENV_RGB = np.array([1.0, 0.5, 0.25], np.float32)


def _receiver(verts, tris, korm=(1.0, 0.5, 0.3), kd=(0.5, 0.5, 0.5), eye=(0.0, 1.0, 2.0), tau=1.0):
    """N_SIDE^2 identical pixels at the origin facing +Y under a constant probe."""
    N = N_SIDE * N_SIDE
    env = np.ones((8, 16, 3), np.float32) * ENV_RGB
    pos = np.zeros((N, 3))
    nrm = np.tile([0.0, 1.0, 0.0], (N, 1))
    return from_arrays("edge", verts, tris, env, pos, nrm, np.tile(kd, (N, 1)), np.tile(korm, (N, 1)),
                       eye=[list(eye)], height=N_SIDE, width=N_SIDE, ray_eps=1e-4, tau=tau)


def _mean_grad(w, ud, us, n_es=16, seeds=8, **kw):
    E = oracle.mesh_edges(w.tris, len(w.verts))
    runs = np.array([oracle.edge_grad(w, E, n_es, ud, us, seed=s, **kw)["g_verts"] for s in range(seeds)])
    return runs.mean(0), runs.std(0, ddof=1) / np.sqrt(seeds)


def _lambert(o, n, V):
    """Cosine-weighted solid angle of a planar polygon seen from o (all of it
    above the plane through o normal to n): half the sum over edges of the
    angle the edge subtends times n . (unit normal of the edge's plane)."""
    q = [np.asarray(v, float) - o for v in V]
    tot = 0.0
    for i in range(len(q)):
        a, b = q[i], q[(i + 1) % len(q)]
        c = np.cross(a, b)
        tot += np.arctan2(np.linalg.norm(c), a @ b) * (n @ c) / np.linalg.norm(c)
    return abs(0.5 * tot)


def _fd(fun, V, h=1e-6):
    g = np.zeros_like(V, dtype=float)
    for i in range(V.shape[0]):
        for k in range(3):
            P, M = V.astype(float).copy(), V.astype(float).copy()
            P[i, k] += h
            M[i, k] -= h
            g[i, k] = (fun(P) - fun(M)) / (2 * h)
    return g


O = np.array([0.0, 1e-4, 0.0])
NY = np.array([0.0, 1.0, 0.0])
TRI = np.array([[-0.3, 1.0, -0.2], [0.4, 1.1, -0.1], [0.0, 0.9, 0.5]])


def _diffuse_expect(V, m=0.3, tau=1.0):
    # c_d = (1 - m)/pi * L * (pi - tau * Phi): d/dV = -(1 - m)/pi * L * tau * dPhi/dV
    return -(1 - m) / np.pi * tau * _fd(lambda P: _lambert(O, NY, P), V)


def _ud_us(w, ud_rgb=(1.0, 1.0, 1.0), us_rgb=(0.0, 0.0, 0.0)):
    N = w.n_pixels
    ud = np.tile(np.asarray(ud_rgb, float)[:, None], (1, N)) / N
    us = np.tile(np.asarray(us_rgb, float)[:, None], (1, N)) / N
    return ud, us


def _check_stat(mean, se, expect, rel=2e-3, z=5.0):
    err = np.abs(mean - expect)
    lim = z * se + rel * np.abs(expect).max()
    assert (err <= lim).all(), (mean, expect, se)


def test_lambert_closed_form_diffuse():
    """Diffuse receiver under a constant probe, one occluding triangle."""
    w = _receiver(TRI, [[0, 1, 2]])
    ud, us = _ud_us(w)
    mean, se = _mean_grad(w, ud, us)
    Lsum = float(ENV_RGB.sum())
    _check_stat(mean, se, Lsum * _diffuse_expect(TRI))
    # reversed winding: the same gradient (the estimator does not depend on it)
    w2 = _receiver(TRI, [[0, 2, 1]])
    mean2, se2 = _mean_grad(w2, ud, us)
    _check_stat(mean2, se2, Lsum * _diffuse_expect(TRI))


def test_tau_scales_and_zero():
    w = _receiver(TRI, [[0, 1, 2]], tau=0.5)
    ud, us = _ud_us(w)
    mean, se = _mean_grad(w, ud, us, seeds=4)
    _check_stat(mean, se, float(ENV_RGB.sum()) * _diffuse_expect(TRI, tau=0.5))
    E = oracle.mesh_edges(w.tris, 3)
    r = oracle.edge_grad(w, E, 8, ud, us, tau=0.0)
    assert (r["g_verts"] == 0).all() and r["samples"] == 0


def test_quad_interior_edge_is_no_silhouette():
    """A planar quad in two triangles: the shared diagonal is covered on both
    sides and adds nothing; the result is the quad's closed form."""
    Q = np.array([[-0.4, 1.0, -0.3], [0.5, 1.0, -0.35], [0.45, 1.05, 0.4], [-0.35, 1.05, 0.45]])
    # make it planar: project the last corner onto the plane of the first three
    nq = np.cross(Q[1] - Q[0], Q[2] - Q[0])
    nq /= np.linalg.norm(nq)
    Q[3] -= ((Q[3] - Q[0]) @ nq) * nq
    w = _receiver(Q, [[0, 1, 2], [0, 2, 3]])
    ud, us = _ud_us(w)
    mean, se = _mean_grad(w, ud, us)
    expect = -(1 - 0.3) / np.pi * _fd(lambda P: _lambert(O, NY, P), Q) * float(ENV_RGB.sum())
    _check_stat(mean, se, expect)


def test_hidden_edge_contributes_nothing():
    """A small triangle entirely behind a large one (seen from o) gets exactly
    zero; the large one keeps its closed-form gradient."""
    big = np.array([[-0.8, 1.0, -0.8], [0.8, 1.0, -0.8], [0.0, 1.0, 0.9]])
    small = np.array([[-0.05, 2.0, 0.0], [0.05, 2.0, 0.0], [0.0, 2.1, 0.05]])
    V = np.vstack([big, small])
    w = _receiver(V, [[0, 1, 2], [3, 4, 5]])
    ud, us = _ud_us(w)
    mean, se = _mean_grad(w, ud, us, seeds=4)
    assert (mean[3:] == 0.0).all()
    _check_stat(mean[:3], se[:3], float(ENV_RGB.sum()) * _diffuse_expect(big))


def test_below_horizon_is_zero():
    V = TRI.copy()
    V[:, 1] = -V[:, 1]
    w = _receiver(V, [[0, 1, 2]])
    ud, us = _ud_us(w)
    E = oracle.mesh_edges(w.tris, 3)
    r = oracle.edge_grad(w, E, 16, ud, us)
    assert (r["g_verts"] == 0.0).all() and r["silhouettes"] == 0


def _gl_triangle(V, n=40):
    """Gauss-Legendre nodes over a triangle (collapsed square): points [K,3]
    and area weights [K]."""
    x, wx = np.polynomial.legendre.leggauss(n)
    s, ws = 0.5 * (x + 1), 0.5 * wx
    S, T = np.meshgrid(s, s, indexing="ij")
    W2 = np.outer(ws, ws)
    a, b, c = V
    P = a + S[..., None] * (b - a) + (S * T)[..., None] * (c - b)
    J = np.linalg.norm(np.cross(b - a, c - b)) * S
    return P.reshape(-1, 3), (W2 * J).reshape(-1)


def test_glossy_receiver_against_quadrature():
    """Glossy receiver: the expectation equals -tau times the derivative of the
    unshadowed integrand's integral over the directions the triangle covers,
    taken by quadrature over the triangle (solid angle = |n_T . q| / |q|^3 dA)."""
    korm = (1.0, 0.35, 0.8)
    w = _receiver(TRI, [[0, 1, 2]], korm=korm, kd=(0.9, 0.6, 0.3), eye=(0.3, 1.2, 1.5))
    ud, us = _ud_us(w, ud_rgb=(0.3, 0.2, 0.1), us_rgb=(1.0, 0.7, 0.4))
    mean, se = _mean_grad(w, ud, us, n_es=32, seeds=8)
    empty = oracle.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))
    tables = oracle.EnvTables(w.env)
    o = np.array([0.0, np.float32(1e-4), 0.0])

    def covered(P):
        pts, wts = _gl_triangle(P)
        q = pts - o
        r = np.linalg.norm(q, axis=1)
        nt = np.cross(P[1] - P[0], P[2] - P[0])
        nt /= np.linalg.norm(nt)
        dom = np.abs(q @ nt) / r ** 3 * wts
        gd, gs = oracle.integrand(w, 0, q / r[:, None], scene=empty, tables=tables, tau=0.0)
        g = gd @ ud[:, 0] + gs @ us[:, 0]
        return float((g * dom).sum()) * w.n_pixels   # every pixel sees the same integral

    expect = -1.0 * _fd(covered, TRI, h=1e-5)
    _check_stat(mean, se, expect, rel=3e-3)


def test_shared_silhouette_edge_counts_once():
    """Two faces folded about a shared edge, the second hidden behind the
    first as seen from o: the shared edge is a silhouette of both faces and
    must count once.  The union of the faces' directions is the front face's,
    so its closed form applies, and the hidden corner gets (almost) zero."""
    A, B, Cc = TRI
    inner = (A + B + Cc) / 3.0 + 0.2 * (A - (A + B + Cc) / 3.0)
    D = O + 2.0 * (inner - O)                  # behind the front face, inside its outline
    V = np.vstack([TRI, D[None]])
    w = _receiver(V, [[0, 1, 2], [1, 0, 3]])
    ud, us = _ud_us(w)
    E = oracle.mesh_edges(w.tris, 4)
    assert tuple(E[0]) == (0, 1, 2, 3)
    mean, se = _mean_grad(w, ud, us)
    expect = float(ENV_RGB.sum()) * _diffuse_expect(TRI)
    # the hidden edges' out-side rays leave the front face only within the
    # out-side offset of the shared corners: a vanishing remainder
    assert np.abs(mean[3]).max() <= 1e-5 * np.abs(expect).max()
    _check_stat(mean[:3], se[:3], expect)


def test_non_finite_vertex_adds_nothing():
    """A triangle with a non-finite corner contributes nothing; the others
    keep their closed form."""
    V = np.vstack([TRI, [[np.nan, 1.0, 0.0], [0.5, 1.5, 0.5], [0.6, 1.4, 0.4]]])
    w = _receiver(V, [[0, 1, 2], [3, 4, 5]])
    ud, us = _ud_us(w)
    mean, se = _mean_grad(w, ud, us, seeds=4)
    assert np.isfinite(mean).all()
    assert (mean[3:] == 0.0).all() or np.abs(mean[3:]).max() < 1e-12


def test_edge_classes():
    """Sharp: a box's edges (not its face diagonals), an icosahedron's
    (normals 41.8 degrees apart), the boundary of a flat grid.  Not sharp: a
    fine icosphere's, the inside of a flat grid."""
    v, f = meshes.box([0.0, 0.0, 0.0], [0.3, 0.2, 0.1], 0.4)
    E = oracle.mesh_edges(f, len(v))
    sharp = oracle.edge_sharp(v, E)
    assert sharp.sum() == 12 and len(E) == 18
    # corner index = 4 ix + 2 iy + iz: a box edge flips one bit, a face
    # diagonal two
    flips = np.array([bin(int(a) ^ int(b)).count("1") for a, b in E[:, :2]])
    assert ((flips == 1) == sharp).all()
    v, f = meshes.icosphere(0)
    assert oracle.edge_sharp(v, oracle.mesh_edges(f, len(v))).all()
    v, f = meshes.icosphere(3)
    assert not oracle.edge_sharp(v, oracle.mesh_edges(f, len(v))).any()
    n = 4
    idx = np.arange(n * n).reshape(n, n)
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 2)
    v = np.stack([g[:, 0], np.zeros(n * n), g[:, 1]], 1).astype(np.float32)
    f = np.array([[idx[i, j], idx[i + 1, j], idx[i + 1, j + 1]] for i in range(n - 1) for j in range(n - 1)] +
                 [[idx[i, j], idx[i + 1, j + 1], idx[i, j + 1]] for i in range(n - 1) for j in range(n - 1)])
    E = oracle.mesh_edges(f, n * n)
    assert (oracle.edge_sharp(v, E) == (E[:, 3] < 0)).all()


def test_class_weights_keep_the_expectation():
    """A box (sharp and smooth edges) and a smooth icosphere shell above the
    receiver: the two-class choice (gain 64) and a uniform choice (gain 1)
    have the same expectation, and the two-class one draws the box's
    silhouettes far more often."""
    bv, bf = meshes.box([0.0, 1.0, 0.0], [0.2, 0.05, 0.2], 0.3)
    sv, sf = meshes.icosphere(3)
    sv = sv * 0.25 + np.array([0.35, 1.6, 0.2])
    V, F = meshes.merge([(bv, bf), (sv, sf)])
    w = _receiver(V, F)
    ud, us = _ud_us(w)
    E = oracle.mesh_edges(w.tris, len(w.verts))
    sharp = oracle.edge_sharp(w.verts, E)
    assert 0 < sharp.sum() < len(E)
    m64, s64 = _mean_grad(w, ud, us, n_es=64, seeds=8, sharp_gain=64)
    m1, s1 = _mean_grad(w, ud, us, n_es=64, seeds=8, sharp_gain=1)
    scale = np.abs(m64).max()
    assert scale > 0
    assert (np.abs(m64 - m1) <= 5 * np.sqrt(s64 ** 2 + s1 ** 2) + 2e-3 * scale).all()
    # the box's vertices: the two-class estimate is much less noisy
    nb = len(bv)
    assert np.median(s64[:nb][np.abs(m64[:nb]) > 0]) < 0.5 * np.median(s1[:nb][np.abs(m64[:nb]) > 0])

"""Pins of the oracle's bilinear probe lookup (technique flag BILINEAR).

The paper keeps the probe as a float texture (section 3.1) and samples it with
a piecewise-constant 2D distribution (section 4.1); the lookup filter is not
named.  The filtered reading reconstructs the radiance with tent weights
centred on texel centres, wrapping across the phi seam and clamping at the
poles, while the light technique keeps its per-texel density.  What pins it:

  texel centres      the reconstruction returns the texel itself there;
  affine probes      bilinear interpolation of an affine function is that
                     function (closed form, interior of the probe);
  seam and poles     hand-computed tent weights across phi = 0 and above the
                     first row centre;
  partition of unity a constant probe reconstructs to the constant everywhere;
  coordinates        the texel coordinates of a direction are (u W, v H) for
                     the direction of (u, v), and a light sample is looked up
                     at the coordinates of its own direction;
  quadrature         the estimator with the filtered lookup converges to a
                     dense quadrature of the filtered integrand (MIS, BSDF-only
                     and light-only; light-only ties the sampled coordinates to
                     those of the integrand);
  finite differences the probe gradient spreads over the four taps, and the
                     estimator is linear in each texel, so a finite difference
                     is exact.
"""

import numpy as np
import pytest

import oracle
from workloads import make_workload, from_arrays

RNG = np.random.Generator(np.random.PCG64(2206))


def _probe(H=16, W=32):
    return RNG.lognormal(0.0, 1.0, (H, W, 3)).astype(np.float32)


def test_bilinear_texel_centres_are_exact():
    env = _probe()
    H, W = env.shape[:2]
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    L = oracle.probe_bilinear(env, j.reshape(-1) + 0.5, i.reshape(-1) + 0.5)
    assert np.array_equal(L, env.reshape(-1, 3).astype(np.float64))


def test_bilinear_affine_probe_interior():
    H, W = 16, 32
    a, b, d = np.array([0.5, 1.0, 2.0]), np.array([0.25, -0.125, 0.5]), np.array([-0.75, 0.375, 0.0625])
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    env = (a + b * j[..., None] + d * i[..., None]).astype(np.float32)
    x = RNG.uniform(0.5, W - 0.5, 4000)
    y = RNG.uniform(0.5, H - 0.5, 4000)
    L = oracle.probe_bilinear(env, x, y)
    ref = a + b * (x - 0.5)[:, None] + d * (y - 0.5)[:, None]
    assert np.allclose(L, ref, rtol=1e-12, atol=1e-12)


def test_bilinear_seam_and_pole_weights():
    H, W = 8, 16
    one = lambda i, j: np.eye(H * W, dtype=np.float32)[i * W + j].reshape(H, W, 1).repeat(3, 2)  # noqa: E731
    # across the phi seam: the centres of columns W-1 and 0 are at -1/2 and 1/2
    assert oracle.probe_bilinear(one(3, 0), [0.25], [3.5])[0, 0] == 0.75
    assert oracle.probe_bilinear(one(3, W - 1), [0.25], [3.5])[0, 0] == 0.25
    assert oracle.probe_bilinear(one(3, 0), [W - 0.25], [3.5])[0, 0] == 0.25
    assert oracle.probe_bilinear(one(3, W - 1), [W - 0.25], [3.5])[0, 0] == 0.75
    # x = 0 and x = W are the same meridian
    env = _probe(H, W)
    y = RNG.uniform(0, H, 50)
    assert np.array_equal(oracle.probe_bilinear(env, np.zeros(50), y), oracle.probe_bilinear(env, np.full(50, W), y))
    # above the first row centre the rows clamp: the first row's value, any y
    for y in (0.0, 0.2, 0.5):
        assert oracle.probe_bilinear(one(0, 5), [5.5], [y])[0, 0] == 1.0
        assert oracle.probe_bilinear(one(H - 1, 5), [5.5], [H - y])[0, 0] == 1.0
    # between row centres 0 and 1: linear in y
    assert oracle.probe_bilinear(one(1, 5), [5.5], [1.25])[0, 0] == 0.75
    assert oracle.probe_bilinear(one(0, 5), [5.5], [1.25])[0, 0] == 0.25
    # between column centres: linear in x
    assert oracle.probe_bilinear(one(2, 6), [6.0], [2.5])[0, 0] == 0.5


def test_bilinear_partition_of_unity():
    env = np.ones((8, 16, 3), np.float32) * np.array([0.7, 1.0, 1.3], np.float32)
    x = np.concatenate([RNG.uniform(0, 16, 500), [0.0, 16.0, 0.5, 15.5]])
    y = np.concatenate([RNG.uniform(0, 8, 500), [0.0, 8.0, 0.25, 7.75]])
    L = oracle.probe_bilinear(env, x, y)
    assert np.allclose(L, env[0, 0].astype(np.float64), rtol=1e-14, atol=0)


def test_texel_coordinates_of_directions():
    H, W = 16, 32
    t = oracle.EnvTables(_probe(H, W))
    u = RNG.uniform(0, 1, 2000)
    v = RNG.uniform(0.01, 0.99, 2000)
    th, ph = np.pi * v, 2 * np.pi * u
    d = np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], -1)
    ti, tj, _, x, y = t.texel_of_dir(d, coords=True)
    assert np.allclose(x, u * W, atol=1e-9) and np.allclose(y, v * H, atol=1e-9)
    assert np.array_equal(ti, np.floor(y).astype(np.int32)) and np.array_equal(tj, np.floor(x).astype(np.int32))


def test_light_sample_coordinates_match_direction():
    """The coordinates a light sample looks the probe up at are those of its
    own direction, inside its own texel."""
    t = oracle.EnvTables(_probe(16, 32))
    xi0, xi1 = RNG.random(5000), RNG.random(5000)
    w, p, ti, tj, x, y = t.sample(xi0, xi1, coords=True)
    _, _, _, xd, yd = t.texel_of_dir(w, coords=True)
    assert np.allclose(x, xd, atol=1e-9) and np.allclose(y, yd, atol=1e-9)
    assert np.all((x >= tj) & (x < tj + 1) & (y >= ti) & (y < ti + 1))


def test_bilinear_white_furnace_equals_nearest():
    """A constant probe reconstructs to itself, so the filtered estimator
    equals the nearest-texel one up to the rounding of the weights."""
    n = 512
    env = np.ones((8, 16, 3), np.float32) * np.array([0.7, 1.0, 1.3], np.float32)
    nrm = RNG.normal(size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    pos = RNG.normal(size=(n, 3))
    kd = RNG.random((n, 3))
    korm = np.stack([np.ones(n), RNG.uniform(0.08, 1, n), RNG.random(n)], 1)
    w = from_arrays("furnace", np.zeros((3, 3), np.float32), np.zeros((0, 3), np.int32), env, pos, nrm, kd,
                    korm, eye=np.zeros(3), spp=16)
    a = oracle.shade(w)
    b = oracle.shade(w, flags=oracle.BILINEAR)
    assert np.allclose(a["c_d"], b["c_d"], rtol=1e-13, atol=0)
    assert np.allclose(a["c_s"], b["c_s"], rtol=1e-13, atol=0)


def test_bilinear_differs_from_nearest():
    w = make_workload("tiny")
    pix = np.nonzero(w.mask)[0][:256]
    a = oracle.shade(w, pixels=pix)
    b = oracle.shade(w, pixels=pix, flags=oracle.BILINEAR)
    # same samples and visibility, different radiance
    assert np.array_equal(a["hitbits"], b["hitbits"])
    rel = np.abs(a["c_d"] - b["c_d"]).sum() / np.abs(a["c_d"]).sum()
    assert rel > 0.05


def _sphere_dirs(H, W, S):
    U = (np.arange(W * S) + 0.5) / (W * S)
    V = (np.arange(H * S) + 0.5) / (H * S)
    U, V = np.meshgrid(U, V)
    th, ph = np.pi * V, 2 * np.pi * U
    d = np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], -1).reshape(-1, 3)
    wt = (2 * np.pi ** 2 * np.sin(th) / (H * S * W * S)).reshape(-1)
    return d, wt


@pytest.mark.parametrize("tech", ["mis", "bsdf", "light"])
def test_bilinear_mc_converges_to_quadrature(tech):
    flags = {"mis": 0, "bsdf": oracle.LIGHT_OFF, "light": oracle.BSDF_OFF}[tech] | oracle.BILINEAR
    w = make_workload("tiny")
    # a glossy metal pixel: its specular lobe is narrower than a texel, so the
    # filtered and the nearest-texel integrals differ visibly
    valid = np.nonzero((w.mask > 0) & (w.korm[1] > 0.15) & (w.korm[1] < 0.25) & (w.korm[2] > 0.6))[0]
    pix = valid[0]
    sc = oracle.Scene(w.verts, w.tris)
    tab = oracle.EnvTables(w.env)
    # the filtered integrand varies inside a texel: a finer grid than the
    # nearest-texel quadrature
    d, wt = _sphere_dirs(w.env.shape[0], w.env.shape[1], 32)
    gd, gs = oracle.integrand(w, pix, d, scene=sc, tables=tab, brute=False, flags=oracle.BILINEAR)
    gdn, gsn = oracle.integrand(w, pix, d, scene=sc, tables=tab, brute=False)
    quad_d, quad_s = (gd * wt[:, None]).sum(0), (gs * wt[:, None]).sum(0)
    N, spp = 8192, 8
    col = lambda a: np.tile(a[:, pix], (N, 1))  # noqa: E731
    rep = from_arrays("rep", w.verts, w.tris, w.env, col(w.pos), col(w.nrm), col(w.kd), col(w.korm),
                      eye=w.eye[0], spp=spp, ray_eps=w.ray_eps, tau=w.tau)
    o = oracle.shade(rep, scene=sc, tables=tab, flags=flags)
    for est, quad, near in ((o["c_d"], quad_d, (gdn * wt[:, None]).sum(0)),
                            (o["c_s"], quad_s, (gsn * wt[:, None]).sum(0))):
        mean = est.mean(1)
        se = est.std(1, ddof=1) / np.sqrt(N)
        assert np.all(np.abs(mean - quad) < 4 * se + 2e-3 * np.abs(quad)), (mean, quad, se)
        if est is o["c_s"] and tech != "light":
            # the two integrals differ by more than the test resolves
            assert np.any(np.abs(quad - near) > 8 * se + 4e-3 * np.abs(quad)), (quad, near, se)


def _grad_setup():
    rng = np.random.Generator(np.random.PCG64(2207))
    w = make_workload("tiny")
    valid = np.nonzero((w.mask > 0) & (w.korm[1] > 0.12))[0]
    pix = rng.choice(valid, 64, replace=False)
    n = len(pix)
    return w, pix, rng.normal(size=(3, n)), rng.normal(size=(3, n))


def _loss(o, Ud, Us):
    return (Ud * o["c_d"]).sum(0) + (Us * o["c_s"]).sum(0)


def test_bilinear_env_gradient_matches_fd():
    w, pix, Ud, Us = _grad_setup()
    sc = oracle.Scene(w.verts, w.tris)
    tab = oracle.EnvTables(w.env)
    g = oracle.shade(w, pixels=pix, scene=sc, tables=tab, grad=True, u_d=Ud, u_s=Us, flags=oracle.BILINEAR)
    ge = g["g_env"]
    nz = np.count_nonzero(np.abs(ge).sum(2))
    gn = oracle.shade(w, pixels=pix, scene=sc, tables=tab, grad=True, u_d=Ud, u_s=Us)
    # four taps per sample: more texels touched than by the nearest lookup
    assert nz > 2 * np.count_nonzero(np.abs(gn["g_env"]).sum(2))
    flat_top = np.argsort(-np.abs(ge).reshape(-1))[:6]
    # also texels the nearest lookup never touches
    untouched = np.nonzero((np.abs(gn["g_env"]).reshape(-1) == 0) & (np.abs(ge).reshape(-1) > 0))[0]
    for flat in list(flat_top) + list(untouched[:6]):
        i, j, c = np.unravel_index(flat, ge.shape)
        vals, xs = [], []
        for sgn in (1, -1):
            e2 = w.env.copy()
            e2[i, j, c] += np.float32(sgn * 0.25)
            xs.append(float(e2[i, j, c]))
            o = oracle.shade(w, pixels=pix, scene=sc, tables=tab, env_eval=e2, flags=oracle.BILINEAR)
            vals.append(_loss(o, Ud, Us).sum())
        fd = (vals[0] - vals[1]) / (xs[0] - xs[1])
        assert abs(fd - ge[i, j, c]) <= 1e-9 * max(1.0, abs(fd)), (fd, ge[i, j, c])
    assert np.all(g["s_env"] >= np.abs(ge) - 1e-15)


@pytest.mark.parametrize("field,ch", [("kd", 1), ("korm", 1), ("korm", 2), ("nrm", 0)])
def test_bilinear_backward_matches_frozen_fd(field, ch):
    w, pix, Ud, Us = _grad_setup()
    sc = oracle.Scene(w.verts, w.tris)
    tab = oracle.EnvTables(w.env)
    g = oracle.shade(w, pixels=pix, scene=sc, tables=tab, grad=True, u_d=Ud, u_s=Us, flags=oracle.BILINEAR)
    an = g[{"kd": "g_kd", "korm": "g_korm", "nrm": "g_nrm"}[field]][ch]
    eps = 1e-5
    res = []
    for sgn in (1, -1):
        arr = getattr(w, field).astype(np.float64).copy()
        arr[ch, pix] += sgn * eps
        o = oracle.shade(w, pixels=pix, scene=sc, tables=tab, eval_override={field: arr.astype(np.float32)},
                         flags=oracle.BILINEAR)
        res.append(_loss(o, Ud, Us))
    base = getattr(w, field).astype(np.float64)[ch, pix]
    h = ((base + eps).astype(np.float32).astype(np.float64) - base) + \
        (base - (base - eps).astype(np.float32).astype(np.float64))
    fd = (res[0] - res[1]) / h
    scale = np.abs(an).max() + 1e-12
    assert np.allclose(an, fd, rtol=2e-3, atol=2e-4 * scale), np.abs(an - fd).max() / scale

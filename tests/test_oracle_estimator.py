"""Estimator-level pins of the FP64 oracle.

  lobe choice        the BSDF technique picks the cosine lobe with frequency
                     q = (1 - m)/2 where n.v > 0 and always where n.v <= 0
                     (every q in (0, 1) is unbiased, so the expectation pins
                     below cannot see it);
  white furnace      uniform probe, no occluder: E[c_d] = (1 - m) L0, and with
                     the light technique off and q = 1 every sample equals it;
  Lambert occluder   uniform probe, a convex polyhedron above a receiver:
                     E[c_d] = (1 - m) L0 (1 - tau F), F the point-to-polygon
                     form factor (Lambert's contour formula) summed over the
                     front-facing faces;
  quadrature         non-uniform probe and an occluding mesh: the Monte Carlo
                     mean converges to a dense quadrature of the integrand;
  finite differences the backward pass equals central differences of the
                     frozen-sample estimator (samples, pdfs, q and visibility
                     fixed; paper: detached sampling and visibility);
  linearity          doubling the probe doubles c_d, c_s bit for bit; tau = 0
                     equals a scene without triangles bit for bit.
"""

import numpy as np
import pytest

import oracle
from workloads import make_workload, from_arrays
from workloads import meshes
from tests.parity_util import occluder_with_hidden_infinity

RNG = np.random.Generator(np.random.PCG64(1185))


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _empty_mesh():
    return np.zeros((3, 3), np.float32), np.zeros((0, 3), np.int32)


# ---------------------------------------------------------------------------
# white furnace
# ---------------------------------------------------------------------------
def _furnace(n=2048, spp=64, L0=(0.7, 1.0, 1.3)):
    env = np.ones((8, 16, 3), np.float32) * np.array(L0, np.float32)
    nrm = _unit(RNG.normal(size=(n, 3)))
    pos = RNG.normal(size=(n, 3))
    eye = np.zeros(3)
    # keep some back-facing pixels (n.v <= 0 path)
    kd = RNG.random((n, 3))
    korm = np.stack([np.ones(n), RNG.uniform(0.08, 1, n), RNG.random(n)], 1)
    v, f = _empty_mesh()
    w = from_arrays("furnace", v, f, env, pos, nrm, kd, korm, eye=eye, spp=spp)
    return w, env[0, 0].astype(np.float64)


def test_white_furnace_expectation():
    w, L0 = _furnace()
    o = oracle.shade(w)
    m = w.korm[2].astype(np.float64)
    ratio = o["c_d"] / (1.0 - m)[None, :]
    # per-channel results are exactly proportional to L0 (same samples)
    r = ratio / L0[:, None]
    assert np.allclose(r[0], r[1], rtol=1e-12) and np.allclose(r[0], r[2], rtol=1e-12)
    mean = r[0].mean()
    se = r[0].std(ddof=1) / np.sqrt(r.shape[1])
    assert abs(mean - 1.0) < 4 * se + 1e-12, (mean, se)
    assert se < 0.01


def test_white_furnace_cosine_only_is_exact():
    w, L0 = _furnace(n=256, spp=8)
    o = oracle.shade(w, flags=oracle.LIGHT_OFF | oracle.FORCE_COS)
    m = w.korm[2].astype(np.float64)
    assert np.allclose(o["c_d"], (1 - m)[None, :] * L0[:, None], rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------
# lobe-selection probability (the paper leaves the mixture weight open; the
# reading is q = (1 - m)/2 where the view is above the surface, else 1)
# ---------------------------------------------------------------------------
def _lobe_workload(m, n=1024, spp=64):
    """Half the pixels face the eye (n.v > 0), half face away (n.v < 0);
    metallic m everywhere, albedo and roughness random (q must not depend on
    them)."""
    eye = np.array([0.0, 0.0, 5.0])
    pos = RNG.uniform(-0.5, 0.5, (n, 3)) * np.array([1.0, 1.0, 0.0])
    tilt = _unit(np.concatenate([RNG.normal(size=(n, 2)) * 0.4, np.ones((n, 1))], 1))
    nrm = tilt.copy()
    nrm[n // 2:] *= -1.0
    kd = RNG.random((n, 3))
    korm = np.stack([np.ones(n), RNG.uniform(0.08, 1, n), np.full(n, m)], 1)
    env = np.ones((8, 16, 3), np.float32)
    v, f = _empty_mesh()
    return from_arrays("lobes", v, f, env, pos, nrm, kd, korm, eye=eye, spp=spp)


@pytest.mark.parametrize("m", [0.0, 0.3, 1.0])
def test_lobe_choice_frequency(m):
    """The BSDF sample takes the cosine lobe with frequency q = (1 - m)/2
    where n.v > 0 (binomial, within 4 standard deviations; exactly never at
    m = 1), and always where n.v <= 0.  A q that depended on kd or on the
    roughness, or a weight like m/2 or 1 - m, fails."""
    w = _lobe_workload(m)
    o = oracle.shade(w, want_decisions=True)
    cos = (o["decisions"][..., 2] & oracle.DEC_LOBE_COS) != 0
    nov_pos = (o["decisions"][..., 2] & oracle.DEC_NOV_POS) != 0
    front = nov_pos.all(axis=1)
    assert front.sum() == w.n_pixels // 2 and (~nov_pos[~front]).all()
    q = float(np.float32(0.5) * (np.float32(1.0) - np.float32(m)))
    k = cos[front]
    freq = k.mean()
    if q == 0.0:
        assert not k.any()
    else:
        sd = np.sqrt(q * (1 - q) / k.size)
        assert abs(freq - q) < 4 * sd, (freq, q, sd)
    # q does not depend on albedo or roughness: the frequency is the same in
    # the two halves of the pixels sorted by roughness
    order = np.argsort(w.korm[1][: w.n_pixels // 2])
    lo, hi = k[order[: len(order) // 2]].mean(), k[order[len(order) // 2:]].mean()
    if q > 0:
        assert abs(lo - hi) < 6 * np.sqrt(q * (1 - q) / (k.size / 2))
    assert cos[~front].all()


def test_lobe_choice_forced():
    """FORCE_COS: q = 1 everywhere; FORCE_GGX: q = 0 where n.v > 0 (cosine
    where the view is below the surface, where GGX visible-normal sampling
    has no density)."""
    w = _lobe_workload(0.3, n=256, spp=16)
    for flag, want_front in ((oracle.FORCE_COS, True), (oracle.FORCE_GGX, False)):
        o = oracle.shade(w, want_decisions=True, flags=oracle.LIGHT_OFF | flag)
        cos = (o["decisions"][..., 2] & oracle.DEC_LOBE_COS) != 0
        front = ((o["decisions"][..., 2] & oracle.DEC_NOV_POS) != 0).all(axis=1)
        assert (cos[front] == want_front).all() and cos[~front].all()


# ---------------------------------------------------------------------------
# smooth specular limit: Schlick's Fresnel at the view angle
# ---------------------------------------------------------------------------
def _mirror_limit(metallic, n=256, spp=64):
    """A flat receiver seen at 60 degrees (n.v = 1/2) under a constant probe,
    roughness at its clamp (alpha = 0.0064), kd = 1/2, no occluder."""
    env = np.ones((8, 16, 3), np.float32)
    pos = np.zeros((n, 3))
    nrm = np.tile([0.0, 1.0, 0.0], (n, 1))
    eye = np.array([10.0 * np.sin(np.pi / 3), 10.0 * np.cos(np.pi / 3), 0.0])
    kd = np.full((n, 3), 0.5)
    korm = np.tile([1.0, 0.08, metallic], (n, 1))
    v, f = _empty_mesh()
    return from_arrays("mirror", v, f, env, pos, nrm, kd, korm, eye=eye, spp=spp)


@pytest.mark.parametrize("metallic, F", [(0.0, 0.04 + 0.96 / 32), (1.0, 0.5 + 0.5 / 32)])
def test_smooth_specular_reflects_schlick_fresnel(metallic, F):
    """Near the mirror limit the specular output is the Fresnel reflectance at
    the view angle times the lobe's directional albedo, and at alpha = 0.0064
    that albedo is 1 within 1e-4 (Smith Lambda ~ 3e-5, no mass below the
    horizon).  Schlick's approximation at n.v = 1/2 gives F0 + (1 - F0)/32:
    0.07 for a dielectric (F0 = 0.04) and 0.515625 for a metal with
    kd = 1/2 (an exponent of 4 would give 0.1 and 0.53125).  With GGX
    sampling alone every sample is F(v.h) G2/G1, and over the 16k samples the
    symmetric spread of v.h about 1/2 moves the mean of F by < 1e-3 (GGX's
    tail of far half vectors holds ~2% of them); with the full MIS estimator
    the mean is also within 4 standard errors."""
    w = _mirror_limit(metallic)
    cs = oracle.shade(w, flags=oracle.LIGHT_OFF | oracle.FORCE_GGX)["c_s"]
    assert abs(cs.mean() - F) < 1e-3, (cs.mean(), F)
    cs = oracle.shade(w)["c_s"][0]
    se = cs.std(ddof=1) / np.sqrt(cs.size)
    assert abs(cs.mean() - F) < 4 * se + 1e-3, (cs.mean(), se, F)
    assert se < 0.02 * F


# ---------------------------------------------------------------------------
# Lambert: convex polyhedron over a receiver
# ---------------------------------------------------------------------------
def lambert_form_factor(p, n, poly):
    """Point-to-polygon form factor by Lambert's contour integral:
    F = 1/(2 pi) |sum_k angle(R_k, R_k+1) * (n . unit(R_k x R_k+1))|."""
    R = poly - p
    tot = 0.0
    for k in range(len(R)):
        a, b = R[k], R[(k + 1) % len(R)]
        g = np.cross(a, b)
        gl = np.linalg.norm(g)
        if gl == 0:
            continue
        ang = np.arccos(np.clip(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)), -1, 1))
        tot += ang * (n @ (g / gl))
    return abs(tot) / (2 * np.pi)


def _occluder_setup(level=4, center=(0.0, 0.2, 0.0), recv=(0.5, -1.0, 0.0)):
    v, f = meshes.icosphere(level)
    v = v + np.array(center)
    p = np.array(recv)
    n = np.array([0.0, 1.0, 0.0])
    return v, f, p, n


def test_lambert_formula_matches_sphere():
    """The polygon formula summed over the front faces of a fine icosphere is
    close to the sphere's closed form (R/d)^2 cos(beta)."""
    v, f, p, n = _occluder_setup(level=5)
    tri = v[f]
    nf = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    front = ((tri[:, 0] - p) * nf).sum(-1) < 0
    F = sum(lambert_form_factor(p, n, t) for t in tri[front])
    c = np.array([0.0, 0.2, 0.0])
    d = np.linalg.norm(c - p)
    F_sphere = (1.0 / d) ** 2 * ((c - p) @ n / d)
    assert abs(F - F_sphere) < 0.01 * F_sphere


@pytest.mark.parametrize("tau", [1.0, 0.5])
def test_lambert_occluder_expectation(tau):
    v, f, p, n = _occluder_setup(level=3)
    N, spp = 4096, 16
    eps = 1e-4
    L0 = np.array([1.0, 2.0, 0.5])
    env = np.ones((16, 32, 3), np.float32) * L0.astype(np.float32)
    m = 0.3
    korm = np.tile([1.0, 0.5, m], (N, 1))
    w = from_arrays("occluder", v, f, env, np.tile(p, (N, 1)), np.tile(n, (N, 1)),
                    np.full((N, 3), 0.5), korm, eye=np.array([3.0, 2.0, 1.0]), spp=spp,
                    ray_eps=eps, tau=tau)
    o = oracle.shade(w)
    # form factor of the mesh actually traced, seen from the ray origin
    origin = (p.astype(np.float32).astype(np.float64) + eps * n)
    vv = w.verts.astype(np.float64)
    tri = vv[w.tris]
    nf = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    front = ((tri[:, 0] - origin) * nf).sum(-1) < 0
    F = sum(lambert_form_factor(origin, n, t) for t in tri[front])
    expect = (1 - m) * L0 * (1 - tau * F)
    est = o["c_d"].mean(1)
    se = o["c_d"].std(1, ddof=1) / np.sqrt(N)
    assert np.all(np.abs(est - expect) < 4 * se), (est, expect, se)
    # rays passing within the tolerance of an edge are undecided: rare
    assert o["info"][:, 1].sum() < 1e-3 * N * spp


def test_blocked_directions_carry_no_radiance():
    """With tau = 1 a direction the occluder blocks carries no radiance
    (appendix A: the incident radiance is the probe's times H, H = 0 on
    blocked directions), whatever the probe holds there: BSDF-only estimates
    with infinite radiance in probe texels that the occluder covers entirely
    equal those with finite radiance, bit for bit.  With tau = 0.5 the
    infinity shows."""
    v, f, p, n, env, env_inf = occluder_with_hidden_infinity()
    N, spp = 256, 16
    korm = np.tile([1.0, 0.5, 0.3], (N, 1))

    def run(e, tau):
        w = from_arrays("occluder", v, f, e, np.tile(p, (N, 1)), np.tile(n, (N, 1)), np.full((N, 3), 0.5), korm,
                        eye=np.array([3.0, 2.0, 1.0]), spp=spp, ray_eps=1e-4, tau=tau)
        return oracle.shade(w, flags=oracle.LIGHT_OFF)

    a, b = run(env, 1.0), run(env_inf, 1.0)
    for k in ("c_d", "c_s"):
        assert np.all(np.isfinite(b[k]))
        assert np.array_equal(a[k], b[k]), k
    assert not np.all(np.isfinite(run(env_inf, 0.5)["c_d"]))


# ---------------------------------------------------------------------------
# quadrature convergence
# ---------------------------------------------------------------------------
def _sphere_dirs(H, W, S):
    """Midpoint nodes S x S per probe texel and their solid-angle weights."""
    v = (np.arange(H * S) + 0.5) / (H * S)
    u = (np.arange(W * S) + 0.5) / (W * S)
    V, U = np.meshgrid(v, u, indexing="ij")
    th, ph = np.pi * V, 2 * np.pi * U
    d = np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], -1).reshape(-1, 3)
    wt = (2 * np.pi ** 2 * np.sin(th) / (H * S * W * S)).reshape(-1)
    return d, wt


TECHNIQUES = {"mis": 0, "bsdf": oracle.LIGHT_OFF, "light": oracle.BSDF_OFF,
              "cosine": oracle.LIGHT_OFF | oracle.FORCE_COS, "ggx": oracle.LIGHT_OFF | oracle.FORCE_GGX}


@pytest.mark.parametrize("tech", sorted(TECHNIQUES))
@pytest.mark.parametrize("pix_sel", [0, 1, 2])
def test_mc_converges_to_quadrature(pix_sel, tech):
    """Every technique subset of the sampling ablation (cosine, BSDF, light,
    GGX alone, and MIS) is an unbiased estimator of the same integral."""
    w = make_workload("tiny")
    valid = np.nonzero((w.mask > 0) & (w.korm[1] > 0.35))[0]
    pix = valid[[len(valid) // 5, len(valid) // 2, (4 * len(valid)) // 5][pix_sel]]
    sc = oracle.Scene(w.verts, w.tris)
    tab = oracle.EnvTables(w.env)
    d, wt = _sphere_dirs(w.env.shape[0], w.env.shape[1], 24)
    gd, gs = oracle.integrand(w, pix, d, scene=sc, tables=tab, brute=False)
    quad_d = (gd * wt[:, None]).sum(0)
    quad_s = (gs * wt[:, None]).sum(0)
    # replicate the pixel: independent Philox streams per copy
    N, spp = 8192, 8
    col = lambda a: np.tile(a[:, pix], (N, 1))  # noqa: E731
    rep = from_arrays("rep", w.verts, w.tris, w.env, col(w.pos), col(w.nrm), col(w.kd), col(w.korm),
                      eye=w.eye[0], spp=spp, ray_eps=w.ray_eps, tau=w.tau)
    o = oracle.shade(rep, scene=sc, tables=tab, flags=TECHNIQUES[tech])
    for est, quad in ((o["c_d"], quad_d), (o["c_s"], quad_s)):
        mean = est.mean(1)
        se = est.std(1, ddof=1) / np.sqrt(N)
        assert np.all(np.abs(mean - quad) < 4 * se + 2e-3 * np.abs(quad)), (mean, quad, se)
        # and the error shrinks like 1/sqrt(N): half the copies, ~sqrt(2) larger SE
        se_half = est[:, : N // 4].std(1, ddof=1) / np.sqrt(N // 4)
        assert np.all(se_half > 1.5 * se) and np.all(se_half < 2.6 * se)


# ---------------------------------------------------------------------------
# gradients: analytic backward vs frozen-sample central differences
# ---------------------------------------------------------------------------
def _grad_setup():
    # its own generator: the same pixels whatever ran before
    rng = np.random.Generator(np.random.PCG64(1186))
    w = make_workload("tiny")
    valid = np.nonzero((w.mask > 0) & (w.korm[1] > 0.12))[0]
    pix = rng.choice(valid, 96, replace=False)
    n = len(pix)
    Ud = rng.normal(size=(3, n))
    Us = rng.normal(size=(3, n))
    return w, pix, Ud, Us


def _loss(o, Ud, Us):
    return (Ud * o["c_d"]).sum(0) + (Us * o["c_s"]).sum(0)


@pytest.mark.parametrize("field,ch", [("kd", 0), ("kd", 2), ("korm", 1), ("korm", 2), ("korm", 0),
                                      ("nrm", 0), ("nrm", 1), ("nrm", 2)])
def test_backward_matches_frozen_fd(field, ch):
    w, pix, Ud, Us = _grad_setup()
    sc = oracle.Scene(w.verts, w.tris)
    tab = oracle.EnvTables(w.env)
    g = oracle.shade(w, pixels=pix, scene=sc, tables=tab, grad=True, u_d=Ud, u_s=Us)
    gkey = {"kd": "g_kd", "korm": "g_korm", "nrm": "g_nrm"}[field]
    an = g[gkey][ch]
    eps = 1e-5
    res = []
    for sgn in (1, -1):
        arr = getattr(w, field).astype(np.float64).copy()
        arr[ch, pix] += sgn * eps
        # the perturbation is applied on the evaluation side only
        o = oracle.shade(w, pixels=pix, scene=sc, tables=tab,
                         eval_override={field: arr.astype(np.float32)})
        res.append(_loss(o, Ud, Us))
    # float32 storage of the perturbed input: use the realised step
    arr_p = getattr(w, field).astype(np.float64).copy()
    h_p = (arr_p[ch, pix] + eps).astype(np.float32).astype(np.float64) - arr_p[ch, pix]
    h_m = arr_p[ch, pix] - (arr_p[ch, pix] - eps).astype(np.float32).astype(np.float64)
    fd = (res[0] - res[1]) / (h_p + h_m)
    scale = np.abs(an).max() + 1e-12
    assert np.allclose(an, fd, rtol=2e-3, atol=2e-4 * scale), np.abs(an - fd).max() / scale


def test_backward_fd_float64_inputs_tight():
    """Same check with a float64-exact perturbation path: perturb a roughness
    value that is exactly representable so the FD step is exact, and ask for
    1e-6 relative agreement away from kinks."""
    w, pix, Ud, Us = _grad_setup()
    sc = oracle.Scene(w.verts, w.tris)
    tab = oracle.EnvTables(w.env)
    g = oracle.shade(w, pixels=pix, scene=sc, tables=tab, grad=True, u_d=Ud, u_s=Us)
    h = 2.0 ** -12
    res = []
    for sgn in (1, -1):
        arr = w.kd.copy()
        arr[1, pix] = (arr[1, pix] + np.float32(sgn * h)).astype(np.float32)
        o = oracle.shade(w, pixels=pix, scene=sc, tables=tab, eval_override={"kd": arr})
        res.append(_loss(o, Ud, Us))
    step = (w.kd[1, pix].astype(np.float64) + h) - (w.kd[1, pix].astype(np.float64) - h)
    fd = (res[0] - res[1]) / step
    # c_s is affine in kd (Schlick), so central differences are exact up to rounding
    assert np.allclose(g["g_kd"][1], fd, rtol=1e-8, atol=1e-12)


def test_env_gradient_matches_fd():
    """The estimator is linear in each texel under frozen sampling, so the
    texel gradient equals a finite difference exactly (up to rounding)."""
    w, pix, Ud, Us = _grad_setup()
    sc = oracle.Scene(w.verts, w.tris)
    tab = oracle.EnvTables(w.env)
    g = oracle.shade(w, pixels=pix, scene=sc, tables=tab, grad=True, u_d=Ud, u_s=Us)
    ge = g["g_env"]
    top = np.argsort(-np.abs(ge).reshape(-1))[:12]
    h = 0.25
    for flat in top:
        i, j, c = np.unravel_index(flat, ge.shape)
        vals, xs = [], []
        for sgn in (1, -1):
            e2 = w.env.copy()
            e2[i, j, c] += np.float32(sgn * h)
            xs.append(float(e2[i, j, c]))
            o = oracle.shade(w, pixels=pix, scene=sc, tables=tab, env_eval=e2)
            vals.append(_loss(o, Ud, Us).sum())
        fd = (vals[0] - vals[1]) / (xs[0] - xs[1])
        assert abs(fd - ge[i, j, c]) <= 1e-9 * max(1.0, abs(fd)), (fd, ge[i, j, c])
    assert np.all(g["s_env"] >= np.abs(ge) - 1e-15)


def test_occlusion_channel_has_no_effect():
    w, pix, Ud, Us = _grad_setup()
    a = oracle.shade(w, pixels=pix)
    k2 = w.korm.copy()
    k2[0] = RNG.random(k2.shape[1])
    b = oracle.shade(w, pixels=pix, eval_override={"korm": k2})
    assert np.array_equal(a["c_d"], b["c_d"]) and np.array_equal(a["c_s"], b["c_s"])


# ---------------------------------------------------------------------------
# exact identities
# ---------------------------------------------------------------------------
def test_probe_linearity_bitwise():
    w = make_workload("tiny")
    a = oracle.shade(w)
    w2 = make_workload("tiny")
    w2.env = (w2.env * 2).astype(np.float32)
    b = oracle.shade(w2)
    assert np.array_equal(2 * a["c_d"], b["c_d"]) and np.array_equal(2 * a["c_s"], b["c_s"])
    assert np.array_equal(a["hitbits"], b["hitbits"])


def test_tau_zero_equals_empty_scene():
    w = make_workload("tiny")
    a = oracle.shade(w, tau=0.0)
    v, f = _empty_mesh()
    b = oracle.shade(w, scene=oracle.Scene(v, f), tau=1.0)
    assert np.array_equal(a["c_d"], b["c_d"]) and np.array_equal(a["c_s"], b["c_s"])
    assert not a["hitbits"].any()


def test_invalid_pixels_are_zero():
    w = make_workload("tiny")
    pos = w.pos.copy()
    nrm = w.nrm.copy()
    valid = np.nonzero(w.mask)[0]
    pos[0, valid[0]] = np.nan
    nrm[:, valid[1]] = 0.0
    w.pos, w.nrm = pos, nrm
    o = oracle.shade(w, grad=True, u_d=np.ones((3, w.n_pixels)), u_s=np.ones((3, w.n_pixels)))
    for k in ("c_d", "c_s", "g_kd", "g_korm", "g_nrm"):
        assert np.all(o[k][:, w.mask == 0] == 0)
        assert np.all(o[k][:, valid[:2]] == 0)
    assert o["nonfinite"] == 1


def test_decisions_and_hitbits_consistent():
    w = make_workload("tiny")
    o = oracle.shade(w, want_decisions=True)
    dec = o["decisions"]
    hb = o["hitbits"][:, 0]
    for s in range(w.spp):
        fl = dec[:, s, 2]
        for tech, bit in ((0, oracle.DEC_L_HIT), (1, oracle.DEC_B_HIT)):
            assert np.array_equal(((hb >> (2 * s + tech)) & 1) != 0, (fl & bit) != 0)
    valid = w.mask > 0
    assert np.all((dec[valid, :, 2] & oracle.DEC_VALID) != 0)
    assert np.all(dec[~valid, :, 0] == oracle.DEC_NONE)


def _views(w, v0, v1, view_base):
    """The workload's views v0..v1-1 on their own, numbered from view_base."""
    import dataclasses
    hw = w.height * w.width
    sl = slice(v0 * hw, v1 * hw)
    return dataclasses.replace(w, n_views=v1 - v0, pos=w.pos[:, sl].copy(), nrm=w.nrm[:, sl].copy(),
                               kd=w.kd[:, sl].copy(), korm=w.korm[:, sl].copy(), mask=w.mask[sl].copy(),
                               eye=w.eye[v0:v1].copy(), view_base=view_base, depth=None)


def test_view_base_is_the_global_view_id():
    """Views 6 and 7 of an 8-view render, rendered on their own with
    view_base = 6, give the same values bit for bit: the counter's second
    word is the global view id.  With view_base = 0 instead they draw other
    samples."""
    w = make_workload("sphere8", H=16, W=16, n_views=8, spp=4)
    hw = 16 * 16
    full = oracle.shade(w)
    part = oracle.shade(_views(w, 6, 8, 6))
    other = oracle.shade(_views(w, 6, 8, 0))
    for key in ("c_d", "c_s"):
        assert np.array_equal(full[key][:, 6 * hw:], part[key])
        assert not np.array_equal(part[key], other[key])
    assert np.array_equal(full["hitbits"][6 * hw:], part["hitbits"])


def test_largest_spp_keeps_the_sample_sequence():
    """spp = 1024 (the library's largest): sample s draws from counter s
    whatever spp is, so the first 512 samples' decisions and hit words equal
    those of spp = 512; every hit bit, up to word 63, agrees with its sample's
    decision; spp = 1025 is rejected."""
    w = make_workload("tiny", H=12, W=12)
    a = oracle.shade(w, spp=1024, want_decisions=True)
    b = oracle.shade(w, spp=512, want_decisions=True)
    assert a["hitbits"].shape[1] == 64
    assert np.array_equal(a["decisions"][:, :512], b["decisions"])
    assert np.array_equal(a["hitbits"][:, :32], b["hitbits"])
    dec, hb = a["decisions"], a["hitbits"]
    for s in range(1024):
        fl = dec[:, s, 2]
        word = hb[:, s // 16]
        for tech, bit in ((0, oracle.DEC_L_HIT), (1, oracle.DEC_B_HIT)):
            assert np.array_equal(((word >> (2 * s % 32 + tech)) & 1) != 0, (fl & bit) != 0)
    assert (hb[:, 32:] != 0).any()
    with pytest.raises(ValueError):
        oracle.shade(w, spp=1025)


def test_brute_force_equals_bvh_render():
    w = make_workload("tiny")
    a = oracle.shade(w)
    b = oracle.shade(w, brute=True)
    assert np.array_equal(a["c_d"], b["c_d"]) and np.array_equal(a["hitbits"], b["hitbits"])


# ---------------------------------------------------------------------------
# tolerance quantities the oracle reports beside its outputs
# ---------------------------------------------------------------------------
def test_abs_sums_and_direction_conditioning():
    """Per output, the sum of the summands' magnitudes bounds the value (and
    equals it where every summand is positive: the values under a positive
    probe); without a direction model no conditioning is reported, with one
    it scales linearly with the model's counts."""
    from workloads import upstream_grads
    w = make_workload("tiny", H=32, W=32)
    ud, us = upstream_grads(w)
    base = dict(grad=True, u_d=ud.astype(np.float64), u_s=us.astype(np.float64))
    o0 = oracle.shade(w, **base)
    for k in ("c_d", "c_s", "g_kd", "g_korm", "g_nrm"):
        assert np.all(o0[k + "_abs"] >= np.abs(o0[k]) * (1 - 1e-12))
        assert np.all(o0[k + "_cond"] == 0.0)
    for k in ("c_d", "c_s"):
        assert np.allclose(o0[k + "_abs"], np.abs(o0[k]), rtol=1e-12, atol=0)
    counts = {"light": 32, "cos": 16, "ggx0": 16, "ggx1": 16, "arg": 16}
    o1 = oracle.shade(w, tol=oracle.Tolerances(dir=counts), **base)
    o2 = oracle.shade(w, tol=oracle.Tolerances(dir={k: 2 * v for k, v in counts.items() if k != "arg"} |
                                               {"arg": 16}), **base)
    for k in ("c_d", "c_s", "g_kd", "g_nrm"):
        assert np.array_equal(o1[k], o0[k])
        c1, c2 = o1[k + "_cond"], o2[k + "_cond"]
        assert (c1 > 0).mean() > 0.5
        assert np.allclose(c2, 2 * c1, rtol=1e-9, atol=1e-300)
    assert np.all(o1["c_env"] >= 0) and o1["c_env"].max() > 0

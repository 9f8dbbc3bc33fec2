"""Pins of the FP64 oracle against things other than itself.

Each test names what it pins: a library routine (rocRAND's Philox), a closed
form (white furnace, Lambert's polygon form factor, GGX normalisation), a
dense quadrature of the integral the estimator targets, brute force on small
inputs, exact identities (linearity in the probe) and frozen-sample finite
differences of the estimator's own value.
"""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from workloads import make_workload
from workloads import meshes

RNG = np.random.Generator(np.random.PCG64(20220607))


# ---------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's independent implementation
# ---------------------------------------------------------------------------
ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand():
    """Raw Philox4x32-10 blocks equal rocRAND's engine output bit for bit
    (rocRAND's counter = (offset/4 as 64 bits, subsequence as 64 bits))."""
    n = 2000
    ctr = RNG.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] &= (1 << 30) - 1          # keep 4*offset inside 64 bits
    ctr[:8] = 0
    ctr[8:16, 1] = 0
    keys = RNG.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    keys[:4] = 0
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "rr.hip")
        exe = os.path.join(d, "rr")
        open(src, "w").write(ROCRAND_PROG)
        subprocess.check_call(["hipcc", "--offload-host-only", "-O1", "-o", exe, src])
        inp = "\n".join(" ".join(str(int(x)) for x in list(c) + list(k)) for c, k in zip(ctr, keys))
        res = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in res.strip().splitlines()], np.uint64)
    mine = np.stack([oracle.philox(c, k)[0] for c, k in zip(ctr, keys)]).astype(np.uint64)
    assert mine.shape == ref.shape
    assert np.array_equal(mine, ref)


def test_uniforms_are_24bit_grid():
    """xi = (x >> 8) 2^-24: in [0,1), on the 2^-24 grid, uniform (KS) and the
    two blocks of a sample differ in the last counter word only."""
    n = 200000
    pix = RNG.integers(0, 2**20, n)
    xi = oracle.uniforms(0, pix, np.zeros(n), RNG.integers(0, 64, n))
    assert xi.min() >= 0.0 and xi.max() < 1.0
    assert np.all(xi * 2**24 == np.floor(xi * 2**24))
    for k in range(8):
        s = np.sort(xi[:, k])
        ks = np.max(np.abs(s - (np.arange(n) + 0.5) / n))
        assert ks < 1.63 / np.sqrt(n) * 1.5
    raw = oracle.philox(np.array([[5, 3, 7, 0], [5, 3, 7, 1]]), [11, 0])
    xi2 = oracle.uniforms(11, [5], [3], [7])[0]
    assert np.array_equal(xi2 * 2**24, np.concatenate([raw[0] >> 8, raw[1] >> 8]).astype(np.float64))


# ---------------------------------------------------------------------------
# probe sampling tables
# ---------------------------------------------------------------------------
def _env(H=16, W=32, seed=3):
    r = np.random.Generator(np.random.PCG64(seed))
    e = r.lognormal(0, 1.0, size=(H, W, 3)).astype(np.float32)
    e[3:5, 10:12] *= 50
    e[H - 2, :] = 0.0          # an all-black row: zero-width marginal bin
    e[5, 3:9] = 0.0            # zero-width conditional bins
    return e


def test_env_tables_invariants():
    t = oracle.EnvTables(_env())
    assert t.light_enabled
    assert t.marg[0] == 0.0 and t.marg[-1] == 1.0
    assert np.all(np.diff(t.marg) >= 0)
    assert np.all(t.cond[:, 0] == 0.0) and np.all(t.cond[:, -1] == 1.0)
    assert np.all(np.diff(t.cond, axis=1) >= 0)
    # black row keeps a uniform conditional CDF and zero pdf
    H, W = t.H, t.W
    assert np.allclose(t.cond[H - 2], np.arange(W + 1) / W)
    assert np.all(t.pdf[H - 2] == 0)
    # pdf table integrates to 1 over (u, v)
    assert abs(t.pdf.astype(np.float64).sum() / (H * W) - 1.0) < 1e-6


def test_env_tables_negative_texels_and_edge_ties():
    """Negative texels weigh 0 (zero density, flat CDF steps).  With the
    first row and the first column black, the first bins have zero width:
    xi = 0 and xi equal to any table entry must still select a texel of
    positive density (the search takes the largest k with cdf[k] <= xi)."""
    e = _env()
    e[0] = 0.0
    e[:, 0] = 0.0
    e[7, 5] = -2.0
    e[8, 9] = np.float32(-1e-3)
    t = oracle.EnvTables(e)
    H, W = t.H, t.W
    assert t.pdf[7, 5] == 0 and t.pdf[8, 9] == 0
    assert np.all(t.pdf[0] == 0) and np.all(t.pdf[:, 0] == 0)
    assert np.all(np.diff(t.cond, axis=1) >= 0) and np.all(np.diff(t.marg) >= 0)
    xi0 = np.unique(np.concatenate([[0.0], t.marg[:-1].astype(np.float64)]))
    xi1 = np.unique(np.concatenate([[0.0], t.cond[:, :-1].astype(np.float64).ravel()]))
    a, b = np.meshgrid(xi0, xi1, indexing="ij")
    w, p, ti, tj = t.sample(a.ravel(), b.ravel())
    assert np.all(t.pdf[ti, tj] > 0) and np.all(p > 0)
    # and the same on random uniforms of the 24-bit grid
    u = np.floor(RNG.random((2, 100_000)) * 2 ** 24) / 2 ** 24
    w, p, ti, tj = t.sample(u[0], u[1])
    assert np.all(t.pdf[ti, tj] > 0)


def test_env_tables_zero_env_disables_light():
    t = oracle.EnvTables(np.zeros((8, 16, 3), np.float32))
    assert not t.light_enabled and t.total == 0.0
    assert np.all(t.pdf == 0)
    assert np.allclose(t.marg, np.arange(9) / 8)


def test_env_tables_scale_invariant():
    """Doubling the probe leaves every table entry bit-identical."""
    e = _env()
    a, b = oracle.EnvTables(e), oracle.EnvTables(2 * e)
    assert np.array_equal(a.cond, b.cond) and np.array_equal(a.marg, b.marg)
    assert np.array_equal(a.pdf, b.pdf)


def test_light_sampler_chi_square():
    """Texel frequencies of the light sampler match w_ij / sum(w), with
    w = max(0, (r+g+b)/3) * sin(theta at the row centre)."""
    e = _env()
    t = oracle.EnvTables(e)
    H, W = t.H, t.W
    n = 2_000_000
    w, p, ti, tj = t.sample(RNG.random(n), RNG.random(n))
    counts = np.bincount(ti * W + tj, minlength=H * W).astype(np.float64)
    y = np.maximum(e.astype(np.float64).sum(-1) / 3, 0)
    wt = y * np.sin(np.pi * (np.arange(H) + 0.5) / H)[:, None]
    expect = (wt / wt.sum()).reshape(-1) * n
    assert counts[expect == 0].sum() == 0
    m = expect > 20
    chi2 = ((counts[m] - expect[m]) ** 2 / expect[m]).sum()
    dof = m.sum() - 1
    assert chi2 < dof + 6 * np.sqrt(2 * dof)
    # the sampled direction lies in the sampled texel and its density is the
    # texel density over 2 pi^2 sin(theta)
    ti2, tj2, marg = t.texel_of_dir(w)
    ok = marg > 1e-9
    assert np.all(ti2[ok] == ti[ok]) and np.all(tj2[ok] == tj[ok])
    assert np.allclose(t.pdf_dir(w[ok]), p[ok], rtol=1e-12)


def test_light_pdf_normalised_on_sphere():
    """Integral of p_light over the sphere = 1 (midpoint rule on a grid 8x
    finer than the texels, d omega = sin(theta) dtheta dphi)."""
    t = oracle.EnvTables(_env())
    H, W = t.H, t.W
    S = 8
    th = (np.arange(H * S) + 0.5) * np.pi / (H * S)
    ph = (np.arange(W * S) + 0.5) * 2 * np.pi / (W * S)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.cos(TH), np.sin(TH) * np.sin(PH)], -1).reshape(-1, 3)
    p = t.pdf_dir(d)
    integral = (p * np.sin(TH).reshape(-1)).sum() * (np.pi / (H * S)) * (2 * np.pi / (W * S))
    assert abs(integral - 1.0) < 1e-6


# ---------------------------------------------------------------------------
# BSDF sampling densities
# ---------------------------------------------------------------------------
def _hemi_grid(n_th, n_ph, alpha=None):
    """Quadrature nodes/weights over the upper hemisphere; theta spacing is
    warped toward the pole for peaked lobes (tan(theta) = alpha * tan(pi t/2))."""
    t = (np.arange(n_th) + 0.5) / n_th
    if alpha is None:
        th = t * np.pi / 2
        dth = np.full(n_th, np.pi / 2 / n_th)
    else:
        x = np.tan(np.pi * t / 2)
        th = np.arctan(alpha * x)
        dth = alpha * (np.pi / 2) / np.cos(np.pi * t / 2) ** 2 / (1 + (alpha * x) ** 2) / n_th
    ph = (np.arange(n_ph) + 0.5) * 2 * np.pi / n_ph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    wts = (np.sin(th) * dth)[:, None] * (2 * np.pi / n_ph) * np.ones_like(PH)
    d = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    return d.reshape(-1, 3), wts.reshape(-1)


@pytest.mark.parametrize("alpha", [0.0064, 0.1, 0.5, 1.0])
def test_ggx_D_normalised(alpha):
    """Integral over the hemisphere of D(h) (n.h) dh = 1 (Walter et al.)."""
    h, wt = _hemi_grid(4000, 8, alpha)
    s2 = h[:, 0] ** 2 + h[:, 1] ** 2
    D, _ = oracle.ggx(h[:, 2], s2, np.full(len(h), 0.5), alpha)
    assert abs((D * h[:, 2] * wt).sum() - 1.0) < 1e-6


@pytest.mark.parametrize("alpha", [0.0064, 0.05, 0.3, 1.0])
@pytest.mark.parametrize("theta_o", [0.0, 0.4, 1.2, 1.55])
def test_ggx_pdf_weak_white_furnace(alpha, theta_o):
    """The VNDF reflection density G1(v) D(h) / (4 n.v) integrates to 1 over
    the whole sphere of directions (weak white furnace, Heitz 2014/2018).
    Integrated in half-vector space with the reflection Jacobian 4 (v.h)."""
    V = np.array([np.sin(theta_o), 0.0, np.cos(theta_o)])
    h, wt = _hemi_grid(3000, 720, alpha)
    vh = h @ V
    L = 2 * vh[:, None] * h - V
    p = oracle.pdf_ggx_local(V, alpha, L)
    integral = (p * 4 * np.maximum(vh, 0) * wt)[vh > 0].sum()
    assert abs(integral - 1.0) < 2e-4


def test_cos_pdf_normalised():
    d, wt = _hemi_grid(2000, 64)
    assert abs((oracle.pdf_cos_local(d) * wt).sum() - 1.0) < 1e-6


def _chi2_sphere(samples, pdf_fn, nb_t=24, nb_p=48, sub=6):
    """Chi-square of samples in equal-solid-angle bins (uniform in cos(theta)
    and phi) against the bin integrals of pdf_fn (sub x sub midpoint rule)."""
    n = len(samples)
    ct = np.clip(samples[:, 2], -1, 1)
    ph = np.mod(np.arctan2(samples[:, 1], samples[:, 0]), 2 * np.pi)
    bi = np.minimum(((1 - ct) / 2 * nb_t).astype(int), nb_t - 1)
    bj = np.minimum((ph / (2 * np.pi) * nb_p).astype(int), nb_p - 1)
    counts = np.bincount(bi * nb_p + bj, minlength=nb_t * nb_p).astype(np.float64)
    u = (np.arange(nb_t * sub) + 0.5) / (nb_t * sub)
    v = (np.arange(nb_p * sub) + 0.5) / (nb_p * sub)
    U, Vv = np.meshgrid(u, v, indexing="ij")
    cth = 1 - 2 * U
    sth = np.sqrt(np.maximum(0, 1 - cth ** 2))
    phi = 2 * np.pi * Vv
    d = np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], -1).reshape(-1, 3)
    p = pdf_fn(d).reshape(nb_t * sub, nb_p * sub) * (4 * np.pi / (nb_t * sub * nb_p * sub))
    expect = p.reshape(nb_t, sub, nb_p, sub).sum(axis=(1, 3)).reshape(-1) * n
    m = expect > 20
    chi2 = ((counts[m] - expect[m]) ** 2 / expect[m]).sum()
    dof = m.sum() - 1
    return chi2, dof, counts[~m].sum(), expect[~m].sum()


@pytest.mark.parametrize("alpha,theta_o", [(0.2, 0.3), (0.5, 1.0), (1.0, 0.0), (0.35, 1.4)])
def test_vndf_sampler_matches_pdf(alpha, theta_o):
    """Histogram of visible-normal samples agrees with the closed-form density
    (a right density with a wrong warp fails here)."""
    V = np.array([np.sin(theta_o), 0.0, np.cos(theta_o)])
    n = 1_000_000
    L = oracle.sample_vndf_local(V, alpha, RNG.random(n), RNG.random(n))
    assert np.allclose(np.linalg.norm(L, axis=1), 1.0, atol=1e-12)
    chi2, dof, c_lo, e_lo = _chi2_sphere(L, lambda d: oracle.pdf_ggx_local(V, alpha, d))
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)
    # sparse bins (incl. those cut by the support boundary h.n = 0, where the
    # midpoint rule is coarse) hold the same small mass
    assert abs(c_lo - e_lo) < 6 * np.sqrt(e_lo + 20) + 1e-3 * n


def test_cos_sampler_matches_pdf():
    n = 1_000_000
    L = oracle.sample_cos_local(RNG.random(n), RNG.random(n))
    chi2, dof, _, _ = _chi2_sphere(L, oracle.pdf_cos_local)
    assert chi2 < dof + 6 * np.sqrt(2 * dof)


# ---------------------------------------------------------------------------
# visibility
# ---------------------------------------------------------------------------
def test_visibility_bvh_equals_brute_force():
    w = make_workload("sphere8", H=8, W=8, n_views=1, freq=12)
    sc = oracle.Scene(w.verts, w.tris)
    n = 20000
    o = RNG.uniform(-3, 3, size=(n, 3))
    d = RNG.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for da, dr in [(0.0, 0.0), (1e-5, 1e-5), (1e-3, 0.0)]:
        a = sc.anyhit(o, d, da, dr, brute=False)
        b = sc.anyhit(o, d, da, dr, brute=True)
        assert np.array_equal(a, b)
    assert 0.05 < (a == oracle.TRI_HIT).mean() < 0.95


def test_visibility_triangle_straddling_the_origin_plane():
    """A triangle with vertices on both sides of the plane through the ray
    origin: (-1,-1,-10), (1,-1,2), (0,1,5).  The line x = y = 0 meets it at
    barycentric weights (1/4, 1/4, 1/2), so at z = 0.5 (plane geometry).
    Rays along +z hit it from below z = 0.5 and miss from above; rays along
    -z do the opposite."""
    V = np.array([[-1.0, -1.0, -10.0], [1.0, -1.0, 2.0], [0.0, 1.0, 5.0]])
    sc = oracle.Scene(V.astype(np.float32), np.array([[0, 1, 2]], np.int32))
    zs = np.array([-3.0, 0.0, 0.4, 0.6, 1.0, 4.0])
    o = np.stack([np.zeros_like(zs), np.zeros_like(zs), zs], 1)
    up = np.tile([0.0, 0.0, 1.0], (len(zs), 1))
    hit_up = sc.anyhit(o, up, 1e-9, 1e-9)
    hit_down = sc.anyhit(o, -up, 1e-9, 1e-9)
    below = zs < 0.5
    assert np.all((hit_up == oracle.TRI_HIT) == below) and np.all((hit_up == oracle.TRI_MISS) == ~below)
    assert np.all((hit_down == oracle.TRI_HIT) == ~below) and np.all((hit_down == oracle.TRI_MISS) == below)


def test_visibility_closed_mesh_geometry():
    """Rays from outside a closed icosphere aimed inside its inscribed ball
    hit; rays aimed away miss; rays from the centre always hit (a centre ray
    that crosses the mesh within the tolerance of an edge is undecided)."""
    rng = np.random.Generator(np.random.PCG64(282))
    v, f = meshes.icosphere(3)
    sc = oracle.Scene(v, f)
    n = 5000
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    o = 3.0 * dirs
    tgt = rng.normal(size=(n, 3))
    tgt = 0.9 * tgt / np.linalg.norm(tgt, axis=1, keepdims=True) * rng.random((n, 1))
    into = tgt - o
    assert np.all(sc.anyhit(o, into, 1e-6, 1e-6) == oracle.TRI_HIT)
    assert np.all(sc.anyhit(o, dirs, 1e-6, 1e-6) == oracle.TRI_MISS)
    rc = sc.anyhit(np.zeros((n, 3)), dirs, 1e-6, 1e-6)
    assert np.all(rc != oracle.TRI_MISS) and np.mean(rc == oracle.TRI_HIT) > 0.99
    # a ray through a shared vertex or edge is undecided, never a robust miss
    r = sc.anyhit(np.array([[0, 0, 0.0]]), v[:1] * 2.0, 1e-6, 1e-6)
    assert r[0] in (oracle.TRI_HIT, oracle.TRI_NEAR)


def test_visibility_triangle_edge_margins():
    tri_v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    sc = oracle.Scene(tri_v, np.array([[0, 1, 2]], np.int32))
    d = np.array([[0, 0, -1.0]])
    cases = [((0.25, 0.25, 1), oracle.TRI_HIT), ((0.5 + 1e-3, 0.5 + 1e-3, 1), oracle.TRI_MISS),
             ((0.5, 0.5 + 1e-8, 1), oracle.TRI_NEAR), ((0.25, 0.25, -1), oracle.TRI_MISS),
             ((0.25, 0.25, 1e-9), oracle.TRI_NEAR), ((-1e-8, 0.3, 1), oracle.TRI_NEAR)]
    for o, want in cases:
        assert sc.anyhit(np.array([o], float), d, 1e-6, 1e-6)[0] == want, o

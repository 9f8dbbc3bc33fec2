"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, compare at the stated tolerance.

Tolerance of every per-pixel output (c_d, c_s and the gradients to kd, korm
and the normal), per channel and valid pixel:

    |gpu - oracle| <= REL_TOL * A + ABS_TOL * mean|oracle| + COND_K * cond + LERR_K * lerr

  A     the sum, over the pixel's samples, of the absolute values of the
        summands of each sample's term (`<name>_abs` from the oracle).  An FP32
        evaluation of a sum of products in any order is within a small
        multiple of u = 2^-24 times that sum (Higham); REL_TOL = 1e-4 is the
        target's relative tolerance and leaves room for ~1000 roundings.  For
        sums of like sign A = |oracle|, the plain 1e-4 relative bound.
  cond  the direction allowance (`<name>_cond`): for every sample,
        |gradient of its term over directions| times the sample's
        direction-error bound, summed.  The kernel samples each direction in
        FP32; the bound is the count of rounded operations of that sampling
        chain (DIR_COUNTS) times the amplification of the chain's square roots
        and normalisation at that sample, evaluated from the exact
        intermediates.  The gradient is a first-order sensitivity; COND_K = 2
        covers the linearisation.
  lerr  the bilinear lookup's own FP32 error (`<name>_lerr`, already a bound:
        LERR_K = 2); zero for the nearest texel.

Every comparison also reports the fraction of elements within the plain
bound 1e-4 |oracle| + 1e-6 mean|oracle| and the largest relative error over
elements above 1% of the mean magnitude.
"""

import numpy as np

import oracle

REL_TOL = 1e-4
ABS_TOL = 1e-6
COND_K = 2
LERR_K = 2
U = 2.0 ** -24

# Direction-error model of the kernel's FP32 sampling chains, in units of u
# (counts of rounded operations, each moving the direction by at most about
# one unit in the last place of an O(1) quantity):
#  light  the in-texel offsets (two differences and a quotient per
#         coordinate, plus the integer part: 4), the scaling to (u, v) (1),
#         sincospi of theta and phi (2 ulp each, i.e. 4 u), the two products of
#         the spherical coordinates (2), times pi and 2 pi of the angle
#         derivatives, and the local frame (3 rounded dot products of rounded
#         frame vectors): <= 32.
#  cos    sqrt of xi4 (2), sincospi of 2 pi xi5 (4), two products (2), the
#         exact 1 - xi4 and its sqrt (2), the world frame (3 fused sums of
#         rounded frame vectors: 3) and the normalisation (3): <= 16.
#  ggx0   the operations after the hemisphere point with unit gain: the
#         reflection 2 (v.n) n - v (5), the world frame (3 fused sums: 3) and
#         two normalisations (6): <= 16.
#  ggx1   the operations up to the un-stretched normal (sqrt, sincospi, the
#         products of the disk point, the blend, the three fused sums of the
#         rounded visible-normal frame, the stretch), whose error the
#         normalisation divides by |m| and the square roots amplify: <= 16.
#  arg    the absolute error of the square roots' arguments g = 1 - t1^2 and
#         h = 1 - t1^2 - t2^2 (two squares and two differences of O(1) terms,
#         with t2's own error): <= 16.
DIR_COUNTS = {"light": 32, "cos": 16, "ggx0": 16, "ggx1": 16, "arg": 16}
TOL = oracle.Tolerances(dir=DIR_COUNTS)


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_forward(w, scene=None, env=None, gb=None, spp=None, seed=None, tau=None, dump=True, flags=0):
    import torch
    import paper_2206_03380_amd as M
    dev = "cuda"
    if scene is None:
        scene = M.Scene(torch.from_numpy(w.verts).to(dev), torch.from_numpy(w.tris).to(dev))
    if env is None:
        env = M.Env(torch.from_numpy(w.env).to(dev))
    if gb is None:
        gb = M.GBuffer.from_workload(w, dev)
    spp = w.spp if spp is None else spp
    seed = w.seed if seed is None else seed
    tau = w.tau if tau is None else tau
    c_d, c_s, hb, dec = M.shade_fwd(scene, env, gb, spp, seed=seed, tau=tau, ray_eps=w.ray_eps,
                                    flags=flags, decisions="dirs" if dump else False)
    torch.cuda.synchronize()
    out = {"c_d": to_np(c_d), "c_s": to_np(c_s), "hitbits": to_np(hb).view(np.uint32),
           "decisions": None, "dirs": None}
    if dec is not None:
        d = to_np(dec).view(np.uint32)
        out["decisions"] = np.ascontiguousarray(d[..., :3])
        out["dirs"] = np.ascontiguousarray(d[..., 3:]).view(np.float32).reshape(d.shape[0], d.shape[1], 2, 3)
    return out, (scene, env, gb, hb)


def hitbits_per_pixel(hb_planar):
    """[words][N] -> [N][words]"""
    return np.ascontiguousarray(hb_planar.T)


def compare(gpu, o, key, valid, rel=REL_TOL, absf=ABS_TOL, med=None, name=None):
    """Compare a [3, n] kernel result with the oracle's `key` on the oracle's
    pixel list (elements `valid`).  Returns (ok, worst error / bound, report).
    med: also require the median relative error (over elements above 1% of
    the mean magnitude) to stay below med, so that an allowance widened for
    ill-conditioned elements cannot hide a systematic error."""
    g = gpu[:, valid].astype(np.float64)
    ref = o[key][:, valid]
    scale = np.abs(ref).mean(axis=1, keepdims=True)
    bound = (rel * o[key + "_abs"][:, valid] + absf * scale + COND_K * o[key + "_cond"][:, valid] +
             LERR_K * o[key + "_lerr"][:, valid])
    err = np.abs(g - ref)
    ok = err <= bound
    plain = REL_TOL * np.abs(ref) + ABS_TOL * scale
    frac_plain = float((err <= plain).mean()) if err.size else 1.0
    worst = float((err / np.maximum(bound, 1e-300)).max()) if err.size else 0.0
    big = np.abs(ref) > 1e-2 * scale
    rel_big = err[big] / np.abs(ref[big])
    max_rel = float(rel_big.max()) if rel_big.size else 0.0
    med_rel = float(np.median(rel_big)) if rel_big.size else 0.0
    rep = ("%s: within plain 1e-4 bound %.5f of %d, max rel (|o| > 1%% of mean) %.3g, median rel %.3g, "
           "max|err| %.3g, fail %d, worst/bound %.3g") % (
        name or key, frac_plain, ok.size, max_rel, med_rel, err.max() if err.size else 0.0, int((~ok).sum()), worst)
    good = bool(ok.all()) and (med is None or med_rel <= med)
    return good, worst, rep


def check_dirs(g_dirs, o_dirs, name=""):
    """Distance between the kernel's FP32 sampled directions and the
    oracle's FP64 ones against the oracle's per-sample bound (the direction
    model of DIR_COUNTS), over every sample both sides drew.  Returns (worst
    distance / bound, largest distance in units of u, samples compared)."""
    g = g_dirs.astype(np.float64)
    od, eb = o_dirs[..., :3], o_dirs[..., 3]
    both = np.isfinite(g).all(-1) & np.isfinite(od).all(-1)
    d = np.linalg.norm(g - od, axis=-1)[both]
    e = eb[both]
    if d.size == 0:
        return 0.0, 0.0, 0
    ratio = float((d / e).max())
    print("%s directions: %d samples, largest distance %.1f u, worst distance/bound %.3f, median bound %.1f u" % (
        name, d.size, d.max() / U, ratio, float(np.median(e)) / U))
    return ratio, float(d.max() / U), int(d.size)


def occluder_with_hidden_infinity(level=3, H=16, W=32, seed=31):
    """A unit icosphere at (0, 0.2, 0) over a receiver point at (0.5, -1, 0)
    (normal +y), a lognormal probe, and a copy of the probe with +inf in every
    texel whose corners all lie within 35 degrees of the direction to the
    sphere's centre (the sphere's angular radius there is 50 degrees), so that
    the receiver sees those texels only through the sphere.
    Returns (verts, tris, p, n, env, env_inf)."""
    from workloads import meshes
    v, f = meshes.icosphere(level)
    v = v + np.array([0.0, 0.2, 0.0])
    p = np.array([0.5, -1.0, 0.0])
    n = np.array([0.0, 1.0, 0.0])
    rng = np.random.Generator(np.random.PCG64(seed))
    env = rng.lognormal(0, 1, (H, W, 3)).astype(np.float32)
    c = np.array([0.0, 0.2, 0.0]) - p
    c /= np.linalg.norm(c)
    inside = np.zeros((H, W), bool)
    for i in range(H):
        for j in range(W):
            th = np.pi * np.array([i, i, i + 1, i + 1]) / H
            ph = 2 * np.pi * np.array([j, j + 1, j, j + 1]) / W
            d = np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], -1)
            inside[i, j] = np.all(d @ c > np.cos(np.radians(35.0)))
    assert inside.sum() >= 4
    env_inf = env.copy()
    env_inf[inside] = np.inf
    return v, f, p, n, env, env_inf


def big_tris(v, f):
    """The scene builder's big triangles, in its own FP32 operations: the
    triangle box's longest side times 8 at least the longest side of the
    bounds of the triangle centroids."""
    t = v[f].astype(np.float32)                                # [nt, 3, 3]
    cen = ((t[:, 0] + t[:, 1]) + t[:, 2]) * np.float32(1.0 / 3.0)
    cext = (cen.max(0) - cen.min(0)).max()
    side = (t.max(1) - t.min(1)).max(1)
    return side * np.float32(8.0) >= cext

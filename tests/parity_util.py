"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, compare at the stated tolerance."""

import numpy as np

# c_d, c_s and per-pixel gradients: |gpu - oracle| <= REL * |oracle| + ABS * mean|oracle|
# (per channel, valid pixels).  FP32 per-sample terms carry ~1e-6 relative
# error, and the sums run over 2*spp terms of like sign.
REL_TOL = 1e-4
ABS_TOL = 1e-6


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
                                    flags=flags, decisions=dump)
    torch.cuda.synchronize()
    out = {"c_d": to_np(c_d), "c_s": to_np(c_s), "hitbits": to_np(hb).view(np.uint32),
           "decisions": to_np(dec).view(np.uint32) if dec is not None else None}
    return out, (scene, env, gb, hb)


def hitbits_per_pixel(hb_planar):
    """[words][N] -> [N][words]"""
    return np.ascontiguousarray(hb_planar.T)


# Grazing samples: an absolute FP32 error of the sampled direction (<= 32u,
# with a factor 2 margin) changes a term by its log-derivative in n.l (<= 2)
# times that error over n.l; the oracle sums |term| u / (n.l) per output as
# `<name>_cond`, and the bound adds COND_K times it.
COND_K = 64


# The bilinear lookup adds an absolute bound of its own (`<name>_lerr`: the
# FP32 error of the texel coordinates through the reconstruction's slope, and
# the rounding of the tap sum), already a bound: the tolerance adds twice it.
LERR_K = 2


def compare(gpu, orc, valid, rel=REL_TOL, absf=ABS_TOL, name="", cond=None, lerr=None, med=None):
    """Return (ok, worst relative excess, report).  cond: the oracle's
    per-element conditioning sum (same shape as orc), or None; lerr: its
    absolute lookup-error bound, or None.  med: also require the median
    relative error (over elements above 1% of the mean magnitude) to stay
    below med, so that a tolerance widened for ill-conditioned elements
    cannot hide a systematic error."""
    g = gpu[:, valid].astype(np.float64)
    o = orc[:, valid]
    scale = np.abs(o).mean(axis=1, keepdims=True)
    bound = rel * np.abs(o) + absf * scale
    if cond is not None:
        bound = bound + COND_K * cond[:, valid]
    if lerr is not None:
        bound = bound + LERR_K * lerr[:, valid]
    err = np.abs(g - o)
    ok = err <= bound
    worst = float((err / np.maximum(bound, 1e-300)).max()) if err.size else 0.0
    big = np.abs(o) > 1e-2 * scale
    med_rel = float(np.median(err[big] / np.abs(o[big]))) if big.any() else 0.0
    rep = "%s: max|err|=%.3g, max rel=%.3g, median rel=%.3g, fail=%d/%d, worst/bound=%.3g" % (
        name, err.max() if err.size else 0, (err / np.maximum(np.abs(o), 1e-30)).max() if err.size else 0,
        med_rel, int((~ok).sum()), ok.size, worst)
    good = bool(ok.all()) and (med is None or med_rel <= med)
    return good, worst, rep

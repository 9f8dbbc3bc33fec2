"""Sampling techniques (appendix D ablation: cosine, BSDF, light-probe
sampling and MIS with the balance heuristic) and correlated/decorrelated
backward seeds (section 4.1), on the GPU.

Every technique subset estimates the same integral, so the image means over
many seeds agree within their standard errors; the variances differ, and the
balance heuristic is never far from the best single technique.  The backward
with a separate seed re-draws and re-traces its own samples and equals a
direct adjoint call with that seed.
"""

import numpy as np
import pytest

from workloads import make_workload, upstream_grads
from tests.parity_util import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TECHS = ("mis", "bsdf", "light", "cosine", "ggx")


def _flags(M, name):
    return {"mis": 0, "bsdf": M.FLAG_LIGHT_OFF, "light": M.FLAG_BSDF_OFF,
            "cosine": M.FLAG_LIGHT_OFF | M.FLAG_FORCE_COS, "ggx": M.FLAG_LIGHT_OFF | M.FLAG_FORCE_GGX}[name]


@pytest.fixture(scope="module")
def runs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_03380_amd as M
    w = make_workload("tiny")
    sc = M.Scene(torch.from_numpy(w.verts).cuda(), torch.from_numpy(w.tris).cuda())
    env = M.Env(torch.from_numpy(w.env).cuda())
    gb = M.GBuffer.from_workload(w, "cuda")
    K, spp = 48, 4
    out = {}
    for t in TECHS:
        c = []
        for k in range(K):
            cd, cs, _, _ = M.shade_fwd(sc, env, gb, spp, seed=1000 + k, tau=w.tau, ray_eps=w.ray_eps,
                                       flags=_flags(M, t), hitbits=False)
            c.append(to_np(gb.kd * cd + cs).astype(np.float64))
        out[t] = np.stack(c)            # [K, 3, N]
    torch.cuda.synchronize()
    return M, w, out


def test_all_techniques_estimate_the_same_image(runs):
    M, w, out = runs
    m = w.mask > 0
    K = out["mis"].shape[0]
    im = {t: out[t][:, :, m].mean(axis=(1, 2)) for t in TECHS}      # per-seed image means [K]
    for t in TECHS:
        se = np.sqrt(im[t].var(ddof=1) / K + im["mis"].var(ddof=1) / K)
        diff = abs(im[t].mean() - im["mis"].mean())
        print("%-7s image mean %.6f  (mis %.6f)  diff/se %.2f" % (t, im[t].mean(), im["mis"].mean(), diff / se))
        assert diff < 5 * se


def test_variance_ablation(runs):
    M, w, out = runs
    m = w.mask > 0
    metal, rough = w.korm[2], w.korm[1]
    classes = {"diffuse": m & (metal < 0.25) & (rough > 0.5), "glossy_metal": m & (metal > 0.75) & (rough < 0.35),
               "all": m}
    var = {}
    for cname, sel in classes.items():
        assert sel.sum() > 20, cname
        for t in TECHS:
            v = out[t][:, :, sel].var(axis=0, ddof=1).sum(0)               # per-pixel variance (summed over RGB)
            mu = out["mis"][:, :, sel].mean(axis=0).sum(0)
            var[(cname, t)] = float(np.mean(v / np.maximum(mu, 1e-3) ** 2))  # relative variance
        print(cname, {t: "%.3g" % var[(cname, t)] for t in TECHS})
    # cosine sampling is poor for sharp specular lobes; light sampling for
    # glossy metal picks directions the lobe rejects
    assert var[("glossy_metal", "mis")] < var[("glossy_metal", "cosine")]
    assert var[("glossy_metal", "mis")] < var[("glossy_metal", "light")]
    # the balance heuristic is within a small factor of the best single technique
    for cname in classes:
        best = min(var[(cname, t)] for t in TECHS if t != "mis")
        assert var[(cname, "mis")] <= 2.0 * best, cname


def test_decorrelated_backward_equals_direct_call():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_03380_amd as M
    w = make_workload("tiny")
    sc = M.Scene(torch.from_numpy(w.verts).cuda(), torch.from_numpy(w.tris).cuda())
    e = torch.from_numpy(w.env).cuda().requires_grad_(True)
    envt = e.detach()
    env = M.Env(envt)
    gb = M.GBuffer.from_workload(w, "cuda")
    ud, us = (torch.from_numpy(a).cuda() for a in upstream_grads(w))
    bs = M.decorrelated_seed(w.seed)
    assert bs != w.seed
    kd, korm, nrm = (t.clone().requires_grad_(True) for t in (gb.kd, gb.korm, gb.nrm))
    cd, cs = M.MCDIShade.apply(kd, korm, nrm, e, sc, env, gb, w.spp, w.seed, w.tau, w.ray_eps, 0, bs)
    ((cd * ud).sum() + (cs * us).sum()).backward()
    g = M.shade_bwd(sc, env, gb, w.spp, ud, us, hitbits=None, seed=bs, tau=w.tau, ray_eps=w.ray_eps)
    for a, b in zip((kd.grad, korm.grad, nrm.grad), g[:3]):
        assert torch.equal(a, b)
    assert torch.allclose(e.grad, g[3], rtol=1e-5, atol=1e-7 * float(g[3].abs().max()))
    # and differs from the correlated backward
    kd2 = gb.kd.clone().requires_grad_(True)
    cd2, cs2 = M.MCDIShade.apply(kd2, gb.korm, gb.nrm, envt, sc, env, gb, w.spp, w.seed, w.tau, w.ray_eps, 0)
    ((cd2 * ud).sum() + (cs2 * us).sum()).backward()
    assert not torch.equal(kd.grad, kd2.grad)


def test_technique_flags_through_autograd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_03380_amd as M
    w = make_workload("tiny")
    sc = M.Scene(torch.from_numpy(w.verts).cuda(), torch.from_numpy(w.tris).cuda())
    envt = torch.from_numpy(w.env).cuda()
    env = M.Env(envt)
    gb = M.GBuffer.from_workload(w, "cuda")
    ud, us = (torch.from_numpy(a).cuda() for a in upstream_grads(w))
    f = M.FLAG_BSDF_OFF
    kd = gb.kd.clone().requires_grad_(True)
    cd, cs = M.MCDIShade.apply(kd, gb.korm, gb.nrm, envt, sc, env, gb, w.spp, w.seed, w.tau, w.ray_eps, f)
    ((cd * ud).sum() + (cs * us).sum()).backward()
    _, _, hb, _ = M.shade_fwd(sc, env, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps, flags=f)
    g = M.shade_bwd(sc, env, gb, w.spp, ud, us, hitbits=hb, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps, flags=f)
    assert torch.equal(kd.grad, g[0])

"""Serving: continuous batching over resident scenes.

Each request's result is the same served alone, served in a mix, and shaded
by the plain staged forward/backward launches: per-pixel outputs and
gradients bit for bit (identical per-pixel code, random numbers keyed by the
pixel and the request's view id); the probe gradient within the FP32
summation-order bound.  Admission keeps the admitted requests' memory under
the budget.
"""

import numpy as np
import pytest

from workloads import serving, upstream_grads
from tests.parity_util import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_03380_amd as M
    scenes_np = serving.make_scenes(full=False, res=(64, 128))
    # a second resident scene: the tiny icosphere
    from workloads import make_workload
    scenes_np["T"] = {64: make_workload("tiny"), 128: make_workload("tiny", H=128, W=128)}
    resident = {}
    for name, views in scenes_np.items():
        w = next(iter(views.values()))
        resident[name] = (M.Scene(torch.from_numpy(w.verts).cuda(), torch.from_numpy(w.tris).cuda()),
                          M.Env(torch.from_numpy(w.env).cuda()))
    return M, scenes_np, resident


def build_requests(M, scenes_np, draws, flags=None):
    from paper_2206_03380_amd.serve import Request
    reqs = []
    for k, (name, res, spp, grad, vb) in enumerate(draws):
        w = scenes_np[name][res]
        gb = M.GBuffer.from_workload(w, "cuda")
        gb.view_base = vb
        r = Request(scene=name, gb=gb, spp=spp, seed=3, tau=w.tau, ray_eps=w.ray_eps,
                    flags=0 if flags is None else flags[k % len(flags)])
        if grad:
            ud, us = upstream_grads(w, seed=vb)
            r.g_cd, r.g_cs = torch.from_numpy(ud).cuda(), torch.from_numpy(us).cuda()
        reqs.append(r)
    torch.cuda.synchronize()
    return reqs


def results(r):
    out = {"c_d": to_np(r.c_d), "c_s": to_np(r.c_s)}
    if r.grad:
        for k in ("g_kd", "g_korm", "g_nrm", "g_env"):
            out[k] = to_np(getattr(r, k))
    return out


def check_same(a, b, env_rtol=1e-4):
    for k in ("c_d", "c_s", "g_kd", "g_korm", "g_nrm"):
        if k in a:
            assert np.array_equal(a[k], b[k]), k
    if "g_env" in a:
        scale = np.abs(a["g_env"]).max() + 1e-30
        assert np.allclose(a["g_env"], b["g_env"], rtol=env_rtol, atol=1e-6 * scale)


def test_served_equals_staged_and_alone(env):
    M, scenes_np, resident = env
    from paper_2206_03380_amd.serve import Server, PerRequest
    draws = serving.make_requests(scenes_np, 14, res=(64, 128), spps=(1, 4, 8, 32))
    # the reference: plain staged launches, one request at a time
    base = PerRequest(resident)
    ref = build_requests(M, scenes_np, draws)
    for r in ref:
        base.submit(r)
    base.drain()
    ref_res = [results(r) for r in ref]
    # all in one mix, small launches so requests spread over many launches
    srv = Server(resident, budget_bytes=1 << 34, max_slots=8, launch_samples=200_000, spp_max=64)
    mix = build_requests(M, scenes_np, draws)
    for r in mix:
        srv.submit(r)
    srv.drain()
    torch.cuda.synchronize()
    assert len(srv.completed) == len(mix) and srv.n_launches > 3
    for a, r in zip(ref_res, mix):
        check_same(a, results(r))
    # each request alone
    for i in (0, 5, 11):
        s1 = Server(resident, launch_samples=10_000_000, spp_max=64)
        alone = build_requests(M, scenes_np, [draws[i]])[0]
        s1.submit(alone)
        s1.drain()
        check_same(ref_res[i], results(alone))


def test_served_technique_flags_equal_staged(env):
    """Requests with technique subsets and the bilinear lookup, mixed in one
    launch: each equals its own staged forward/backward (the served adjoint
    scatters the bilinear taps with atomics, the staged one through records)."""
    M, scenes_np, resident = env
    from paper_2206_03380_amd.serve import Server, PerRequest
    flags = [0, M.FLAG_BILINEAR, M.FLAG_LIGHT_OFF, M.FLAG_BSDF_OFF | M.FLAG_BILINEAR,
             M.FLAG_LIGHT_OFF | M.FLAG_FORCE_GGX | M.FLAG_BILINEAR]
    draws = serving.make_requests(scenes_np, 10, seed=21, res=(64, 128), spps=(2, 8))
    draws = [(n, r, s, True, vb) for (n, r, s, g, vb) in draws]
    base = PerRequest(resident)
    ref = build_requests(M, scenes_np, draws, flags)
    for r in ref:
        base.submit(r)
    base.drain()
    ref_res = [results(r) for r in ref]
    srv = Server(resident, budget_bytes=1 << 34, max_slots=8, launch_samples=200_000, spp_max=64)
    mix = build_requests(M, scenes_np, draws, flags)
    for r in mix:
        srv.submit(r)
    srv.drain()
    torch.cuda.synchronize()
    assert len(srv.completed) == len(mix)
    for a, r in zip(ref_res, mix):
        check_same(a, results(r))
    # the bilinear requests differ from the same requests with the nearest lookup
    near = build_requests(M, scenes_np, draws[1:2], [0])[0]
    b2 = PerRequest(resident)
    b2.submit(near)
    b2.drain()
    assert not np.array_equal(results(near)["c_d"], ref_res[1]["c_d"])


def test_admission_respects_budget(env):
    """The server's scratch stays under the budget and the admitted requests
    under the slot count at every poll; every request completes once."""
    M, scenes_np, resident = env
    from paper_2206_03380_amd.serve import Server, request_bytes
    draws = serving.make_requests(scenes_np, 20, seed=9, res=(64, 128))
    reqs = build_requests(M, scenes_np, draws)
    sizes = [request_bytes(r.gb.n, r.spp) for r in reqs]
    budget = 3 * max(sizes)
    srv = Server(resident, budget_bytes=budget, max_slots=3, launch_samples=100_000, spp_max=64)
    peak, peak_slots, peak_queue = 0, 0, 0
    for r in reqs:
        srv.submit(r)
        i = srv.info()
        peak_queue = max(peak_queue, i["queued"])
    while srv.pump():
        i = srv.info()
        peak = max(peak, i["used_bytes"])
        peak_slots = max(peak_slots, i["admitted"])
    assert 0 < peak <= budget and 0 < peak_slots <= 3 and peak_queue > 0
    i = srv.info()
    assert i["used_bytes"] == 0 and i["admitted"] == 0 and i["queued"] == 0
    assert len(srv.completed) == len(reqs) and len({id(r) for r in srv.completed}) == len(reqs)
    assert all(r.done and r.latency > 0 for r in reqs)


def test_server_rejects_bad_requests(env):
    M, scenes_np, resident = env
    from paper_2206_03380_amd.serve import Server, request_bytes
    from paper_2206_03380_amd._lib import MCDIError, MCDI_E_INVALID, MCDI_E_UNSUPPORTED
    srv = Server(resident, spp_max=8)
    r = build_requests(M, scenes_np, [("A", 64, 16, False, 1)])[0]
    with pytest.raises(MCDIError) as ei:
        srv.submit(r)
    assert ei.value.status == MCDI_E_INVALID
    r3 = build_requests(M, scenes_np, [("A", 64, 4, False, 3)])[0]
    r3.flags = M.FLAG_DUMP
    with pytest.raises(MCDIError) as ei:
        srv.submit(r3)
    assert ei.value.status == MCDI_E_INVALID
    small = Server(resident, budget_bytes=1024, spp_max=8)
    r2 = build_requests(M, scenes_np, [("A", 64, 4, False, 2)])[0]
    assert request_bytes(r2.gb.n, r2.spp) > 1024
    with pytest.raises(MCDIError) as ei:
        small.submit(r2)
    assert ei.value.status == MCDI_E_UNSUPPORTED
    assert small.info()["queued"] == 0 and not small.pending
    # nothing was queued: both servers drain at once
    assert srv.drain() == [] and small.drain() == []


def test_submit_orders_after_the_callers_stream(env):
    """Inputs written on the caller's stream right before submit() (no
    synchronisation in between, the stream still busy): the serving stream
    waits for them, so the results equal the staged path's, for the batched
    server and for per-request launches."""
    M, scenes_np, resident = env
    from paper_2206_03380_amd.serve import Server, PerRequest, Request
    draws = serving.make_requests(scenes_np, 6, seed=33, res=(64, 128), spps=(4, 8))
    draws = [(n, r, s, True, vb) for (n, r, s, g, vb) in draws]
    base = PerRequest(resident)
    ref = build_requests(M, scenes_np, draws)
    for r in ref:
        base.submit(r)
    base.drain()
    torch.cuda.synchronize()
    ref_res = [results(r) for r in ref]
    makers = (lambda: Server(resident, budget_bytes=1 << 34, max_slots=8, launch_samples=200_000, spp_max=64),
              lambda: PerRequest(resident))
    for make in makers:
        sysm = make()
        src = build_requests(M, scenes_np, draws)      # synchronised copies
        torch.cuda._sleep(50_000_000)                  # keep the caller's stream busy
        reqs = []
        for r in src:
            gb = r.gb
            g2 = M.GBuffer(gb.pos.clone(), gb.nrm.clone(), gb.kd.clone(), gb.korm.clone(), gb.mask.clone(),
                           gb.eye.clone(), gb.n_views, gb.height, gb.width, gb.view_base)
            r2 = Request(scene=r.scene, gb=g2, spp=r.spp, seed=r.seed, tau=r.tau, ray_eps=r.ray_eps,
                         g_cd=r.g_cd * 1.0, g_cs=r.g_cs * 1.0)
            reqs.append(sysm.submit(r2))
        del src
        sysm.drain()
        torch.cuda.synchronize()
        assert len(sysm.completed) == len(reqs)
        for a, r in zip(ref_res, reqs):
            check_same(a, results(r))

#!/usr/bin/env python3
"""Benchmark of the differentiable Monte Carlo direct-illumination hot path.

One step = one optimisation iteration of the path on one batch: rebuild the
shadow-ray BVH from the mesh, rebuild the probe sampling tables, forward
shading (samples, MIS, shadow rays), the fused image loss (tonemapped L1 +
light regulariser, value and gradients in one kernel pass) and the backward
pass through the autograd Function (adjoint kernel with the probe-texel
scatter); with --denoise the cross-bilateral denoiser (sigma 2) sits between
shading and loss.  Inputs are resident in HBM before timing starts.

Default workload (the headline): the heavy-occlusion lattice room, 4 views
at 1024x1024 of a 1.0M-triangle lattice, a 2048x1024 probe, 32 samples per
pixel, forward + backward -- the largest single-GPU configuration, shaped
like the paper's multi-view batches and mesh sizes (synthetic data).  The
line also carries, as secondary keys, the 8 x 512^2 displaced-sphere
workload at 12 spp, the three-scene serving mix (batched persistent
launches against per-request launches at 0.5/0.7/0.9 of the saturated
rate), the next rows' kernels (denoiser, loss, sampling study, visibility
gradient) and the FP64 oracle's rate on the host cores.

Prints ONE JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shaded samples/s fwd+bwd (px×spp) + shadow rays/s; served p50/p99 latency"

# MI355X public peaks
CU, LANES, CLOCK = 256, 64, 2.4e9
VALU_PEAK = CU * LANES * CLOCK       # 32-bit lane operations per second, non-packed
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lattice")
    ap.add_argument("--secondary", default="sphere8_grad",
                    help="workload measured as a secondary key with fewer steps ('' to skip)")
    ap.add_argument("--secondary-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark on the three-scene mix (50k/300k/1M triangles)")
    ap.add_argument("--serve-requests", type=int, default=None,
                    help="measured requests per load of the serving mix (default 400 in the line, 2000 with --serve)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving mix of the default line")
    ap.add_argument("--serve-launch-samples", type=int, default=40_000_000,
                    help="work of one batched serving launch, in samples")
    ap.add_argument("--denoise", action="store_true", help="cross-bilateral denoiser (sigma 2) inside the step")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the denoiser, loss and sampling-study measurements (profiling runs of the step's "
                         "kernels: the study launches the traversal with other technique flags)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB device copy (counter calibration)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (pixels are independent, so "
              "sharding by views would only add an all-reduce of the probe gradient); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2206_03380_amd as M
    from workloads import make_workload

    torch.cuda.set_device(0)
    if args.serve:
        print(json.dumps(serve_mix(args, M, args.serve_requests or 2000)), flush=True)
        return
    t0 = time.time()
    w = make_workload(args.workload)
    log(args, "workload %s generated in %.1fs: %d px (%d valid), %d tris, env %s, spp %d" % (
        w.name, time.time() - t0, w.n_pixels, w.n_valid, len(w.tris), w.env.shape[:2], w.spp))
    m = measure(args, M, w, args.steps, args.warmup)
    result = {
        "metric": METRIC, "value": m["value"], "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": m["config"],
    }
    for k in ("shadow_rays_per_s", "fwd_ms", "bwd_ms", "trace_ms", "adjoint_ms", "bvh_build_ms", "env_cdf_ms",
              "shade_only_samples_per_s", "work", "roofline", "adjoint_roofline"):
        result[k] = m[k]
    gb = m["gb"]
    if not args.no_next_rows:
        result["next_rows"] = next_rows(args, M, gb, m["c_d"], m["c_s"], m["target"], m["timed"])
    del m
    torch.cuda.empty_cache()
    if args.secondary and args.secondary != args.workload:
        t0 = time.time()
        w2 = make_workload(args.secondary)
        log(args, "secondary workload %s generated in %.1fs" % (w2.name, time.time() - t0))
        m2 = measure(args, M, w2, args.secondary_steps, 2)
        result["secondary"] = {w2.name: {k: m2[k] for k in (
            "config", "value", "ms_per_step", "shadow_rays_per_s", "fwd_ms", "bwd_ms", "trace_ms", "adjoint_ms",
            "roofline", "adjoint_roofline")}}
        result["secondary"][w2.name]["steps"] = args.secondary_steps
        del m2, w2
        torch.cuda.empty_cache()
    if not args.no_serve:
        result["serving"] = serve_mix(args, M, args.serve_requests or 400)
    if args.copy_calibration:
        result["copy_calibration_bytes"] = copy_calibration("cuda:0")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, w)
    print(json.dumps(result), flush=True)


def measure(args, M, w, steps, warmup):
    """Time `steps` optimisation steps of workload w (after `warmup`), then
    the forward and backward calls, the BVH and table builds on their own,
    the work counts of the statistics instantiation, and the rooflines of the
    traversal and adjoint kernels (their HIP-event durations over the timed
    steps)."""
    import numpy as np
    import torch
    dev = "cuda:0"
    verts = torch.from_numpy(w.verts).to(dev)
    tris = torch.from_numpy(w.tris).to(dev)
    env_p = torch.from_numpy(w.env).to(dev)
    gb = M.GBuffer.from_workload(w, dev)
    kd = gb.kd.clone().requires_grad_(True)
    korm = gb.korm.clone().requires_grad_(True)
    nrm = gb.nrm.clone().requires_grad_(True)
    env_t = env_p.clone().requires_grad_(True)
    mask = gb.mask.bool()
    n_valid = int(mask.sum())

    # target image: one render with perturbed materials/probe (fixed seed)
    rng = np.random.Generator(np.random.PCG64(7))
    kd_t = np.clip(w.kd * (1 + 0.1 * rng.normal(size=w.kd.shape)), 0, 1).astype(np.float32)
    korm_t = w.korm.copy()
    korm_t[1] = np.clip(korm_t[1] + 0.05 * rng.normal(size=korm_t[1].shape), 0.08, 1).astype(np.float32)
    env_tgt = (w.env * np.exp(0.1 * rng.normal(size=w.env.shape))).astype(np.float32)
    with torch.no_grad():
        sc0 = M.Scene(verts, tris)
        ev0 = M.Env(torch.from_numpy(env_tgt).to(dev))
        gbt = M.GBuffer(gb.pos, gb.nrm, torch.from_numpy(kd_t).to(dev), torch.from_numpy(korm_t).to(dev), gb.mask,
                        gb.eye, gb.n_views, gb.height, gb.width)
        cd_t, cs_t, _, _ = M.shade_fwd(sc0, ev0, gbt, w.spp, seed=0, tau=w.tau, ray_eps=w.ray_eps, hitbits=False)
        target = (gbt.kd * cd_t + cs_t).detach()
        del sc0, ev0, cd_t, cs_t

    side = torch.cuda.Stream()
    timing = M.FLAG_TIME_TRACE | M.FLAG_TIME_ADJOINT

    def step():
        # BVH rebuild (the mesh changes every iteration) on a side stream: the
        # traversal waits for it, the ray generation before it does not
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            scene = M.Scene(verts, tris)
        envh = M.Env(env_t.detach())                      # probe tables rebuild
        c_d, c_s = M.MCDIShade.apply(kd, korm, nrm, env_t, scene, envh, gb, w.spp, w.seed, w.tau, w.ray_eps,
                                     timing)
        if args.denoise:
            guide = M.BilateralGuide.from_gbuffer(gb, sigma=2.0)
            y = M.Bilateral.apply(torch.cat([c_d, c_s]), guide)
            c_d, c_s = y[:3], y[3:]
        loss = M.ImageLoss.apply(kd, c_d, c_s, target, gb.mask, 0.15)
        loss.backward()
        for t in (kd, korm, nrm, env_t):
            t.grad = None

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    M.trace_times()                                       # forget warm-up timings
    M.adjoint_times()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    # traversal and adjoint kernels: HIP events on the stream they run on
    trace_ms_list, adj_ms_list = M.trace_times(), M.adjoint_times()
    trace_ms = sum(trace_ms_list) / max(len(trace_ms_list), 1)
    adj_ms = sum(adj_ms_list) / max(len(adj_ms_list), 1)
    samples = n_valid * w.spp
    value = samples / (ms * 1e-3)
    log(args, "%s: step %.3f ms -> %.3g samples/s; trace kernel %.3f ms (%d launches), adjoint kernel %.3f ms" % (
        w.name, ms, value, trace_ms, len(trace_ms_list), adj_ms))

    # ---- per-call timing on the launch stream (HIP events) ----
    scene = M.Scene(verts, tris)
    envh = M.Env(env_p)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    live = torch.empty((M.hit_words(w.spp), gb.n), dtype=torch.int32, device=dev)
    out = M.shade_fwd(scene, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps, live=live)
    hb = out[2]
    g_cd = torch.randn((3, gb.n), device=dev) * mask / n_valid
    g_cs = torch.randn((3, gb.n), device=dev) * mask / n_valid
    g_env = torch.zeros_like(env_p)
    bwd_out = (torch.empty_like(g_cd), torch.empty_like(g_cd), torch.empty_like(g_cd))
    reps = max(3, min(args.kernel_reps, int(2000 / max(ms, 1.0))))
    fwd_ms = timed(lambda: M.shade_fwd(scene, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps,
                                       out=out[:3], live=live), reps)
    bwd_ms = timed(lambda: M.shade_bwd(scene, envh, gb, w.spp, g_cd, g_cs, hitbits=hb, seed=w.seed, tau=w.tau,
                                       ray_eps=w.ray_eps, g_env=g_env, out=bwd_out, live=live), reps)
    bvh_ms = timed(lambda: M.Scene(verts, tris), max(3, reps // 2))
    cdf_ms = timed(lambda: M.Env(env_p), max(3, reps // 2))

    # ---- statistics instantiation (same rays): work counts ----
    st = M.new_stats(dev)
    M.shade_fwd(scene, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps, stats=st, hitbits=False)
    stats = M.read_stats(st)
    rays = stats["rays_traced"]

    # ---- roofline of the dominant kernel (any-hit traversal) ----
    # VALU lane-operations the method performs per launch, from the work counts
    ops = OPS_PER_RAY * rays + OPS_PER_BOX * stats["box_tests"] + OPS_PER_TRI * stats["tri_tests"]
    achieved = ops / (trace_ms * 1e-3)
    tfile = os.path.join(ROOT, "profiles", "trace_rays_%s_pmc.md" % w.name)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK, "traffic": measured_traffic(tfile),
                "kernel": "trace_rays_kernel", "ops_per_launch": ops, "kernel_ms": trace_ms,
                "units": {"rays": rays, "box_tests": stats["box_tests"], "tri_tests": stats["tri_tests"]},
                "lane_utilisation": {"box": stats["box_lanes"] / max(stats["box_slots"], 1),
                                     "tri": stats["tri_tests"] / max(stats["tri_slots"], 1)},
                "box_tests_per_lane_step": stats["box_tests"] / max(stats["box_lanes"], 1)}
    # ---- roofline of the adjoint kernel (shade_kernel<true>) ----
    adj_units = adjoint_units(hb, live, stats, w)
    adj_ops = (ADJ_OPS_PHILOX * adj_units["pairs_drawn"] + ADJ_OPS_LIGHT * adj_units["light_draws"] +
               ADJ_OPS_BSDF * adj_units["bsdf_draws"] + ADJ_OPS_PER_EVAL * adj_units["evaluated_directions"])
    adj_a = adj_ops / (adj_ms * 1e-3) if adj_ms > 0 else 0.0
    adjoint_roofline = {"bound": "alu", "achieved": adj_a / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TOP/s",
                        "frac": adj_a / VALU_PEAK, "traffic": None, "kernel": "shade_kernel<true>",
                        "ops_per_launch": adj_ops, "kernel_ms": adj_ms, "units": adj_units}
    STATE.update(scene=scene, env=envh, w=w, verts=verts, tris=tris)
    return {
        "config": {"workload": "%s: %d views %dx%d, %d tris, env %dx%d, %d spp, fwd+bwd" % (
            w.name, w.n_views, w.width, w.height, len(w.tris), w.env.shape[1], w.env.shape[0], w.spp),
            "views": w.n_views, "height": w.height, "width": w.width, "spp": w.spp, "tris": int(len(w.tris)),
            "env": [int(w.env.shape[0]), int(w.env.shape[1])], "valid_px": n_valid,
            "parallelism": "single-gpu"},
        "value": value, "ms_per_step": ms,
        "shadow_rays_per_s": rays / (fwd_ms * 1e-3),
        "fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "trace_ms": trace_ms, "adjoint_ms": adj_ms, "bvh_build_ms": bvh_ms,
        "env_cdf_ms": cdf_ms, "shade_only_samples_per_s": samples / ((fwd_ms + bwd_ms) * 1e-3),
        "work": stats, "roofline": roofline, "adjoint_roofline": adjoint_roofline,
        "gb": gb, "c_d": out[0], "c_s": out[1], "target": target, "timed": timed,
    }


# Adjoint kernel (shade_kernel<true>), VALU lane operations of the method.
# Per drawn sample pair of a valid pixel: the first Philox4x32-10 block (ten
# rounds of two 32x32->64 products, two xors and the key schedule: 80).  Per
# light draw (marginal and guided conditional searches, in-texel offsets, two
# sincospi, the direction and its density: 50).  Per BSDF draw (the second
# Philox block: 80; lobe choice, cosine or visible-normal warp, world frame,
# normalisation, two atan2 for the texel and its density: 100).  Per
# evaluated direction: the balance heuristic and the BSDF (half vector, D,
# both Smith Lambdas, G2, Schlick F, three densities: 60) and the
# derivatives (D and Lambda in alpha, S in alpha, n.v, n.l and n.h, the
# normal gradient in the tangent frame, kd/m/r terms, the probe coefficient
# and its scatter: 85) = 145.
ADJ_OPS_PHILOX = 80
ADJ_OPS_LIGHT = 50
ADJ_OPS_BSDF = 180
ADJ_OPS_PER_EVAL = 145


def adjoint_units(hb, live, stats, w):
    """The adjoint's units of work, counted from the step's hit bits and
    live bits ([words][N] u32 each, bit 2s the light sample of sample s,
    bit 2s + 1 its BSDF sample).  Given the live bits, the adjoint draws and
    differentiates the live samples -- with tau = 1 only those not blocked
    (a blocked one adds nothing) -- and a sample pair draws its first Philox
    block once.  Without tracing every sample of a valid pixel is drawn."""
    import numpy as np
    pairs = stats["valid_pixels"] * w.spp
    if w.tau == 0.0 or live is None:
        return {"pairs_drawn": pairs, "light_draws": pairs, "bsdf_draws": pairs,
                "evaluated_directions": stats["rays_traced"]}
    need = live.cpu().numpy().view(np.uint32)
    if w.tau == 1.0:
        need = need & ~hb.cpu().numpy().view(np.uint32)
    even = np.uint32(0x55555555)
    light, bsdf = need & even, (need >> np.uint32(1)) & even
    return {"pairs_drawn": int(np.bitwise_count(light | bsdf).sum()), "light_draws": int(np.bitwise_count(light).sum()),
            "bsdf_draws": int(np.bitwise_count(bsdf).sum()), "evaluated_directions": int(np.bitwise_count(need).sum())}


# per-unit VALU lane-operation counts of the traversal: slab test of one
# child box (6 sub, 6 mul, 6 min/max per axis, 5 min/max for the interval, 1
# compare), watertight test of one triangle (9 sub, 6 shear FMA, 6 mul + 3 sub
# for the edge functions, 6 sign compares, 2 add, 6 for the hit distance, 1
# compare), ray setup
OPS_PER_BOX = 24
OPS_PER_TRI = 39
OPS_PER_RAY = 25

# Cross-bilateral denoiser, per footprint tap of a valid pixel with six
# channels, in single-rate VALU issue slots: 15 FP32 ops (normal dot 3, clamp,
# depth difference, scale, two exponent FMAs, weight sum, 6 colour FMAs), one
# FP64->FP32 convert (2), two FP64 FMAs (half rate: 4) and three quarter-rate
# transcendentals (log2, rcp, exp2: 12).  The adjoint has no weight sum.
BILAT_OPS_FWD = 33
BILAT_OPS_BWD = 32
# Image loss: bytes per pixel that must cross HBM: kd, c_d, c_s, ref in
# (48), mask twice (count pass and loss pass, 2), three gradients out (36).
LOSS_BYTES_PER_PX = 86


def sampling_study(args, M, gb, timed, seeds=4):
    """Variance study of the sampling techniques on the step's workload:
    forward time at the workload's spp, and the mean per-pixel relative
    variance of the shaded colour over independent seeds; efficiency is
    1 / (variance x time) relative to MIS."""
    import torch
    sc, envh, w = STATE["scene"], STATE["env"], STATE["w"]
    techs = {"mis": 0, "bsdf": M.FLAG_LIGHT_OFF, "light": M.FLAG_BSDF_OFF,
             "cosine": M.FLAG_LIGHT_OFF | M.FLAG_FORCE_COS, "ggx": M.FLAG_LIGHT_OFF | M.FLAG_FORCE_GGX,
             "mis_bilinear": M.FLAG_BILINEAR}
    m = gb.mask.bool()
    res = {}
    for name, f in techs.items():
        cols = []
        for k in range(seeds):
            cd, cs, _, _ = M.shade_fwd(sc, envh, gb, w.spp, seed=100 + k, tau=w.tau, ray_eps=w.ray_eps, flags=f,
                                       hitbits=False)
            cols.append((gb.kd * cd + cs)[:, m].sum(0))
        c = torch.stack(cols).double()
        res[name] = {"rel_var": float((c.var(0) / c.mean(0).clamp_min(1e-3) ** 2).mean())}
        out = M.shade_fwd(sc, envh, gb, w.spp, seed=0, tau=w.tau, ray_eps=w.ray_eps, flags=f)
        res[name]["fwd_ms"] = timed(lambda: M.shade_fwd(sc, envh, gb, w.spp, seed=0, tau=w.tau, ray_eps=w.ray_eps,
                                                        flags=f, out=out[:3]), max(3, args.kernel_reps // 2))
    ref = res["mis"]["rel_var"] * res["mis"]["fwd_ms"]
    for name in res:
        res[name]["efficiency_vs_mis"] = ref / (res[name]["rel_var"] * res[name]["fwd_ms"])
    # the backward pass with either lookup (the bilinear one scatters each
    # sample's probe gradient to four texels)
    n = gb.n
    g_cd = torch.randn((3, n), device=gb.kd.device) * m / max(int(m.sum()), 1)
    g_cs = torch.randn((3, n), device=gb.kd.device) * m / max(int(m.sum()), 1)
    bwd = {}
    for name, f in (("nearest", 0), ("bilinear", M.FLAG_BILINEAR)):
        live = torch.empty((M.hit_words(w.spp), n), dtype=torch.int32, device=gb.kd.device)
        hb = M.shade_fwd(sc, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps, flags=f, live=live)[2]
        g_env = torch.zeros_like(envh.env)
        bo = tuple(torch.empty_like(g_cd) for _ in range(3))
        bwd[name] = timed(lambda: M.shade_bwd(sc, envh, gb, w.spp, g_cd, g_cs, hitbits=hb, seed=w.seed, tau=w.tau,
                                              ray_eps=w.ray_eps, flags=f, g_env=g_env, out=bo, live=live),
                          max(3, args.kernel_reps // 2))
    return {"spp": w.spp, "seeds": seeds, "techniques": res, "bwd_ms": bwd}


STATE = {}

# Edge-sampled visibility gradient, VALU lane-operations per edge sample
# (every sample): Philox4x32-10 (ten rounds of two 32x32->64 products = 4
# lane ops, and 4 xors: 80), class choice (a 64-bit product and a compare: 4),
# edge choice and t (4), the differences from o and along the edge (6), the
# arc normal (6), the two face-side determinants (24), sign logic and |m|^2
# (7) = 131.  Per sample that reaches the queue
# (silhouette, above the horizon): direction and distance (14), arc normal and
# Jacobian (18), probe lookup (two atan2 and the texel, 50), the BSDF terms
# (50), out-side direction and record (18) = 150.
EDGE_OPS_PER_SAMPLE = 131
EDGE_OPS_PER_QUEUED = 150
EDGE_SPP = 8


def visibility_gradient(args, M, gb, timed):
    """Edge-sampled shadow-visibility gradient on the step's workload: edge
    list build, and one gradient pass of EDGE_SPP edge samples per pixel, with
    a uniform edge choice and with sharp edges 64 times as likely."""
    import torch
    sc, envh, w = STATE["scene"], STATE["env"], STATE["w"]
    verts, tris = STATE["verts"], STATE["tris"]
    nv = verts.shape[0]
    m = gb.mask.bool()
    nval = max(int(m.sum()), 1)
    reps = max(3, args.kernel_reps // 2)
    ed = M.Edges(tris, nv)
    n_edges = ed.count()
    build_ms = timed(lambda: M.Edges(tris, nv), reps)
    gen = torch.Generator(device=gb.kd.device)
    gen.manual_seed(11)
    g_cd = torch.randn((3, gb.n), device=gb.kd.device, generator=gen) * m / nval
    g_cs = torch.randn((3, gb.n), device=gb.kd.device, generator=gen) * m / nval
    samples = nval * EDGE_SPP

    def measure(gain):
        gv = torch.zeros_like(verts)
        st = M.new_stats(verts.device)
        M.shade_bwd_edges(sc, envh, ed, verts, gb, EDGE_SPP, g_cd, g_cs, seed=w.seed, tau=w.tau,
                          ray_eps=w.ray_eps, g_verts=gv, stats=st, sharp_gain=gain)
        stats = M.read_stats(st)
        M.adjoint_times()
        ms = timed(lambda: M.shade_bwd_edges(sc, envh, ed, verts, gb, EDGE_SPP, g_cd, g_cs, seed=w.seed,
                                             tau=w.tau, ray_eps=w.ray_eps, g_verts=gv, sharp_gain=gain,
                                             flags=M.FLAG_TIME_ADJOINT), reps)
        # the edge-sample kernel of every pass of the timed calls (HIP events)
        gen = M.adjoint_times()
        calls = reps + 1
        return ms, stats, sum(gen) / calls, len(gen) // calls

    ms, stats, gen_ms, passes = measure(1)
    ms64, stats64, _, _ = measure(64)

    queued = stats["rays_traced"]
    ops = EDGE_OPS_PER_SAMPLE * samples + EDGE_OPS_PER_QUEUED * queued
    a = ops / (ms * 1e-3)
    # the edge-sample kernel streams one random 64-byte line (the drawn edge's
    # packed corners) per sample past the L2, plus the G-buffer position and
    # normal of each valid pixel, the mask of every pixel and a 4-byte record
    # per queued candidate: bound by memory bandwidth
    gen_bytes = 64 * samples + 24 * nval + gb.n + 4 * queued
    gen_a = gen_bytes / (gen_ms * 1e-3) if gen_ms > 0 else 0.0
    efile = os.path.join(ROOT, "profiles", "edge_grad_%s_pmc.md" % w.name)
    return {"edge_spp": EDGE_SPP, "edges": n_edges, "edge_build_ms": build_ms, "ms": ms,
            "edge_samples_per_s": samples / (ms * 1e-3), "samples": samples,
            "silhouette_rays": queued, "silhouette_rays_blocked": stats["rays_hit"],
            "sharp_gain_64": {"ms": ms64, "silhouette_rays": stats64["rays_traced"],
                              "silhouette_rays_blocked": stats64["rays_hit"]},
            "roofline": {"bound": "hbm", "achieved": gen_a / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": gen_a / HBM_PEAK,
                         "traffic": measured_traffic(efile, EDGE_SOURCES, "sample-kernel-bytes-per-call"),
                         "kernel": "edge_gen_kernel", "kernel_ms": gen_ms, "passes": passes,
                         "bytes_per_call": gen_bytes},
            "call_alu": {"bound": "alu", "achieved": a / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TOP/s",
                         "frac": a / VALU_PEAK,
                         "traffic": measured_traffic(efile, EDGE_SOURCES, "traffic-bytes-per-call"),
                         "ops_per_call": ops,
                         "note": "whole call, uniform edge choice: classes and corners packed, sample kernel, "
                                 "out-side-ray kernel"}}


def next_rows(args, M, gb, c_d, c_s, target, timed):
    """Denoiser and image-loss kernels on the step's own outputs, each timed
    alone with HIP events on the launch stream."""
    import torch
    n = gb.n
    valid = int(gb.mask.sum())
    reps = max(args.kernel_reps, 5)
    sigma = 2.0
    guide = M.BilateralGuide.from_gbuffer(gb, sigma=sigma)
    x = torch.cat([c_d, c_s]).contiguous()
    fo = (torch.empty_like(x), torch.empty(n, dtype=torch.float32, device=x.device))
    M.bilateral_fwd(guide, x, out=fo)
    g = torch.randn_like(x) * gb.mask
    gi = torch.empty_like(x)
    f_ms = timed(lambda: M.bilateral_fwd(guide, x, out=fo), reps)
    b_ms = timed(lambda: M.bilateral_bwd(guide, g, fo[1], out=gi), reps)
    d_ms = timed(lambda: M.view_depth(gb), reps)
    R = M.bilateral_radius(sigma)
    taps = valid * (2 * R + 1) ** 2

    def alu(ops, ms):
        a = ops / (ms * 1e-3)
        return {"bound": "alu", "achieved": a / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TOP/s",
                "frac": a / VALU_PEAK, "traffic": None}

    sampling = sampling_study(args, M, gb, timed)
    vis = visibility_gradient(args, M, gb, timed)
    lo = (torch.empty(3, dtype=torch.float32, device=x.device),) + tuple(torch.empty_like(c_d) for _ in range(3))
    l_ms = timed(lambda: M.image_loss(gb.kd, c_d, c_s, target, gb.mask, out=lo), reps)
    lbytes = LOSS_BYTES_PER_PX * n
    return {
        "bilateral": {"sigma": sigma, "radius": R, "channels": 6, "taps": taps,
                      "fwd_ms": f_ms, "bwd_ms": b_ms, "view_depth_ms": d_ms,
                      "fwd_roofline": alu(taps * BILAT_OPS_FWD, f_ms),
                      "bwd_roofline": alu(taps * BILAT_OPS_BWD, b_ms)},
        "sampling": sampling,
        "visibility_gradient": vis,
        "image_loss": {"ms": l_ms, "bytes_per_launch": lbytes,
                       "roofline": {"bound": "hbm", "achieved": lbytes / (l_ms * 1e-3) / 1e9,
                                    "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                    "frac": lbytes / (l_ms * 1e-3) / HBM_PEAK, "traffic": None}},
    }


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2206_03380_amd", "csrc", f)
                  for f in ("shade.hip", "shade_common.h", "device_common.h", "mcdi_internal.h", "bvh_build.hip")]
# the edge-gradient call's kernels (classes, packing, samples, out-side rays)
EDGE_SOURCES = [os.path.join(ROOT, "paper_2206_03380_amd", "csrc", f)
                for f in ("edge_grad.hip", "edge_internal.h", "shade_common.h", "device_common.h", "mcdi_internal.h")]


def kernel_source_hash(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES if files is None else files):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path, files=None, key="traffic-bytes-per-launch"):
    """HBM bytes per launch (or per call) from a committed FETCH_SIZE /
    WRITE_SIZE summary, scaled by the copy-kernel calibration; None when the
    kernel sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source-sha256") != kernel_source_hash(files):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def copy_calibration(dev):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    n = 128 * 1024 * 1024          # 512 MiB of float32
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 4 * n


def _serve_run(M, make_system, requests, arrivals):
    """Drive a serving system with the given arrivals; returns metrics."""
    import torch
    from paper_2206_03380_amd.serve import run_arrivals, percentile
    for r in requests:
        r.t_done = None
    sysm = make_system()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = run_arrivals(sysm, requests, arrivals)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [r.latency * 1e3 for r in done]
    samples = sum(r._valid * r.spp for r in done)
    return {"requests": len(done), "wall_s": wall, "samples_per_s": samples / wall,
            "p50_ms": percentile(lat, 0.5), "p99_ms": percentile(lat, 0.99), "launches": sysm.n_launches}


def _serving_compare(args, M, resident, requests, label, fracs=(0.5, 0.7, 0.9), warm=10):
    import numpy as np
    from paper_2206_03380_amd.serve import Server, PerRequest
    from workloads.serving import poisson_arrivals
    mk_srv = lambda: Server(resident, budget_bytes=64 << 30, max_slots=64, spp_max=32,  # noqa: E731
                            launch_samples=args.serve_launch_samples)
    mk_base = lambda: PerRequest(resident)  # noqa: E731
    # warm-up, then the saturated rates: everything arrives at once
    _serve_run(M, mk_srv, requests[:warm], np.zeros(warm))
    _serve_run(M, mk_base, requests[:warm], np.zeros(warm))
    sat = _serve_run(M, mk_srv, requests, np.zeros(len(requests)))
    sat_base = _serve_run(M, mk_base, requests, np.zeros(len(requests)))
    rate = sat["requests"] / sat["wall_s"]
    out = {"workload": label, "requests_per_load": len(requests), "budget_bytes": 64 << 30, "slots": 64,
           "launch_samples": args.serve_launch_samples,
           "saturated": {"batched": {"requests_per_s": rate, "samples_per_s": sat["samples_per_s"]},
                         "per_request_launches": {"requests_per_s": sat_base["requests"] / sat_base["wall_s"],
                                                  "samples_per_s": sat_base["samples_per_s"]}},
           "loads": []}
    for f in fracs:
        arr = poisson_arrivals(len(requests), f * rate)
        srv = _serve_run(M, mk_srv, requests, arr)
        base = _serve_run(M, mk_base, requests, arr)
        out["loads"].append({"load": f, "qps": f * rate, "batched": srv, "per_request_launches": base})
    return out


def serve_mix(args, M, n_requests):
    """Serving mix: resident scenes of ~50k, ~298k and ~1.0M triangles (probes
    512x256 to 2048x1024); requests draw scene, resolution in {128..1024}^2,
    spp in {4, 8, 16, 32}, forward or forward+backward; the saturated request
    rate of batched persistent launches and of one launch per request, then
    Poisson arrivals at 0.5/0.7/0.9 of the batched saturated rate through
    both (the same requests and seeds, hence identical results)."""
    import torch
    from paper_2206_03380_amd.serve import Request
    from workloads import serving, upstream_grads
    dev = "cuda:0"
    t0 = time.time()
    scenes_np = serving.make_scenes(full=True)
    log(args, "serving scenes generated in %.1fs" % (time.time() - t0))
    resident = {}
    gbs = {}
    for name, views in scenes_np.items():
        w0 = next(iter(views.values()))
        resident[name] = (M.Scene(torch.from_numpy(w0.verts).to(dev), torch.from_numpy(w0.tris).to(dev)),
                          M.Env(torch.from_numpy(w0.env).to(dev)))
        for res, w in views.items():
            ud, us = upstream_grads(w)
            gbs[(name, res)] = (M.GBuffer.from_workload(w, dev), torch.from_numpy(ud).to(dev),
                                torch.from_numpy(us).to(dev), w.n_valid, w.tau, w.ray_eps)
    warm = 50
    draws = serving.make_requests(scenes_np, n_requests + warm)
    reqs = []
    for (name, res, spp, grad, vb) in draws:
        gb, gd, gs, nv, tau, eps = gbs[(name, res)]
        g1 = M.GBuffer(gb.pos, gb.nrm, gb.kd, gb.korm, gb.mask, gb.eye, 1, res, res, vb)
        r = Request(scene=name, gb=g1, spp=spp, seed=0, tau=tau, ray_eps=eps)
        if grad:
            r.g_cd, r.g_cs = gd, gs
        r._valid = nv
        reqs.append(r)
    torch.cuda.synchronize()
    out = _serving_compare(args, M, resident, reqs[warm:], "three-scene serving mix (50k/298k/1.0M triangles)",
                           warm=warm)
    out["metric"] = METRIC
    out["tris"] = {n: int(len(next(iter(v.values())).tris)) for n, v in scenes_np.items()}
    return out


def cpu_baseline(args, w):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload."""
    import numpy as np
    import oracle
    from workloads import upstream_grads
    nthreads = oracle.max_threads()
    rng = np.random.Generator(np.random.PCG64(11))
    valid = np.nonzero(w.mask)[0]
    scene = oracle.Scene(w.verts, w.tris)
    tables = oracle.EnvTables(w.env)
    ud, us = upstream_grads(w)

    def run(n, threads=0):
        pix = np.sort(rng.choice(valid, n, replace=False))
        t = time.time()
        oracle.shade(w, pixels=pix, scene=scene, tables=tables, threads=threads)
        oracle.shade(w, pixels=pix, scene=scene, tables=tables, grad=True, u_d=ud[:, pix].astype(np.float64),
                     u_s=us[:, pix].astype(np.float64), threads=threads)
        return time.time() - t

    # size the sample from a calibration run large enough that per-call
    # overheads do not dominate; the whole workload when it fits the budget
    n = int(min(len(valid), 65536))
    dt = run(n)
    n2 = int(min(len(valid), max(n, n * args.cpu_seconds / max(dt, 1e-3))))
    dt2 = run(n2)
    what = ("all %d valid pixels" % n2 if n2 == len(valid) else
            "%d random valid pixels of the %d (rate extrapolated to the whole workload)" % (n2, len(valid)))
    res = {"value": n2 * w.spp / dt2, "unit": "samples/s", "cores": nthreads, "kind": "oracle",
           "sample": "%s of the same workload, forward + backward, %.1f s" % (what, dt2)}
    n1 = int(min(len(valid), 8192))
    dt1 = run(n1, threads=1)
    res["single_thread"] = {"value": n1 * w.spp / dt1, "unit": "samples/s", "cores": 1,
                            "sample": "%d random valid pixels, forward + backward, %.1f s" % (n1, dt1)}
    if not args.no_next_rows:
        # the oracle's edge-sampled visibility gradient beside the kernels' (row f4)
        edges = oracle.mesh_edges(w.tris, len(w.verts))
        # up to 2^18 random valid pixels (all of them on smaller workloads)
        pe = valid if len(valid) <= (1 << 18) else np.sort(rng.choice(valid, 1 << 18, replace=False))
        t = time.time()
        oracle.edge_grad(w, edges, EDGE_SPP, ud[:, pe].astype(np.float64), us[:, pe].astype(np.float64),
                         pixels=pe, scene=scene, tables=tables)
        dte = time.time() - t
        res["visibility_gradient"] = {"value": len(pe) * EDGE_SPP / dte, "unit": "edge samples/s",
                                      "cores": nthreads, "kind": "oracle",
                                      "sample": "%d of the %d valid pixels x %d edge samples, %.2f s" % (
                                          len(pe), len(valid), EDGE_SPP, dte)}
    return res


if __name__ == "__main__":
    main()

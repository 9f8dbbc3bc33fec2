#!/usr/bin/env python3
"""Benchmark of the differentiable Monte Carlo direct-illumination hot path.

One step = one optimisation iteration of the path on one batch: rebuild the
shadow-ray BVH from the mesh, rebuild the probe sampling tables, forward
shading (samples, MIS, shadow rays), the fused image loss (tonemapped L1 +
light regulariser, value and gradients in one kernel pass) and the backward
pass through the autograd Function (adjoint kernel with the probe-texel
scatter); with --denoise the cross-bilateral denoiser (sigma 2) sits between
shading and loss.  Inputs are resident in HBM before timing starts.  The
denoiser and the loss kernels are also timed on their own, each with its
roofline, under "next_rows".

Default workload: 8 views at 512x512 of a 101,060-triangle displaced sphere
with 20 box occluders, a 512x256 probe, 12 samples per pixel, forward +
backward (synthetic data shaped like the paper's multi-view batches).

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
    ap.add_argument("--workload", default="sphere8_grad")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark on the three-scene mix (50k/300k/1M triangles)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-serve", action="store_true", help="skip the short serving run of the default line")
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
    import numpy as np
    import torch
    import paper_2206_03380_amd as M
    from workloads import make_workload

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.serve:
        print(json.dumps(serve_full(args, M)), flush=True)
        return
    t0 = time.time()
    w = make_workload(args.workload)
    log(args, "workload %s generated in %.1fs: %d px (%d valid), %d tris, env %s, spp %d" % (
        w.name, time.time() - t0, w.n_pixels, w.n_valid, len(w.tris), w.env.shape[:2], w.spp))

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
        del sc0, ev0

    side = torch.cuda.Stream()

    def step():
        # BVH rebuild (the mesh changes every iteration) on a side stream: the
        # traversal waits for it, the ray generation before it does not
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            scene = M.Scene(verts, tris)
        envh = M.Env(env_t.detach())                      # probe tables rebuild
        c_d, c_s = M.MCDIShade.apply(kd, korm, nrm, env_t, scene, envh, gb, w.spp, w.seed, w.tau, w.ray_eps,
                                     M.FLAG_TIME_TRACE)
        if args.denoise:
            guide = M.BilateralGuide.from_gbuffer(gb, sigma=2.0)
            y = M.Bilateral.apply(torch.cat([c_d, c_s]), guide)
            c_d, c_s = y[:3], y[3:]
        loss = M.ImageLoss.apply(kd, c_d, c_s, target, gb.mask, 0.15)
        loss.backward()
        return scene, envh

    # warmup
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    M.trace_times()                                       # forget warm-up timings
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    trace_ms_list = M.trace_times()                       # traversal kernel, HIP events on its stream
    trace_ms = sum(trace_ms_list) / max(len(trace_ms_list), 1)
    samples = n_valid * w.spp
    value = samples / (ms * 1e-3)
    log(args, "step %.3f ms -> %.3g samples/s; trace kernel %.3f ms (%d launches)" % (
        ms, value, trace_ms, len(trace_ms_list)))

    # ---- per-kernel timing on the launch stream (HIP events) ----
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

    out = M.shade_fwd(scene, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps)
    hb = out[2]
    g_cd = torch.randn((3, gb.n), device=dev) * mask / n_valid
    g_cs = torch.randn((3, gb.n), device=dev) * mask / n_valid
    g_env = torch.zeros_like(env_p)
    bwd_out = (torch.empty_like(g_cd), torch.empty_like(g_cd), torch.empty_like(g_cd))
    fwd_ms = timed(lambda: M.shade_fwd(scene, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps,
                                       out=out[:3]), args.kernel_reps)
    bwd_ms = timed(lambda: M.shade_bwd(scene, envh, gb, w.spp, g_cd, g_cs, hitbits=hb, seed=w.seed, tau=w.tau,
                                       ray_eps=w.ray_eps, g_env=g_env, out=bwd_out), args.kernel_reps)
    bvh_ms = timed(lambda: M.Scene(verts, tris), max(3, args.kernel_reps // 2))
    cdf_ms = timed(lambda: M.Env(env_p), max(3, args.kernel_reps // 2))

    # ---- statistics instantiation (same rays): work counts ----
    st = M.new_stats(dev)
    M.shade_fwd(scene, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps, stats=st, hitbits=False)
    stats = M.read_stats(st)
    rays = stats["rays_traced"]

    # ---- roofline of the dominant kernel (any-hit traversal) ----
    # VALU lane-operations the method performs per launch, from the work counts
    ops = OPS_PER_RAY * rays + OPS_PER_BOX * stats["box_tests"] + OPS_PER_TRI * stats["tri_tests"]
    achieved = ops / (trace_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK, "traffic": measured_traffic(),
                "kernel": "trace_rays_kernel", "ops_per_launch": ops, "kernel_ms": trace_ms,
                "units": {"rays": rays, "box_tests": stats["box_tests"], "tri_tests": stats["tri_tests"]},
                "lane_utilisation": {"box": stats["box_tests"] / max(stats["box_slots"], 1),
                                     "tri": stats["tri_tests"] / max(stats["tri_slots"], 1)}}

    result = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s: %d views %dx%d, %d tris, env %dx%d, %d spp, fwd+bwd" % (
            w.name, w.n_views, w.width, w.height, len(w.tris), w.env.shape[1], w.env.shape[0], w.spp),
            "views": w.n_views, "height": w.height, "width": w.width, "spp": w.spp, "tris": int(len(w.tris)),
            "env": [int(w.env.shape[0]), int(w.env.shape[1])], "valid_px": n_valid,
            "parallelism": "single-gpu"},
        "shadow_rays_per_s": rays / (fwd_ms * 1e-3),
        "fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "trace_ms": trace_ms, "bvh_build_ms": bvh_ms, "env_cdf_ms": cdf_ms,
        "shade_only_samples_per_s": samples / ((fwd_ms + bwd_ms) * 1e-3),
        "work": stats,
        "roofline": roofline,
    }

    STATE.update(scene=scene, env=envh, w=w, verts=verts, tris=tris)
    if not args.no_next_rows:
        result["next_rows"] = next_rows(args, M, gb, out[0], out[1], target, timed)
    if not args.no_serve:
        result["serving"] = serve_quick(args, M, w, gb)
    if args.copy_calibration:
        result["copy_calibration_bytes"] = copy_calibration(dev)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, w)
    print(json.dumps(result), flush=True)


# per-unit VALU lane-operation counts of the traversal: slab test of one node
# box (6 sub, 6 mul, 6 min/max per axis, 5 min/max for the interval, 1 mul for
# the slack, 1 compare), watertight test of one triangle (9 sub, 6 shear FMA,
# 6 mul + 3 sub for the edge functions, 6 sign compares, 2 add, 6 for the hit
# distance, 1 compare), ray setup
OPS_PER_BOX = 25
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
        hb = M.shade_fwd(sc, envh, gb, w.spp, seed=w.seed, tau=w.tau, ray_eps=w.ray_eps, flags=f)[2]
        g_env = torch.zeros_like(envh.env)
        bo = tuple(torch.empty_like(g_cd) for _ in range(3))
        bwd[name] = timed(lambda: M.shade_bwd(sc, envh, gb, w.spp, g_cd, g_cs, hitbits=hb, seed=w.seed, tau=w.tau,
                                              ray_eps=w.ray_eps, flags=f, g_env=g_env, out=bo),
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
        ms = timed(lambda: M.shade_bwd_edges(sc, envh, ed, verts, gb, EDGE_SPP, g_cd, g_cs, seed=w.seed,
                                             tau=w.tau, ray_eps=w.ray_eps, g_verts=gv, sharp_gain=gain), reps)
        return ms, stats

    ms, stats = measure(1)
    ms64, stats64 = measure(64)

    queued = stats["rays_traced"]
    ops = EDGE_OPS_PER_SAMPLE * samples + EDGE_OPS_PER_QUEUED * queued
    a = ops / (ms * 1e-3)
    return {"edge_spp": EDGE_SPP, "edges": n_edges, "edge_build_ms": build_ms, "ms": ms,
            "edge_samples_per_s": samples / (ms * 1e-3), "samples": samples,
            "silhouette_rays": queued, "silhouette_rays_blocked": stats["rays_hit"],
            "sharp_gain_64": {"ms": ms64, "silhouette_rays": stats64["rays_traced"],
                              "silhouette_rays_blocked": stats64["rays_hit"]},
            "roofline": {"bound": "alu", "achieved": a / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TOP/s",
                         "frac": a / VALU_PEAK, "traffic": measured_traffic(EDGE_TRAFFIC_FILE, EDGE_SOURCES,
                                                                            "traffic-bytes-per-call"),
                         "ops_per_launch": ops,
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "trace_rays_sphere8_grad_pmc.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2206_03380_amd", "csrc", f)
                  for f in ("shade.hip", "shade_common.h", "device_common.h", "mcdi_internal.h", "bvh_build.hip")]
# the edge-gradient call's kernels (classes, packing, samples, out-side rays)
EDGE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "edge_grad_sphere8_grad_pmc.md")
EDGE_SOURCES = [os.path.join(ROOT, "paper_2206_03380_amd", "csrc", f)
                for f in ("edge_grad.hip", "edge_internal.h", "shade_common.h", "device_common.h", "mcdi_internal.h")]


def kernel_source_hash(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES if files is None else files):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE, files=None, key="traffic-bytes-per-launch"):
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


def _serving_compare(args, M, resident, requests, label, fracs=(0.7,), warm=10):
    import numpy as np
    from paper_2206_03380_amd.serve import Server, PerRequest
    from workloads.serving import poisson_arrivals
    mk_srv = lambda: Server(resident, budget_bytes=64 << 30, max_slots=64, spp_max=32)  # noqa: E731
    mk_base = lambda: PerRequest(resident)  # noqa: E731
    # warm-up, then the saturated rate: everything arrives at once
    _serve_run(M, mk_srv, requests[:warm], np.zeros(warm))
    _serve_run(M, mk_base, requests[:warm], np.zeros(warm))
    sat = _serve_run(M, mk_srv, requests, np.zeros(len(requests)))
    rate = sat["requests"] / sat["wall_s"]
    out = {"workload": label, "saturated_requests_per_s": rate, "saturated_samples_per_s": sat["samples_per_s"],
           "loads": []}
    for f in fracs:
        arr = poisson_arrivals(len(requests), f * rate)
        srv = _serve_run(M, mk_srv, requests, arr)
        base = _serve_run(M, mk_base, requests, arr)
        out["loads"].append({"load": f, "qps": f * rate, "batched": srv, "per_request_launches": base})
    return out


def serve_quick(args, M, w, gb):
    """Short serving run on the main scene: each request is one 512x512 view
    with spp in {4, 8, 16, 32}, forward or forward+backward (50/50), Poisson
    arrivals at 0.7x the batched saturated rate; same requests through plain
    per-request launches."""
    import numpy as np
    import torch
    from paper_2206_03380_amd.serve import Request
    from workloads import upstream_grads
    dev = "cuda:0"
    resident = {"main": (M.Scene(torch.from_numpy(w.verts).to(dev), torch.from_numpy(w.tris).to(dev)),
                         M.Env(torch.from_numpy(w.env).to(dev)))}
    hw = w.height * w.width
    ud, us = upstream_grads(w)
    rng = np.random.Generator(np.random.PCG64(5))
    views = []
    for v in range(w.n_views):
        sl = slice(v * hw, (v + 1) * hw)
        g1 = M.GBuffer(gb.pos[:, sl].contiguous(), gb.nrm[:, sl].contiguous(), gb.kd[:, sl].contiguous(),
                       gb.korm[:, sl].contiguous(), gb.mask[sl].contiguous(), gb.eye[v:v + 1].contiguous(), 1,
                       w.height, w.width, v)
        views.append((g1, torch.from_numpy(np.ascontiguousarray(ud[:, sl])).to(dev),
                      torch.from_numpy(np.ascontiguousarray(us[:, sl])).to(dev), int(w.mask[sl].sum())))
    reqs = []
    for i in range(120):
        v = int(rng.integers(w.n_views))
        g1, gd, gs, nv = views[v]
        r = Request(scene="main", gb=g1, spp=int(rng.choice([4, 8, 16, 32])), seed=i, tau=w.tau,
                    ray_eps=w.ray_eps)
        if rng.random() < 0.5:
            r.g_cd, r.g_cs = gd, gs
        r._valid = nv
        reqs.append(r)
    torch.cuda.synchronize()
    return _serving_compare(args, M, resident, reqs, "one 512x512 view of the main scene per request")


def serve_full(args, M):
    """Serving mix: resident scenes of ~50k, ~298k and ~1.0M triangles (probes
    512x256 to 2048x1024); requests draw scene, resolution in {128..1024}^2,
    spp in {4, 8, 16, 32}, forward or forward+backward; Poisson arrivals at
    0.5/0.7/0.9 of the saturated request rate."""
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
    draws = serving.make_requests(scenes_np, args.serve_requests + 50)
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
    out = _serving_compare(args, M, resident, reqs[50:], "three-scene serving mix (50k/298k/1.0M triangles)",
                           fracs=(0.5, 0.7, 0.9), warm=50)
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
    what = "all %d valid pixels" % n2 if n2 == len(valid) else "%d random valid pixels" % n2
    res = {"value": n2 * w.spp / dt2, "unit": "samples/s", "cores": nthreads, "kind": "oracle",
           "sample": "%s of the same workload, forward + backward, %.1f s" % (what, dt2)}
    n1 = int(min(len(valid), 8192))
    dt1 = run(n1, threads=1)
    res["single_thread"] = {"value": n1 * w.spp / dt1, "unit": "samples/s", "cores": 1,
                            "sample": "%d random valid pixels, forward + backward, %.1f s" % (n1, dt1)}
    if not args.no_next_rows:
        # the oracle's edge-sampled visibility gradient beside the kernels' (row f4)
        edges = oracle.mesh_edges(w.tris, len(w.verts))
        # every valid pixel: the same work as the kernels' measurement
        t = time.time()
        oracle.edge_grad(w, edges, EDGE_SPP, ud[:, valid].astype(np.float64), us[:, valid].astype(np.float64),
                         pixels=valid, scene=scene, tables=tables)
        dte = time.time() - t
        res["visibility_gradient"] = {"value": len(valid) * EDGE_SPP / dte, "unit": "edge samples/s",
                                      "cores": nthreads, "kind": "oracle",
                                      "sample": "all %d valid pixels x %d edge samples, %.2f s" % (
                                          len(valid), EDGE_SPP, dte)}
    return res


if __name__ == "__main__":
    main()

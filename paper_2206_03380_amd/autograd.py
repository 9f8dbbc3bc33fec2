"""torch.autograd.Function over the forward/backward kernels.

Forward saves only the shadow-ray hit bits (2 bits per sample and pixel);
backward replays the same random numbers and recomputes every BSDF, pdf and
MIS term instead of storing them per sample (paper: section 4.1, the forward
seed is re-used during backpropagation; sampling and visibility detached).
"""

import torch

from . import _lib as L


class MCDIShade(torch.autograd.Function):
    """c_d, c_s = MCDIShade.apply(kd, korm, nrm, env, scene, env_tables, gbuf, spp, seed, tau, ray_eps, flags,
                                 bwd_seed, verts, edges, edge_spp, sharp_gain)

    kd, korm, nrm: [3, N] float32 (differentiable); env: the [H, W, 3] probe
    tensor the tables were built from (differentiable; its gradient is the
    texel scatter).  Positions, mask and eyes come from gbuf (not
    differentiated: shape gradients come from primary visibility).
    bwd_seed None (default): the backward replays the forward's samples
    (correlated, section 4.1); otherwise it draws and traces its own samples
    from bwd_seed (decorrelated, unbiased; see decorrelated_seed).
    verts, edges, edge_spp: optionally the mesh's vertex positions [Nv, 3]
    (the ones scene was built from; differentiable), its Edges and a number
    of edge samples per pixel: the backward then also returns the
    edge-sampled visibility gradient of the shadow term for verts (the paper
    detaches it by default, section 3.1 "Shadow gradients").  sharp_gain: how
    many times as likely a sharp edge is drawn as a smooth one (1 = uniform
    over the edges; see shade_bwd_edges)."""

    @staticmethod
    def forward(ctx, kd, korm, nrm, env, scene, env_tables, gbuf, spp, seed=0, tau=1.0, ray_eps=1e-3, flags=0,
                bwd_seed=None, verts=None, edges=None, edge_spp=0, sharp_gain=1):
        from . import _ptr, _stream, hit_words, _params
        import ctypes as C
        n = gbuf.n
        dev = kd.device
        kd, korm, nrm = kd.contiguous(), korm.contiguous(), nrm.contiguous()
        if env_tables.env.data_ptr() != env.data_ptr():
            raise ValueError("env_tables must be built from the env tensor passed in")
        c_d = torch.empty((3, n), dtype=torch.float32, device=dev)
        c_s = torch.empty((3, n), dtype=torch.float32, device=dev)
        need_bits = tau != 0.0 and any(ctx.needs_input_grad[:4]) and bwd_seed is None
        hb = torch.empty((hit_words(spp), n), dtype=torch.int32, device=dev) if need_bits else None
        # the live samples go with the hit bits: the adjoint draws only those
        live = torch.empty_like(hb) if need_bits else None
        gs = gbuf.struct(kd=kd, korm=korm, nrm=nrm)
        prm = _params(spp, seed, tau, ray_eps, flags, None, live)
        L.check(L.lib().mcdi_shade_fwd(scene.handle, env_tables.handle, C.byref(gs), C.byref(prm), _ptr(c_d),
                                       _ptr(c_s), _ptr(hb), None, _stream()))
        vis = verts is not None and edges is not None and edge_spp > 0
        empty = torch.empty(0, device=dev)
        ctx.save_for_backward(kd, korm, nrm, hb if hb is not None else empty, live if live is not None else empty,
                              verts if vis else empty)
        ctx.meta = (scene, env_tables, gbuf, spp, seed if bwd_seed is None else bwd_seed, tau, ray_eps,
                    hb is not None, flags & ~(L.FLAG_DUMP | L.FLAG_TIME_TRACE))
        ctx.vis = (edges, edge_spp, sharp_gain) if vis else None
        return c_d, c_s

    @staticmethod
    def backward(ctx, g_cd, g_cs):
        from . import _ptr, _stream, _params
        import ctypes as C
        kd, korm, nrm, hb, live, verts = ctx.saved_tensors
        scene, env_tables, gbuf, spp, seed, tau, ray_eps, has_bits, flags = ctx.meta
        n = gbuf.n
        dev = kd.device
        g_cd = (g_cd if g_cd is not None else torch.zeros((3, n), device=dev)).contiguous().float()
        g_cs = (g_cs if g_cs is not None else torch.zeros((3, n), device=dev)).contiguous().float()
        g_kd = torch.empty((3, n), dtype=torch.float32, device=dev)
        g_korm = torch.empty((3, n), dtype=torch.float32, device=dev)
        g_nrm = torch.empty((3, n), dtype=torch.float32, device=dev)
        g_env = torch.zeros((env_tables.H, env_tables.W, 3), dtype=torch.float32, device=dev)
        if any(ctx.needs_input_grad[:4]):
            gs = gbuf.struct(kd=kd, korm=korm, nrm=nrm)
            prm = _params(spp, seed, tau, ray_eps, flags, None, live if has_bits else None)
            L.check(L.lib().mcdi_shade_bwd(scene.handle, env_tables.handle, C.byref(gs), C.byref(prm), _ptr(g_cd),
                                           _ptr(g_cs), _ptr(hb) if has_bits else None, _ptr(g_kd), _ptr(g_korm),
                                           _ptr(g_nrm), _ptr(g_env), None, _stream()))
        else:
            g_kd = g_korm = g_nrm = g_env = None
        g_verts = None
        if ctx.vis is not None and ctx.needs_input_grad[13]:
            from . import shade_bwd_edges
            edges, edge_spp, sharp_gain = ctx.vis
            g_verts = shade_bwd_edges(scene, env_tables, edges, verts.detach().contiguous(), gbuf, edge_spp, g_cd,
                                      g_cs, seed=seed, tau=tau, ray_eps=ray_eps, flags=flags & L.FLAG_BILINEAR,
                                      sharp_gain=sharp_gain)
        return (g_kd, g_korm, g_nrm, g_env, None, None, None, None, None, None, None, None, None, g_verts, None,
                None, None)


class Bilateral(torch.autograd.Function):
    """out = Bilateral.apply(x, guide): cross-bilateral denoiser on x [C, N]
    (C in 1, 3, 6) with the guide's depth/normal edge-stopping weights.  The
    weights are constants: the gradient flows to x only (appendix B)."""

    @staticmethod
    def forward(ctx, x, guide):
        from . import bilateral_fwd
        out, wsum = bilateral_fwd(guide, x.contiguous())
        ctx.save_for_backward(wsum)
        ctx.guide = guide
        return out

    @staticmethod
    def backward(ctx, g_out):
        from . import bilateral_bwd
        (wsum,) = ctx.saved_tensors
        return bilateral_bwd(ctx.guide, g_out.contiguous().float(), wsum), None


class ImageLoss(torch.autograd.Function):
    """L = ImageLoss.apply(kd, c_d, c_s, ref, mask, w_light): tonemapped L1 of
    the composed image kd*c_d + c_s against ref plus w_light times the light
    regulariser (appendix A).  One kernel pass computes the loss and its
    gradients; backward only scales them by the upstream gradient."""

    @staticmethod
    def forward(ctx, kd, c_d, c_s, ref, mask, w_light=0.15):
        from . import image_loss
        loss, g_kd, g_cd, g_cs = image_loss(kd.contiguous(), c_d.contiguous(), c_s.contiguous(),
                                            ref.contiguous(), mask, w_light)
        ctx.save_for_backward(g_kd, g_cd, g_cs)
        return loss[2]

    @staticmethod
    def backward(ctx, g):
        g_kd, g_cd, g_cs = ctx.saved_tensors
        return g_kd * g, g_cd * g, g_cs * g, None, None, None

"""Continuous-batching request loop over resident scenes.

Scenes (BVH) and probe tables stay resident on the device.  Requests (a
G-buffer already on the device, spp, seed, forward-only or forward+backward
with upstream gradients) go to the library's server (mcdi_server_*), which
admits them while its scratch budget and slot count allow, packs their tiles
(256 pixels), oldest request first, into persistent launches of bounded work
on two alternating streams (one launch's tail overlaps the next launch), and
reports completed requests by ticket.  This module only allocates each request's outputs and marshals the
calls; latency is measured from submit() to the poll that reports the
request's ticket, on the host clock.

Every pixel is computed by the same code as the staged forward/backward with
random numbers keyed by (pixel, view_base, sample), so a request's results do
not depend on the mix it was served in (the probe gradient up to FP32
summation order).
"""

import ctypes as C
import time
from collections import deque
from dataclasses import dataclass

import torch

from . import _lib as L
from . import _ptr, GBuffer, _TORCH_ALLOCATOR

TILE = 256


@dataclass
class Request:
    scene: str
    gb: GBuffer
    spp: int
    seed: int = 0
    tau: float = 1.0
    ray_eps: float = 1e-3
    flags: int = 0                     # technique / probe-lookup flags (FLAG_*; not DUMP or TIME_*)
    g_cd: torch.Tensor = None          # upstream gradients: forward+backward request
    g_cs: torch.Tensor = None
    # filled by the server
    rid: int = -1
    t_submit: float = 0.0
    t_done: float = None
    c_d: torch.Tensor = None
    c_s: torch.Tensor = None
    g_kd: torch.Tensor = None
    g_korm: torch.Tensor = None
    g_nrm: torch.Tensor = None
    g_env: torch.Tensor = None

    @property
    def grad(self):
        return self.g_cd is not None

    @property
    def done(self):
        return self.t_done is not None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_submit


def _alloc_outputs(req, env):
    """Outputs on the caller's stream (the server's first read of the request
    waits for that stream's work so far, the zero fill of g_env included)."""
    n, dev = req.gb.n, req.gb.pos.device
    req.c_d = torch.empty((3, n), dtype=torch.float32, device=dev)
    req.c_s = torch.empty((3, n), dtype=torch.float32, device=dev)
    if req.grad:
        req.g_kd = torch.empty((3, n), dtype=torch.float32, device=dev)
        req.g_korm = torch.empty((3, n), dtype=torch.float32, device=dev)
        req.g_nrm = torch.empty((3, n), dtype=torch.float32, device=dev)
        req.g_env = torch.zeros((env.H, env.W, 3), dtype=torch.float32, device=dev)


def request_bytes(n_pixels, spp):
    """Server scratch a request holds while admitted (hit bits and ray
    origins)."""
    return int(L.lib().mcdi_server_request_bytes(int(n_pixels), int(spp)))


class Server:
    def __init__(self, scenes, budget_bytes=64 << 30, max_slots=64, launch_samples=40_000_000, spp_max=64,
                 n_workgroups=0, stream=None):
        """scenes: {name: (Scene, Env)} resident on the device.  stream: the
        server's allocation stream (its launches run on two streams of the
        library's own)."""
        self.scenes = scenes
        self.stream = stream or torch.cuda.Stream()
        cfg = L.ServerConfig(int(budget_bytes), int(launch_samples), int(max_slots), int(spp_max), int(n_workgroups), 0)
        h = C.c_void_p()
        L.check(L.lib().mcdi_server_create(C.byref(cfg), C.byref(_TORCH_ALLOCATOR),
                                           C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self.pending = {}             # ticket -> request
        self.completed = []
        self._rid = 0
        self._buf = (C.c_int64 * 256)()

    def close(self):
        if getattr(self, "handle", None):
            L.lib().mcdi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = L.ServerInfo()
        L.check(L.lib().mcdi_server_info(self.handle, C.byref(i)))
        return {"used_bytes": i.used_bytes, "launches": i.launches, "queued": i.queued, "admitted": i.admitted,
                "in_flight": i.in_flight}

    @property
    def n_launches(self):
        return self.info()["launches"]

    # ------------------------------------------------------------------
    def submit(self, req):
        scene, env = self.scenes[req.scene]
        req.t_submit = time.perf_counter()
        _alloc_outputs(req, env)
        q = L.Request()
        q.scene, q.env = scene.handle, env.handle
        q.gbuf = req.gb.struct()
        q.params = L.Params(req.spp, int(req.flags), req.seed, float(req.tau), float(req.ray_eps), None)
        q.c_d, q.c_s = _ptr(req.c_d), _ptr(req.c_s)
        if req.grad:
            q.g_cd, q.g_cs = _ptr(req.g_cd), _ptr(req.g_cs)
            q.g_kd, q.g_korm, q.g_nrm, q.g_env = _ptr(req.g_kd), _ptr(req.g_korm), _ptr(req.g_nrm), _ptr(req.g_env)
        ticket = C.c_int64()
        caller = torch.cuda.current_stream()
        L.check(L.lib().mcdi_server_submit(self.handle, C.byref(q), C.c_void_p(caller.cuda_stream),
                                           C.byref(ticket)))
        # the request (and through it every buffer the server reads or
        # writes) stays referenced until its ticket is reported
        req.rid = self._rid
        self._rid += 1
        self.pending[ticket.value] = req
        return req

    def _collect(self, fn):
        n = C.c_int32()
        L.check(fn(self.handle, self._buf, len(self._buf), C.byref(n)))
        now = time.perf_counter()
        for k in range(n.value):
            r = self.pending.pop(self._buf[k])
            r.t_done = now
            self.completed.append(r)
        return n.value

    def pump(self):
        """Completions, admission and launches, without blocking.  Returns
        True while requests are outstanding."""
        while self._collect(L.lib().mcdi_server_poll) == len(self._buf):
            pass
        return bool(self.pending)

    def drain(self):
        while self.pending:
            self._collect(L.lib().mcdi_server_wait)
        return self.completed


class PerRequest:
    """Baseline with the same interface: every request is shaded by its own
    staged launches (forward, then backward for gradient requests) on one
    stream, in arrival order, as soon as it is submitted."""

    def __init__(self, scenes, stream=None):
        self.scenes = scenes
        self.stream = stream or torch.cuda.Stream()
        self.in_flight = deque()
        self.completed = []
        self._rid = 0
        self.n_launches = 0

    def submit(self, req):
        from . import shade_fwd, shade_bwd, hit_words
        req.rid = self._rid
        self._rid += 1
        req.t_submit = time.perf_counter()
        scene, env = self.scenes[req.scene]
        # the inputs were written on the caller's stream: order after it, and
        # keep their memory from being reused while this stream reads them
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream())
        self.stream.wait_event(ready)
        gb = req.gb
        for t in [gb.pos, gb.nrm, gb.kd, gb.korm, gb.mask, gb.eye] + ([req.g_cd, req.g_cs] if req.grad else []):
            t.record_stream(self.stream)
        with torch.cuda.stream(self.stream):
            # the adjoint gets the forward's live samples with its hit bits
            live = (torch.empty((hit_words(req.spp), req.gb.n), dtype=torch.int32, device=req.gb.pos.device)
                    if req.grad and req.tau != 0.0 else None)
            req.c_d, req.c_s, hb, _ = shade_fwd(scene, env, req.gb, req.spp, seed=req.seed, tau=req.tau,
                                                ray_eps=req.ray_eps, flags=req.flags, hitbits=req.grad,
                                                stream=self.stream, live=live)
            self.n_launches += 1
            if req.grad:
                req.g_kd, req.g_korm, req.g_nrm, req.g_env = shade_bwd(
                    scene, env, req.gb, req.spp, req.g_cd, req.g_cs, hitbits=hb, seed=req.seed, tau=req.tau,
                    ray_eps=req.ray_eps, flags=req.flags, stream=self.stream, live=live)
                self.n_launches += 1
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self.in_flight.append((ev, req))
        return req

    def pump(self):
        while self.in_flight and self.in_flight[0][0].query():
            _, r = self.in_flight.popleft()
            r.t_done = time.perf_counter()
            self.completed.append(r)
        return bool(self.in_flight)

    def drain(self):
        while self.pump():
            time.sleep(0)
        return self.completed


def run_arrivals(system, requests, arrivals):
    """Submit requests at their arrival times (seconds from now) and drive the
    system until all complete.  Returns the completed requests."""
    t0 = time.perf_counter()
    i = 0
    n = len(requests)
    while i < n or system.pump():
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            system.submit(requests[i])
            i += 1
        if i < n and not system.pump():
            # idle: wait for the next arrival
            while time.perf_counter() - t0 < arrivals[i]:
                pass
    return system.completed


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    f = int(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)

"""Continuous-batching request loop over resident scenes.

Scenes (BVH) and probe tables stay resident on the device.  Requests (a
G-buffer already on the device, spp, seed, forward-only or forward+backward
with upstream gradients) are admitted while a device-memory budget and a slot
count allow, and their tiles (256 pixels) are packed, oldest request first,
into persistent launches of bounded work; requests that arrive while earlier
ones are on the GPU join the next launch.  Two launches are kept in flight on
one stream so the device never waits for the host.  A request completes when
the launch holding its last tile has finished (HIP event); latency is
measured from submit() to that moment on the host clock.

Every pixel is computed by the same code as the staged forward/backward with
random numbers keyed by (pixel, view_base, sample), so a request's results do
not depend on the mix it was served in (the probe gradient up to FP32
summation order).
"""

import ctypes as C
import time
from collections import deque
from dataclasses import dataclass, field

import torch

from . import _lib as L
from . import _ptr, _stream, hit_words, GBuffer, _TORCH_ALLOCATOR

TILE = 256


@dataclass
class Request:
    scene: str
    gb: GBuffer
    spp: int
    seed: int = 0
    tau: float = 1.0
    ray_eps: float = 1e-3
    flags: int = 0                     # technique / probe-lookup flags (FLAG_*; not DUMP or TIME_TRACE)
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
    _hb: torch.Tensor = None
    _org: torch.Tensor = None
    _next_tile: int = 0
    _tiles: int = 0
    _bytes: int = 0
    _last_launch: int = -1
    _ready: object = None              # event on the submitting stream: inputs written

    @property
    def grad(self):
        return self.g_cd is not None

    @property
    def done(self):
        return self.t_done is not None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_submit



def _inputs(req):
    """Device tensors a request reads: its G-buffer planes and upstream
    gradients."""
    gb = req.gb
    ts = [gb.pos, gb.nrm, gb.kd, gb.korm, gb.mask, gb.eye]
    if req.grad:
        ts += [req.g_cd, req.g_cs]
    return ts


def _order_after_caller(req, stream):
    """The server's stream must not read a request's inputs (or the probe
    tables built before it) before the caller's stream has written them: an
    event recorded on the submitting stream, waited for by `stream` before
    the first launch that reads the request.  The inputs are also marked as
    used on `stream`, so the caching allocator does not hand their memory out
    again while that stream may still read it."""
    ev = torch.cuda.Event()
    ev.record(torch.cuda.current_stream())
    req._ready = ev
    for t in _inputs(req):
        t.record_stream(stream)


def request_bytes(n_pixels, spp, grad, env_hw):
    """Device memory a request holds while admitted."""
    b = n_pixels * (24 + 4 * hit_words(spp) + 16)
    if grad:
        b += n_pixels * 36 + env_hw[0] * env_hw[1] * 12
    return b


class Server:
    def __init__(self, scenes, budget_bytes=64 << 30, max_slots=64, launch_samples=40_000_000, spp_max=64,
                 n_workgroups=0, stream=None):
        """scenes: {name: (Scene, Env)} resident on the device."""
        self.scenes = scenes
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.launch_samples = launch_samples
        self.spp_max = spp_max
        self.stream = stream or torch.cuda.Stream()
        h = C.c_void_p()
        L.check(L.lib().mcdi_server_create(spp_max, n_workgroups, C.byref(_TORCH_ALLOCATOR),
                                           C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self.queue = deque()          # submitted, not admitted
        self.admitted = []            # admitted, tiles pending or in flight
        self.in_flight = deque()      # (launch id, event, [requests completing in it])
        self.used = 0
        self.launch_id = 0
        self.n_launches = 0
        self._rid = 0
        self.completed = []

    def close(self):
        if getattr(self, "handle", None):
            L.lib().mcdi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def submit(self, req):
        if req.spp > self.spp_max:
            raise ValueError("spp above the server's spp_max")
        if req.scene not in self.scenes:
            raise KeyError(req.scene)
        req.rid = self._rid
        self._rid += 1
        req.t_submit = time.perf_counter()
        env = self.scenes[req.scene][1]
        req._bytes = request_bytes(req.gb.n, req.spp, req.grad, (env.H, env.W))
        if req._bytes > self.budget:
            raise ValueError("request larger than the memory budget")
        _order_after_caller(req, self.stream)
        self.queue.append(req)
        return req

    def _admit(self):
        while self.queue and len(self.admitted) < self.max_slots and self.used + self.queue[0]._bytes <= self.budget:
            r = self.queue.popleft()
            env = self.scenes[r.scene][1]
            n, dev = r.gb.n, r.gb.pos.device
            with torch.cuda.stream(self.stream):
                r.c_d = torch.empty((3, n), dtype=torch.float32, device=dev)
                r.c_s = torch.empty((3, n), dtype=torch.float32, device=dev)
                r._hb = torch.empty((hit_words(r.spp), n), dtype=torch.int32, device=dev)
                r._org = torch.empty((n, 4), dtype=torch.float32, device=dev)
                if r.grad:
                    r.g_kd = torch.empty((3, n), dtype=torch.float32, device=dev)
                    r.g_korm = torch.empty((3, n), dtype=torch.float32, device=dev)
                    r.g_nrm = torch.empty((3, n), dtype=torch.float32, device=dev)
                    r.g_env = torch.zeros((env.H, env.W, 3), dtype=torch.float32, device=dev)
            r._tiles = (n + TILE - 1) // TILE
            r._next_tile = 0
            self.used += r._bytes
            self.admitted.append(r)

    def _item(self, r, first, count):
        scene, env = self.scenes[r.scene]
        it = L.ServeItem()
        it.scene, it.env = scene.handle, env.handle
        it.gbuf = r.gb.struct()
        it.params = L.Params(r.spp, int(r.flags), r.seed, float(r.tau), float(r.ray_eps), None)
        it.c_d, it.c_s, it.hitbits, it.origins = (r.c_d.data_ptr(), r.c_s.data_ptr(), r._hb.data_ptr(),
                                                  r._org.data_ptr())
        if r.grad:
            it.g_cd, it.g_cs = r.g_cd.data_ptr(), r.g_cs.data_ptr()
            it.g_kd, it.g_korm, it.g_nrm, it.g_env = (r.g_kd.data_ptr(), r.g_korm.data_ptr(), r.g_nrm.data_ptr(),
                                                      r.g_env.data_ptr())
        it.first_tile, it.n_tiles = first, count
        return it

    def _launch(self):
        """Pack pending tiles, oldest request first, up to the launch's work budget."""
        items, finishing = [], []
        budget = self.launch_samples
        for r in self.admitted:
            if r._next_tile >= r._tiles or budget <= 0:
                continue
            per_tile = TILE * r.spp * (2 if r.grad else 1)
            take = min(r._tiles - r._next_tile, max(1, budget // per_tile))
            items.append(self._item(r, r._next_tile, take))
            r._next_tile += take
            budget -= take * per_tile
            if r._next_tile >= r._tiles:
                finishing.append(r)
        if not items:
            return False
        # first launch of a request: after the caller's writes of its inputs
        for r in self.admitted:
            if r._ready is not None and r._next_tile > 0:
                self.stream.wait_event(r._ready)
                r._ready = None
        arr = (L.ServeItem * len(items))(*items)
        L.check(L.lib().mcdi_server_launch(self.handle, arr, len(items)))
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self.in_flight.append((self.launch_id, ev, finishing))
        self.launch_id += 1
        self.n_launches += 1
        return True

    def _poll(self):
        while self.in_flight and self.in_flight[0][1].query():
            _, _, finishing = self.in_flight.popleft()
            now = time.perf_counter()
            for r in finishing:
                r.t_done = now
                self.used -= r._bytes
                self.admitted.remove(r)
                r._hb = None
                r._org = None
                self.completed.append(r)

    def pump(self):
        """One scheduling step: completions, admission, and a launch if fewer
        than two are in flight.  Returns True if work remains."""
        self._poll()
        self._admit()
        while len(self.in_flight) < 2 and self._launch():
            pass
        return bool(self.queue or self.admitted or self.in_flight)

    def drain(self):
        while self.pump():
            time.sleep(0)
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
        from . import shade_fwd, shade_bwd
        req.rid = self._rid
        self._rid += 1
        req.t_submit = time.perf_counter()
        scene, env = self.scenes[req.scene]
        _order_after_caller(req, self.stream)
        self.stream.wait_event(req._ready)
        with torch.cuda.stream(self.stream):
            req.c_d, req.c_s, hb, _ = shade_fwd(scene, env, req.gb, req.spp, seed=req.seed, tau=req.tau,
                                                ray_eps=req.ray_eps, flags=req.flags, hitbits=req.grad,
                                                stream=self.stream)
            self.n_launches += 1
            if req.grad:
                req.g_kd, req.g_korm, req.g_nrm, req.g_env = shade_bwd(
                    scene, env, req.gb, req.spp, req.g_cd, req.g_cs, hitbits=hb, seed=req.seed, tau=req.tau,
                    ray_eps=req.ray_eps, flags=req.flags, stream=self.stream)
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

"""Primary-visibility G-buffer by analytic ray casting (float64, numpy).

The method consumes a G-buffer produced upstream by a rasterizer; here it is
produced by intersecting camera rays with the analytic surfaces the meshes
tessellate.  Closest hit only; this is not the estimator's shadow-ray test.
"""

import numpy as np


def mat3(a, m):
    """a [N, 3] times m [3, K] as an explicit sum over the three terms, in a
    fixed order: the result does not depend on how many threads a BLAS
    library happens to use (the generated inputs are bit-reproducible)."""
    return a[:, 0, None] * m[0] + a[:, 1, None] * m[1] + a[:, 2, None] * m[2]


def look_at_rays(eye, target, fov_deg, height, width, up=(0.0, 1.0, 0.0)):
    """Unit ray directions through pixel centres, row-major (y down)."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    th = np.tan(np.radians(fov_deg) / 2.0)
    aspect = width / height
    xs = ((np.arange(width) + 0.5) / width * 2.0 - 1.0) * th * aspect
    ys = (1.0 - (np.arange(height) + 0.5) / height * 2.0) * th
    X, Y = np.meshgrid(xs, ys)
    d = fwd[None, None, :] + X[..., None] * right + Y[..., None] * upv
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return d.reshape(-1, 3)


class Hits:
    def __init__(self, n):
        self.t = np.full(n, np.inf)
        self.nrm = np.zeros((n, 3))
        self.obj = np.full(n, -1, np.int64)

    def take(self, t, nrm, obj):
        better = t < self.t
        self.t[better] = t[better]
        self.nrm[better] = nrm[better]
        self.obj[better] = obj


def hit_sphere(o, d, center, radius):
    oc = o - center
    b = (oc * d).sum(-1)
    c = (oc * oc).sum(-1) - radius * radius
    disc = b * b - c
    t = np.full(len(d), np.inf)
    ok = disc >= 0
    sq = np.sqrt(np.where(ok, disc, 0.0))
    t0 = -b - sq
    t1 = -b + sq
    tt = np.where(t0 > 1e-9, t0, np.where(t1 > 1e-9, t1, np.inf))
    t[ok] = tt[ok]
    p = o + d * np.where(np.isfinite(t), t, 0.0)[:, None]
    n = (p - center) / radius
    return t, n


def hit_rect_y(o, d, y, x0, x1, z0, z1, up=True):
    """Horizontal rectangle at height y; normal +Y (up) or -Y."""
    t = np.full(len(d), np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        tt = (y - o[:, 1]) / d[:, 1]
    p = o + d * np.nan_to_num(tt, posinf=0, neginf=0)[:, None]
    ok = (tt > 1e-9) & (p[:, 0] >= x0) & (p[:, 0] <= x1) & (p[:, 2] >= z0) & (p[:, 2] <= z1)
    t[ok] = tt[ok]
    n = np.zeros_like(d)
    n[:, 1] = 1.0 if up else -1.0
    return t, n


def hit_box(o, d, center, half, yaw=0.0):
    """Box rotated by yaw about +Y: slab test in the box frame."""
    c = np.asarray(center, np.float64)
    cy, sy = np.cos(yaw), np.sin(yaw)
    rot = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])  # local -> world
    ol = mat3(o - c, rot)
    dl = mat3(d, rot)
    half = np.asarray(half, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dl
        t0 = (-half - ol) * inv
        t1 = (half - ol) * inv
    tmin = np.minimum(t0, t1)
    tmax = np.maximum(t0, t1)
    tmin = np.nan_to_num(tmin, nan=-np.inf)
    tmax = np.nan_to_num(tmax, nan=np.inf)
    tn = tmin.max(-1)
    tf = tmax.min(-1)
    t = np.full(len(d), np.inf)
    ok = (tn <= tf) & (tf > 1e-9)
    tt = np.where(tn > 1e-9, tn, tf)
    t[ok] = tt[ok]
    # normal: axis of the entering (or exiting) slab
    ax = np.where(tn > 1e-9, tmin.argmax(-1), tmax.argmin(-1))
    nl = np.zeros_like(d)
    rows = np.arange(len(d))
    sgn = np.where(tn > 1e-9, -np.sign(dl[rows, ax]), np.sign(dl[rows, ax]))
    nl[rows, ax] = sgn
    return t, mat3(nl, rot.T)


class DisplacedSphere:
    """Implicit surface |x| = 1 + amp * n(x/|x|), n a normalised sum of
    random-direction sinusoids, values in [-1, 1]."""

    def __init__(self, rng, amp=0.05, n_waves=8):
        u = rng.normal(size=(n_waves, 3))
        self.u = u / np.linalg.norm(u, axis=1, keepdims=True)
        self.freq = rng.uniform(2.0, 6.0, n_waves)
        self.phase = rng.uniform(0.0, 2 * np.pi, n_waves)
        self.amp = amp
        self.n_waves = n_waves

    def noise(self, dirs):
        arg = mat3(dirs, self.u.T) * self.freq + self.phase
        return np.sin(arg).sum(-1) / self.n_waves

    def radius(self, dirs):
        return 1.0 + self.amp * self.noise(dirs)

    def f(self, x):
        r = np.linalg.norm(x, axis=-1)
        return r - self.radius(x / r[:, None])

    def grad(self, x):
        r = np.linalg.norm(x, axis=-1, keepdims=True)
        xh = x / r
        arg = mat3(xh, self.u.T) * self.freq + self.phase
        c = np.cos(arg) * self.freq / self.n_waves  # d noise / d(xh.u_k)
        proj = self.u[None, :, :] - mat3(xh, self.u.T)[:, :, None] * xh[:, None, :]
        dn = (c[:, :, None] * proj).sum(1) / r
        return xh - self.amp * dn

    def intersect(self, o, d):
        n = len(d)
        rmax = 1.0 + self.amp * 1.01
        t, _ = hit_sphere(o, d, np.zeros(3), rmax)
        alive = np.isfinite(t)
        tt = np.where(alive, t, 0.0)
        lip = 1.0 + self.amp * self.freq.max() / (1.0 - self.amp) + 0.1
        for _ in range(400):
            if not alive.any():
                break
            idx = np.nonzero(alive)[0]
            x = o[idx] + d[idx] * tt[idx, None]
            fx = self.f(x)
            done = fx < 1e-9
            tt[idx] += np.where(done, 0.0, fx / lip)
            r = np.linalg.norm(o[idx] + d[idx] * tt[idx, None], axis=-1)
            gone = (r > rmax + 1e-6) & ~done
            alive[idx[done | gone]] = False
            tt[idx[gone]] = np.inf
        hitm = np.isfinite(tt) & np.isfinite(t)
        # Newton polish along the ray
        idx = np.nonzero(hitm)[0]
        for _ in range(4):
            x = o[idx] + d[idx] * tt[idx, None]
            g = self.grad(x)
            den = (g * d[idx]).sum(-1)
            step = np.where(np.abs(den) > 1e-6, self.f(x) / den, 0.0)
            step = np.clip(step, -1e-3, 1e-3)
            tt[idx] -= step
        out = np.full(n, np.inf)
        out[hitm] = tt[hitm]
        nrm = np.zeros((n, 3))
        if len(idx):
            g = self.grad(o[idx] + d[idx] * out[idx, None])
            nrm[idx] = g / np.linalg.norm(g, axis=-1, keepdims=True)
        return out, nrm

    def mesh(self, freq):
        from .meshes import geodesic_sphere
        v, f = geodesic_sphere(freq)
        return v * self.radius(v)[:, None], f

"""FP64 oracle of the differentiable cross-bilateral denoiser (appendix B,
"Bilateral Denoiser": the spatial part of SVGF evaluated densely).

TEST INFRASTRUCTURE (imported by tests and the benchmark's CPU leg only).

  out(p) = sum_q c(q) w(p,q) / sum_q w(p,q),  q in the (2R+1)^2 footprint of p
  w(p,q) = exp(-|p-q|^2 / (2 sigma^2))
         * exp(-|z(p) - z(q)| / (sigma_z |grad z(p) . (p - q)| + eps))
         * max(0, n(p) . n(q))^sigma_n
with R = min(8, max(1, ceil(3 sigma))), eps = 1e-5, n normalised, grad z by
central differences in the image (one-sided where a neighbour is outside the
view or invalid, 0 if both are).  Only valid pixels (mask) contribute or
receive; invalid pixels output 0.  Gradients flow to the colours only:
  dL/dc(q) = sum_p dL/dout(p) w(p,q) / W(p),  W(p) = sum_q w(p,q).
Readings of points the paper leaves open: the footprint radius, eps, the
depth-gradient stencil and the masking.
"""

import math

import numpy as np

EPS = 1e-5


def radius(sigma):
    return int(min(8, max(1, math.ceil(3.0 * sigma))))


def _views(a, V, H, W):
    return np.asarray(a, np.float64).reshape(-1, V, H, W)


def depth_gradient(z, mask):
    """z, mask [V][H][W] -> (gx, gy), depth change per pixel along x and y:
    central difference where both neighbours are valid and inside the view,
    one-sided where only one is, 0 where neither is."""
    def along(dy, dx):
        zp, mp = _shift(z, dy, dx, 0.0), _shift(mask, dy, dx, False)
        zm, mm = _shift(z, -dy, -dx, 0.0), _shift(mask, -dy, -dx, False)
        return np.where(mp & mm, (zp - zm) / 2,
                        np.where(mp, zp - z, np.where(mm, z - zm, 0.0)))
    return along(0, 1), along(1, 0)


def weights_setup(depth, nrm, mask, V, H, W):
    """Guides of valid pixels (values at invalid pixels are never used)."""
    m = _views(mask, V, H, W)[0] > 0
    z = np.where(m, _views(depth, V, H, W)[0], 0.0)
    n = np.where(m, _views(nrm, V, H, W), 0.0)
    ln = np.sqrt((n ** 2).sum(0))
    n = np.where(ln > 0, n / np.where(ln > 0, ln, 1), 0)
    gx, gy = depth_gradient(z, m)
    return z, m, n, gx, gy


def _shift(a, dy, dx, fill):
    """out[..., y, x] = a[..., y + dy, x + dx] (fill outside)."""
    out = np.full_like(a, fill)
    H, W = a.shape[-2], a.shape[-1]
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    ys2 = slice(max(0, dy), min(H, H + dy))
    xs2 = slice(max(0, dx), min(W, W + dx))
    out[..., ys, xs] = a[..., ys2, xs2]
    return out


def tap_weight(z, m, n, gx, gy, dy, dx, sigma, sigma_z, sigma_n):
    """w(p, p + (dx, dy)) for every p, [V][H][W] (0 where q invalid)."""
    zq = _shift(z, dy, dx, 0.0)
    mq = _shift(m, dy, dx, False)
    nq = _shift(n, dy, dx, 0.0)
    ws = math.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))
    pred = np.abs(gx * (-dx) + gy * (-dy))         # grad z(p) . (p - q)
    wz = np.exp(-np.abs(z - zq) / (sigma_z * pred + EPS))
    wn = np.maximum(0.0, (n * nq).sum(0)) ** sigma_n
    return np.where(m & mq, ws * wz * wn, 0.0)


def bilateral_fwd(color, depth, nrm, mask, V, H, W, sigma, sigma_z=1.0, sigma_n=128.0):
    """Returns (out [3][N], wsum [N])."""
    z, m, n, gx, gy = weights_setup(depth, nrm, mask, V, H, W)
    c = np.where(m, _views(color, V, H, W), 0.0)
    R = radius(sigma)
    num = np.zeros_like(c)
    den = np.zeros_like(z)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            w = tap_weight(z, m, n, gx, gy, dy, dx, sigma, sigma_z, sigma_n)
            num += w * _shift(c, dy, dx, 0.0)
            den += w
    out = np.where(m, num / np.where(den > 0, den, 1), 0.0)
    return out.reshape(c.shape[0], -1), den.reshape(-1)


def view_depth(pos, eye, mask, V, H, W):
    """Depth guide of a G-buffer: distance from the view's eye, 0 where
    mask is 0.  pos [3][N], eye [V][3] -> [N]."""
    p = np.asarray(pos, np.float64).reshape(3, V, H * W)
    e = np.asarray(eye, np.float64).reshape(V, 3).T[:, :, None]
    d = np.sqrt(((p - e) ** 2).sum(0)).reshape(-1)
    return np.where(np.asarray(mask).reshape(-1) > 0, d, 0.0)


def bilateral_bwd(g_out, depth, nrm, mask, V, H, W, sigma, sigma_z=1.0, sigma_n=128.0):
    """dL/dcolor [3][N] for upstream dL/dout [3][N]."""
    z, m, n, gx, gy = weights_setup(depth, nrm, mask, V, H, W)
    g = np.where(m, _views(g_out, V, H, W), 0.0)
    R = radius(sigma)
    den = np.zeros_like(z)
    taps = []
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            w = tap_weight(z, m, n, gx, gy, dy, dx, sigma, sigma_z, sigma_n)
            taps.append((dy, dx, w))
            den += w
    gp = np.where(m, g / np.where(den > 0, den, 1), 0.0)   # dL/dout(p) / W(p)
    gc = np.zeros_like(g)
    for dy, dx, w in taps:
        # w[p] = w(p, p + d): contributes to q = p + d
        gc += _shift(gp * w, -dy, -dx, 0.0)
    return gc.reshape(g.shape[0], -1)

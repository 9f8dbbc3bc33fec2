"""FP64 oracle of the image loss on the estimator's outputs (appendix A,
"Optimization and Regularization": image loss and light regulariser).

TEST INFRASTRUCTURE (imported by tests and the benchmark's CPU leg only).

  c       = kd * c_d + c_s                               (section 4.2, composition)
  T(x)    = Gamma(log(max(x, 0) + 1)), Gamma = sRGB transfer function
  L_image = mean over valid pixels and channels of |T(c) - T(ref)|
  L_light = mean over valid pixels of |Y(T(c_d + c_s)) - V(T(ref))|,
            Y(x) = (r + g + b) / 3, V(x) = max(r, g, b)
  L       = L_image + w_light * L_light
Gradients with respect to kd, c_d, c_s; sign(0) = 0; the clamp at 0 passes no
gradient for x < 0.
"""

import numpy as np

A = 0.055
LIN = 0.0031308


def srgb(y):
    y = np.asarray(y, np.float64)
    return np.where(y <= LIN, 12.92 * y, (1 + A) * np.power(np.maximum(y, LIN), 1 / 2.4) - A)


def srgb_d(y):
    y = np.asarray(y, np.float64)
    return np.where(y <= LIN, 12.92, (1 + A) / 2.4 * np.power(np.maximum(y, LIN), 1 / 2.4 - 1))


def tonemap(x):
    x = np.asarray(x, np.float64)
    return srgb(np.log(np.maximum(x, 0) + 1))


def tonemap_d(x):
    x = np.asarray(x, np.float64)
    xp = np.maximum(x, 0)
    return np.where(x > 0, srgb_d(np.log(xp + 1)) / (xp + 1), 0.0)


def image_loss(kd, c_d, c_s, ref, mask, w_light=0.15):
    """All per-pixel inputs [3][N]; mask [N].  Returns (L_image, L_light,
    g_kd, g_cd, g_cs) of L = L_image + w_light * L_light."""
    kd, c_d, c_s, ref = (np.asarray(a, np.float64) for a in (kd, c_d, c_s, ref))
    m = np.asarray(mask) > 0
    n = max(int(m.sum()), 1)
    c = kd * c_d + c_s
    diff = tonemap(c) - tonemap(ref)
    L_img = float(np.abs(diff)[:, m].sum() / (3 * n))
    gc = np.sign(diff) * tonemap_d(c) / (3 * n) * m
    lsum = c_d + c_s
    y = tonemap(lsum).mean(0)
    v = tonemap(ref).max(0)
    dl = y - v
    L_light = float(np.abs(dl)[m].sum() / n)
    gl = (np.sign(dl) / n * m)[None, :] * tonemap_d(lsum) / 3.0 * w_light
    g_kd = gc * c_d
    g_cd = gc * kd + gl
    g_cs = gc + gl
    return L_img, L_light, g_kd, g_cd, g_cs

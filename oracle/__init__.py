"""FP64 CPU oracle of the Monte Carlo direct-illumination estimator.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline leg import this package.  The product (the HIP library and its
binding) never does.  The C source `mcdi_oracle.c` is compiled with gcc into
`liboracle.so` next to it; nothing here is shared with the HIP path.
"""

import ctypes as C
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcdi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# decision-record flag bits
DEC_LOBE_COS, DEC_L_CULL, DEC_B_CULL = 1 << 0, 1 << 1, 1 << 2
DEC_L_TRACED, DEC_B_TRACED, DEC_L_HIT, DEC_B_HIT = 1 << 3, 1 << 4, 1 << 5, 1 << 6
DEC_NOV_POS, DEC_VALID = 1 << 7, 1 << 8
DEC_NONE = 0xFFFFFFFF
LIGHT_OFF, FORCE_COS, BSDF_OFF, FORCE_GGX, BILINEAR = 1, 2, 4, 8, 16
TRI_MISS, TRI_HIT, TRI_NEAR = 0, 1, 2


def build(force=True):
    """Compile the oracle (-O2, no fast-math, no FP contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class Env(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("env", C.c_void_p), ("cond", C.c_void_p),
                ("marg", C.c_void_p), ("pdf", C.c_void_p), ("light_enabled", C.c_int32)]


class GBuf(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("height", C.c_int32), ("width", C.c_int32),
                ("view_base", C.c_int32), ("pos", C.c_void_p), ("nrm", C.c_void_p),
                ("kd", C.c_void_p), ("korm", C.c_void_p), ("mask", C.c_void_p), ("eye", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("spp", C.c_int32), ("flags", C.c_uint32), ("seed", C.c_uint64), ("tau", C.c_double),
                ("ray_eps", C.c_double), ("delta_vis_abs", C.c_double), ("delta_vis_rel", C.c_double),
                ("delta_ang", C.c_double), ("delta_cos", C.c_double), ("brute", C.c_int32),
                ("dir_light", C.c_double), ("dir_cos", C.c_double), ("dir_ggx0", C.c_double),
                ("dir_ggx1", C.c_double), ("dir_arg", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.orc_scene_build.restype = vp
        L.orc_scene_build.argtypes = [vp, C.c_int64, vp, C.c_int64]
        L.orc_scene_free.argtypes = [vp]
        L.orc_env_tables.restype = C.c_int
        L.orc_env_tables.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp]
        L.orc_shade.restype = C.c_int64
        L.orc_shade.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, vp, vp, C.c_int, vp, vp, vp, vp, vp,
                                vp, vp, vp, vp, vp, vp, vp, vp, C.c_int32, vp, vp, vp, C.c_int]
        L.orc_batch_philox.argtypes = [C.c_int64, vp, vp, vp]
        L.orc_batch_uniforms.argtypes = [C.c_int64, C.c_uint64, vp, vp, vp, vp]
        L.orc_batch_sample_light.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_batch_pdf_light.argtypes = [vp, C.c_int64, vp, vp]
        L.orc_batch_texel_of_dir.argtypes = [C.c_int, C.c_int, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.orc_batch_pdf_ggx_local.argtypes = [C.c_int64, vp, C.c_double, vp, vp]
        L.orc_batch_pdf_cos_local.argtypes = [C.c_int64, vp, vp]
        L.orc_batch_sample_vndf_local.argtypes = [C.c_int64, vp, C.c_double, vp, vp, vp]
        L.orc_batch_sample_cos_local.argtypes = [C.c_int64, vp, vp, vp]
        L.orc_batch_ggx.argtypes = [C.c_int64, vp, vp, vp, C.c_double, vp, vp]
        L.orc_batch_anyhit.argtypes = [vp, C.c_int64, vp, vp, C.c_double, C.c_double, C.c_int, vp]
        L.orc_integrand.argtypes = [vp, vp, vp, C.c_int64, vp, C.c_int64, vp, vp, vp]
        L.orc_batch_probe_bilinear.argtypes = [vp, C.c_int, C.c_int, C.c_int64, vp, vp, vp]
        L.orc_max_threads.restype = C.c_int
        L.orc_edge_grad.restype = C.c_int
        L.orc_edge_sharp.argtypes = [vp, vp, C.c_int64, vp]
        L.orc_edge_grad.argtypes = [vp, vp, vp, vp, C.c_int64, vp, C.c_int32, vp, C.c_int64, vp, C.c_int64,
                                    vp, vp, vp, vp, vp, vp, vp, C.c_int, C.c_uint32]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------

def philox(ctr, key):
    ctr = _c(ctr, np.uint32).reshape(-1, 4)
    key = _c(key, np.uint32).reshape(2)
    out = np.empty_like(ctr)
    lib().orc_batch_philox(len(ctr), _p(ctr), _p(key), _p(out))
    return out


def uniforms(seed, pix, view, s):
    pix, view, s = (_c(x, np.uint32).reshape(-1) for x in (pix, view, s))
    xi = np.empty((len(pix), 8))
    lib().orc_batch_uniforms(len(pix), C.c_uint64(seed), _p(pix), _p(view), _p(s), _p(xi))
    return xi


class EnvTables:
    """FP32 sampling tables of a lat-long probe, built by the oracle."""

    def __init__(self, env):
        self.env = _c(env, np.float32)
        H, W = self.env.shape[:2]
        self.H, self.W = H, W
        self.cond = np.empty((H, W + 1), np.float32)
        self.marg = np.empty(H + 1, np.float32)
        self.pdf = np.empty((H, W), np.float32)
        tot = C.c_double()
        self.light_enabled = lib().orc_env_tables(_p(self.env), H, W, _p(self.cond), _p(self.marg),
                                                  _p(self.pdf), C.byref(tot))
        self.total = tot.value
        self.struct = Env(H, W, self.env.ctypes.data, self.cond.ctypes.data, self.marg.ctypes.data,
                          self.pdf.ctypes.data, self.light_enabled)

    def sample(self, xi0, xi1, coords=False):
        """Light-technique samples: direction, density, texel (i, j) and,
        with coords, the continuous texel coordinates (x, y) of the sample."""
        xi0, xi1 = _c(xi0, np.float64), _c(xi1, np.float64)
        n = len(xi0)
        w, p = np.empty((n, 3)), np.empty(n)
        ti, tj = np.empty(n, np.int32), np.empty(n, np.int32)
        x, y = np.empty(n), np.empty(n)
        lib().orc_batch_sample_light(C.byref(self.struct), n, _p(xi0), _p(xi1), _p(w), _p(p), _p(ti), _p(tj),
                                     _p(x), _p(y))
        return (w, p, ti, tj, x, y) if coords else (w, p, ti, tj)

    def pdf_dir(self, w):
        w = _c(w, np.float64).reshape(-1, 3)
        p = np.empty(len(w))
        lib().orc_batch_pdf_light(C.byref(self.struct), len(w), _p(w), _p(p))
        return p

    def texel_of_dir(self, w, coords=False):
        """Nearest texel (i, j) of unit directions and the angular margin to
        the closest texel boundary; with coords, also the continuous texel
        coordinates (x, y) = (phi W / 2 pi, theta H / pi)."""
        w = _c(w, np.float64).reshape(-1, 3)
        n = len(w)
        ti, tj, m = np.empty(n, np.int32), np.empty(n, np.int32), np.empty(n)
        x, y = np.empty(n), np.empty(n)
        lib().orc_batch_texel_of_dir(self.H, self.W, n, _p(w), _p(ti), _p(tj), _p(m), _p(x), _p(y))
        return (ti, tj, m, x, y) if coords else (ti, tj, m)


def probe_bilinear(env, x, y):
    """Bilinear reconstruction of an [H, W, 3] probe at continuous texel
    coordinates (x, y) = (phi W / 2 pi, theta H / pi); texel centres at
    (j + 1/2, i + 1/2), columns wrap, rows clamp."""
    env = _c(env, np.float32)
    H, W = env.shape[:2]
    x, y = _c(x, np.float64).reshape(-1), _c(y, np.float64).reshape(-1)
    L = np.empty((len(x), 3))
    lib().orc_batch_probe_bilinear(_p(env), H, W, len(x), _p(x), _p(y), _p(L))
    return L


def pdf_ggx_local(V, alpha, L):
    V, L = _c(V, np.float64), _c(L, np.float64).reshape(-1, 3)
    p = np.empty(len(L))
    lib().orc_batch_pdf_ggx_local(len(L), _p(V), alpha, _p(L), _p(p))
    return p


def pdf_cos_local(L):
    L = _c(L, np.float64).reshape(-1, 3)
    p = np.empty(len(L))
    lib().orc_batch_pdf_cos_local(len(L), _p(L), _p(p))
    return p


def sample_vndf_local(V, alpha, u1, u2):
    V, u1, u2 = _c(V, np.float64), _c(u1, np.float64), _c(u2, np.float64)
    L = np.empty((len(u1), 3))
    lib().orc_batch_sample_vndf_local(len(u1), _p(V), alpha, _p(u1), _p(u2), _p(L))
    return L


def sample_cos_local(u1, u2):
    u1, u2 = _c(u1, np.float64), _c(u2, np.float64)
    L = np.empty((len(u1), 3))
    lib().orc_batch_sample_cos_local(len(u1), _p(u1), _p(u2), _p(L))
    return L


def ggx(noh, s2, nov, alpha):
    noh, s2, nov = (_c(x, np.float64) for x in (noh, s2, nov))
    D, lam = np.empty(len(noh)), np.empty(len(noh))
    lib().orc_batch_ggx(len(noh), _p(noh), _p(s2), _p(nov), alpha, _p(D), _p(lam))
    return D, lam


class Scene:
    def __init__(self, verts, tris):
        self.verts = _c(verts, np.float32)
        self.tris = _c(tris, np.int32)
        self.ptr = lib().orc_scene_build(_p(self.verts), len(self.verts), _p(self.tris), len(self.tris))

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.orc_scene_free(self.ptr)
            self.ptr = None

    def anyhit(self, o, d, delta_abs=0.0, delta_rel=0.0, brute=False):
        o, d = _c(o, np.float64).reshape(-1, 3), _c(d, np.float64).reshape(-1, 3)
        out = np.empty(len(o), np.int32)
        lib().orc_batch_anyhit(self.ptr, len(o), _p(o), _p(d), delta_abs, delta_rel, int(brute), _p(out))
        return out


# ---------------------------------------------------------------------------
# the estimator
# ---------------------------------------------------------------------------

class Tolerances:
    """Decision tolerances of the parity protocol: a discrete decision whose
    margin is below these (visibility: absolute and relative edge distance;
    texel boundaries: radians of arc; signs of n.v and n.l: cosine) is
    undecided in FP32, so the oracle adopts the kernel's dumped decision
    there or flags it.

    dir: the direction-error model of an FP32 evaluation of the sampling
    chains, a dict of counts in units of u = 2^-24 (keys light, cos, ggx0,
    ggx1, arg; see orc_params in mcdi_oracle.c), or None.  With it the oracle
    reports, per output, the conditioning of its terms in their sampled
    directions (`<name>_cond`), widens the texel and horizon decisions by twice
    each sample's bound, and bounds the bilinear lookup's coordinate error by
    it.  Without it no conditioning is computed."""

    def __init__(self, vis_abs=1e-5, vis_rel=1e-5, ang=2e-5, cos=1e-5, dir=None):
        self.vis_abs, self.vis_rel, self.ang, self.cos = vis_abs, vis_rel, ang, cos
        self.dir = dict(dir) if dir else None

    def params(self, spp, flags, seed, tau, ray_eps, brute):
        d = self.dir or {}
        return Params(spp, flags, seed, tau, ray_eps, self.vis_abs, self.vis_rel, self.ang, self.cos, int(brute),
                      float(d.get("light", 0.0)), float(d.get("cos", 0.0)), float(d.get("ggx0", 0.0)),
                      float(d.get("ggx1", 0.0)), float(d.get("arg", 0.0)))


def _gbuf_struct(w, arrays):
    pos, nrm, kd, korm, mask, eye = arrays
    return GBuf(w.n_views, w.height, w.width, w.view_base, pos.ctypes.data, nrm.ctypes.data,
                kd.ctypes.data, korm.ctypes.data, mask.ctypes.data, eye.ctypes.data)


def _gb_arrays(w, override=None):
    override = override or {}
    get = lambda k, dt: _c(override.get(k, getattr(w, k)), dt)  # noqa: E731
    return (get("pos", np.float32), get("nrm", np.float32), get("kd", np.float32),
            get("korm", np.float32), get("mask", np.uint8), get("eye", np.float32))


def shade(w, pixels=None, scene=None, tables=None, spp=None, seed=None, tau=None, ray_eps=None,
          flags=0, grad=False, u_d=None, u_s=None, sync=None, eval_override=None, env_eval=None,
          tol=None, brute=False, threads=0, want_decisions=False, want_dirs=False):
    """Run the oracle forward (grad=False) or backward (grad=True) on the
    listed pixels of workload `w` (all pixels if None).

    eval_override: dict of G-buffer arrays replacing the evaluation-side
    inputs (the frozen-sample finite-difference hook); env_eval likewise for
    the probe radiance.  Returns a dict of FP64 arrays in pixel-list order:
    the outputs, and per output `<name>_abs` (sum of the absolute values of
    the summands of its terms), `<name>_cond` (conditioning of its terms in
    their sampled directions; 0 without a direction model in `tol`) and
    `<name>_lerr` (bound on the radiance lookup's own FP32 error); with
    want_dirs, `dirs` [n, spp, 2, 4]: each sample's direction (light, then
    BSDF technique) and its direction-error bound, NaN where none was drawn."""
    L = lib()
    spp = w.spp if spp is None else spp
    seed = w.seed if seed is None else seed
    # tau and ray_eps are FP32 parameters of the library: use the same values
    tau = float(np.float32(w.tau if tau is None else tau))
    ray_eps = float(np.float32(w.ray_eps if ray_eps is None else ray_eps))
    tol = tol or Tolerances()
    pixels = np.arange(w.n_pixels, dtype=np.int64) if pixels is None else _c(pixels, np.int64)
    n = len(pixels)
    scene = scene or Scene(w.verts, w.tris)
    tables = tables or EnvTables(w.env)
    gs_arr = _gb_arrays(w)
    gs = _gbuf_struct(w, gs_arr)
    ge_arr = ge = None
    if eval_override is not None:
        ge_arr = _gb_arrays(w, eval_override)
        ge = _gbuf_struct(w, ge_arr)
    env_ev = _c(env_eval, np.float32) if env_eval is not None else None
    prm = tol.params(spp, flags, seed, tau, ray_eps, brute)
    hw = (2 * spp + 31) // 32
    out = {"c_d": np.zeros((3, n)), "c_s": np.zeros((3, n)), "hitbits": np.zeros((n, hw), np.uint32),
           "info": np.zeros((n, 3), np.int32)}
    sync_arr = _c(sync, np.uint32) if sync is not None else None
    dec = np.zeros((n, spp, 3), np.uint32) if want_decisions else None
    ud = us = None
    if grad:
        ud = _c(u_d, np.float64).reshape(3, n)
        us = _c(u_s, np.float64).reshape(3, n)
        out.update(g_kd=np.zeros((3, n)), g_korm=np.zeros((3, n)), g_nrm=np.zeros((3, n)),
                   g_env=np.zeros(tables.env.shape), s_env=np.zeros(tables.env.shape),
                   c_env=np.zeros(tables.env.shape), l_env=np.zeros(tables.env.shape))
    vaux = np.zeros((3, 15, n))
    dirs = np.zeros((n, spp, 2, 4)) if want_dirs else None
    r = L.orc_shade(scene.ptr, C.byref(tables.struct), _p(env_ev), C.byref(gs),
                    C.byref(ge) if ge is not None else None, _p(pixels), n, C.byref(prm),
                    _p(sync_arr), int(grad), _p(ud), _p(us), _p(out["c_d"]), _p(out["c_s"]), _p(vaux),
                    _p(out.get("g_kd")), _p(out.get("g_korm")), _p(out.get("g_nrm")),
                    _p(out.get("g_env")), _p(out.get("s_env")), _p(out.get("c_env")), _p(out.get("l_env")),
                    _p(out["hitbits"]), hw, _p(dec), _p(dirs),
                    _p(out["info"]), int(threads))
    if r < 0:
        raise ValueError("oracle rejected the parameters (spp must be in [1, 1024])")
    out["nonfinite"] = int(r)
    for kind, suffix in enumerate(("_abs", "_cond", "_lerr")):
        for k, name in enumerate(("c_d", "c_s", "g_kd", "g_korm", "g_nrm")):
            out[name + suffix] = vaux[kind, 3 * k:3 * k + 3]
    if dec is not None:
        out["decisions"] = dec
    if dirs is not None:
        out["dirs"] = dirs
    return out


def integrand(w, pixel, dirs, scene=None, tables=None, tau=None, ray_eps=None, brute=True, flags=0):
    """Direct-illumination integrand (g_d, g_s) of one pixel at unit directions
    (probe radiance by the nearest texel, or bilinear with BILINEAR in flags)."""
    scene = scene or Scene(w.verts, w.tris)
    tables = tables or EnvTables(w.env)
    arr = _gb_arrays(w)
    gs = _gbuf_struct(w, arr)
    tau = w.tau if tau is None else tau
    ray_eps = w.ray_eps if ray_eps is None else ray_eps
    prm = Tolerances(0.0, 0.0, 0.0, 0.0).params(1, flags & BILINEAR, 0, tau, ray_eps, brute)
    dirs = _c(dirs, np.float64).reshape(-1, 3)
    gd, gsp = np.empty((len(dirs), 3)), np.empty((len(dirs), 3))
    lib().orc_integrand(scene.ptr, C.byref(tables.struct), C.byref(gs), int(pixel), C.byref(prm),
                        len(dirs), _p(dirs), _p(gd), _p(gsp))
    return gd, gsp


def max_threads():
    return lib().orc_max_threads()


# ---------------------------------------------------------------------------
# visibility gradients of the shadow term by edge sampling
# ---------------------------------------------------------------------------

def mesh_edges(tris, n_verts):
    """Unique undirected edges of an indexed triangle mesh, [E, 4] int32 rows
    (a, b, c, d): the edge a-b as it first appears (triangle f, side k runs
    from corner k to corner k+1), c the opposite corner of that face, d the
    opposite corner of the second face that has the edge (-1 if none).
    Rows are in order of first appearance, f-major then k.  A triangle with
    a corner outside [0, n_verts) contributes nothing, nor does a side whose
    two corners are the same vertex; faces after the second are ignored."""
    tris = np.asarray(tris, np.int64).reshape(-1, 3)
    first = {}
    rows = []
    for f in range(len(tris)):
        t = tris[f]
        if (t < 0).any() or (t >= n_verts).any():
            continue
        for k in range(3):
            a, b, c = int(t[k]), int(t[(k + 1) % 3]), int(t[(k + 2) % 3])
            if a == b:
                continue
            key = (a, b) if a < b else (b, a)
            at = first.get(key)
            if at is None:
                first[key] = len(rows)
                rows.append([a, b, c, -1])
            elif rows[at][3] == -1:
                rows[at][3] = c
    return np.array(rows, np.int32).reshape(-1, 4)


def edge_sharp(verts, edges):
    """Sampling class of each edge row: True where the edge is sharp (one face,
    or face normals more than 20 degrees apart, decided in FP32)."""
    verts = _c(verts, np.float32)
    edges = _c(edges, np.int32).reshape(-1, 4)
    out = np.empty(len(edges), np.int32)
    lib().orc_edge_sharp(_p(verts), _p(edges), len(edges), _p(out))
    return out.astype(bool)


def edge_grad(w, edges, n_es, u_d, u_s, pixels=None, scene=None, tables=None, seed=None, tau=None,
              ray_eps=None, flags=0, tol=None, brute=False, threads=0, sharp_gain=1):
    """Edge-sampled derivative of sum_pixels (u_d . c_d + u_s . c_s) with
    respect to the mesh vertices through the shadow-ray visibility, from
    n_es edge samples per pixel (sharp edges sharp_gain times as likely per
    edge as the others; 1 is a uniform choice; every gain has the same
    expectation).  Returns a dict: g_verts [Nv, 3] and, per
    element, abs (sum of |term|), cond (FP32 error bound of the terms),
    flag (bound on the terms of samples with an undecided step), plus the
    sample counts."""
    L = lib()
    seed = w.seed if seed is None else seed
    tau = float(np.float32(w.tau if tau is None else tau))
    ray_eps = float(np.float32(w.ray_eps if ray_eps is None else ray_eps))
    tol = tol or Tolerances()
    pixels = np.arange(w.n_pixels, dtype=np.int64) if pixels is None else _c(pixels, np.int64)
    n = len(pixels)
    scene = scene or Scene(w.verts, w.tris)
    tables = tables or EnvTables(w.env)
    arr = _gb_arrays(w)
    gs = _gbuf_struct(w, arr)
    prm = tol.params(1, flags, seed, tau, ray_eps, brute)
    edges = _c(edges, np.int32).reshape(-1, 4)
    verts = _c(w.verts, np.float32)
    nv = len(verts)
    ud = _c(u_d, np.float64).reshape(3, -1)
    us = _c(u_s, np.float64).reshape(3, -1)
    if ud.shape[1] != n:
        ud, us = np.ascontiguousarray(ud[:, pixels]), np.ascontiguousarray(us[:, pixels])
    out = {k: np.zeros((nv, 3)) for k in ("g_verts", "abs", "cond", "flag")}
    counts = np.zeros(5, np.int64)
    r = L.orc_edge_grad(scene.ptr, C.byref(tables.struct), C.byref(gs), _p(pixels), n, C.byref(prm), int(n_es),
                        _p(edges), len(edges), _p(verts), nv, _p(ud), _p(us), _p(out["g_verts"]),
                        _p(out["abs"]), _p(out["cond"]), _p(out["flag"]), _p(counts), int(threads),
                        int(sharp_gain))
    if r < 0:
        raise ValueError("oracle rejected the edge-gradient arguments")
    out.update(samples=int(counts[0]), silhouettes=int(counts[1]), traced=int(counts[2]),
               blocked=int(counts[3]), flagged=int(counts[4]))
    return out

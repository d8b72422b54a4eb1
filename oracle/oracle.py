"""ctypes front-end of the FP64 oracle (``oracle.c``).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It never touches the GPU path and
the GPU path never imports it.

Inputs are the float32 masters produced by ``hg_inputs``; outputs are float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-Wall", "-shared", "-fPIC"]

DIFFUSE_ONLY = 1
HARD_VIS = 2
MIS = 4


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no fast-math, no FMA
    contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


MAXL = 32


class Grid(C.Structure):
    _fields_ = [("L", C.c_int32), ("F", C.c_int32), ("log2_T", C.c_int32),
                ("res", C.c_int32 * MAXL), ("lo", C.c_double), ("extent", C.c_double),
                ("table", C.c_void_p)]


class MLP(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32),
                ("W0", C.c_void_p), ("b0", C.c_void_p), ("W1", C.c_void_p),
                ("b1", C.c_void_p), ("W2", C.c_void_p), ("b2", C.c_void_p)]


class Model(C.Structure):
    _fields_ = [("grid", Grid), ("brdf", MLP), ("irt", MLP), ("t_near", C.c_double),
                ("t_far", C.c_double), ("f0", C.c_double)]


class Env(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("rgb", C.c_void_p)]


class Sampling(C.Structure):
    _fields_ = [("n_dirs", C.c_int32), ("n_dirs2", C.c_int32), ("seed", C.c_uint64),
                ("flags", C.c_uint32)]


class Points(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("nrm", C.c_void_p),
                ("wo", C.c_void_p), ("dir", C.c_void_p), ("pid", C.c_void_p)]


_lib = None


def _set_types(h):
    h.or_l2_loss.restype = C.c_double
    h.or_render.restype = C.c_int32
    h.or_backward.restype = C.c_int32


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _set_types(_lib)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleModel:
    """Holds contiguous float32 copies of a model's parameters and the ctypes
    descriptors pointing at them (kept alive by this object)."""

    def __init__(self, model: dict, box_lo: float, box_extent: float, t_near=0.05, t_far=1.5,
                 f0=0.04):
        self.table = _f32(model["table"])
        self.brdf = [_f32(a) for a in model["brdf"]]
        self.irt = [_f32(a) for a in model["irt"]]
        L, T, F = self.table.shape
        g = Grid()
        g.L, g.F, g.log2_T = L, F, int(T).bit_length() - 1
        for i, r in enumerate(model["res"]):
            g.res[i] = int(r)
        g.lo, g.extent, g.table = box_lo, box_extent, _p(self.table)
        m = Model()
        m.grid = g
        m.brdf = self._mlp(self.brdf)
        m.irt = self._mlp(self.irt)
        m.t_near, m.t_far, m.f0 = t_near, t_far, f0
        self.c = m
        self.L, self.F, self.T = L, F, T

    @staticmethod
    def _mlp(ws):
        m = MLP()
        m.n_hidden, m.n_in = ws[0].shape
        m.n_out = ws[4].shape[0]
        m.W0, m.b0, m.W1, m.b1, m.W2, m.b2 = [_p(a) for a in ws]
        return m

    def n_brdf_params(self):
        return sum(a.size for a in self.brdf)

    def n_irt_params(self):
        return sum(a.size for a in self.irt)


class OracleEnv:
    def __init__(self, env):
        self.rgb = _f32(env)
        e = Env()
        e.H, e.W = self.rgb.shape[:2]
        e.rgb = _p(self.rgb)
        self.c = e


def sampling(n_dirs, n_dirs2=8, seed=7, flags=0):
    s = Sampling()
    s.n_dirs, s.n_dirs2, s.seed, s.flags = n_dirs, n_dirs2, seed, flags
    return s


def _points(pos, nrm=None, wo=None, dirs=None, pid=None):
    keep = [_f32(pos), None if nrm is None else _f32(nrm), None if wo is None else _f32(wo),
            None if dirs is None else _f32(dirs),
            None if pid is None else np.ascontiguousarray(pid, dtype=np.uint32)]
    P = Points()
    P.n = keep[0].shape[0]
    P.pos, P.nrm, P.wo, P.dir, P.pid = [_p(a) for a in keep]
    return P, keep


# --------------------------------------------------------------------------
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return list(o)


def uniforms(seed, pid, q, k, tag):
    pid, q, k = [np.ascontiguousarray(a, np.uint32) for a in (pid, q, k)]
    out = np.empty((pid.size, 2))
    lib().or_uniforms(C.c_uint64(seed), _p(pid), _p(q), _p(k), C.c_uint32(tag),
                      C.c_int64(pid.size), _p(out))
    return out


def sample_dirs(seed, nrm, pid, q, k, tag, nstrata):
    nrm = _f64(nrm)
    pid, q, k = [np.ascontiguousarray(np.broadcast_to(a, (nrm.shape[0],)), np.uint32)
                 for a in (pid, q, k)]
    out = np.empty_like(nrm)
    lib().or_sample_dirs(C.c_uint64(seed), _p(nrm), _p(pid), _p(q), _p(k), C.c_uint32(tag),
                         C.c_int32(nstrata), C.c_int64(nrm.shape[0]), _p(out))
    return out


def encode(om: OracleModel, pos):
    pos = _f32(pos)
    out = np.empty((pos.shape[0], om.L * om.F))
    lib().or_encode(C.byref(om.c.grid), _p(pos), C.c_int64(pos.shape[0]), _p(out))
    return out


def encode_f64(om: OracleModel, pos):
    pos = _f64(pos)
    out = np.empty((pos.shape[0], om.L * om.F))
    lib().or_encode_f64(C.byref(om.c.grid), _p(pos), C.c_int64(pos.shape[0]), _p(out))
    return out


def encode_index(om: OracleModel, pos):
    pos = _f32(pos)
    n = pos.shape[0]
    idx = np.empty((n, om.L, 8), np.uint32)
    w = np.empty((n, om.L, 3))
    lib().or_encode_index(C.byref(om.c.grid), _p(pos), C.c_int64(n), _p(idx), _p(w))
    return idx, w


def mlp_forward(om: OracleModel, which: str, x):
    x = _f64(x)
    m = om.c.brdf if which == "brdf" else om.c.irt
    out = np.empty((x.shape[0], m.n_out))
    lib().or_mlp_forward(C.byref(m), _p(x), C.c_int64(x.shape[0]), _p(out))
    return out


def env_lookup(oe: OracleEnv, dirs):
    dirs = _f64(dirs)
    out = np.empty_like(dirs)
    lib().or_env_lookup(C.byref(oe.c), _p(dirs), C.c_int64(dirs.shape[0]), _p(out))
    return out


def env_dist(oe: OracleEnv):
    """Light-sampling distribution of an environment map: (cos theta at the
    row edges [H+1], marginal CDF [H+1], conditional CDFs [H][W+1], texel
    solid-angle densities [H][W])."""
    H, W = oe.c.H, oe.c.W
    ct, marg = np.empty(H + 1), np.empty(H + 1)
    cond, dens = np.empty((H, W + 1)), np.empty((H, W))
    lib().or_env_dist(C.byref(oe.c), _p(ct), _p(marg), _p(cond), _p(dens))
    return ct, marg, cond, dens


def env_sample(oe: OracleEnv, s):
    """Light samples for uniforms s [n][2] in (0,1): directions [n][3], densities [n]."""
    s = _f64(s)
    n = s.shape[0]
    w, pdf = np.empty((n, 3)), np.empty(n)
    lib().or_env_sample(C.byref(oe.c), _p(s), C.c_int64(n), _p(w), _p(pdf))
    return w, pdf


def env_density(oe: OracleEnv, w):
    w = _f64(w)
    pdf = np.empty(w.shape[0])
    lib().or_env_density(C.byref(oe.c), _p(w), C.c_int64(w.shape[0]), _p(pdf))
    return pdf


def ggx_sample(n, v, r, s):
    """GGX visible-normal samples: reflected directions [cnt][3]."""
    n, v, r, s = _f64(n), _f64(v), _f64(r), _f64(s)
    out = np.empty((n.shape[0], 3))
    lib().or_ggx_sample(_p(n), _p(v), _p(r), _p(s), C.c_int64(n.shape[0]), _p(out))
    return out


def ggx_density(n, v, r, l):
    n, v, r, l = _f64(n), _f64(v), _f64(r), _f64(l)
    out = np.empty(n.shape[0])
    lib().or_ggx_density(_p(n), _p(v), _p(r), _p(l), C.c_int64(n.shape[0]), _p(out))
    return out


def brdf(n, v, l, a, r, m, f0=0.04, diffuse_only=False):
    n, v, l, a = [_f64(x) for x in (n, v, l, a)]
    r, m = _f64(r), _f64(m)
    cnt = n.shape[0]
    f = np.empty((cnt, 3)); dfa = np.empty((cnt, 3)); dfr = np.empty((cnt, 3)); dfm = np.empty((cnt, 3))
    lib().or_brdf(_p(n), _p(v), _p(l), _p(a), _p(r), _p(m), C.c_double(f0), C.c_int32(int(diffuse_only)),
                  C.c_int64(cnt), _p(f), _p(dfa), _p(dfr), _p(dfm))
    return f, dfa, dfr, dfm


def render(om: OracleModel, oe: OracleEnv, samp: Sampling, pos, nrm=None, wo=None, dirs=None,
           indirect=True, want_vis=True, pid=None):
    """Shade mode (dirs None): rgb [n,3], vis/depth [n,N].  Query mode:
    rgb [n,3], vis [n], depth [n].  pid: the points' ids in the sampler's
    counter (default 0..n-1), for evaluating a subset of a larger batch."""
    if dirs is None and (nrm is None or wo is None):
        raise ValueError("shade mode needs nrm and wo (pass dirs= for query mode)")
    P, keep = _points(pos, nrm, wo, dirs, pid)
    n = P.n
    rgb = np.empty((n, 3))
    if dirs is None:
        vis = np.empty((n, samp.n_dirs)) if want_vis else None
        dep = np.empty((n, samp.n_dirs)) if want_vis else None
    else:
        vis = np.empty(n)
        dep = np.empty(n)
    rc = lib().or_render(C.byref(om.c), C.byref(oe.c), C.byref(samp), C.byref(P),
                         C.c_int32(int(indirect)), _p(rgb), _p(vis), _p(dep))
    del keep
    if rc != 0:
        raise ValueError("or_render rejected its arguments (a required pointer is NULL)")
    return rgb, vis, dep


def l2_loss(rgb, vis, dep, tgt):
    rgb, vis, dep, tgt = [_f32(a) for a in (rgb, vis, dep, tgt)]
    n = vis.shape[0]
    g_rgb = np.empty((n, 3)); g_vis = np.empty(n); g_dep = np.empty(n)
    loss = lib().or_l2_loss(_p(rgb), _p(vis), _p(dep), _p(tgt), C.c_int64(n), _p(g_rgb), _p(g_vis),
                            _p(g_dep))
    return loss, g_rgb, g_vis, g_dep


def split_mlp_grad(flat, ws):
    out, o = [], 0
    for a in ws:
        out.append(flat[o:o + a.size].reshape(a.shape))
        o += a.size
    return out


def backward(om: OracleModel, oe: OracleEnv, samp: Sampling, pos, dirs, g_rgb, g_vis, g_dep,
             indirect=True, want_pos=False, pid=None):
    """Gradients of sum_p (g_rgb.rgb + g_vis*vis + g_dep*depth) in query mode.
    Returns dict(table [L,T,F], brdf [6 arrays], irt [6 arrays], pos [n,3]|None).
    Defined for the 5-output decoder (facing normal at the bounce point)."""
    if om.c.brdf.n_out != 5:
        raise ValueError("the oracle backward covers the 5-output decoder only")
    P, keep = _points(pos, None, None, dirs, pid)
    g_rgb, g_vis, g_dep = _f32(g_rgb), _f32(g_vis), _f32(g_dep)
    gt = np.zeros(om.table.shape)
    gb = np.zeros(om.n_brdf_params())
    gi = np.zeros(om.n_irt_params())
    gp = np.zeros((P.n, 3)) if want_pos else None
    rc = lib().or_backward(C.byref(om.c), C.byref(oe.c), C.byref(samp), C.byref(P),
                           C.c_int32(int(indirect)), _p(g_rgb), _p(g_vis), _p(g_dep), _p(gt), _p(gb),
                           _p(gi), _p(gp))
    del keep
    if rc != 0:
        raise ValueError("or_backward rejected its arguments (a required pointer is NULL)")
    return dict(table=gt, brdf=split_mlp_grad(gb, om.brdf), irt=split_mlp_grad(gi, om.irt), pos=gp)


def adam(param, grad, m, v, step, lr=2e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam step in FP64; returns new (param, m, v)."""
    p = _f64(param).copy(); g = _f64(grad); m = _f64(m).copy(); v = _f64(v).copy()
    lib().or_adam(_p(p), _p(g), _p(m), _p(v), C.c_int64(p.size), C.c_int32(step), C.c_double(lr),
                  C.c_double(b1), C.c_double(b2), C.c_double(eps), C.c_double(wd))
    return p, m, v


def denoise(rgb, depth, nrm, iters=5, sigma_z=1.0, sigma_n=128.0, sigma_l=4.0, return_var=False):
    """Spatial SVGF filter of an [H, W, 3] image with depth [H, W] and normal
    [H, W, 3] guides; returns [H, W, 3] float64 (and, with return_var, the
    luminance variance [H, W] carried out of the last iteration)."""
    rgb, depth, nrm = _f32(rgb), _f32(depth), _f32(nrm)
    H, W = depth.shape
    out = np.empty((H, W, 3))
    var = np.empty((H, W)) if return_var else None
    lib().or_denoise(_p(rgb), _p(depth), _p(nrm), C.c_int32(H), C.c_int32(W), C.c_int32(iters),
                     C.c_double(sigma_z), C.c_double(sigma_n), C.c_double(sigma_l), _p(out), _p(var))
    return (out, var) if return_var else out


def brdf_terms(n, v, l, r):
    """Specular factors per sample: GGX D, the height-correlated Smith
    visibility Vis = G2 / (4 n.l n.v) and the Schlick weight (1 - v.h)^5."""
    n, v, l, r = _f64(n), _f64(v), _f64(l), _f64(r)
    cnt = n.shape[0]
    D, Vis, P = np.empty(cnt), np.empty(cnt), np.empty(cnt)
    lib().or_brdf_terms(_p(n), _p(v), _p(l), _p(r), C.c_int64(cnt), _p(D), _p(Vis), _p(P))
    return D, Vis, P

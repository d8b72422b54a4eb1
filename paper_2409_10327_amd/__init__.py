"""Python binding of libhg.so, the gfx950 hash-grid secondary-ray renderer.

Argument marshalling only: every step of the renderer runs in the HIP
kernels behind the C ABI declared in include/hg.h.  PyTorch supplies device
memory (tensors) and the current HIP stream.  If the library is missing the
import of any entry point raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhg.so")

HG_OK, HG_E_INVALID, HG_E_UNSUPPORTED, HG_E_WORKSPACE, HG_E_HIP = range(5)
HG_F32, HG_F16, HG_BF16 = 0, 1, 2
HG_DIFFUSE_ONLY = 1
HG_HARD_VIS = 2
HG_MIS = 4

BOX_LO = -8.0
BOX_EXTENT = 16.0


class HGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hg status {status}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("L", C.c_int32), ("F", C.c_int32), ("log2_T", C.c_int32), ("res", C.c_int32 * 32),
                ("box_lo", C.c_float), ("box_extent", C.c_float), ("dtype", C.c_int32), ("table", C.c_void_p)]


class Mlp(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32), ("dtype", C.c_int32),
                ("W", C.c_void_p * 3), ("b", C.c_void_p * 3)]


class Model(C.Structure):
    _fields_ = [("grid", Grid), ("brdf", Mlp), ("irt", Mlp), ("t_near", C.c_float), ("t_far", C.c_float),
                ("f0", C.c_float)]


class Env(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("rgb", C.c_void_p), ("dist", C.c_void_p)]


class Sampling(C.Structure):
    _fields_ = [("n_dirs", C.c_int32), ("n_dirs2", C.c_int32), ("seed", C.c_uint64), ("flags", C.c_uint32)]


class DenoiseParams(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("sigma_z", C.c_float), ("sigma_n", C.c_float), ("sigma_l", C.c_float)]


class Points(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("nrm", C.c_void_p), ("wo", C.c_void_p),
                ("dir", C.c_void_p)]


EXPORTS = ["hg_encode", "hg_encode_index", "hg_render_direct", "hg_render_indirect", "hg_backward",
           "hg_backward_workspace_size", "hg_morton_order", "hg_morton_order_workspace_size", "hg_l2_loss", "hg_adam_step_multi",
           "hg_adam_step", "hg_denoise", "hg_denoise_noalloc", "hg_denoise_workspace_size", "hg_env_build_sampling",
           "hg_env_sampling_size", "hg_last_error"]

_lib = None


def lib():
    """Load libhg.so (built in-tree by ``python -m paper_2409_10327_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_10327_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.hg_last_error.restype = C.c_char_p
        for name in EXPORTS[:-1]:
            getattr(L, name).restype = C.c_int
        L.hg_env_sampling_size.restype = C.c_size_t
        L.hg_env_sampling_size.argtypes = [C.c_int32, C.c_int32]
        L.hg_env_build_sampling.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]
        L.hg_denoise_workspace_size.restype = C.c_size_t
        L.hg_denoise_workspace_size.argtypes = [C.c_int32, C.c_int32]
        L.hg_denoise.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(DenoiseParams),
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.hg_denoise_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                         C.POINTER(DenoiseParams), C.c_void_p, C.c_void_p]
        L.hg_encode.argtypes = [C.POINTER(Grid), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.hg_encode_index.argtypes = [C.POINTER(Grid), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        for nm in ("hg_render_direct", "hg_render_indirect"):
            getattr(L, nm).argtypes = [C.POINTER(Model), C.POINTER(Env), C.POINTER(Sampling), C.POINTER(Points),
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.hg_backward.argtypes = [C.POINTER(Model), C.POINTER(Env), C.POINTER(Sampling), C.POINTER(Points),
                                  C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p * 6, C.c_void_p * 6, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.hg_backward_workspace_size.restype = C.c_size_t
        L.hg_backward_workspace_size.argtypes = [C.c_int32, C.c_int64]
        L.hg_morton_order_workspace_size.restype = C.c_size_t
        L.hg_morton_order_workspace_size.argtypes = [C.c_int64]
        L.hg_morton_order.argtypes = [C.c_void_p, C.c_int64, C.c_float, C.c_float, C.c_void_p, C.c_void_p,
                                      C.c_size_t, C.c_void_p]
        L.hg_l2_loss.argtypes = [C.c_void_p] * 4 + [C.c_int64] + [C.c_void_p] * 5
        L.hg_adam_step_multi.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                                         C.c_float, C.c_int32, C.c_void_p]
        L.hg_adam_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                   C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p, C.c_int32,
                                   C.c_void_p]
        _lib = L
    return _lib


def _check(status):
    if status != HG_OK:
        raise HGError(status, lib().hg_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _f32c(t, dev):
    return torch.as_tensor(t).to(device=dev, dtype=torch.float32).contiguous()


# --------------------------------------------------------------------------
# Parameter holder
# --------------------------------------------------------------------------
class HashRenderer:
    """Device-resident parameters of the hash renderer.

    FP32 masters (table [L][T][F], decoder B and tracer I as W0,b0,W1,b1,W2,b2)
    plus low-precision shadows for the mixed path (FP16 table, BF16 weights),
    refreshed by :meth:`refresh_shadows` or by the Adam step."""

    def __init__(self, params: dict, device="cuda", box_lo=BOX_LO, box_extent=BOX_EXTENT, t_near=0.05,
                 t_far=1.5, f0=0.04):
        self.device = torch.device(device)
        self.table = _f32c(params["table"], self.device)
        L = self.table.shape[0]
        # the kernels read 16 level slots: first-layer columns of the slots of
        # missing levels are zero (the layout the C ABI documents)
        self.brdf = [_f32c(a, self.device) for a in params["brdf"]]
        self.irt = [_f32c(a, self.device) for a in params["irt"]]
        self.brdf[0] = self._slot_cols(self.brdf[0], L, 0)
        self.irt[0] = self._slot_cols(self.irt[0], L, 3)
        self.res = [int(r) for r in params["res"]]
        self.box_lo, self.box_extent = float(box_lo), float(box_extent)
        self.t_near, self.t_far, self.f0 = float(t_near), float(t_far), float(f0)
        self.table16 = None
        self.brdf16 = None
        self.irt16 = None

    @property
    def L(self):
        return self.table.shape[0]

    @staticmethod
    def _slot_cols(W0, L, n_dir):
        """[64][2L + n_dir] -> [64][32 + n_dir]: features into their level
        slots, the direction columns after the 32 slots."""
        if W0.shape[1] == 32 + n_dir:
            return W0.contiguous()
        out = torch.zeros((W0.shape[0], 32 + n_dir), device=W0.device, dtype=W0.dtype)
        out[:, :2 * L] = W0[:, :2 * L]
        out[:, 32:] = W0[:, 2 * L:]
        return out

    def natural(self, mlp_list, which):
        """Undo the slot layout of a first-layer weight (or its gradient):
        returns the list with W0 as [64][2L (+3)]."""
        L = self.L
        W0 = mlp_list[0]
        n_dir = 3 if which == "irt" else 0
        if W0.shape[1] == 2 * L + n_dir:
            return list(mlp_list)
        return [torch.cat([W0[:, :2 * L], W0[:, 32:]], 1)] + list(mlp_list[1:])

    def refresh_shadows(self):
        self.table16 = self.table.to(torch.float16)
        self.brdf16 = [a.to(torch.bfloat16) if i % 2 == 0 else a for i, a in enumerate(self.brdf)]
        self.irt16 = [a.to(torch.bfloat16) if i % 2 == 0 else a for i, a in enumerate(self.irt)]

    def grid_struct(self, table=None, dtype=HG_F32):
        table = self.table if table is None else table
        g = Grid()
        g.L, g.F = table.shape[0], table.shape[2]
        g.log2_T = int(table.shape[1]).bit_length() - 1
        for i, r in enumerate(self.res):
            g.res[i] = r
        g.box_lo, g.box_extent = self.box_lo, self.box_extent
        g.dtype = dtype
        g.table = table.data_ptr()
        return g

    @staticmethod
    def _mlp(ws, dtype):
        m = Mlp()
        m.n_hidden, m.n_in = ws[0].shape
        m.n_out = ws[4].shape[0]
        m.dtype = dtype
        for k in range(3):
            m.W[k] = ws[2 * k].data_ptr()
            m.b[k] = ws[2 * k + 1].data_ptr()
        return m

    def model_struct(self, precision="fp32"):
        """precision: "fp32" (FP32 table + FP32 MLPs), "mixed" (FP16 table +
        BF16 MLPs) or "f16table" (FP16 table + FP32 MLPs, backward only)."""
        m = Model()
        if precision == "fp32":
            m.grid = self.grid_struct()
            m.brdf = self._mlp(self.brdf, HG_F32)
            m.irt = self._mlp(self.irt, HG_F32)
        else:
            if self.table16 is None:
                self.refresh_shadows()
            m.grid = self.grid_struct(self.table16, HG_F16)
            if precision == "mixed":
                m.brdf = self._mlp(self.brdf16, HG_BF16)
                m.irt = self._mlp(self.irt16, HG_BF16)
            elif precision == "f16table":
                m.brdf = self._mlp(self.brdf, HG_F32)
                m.irt = self._mlp(self.irt, HG_F32)
            else:
                raise ValueError(precision)
        m.t_near, m.t_far, m.f0 = self.t_near, self.t_far, self.f0
        return m


def env_struct(env: torch.Tensor, dist: torch.Tensor | None = None):
    e = Env()
    e.H, e.W = env.shape[0], env.shape[1]
    e.rgb = env.data_ptr()
    e.dist = None if dist is None else dist.data_ptr()
    return e


def env_sampling(env: torch.Tensor) -> torch.Tensor:
    """Light-importance distribution of an environment map [H,W,3] (needed
    by flags=HG_MIS): built by the library on the host from a host copy of
    the map, returned as an opaque FP32 device buffer."""
    H, W = env.shape[0], env.shape[1]
    nbytes = lib().hg_env_sampling_size(H, W)
    if nbytes == 0:
        raise HGError(HG_E_INVALID, f"environment map {H}x{W} is outside [1, 8192]^2")
    host = env.detach().to("cpu", torch.float32).contiguous()
    dist = torch.empty((nbytes + 3) // 4, device=env.device, dtype=torch.float32)
    _check(lib().hg_env_build_sampling(C.c_void_p(host.data_ptr()), H, W, _ptr(dist), dist.numel() * 4,
                                       _stream(env.device)))
    return dist


def sampling_struct(n_dirs=1, n_dirs2=8, seed=7, flags=0):
    s = Sampling()
    s.n_dirs, s.n_dirs2, s.seed, s.flags = n_dirs, n_dirs2, seed, flags
    return s


def points_struct(pos, nrm=None, wo=None, dirs=None):
    p = Points()
    p.n = pos.shape[0]
    p.pos = pos.data_ptr()
    p.nrm = None if nrm is None else nrm.data_ptr()
    p.wo = None if wo is None else wo.data_ptr()
    p.dir = None if dirs is None else dirs.data_ptr()
    return p


# --------------------------------------------------------------------------
# Entry points
# --------------------------------------------------------------------------
def encode(r: HashRenderer, pos: torch.Tensor, precision="fp32") -> torch.Tensor:
    """f = H(x): [n,3] -> [n, L*F] FP32."""
    feat = torch.empty((pos.shape[0], r.L * 2), device=pos.device, dtype=torch.float32)
    if precision == "fp32":
        g = r.grid_struct()
    else:
        if r.table16 is None:
            r.refresh_shadows()
        g = r.grid_struct(r.table16, HG_F16)
    _check(lib().hg_encode(C.byref(g), _ptr(pos), pos.shape[0], _ptr(feat), _stream(pos.device)))
    return feat


def encode_index(r: HashRenderer, pos: torch.Tensor):
    """Corner indices [n,L,8] (int32 view of uint32) and weights [n,L,3]."""
    n = pos.shape[0]
    idx = torch.empty((n, r.L, 8), device=pos.device, dtype=torch.int32)
    w = torch.empty((n, r.L, 3), device=pos.device, dtype=torch.float32)
    g = r.grid_struct()
    _check(lib().hg_encode_index(C.byref(g), _ptr(pos), n, _ptr(idx), _ptr(w), _stream(pos.device)))
    return idx, w


def render(r: HashRenderer, env: torch.Tensor, pos, nrm=None, wo=None, dirs=None, n_dirs=32, n_dirs2=8, seed=7,
           flags=0, indirect=True, want_vis=False, precision="fp32", out=None, env_dist=None):
    """Shade mode (dirs None): rgb [n,3] (+ vis/depth [n,N] if want_vis).
    Query mode: rgb [n,3] = L_in, vis [n], depth [n].  flags=HG_MIS needs
    env_dist = env_sampling(env)."""
    n = pos.shape[0]
    dev = pos.device
    if out is None:
        rgb = torch.empty((n, 3), device=dev, dtype=torch.float32)
        if dirs is not None:
            vis = torch.empty(n, device=dev, dtype=torch.float32)
            dep = torch.empty(n, device=dev, dtype=torch.float32)
        elif want_vis:
            vis = torch.empty((n, n_dirs), device=dev, dtype=torch.float32)
            dep = torch.empty((n, n_dirs), device=dev, dtype=torch.float32)
        else:
            vis = dep = None
    else:
        rgb, vis, dep = out
    m = r.model_struct(precision)
    e = env_struct(env, env_dist)
    s = sampling_struct(n_dirs, n_dirs2, seed, flags)
    p = points_struct(pos, nrm, wo, dirs)
    fn = lib().hg_render_indirect if indirect else lib().hg_render_direct
    _check(fn(C.byref(m), C.byref(e), C.byref(s), C.byref(p), _ptr(rgb), _ptr(vis), _ptr(dep), _stream(dev)))
    return rgb, vis, dep


def backward(r: HashRenderer, env, pos, dirs, g_rgb, g_vis, g_dep, grads, n_dirs2=8, seed=7, flags=0,
             indirect=True, g_pos=None, precision="fp32", ws=None):
    """Adds query-mode gradients into grads = dict(table=..., brdf=[6], irt=[6]).
    ws: optional uint8 device workspace of hg_backward_workspace_size bytes
    (allocated here if None)."""
    m = r.model_struct(precision)
    e = env_struct(env)
    s = sampling_struct(1, n_dirs2, seed, flags)
    p = points_struct(pos, None, None, dirs)
    gb = (C.c_void_p * 6)(*[g.data_ptr() for g in grads["brdf"]])
    gi = (C.c_void_p * 6)(*[g.data_ptr() for g in grads["irt"]])
    need = lib().hg_backward_workspace_size(int(indirect), pos.shape[0])
    if need and (ws is None or ws.numel() * ws.element_size() < need):
        ws = torch.empty(need, device=pos.device, dtype=torch.uint8)
    _check(lib().hg_backward(C.byref(m), C.byref(e), C.byref(s), C.byref(p), int(indirect), _ptr(g_rgb),
                             _ptr(g_vis), _ptr(g_dep), _ptr(grads["table"]), gb, gi, _ptr(g_pos),
                             _ptr(ws) if need else None, need, _stream(pos.device)))


def morton_order(r: HashRenderer, pos, ws=None):
    """int32 permutation of the points pos [n][3] along a Z-order curve over
    the renderer's grid box (hg_morton_order); ws: optional uint8 device
    workspace of hg_morton_order_workspace_size bytes."""
    if pos.dim() != 2 or pos.shape[1] != 3 or pos.dtype != torch.float32 or not pos.is_contiguous():
        raise ValueError("pos must be a contiguous float32 [n][3] tensor")
    n = pos.shape[0]
    perm = torch.empty(n, device=pos.device, dtype=torch.int32)
    if n == 0:
        return perm
    need = lib().hg_morton_order_workspace_size(n)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, device=pos.device, dtype=torch.uint8)
    _check(lib().hg_morton_order(_ptr(pos), n, r.box_lo, r.box_extent, _ptr(perm), _ptr(ws), need,
                                 _stream(pos.device)))
    return perm


class AdamTensor(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("weight_decay", C.c_float), ("shadow_dtype", C.c_int32), ("shadow", C.c_void_p)]


ADAM_MAX_TENSORS = 16


class AdamGroup:
    """The descriptors of hg_adam_step_multi for a fixed list of (param,
    grad, m, v, weight_decay, shadow) tuples (shadow None, or an FP16 / BF16
    tensor of param's size), built once and reused every step."""

    def __init__(self, tensors):
        if len(tensors) > ADAM_MAX_TENSORS:
            raise ValueError(f"at most {ADAM_MAX_TENSORS} tensors per group")
        self.tensors = list(tensors)  # keeps the tensors alive
        self.arr = (AdamTensor * max(1, len(tensors)))()
        self.count = len(tensors)
        self.device = tensors[0][0].device if tensors else None
        for i, (p, g, m_, v_, wd, sh) in enumerate(tensors):
            dt = 0 if sh is None else (HG_F16 if sh.dtype == torch.float16 else HG_BF16)
            self.arr[i] = AdamTensor(p.data_ptr(), g.data_ptr(), m_.data_ptr(), v_.data_ptr(), p.numel(), wd, dt,
                                     None if sh is None else sh.data_ptr())


def adam_step_multi(tensors, step, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8, zero_grad=False):
    """hg_adam_step_multi over an AdamGroup or a list of (param, grad, m, v,
    weight_decay, shadow) tuples."""
    grp = tensors if isinstance(tensors, AdamGroup) else AdamGroup(tensors)
    _check(lib().hg_adam_step_multi(grp.arr, grp.count, step, lr, beta1, beta2, eps, int(bool(zero_grad)),
                                    _stream(grp.device)))


def l2_loss(rgb, vis, dep, tgt):
    n = vis.shape[0]
    dev = vis.device
    loss = torch.empty(1, device=dev, dtype=torch.float32)
    g_rgb = torch.empty_like(rgb)
    g_vis = torch.empty_like(vis)
    g_dep = torch.empty_like(dep)
    _check(lib().hg_l2_loss(_ptr(rgb), _ptr(vis), _ptr(dep), _ptr(tgt), n, _ptr(loss), _ptr(g_rgb), _ptr(g_vis),
                            _ptr(g_dep), _stream(dev)))
    return loss, g_rgb, g_vis, g_dep


def adam_step(param, grad, m, v, step, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0,
              shadow=None):
    sd = HG_F32
    if shadow is not None:
        sd = HG_F16 if shadow.dtype == torch.float16 else HG_BF16
    _check(lib().hg_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), step, lr, beta1, beta2,
                              eps, weight_decay, _ptr(shadow), sd, _stream(param.device)))


def denoise(rgb, depth, nrm, iterations=5, sigma_z=1.0, sigma_n=128.0, sigma_l=4.0, work=None):
    """Spatial SVGF filter: rgb [H,W,3], depth [H,W], nrm [H,W,3] -> [H,W,3]."""
    H, W = depth.shape
    out = torch.empty_like(rgb)
    need = lib().hg_denoise_workspace_size(H, W)
    if work is None or work.numel() * work.element_size() < need:
        work = torch.empty(need // 4, device=rgb.device, dtype=torch.float32)
    prm = DenoiseParams(iterations, sigma_z, sigma_n, sigma_l)
    _check(lib().hg_denoise(_ptr(rgb), _ptr(depth), _ptr(nrm), H, W, C.byref(prm), _ptr(out), _ptr(work),
                            work.numel() * work.element_size(), _stream(rgb.device)))
    return out


DENOISE_NOALLOC_MAX_PIXELS = 1 << 20  # HG_DENOISE_NOALLOC_MAX_PIXELS


def denoise_noalloc(rgb, depth, nrm, out, iterations=5, sigma_z=1.0, sigma_n=128.0, sigma_l=4.0):
    """hg_denoise_noalloc: as denoise() into the caller's ``out`` [H,W,3], with the
    library's static per-device workspace (at most 2^20 pixels; concurrent calls
    on one GPU race)."""
    H, W = depth.shape
    prm = DenoiseParams(iterations, sigma_z, sigma_n, sigma_l)
    _check(lib().hg_denoise_noalloc(_ptr(rgb), _ptr(depth), _ptr(nrm), H, W, C.byref(prm), _ptr(out),
                                    _stream(rgb.device)))
    return out


def zero_grads(r: HashRenderer):
    return dict(table=torch.zeros_like(r.table), brdf=[torch.zeros_like(a) for a in r.brdf],
                irt=[torch.zeros_like(a) for a in r.irt])


# --------------------------------------------------------------------------
# autograd
# --------------------------------------------------------------------------
class HGQueryFn(torch.autograd.Function):
    """Query-mode forward (L_in, V, d) with the hand-written backward.

    forward(renderer, env, pos, dirs, table, *mlp_params) -> (rgb, vis, depth).
    The parameter tensors are passed so that autograd routes their gradients;
    they must be the renderer's own masters."""

    @staticmethod
    def forward(ctx, renderer, env, pos, dirs, n_dirs2, seed, indirect, precision, table, *mlp):
        rgb, vis, dep = render(renderer, env, pos, dirs=dirs, n_dirs2=n_dirs2, seed=seed, indirect=indirect,
                               precision=precision)
        ctx.renderer, ctx.env, ctx.cfg = renderer, env, (n_dirs2, seed, indirect, precision)
        ctx.save_for_backward(pos, dirs)
        return rgb, vis, dep

    @staticmethod
    def backward(ctx, g_rgb, g_vis, g_dep):
        pos, dirs = ctx.saved_tensors
        r = ctx.renderer
        n_dirs2, seed, indirect, precision = ctx.cfg
        grads = zero_grads(r)
        z = lambda t, shape: torch.zeros(shape, device=pos.device) if t is None else t.contiguous()
        backward(r, ctx.env, pos, dirs, z(g_rgb, (pos.shape[0], 3)), z(g_vis, (pos.shape[0],)),
                 z(g_dep, (pos.shape[0],)), grads, n_dirs2=n_dirs2, seed=seed, indirect=indirect,
                 precision=precision)
        return (None, None, None, None, None, None, None, None, grads["table"], *grads["brdf"], *grads["irt"])

"""Seeded synthetic inputs for the hash-grid secondary-ray renderer.

This module is shared by the FP64 oracle's tests and by the GPU path's tests
and benchmark.  It produces *inputs only*: analytic primary surface points,
hash tables, MLP weights, environment maps and training batches.  It holds
none of the renderer's arithmetic (no encode, no MLP evaluation, no BRDF, no
sampling of light directions); those live separately in the oracle and in
the HIP kernels.

Workload shapes follow the paper's evaluation setting (800x800 frames,
3-layer width-64 decoders, 8 secondary rays per bounce point; Sec. 4.1 and the
supplementary "Rendering Details") with the synthetic scene family described
below standing in for the paper's TensoIR-/InvRender-synthetic scenes, which
are not available.

Every array is generated with ``numpy.random.Generator(PCG64(seed))`` and
returned as float32 (the FP32 masters).  Low-precision shadows (FP16 tables,
BF16 weights) are derived from these masters by the product at run time.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

# --------------------------------------------------------------------------
# Seeds (one per input family)
# --------------------------------------------------------------------------
SEED_SCENE = 1
SEED_TABLE = 2
SEED_MLP = 3
SEED_ENV = 4
SEED_TEACHER = 5
SEED_BATCH = 6
SEED_DIRS = 7          # key of the counter-based direction generator

# Domain of the hash grid: the cube [BOX_LO, BOX_LO + BOX_EXTENT]^3.  The
# extent is a power of two so that normalising a coordinate is exact after
# the subtraction of BOX_LO.
BOX_LO = -8.0
BOX_EXTENT = 16.0

T_NEAR = 0.05          # secondary-ray near/far (supplementary, hash renderer)
T_FAR = 1.5
F0_DIELECTRIC = 0.04   # fixed Fresnel reflectance (Sec. 5)


def level_resolutions(n_levels: int, n_min: int, n_max: int) -> list[int]:
    """Per-level grid resolutions N_l, geometric from n_min to n_max.

    The hash encoder follows InstantNGP's multi-resolution layout (Sec. 3.2,
    "Indirect Illumination Renderer"; Sec. 4.1 gives min/max resolutions).
    N_l = floor(n_min * b**l) with b = exp((ln n_max - ln n_min)/(L-1)),
    evaluated once in float64 with a 1e-12 relative guard so that exact
    powers (e.g. 16*2**(15/3) = 512) do not floor to one below.
    """
    if n_levels == 1:
        return [int(n_min)]
    b = math.exp((math.log(n_max) - math.log(n_min)) / (n_levels - 1))
    return [int(math.floor(n_min * b ** l * (1.0 + 1e-12))) for l in range(n_levels)]


@dataclass
class Config:
    name: str
    img_h: int = 64
    img_w: int = 64
    n_levels: int = 16
    n_feat: int = 2
    log2_T: int = 14
    res_min: int = 16
    res_max: int = 512
    hidden: int = 64
    env_h: int = 16
    env_w: int = 32
    n_dirs: int = 32
    n_dirs2: int = 8
    indirect: bool = True
    precision: str = "fp32"          # "fp32" or "mixed"
    batch: int = 0                   # training batch (query mode), 0 = none
    teacher_log2_T: int = 20
    brdf_out: int = 5                # 8: decoder with a normal head (paper shape)
    res: list = field(default_factory=list)

    def __post_init__(self):
        if not self.res:
            self.res = level_resolutions(self.n_levels, self.res_min, self.res_max)

    @property
    def n_points(self) -> int:
        return self.img_h * self.img_w

    def to_dict(self):
        return asdict(self)


def config(name: str) -> Config:
    """The five workload configurations.

    c1: FP32 forward, tiny (64x64 frame, T=2^14, res 16..512, env 16x32, N=32).
    c2: FP32 forward at frame size (800x800, T=2^19, res 16..2048, env 64x128,
        N=128, N'=8): 81.92M secondary queries.
    c3: as c2, mixed precision (FP16 tables, BF16 MLPs, FP32 accumulation).
    c4: distillation training step: 2^18 query-mode samples, teacher T=2^20,
        student T=2^19.
    c5: mixed 800x800 frame at N=512 plus a training step over 2^20 samples.
    paper: the paper's model shape (Sec. 4.1): 14 levels, T=2^17, res
        16..131072 (growth 2, two dense levels), decoder with a normal head
        (8 outputs), 800x800 frame, env 64x128, N=128.
    paper_small: the same model shape on the 64x64 frame (parity sizes).
    """
    if name == "c1":
        return Config("c1")
    frame = dict(img_h=800, img_w=800, log2_T=19, res_max=2048, env_h=64, env_w=128,
                 n_dirs=128)
    if name == "c2":
        return Config("c2", **frame)
    if name == "c3":
        return Config("c3", precision="mixed", **frame)
    if name == "c4":
        return Config("c4", img_h=0, img_w=0, log2_T=19, res_max=2048, env_h=64, env_w=128,
                      n_dirs=1, batch=1 << 18)
    if name in ("paper", "paper_small"):
        size = 800 if name == "paper" else 64
        env = (64, 128) if name == "paper" else (16, 32)
        return Config(name, img_h=size, img_w=size, n_levels=14, log2_T=17, res_min=16, res_max=131072,
                      env_h=env[0], env_w=env[1], n_dirs=128 if name == "paper" else 32, brdf_out=8)
    if name == "c5":
        f = dict(frame)
        f["n_dirs"] = 512
        return Config("c5", precision="mixed", batch=1 << 20, **f)
    raise KeyError(name)


# --------------------------------------------------------------------------
# Analytic scene: unit sphere at the origin resting on the plane y = -1,
# pinhole camera at radius 4 looking at the origin (y is up).
# --------------------------------------------------------------------------
CAM_RADIUS = 4.0
CAM_FOV_DEG = 40.0
CAM_ELEV_DEG = (45.0, 60.0)


def camera(seed: int = SEED_SCENE):
    rng = np.random.Generator(np.random.PCG64(seed))
    el = math.radians(rng.uniform(*CAM_ELEV_DEG))
    az = rng.uniform(0.0, 2.0 * math.pi)
    c = CAM_RADIUS * np.array([math.cos(el) * math.cos(az), math.sin(el),
                               math.cos(el) * math.sin(az)])
    return c


def make_scene(img_h: int, img_w: int, seed: int = SEED_SCENE):
    """Primary surface points of the analytic scene, one per pixel.

    Returns float32 arrays pos [P,3], nrm [P,3] (unit outward normal) and
    wo [P,3] (unit direction from the surface point back to the camera),
    P = img_h*img_w, pixels in row-major order.  Every pixel hits either the
    sphere or the plane (the camera looks down by at least 25 degrees at the
    top edge of the frame).
    """
    c = camera(seed)
    fwd = -c / np.linalg.norm(c)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(CAM_FOV_DEG) / 2)
    ys, xs = np.meshgrid(np.arange(img_h), np.arange(img_w), indexing="ij")
    ndc_x = ((xs + 0.5) / img_w * 2 - 1) * th * (img_w / img_h)
    ndc_y = (1 - (ys + 0.5) / img_h * 2) * th
    d = fwd[None, None, :] + ndc_x[..., None] * right + ndc_y[..., None] * up
    d = d.reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # sphere |c + t d| = 1
    cd = d @ c
    disc = cd * cd - (c @ c - 1.0)
    t_s = np.where(disc >= 0, -cd - np.sqrt(np.maximum(disc, 0)), np.inf)
    t_s = np.where(t_s > 0, t_s, np.inf)
    # plane y = -1
    t_p = np.where(d[:, 1] < 0, (-1.0 - c[1]) / np.where(d[:, 1] < 0, d[:, 1], -1), np.inf)
    hit_s = t_s <= t_p
    t = np.where(hit_s, t_s, t_p)
    if not np.all(np.isfinite(t)):
        raise RuntimeError("camera ray missed the scene")
    pos = c[None, :] + t[:, None] * d
    nrm = np.where(hit_s[:, None], pos, np.array([0.0, 1.0, 0.0]))
    nrm = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)
    wo = -d
    return pos.astype(np.float32), nrm.astype(np.float32), wo.astype(np.float32)


def subset_rows_cols(img_h: int, img_w: int, stride: int = 8):
    """Indices of the pixel subset on every `stride`-th row and column."""
    ys, xs = np.meshgrid(np.arange(0, img_h, stride), np.arange(0, img_w, stride), indexing="ij")
    return (ys * img_w + xs).reshape(-1)


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
def make_table(n_levels: int, log2_T: int, n_feat: int = 2, seed: int = SEED_TABLE,
               std: float = 0.1):
    """Hash tables [L][T][F], entries ~ Normal(0, std^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = 1 << log2_T
    return rng.standard_normal((n_levels, T, n_feat), dtype=np.float32) * np.float32(std)


def make_mlp(n_in: int, n_hidden: int, n_out: int, rng):
    """3-layer MLP n_in -> n_hidden -> n_hidden -> n_out, nn.Linear layout
    W[out][in].  Kaiming-normal weights (std sqrt(2/fan_in)), zero biases."""
    shapes = [(n_hidden, n_in), (n_hidden, n_hidden), (n_out, n_hidden)]
    out = []
    for (o, i) in shapes:
        w = (rng.standard_normal((o, i)) * math.sqrt(2.0 / i)).astype(np.float32)
        out += [w, np.zeros((o,), np.float32)]
    return out


def make_model(cfg: Config, seed_table: int = SEED_TABLE, seed_mlp: int = SEED_MLP,
               log2_T: int | None = None):
    """Tables plus BRDF decoder B (L*F -> 64 -> 64 -> 5, or 8 with the normal
    head) and implicit ray tracer I (L*F+3 -> 64 -> 64 -> 2) as float32
    arrays."""
    lt = cfg.log2_T if log2_T is None else log2_T
    table = make_table(cfg.n_levels, lt, cfg.n_feat, seed_table)
    rng = np.random.Generator(np.random.PCG64(seed_mlp))
    nf = cfg.n_levels * cfg.n_feat
    brdf = make_mlp(nf, cfg.hidden, cfg.brdf_out, rng)
    irt = make_mlp(nf + 3, cfg.hidden, 2, rng)
    return dict(table=table, brdf=brdf, irt=irt, res=list(cfg.res), log2_T=lt,
                n_levels=cfg.n_levels, n_feat=cfg.n_feat)


def make_teacher(cfg: Config):
    """Fixed seed-initialised teacher of the student's architecture with a
    larger table (T = 2^teacher_log2_T)."""
    return make_model(cfg, seed_table=SEED_TEACHER, seed_mlp=SEED_TEACHER + 100,
                      log2_T=cfg.teacher_log2_T)


# --------------------------------------------------------------------------
# Environment map: equirectangular HDR, [H][W][3], y is up, row 0 at the
# zenith, column 0 at azimuth -pi (azimuth measured as atan2(z, x)).
# --------------------------------------------------------------------------
SUN_INTENSITY = 50.0
SUN_SHARPNESS = 100.0


def make_env(h: int, w: int, seed: int = SEED_ENV):
    """Log-normal(0,1) texels per channel plus a sun lobe
    50*exp(100*(w.d_sun - 1)) on all channels, evaluated at texel centres;
    the sun's elevation is uniform in [20, 70] degrees."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.exp(rng.standard_normal((h, w, 3)))
    el = math.radians(rng.uniform(20.0, 70.0))
    az = rng.uniform(-math.pi, math.pi)
    sun = np.array([math.cos(el) * math.cos(az), math.sin(el), math.cos(el) * math.sin(az)])
    th = (np.arange(h) + 0.5) / h * math.pi
    ph = (np.arange(w) + 0.5) / w * 2 * math.pi - math.pi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(TH) * np.cos(PH), np.cos(TH), np.sin(TH) * np.sin(PH)], -1)
    lobe = SUN_INTENSITY * np.exp(SUN_SHARPNESS * (dirs @ sun - 1.0))
    return (base + lobe[..., None]).astype(np.float32)


# --------------------------------------------------------------------------
# Training batch (query mode): surface points uniform in [-1,1]^3 and unit
# directions uniform on the sphere.
# --------------------------------------------------------------------------
def make_train_batch(n: int, seed: int = SEED_BATCH):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(-1.0, 1.0, (n, 3)).astype(np.float32)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return pos, d.astype(np.float32)


def make_targets(n: int, seed: int = SEED_BATCH + 1000):
    """Arbitrary regression targets [n][5] (rgb, visibility, depth) for
    loss/backward parity cases that do not need a teacher."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.empty((n, 5), np.float32)
    t[:, :3] = np.exp(rng.standard_normal((n, 3)))
    t[:, 3] = rng.uniform(0, 1, n)
    t[:, 4] = rng.uniform(0, 1, n)
    return t

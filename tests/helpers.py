"""Shared builders for the parity tests (inputs from hg_inputs only)."""
import numpy as np

import hg_inputs as H


def relerr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def max_rel(a, b, floor_frac=1e-3):
    """Elementwise |a-b| / (|b| + floor_frac * RMS(b))."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    rms = np.sqrt(np.mean(b * b)) if b.size else 1.0
    return float(np.max(np.abs(a - b) / (np.abs(b) + floor_frac * rms))) if b.size else 0.0


def psnr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    mse = np.mean((a - b) ** 2)
    return 10 * np.log10(b.max() ** 2 / mse) if mse > 0 else np.inf


def c1_setup():
    cfg = H.config("c1")
    model = H.make_model(cfg)
    env = H.make_env(cfg.env_h, cfg.env_w)
    pos, nrm, wo = H.make_scene(cfg.img_h, cfg.img_w)
    return cfg, model, env, pos, nrm, wo


def adversarial_positions(res, n_random=20000, seed=0):
    """Random positions plus points on / just next to vertices of every level,
    the box faces and outside the box (FP32)."""
    rng = np.random.default_rng(seed)
    pts = [rng.uniform(H.BOX_LO - 1, H.BOX_LO + H.BOX_EXTENT + 1, (n_random, 3))]
    for N in res:
        k = rng.integers(0, N + 1, (200, 3))
        v = H.BOX_LO + H.BOX_EXTENT * k / N
        pts.append(v)
        pts.append(np.nextafter(v.astype(np.float32), np.float32(-np.inf)))
        pts.append(np.nextafter(v.astype(np.float32), np.float32(np.inf)))
    pts.append(np.array([[H.BOX_LO] * 3, [H.BOX_LO + H.BOX_EXTENT] * 3, [0.0, 0.0, 0.0]]))
    return np.concatenate([np.asarray(p, np.float32) for p in pts]).astype(np.float32)

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


def kink_margin(model, pos, dirs, dep, indirect, seed=7, n_dirs2=8):
    """Per query-mode sample, the smallest relative distance to a kink of the
    network in FP64: every ReLU pre-activation p over |W||z| + |b| (for the
    tracer at (x, w), and with the bounce the decoder at x' and the tracer at
    (x', w'_j)), and the depth clamp |softplus - 1|.  Where it is within FP32
    rounding (~1e-5) the FP32 and FP64 sides may take different branches and
    the gradient jumps, so gradient parity excludes those samples.  With the
    bounce, x' within 2e-4 cells of a cell face of any level also counts
    (the FP32 x' is uncertain by ~1e-6 of the domain).  Uses the
    oracle's encodings and depths (dep) and the 5-output decoder's facing
    normal."""
    import hg_inputs as H
    from oracle import oracle as O
    om = O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT)
    irt = [a.astype(np.float64) for a in model["irt"]]
    brdf = [a.astype(np.float64) for a in model["brdf"]]

    def margins(m, z):  # z [n, k]
        p1 = z @ m[0].T + m[1]
        s1 = np.abs(z) @ np.abs(m[0]).T + np.abs(m[1]) + 1e-300
        h1 = np.maximum(p1, 0)
        p2 = h1 @ m[2].T + m[3]
        s2 = h1 @ np.abs(m[2]).T + np.abs(m[3]) + 1e-300
        out = np.maximum(h1 @ m[2].T + m[3], 0) @ m[4].T + m[5]
        return np.minimum((np.abs(p1) / s1).min(1), (np.abs(p2) / s2).min(1)), out

    n = pos.shape[0]
    w = dirs.astype(np.float64)
    f = O.encode(om, pos)
    mg, o = margins(irt, np.concatenate([f, w], 1))
    sp = np.logaddexp(0.0, o[:, 1])
    mg = np.minimum(mg, np.abs(sp - 1.0))
    if indirect:
        t = 0.05 + 1.45 * np.asarray(dep, np.float64)
        xb = pos.astype(np.float64) + t[:, None] * w
        # the trilinear interpolation's spatial derivative (which carries the
        # depth head's gradient) jumps at cell faces: distance of x' to the
        # nearest face in cells, scaled so that 2e-4 cells maps to 1e-5
        u = np.clip((xb - H.BOX_LO) / H.BOX_EXTENT, 0.0, 1.0)
        for N in model["res"]:
            p = u * N
            mg = np.minimum(mg, np.abs(p - np.round(p)).min(1) * (1e-5 / 2e-4))
        fb = O.encode_f64(om, xb)
        m2, _ = margins(brdf, fb)
        mg = np.minimum(mg, m2)
        for j in range(n_dirs2):
            wj = O.sample_dirs(seed, -w, np.arange(n), np.zeros(n), np.full(n, j), 1, n_dirs2)
            m3, _ = margins(irt, np.concatenate([fb, wj], 1))
            mg = np.minimum(mg, m3)
    return mg


def grad_condition(om, oe, samp, pos, dirs, g_rgb, g_vis, g_dep, indirect):
    """Condition number of each MLP parameter gradient as a sum over samples:
    ||sum_s |g_s| || / ||sum_s g_s|| with g_s the FP64 oracle's contribution
    of sample s (one backward per sample, with its own point id).  An FP32
    implementation whose per-sample terms carry a relative rounding error
    delta is off by up to this factor times delta."""
    from oracle import oracle as O
    tot = O.backward(om, oe, samp, pos, dirs, g_rgb, g_vis, g_dep, indirect=indirect)
    ab = {k: [np.zeros_like(a) for a in tot[k]] for k in ("irt", "brdf")}
    for s in range(pos.shape[0]):
        r = O.backward(om, oe, samp, pos[s:s + 1], dirs[s:s + 1], g_rgb[s:s + 1], g_vis[s:s + 1], g_dep[s:s + 1],
                       indirect=indirect, pid=np.array([s]))
        for k in ab:
            for i in range(6):
                ab[k][i] += np.abs(r[k][i])
    return {(k, i): float(np.linalg.norm(ab[k][i]) / max(np.linalg.norm(tot[k][i]), 1e-300))
            for k in ab for i in range(6)}

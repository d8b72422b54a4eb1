"""Multiple importance sampling of the primary directions (light-importance
rays from the environment map plus GGX visible-normal rays, balance
heuristic; Sec. 4.1) against the FP64 oracle.

The light distribution is compared entry by entry.  In the frames, a GGX
ray whose direction lies within FP32 rounding of a texel edge of the
environment map may look up the neighbouring texel's density, which changes
that sample's weight: such pixels are counted and bounded, the rest are
compared at the FP32 bar."""
import numpy as np
import pytest
import torch

import hg_inputs as H
import paper_2409_10327_amd as hg
from oracle import oracle as O
from helpers import c1_setup, psnr, relerr

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def c1():
    cfg, model, env, pos, nrm, wo = c1_setup()
    r = hg.HashRenderer(model, DEV)
    r.refresh_shadows()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    env_t = t(env)
    return dict(cfg=cfg, model=model, env=env, pos=pos, nrm=nrm, wo=wo, r=r, t=t, env_t=env_t,
                dist=hg.env_sampling(env_t), om=O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT), oe=O.OracleEnv(env))


def unpack(dist, Hh, Ww):
    """Device layout: rows float4 [H], marginal and conditional CDFs as
    (hi, lo) float2 pairs, densities [H][W]; CDF values returned as hi + lo
    in float64."""
    d = dist.cpu().numpy().view(np.float32)
    rows = d[:4 * Hh].reshape(Hh, 4).astype(np.float64)
    o = 4 * Hh
    mp = d[o:o + 2 * (Hh + 1)].reshape(Hh + 1, 2).astype(np.float64)
    o += 2 * (Hh + 1)
    cp = d[o:o + 2 * Hh * (Ww + 1)].reshape(Hh, Ww + 1, 2).astype(np.float64)
    o += 2 * Hh * (Ww + 1)
    dens = d[o:o + Hh * Ww].reshape(Hh, Ww)
    return rows, mp[:, 0] + mp[:, 1], cp[..., 0] + cp[..., 1], dens


def env_cases():
    rng = np.random.default_rng(3)
    black_row = np.exp(rng.standard_normal((8, 16, 3))).astype(np.float32)
    black_row[3] = 0.0
    return {"sun 16x32": H.make_env(16, 32), "sun 64x128": H.make_env(64, 128, seed=9),
            "black row 8x16": black_row, "all black 4x8": np.zeros((4, 8, 3), np.float32),
            "single texel": np.full((1, 1, 3), 2.0, np.float32), "ragged 5x7": np.exp(rng.standard_normal((5, 7, 3))).astype(np.float32)}


@pytest.mark.parametrize("name", list(env_cases()))
def test_env_distribution(name):
    print(f"case: env distribution {name}", flush=True)
    env = env_cases()[name]
    Hh, Ww = env.shape[:2]
    dist = hg.env_sampling(torch.from_numpy(env).to(DEV))
    rows, marg, cond, dens = unpack(dist, Hh, Ww)
    oct_, omarg, ocond, odens = O.env_dist(O.OracleEnv(env))
    # row geometry in FP32: cos at the top edge, 1 - cos(top), 1 + cos(bottom), span
    assert np.all(np.abs(rows[:, 0] - oct_[:-1]) <= 6e-8)
    for got, want in ((rows[:, 1], 1 - oct_[:-1]), (rows[:, 2], 1 + oct_[1:]), (rows[:, 3], oct_[:-1] - oct_[1:])):
        assert np.all(np.abs(got - want) <= 1.2e-7 * np.abs(want) + 1e-15)
    # the CDFs as (hi, lo) pairs carry the double values to ~2^-48
    assert np.max(np.abs(marg - omarg)) < 1e-14 and marg[0] == 0 and marg[-1] == 1
    assert np.max(np.abs(cond - ocond)) < 1e-14 and np.all(cond[:, 0] == 0) and np.all(cond[:, -1] == 1)
    assert np.all(np.diff(marg) >= 0) and np.all(np.diff(cond, axis=1) >= 0)
    assert np.allclose(dens, odens, rtol=1e-6, atol=0)


@pytest.mark.parametrize("N,precision", [(2, "fp32"), (8, "fp32"), (32, "fp32"), (128, "fp32"), (2, "mixed"),
                                         (128, "mixed"), (256, "mixed")])
def test_mis_frame(c1, N, precision):
    """N = 2 is the paper's one light ray + one GGX ray; fewer than 16
    directions take the matrix-core kernel's per-lane mode."""
    print(f"case: MIS frame 64x64 N={N} {precision}", flush=True)
    t = c1["t"]
    rgb, vis, _ = hg.render(c1["r"], c1["env_t"], t(c1["pos"]), t(c1["nrm"]), t(c1["wo"]), n_dirs=N,
                            flags=hg.HG_MIS, want_vis=True, precision=precision, env_dist=c1["dist"])
    rgb, vis = rgb.cpu().numpy(), vis.cpu().numpy()
    orgb, ovis, _ = O.render(c1["om"], c1["oe"], O.sampling(N, 8, 7, O.MIS), c1["pos"], c1["nrm"], c1["wo"])
    if precision == "fp32":
        e = np.linalg.norm(rgb - orgb, axis=1) / (np.linalg.norm(orgb, axis=1) + 1e-6)
        ok = e < 1e-4
        print(f"MIS N={N}: {ok.mean():.5f} of pixels within 1e-4, rel err on them {relerr(rgb[ok], orgb[ok]):.3g}, "
              f"all {relerr(rgb, orgb):.3g}; vis rel err {relerr(vis[ok], ovis[ok]):.3g}")
        assert ok.mean() > 0.995
        assert relerr(rgb[ok], orgb[ok]) < 1e-5
        assert relerr(vis[ok], ovis[ok]) < 1e-5
    else:
        p = psnr(rgb, orgb)
        print(f"MIS N={N} mixed: PSNR {p:.1f} dB, rel err {relerr(rgb, orgb):.3g}")
        assert p >= 45.0


def test_mis_is_unbiased_against_cosine(c1):
    """Both estimators target the same rendering integral: over the 64x64
    frame their means agree within the Monte Carlo noise of the two."""
    print("case: MIS vs cosine frame means", flush=True)
    t = c1["t"]
    args = (c1["r"], c1["env_t"], t(c1["pos"]), t(c1["nrm"]), t(c1["wo"]))
    a = hg.render(*args, n_dirs=512, flags=hg.HG_MIS, env_dist=c1["dist"])[0].cpu().numpy()
    b = hg.render(*args, n_dirs=512)[0].cpu().numpy()
    d = (a - b).mean(0)
    sem = (a - b).std(0) / np.sqrt(a.shape[0])
    print(f"mean MIS {a.mean(0)}, cosine {b.mean(0)}, diff {d}, sem {sem}")
    assert np.all(np.abs(d) < 5 * sem + 1e-6)


def test_mis_deterministic_and_ragged(c1):
    print("case: MIS determinism and ragged sizes", flush=True)
    t = c1["t"]
    for npix, N in ((1, 2), (37, 16), (130, 64)):
        sl = slice(200, 200 + npix)
        args = (c1["r"], c1["env_t"], t(c1["pos"][sl]), t(c1["nrm"][sl]), t(c1["wo"][sl]))
        a = hg.render(*args, n_dirs=N, flags=hg.HG_MIS, env_dist=c1["dist"])[0]
        b = hg.render(*args, n_dirs=N, flags=hg.HG_MIS, env_dist=c1["dist"])[0]
        assert torch.equal(a, b)
        o = O.render(c1["om"], c1["oe"], O.sampling(N, 8, 7, O.MIS), c1["pos"][sl], c1["nrm"][sl], c1["wo"][sl],
                     want_vis=False)[0]
        e = np.linalg.norm(a.cpu().numpy() - o, axis=1) / (np.linalg.norm(o, axis=1) + 1e-6)
        assert np.mean(e < 1e-4) >= (npix - 1) / npix

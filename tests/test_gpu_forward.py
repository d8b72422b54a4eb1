"""GPU parity of the forward entry points against the FP64 oracle (c1 sizes
and edge cases).  The FP32 path must match within 1e-5 norm-wise relative
error per output; hash indices must match bit-exactly."""
import math

import numpy as np
import pytest
import torch

import hg_inputs as H
import paper_2409_10327_amd as hg
from oracle import oracle as O
from helpers import adversarial_positions, c1_setup, max_rel, relerr

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-5


@pytest.fixture(scope="module")
def c1():
    cfg, model, env, pos, nrm, wo = c1_setup()
    om = O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT)
    oe = O.OracleEnv(env)
    r = hg.HashRenderer(model, DEV)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return dict(cfg=cfg, model=model, env=env, pos=pos, nrm=nrm, wo=wo, om=om, oe=oe, r=r,
                env_t=t(env), pos_t=t(pos), nrm_t=t(nrm), wo_t=t(wo), t=t)


def test_encode_indices_bit_exact(c1):
    print("case: encode index, c1 grid", flush=True)
    pos = adversarial_positions(c1["model"]["res"])
    idx, w = hg.encode_index(c1["r"], c1["t"](pos))
    torch.cuda.synchronize()
    oidx, ow = O.encode_index(c1["om"], pos)
    gi = idx.cpu().numpy().view(np.uint32)
    assert np.array_equal(gi, oidx), np.argwhere(gi != oidx)[:5]
    assert np.max(np.abs(w.cpu().numpy() - ow)) < 2e-7


def test_encode_features(c1):
    print("case: encode features, c1 grid", flush=True)
    pos = adversarial_positions(c1["model"]["res"], seed=1)
    f = hg.encode(c1["r"], c1["t"](pos)).cpu().numpy()
    of = O.encode(c1["om"], pos)
    assert relerr(f, of) < 1e-6
    # element-wise: a feature is a sum of 8 weight products w_k e_k; FP32
    # weights and accumulation bound its error by a few ulp of max|e|
    tmax = np.abs(c1["model"]["table"]).max(axis=(1, 2))  # per level
    bound = 2.0 ** -20 * np.repeat(tmax, 2)[None, :]
    assert np.all(np.abs(f - of) <= bound), np.max(np.abs(f - of) / bound)
    # exact reproduction at vertices of a level: weights are exactly 0/1
    N = c1["model"]["res"][9]  # 128
    k = np.random.default_rng(3).integers(0, N + 1, (500, 3))
    v = (H.BOX_LO + H.BOX_EXTENT * k / N).astype(np.float32)
    fv = hg.encode(c1["r"], c1["t"](v)).cpu().numpy()
    oidx, ow = O.encode_index(c1["om"], v)
    corner = (ow[:, 9, 0] == 1) * 1 + (ow[:, 9, 1] == 1) * 2 + (ow[:, 9, 2] == 1) * 4
    assert np.all(np.isin(ow[:, 9], [0.0, 1.0]))
    e = c1["model"]["table"][9][oidx[np.arange(500), 9, corner]]
    assert np.array_equal(fv[:, 18:20], e)


@pytest.mark.parametrize("indirect", [False, True])
def test_query_mode_parity(c1, indirect):
    print(f"case: query mode indirect={indirect}, c1 model, 4099 queries", flush=True)
    pos, dirs = H.make_train_batch(4099, seed=11)
    rgb, vis, dep = hg.render(c1["r"], c1["env_t"], c1["t"](pos), dirs=c1["t"](dirs), indirect=indirect)
    s = O.sampling(1, 8, 7, 0)
    orgb, ovis, odep = O.render(c1["om"], c1["oe"], s, pos, dirs=dirs, indirect=indirect)
    rgb, vis, dep = rgb.cpu().numpy(), vis.cpu().numpy(), dep.cpu().numpy()
    for a, b in ((rgb, orgb), (vis, ovis), (dep, odep)):
        assert relerr(a, b) < TOL, relerr(a, b)
        assert max_rel(a, b) < 1e-3


@pytest.mark.parametrize("indirect", [False, True])
def test_shade_mode_parity_c1(c1, indirect):
    print(f"case: shade mode indirect={indirect}, c1 frame 64x64 N=32", flush=True)
    cfg = c1["cfg"]
    rgb, vis, dep = hg.render(c1["r"], c1["env_t"], c1["pos_t"], c1["nrm_t"], c1["wo_t"], n_dirs=cfg.n_dirs,
                              n_dirs2=8, seed=H.SEED_DIRS, indirect=indirect, want_vis=True)
    s = O.sampling(cfg.n_dirs, 8, H.SEED_DIRS, 0)
    orgb, ovis, odep = O.render(c1["om"], c1["oe"], s, c1["pos"], c1["nrm"], c1["wo"], indirect=indirect)
    rgb, vis, dep = rgb.cpu().numpy(), vis.cpu().numpy(), dep.cpu().numpy()
    print("rel rgb %.3g vis %.3g dep %.3g; max_rel rgb %.3g" % (relerr(rgb, orgb), relerr(vis, ovis),
                                                                   relerr(dep, odep), max_rel(rgb, orgb)))
    for a, b in ((rgb, orgb), (vis, ovis), (dep, odep)):
        assert relerr(a, b) < TOL
        assert max_rel(a, b) < 1e-3


def test_shade_deterministic(c1):
    print("case: shade determinism", flush=True)
    cfg = c1["cfg"]
    a = hg.render(c1["r"], c1["env_t"], c1["pos_t"], c1["nrm_t"], c1["wo_t"], n_dirs=cfg.n_dirs)[0]
    b = hg.render(c1["r"], c1["env_t"], c1["pos_t"], c1["nrm_t"], c1["wo_t"], n_dirs=cfg.n_dirs)[0]
    assert torch.equal(a, b)


@pytest.mark.parametrize("N,npix", [(1, 37), (2, 65), (4, 130), (64, 3), (128, 5), (512, 2)])
def test_shade_sample_counts_and_ragged(c1, N, npix):
    print(f"case: shade N={N} npix={npix}", flush=True)
    sl = slice(100, 100 + npix)
    pos, nrm, wo = c1["pos"][sl], c1["nrm"][sl], c1["wo"][sl]
    t = c1["t"]
    rgb, vis, dep = hg.render(c1["r"], c1["env_t"], t(pos), t(nrm), t(wo), n_dirs=N, indirect=True,
                              want_vis=True)
    s = O.sampling(N, 8, 7, 0)
    orgb, ovis, odep = O.render(c1["om"], c1["oe"], s, pos, nrm, wo, indirect=True)
    assert relerr(rgb.cpu().numpy(), orgb) < TOL
    assert relerr(vis.cpu().numpy(), ovis) < TOL



@pytest.mark.parametrize("N,npix", [(1, 70), (8, 33)])
def test_shade_small_n_direct(c1, N, npix):
    """The per-lane mode (fewer than 16 directions) without the bounce."""
    print(f"case: direct shade N={N} npix={npix}", flush=True)
    sl = slice(300, 300 + npix)
    pos, nrm, wo = c1["pos"][sl], c1["nrm"][sl], c1["wo"][sl]
    t = c1["t"]
    rgb, vis, dep = hg.render(c1["r"], c1["env_t"], t(pos), t(nrm), t(wo), n_dirs=N, indirect=False,
                              want_vis=True)
    orgb, ovis, odep = O.render(c1["om"], c1["oe"], O.sampling(N, 8, 7, 0), pos, nrm, wo, indirect=False)
    assert relerr(rgb.cpu().numpy(), orgb) < TOL
    assert relerr(vis.cpu().numpy(), ovis) < TOL
    assert relerr(dep.cpu().numpy(), odep) < TOL


def test_empty_input_is_noop(c1):
    pos = torch.empty((0, 3), device=DEV)
    rgb, vis, dep = hg.render(c1["r"], c1["env_t"], pos, pos, pos, n_dirs=32)
    assert rgb.shape == (0, 3)
    assert hg.encode(c1["r"], pos).shape == (0, 32)


def furnace_params(model, v_logit, albedo, d_raw=0.0):
    p = dict(model)
    nf = 32

    def const(n_in, n_out, bias):
        return [np.zeros((64, n_in), np.float32), np.zeros(64, np.float32), np.zeros((64, 64), np.float32),
                np.zeros(64, np.float32), np.zeros((n_out, 64), np.float32), np.asarray(bias, np.float32)]
    lg = [math.log(a / (1 - a)) for a in albedo]
    p["brdf"] = const(nf, 5, lg + [0.0, -40.0])
    p["irt"] = const(nf + 3, 2, [v_logit, d_raw])
    return p


def test_furnace_and_two_bounce_on_gpu(c1):
    """Constant environment L, constant visibility c and albedo a, diffuse:
    L_o = a c L (1 + (1 - c) a) (c -> 1: the white furnace a L)."""
    print("case: furnace / two-bounce closed forms", flush=True)
    alb = (0.3, 0.6, 0.9)
    L_ = 2.0
    env = torch.full((8, 16, 3), L_, device=DEV)
    t = c1["t"]
    for c in (1.0 - 1e-12, 0.35):
        vl = 40.0 if c > 0.5 else math.log(c / (1 - c))
        r = hg.HashRenderer(furnace_params(c1["model"], vl, alb), DEV)
        rgb = hg.render(r, env, c1["pos_t"], c1["nrm_t"], c1["wo_t"], n_dirs=16, flags=hg.HG_DIFFUSE_ONLY)[0]
        aa = 1 / (1 + np.exp(-np.array([np.float32(math.log(a / (1 - a))) for a in alb], np.float64)))
        cc = 1 / (1 + math.exp(-float(np.float32(vl))))
        ref = aa * cc * L_ * (1 + (1 - cc) * aa)
        assert np.max(np.abs(rgb.cpu().numpy() / ref - 1)) < 2e-6
    del t

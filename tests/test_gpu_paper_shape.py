"""The paper's model shape (Sec. 4.1): 14 levels, T = 2^17, resolutions 16 to
131072, decoder with a normal head, against the FP64 oracle (64x64 frame).

Bars.  Encode indices are bit-exact and the direct path meets the FP32 bar
(1e-5 norm-wise).  The bounce is ill-conditioned at this shape: a cell of
the finest level spans 128 FP32 steps of a coordinate near 8, and the bounce
point x' = x + t w moves with the tracer's depth output t, which an FP32
implementation only has to a few 1e-7 relative.  Perturbing t by a relative
1e-7 / 1e-6 inside a copy of the oracle moves the 64x64 frame by 2.2e-4 /
1.7e-3 and query-mode radiance by 6.5e-4 / 4.6e-3 (norm-wise), so the
indirect bars are 5e-3 (frame) and 1e-2 (query).  The query-mode gradients
move by 1.4e-2 (table) at 1e-7 already, so with the finest level at 131072
the indirect gradient check is only a sanity bound; 14 levels up to 2048
keep the FP32 bar.  The mixed path is held to 45 dB PSNR."""
import numpy as np
import pytest
import torch

import hg_inputs as H
import paper_2409_10327_amd as hg
from oracle import oracle as O
from helpers import kink_margin, psnr, relerr

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL_DIRECT = 1e-5
TOL_FRAME = 5e-3
TOL_QUERY = 1e-2


@pytest.fixture(scope="module")
def ps():
    cfg = H.config("paper_small")
    model = H.make_model(cfg)
    env = H.make_env(cfg.env_h, cfg.env_w)
    pos, nrm, wo = H.make_scene(cfg.img_h, cfg.img_w)
    r = hg.HashRenderer(model, DEV)
    r.refresh_shadows()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return dict(cfg=cfg, model=model, env=env, pos=pos, nrm=nrm, wo=wo, r=r, t=t, env_t=t(env),
                om=O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT), oe=O.OracleEnv(env))


def test_encode_paper_levels(ps):
    print("case: encode, 14 levels to 131072", flush=True)
    rng = np.random.default_rng(2)
    pos = rng.uniform(-9, 9, (20000, 3)).astype(np.float32)
    f = hg.encode(ps["r"], ps["t"](pos)).cpu().numpy()
    assert f.shape == (20000, 28)
    assert relerr(f, O.encode(ps["om"], pos)) < 1e-6
    idx, w = hg.encode_index(ps["r"], ps["t"](pos))
    oidx, ow = O.encode_index(ps["om"], pos)
    assert np.array_equal(idx.cpu().numpy().view(np.uint32), oidx)
    assert np.max(np.abs(w.cpu().numpy() - ow)) < 1e-6


@pytest.mark.parametrize("indirect", [False, True])
def test_frame_fp32(ps, indirect):
    print(f"case: paper-shape frame 64x64 N=32 indirect={indirect}", flush=True)
    t = ps["t"]
    rgb, vis, dep = hg.render(ps["r"], ps["env_t"], t(ps["pos"]), t(ps["nrm"]), t(ps["wo"]), n_dirs=32,
                              indirect=indirect, want_vis=True)
    orgb, ovis, odep = O.render(ps["om"], ps["oe"], O.sampling(32, 8, 7, 0), ps["pos"], ps["nrm"], ps["wo"],
                                indirect=indirect)
    rgb, vis, dep = rgb.cpu().numpy(), vis.cpu().numpy(), dep.cpu().numpy()
    e = relerr(rgb, orgb)
    print(f"paper shape indirect={indirect}: rgb {e:.3g}, vis {relerr(vis, ovis):.3g}, dep {relerr(dep, odep):.3g}")
    assert relerr(vis, ovis) < TOL_DIRECT and relerr(dep, odep) < TOL_DIRECT
    assert e < (TOL_FRAME if indirect else TOL_DIRECT)


def test_frame_mixed(ps):
    print("case: paper-shape frame mixed N=32", flush=True)
    t = ps["t"]
    rgb = hg.render(ps["r"], ps["env_t"], t(ps["pos"]), t(ps["nrm"]), t(ps["wo"]), n_dirs=32,
                    precision="mixed")[0].cpu().numpy()
    orgb = O.render(ps["om"], ps["oe"], O.sampling(32, 8, 7, 0), ps["pos"], ps["nrm"], ps["wo"], want_vis=False)[0]
    p = psnr(rgb, orgb)
    print(f"paper shape mixed: PSNR {p:.1f} dB, rel err {relerr(rgb, orgb):.3g}")
    assert p >= 45.0


@pytest.mark.parametrize("n", [1, 4099])
def test_query_mode(ps, n):
    print(f"case: paper-shape query mode n={n}", flush=True)
    pos, dirs = H.make_train_batch(n, seed=12)
    t = ps["t"]
    rgb, vis, dep = hg.render(ps["r"], ps["env_t"], t(pos), dirs=t(dirs))
    orgb, ovis, odep = O.render(ps["om"], ps["oe"], O.sampling(1, 8, 7, 0), pos, dirs=dirs)
    assert relerr(vis.cpu().numpy(), ovis) < TOL_DIRECT
    assert relerr(rgb.cpu().numpy(), orgb) < TOL_QUERY


def test_normal_head_changes_the_bounce(ps):
    """The same weights with the normal head dropped (5 outputs, facing
    normal) render a different frame, and each variant matches its oracle."""
    print("case: normal head vs facing normal", flush=True)
    m5 = dict(ps["model"])
    m5["brdf"] = ps["model"]["brdf"][:4] + [ps["model"]["brdf"][4][:5], ps["model"]["brdf"][5][:5]]
    r5 = hg.HashRenderer(m5, DEV)
    t = ps["t"]
    args = (ps["env_t"], t(ps["pos"]), t(ps["nrm"]), t(ps["wo"]))
    a = hg.render(ps["r"], *args, n_dirs=32)[0].cpu().numpy()
    b = hg.render(r5, *args, n_dirs=32)[0].cpu().numpy()
    ob = O.render(O.OracleModel(m5, H.BOX_LO, H.BOX_EXTENT), ps["oe"], O.sampling(32, 8, 7, 0), ps["pos"],
                  ps["nrm"], ps["wo"], want_vis=False)[0]
    print(f"normal head vs facing: {relerr(a, b):.3g}; facing vs oracle {relerr(b, ob):.3g}")
    assert relerr(a, b) > 1e-2
    assert relerr(b, ob) < TOL_FRAME


def _grads_natural(r, g):
    return dict(table=g["table"].cpu().numpy(), brdf=[x.cpu().numpy() for x in r.natural(g["brdf"], "brdf")],
                irt=[x.cpu().numpy() for x in r.natural(g["irt"], "irt")])


@pytest.mark.parametrize("res_max,indirect", [(2048, False), (2048, True), (131072, False), (131072, True)])
def test_backward_14_levels(ps, res_max, indirect):
    """14 levels with the 5-output decoder (the normal head is forward
    only): gradients against the oracle, with the level-slot columns of the
    missing levels receiving exactly zero.  Samples within FP32 rounding of
    a network kink are excluded.  With the finest level at 131072 the
    indirect gradients are ill-conditioned (see the module docstring: the
    depth head's gradient carries the finest level's spatial derivative,
    8192 per unit, and the decoder's first-layer gradient the finest
    features), so that case only checks the table gradient to 0.25; with the
    finest level at 2048 the FP32 bar holds."""
    print(f"case: backward, 14 levels to {res_max}, indirect={indirect}", flush=True)
    cfg = H.Config("b14", n_levels=14, log2_T=17, res_min=16, res_max=res_max)
    m5 = H.make_model(cfg)
    m5["irt"][5] = np.array([0.2, -0.5], np.float32)
    r5 = hg.HashRenderer(m5, DEV)
    n = 1030
    pos, dirs = H.make_train_batch(n, seed=21)
    rng = np.random.default_rng(5)
    g_rgb = rng.standard_normal((n, 3)).astype(np.float32)
    g_vis = rng.standard_normal(n).astype(np.float32)
    g_dep = rng.standard_normal(n).astype(np.float32)
    om5 = O.OracleModel(m5, H.BOX_LO, H.BOX_EXTENT)
    dep = O.render(om5, ps["oe"], O.sampling(1, 8, 7, 0), pos, dirs=dirs, indirect=indirect)[2]
    # indirect with the finest level at 2048: margin 1e-4 and bar 3e-4 (a
    # relative depth perturbation of 4e-7 / 1e-6 in a copy of the oracle
    # moves the worst array by 8.5e-5 / 2.1e-4); the direct path keeps 1e-5
    thr = 1e-4 if indirect else 1e-5
    keep = (kink_margin(m5, pos, dirs, dep, indirect) >= thr).astype(np.float32)
    g_rgb, g_vis, g_dep = g_rgb * keep[:, None], g_vis * keep, g_dep * keep
    t = ps["t"]
    grads = hg.zero_grads(r5)
    hg.backward(r5, ps["env_t"], t(pos), t(dirs), t(g_rgb), t(g_vis), t(g_dep), grads, indirect=indirect)
    assert torch.all(grads["brdf"][0][:, 28:] == 0) and torch.all(grads["irt"][0][:, 28:32] == 0)
    G = _grads_natural(r5, grads)
    ref = O.backward(om5, ps["oe"], O.sampling(1, 8, 7, 0), pos, dirs, g_rgb, g_vis, g_dep, indirect=indirect)
    e = relerr(G["table"], ref["table"])
    print(f"backward 14 levels to {res_max} indirect={indirect}: table {e:.3g}")
    if indirect and res_max > 2048:
        assert e < 0.25
        return
    tol = 3e-4 if indirect else TOL_DIRECT
    assert e < tol
    for k in ("brdf", "irt"):
        for i in range(6):
            if not indirect and k == "brdf":
                continue
            assert relerr(G[k][i], ref[k][i]) < tol, (k, i, relerr(G[k][i], ref[k][i]))


def test_backward_rejects_normal_head(ps):
    n = 64
    pos, dirs = H.make_train_batch(n, seed=3)
    t = ps["t"]
    z = torch.zeros(n, device=DEV)
    with pytest.raises(hg.HGError) as ei:
        hg.backward(ps["r"], ps["env_t"], t(pos), t(dirs), torch.zeros((n, 3), device=DEV), z, z,
                    hg.zero_grads(ps["r"]))
    assert ei.value.status == hg.HG_E_UNSUPPORTED

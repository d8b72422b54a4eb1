"""GPU parity of the spatial SVGF filter (hg_denoise) against the FP64 oracle,
on the oracle's own render of the 64x64 analytic frame and on ragged sizes."""
import numpy as np
import pytest
import torch

import hg_inputs as H
import paper_2409_10327_amd as hg
from oracle import oracle as O
from helpers import c1_setup, relerr

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def frame():
    cfg, model, env, pos, nrm, wo = c1_setup()
    om, oe = O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT), O.OracleEnv(env)
    rgb = O.render(om, oe, O.sampling(16, 8, 7, 0), pos, nrm, wo, want_vis=False)[0].astype(np.float32)
    cam = H.camera()
    depth = np.linalg.norm(pos.astype(np.float64) - cam, axis=1).astype(np.float32)
    h, w = cfg.img_h, cfg.img_w
    return rgb.reshape(h, w, 3), depth.reshape(h, w), nrm.reshape(h, w, 3)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("iters", [0, 1, 5])
def test_denoise_frame(frame, iters):
    print(f"case: denoise 64x64 iters={iters}", flush=True)
    rgb, depth, nrm = frame
    out = hg.denoise(gpu(rgb), gpu(depth), gpu(nrm), iterations=iters).cpu().numpy()
    ref = O.denoise(rgb, depth, nrm, iters=iters) if iters else rgb
    e = relerr(out, ref)
    print(f"denoise iters={iters}: rel err {e:.3g}, noise std in {np.std(rgb):.3g} out {np.std(out):.3g}")
    assert e < 1e-4


@pytest.mark.parametrize("h,w", [(1, 1), (17, 33), (5, 200)])
def test_denoise_ragged(h, w):
    print(f"case: denoise ragged {h}x{w}", flush=True)
    rng = np.random.default_rng(h * 1000 + w)
    rgb = np.exp(rng.standard_normal((h, w, 3))).astype(np.float32)
    depth = rng.uniform(1, 3, (h, w)).astype(np.float32)
    n = rng.standard_normal((h, w, 3))
    n = (n / np.linalg.norm(n, axis=2, keepdims=True)).astype(np.float32)
    out = hg.denoise(gpu(rgb), gpu(depth), gpu(n)).cpu().numpy()
    assert relerr(out, O.denoise(rgb, depth, n)) < 1e-4


def test_denoise_workspace_checked(frame):
    rgb, depth, nrm = frame
    small = torch.empty(16, device=DEV)
    prm = hg.DenoiseParams(5, 1.0, 128.0, 4.0)
    st = hg.lib().hg_denoise(hg._ptr(gpu(rgb)), hg._ptr(gpu(depth)), hg._ptr(gpu(nrm)), 64, 64, hg.C.byref(prm),
                             hg._ptr(gpu(rgb)), hg._ptr(small), 64, None)
    assert st == hg.HG_E_INVALID

"""hg_denoise_noalloc (static device workspace, for callers that cannot
allocate) against hg_denoise with a caller workspace: the same kernels, so the
frames must agree bit for bit.  Two calls in a row, the second smaller, so the
second runs on a workspace that still holds the first call's contents."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2409_10327_amd as hg

pytestmark = pytest.mark.gpu
DEV = "cuda"


def inputs(h, w, seed):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float32)
    rgb = rng.lognormal(0.0, 1.0, (h, w, 3)).astype(np.float32)
    depth = (3.0 + 0.01 * xx + 0.02 * yy + 0.05 * (xx > w // 2)).astype(np.float32)
    n = rng.normal(size=(h, w, 3)) + np.array([0.0, 0.0, 3.0])
    n = (n / np.linalg.norm(n, axis=-1, keepdims=True)).astype(np.float32)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return g(rgb), g(depth), g(n)


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    L = hg.lib()
    prm = hg.DenoiseParams(5, 1.0, 128.0, 4.0)
    # one pixel past the static workspace: rejected on the host, nothing launched
    f = torch.zeros(16, device=DEV)
    assert L.hg_denoise_noalloc(hg._ptr(f), hg._ptr(f), hg._ptr(f), 1024, 1025, C.byref(prm), hg._ptr(f),
                                None) == hg.HG_E_INVALID
    assert "static workspace" in L.hg_last_error().decode()
    for h, w, seed, iters in ((1024, 1024, 11, 5), (37, 53, 12, 5), (37, 53, 13, 0)):
        print(f"case: hg_denoise_noalloc {h}x{w} iters={iters} seed={seed}", flush=True)
        rgb, depth, nrm = inputs(h, w, seed)
        out = torch.full_like(rgb, float("nan"))
        hg.denoise_noalloc(rgb, depth, nrm, out, iterations=iters)
        ref = hg.denoise(rgb, depth, nrm, iterations=iters)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), (h, w, (out - ref).abs().max().item())

"""GPU parity of the training entry points (backward, loss, Adam) against the
FP64 oracle, plus the FP64 central-difference check of the GPU gradients."""
import numpy as np
import pytest
import torch

import hg_inputs as H
import paper_2409_10327_amd as hg
from oracle import oracle as O
from helpers import grad_condition, kink_margin, relerr

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def setup():
    cfg = H.config("c1")
    model = H.make_model(cfg)
    # keep the depth head off its clamp so the bounce-point path is exercised
    model["irt"][5] = np.array([0.2, -0.5], np.float32)
    env = H.make_env(cfg.env_h, cfg.env_w)
    r = hg.HashRenderer(model, DEV)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    om, oe = O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT), O.OracleEnv(env)
    return dict(cfg=cfg, model=model, env=env, r=r, t=t, om=om, oe=oe, env_t=t(env))


@pytest.mark.parametrize("indirect", [True, False])
@pytest.mark.parametrize("n", [1, 77, 1030])
def test_backward_parity(setup, indirect, n):
    print(f"case: backward indirect={indirect} n={n}", flush=True)
    t = setup["t"]
    pos, dirs = H.make_train_batch(n, seed=21)
    rng = np.random.default_rng(5)
    g_rgb = rng.standard_normal((n, 3)).astype(np.float32)
    g_vis = rng.standard_normal(n).astype(np.float32)
    g_dep = rng.standard_normal(n).astype(np.float32)
    # samples within FP32 rounding of a ReLU kink (or the depth clamp) take
    # different branches in FP32 and FP64: their gradients are excluded
    dep = O.render(setup["om"], setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs=dirs, indirect=indirect)[2]
    keep = (kink_margin(setup["model"], pos, dirs, dep, indirect) >= 1e-5).astype(np.float32)
    print(f"{int(n - keep.sum())} of {n} samples within FP32 rounding of a kink")
    g_rgb, g_vis, g_dep = g_rgb * keep[:, None], g_vis * keep, g_dep * keep
    grads = hg.zero_grads(setup["r"])
    g_pos = torch.empty((n, 3), device=DEV)
    hg.backward(setup["r"], setup["env_t"], t(pos), t(dirs), t(g_rgb), t(g_vis), t(g_dep), grads,
                indirect=indirect, g_pos=g_pos)
    ref = O.backward(setup["om"], setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs, g_rgb, g_vis, g_dep,
                     indirect=indirect, want_pos=True)
    assert relerr(grads["table"].cpu().numpy(), ref["table"]) < 1e-5
    for k in ("brdf", "irt"):
        for i in range(6):
            a, b = grads[k][i].cpu().numpy(), ref[k][i]
            if not indirect and k == "brdf":
                assert np.all(a == 0) and np.all(b == 0)
                continue
            assert relerr(a, b) < 1e-5, (k, i, relerr(a, b))
    k = keep > 0
    assert relerr(g_pos.cpu().numpy()[k], ref["pos"][k]) < 1e-5


def test_gpu_gradients_vs_central_differences(setup):
    """64 sampled parameters (32 table entries across levels, 32 MLP
    weights/biases across both MLPs and all layers): GPU analytic gradient
    of L = sum(g . outputs) vs FP64 central differences of the oracle."""
    print("case: GPU gradients vs FP64 central differences", flush=True)
    from test_oracle_pins import _fd
    model, env = setup["model"], setup["env"]
    n = 64
    pos, dirs = H.make_train_batch(n, seed=31)
    rng = np.random.default_rng(7)
    g_rgb = rng.standard_normal((n, 3)).astype(np.float32)
    g_vis = rng.standard_normal(n).astype(np.float32)
    g_dep = rng.standard_normal(n).astype(np.float32)
    t = setup["t"]
    grads = hg.zero_grads(setup["r"])
    hg.backward(setup["r"], setup["env_t"], t(pos), t(dirs), t(g_rgb), t(g_vis), t(g_dep), grads)
    G = dict(table=grads["table"].cpu().numpy(), brdf=[g.cpu().numpy() for g in grads["brdf"]],
             irt=[g.cpu().numpy() for g in grads["irt"]])
    samp = O.sampling(1, 8, 7, 0)
    cand = []
    nz = np.argwhere(np.abs(G["table"]) > 1e-5)
    levels = np.unique(nz[:, 0])
    per = max(1, 32 // len(levels))
    for l in levels:
        rows = nz[nz[:, 0] == l]
        for r in rows[rng.permutation(len(rows))[:per]]:
            cand.append(("table", tuple(r)))
    for k in ("brdf", "irt"):
        for i in range(6):
            flat = np.argwhere(np.abs(G[k][i]) > 1e-6)
            for r in flat[rng.permutation(len(flat))[:6]]:
                cand.append(((k, i), tuple(r)))
    checked = 0
    for key, index in cand:
        if checked >= 64:
            break
        ana = G["table"][index] if key == "table" else G[key[0]][key[1]][index]
        fd1 = _fd(model, key, index, env, pos, dirs, g_rgb, g_vis, g_dep, samp, 1e-4)
        fd2 = _fd(model, key, index, env, pos, dirs, g_rgb, g_vis, g_dep, samp, 2.5e-5)
        scale = max(abs(fd1), abs(fd2), 1e-3)
        if abs(fd1 - fd2) > 1e-6 * scale:
            continue
        assert abs(ana - fd1) <= 1e-4 * scale + 1e-6, (key, index, ana, fd1)
        checked += 1
    assert checked >= 48, checked


@pytest.mark.parametrize("n", [1, 1 << 14, 300001])  # 300001: more samples than threads of the capped grid
def test_l2_loss_parity(setup, n):
    t = setup["t"]
    rng = np.random.default_rng(2)
    rgb = rng.standard_normal((n, 3)).astype(np.float32)
    vis = rng.uniform(0, 1, n).astype(np.float32)
    dep = rng.uniform(0, 1, n).astype(np.float32)
    tgt = H.make_targets(n)
    loss, gr, gv, gd = hg.l2_loss(t(rgb), t(vis), t(dep), t(tgt))
    ol, ogr, ogv, ogd = O.l2_loss(rgb, vis, dep, tgt)
    assert abs(loss.item() / ol - 1) < 1e-5
    for a, b in ((gr, ogr), (gv, ogv), (gd, ogd)):
        assert relerr(a.cpu().numpy(), b) < 1e-6


@pytest.mark.parametrize("n,shadow", [(1, None), (1027, "f16"), (4096, "bf16")])
def test_adam_parity(setup, n, shadow):
    t = setup["t"]
    rng = np.random.default_rng(3)
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (rng.standard_normal(n) * 0.1).astype(np.float32)
    v = rng.uniform(0, 0.1, n).astype(np.float32)
    pt, mt, vt = t(p), t(m), t(v)
    sh = None
    if shadow == "f16":
        sh = torch.empty(n, dtype=torch.float16, device=DEV)
    elif shadow == "bf16":
        sh = torch.empty(n, dtype=torch.bfloat16, device=DEV)
    hg.adam_step(pt, t(g), mt, vt, 3, lr=2e-3, weight_decay=1e-6, shadow=sh)
    # the library receives FP32 hyper-parameters; the oracle gets the same values
    f = lambda x: float(np.float32(x))
    op, om_, ov = O.adam(p, g, m, v, 3, lr=f(2e-3), b1=f(0.9), b2=f(0.999), eps=f(1e-8), wd=f(1e-6))
    assert relerr(pt.cpu().numpy(), op) < 1e-6
    assert relerr(mt.cpu().numpy(), om_) < 1e-6 and relerr(vt.cpu().numpy(), ov) < 1e-6
    if sh is not None:
        assert torch.equal(sh, pt.to(sh.dtype))


def test_autograd_function_matches_backward(setup):
    t = setup["t"]
    r = setup["r"]
    n = 300
    pos, dirs = H.make_train_batch(n, seed=41)
    params = [r.table] + r.brdf + r.irt
    for p_ in params:
        p_.requires_grad_(True)
    try:
        rgb, vis, dep = hg.HGQueryFn.apply(r, setup["env_t"], t(pos), t(dirs), 8, 7, True, "fp32", *params)
        (rgb.sum() + 2 * vis.sum() - dep.sum()).backward()
        grads = hg.zero_grads(r)
        ones = torch.ones((n, 3), device=DEV)
        hg.backward(r, setup["env_t"], t(pos), t(dirs), ones, torch.full((n,), 2.0, device=DEV),
                    torch.full((n,), -1.0, device=DEV), grads)
        assert relerr(r.table.grad.cpu().numpy(), grads["table"].cpu().numpy()) < 1e-6
        for a, b in zip(r.irt, grads["irt"]):
            assert relerr(a.grad.cpu().numpy(), b.cpu().numpy()) < 1e-6
    finally:
        for p_ in params:
            p_.requires_grad_(False)
            p_.grad = None


@pytest.mark.parametrize("indirect", [True, False])
def test_backward_f16_table(setup, indirect):
    """The mixed training step's backward gathers the FP16 table shadow with
    the FP32 master MLPs: it equals the oracle's backward on the FP16-rounded
    table (same kink mask and bar as the FP32 backward)."""
    print(f"case: backward with FP16 tables, indirect={indirect}", flush=True)
    t = setup["t"]
    r = setup["r"]
    r.refresh_shadows()
    m16 = dict(setup["model"])
    m16["table"] = setup["model"]["table"].astype(np.float16).astype(np.float32)
    om16 = O.OracleModel(m16, H.BOX_LO, H.BOX_EXTENT)
    n = 1030
    pos, dirs = H.make_train_batch(n, seed=23)
    rng = np.random.default_rng(6)
    g_rgb = rng.standard_normal((n, 3)).astype(np.float32)
    g_vis = rng.standard_normal(n).astype(np.float32)
    g_dep = rng.standard_normal(n).astype(np.float32)
    dep = O.render(om16, setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs=dirs, indirect=indirect)[2]
    keep = (kink_margin(m16, pos, dirs, dep, indirect) >= 1e-5).astype(np.float32)
    g_rgb, g_vis, g_dep = g_rgb * keep[:, None], g_vis * keep, g_dep * keep
    grads = hg.zero_grads(r)
    hg.backward(r, setup["env_t"], t(pos), t(dirs), t(g_rgb), t(g_vis), t(g_dep), grads, indirect=indirect,
                precision="f16table")
    ref = O.backward(om16, setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs, g_rgb, g_vis, g_dep, indirect=indirect)
    assert relerr(grads["table"].cpu().numpy(), ref["table"]) < 1e-5
    for k in ("brdf", "irt"):
        for i in range(6):
            if not indirect and k == "brdf":
                continue
            assert relerr(grads[k][i].cpu().numpy(), ref[k][i]) < 1e-5, (k, i)


def morton_sorted(pos, dirs):
    """Batch reordered along a Morton curve (what the benchmark's training
    step does): lanes of a wave then share cells at most levels."""
    lo, hi = pos.min(0), pos.max(0)
    q = np.clip(((pos - lo) / (hi - lo) * 1023).astype(np.int64), 0, 1023)

    def spread(v):
        v = (v | (v << 16)) & 0x030000FF
        v = (v | (v << 8)) & 0x0300F00F
        v = (v | (v << 4)) & 0x030C30C3
        return (v | (v << 2)) & 0x09249249
    order = np.argsort(spread(q[:, 0]) | (spread(q[:, 1]) << 1) | (spread(q[:, 2]) << 2), kind="stable")
    return pos[order], dirs[order]


@pytest.mark.parametrize("indirect", [True, False])
def test_backward_parity_spatially_sorted_batch(setup, indirect):
    """A Morton-ordered batch drives the backward's per-cell summation of the
    table gradient at most levels (groups of lanes sharing a cell); gradients
    still match the oracle at the FP32 bar.  Each MLP parameter gradient is a
    sum over samples; where its terms cancel, FP32 rounding of the terms
    (a few ulps each, 2^-20) is amplified by the sum's condition number
    kappa (measured with the oracle), so the bar is max(1e-5, kappa 2^-20)
    (kappa reaches about 90 for the tracer's output bias here)."""
    print(f"case: backward on a Morton-ordered batch, indirect={indirect}", flush=True)
    t = setup["t"]
    n = 4096
    pos, dirs = morton_sorted(*H.make_train_batch(n, seed=29))
    rng = np.random.default_rng(8)
    g_rgb = rng.standard_normal((n, 3)).astype(np.float32)
    g_vis = rng.standard_normal(n).astype(np.float32)
    g_dep = rng.standard_normal(n).astype(np.float32)
    dep = O.render(setup["om"], setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs=dirs, indirect=indirect)[2]
    keep = (kink_margin(setup["model"], pos, dirs, dep, indirect) >= 1e-5).astype(np.float32)
    g_rgb, g_vis, g_dep = g_rgb * keep[:, None], g_vis * keep, g_dep * keep
    grads = hg.zero_grads(setup["r"])
    hg.backward(setup["r"], setup["env_t"], t(pos), t(dirs), t(g_rgb), t(g_vis), t(g_dep), grads, indirect=indirect)
    ref = O.backward(setup["om"], setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs, g_rgb, g_vis, g_dep,
                     indirect=indirect)
    assert relerr(grads["table"].cpu().numpy(), ref["table"]) < 1e-5
    kappa = grad_condition(setup["om"], setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs, g_rgb, g_vis, g_dep, indirect)
    for k in ("brdf", "irt"):
        for i in range(6):
            if not indirect and k == "brdf":
                continue
            bar = max(1e-5, kappa[(k, i)] * 2.0 ** -20)
            e = relerr(grads[k][i].cpu().numpy(), ref[k][i])
            print(f"{k}[{i}]: rel err {e:.3g}, kappa {kappa[(k, i)]:.3g}, bar {bar:.3g}")
            assert e < bar, (k, i, e, bar)


def _cos(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("indirect", [True, False])
@pytest.mark.parametrize("n", [77, 1030])
def test_backward_bf16_parity(setup, indirect, n):
    """BF16 matrix-core backward of the mixed MLPs (FP16 tables, BF16
    weights, activations and deltas, FP32 accumulation and gradients) against
    the FP64 oracle on the FP32 masters.  BF16 keeps 8 significand bits, so a
    per-sample gradient term carries ~2^-8 relative rounding, and a gradient
    array (a sum over samples with random upstream gradients) moves by that
    times its cancellation, and a pre-activation within BF16 rounding of zero
    can flip its ReLU mask against FP64 (with few samples a few flips weigh
    more): measured 4e-5 .. 0.2 norm-wise at c1 (about 8x the FP16-table
    backward's error, as the 3 fewer significand bits give; the first layer
    and the table at 77 samples the worst), cosines 0.983 and above.  A
    mapping mistake (a transposed tile, a missing ReLU mask, a shifted bias
    or direction column) would turn an array away from the oracle's instead:
    every array, and the tracer's direction columns on their own, must keep a
    cosine of at least 0.97 with it and a relative error of at most 0.3."""
    print(f"case: BF16 backward indirect={indirect} n={n}", flush=True)
    t = setup["t"]
    r = setup["r"]
    r.refresh_shadows()
    pos, dirs = H.make_train_batch(n, seed=23)
    rng = np.random.default_rng(6)
    g_rgb = rng.standard_normal((n, 3)).astype(np.float32)
    g_vis = rng.standard_normal(n).astype(np.float32)
    g_dep = rng.standard_normal(n).astype(np.float32)
    grads = hg.zero_grads(r)
    hg.backward(r, setup["env_t"], t(pos), t(dirs), t(g_rgb), t(g_vis), t(g_dep), grads, indirect=indirect,
                precision="mixed")
    ref = O.backward(setup["om"], setup["oe"], O.sampling(1, 8, 7, 0), pos, dirs, g_rgb, g_vis, g_dep,
                     indirect=indirect)
    pairs = [("table", grads["table"].cpu().numpy(), ref["table"])]
    for k in ("brdf", "irt"):
        for i in range(6):
            pairs.append((f"{k}{i}", grads[k][i].cpu().numpy(), ref[k][i]))
    pairs.append(("irt0 direction columns", grads["irt"][0].cpu().numpy()[:, 32:], ref["irt"][0][:, 32:]))
    for name, a, b in pairs:
        if not indirect and name.startswith("brdf"):
            assert np.all(a == 0) and np.all(b == 0), name
            continue
        e, c = relerr(a, b), _cos(a, b)
        print(f"  {name}: rel {e:.3g} cos {c:.5f}")
        assert np.all(np.isfinite(a)), name
        assert c >= 0.97 and e <= 0.3, (name, e, c)


def _morton63_ref(pos, lo, extent):
    """Keys of hg_morton_order written out in numpy: the FP32 cell per axis
    (subtract, then multiply by the power of two 2^21 / extent: both steps
    round as on the GPU), clamped, NaN to cell 0, bits interleaved x lowest."""
    f = (pos - np.float32(lo)) * np.float32(2.0 ** 21 / extent)
    f = np.where(np.isnan(f), np.float32(0), f)
    q = np.clip(f, 0, 2 ** 21 - 1).astype(np.uint64)
    key = np.zeros(pos.shape[0], np.uint64)
    for d in range(3):
        for b in range(21):
            key |= ((q[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return key


@pytest.mark.parametrize("n", [1, 7, 1000, 262147])
def test_morton_order_is_stable_key_order(n):
    rng = np.random.default_rng(n)
    pos = rng.uniform(-1.0, 1.0, (n, 3)).astype(np.float32)
    if n >= 7:
        # outside the box, on its faces, non-finite, and repeated points (ties)
        pos[0] = (-9.0, 9.0, 0.0)
        pos[1] = (-8.0, 8.0, 7.9999995)
        pos[2] = (np.nan, 0.5, -0.5)
        pos[3] = (np.inf, -np.inf, 0.0)
        pos[5] = pos[4]
        pos[6] = pos[4]
    r = hg.HashRenderer(H.make_model(H.config("c1")), "cuda")
    perm = hg.morton_order(r, torch.from_numpy(pos).cuda()).cpu().numpy()
    ref = np.argsort(_morton63_ref(pos, r.box_lo, r.box_extent), kind="stable")
    assert perm.dtype == np.int32
    assert np.array_equal(perm, ref.astype(np.int32))


def test_morton_order_empty():
    r = hg.HashRenderer(H.make_model(H.config("c1")), "cuda")
    assert hg.morton_order(r, torch.empty((0, 3), device="cuda")).numel() == 0


@pytest.mark.parametrize("zero_grad", [False, True])
def test_adam_multi_matches_single(zero_grad):
    """hg_adam_step_multi against hg_adam_step tensor by tensor: parameters,
    moments and shadows bit-identical over ragged sizes and both shadow
    types; gradients cleared exactly when asked."""
    rng = np.random.default_rng(11)
    sizes = [1, 3, 4, 5, 1000, 4097, 262147]
    kinds = [None, torch.float16, torch.bfloat16, None, torch.bfloat16, torch.float16, None]
    def make():
        out = []
        for i, (n, k) in enumerate(zip(sizes, kinds)):
            r = np.random.default_rng(100 + i)
            p = torch.from_numpy(r.standard_normal(n).astype(np.float32)).cuda()
            g = torch.from_numpy(r.standard_normal(n).astype(np.float32)).cuda()
            m = torch.from_numpy(r.standard_normal(n).astype(np.float32) * 0.1).cuda()
            v = torch.from_numpy(np.abs(r.standard_normal(n)).astype(np.float32) * 0.01).cuda()
            sh = None if k is None else torch.empty(n, device="cuda", dtype=k)
            out.append([p, g, m, v, 1e-6 * (i % 2), sh])
        return out
    a, b = make(), make()
    for step in (1, 2):
        for p, g, m, v, wd, sh in a:
            hg.adam_step(p, g, m, v, step, lr=2e-3, weight_decay=wd, shadow=sh)
        gb = [x[1].clone() for x in b]
        hg.adam_step_multi([tuple(x) for x in b], step, lr=2e-3, zero_grad=zero_grad)
        torch.cuda.synchronize()
        for x, y, g0 in zip(a, b, gb):
            for u, w in zip((x[0], x[2], x[3]), (y[0], y[2], y[3])):
                assert torch.equal(u, w)
            if x[5] is not None:
                assert torch.equal(x[5].view(torch.int16), y[5].view(torch.int16))
            if zero_grad:
                assert torch.count_nonzero(y[1]).item() == 0
                y[1].copy_(g0)  # the next step reuses the same gradients
            else:
                assert torch.equal(y[1], g0)

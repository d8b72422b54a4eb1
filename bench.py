"""Benchmark of the hash-grid secondary-ray renderer on one MI355X.

A step renders one 800x800 frame of the analytic scene with 128 stratified
directions per pixel and one indirect bounce with 8 secondary directions
(81.92M secondary queries, FP32 path), the frame-size workload.  The same
run also times the mixed-precision frame (FP16 tables, BF16 matrix-core
MLPs) when available, and one distillation training step (query-mode forward
over 2^18 samples, L2 loss, hand-written backward, Adam), and reports the
FP64 oracle on a bounded pixel subset on the host's cores.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0

# Algorithmic work per secondary query (one (pixel, direction) pair):
# tracer at x with the first layer split into a per-point part and a
# direction part (3*64 + 64*64 + 64*2 MAC), decoder at x' (32*64 + 64*64 +
# 64*5), the per-point part at x' (32*64) and N' = 8 direction parts:
# 4416 + 6464 + 2048 + 8*4416 = 48,256 MAC = 96,512 FLOP.
FLOP_PER_QUERY = 2 * (4416 + 6464 + 2048 + 8 * 4416)

# Backward of one query-mode training sample (hg_backward): the recomputed
# forward (tracer at (x, w) 35*64 + 64*64 + 64*2, decoder at x', the tracer's
# point part at x' and 8 direction parts) plus, per layer, the weight
# gradient (fan_in * fan_out MAC) and the input gradient (the same, except
# for the direction inputs of the tracer): tracer at x 6464 + 6464 + 6272,
# decoder 6464 + 6464 + 6464, bounce tracer 37376 + 51712 + 50176
# = 177,856 MAC.  Table-gradient scatter: 2 encodes x 16 levels x 8 corners
# x 2 features = 512 FP32 adds per sample before any aggregation.
BWD_FLOP_PER_SAMPLE = 2 * (6464 + 6464 + 6272 + 6464 + 6464 + 6464 + 37376 + 51712 + 50176)
ATOMICS_PER_SAMPLE = 512


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--img", type=int, default=800)
    ap.add_argument("--n-dirs", type=int, default=128)
    ap.add_argument("--train-batch", type=int, default=1 << 18)
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-encode", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=3)
    ap.add_argument("--no-denoise", action="store_true")
    ap.add_argument("--no-errors", action="store_true", help="skip the per-output errors against the oracle")
    ap.add_argument("--no-mis", action="store_true")
    ap.add_argument("--no-hardvis", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the mixed N=512 frame + 2^20-query training step")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def profile_value(name, key):
    """A figure from a committed rocprofv3 summary profiles/<name>.txt (its
    `key: value` lines); None if the file is missing or the kernel sources it
    lists changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name + ".txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for f in kv["kernel_sources"].split():
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != kv["source_sha256"]:
            return None
        return float(kv[key])
    except (KeyError, OSError, ValueError):
        return None


def measured_traffic(img, n_dirs):
    """HBM-side bytes per launch of the headline kernel, from the committed
    FETCH_SIZE/WRITE_SIZE summary (copy-calibrated); None if the workload
    differs or the kernel sources changed since the counters were taken."""
    if img != 800 or n_dirs != 128:
        return None
    return profile_value("k_render_mma_f32_frame800_n128_traffic", "traffic_bytes_per_launch")


def issued_backward_atomics(precision, batch):
    """Atomic requests one backward call issues (k_backward's MLP-gradient
    flushes plus k_scatter_records' merged table-gradient adds; a request is
    the lanes of one instruction that fall in one 64-byte line), counted with
    TCP_TCC_ATOMIC_WITHOUT_RET_REQ on the benchmark's training batches (2^18
    FP32 and mixed, 2^20 mixed); None for another batch or stale counters."""
    names = ((f"k_backward_f32_train{batch}", f"k_scatter_records_f32_train{batch}") if precision == "fp32" else
             (f"k_backward_bf16_train{batch}", f"k_scatter_records_f16_train{batch}"))
    v = [profile_value(n, "issued_atomic_requests_per_launch") for n in names]
    return None if None in v else {"k_backward": v[0], "k_scatter_records": v[1]}


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    n = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / n) if n > 0 else float(np.linalg.norm(a.ravel()))


def _max_rel(a, b, floor_frac=1e-3):
    """Element-wise |a - b| / (|b| + floor_frac RMS(b))."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    rms = np.sqrt(np.mean(b * b))
    return float(np.max(np.abs(a - b) / (np.abs(b) + floor_frac * rms)))


def _psnr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    mse = np.mean((a - b) ** 2)
    return float(10 * np.log10(b.max() ** 2 / mse)) if mse > 0 else float("inf")


def _frame_errors(g, o):
    (grgb, gvis, gdep), (orgb, ovis, odep) = g, o
    return {"rgb": {"rel": _rel(grgb, orgb), "max_rel": _max_rel(grgb, orgb), "psnr_db": _psnr(grgb, orgb)},
            "vis": {"rel": _rel(gvis, ovis), "max_rel": _max_rel(gvis, ovis)},
            "depth": {"rel": _rel(gdep, odep), "max_rel": _max_rel(gdep, odep)}}


def output_errors(args, cfg, model, env, pos, nrm, wo, sub, oracle_out, O, H, hg, torch, dev):
    """Error per output against the FP64 oracle, outside every timed region:
    the benchmark frame (FP32 and mixed paths) on the oracle's pixel subset
    (rgb, and visibility and depth of every primary direction), the mixed
    N = 512 frame on a sparser subset, and the gradients of one 4096-sample
    training sub-batch (FP32 backward, and the FP16-table backward after the
    mixed forward), norm-wise per parameter array.  The renderer is rebuilt
    from the seeded model (the training leg has updated its own)."""
    print("[bench] errors against the oracle", file=sys.stderr, flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    re_ = hg.HashRenderer(model, dev)
    re_.refresh_shadows()
    env_t, pos_t, nrm_t, wo_t = t(env), t(pos), t(nrm), t(wo)
    res = {"pixels": int(len(sub)), "note": "norm-wise relative (rel), element-wise |d|/(|ref| + 1e-3 RMS(ref)) "
                                             "(max_rel), PSNR on HDR rgb; vis/depth per primary direction"}
    for prec in ("fp32", "mixed"):
        g = hg.render(re_, env_t, pos_t, nrm_t, wo_t, n_dirs=cfg.n_dirs, n_dirs2=cfg.n_dirs2, seed=H.SEED_DIRS,
                      indirect=True, want_vis=True, precision=prec)
        g = tuple(a[torch.from_numpy(sub).to(dev)].cpu().numpy() for a in g)
        res[f"frame_n{cfg.n_dirs}_{prec}"] = _frame_errors(g, oracle_out)
        del g
    if not (args.no_mixed or args.no_c5):
        sub5 = H.subset_rows_cols(cfg.img_h, cfg.img_w, 3 * args.cpu_stride)
        o5 = O.render(O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT), O.OracleEnv(env),
                      O.sampling(512, cfg.n_dirs2, H.SEED_DIRS, 0), pos[sub5], nrm[sub5], wo[sub5], indirect=True,
                      want_vis=True, pid=sub5)
        g = hg.render(re_, env_t, pos_t, nrm_t, wo_t, n_dirs=512, n_dirs2=cfg.n_dirs2, seed=H.SEED_DIRS,
                      indirect=True, want_vis=True, precision="mixed")
        g = tuple(a[torch.from_numpy(sub5).to(dev)].cpu().numpy() for a in g)
        res["frame_n512_mixed"] = dict(_frame_errors(g, o5), pixels=int(len(sub5)))
        del g
    # gradients of one training sub-batch
    nb = 4096
    bp, bd = H.make_train_batch(nb, seed=31)
    tgt = t(H.make_targets(nb))
    om = O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT)
    oe = O.OracleEnv(env)
    for fwd, bwd in (("fp32", "fp32"), ("mixed", "mixed")):
        rgb_, vis_, dep_ = hg.render(re_, env_t, t(bp), dirs=t(bd), precision=fwd)
        _, g_rgb, g_vis, g_dep = hg.l2_loss(rgb_, vis_, dep_, tgt)
        grads = hg.zero_grads(re_)
        hg.backward(re_, env_t, t(bp), t(bd), g_rgb, g_vis, g_dep, grads, precision=bwd)
        ref = O.backward(om, oe, O.sampling(1, cfg.n_dirs2, 7, 0), bp, bd, g_rgb.cpu().numpy(),
                         g_vis.cpu().numpy(), g_dep.cpu().numpy(), indirect=True)
        e = {"table": _rel(grads["table"].cpu().numpy(), ref["table"])}
        for k in ("brdf", "irt"):
            for i, nm in enumerate(("W0", "b0", "W1", "b1", "W2", "b2")):
                e[f"{k}.{nm}"] = _rel(grads[k][i].cpu().numpy(), ref[k][i])
        res[f"grad_batch{nb}_{bwd}"] = e
    return res


def time_events(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        s.record()
        fn()
        e.record()
        e.synchronize()
        per.append(s.elapsed_time(e))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return float(np.mean(per)), per, wall


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (rendering shards by pixel with "
              "no exchange between GPUs).", file=sys.stderr)
        sys.exit(2)
    import torch

    import hg_inputs as H
    import paper_2409_10327_amd as hg

    dev = "cuda:0"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    cfg = H.config("c2")
    cfg.img_h = cfg.img_w = args.img
    cfg.n_dirs = args.n_dirs
    print(f"[bench] building inputs {args.img}x{args.img} N={args.n_dirs}", file=sys.stderr, flush=True)
    model = H.make_model(cfg)
    env = H.make_env(cfg.env_h, cfg.env_w)
    pos, nrm, wo = H.make_scene(cfg.img_h, cfg.img_w)
    r = hg.HashRenderer(model, dev)
    env_t, pos_t, nrm_t, wo_t = t(env), t(pos), t(nrm), t(wo)
    P = pos.shape[0]
    S = P * cfg.n_dirs
    rgb = torch.empty((P, 3), device=dev)

    def frame_fp32():
        hg.render(r, env_t, pos_t, nrm_t, wo_t, n_dirs=cfg.n_dirs, n_dirs2=cfg.n_dirs2, seed=H.SEED_DIRS,
                  indirect=True, out=(rgb, None, None))

    print("[bench] FP32 frame", file=sys.stderr, flush=True)
    ms, per, wall = time_events(frame_fp32, args.steps, args.warmup, torch)
    out = {
        "metric": "secondary-ray queries/s (FP32 forward, 800x800 frame, 128 dirs + 1 bounce x 8)",
        "value": S / (ms * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"frame {args.img}x{args.img}, N={cfg.n_dirs}, N'={cfg.n_dirs2}, L=16, "
                               f"T=2^{cfg.log2_T}, res 16..2048, env 64x128 (FP32 path)",
                   "shaded_px_per_s": P / (ms * 1e-3), "secondary_queries": S,
                   "tertiary_irt_per_s": S * cfg.n_dirs2 / (ms * 1e-3)},
    }
    achieved = FLOP_PER_QUERY * S / (ms * 1e-3) / 1e12
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                       "traffic": measured_traffic(args.img, cfg.n_dirs),
                       "kernel": "k_render_mma<F32Path, indirect, shade>"}

    if args.copy_probe:
        src = torch.ones(1 << 28, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
        del src, dst

    if not args.no_mixed:
        try:
            rgbm = torch.empty((P, 3), device=dev)
            r.refresh_shadows()

            def frame_mixed():
                hg.render(r, env_t, pos_t, nrm_t, wo_t, n_dirs=cfg.n_dirs, n_dirs2=cfg.n_dirs2,
                          seed=H.SEED_DIRS, indirect=True, precision="mixed", out=(rgbm, None, None))
            print("[bench] mixed frame", file=sys.stderr, flush=True)
            msm, _, _ = time_events(frame_mixed, args.steps, args.warmup, torch)
            a_m = FLOP_PER_QUERY * S / (msm * 1e-3) / 1e12
            out["mixed"] = {"value": S / (msm * 1e-3), "ms_per_step": msm, "shaded_px_per_s": P / (msm * 1e-3),
                            "dtype": "bf16-mfma/f16-table/f32-acc",
                            "roofline": {"bound": "mfma", "achieved": a_m, "peak": BF16_MFMA_PEAK_TFLOPS,
                                         "unit": "TFLOP/s", "frac": a_m / BF16_MFMA_PEAK_TFLOPS,
                                         "kernel": "k_render_mma<Bf16PathT<true>, indirect, shade>"}}
        except hg.HGError as e:
            out["mixed"] = {"unavailable": str(e)}

    if not (args.no_mixed or args.no_hardvis):
        # hard visibility: the bounce runs only for shadow rays
        def frame_hard(prec):
            def f():
                hg.render(r, env_t, pos_t, nrm_t, wo_t, n_dirs=cfg.n_dirs, n_dirs2=cfg.n_dirs2, seed=H.SEED_DIRS,
                          indirect=True, flags=hg.HG_HARD_VIS, precision=prec, out=(rgb, None, None))
            return f
        print("[bench] hard-visibility frames", file=sys.stderr, flush=True)
        msh32, _, _ = time_events(frame_hard("fp32"), args.steps, args.warmup, torch)
        mshm, _, _ = time_events(frame_hard("mixed"), args.steps, args.warmup, torch)
        out["hard_visibility"] = {"fp32_ms": msh32, "mixed_ms": mshm,
                                  "fp32_queries_per_s": S / (msh32 * 1e-3), "mixed_queries_per_s": S / (mshm * 1e-3)}

    if not args.no_mis:
        # MIS primary directions (light-importance + GGX visible-normal rays):
        # the paper's one + one rays per pixel (the matrix-core kernel's
        # per-lane mode) and the 128-direction frame
        dist = hg.env_sampling(env_t)

        def frame_mis(n, prec):
            def f():
                hg.render(r, env_t, pos_t, nrm_t, wo_t, n_dirs=n, n_dirs2=cfg.n_dirs2, seed=H.SEED_DIRS,
                          indirect=True, flags=hg.HG_MIS, precision=prec, env_dist=dist, out=(rgb, None, None))
            return f
        print("[bench] MIS frames", file=sys.stderr, flush=True)
        ms2, _, _ = time_events(frame_mis(2, "fp32"), args.steps, args.warmup, torch)
        ms128, _, _ = time_events(frame_mis(cfg.n_dirs, "fp32"), args.steps, args.warmup, torch)
        out["mis"] = {"paper_1plus1_fp32_ms": ms2, "paper_1plus1_fps": 1e3 / ms2,
                      "paper_1plus1_queries_per_s": 2 * P / (ms2 * 1e-3),
                      "n128_fp32_ms": ms128, "n128_fp32_queries_per_s": S / (ms128 * 1e-3)}
        if not args.no_mixed:
            ms2m, _, _ = time_events(frame_mis(2, "mixed"), args.steps, args.warmup, torch)
            ms128m, _, _ = time_events(frame_mis(cfg.n_dirs, "mixed"), args.steps, args.warmup, torch)
            out["mis"]["paper_1plus1_mixed_ms"] = ms2m
            out["mis"]["paper_1plus1_mixed_fps"] = 1e3 / ms2m
            out["mis"]["n128_mixed_ms"] = ms128m
            out["mis"]["n128_mixed_queries_per_s"] = S / (ms128m * 1e-3)
        del dist

    if not args.no_paper:
        # the paper's model shape (14 levels, T = 2^17, res 16..131072, decoder
        # normal head) on the same 800x800 frame
        pcfg = H.config("paper")
        rp = hg.HashRenderer(H.make_model(pcfg), dev)
        rp.refresh_shadows()
        pdist = hg.env_sampling(env_t)

        def frame_paper(n, prec, flags=0):
            def f():
                hg.render(rp, env_t, pos_t, nrm_t, wo_t, n_dirs=n, n_dirs2=cfg.n_dirs2, seed=H.SEED_DIRS,
                          indirect=True, flags=flags, precision=prec, env_dist=pdist, out=(rgb, None, None))
            return f
        print("[bench] paper-shape frames", file=sys.stderr, flush=True)
        mp32, _, _ = time_events(frame_paper(cfg.n_dirs, "fp32"), args.steps, args.warmup, torch)
        mpm, _, _ = time_events(frame_paper(cfg.n_dirs, "mixed"), args.steps, args.warmup, torch)
        mpmis, _, _ = time_events(frame_paper(2, "fp32", hg.HG_MIS), args.steps, args.warmup, torch)
        mpmism, _, _ = time_events(frame_paper(2, "mixed", hg.HG_MIS), args.steps, args.warmup, torch)
        out["paper_shape"] = {"n128_fp32_ms": mp32, "n128_fp32_queries_per_s": S / (mp32 * 1e-3),
                              "n128_mixed_ms": mpm, "n128_mixed_queries_per_s": S / (mpm * 1e-3),
                              "mis_1plus1_fp32_ms": mpmis, "mis_1plus1_fps": 1e3 / mpmis,
                              "mis_1plus1_mixed_ms": mpmism, "mis_1plus1_mixed_fps": 1e3 / mpmism}
        del rp, pdist

    if not args.no_denoise:
        # spatial SVGF (5 a-trous iterations) on the FP32 frame, guided by the
        # primary depth and normals.  Algorithmic bytes per pixel: init 44
        # (rgb, depth, colour+luminance, variance, depth gradient), each
        # iteration 64 (colour+luminance, variance, gradient, depth, normal in;
        # colour+luminance, variance out), 12 for the output colour.
        frame_fp32()
        cam = torch.tensor(H.camera(), device=dev, dtype=torch.float64)
        dmap = torch.linalg.norm(pos_t.double() - cam, dim=1).float().view(cfg.img_h, cfg.img_w)
        rgb_img, nrm_img = rgb.view(cfg.img_h, cfg.img_w, 3), nrm_t.view(cfg.img_h, cfg.img_w, 3)
        work = torch.empty(hg.lib().hg_denoise_workspace_size(cfg.img_h, cfg.img_w) // 4, device=dev)
        its = 5

        def dn():
            hg.denoise(rgb_img, dmap, nrm_img, iterations=its, work=work)
        print("[bench] denoise", file=sys.stderr, flush=True)
        msd, _, _ = time_events(dn, args.steps, args.warmup, torch)
        alg_d = P * (44 + 64 * its + 12)
        out["denoise"] = {"ms": msd, "iterations": its, "px_per_s": P / (msd * 1e-3),
                          "roofline": {"bound": "hbm", "achieved": alg_d / (msd * 1e-3) / 1e9,
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": alg_d / (msd * 1e-3) / 1e9 / HBM_PEAK_GBS}}

    if not args.no_encode:
        # hg_encode gather bandwidth: 2^24 points uniform in the scene's
        # bounding region, FP32 tables (T = 2^19, 64 MiB).  Algorithmic bytes
        # per point: 16 levels x 8 corners x 8 B gathered + 12 B position +
        # 128 B features.  Ceiling: the same kernel grid gathering exactly the
        # encoder's own corner addresses (indices recorded by hg_encode_index
        # and streamed from HBM, no arithmetic) -- the achievable rate for this
        # access stream; for context, fully random 8-byte gathers over a table
        # of the same size (every load a different cache line).
        from paper_2409_10327_amd import membench as MB
        print("[bench] encode", file=sys.stderr, flush=True)
        ne = 1 << 24
        gen = torch.Generator(device=dev)
        gen.manual_seed(3)
        epos = (torch.rand((ne, 3), device=dev, generator=gen) * 8.0 - 4.0).contiguous()

        def enc():
            hg.encode(r, epos)
        mse, _, _ = time_events(enc, args.steps, 1, torch)
        alg = ne * (16 * 8 * 8 + 12 + 128)
        gbytes = ne * 16 * 8 * 8
        idx, _w = hg.encode_index(r, epos)
        del _w
        lvl_off = (torch.arange(16, device=dev, dtype=torch.int32) << cfg.log2_T).view(1, 16, 1)
        gidx = (idx + lvl_off).view(-1)
        del idx
        ms_replay = min(MB.gather_indexed_ms(r.table, 8, gidx, blocks_per_cu=b) for b in (2, 4, 8))
        # the replay's own index stream, timed with every gather an L1 hit
        ms_stream = MB.gather_indexed_ms(torch.zeros(32, device=dev, dtype=torch.int32), 8, torch.zeros_like(gidx),
                                         blocks_per_cu=2)
        del gidx
        rnd = MB.gather(64 << 20, 8)
        # the pure gather time of the stream lies in [replay - index stream, replay]
        out["encode"] = {"points": ne, "ms": mse, "gather_GBps": alg / (mse * 1e-3) / 1e9,
                         "corner_gathers_per_s": ne * 128 / (mse * 1e-3),
                         "achievable": {"kind": "replay of the encoder's own corner addresses in its order (persistent "
                                                "grid, indices streamed non-temporally and prefetched, no arithmetic; "
                                                "fastest of 2, 4, 8 blocks per CU)",
                                        "replay_ms": ms_replay, "index_stream_ms": ms_stream,
                                        "gather_ms_bounds": [ms_replay - ms_stream, ms_replay]},
                         "frac_of_achievable": (ms_replay - ms_stream) / mse,
                         "frac_of_achievable_bounds": [(ms_replay - ms_stream) / mse, ms_replay / mse],
                         "random_8B_gather_64MiB": {"items_per_s": rnd["items_per_s"],
                                                    "useful_GBps": rnd["useful_GBps"]},
                         "hbm_peak_GBps": HBM_PEAK_GBS, "frac_of_hbm_peak": alg / (mse * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del epos

    if not args.no_train:
        B = args.train_batch
        print(f"[bench] training step B={B}", file=sys.stderr, flush=True)
        teacher = hg.HashRenderer(H.make_teacher(cfg), dev)
        bp, bd = H.make_train_batch(B)
        bp_t, bd_t = t(bp), t(bd)
        trgb, tvis, tdep = hg.render(teacher, env_t, bp_t, dirs=bd_t)
        tgt = torch.cat([trgb, tvis[:, None], tdep[:, None]], 1).contiguous()
        del teacher
        grads = hg.zero_grads(r)
        params = [r.table] + r.brdf + r.irt
        gl = [grads["table"]] + grads["brdf"] + grads["irt"]
        ms_ = [torch.zeros_like(p) for p in params]
        vs_ = [torch.zeros_like(p) for p in params]
        step = [0]

        # batch order along a Morton curve (hg_morton_order: 21 bits per axis over
        # the hash grid's domain box, no reduction over the batch): queries of a
        # wave then share cells down to finer levels
        morton_ws = torch.empty(hg.lib().hg_morton_order_workspace_size(1 << 20), device=dev, dtype=torch.uint8)

        def morton_order(p):
            return hg.morton_order(r, p, ws=morton_ws)

        def train_step():
            # a training loop draws a new batch each step: its ordering is part of the step
            step[0] += 1
            order = morton_order(bp_t)
            sp, sd, st = bp_t[order], bd_t[order], tgt[order]
            rgb_, vis_, dep_ = hg.render(r, env_t, sp, dirs=sd)
            loss, g_rgb, g_vis, g_dep = hg.l2_loss(rgb_, vis_, dep_, st)
            hg.backward(r, env_t, sp, sd, g_rgb, g_vis, g_dep, grads)
            # Adam over the 13 arrays in one launch, clearing each gradient
            # after use for the next step's backward
            hg.adam_step_multi(adam_fp32, step[0], lr=2e-3, zero_grad=True)
            return loss

        adam_fp32 = hg.AdamGroup([(p_, g_, ms_[i], vs_[i], 0.0 if i == 0 else 1e-6, None)
                                  for i, (p_, g_) in enumerate(zip(params, gl))])
        for g in gl:  # cleared once; every step leaves them cleared
            g.zero_()
        mst, _, _ = time_events(train_step, max(5, args.steps), 2, torch)
        out["train"] = {"samples_per_s": B / (mst * 1e-3), "ms_per_step": mst, "batch": B,
                        "secondary_queries_per_s_fwd_bwd": B / (mst * 1e-3), "dtype": "f32"}

        def backward_roofline(precision, B=B):
            """Time the backward call alone (k_backward, the record sort and
            k_scatter_records) on one Morton-ordered batch.  Its binding
            resource is the FP32 atomic adds, which the hardware executes past
            the L2 at a rate of requests (the lanes of one instruction in one
            64-byte line) that does not depend on addresses: the roofline is
            the requests it issues (counted by rocprofv3) over the measured
            random-atomic request rate.  The 512 table-gradient adds per sample
            of the definition are merged in LDS before they are issued, so
            they are reported beside it, not as the achieved rate."""
            order = morton_order(bp_t)
            sp, sd, st = bp_t[order], bd_t[order], tgt[order]
            fwd_prec = "fp32" if precision == "fp32" else "mixed"
            rgb_, vis_, dep_ = hg.render(r, env_t, sp, dirs=sd, precision=fwd_prec)
            _, g_rgb, g_vis, g_dep = hg.l2_loss(rgb_, vis_, dep_, st)

            def bwd():
                hg.backward(r, env_t, sp, sd, g_rgb, g_vis, g_dep, grads, precision=precision)
            msb, _, _ = time_events(bwd, max(5, args.steps), 1, torch)
            issued = issued_backward_atomics(precision, B)
            ceil = atomic_ceiling["lane_atomics_per_s"]
            rate = None if issued is None else sum(issued.values()) / (msb * 1e-3)
            mfma_peak = FP32_MFMA_PEAK_TFLOPS if precision == "fp32" else BF16_MFMA_PEAK_TFLOPS
            fl = BWD_FLOP_PER_SAMPLE * B / (msb * 1e-3) / 1e12
            return msb, {"bound": "atomics", "kernel": "backward call: k_backward + record sort + k_scatter_records",
                         "ms": msb, "achieved": rate, "peak": ceil, "unit": "FP32 atomic requests/s",
                         "frac": None if rate is None else rate / ceil,
                         "peak_kind": "measured random FP32 atomic adds over 64 MiB (hgmb_atomic), one lane "
                                      "per request",
                         "issued_atomic_requests_per_launch": issued,
                         "table_adds_before_merging_per_launch": ATOMICS_PER_SAMPLE * B,
                         "mfma": {"achieved": fl, "peak": mfma_peak, "unit": "TFLOP/s", "frac": fl / mfma_peak}}

        def step_mfma(ms_step, precision, B=B):
            # the whole training step's matrix work (forward + backward per
            # sample) against the matrix-core peak of the MLP precision
            peak = FP32_MFMA_PEAK_TFLOPS if precision == "fp32" else BF16_MFMA_PEAK_TFLOPS
            fl = (FLOP_PER_QUERY + BWD_FLOP_PER_SAMPLE) * B / (ms_step * 1e-3) / 1e12
            return {"bound": "mfma", "flop_per_sample": FLOP_PER_QUERY + BWD_FLOP_PER_SAMPLE, "achieved": fl,
                    "peak": peak, "unit": "TFLOP/s", "frac": fl / peak}

        from paper_2409_10327_amd import membench as MB
        atomic_ceiling = MB.atomic(64 << 20, 1)
        _, out["train"]["roofline"] = backward_roofline("fp32")
        out["train"]["step_roofline"] = step_mfma(mst, "fp32")

        # mixed-precision step: forward and backward with FP16 tables and BF16
        # MLPs on the matrix cores (FP32 accumulation, FP32 master gradients),
        # Adam on the FP32 masters refreshing the FP16/BF16 shadows
        r.refresh_shadows()
        shadows = [r.table16] + [r.brdf16[i] if i % 2 == 0 else None for i in range(6)] + \
                  [r.irt16[i] if i % 2 == 0 else None for i in range(6)]

        def train_step_mixed():
            step[0] += 1
            order = morton_order(bp_t)
            sp, sd, st = bp_t[order], bd_t[order], tgt[order]
            rgb_, vis_, dep_ = hg.render(r, env_t, sp, dirs=sd, precision="mixed")
            loss, g_rgb, g_vis, g_dep = hg.l2_loss(rgb_, vis_, dep_, st)
            hg.backward(r, env_t, sp, sd, g_rgb, g_vis, g_dep, grads, precision="mixed")
            hg.adam_step_multi(adam_mixed, step[0], lr=2e-3, zero_grad=True)
            return loss

        adam_mixed = hg.AdamGroup([(p_, g_, ms_[i], vs_[i], 0.0 if i == 0 else 1e-6, shadows[i])
                                   for i, (p_, g_) in enumerate(zip(params, gl))])
        for g in gl:  # the backward roofline above added into them
            g.zero_()
        mstm, _, _ = time_events(train_step_mixed, max(5, args.steps), 2, torch)
        out["train"]["mixed"] = {"samples_per_s": B / (mstm * 1e-3), "ms_per_step": mstm,
                                 "dtype": "bf16-mfma fwd+bwd / f16 tables / f32 masters and gradients"}
        _, out["train"]["mixed"]["roofline"] = backward_roofline("mixed")
        out["train"]["mixed"]["step_roofline"] = step_mfma(mstm, "mixed")
        out["train"]["random_atomic_ceiling"] = atomic_ceiling
        # the same rate per request when two or sixteen lanes share a line
        out["train"]["atomic_lines"] = [MB.atomic_lines(64 << 20, g) for g in (2, 16)]
        del bp_t, bd_t, tgt

        if not (args.no_mixed or args.no_c5):
            # the combined mixed workload: the 800x800 frame at N = 512 (327.68M
            # secondary queries) and a mixed training step over 2^20 queries
            # (teacher targets, Morton order, recomputed bounce)
            print("[bench] mixed frame N=512 and mixed step B=2^20", file=sys.stderr, flush=True)
            N5 = 512
            rgb5 = torch.empty((P, 3), device=dev)
            r.refresh_shadows()

            def frame5():
                hg.render(r, env_t, pos_t, nrm_t, wo_t, n_dirs=N5, n_dirs2=cfg.n_dirs2, seed=H.SEED_DIRS,
                          indirect=True, precision="mixed", out=(rgb5, None, None))
            ms5, _, _ = time_events(frame5, max(2, args.steps // 2), 1, torch)
            B5 = 1 << 20
            teacher = hg.HashRenderer(H.make_teacher(cfg), dev)
            bp5, bd5 = H.make_train_batch(B5)
            bp_t, bd_t = t(bp5), t(bd5)
            trgb, tvis, tdep = hg.render(teacher, env_t, bp_t, dirs=bd_t)
            tgt = torch.cat([trgb, tvis[:, None], tdep[:, None]], 1).contiguous()
            del teacher, trgb, tvis, tdep
            for g in gl:  # the backward roofline above added into them
                g.zero_()
            ms5t, _, _ = time_events(train_step_mixed, max(2, args.steps // 2), 1, torch)
            a5 = FLOP_PER_QUERY * P * N5 / (ms5 * 1e-3) / 1e12
            out["mixed_n512_train_2e20"] = {
                "frame_ms": ms5, "frame_queries_per_s": P * N5 / (ms5 * 1e-3), "frame_px_per_s": P / (ms5 * 1e-3),
                "frame_roofline": {"bound": "mfma", "kernel": "k_render_mma<Bf16PathT<false>, indirect, shade>",
                                   "achieved": a5, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": a5 / BF16_MFMA_PEAK_TFLOPS},
                "train_ms": ms5t, "train_samples_per_s": B5 / (ms5t * 1e-3),
                "train_step_roofline": step_mfma(ms5t, "mixed", B5),
                "dtype": "bf16-mfma/f16-table/f32-acc; f32 masters"}
            _, out["mixed_n512_train_2e20"]["train_roofline"] = backward_roofline("mixed", B5)
            del bp_t, bd_t, tgt

    if not args.no_cpu:
        from oracle import oracle as O
        sub = H.subset_rows_cols(cfg.img_h, cfg.img_w, args.cpu_stride)
        om, oe = O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT), O.OracleEnv(env)
        samp = O.sampling(cfg.n_dirs, cfg.n_dirs2, H.SEED_DIRS, 0)
        print(f"[bench] oracle on {len(sub)} px", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        orgb, ovis, odep = O.render(om, oe, samp, pos[sub], nrm[sub], wo[sub], indirect=True, want_vis=True, pid=sub)
        dt = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": len(sub) * cfg.n_dirs / dt, "unit": "queries/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"every {args.cpu_stride}th row and column ({len(sub)} px x "
                                         f"{cfg.n_dirs} dirs), FP64, {dt:.1f} s"}
        if not args.no_errors:
            out["errors"] = output_errors(args, cfg, model, env, pos, nrm, wo, sub, (orgb, ovis, odep), O, H, hg,
                                          torch, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

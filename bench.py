"""Benchmark of the semantic Gaussian rasterizer on one MI355X.

Step = one mapping iteration on 1M Gaussians in a 10x8x3 m room seen by one
1200x680 keyframe (fx=fy=600): project -> bin -> render_forward with the
fused loss gradient -> render_backward, whose gather applies the Adam step
where each Gaussian's gradient is formed.  The loss is the mapping loss with the
silhouette mask (S > 0.99: L1 depth + 0.5 L1 colour), plus L1(S, 1) and a
cross-entropy on the semantic map.  Throughput is Gaussian-pixel blends per
second (blends = sum of n_contrib, exact).  Candidate-view scoring (500k
Gaussians, 64 views of mixed resolution) is timed batched and one view per
launch.  Synthetic, seeded inputs; everything is resident in HBM before the
timed region starts.

    python bench.py [--gpus 1] [--steps 40] [--warmup 5]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/iter & Gaussian-pixel blends/s @1M G 1200x680; views/s"
HBM_PEAK_GBS = 8000.0
# fp32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (packed pair) x 2 flops (FMA) x 2.4 GHz; the HIP
# code here is built without packed fp32, which halves what it can reach
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_TFLOPS = 78.6
# Algorithmic fp32 flops per blend (an FMA counts as 2, exp2 and rcp as 1):
#   evaluation of a blended pair: offset 2, u = dx + cb dy 2, exponent ca u^2 + cc dy^2 5, exp2 1,
#     alpha = min(alpha_max, o G) 2                                                          = 12
#   forward blend: w = alpha T 1, T (1 - alpha) 2, colour 6, depth 2, silhouette 1, the label's
#     class sum 2                                                                             = 14
#   backward blend (one-class semantic gradient): T in front 3, w 1, e over the channels 8,
#     dL/dalpha 3, suffix sum 2, dL/dQ and dL/do 3, whitened offset 4, its products 5, colour
#     and depth terms 4, semantic term 1, the per-key sums of the 11 values 11              = 45
FLOPS_PER_BLEND = {"fwd": 12 + 14, "bwd_tiles": 12 + 45}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--score-views", type=int, default=64)
    ap.add_argument("--score-n", type=int, default=500_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-score", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library defaults)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run a plain streaming kernel over this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--no-mapping", action="store_true",
                    help="skip the mapping leg (then only the other legs' results are printed; for profiling them)")
    ap.add_argument("--no-plan", action="store_true", help="skip the planning leg")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-vs-sparse leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the legs of the other workloads (64x64 forward, 200k fwd+bwd, 3M large scene)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


class Timer:
    """HIP events on torch's current stream (the stream every library call
    is enqueued on)."""

    def __init__(self, torch, names):
        self.torch = torch
        self.names = names
        self.ev = {nm: [] for nm in names}

    def mark(self, name):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.ev[name].append(e)
        return e

    def pairs_ms(self, a, b):
        return [x.elapsed_time(y) for x, y in zip(self.ev[a], self.ev[b])]


def mapping_bench(args, torch, out):
    from paper_2506_00225_amd import Frame, FusedAdam, Gaussians, autotune, loss_config, make_config, scenes

    log("generating room scene", args.n)
    sc = scenes.room_scene(n=args.n)
    cam = sc.cameras[0]
    H, W, C, k = cam.height, cam.width, sc.num_classes, sc.k
    P = H * W
    g = Gaussians.from_scene(sc)
    params = [g.means, g.scales, g.quats, g.opacity, g.rgb, g.sem_val]
    cfg = make_config(C, k)
    fr = Frame(sc.n, [cam], cfg)
    fr.prepare(g, check=True)
    st, nvis, nkeys = fr.status()
    fr.key_capacity = int(nkeys * 1.5) + 4096
    fr._alloc()
    fr.prepare(g, check=True)
    dev = g.means.device
    t_rgb = torch.from_numpy(sc.targets["rgb"]).to(dev).reshape(P, 3)
    t_depth = torch.from_numpy(sc.targets["depth"]).to(dev).reshape(P)
    label = torch.from_numpy(sc.targets["label"]).to(dev).reshape(P).int().contiguous()
    # cross-entropy's semantic gradient is one class per pixel: kept in that sparse form
    grads_in = {"rgb": torch.empty(P, 3, device=dev), "depth": torch.empty(P, device=dev),
                "sil": torch.empty(P, device=dev), "sem_at_label": torch.empty(P, device=dev), "sem_label": label}
    gout = {nm: torch.empty_like(getattr(g, nm)) for nm in ("means", "scales", "quats", "opacity", "rgb", "sem_val")}
    inf = float("inf")
    opt = FusedAdam([(g.means, gout["means"], -inf, inf), (g.scales, gout["scales"], -inf, inf),
                     (g.quats, gout["quats"], -inf, inf), (g.opacity, gout["opacity"], 1e-4, 0.9999),
                     (g.rgb, gout["rgb"], -inf, inf), (g.sem_val, gout["sem_val"], 0.0, inf)],
                    lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    blends = torch.zeros(2 * args.steps + args.warmup, dtype=torch.int64, device=dev)

    targets = {"rgb": t_rgb, "depth": t_depth, "label": label}
    lcfg = loss_config()  # Sec. 3.1 masked depth + 0.5 colour L1, |S - 1|, cross-entropy
    ncon = {"n_contrib": torch.empty(P, dtype=torch.int32, device=dev)}
    losses = torch.zeros(2 * args.steps + args.warmup, dtype=torch.float64, device=dev)

    if not args.no_tune:  # times the fused forward + loss and the backward, as the step runs them
        rep = autotune.tune_mapping(fr, g, reps=3, targets=targets, loss_cfg=lcfg)
        out["autotune_mapping"] = rep
        log("autotune mapping", json.dumps(rep["candidates"]))

    names = ["s0", "proj", "bin", "fwd", "bwd_tiles", "bwd_gather", "adam"]
    tm = Timer(torch, names)

    def step(i, marked, fused=True):
        """One mapping iteration.  fused: the gather and the Adam step in one
        pass (sgr_render_backward_gather_adam), as the timed steps run it;
        the steps with stage events run them apart, so the breakdown shows
        each."""
        mk = tm.mark if marked else (lambda _n: None)
        mk("s0")
        fr.project(g)
        mk("proj")
        fr.bin(g)
        mk("bin")
        _, loss = fr.forward_loss(g, targets, lcfg, maps=ncon, grads=grads_in)  # forward + fused loss gradient
        mk("fwd")
        fr.backward_tiles(g, grads_in)
        mk("bwd_tiles")
        if fused and not marked:
            fr.backward_gather_adam(g, opt)
        else:
            fr.backward_gather(g, gout)
            mk("bwd_gather")
            opt.step()
        mk("adam")
        if marked:  # bookkeeping, after the step's last event
            blends[i].copy_(ncon["n_contrib"].sum(dtype=torch.int64))
            losses[i].copy_(loss[0])

    log("warmup", args.warmup)
    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    # The timed steps carry no events between stages (each event costs a few
    # microseconds of idle GPU); the per-stage breakdown, the blend count B
    # and the losses come from the same steps run again with an event at
    # every stage boundary.  Each run starts from the parameters and moments
    # left by the warmup, and the gather with Adam gives the bits of the
    # gather followed by Adam, so all three runs take the same trajectory and
    # B is the timed steps' own blend count.
    snap = [x.clone() for x in params + opt.m + opt.v]
    t_snap = opt.t

    def restore():
        for x, y in zip(params + opt.m + opt.v, snap):
            x.copy_(y)
        opt.t = t_snap

    log("timed", args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        step(args.warmup + i, False)
    e1.record()
    enqueue = time.perf_counter() - t0  # host time to issue the steps (well below the GPU time: GPU-bound)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / args.steps
    # the same steps with the gather and Adam as two launches
    restore()
    e0.record()
    for i in range(args.steps):
        step(args.warmup + i, False, fused=False)
    e1.record()
    torch.cuda.synchronize()
    step_unfused_ms = e0.elapsed_time(e1) / args.steps
    log("breakdown", args.steps)
    restore()
    for i in range(args.steps):
        step(args.warmup + args.steps + i, True)
    torch.cuda.synchronize()
    st, nvis, nkeys = fr.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after the timed steps (key capacity {fr.key_capacity}, K {nkeys})")
    stage = {}
    for a, b in zip(names[:-1], names[1:]):
        stage[b] = float(np.mean(tm.pairs_ms(a, b)))
    stage["bwd"] = stage["bwd_tiles"] + stage["bwd_gather"]
    marked_ms = float(np.mean(tm.pairs_ms("s0", "adam")))
    B = blends[args.warmup + args.steps:].double().mean().item()
    fwd_bwd_ms = stage["proj"] + stage["bin"] + stage["fwd"] + stage["bwd"]
    out.update(dict(step_ms=step_ms, step_unfused_ms=step_unfused_ms, step_ms_with_stage_events=marked_ms,
                    wall_ms=wall * 1e3 / args.steps,
                    enqueue_ms=enqueue * 1e3 / args.steps,
                    stage_ms=stage, blends=B, nvis=nvis, keys=nkeys, fwd_bwd_ms=fwd_bwd_ms, pixels=P, C=C, k=k,
                    n=sc.n, loss_first_last=[float(losses[args.warmup + args.steps]), float(losses[-1])]))
    log("stages ms", json.dumps({k_: round(v, 4) for k_, v in stage.items()}), "K", nkeys, "Nv", nvis, "B", B)
    return sc


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_kernels_1M_traffic.json")
KERNEL_SOURCES = {"bwd_tiles": ("render_bwd.hip", "render_common.h", "pipeline.h", "sgr_internal.h"),
                  "fwd": ("render_fwd.hip", "render_common.h", "pipeline.h", "sgr_internal.h")}


def source_sha(stage):
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[stage]:
        with open(os.path.join(ROOT, "paper_2506_00225_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(stage):
    """HBM bytes per launch of the stage's kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a plain
    streaming kernel of known size), if the summary was taken on the current
    kernel sources; else None."""
    if stage not in KERNEL_SOURCES or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f).get(stage)
    if not rec or rec.get("source_sha256") != source_sha(stage):
        return None
    return rec.get("bytes_per_launch")


def roofline(out):
    """Roofline of the stage with the longest HIP-event time.

    The compositing stages are bound by vector ALU issue, not HBM, so they
    are reported against the fp32 vector peak with the algorithmic flops
    per blend of FLOPS_PER_BLEND (an FMA counts as 2; B blends per launch,
    the same B as the oracle's), and beside it against the unpacked fp32
    ceiling the code is built for.  Their algorithmic bytes (every input
    read once, every output and compulsory intermediate written once) are
    reported beside it.  Other stages are HBM-bound and reported against
    the HBM peak."""
    P, C, k, K, Nv, n = out["pixels"], out["C"], out["k"], out["keys"], out["nvis"], out["n"]
    B = out["blends"]
    rec = 48 + 16 + 4 * k + ((k + 3) // 4) * 4  # projected record + rgb/z + top-k values + indices
    g2d = (10 + k) * 4  # per visible Gaussian: 2D mean, conic, opacity, rgb, depth, top-k values
    alg = {
        "proj": 44 * n + 8 * n + 12 * Nv,
        "bin": 12 * K * 3 + 8 * Nv,
        # forward with the fused loss: read records and sorted ids once and the targets (rgb, depth,
        # label); write dL/d(rgb, depth, sil), the label-class semantic gradient, n_contrib and the
        # two per-pixel words
        "fwd": rec * Nv + 4 * K + 20 * P + 6 * 4 * P + 12 * P,
        # read dL/dmaps (label-class form), the per-pixel words, sorted ids and records once;
        # write 2D gradients once
        "bwd_tiles": 7 * 4 * P + 8 * P + 4 * K + rec * Nv + g2d * Nv,
        # read 2D gradients and parameters once; write per-Gaussian gradients once
        "bwd_gather": g2d * Nv + 44 * n + (14 + k) * 4 * n,
    }
    ops_per_blend = FLOPS_PER_BLEND
    stage = out["stage_ms"]
    dom = max(alg, key=lambda s: stage[s])
    sec = stage[dom] * 1e-3
    gbs = alg[dom] / sec / 1e9
    kern = {"fwd": "render_fwd_label_kernel", "bwd_tiles": "render_bwd_kernel"}.get(dom, dom)
    common = {"traffic": counted_traffic(dom), "kernel": kern, "alg_bytes": int(alg[dom]), "ms": round(stage[dom], 4)}
    if dom in ops_per_blend:
        flops = B * ops_per_blend[dom]
        tf = flops / sec / 1e12
        return dom, {"bound": "alu", "achieved": round(tf, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / FP32_PEAK_TFLOPS, 4), **common, "alg_flops": int(flops),
                     "flops_per_blend": ops_per_blend[dom], "peak_unpacked": FP32_UNPACKED_TFLOPS,
                     "frac_unpacked": round(tf / FP32_UNPACKED_TFLOPS, 4), "hbm_gbs": round(gbs, 2),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return dom, {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(gbs / HBM_PEAK_GBS, 4), **common}


def hbm_path(out):
    """Forward + backward of the mapping iteration (proj, bin, fwd, bwd_tiles,
    bwd_gather) against the HBM roofline, with two byte counts:
    * the compulsory-byte formula of the hot-path scope (every input read
      once, every output and intermediate written once and read once, the
      dense C-class maps and their gradients included), with the measured
      key count K and visible pairs N_v;
    * this path's own algorithmic bytes (the fused loss keeps the class maps
      and their gradients on chip), the sum of the per-stage figures."""
    P, C, k, K, Nv, n = out["pixels"], out["C"], out["k"], out["keys"], out["nvis"], out["n"]
    b_fwd = 44 * n + 36 * n + 8 * n + 36 * K + 4 * K + (36 + 12 + 5 * k) * Nv + P * (5 + C) * 4 + 8 * P
    b_bwd = P * (5 + C) * 4 + 8 * P + 4 * K + (48 + 5 * k) * Nv + (40 + 4 * k) * n + 72 * n + 44 * n
    rec = 48 + 16 + 4 * k + ((k + 3) // 4) * 4
    g2d = (10 + k) * 4
    fused = (44 * n + 8 * n + 12 * Nv) + (12 * K * 3 + 8 * Nv) + (rec * Nv + 4 * K + 20 * P + 6 * 4 * P + 12 * P) + \
            (7 * 4 * P + 8 * P + 4 * K + rec * Nv + g2d * Nv) + (g2d * Nv + 44 * n + (14 + k) * 4 * n)
    sec = out["fwd_bwd_ms"] * 1e-3
    return {"fwd_bwd_ms": round(out["fwd_bwd_ms"], 4),
            "scope_formula_bytes": int(b_fwd + b_bwd), "scope_formula_gbs": round((b_fwd + b_bwd) / sec / 1e9, 1),
            "scope_formula_frac": round((b_fwd + b_bwd) / sec / 1e9 / HBM_PEAK_GBS, 4),
            "fused_path_bytes": int(fused), "fused_path_gbs": round(fused / sec / 1e9, 1),
            "fused_path_frac": round(fused / sec / 1e9 / HBM_PEAK_GBS, 4),
            "target_ms_at_half_peak": round((b_fwd + b_bwd) / (0.5 * HBM_PEAK_GBS * 1e9) * 1e3, 4)}


def score_bench(args, torch, out):
    from paper_2506_00225_amd import Frame, Gaussians, autotune, make_config, scenes, score_maps

    log("generating candidate scene", args.score_n, args.score_views)
    sc = scenes.candidate_scene(n=args.score_n, nviews=args.score_views)
    g = Gaussians.from_scene(sc)
    cfg = make_config(sc.num_classes, sc.k)
    fr = Frame(sc.n, sc.cameras, cfg)
    fr.prepare(g, check=True)
    _, _, nk = fr.status()
    fr.key_capacity = int(nk * 1.3) + 4096
    fr._alloc()
    if not args.no_tune:
        rep = autotune.tune_score(fr, g, reps=2)
        out["autotune_score"] = rep
        log("autotune score", json.dumps(rep["candidates"]))
    ne = torch.empty(fr.V, dtype=torch.int32, device="cuda")
    hs = torch.empty(fr.V, dtype=torch.float64, device="cuda")
    reps = 10
    for _ in range(2):
        fr.score(g, ne, hs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fr.score(g, ne, hs)
    e1.record()
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / reps
    st, _, _ = fr.status()
    assert st == 0
    graph, gne, ghs = fr.capture_score(g)
    graph.replay()
    torch.cuda.synchronize()
    graph_same = bool(torch.equal(gne, ne) and torch.equal(ghs, hs))
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / reps
    # plain: one frame per view, project/bin/render dense maps/score each
    frames = []
    for cam in sc.cameras:
        f1 = Frame(sc.n, [cam], cfg)
        f1.prepare(g, check=True)
        frames.append((f1, f1.alloc_maps(want=("sem",)), cam))
    pe = torch.empty(fr.V, dtype=torch.int32, device="cuda")
    ph = torch.empty(fr.V, dtype=torch.float64, device="cuda")
    scratch = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")

    def plain():
        for v, (f1, mp, cam) in enumerate(frames):
            f1.project(g)
            f1.bin(g)
            f1.forward(g, mp)
            score_maps(mp["sem"].view(cam.height, cam.width, -1), mp["n_contrib"].view(cam.height, cam.width),
                       sc.num_classes, scratch, pe[v:v + 1], ph[v:v + 1])

    plain()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        plain()
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / reps
    P = np.array([c.width * c.height for c in sc.cameras], dtype=np.float64)
    dmean = np.abs(ph.cpu().numpy() - hs.cpu().numpy()) / P
    same_empty = bool(torch.equal(pe, ne))
    out.update(dict(views_per_s_batched=fr.V / (batched_ms * 1e-3), views_per_s_plain=fr.V / (plain_ms * 1e-3),
                    views_per_s_graph=fr.V / (graph_ms * 1e-3), score_graph_ms=graph_ms, score_graph_equal=graph_same,
                    score_batched_ms=batched_ms, score_plain_ms=plain_ms, score_max_mean_entropy_diff=float(dmean.max()),
                    score_n_empty_equal=same_empty, score_views=fr.V))
    log("scoring batched", batched_ms, "ms plain", plain_ms, "ms")


def plan_bench(args, torch, out):
    """Next-best-view planning steps (Sec. 3.2) on the candidate-scene
    Gaussians: candidates from the newly observed voxels of a synthetic
    exploration map (10 x 8 x 3 m at 0.25 m; free within 2 m of (5, 4, 1.5)
    before, within 4 m now for the coarse stage, 2.5 -> 3 m for the fine
    stage), scored at 320 x 240 (fx = 160) and combined (Eq. 7)."""
    import numpy as np_
    from paper_2506_00225_amd import Gaussians, make_config, scenes
    from paper_2506_00225_amd.planner import COARSE, FINE, Grid, Planner, sampling

    sc = scenes.candidate_scene(n=args.score_n, nviews=1)
    g = Gaussians.from_scene(sc)
    vox, dims = 0.25, (40, 32, 12)
    z, y, x = np_.meshgrid(np_.arange(dims[2]), np_.arange(dims[1]), np_.arange(dims[0]), indexing="ij")
    centre = (np_.stack([x, y, z], -1) + 0.5) * vox
    dist = np_.linalg.norm(centre - np_.array([5.0, 4.0, 1.5]), axis=-1).reshape(-1)
    ball = lambda r: torch.from_numpy((dist <= r).astype(np_.uint8)).cuda()
    intr = scenes.Camera(np_.eye(3, dtype=np_.float32), np_.zeros(3, np_.float32), 160.0, 160.0, 160.0, 120.0,
                         320, 240)
    pl = Planner(Grid(dims, vox, (0.0, 0.0, 0.0)), intr, make_config(sc.num_classes, sc.k), capacity=4096)
    res = {}
    for name, st, (r0, r1), zr in (("coarse", COARSE, (2.0, 4.0), (1.5, 1.5)),
                                   ("fine", FINE, (2.5, 3.0), (0.5, 2.5))):
        now, before = ball(r1), ball(r0)
        samp = sampling(st["step"], st["directions"], *zr)
        o = pl.step(g, now, before, samp, (5.0, 4.0, 1.5))  # warm-up, sizes the buffers
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            o = pl.step(g, now, before, samp, (5.0, 4.0, 1.5))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[name] = {"candidates": o["V"], "ms": round(ms, 3), "candidates_per_s": round(o["V"] / (ms * 1e-3), 1),
                     "pruned": int(o["pruned"].sum()), "best": int(o["best"][0])}
        log("plan", name, json.dumps(res[name]))
    out["plan"] = res


def dense_bench(args, torch, out):
    """Dense vs top-k semantic rendering (supplement S.2.2's comparison): one
    forward at 600 x 340 of a room with about 204k Gaussians in view, C = 102,
    with the top-k lists (k = 16) and with a dense 102-class row per Gaussian."""
    from paper_2506_00225_amd import Frame, Gaussians, make_config, scenes

    sc = scenes.room_scene(seed=5, n=730_000, targets=False)
    cam = sc.cameras[0]
    half = scenes.Camera(cam.R, cam.t, cam.fx / 2, cam.fy / 2, cam.cx / 2, cam.cy / 2, cam.width // 2,
                         cam.height // 2)
    g = Gaussians.from_scene(sc)
    gen = torch.Generator(device="cuda").manual_seed(0)
    dense = torch.rand((sc.n, sc.num_classes), generator=gen, device="cuda")
    dense /= dense.sum(1, keepdim=True)
    fr = Frame(sc.n, [half], make_config(sc.num_classes, sc.k))
    fr.prepare(g, check=True)
    _, nvis, _ = fr.status()
    maps = fr.alloc_maps()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"width": half.width, "height": half.height, "gaussians": sc.n, "visible": nvis, "classes": sc.num_classes}
    for name, fn in (("sparse_top16_ms", lambda: fr.forward(g, maps)),
                     ("dense_ms", lambda: fr.forward_dense(g, dense, maps))):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = round(e0.elapsed_time(e1) / 10, 4)
    res["dense_over_sparse"] = round(res["dense_ms"] / res["sparse_top16_ms"], 2)
    log("dense vs sparse", json.dumps(res))
    out["dense_vs_sparse"] = res


def _sized_frame(torch, sc, cams, slack=1.3):
    """A frame whose key capacity is the measured key count times slack."""
    from paper_2506_00225_amd import Frame, Gaussians, make_config
    g = Gaussians.from_scene(sc)
    fr = Frame(sc.n, cams, make_config(sc.num_classes, sc.k))
    fr.prepare(g, check=True)
    _, _, nk = fr.status()
    fr.key_capacity = int(nk * slack) + 4096
    fr._alloc()
    fr.prepare(g, check=True)
    return g, fr


def _l1_step(torch, fr, g, maps, t_rgb, t_depth, onehot):
    """project, bin, forward (every map), the gradient of the mean L1 loss
    of each map (rgb, depth, silhouette against 1, semantics against the
    one-hot label), backward; returns the per-Gaussian gradients."""
    fr.project(g)
    fr.bin(g)
    fr.forward(g, maps)
    P = maps["depth"].numel()
    grads = {"rgb": torch.sign(maps["rgb"] - t_rgb) / (3 * P), "depth": torch.sign(maps["depth"] - t_depth) / P,
             "sil": torch.sign(maps["sil"] - 1.0) / P, "sem": torch.sign(maps["sem"] - onehot) / onehot.numel()}
    return fr.backward(g, grads)


def _time(torch, fn, reps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def config_legs(args, torch, out):
    """The other workloads, one line each:
    * 64x64 forward: 2,000 Gaussians, C = 16, k = 3 (project, bin, forward
      with every map);
    * 200k fwd+bwd: 200k room Gaussians at 1200x680, C = 102, k = 16, the
      mean L1 loss of each map (its gradient computed by torch between the
      two library calls, inside the timed step);
    * large scene: 3M Gaussians, C = 40, 8 keyframes at 1024x1280 rendered
      forward and backward in one batch (gradients summed per Gaussian, L1
      loss as above), then 128 candidate views at 320x240 scored in batches
      of 16 views."""
    from paper_2506_00225_amd import scenes
    res = {}
    # 64x64 forward
    sc = scenes.tiny_scene()
    g, fr = _sized_frame(torch, sc, sc.cameras)
    maps = fr.alloc_maps()

    def fwd0():
        fr.project(g)
        fr.bin(g)
        fr.forward(g, maps)
    ms = _time(torch, fwd0, 200)
    B = int(maps["n_contrib"].sum())
    res["forward_64x64_2k"] = {"ms": round(ms, 4), "blends": B, "blends_per_s": round(B / (ms * 1e-3), 1)}
    log("config 64x64", json.dumps(res["forward_64x64_2k"]))
    # 200k fwd+bwd with the L1 loss
    for name, sc, ncams in (("fwd_bwd_200k_1200x680", scenes.room_scene(n=200_000), 1),
                            ("large_3m_8x1024x1280", scenes.large_scene(), 8)):
        cams = sc.cameras[:ncams]
        g, fr = _sized_frame(torch, sc, cams)
        maps = fr.alloc_maps()
        dev = g.means.device
        if ncams == 1:
            tr = {k_: torch.from_numpy(v).to(dev) for k_, v in sc.targets.items()}
        else:
            rng = np.random.default_rng(1)
            tl = [scenes.l1_targets(rng, c, sc.num_classes) for c in cams]
            tr = {k_: torch.from_numpy(np.concatenate([t[k_].reshape(c.width * c.height, -1) for t, c in zip(tl, cams)])
                                       ).to(dev).squeeze(-1) for k_ in ("rgb", "depth", "label")}
        P = fr.pix_off[-1]
        t_rgb, t_depth = tr["rgb"].reshape(P, 3), tr["depth"].reshape(P)
        onehot = torch.nn.functional.one_hot(tr["label"].reshape(P).long(), sc.num_classes).float()
        step = lambda: _l1_step(torch, fr, g, maps, t_rgb, t_depth, onehot)
        ms = _time(torch, step, 10 if ncams == 1 else 3)
        st, nvis, nk = fr.status()
        assert st == 0, st
        B = int(maps["n_contrib"].sum())
        r = {"views": ncams, "gaussians": sc.n, "classes": sc.num_classes, "ms": round(ms, 4), "blends": B,
             "blends_per_s": round(B / (ms * 1e-3), 1), "keys": nk, "visible": nvis}
        del maps, onehot, fr
        if ncams > 1:
            # candidate scoring from device poses, in launches of 16 views (the
            # planner's chunked path; a status read after each launch)
            from paper_2506_00225_amd import make_config
            from paper_2506_00225_amd.planner import Grid, Planner
            cands = sc.candidates
            pl = Planner(Grid((1, 1, 1), 1.0, (0.0, 0.0, 0.0)), cands[0], make_config(sc.num_classes, sc.k),
                         capacity=len(cands), chunk=16)
            poses = np.stack([np.concatenate([np.asarray(c.R, np.float32).reshape(9),
                                              np.asarray(c.t, np.float32).reshape(3)]) for c in cands])
            pl.poses[:len(cands)].copy_(torch.from_numpy(poses))
            sms = _time(torch, lambda: pl.score_views(g, len(cands)), 3)
            r.update({"candidates": len(cands), "score_ms": round(sms, 3),
                      "views_per_s": round(len(cands) / (sms * 1e-3), 1)})
            del pl
        res[name] = r
        log("config", name, json.dumps(r))
        torch.cuda.empty_cache()
    out["configs"] = res


def cpu_baseline(sc, rows=None, min_s=10.0):
    """The FP64 oracle (as it stands) on the same keyframe and the same 1M
    Gaussians: projection of all Gaussians, forward render and analytic
    backward of `rows` image rows through the middle (all of them by
    default, about 10 s on 16 host threads)."""
    from oracle import oracle as O
    from paper_2506_00225_amd import scenes

    cam = sc.cameras[0]
    rows = cam.height if rows is None else rows
    band = scenes.Camera(cam.R, cam.t, cam.fx, cam.fy, cam.cx, cam.cy - (cam.height - rows) / 2, cam.width, rows)
    cfg = O.config_array()
    rng = np.random.default_rng(0)
    grads = {"rgb": rng.standard_normal((rows, cam.width, 3)), "depth": rng.standard_normal((rows, cam.width)),
             "sil": rng.standard_normal((rows, cam.width)),
             "sem": rng.standard_normal((rows, cam.width, sc.num_classes))}
    # repeat the whole fwd+bwd until about 10 s of host work (at most 16 times)
    reps, t = 0, 0.0
    while reps < 16 and (reps == 0 or t < min_s):
        t0 = time.perf_counter()
        pr, mp = O.forward(O.scene_arrays(sc), band, cfg, sc.num_classes)
        O.backward(O.scene_arrays(sc), band, cfg, sc.num_classes, grads, proj=pr)
        t += time.perf_counter() - t0
        reps += 1
    B = int(mp["n_contrib"].sum()) * reps
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": B / t, "unit": "blends/s", "cores": threads, "kind": "oracle",
            "sample": (f"{reps} x fwd+bwd of the full {cam.width}x{rows} keyframe" if rows == cam.height else
                       f"{reps} x fwd+bwd of a {cam.width}x{rows} band through the keyframe centre") +
                      f", all {sc.n} Gaussians projected each time; {B} blends in {t:.2f} s"}


def oracle_legs(out):
    """The FP64 oracle (as it stands) on the other workloads, on the host
    threads, beside the GPU figures of the same legs: the 64x64 forward
    (repeated to about 1 s), the 200k forward + backward of the full
    keyframe, one 1024x1280 keyframe of the 3M scene forward + backward,
    and the first 8 of the 64 candidate views scored (forward + entropy)."""
    from oracle import oracle as O
    from paper_2506_00225_amd import scenes
    cfg = O.config_array()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    res = {}

    def grads_for(cam, C, seed):
        rng = np.random.default_rng(seed)
        h, w = cam.height, cam.width
        return {"rgb": rng.standard_normal((h, w, 3)), "depth": rng.standard_normal((h, w)),
                "sil": rng.standard_normal((h, w)), "sem": rng.standard_normal((h, w, C))}

    sc = scenes.tiny_scene()
    reps, t = 0, 0.0
    while reps < 200 and (reps == 0 or t < 1.0):
        t0 = time.perf_counter()
        _, mp = O.forward(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes)
        t += time.perf_counter() - t0
        reps += 1
    B = int(mp["n_contrib"].sum())
    res["forward_64x64_2k"] = {"ms": round(t / reps * 1e3, 3), "blends": B, "sample": f"{reps} forward passes"}
    for name, sc, cam in (("fwd_bwd_200k_1200x680", scenes.room_scene(n=200_000, targets=False), None),
                          ("large_3m_8x1024x1280", scenes.large_scene(), None)):
        cam = sc.cameras[0]
        gr = grads_for(cam, sc.num_classes, 1)
        t0 = time.perf_counter()
        pr, mp = O.forward(O.scene_arrays(sc), cam, cfg, sc.num_classes)
        O.backward(O.scene_arrays(sc), cam, cfg, sc.num_classes, gr, proj=pr)
        t = time.perf_counter() - t0
        B = int(mp["n_contrib"].sum())
        res[name] = {"ms": round(t * 1e3, 1), "blends": B, "blends_per_s": round(B / t, 1),
                     "sample": f"forward + backward of one {cam.width}x{cam.height} keyframe, all {sc.n} Gaussians"}
        del mp, gr
    sc = scenes.candidate_scene(n=500_000, nviews=64)
    t0 = time.perf_counter()
    for cam in sc.cameras[:8]:
        _, mp = O.forward(O.scene_arrays(sc), cam, cfg, sc.num_classes)
        O.score(mp, sc.num_classes)
    t = time.perf_counter() - t0
    res["score_64_views"] = {"views_per_s": round(8 / t, 2), "sample": "the first 8 of the 64 candidate views"}
    for k_, v in res.items():
        v["cores"] = threads
    out["oracle_legs"] = res


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline_one_thread(n, rows):
    """The same oracle pass on one host thread (a child process with
    OMP_NUM_THREADS=1: the thread count of the oracle's OpenMP runtime is
    fixed when it starts), over a band of `rows` rows."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, %r); import bench; from paper_2506_00225_amd import scenes; "
            "print(json.dumps(bench.cpu_baseline(scenes.room_scene(n=%d, targets=False), rows=%d, min_s=0.0)))"
            % (ROOT, n, rows))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        log("one-thread oracle failed", r.stderr[-500:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}); the rasterizer in this "
              "repository has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    out = {}
    if args.no_mapping:
        if not args.no_score:
            score_bench(args, torch, out)
        print(json.dumps({k: v for k, v in out.items() if not k.startswith("autotune")}), flush=True)
        return
    sc = mapping_bench(args, torch, out)
    if not args.no_score:
        score_bench(args, torch, out)
        if not args.no_plan:
            plan_bench(args, torch, out)
        if not args.no_dense:
            dense_bench(args, torch, out)
    if not args.no_configs:
        config_legs(args, torch, out)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # reads and writes copy_probe MiB each
        torch.cuda.synchronize()
        log("copy probe", args.copy_probe, "MiB x3")
    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(sc)
        cpu.update(cpu_info())
        log("cpu baseline, one thread")
        one = cpu_baseline_one_thread(sc.n, rows=68)
        if one is not None:
            cpu["one_thread"] = {"value": one["value"], "unit": one["unit"], "sample": one["sample"]}
        if not args.no_configs:
            log("oracle on the other workloads")
            oracle_legs(out)
    dom, roof = roofline(out)
    value = out["blends"] / (out["step_ms"] * 1e-3)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "blends/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(out["step_ms"], 4),
        "ms_per_step_with_stage_events": round(out["step_ms_with_stage_events"], 4),
        "ms_per_step_gather_and_adam_apart": round(out["step_unfused_ms"], 4),
        "host_wall_ms_per_step": round(out["wall_ms"], 4), "host_enqueue_ms_per_step": round(out["enqueue_ms"], 4),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mapping iteration: 1M Gaussians, 10x8x3 m room, 1200x680 keyframe, C=102, k=16, "
                               "fwd + loss + bwd + Adam", "gaussians": out["n"], "width": 1200, "height": 680,
                   "classes": out["C"], "top_k": out["k"]},
        "fwd_bwd_ms": round(out["fwd_bwd_ms"], 4),
        "blends_per_s_fwd_bwd": round(out["blends"] / (out["fwd_bwd_ms"] * 1e-3), 1),
        "blends_per_step": out["blends"], "keys": out["keys"], "visible": out["nvis"],
        "stage_ms": {k_: round(v, 4) for k_, v in out["stage_ms"].items()},
        "loss_first_last": out["loss_first_last"],
        "roofline": roof,
        "hbm_fwd_bwd": hbm_path(out),
        "cpu_baseline": cpu,
    }
    for key in ("views_per_s_batched", "views_per_s_graph", "views_per_s_plain", "score_batched_ms", "score_graph_ms",
                "score_graph_equal", "score_plain_ms",
                "score_max_mean_entropy_diff", "score_n_empty_equal", "score_views", "plan", "dense_vs_sparse",
                "configs", "oracle_legs"):
        if key in out:
            line[key] = out[key]
    tuned = {k: out[k]["chosen"] for k in ("autotune_mapping", "autotune_score") if k in out and "chosen" in out[k]}
    if tuned:
        line["autotune"] = tuned
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

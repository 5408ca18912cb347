"""Benchmark of the semantic Gaussian rasterizer on one MI355X.

Step = one mapping iteration on 1M Gaussians in a 10x8x3 m room seen by one
1200x680 keyframe (fx=fy=600): project -> bin -> render_forward -> loss
gradient -> render_backward -> Adam.  The loss is the mapping loss with the
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
# fp32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (packed pair) x 2 flops (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3


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

    def step(i, marked):
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
    # and the losses come from as many further steps with an event at every
    # stage boundary.
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
    log("breakdown", args.steps)
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
    out.update(dict(step_ms=step_ms, step_ms_with_stage_events=marked_ms, wall_ms=wall * 1e3 / args.steps,
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
    are reported against the fp32 vector peak with the algorithmic
    operation count per blend (B blends per launch, the same B as the
    oracle's): per evaluation of a blended pair 12 fp32 operations and one
    exponential; per forward blend 6 + k accumulations; per backward blend
    40 + 3k operations (transmittance, dL/dalpha over the channels, the
    colour, opacity, conic and mean terms and the top-k semantic terms).
    An FMA counts as one operation, so the figure is a lower bound.
    Their algorithmic bytes (every input read once, every output and
    compulsory intermediate written once) are reported beside it.  Other
    stages are HBM-bound and reported against the HBM peak."""
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
    ops_per_blend = {"fwd": 13 + 6 + k, "bwd_tiles": 13 + 40 + 3 * k}
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
                     "ops_per_blend": ops_per_blend[dom], "hbm_gbs": round(gbs, 2),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return dom, {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(gbs / HBM_PEAK_GBS, 4), **common}


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


def cpu_baseline(sc, rows=None):
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
    while reps < 16 and (reps == 0 or t < 10.0):
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
    sc = mapping_bench(args, torch, out)
    if not args.no_score:
        score_bench(args, torch, out)
        plan_bench(args, torch, out)
        dense_bench(args, torch, out)
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
    dom, roof = roofline(out)
    value = out["blends"] / (out["step_ms"] * 1e-3)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "blends/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(out["step_ms"], 4),
        "ms_per_step_with_stage_events": round(out["step_ms_with_stage_events"], 4),
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
        "cpu_baseline": cpu,
    }
    for key in ("views_per_s_batched", "views_per_s_graph", "views_per_s_plain", "score_batched_ms", "score_graph_ms",
                "score_graph_equal", "score_plain_ms",
                "score_max_mean_entropy_diff", "score_n_empty_equal", "score_views", "plan", "dense_vs_sparse"):
        if key in out:
            line[key] = out[key]
    tuned = {k: out[k]["chosen"] for k in ("autotune_mapping", "autotune_score") if k in out and "chosen" in out[k]}
    if tuned:
        line["autotune"] = tuned
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

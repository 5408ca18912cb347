"""Autotuner for the launch choices that change speed but not results.

The knobs live in `sgr_config` and are read by the library on every call:

* ``sem_accumulators``: per-pixel class sums in LDS or in registers (C <= 128);
* ``tile_order``: XCD-contiguous runs of tiles (each XCD's L2 sees
  neighbouring tiles, which share Gaussians) or plain linear order;
* ``score_workgroups``: size of the persistent scoring grid;
* ``sem_passes``: with the class sums in LDS, how many class ranges a tile
  is composited in (1/passes of the LDS each, so more workgroups share a CU,
  against recompositing the geometry once per range);
* ``bwd_batch``: keys the backward stages per batch (32, 44, 56: LDS per
  workgroup against barriers per key);
* ``radix_bits``: the widest digit of the depth and tile sorts (6 or 8).

Every candidate is run on the caller's own frame and data, timed with HIP
events on the current stream, and its outputs are compared bit for bit with
the first candidate's; a mismatch raises, since these choices must not change
any output.  The search runs in two stages: the product of the first four
knobs, then the batch size and digit width with the stage-one winner fixed.
The winner is written into ``frame.cfg`` and remembered per GPU
architecture and workload shape (number of Gaussians, classes, k, view
sizes), in memory and in a JSON file (``SGR_AUTOTUNE_CACHE``, by default
``~/.cache/sgr/autotune.json``; set it to an empty string to keep the cache
in memory only).

Not searched: the tile shape (16x16: the binning keys, and so the sorted key
lists the parity tests pin, are defined on it), the forward's staging batch
(128 entries, one per lane of two waves), the waves per workgroup (one
pixel per lane of a 16x16 tile), and the order of views in a batched
scoring launch (its tiles are handed out with a static stride, and each
view's sums are reduced in tile order, so neither balance nor results
depend on it).
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import _lib as L

_CACHE: dict = {}

KNOBS = ("sem_accumulators", "tile_order", "score_workgroups", "sem_passes", "bwd_batch", "radix_bits")


def cache_path() -> str | None:
    """The JSON cache file (None: memory only)."""
    p = os.environ.get("SGR_AUTOTUNE_CACHE")
    if p is None:
        p = os.path.join(os.path.expanduser("~"), ".cache", "sgr", "autotune.json")
    return p or None


def _arch(frame) -> str:
    try:
        return str(torch.cuda.get_device_properties(frame.device).gcnArchName)
    except Exception:  # noqa: BLE001 - no device properties: the key still separates shapes
        return "unknown"


def shape_key(arch: str, what: str, n: int, num_classes: int, top_k: int, sizes) -> str:
    """Cache key of one tuning: architecture, what was timed, and the
    workload shape (sizes: (height, width) per view)."""
    views = ",".join(f"{int(h)}x{int(w)}" for h, w in sizes)
    return f"{arch}|{what}|n={int(n)}|C={int(num_classes)}|k={int(top_k)}|views={views}"


def _shape_key(frame, what: str) -> str:
    return shape_key(_arch(frame), what, frame.n, frame.cfg.num_classes, frame.cfg.top_k, frame.sizes)


def load_cached(key: str, path: str | None = None):
    """Knob tuple stored for key (memory, then the JSON file), or None."""
    if key in _CACHE:
        return _CACHE[key]
    path = cache_path() if path is None else path
    if not path or not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not isinstance(rec, dict) or any(k not in rec for k in KNOBS):
        return None
    knobs = tuple(int(rec[k]) for k in KNOBS)
    _CACHE[key] = knobs
    return knobs


def store(key: str, knobs, ms: float | None = None, path: str | None = None):
    """Remembers knobs for key in memory and in the JSON file (rewritten
    whole through a temporary file, so a reader never sees half of it)."""
    _CACHE[key] = tuple(int(x) for x in knobs)
    path = cache_path() if path is None else path
    if not path:
        return
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        data = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
        data[key] = dict(zip(KNOBS, _CACHE[key]), **({} if ms is None else {"ms": round(float(ms), 4)}))
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except (OSError, ValueError):
        pass  # an unwritable cache only costs a re-tune


def _knobs(cfg):
    return tuple(int(getattr(cfg, k)) for k in KNOBS)


def _set(cfg, knobs):
    for k, v in zip(KNOBS, knobs):
        setattr(cfg, k, v)


def _time(fn, reps: int) -> float:
    fn()  # warm-up (first launch of a kernel variant)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _snapshot(outs) -> list:
    return [t.clone() for t in outs if t is not None]


def _same(a: list, b: list) -> bool:
    return len(a) == len(b) and all(torch.equal(x, y) for x, y in zip(a, b))


def _search(frame, candidates, run, reps: int, what: str):
    original = _knobs(frame.cfg)
    report, ref, best = [], None, None  # best: (knobs, ms, index into report)
    try:
        for knobs in candidates:
            _set(frame.cfg, knobs)
            try:
                outs = _snapshot(run())
            except L.SgrError as e:  # e.g. the class sums of one pass exceed the LDS
                if e.status != L.SGR_EUNSUPPORTED:
                    raise
                continue
            if ref is None:
                ref = outs
            elif not _same(ref, outs):
                raise RuntimeError(f"autotune({what}): candidate {knobs} changed the outputs")
            ms = _time(run, reps)
            report.append(dict(zip(KNOBS, knobs), ms=round(ms, 4)))
            if best is None or ms < best[1]:
                best = (knobs, ms, len(report) - 1)
    except Exception:
        _set(frame.cfg, original)
        raise
    if best is None:
        _set(frame.cfg, original)
        raise L.SgrError(L.SGR_EUNSUPPORTED, f"autotune({what}): no candidate runs")
    _set(frame.cfg, best[0])
    return {"what": what, "chosen": report[best[2]], "candidates": report, "knobs": best[0], "ms": best[1]}


def _two_stage(frame, first, run, reps: int, what: str, radix=(8, 6), batches=(44, 32, 56)):
    """Stage one over `first`; stage two over bwd_batch x radix_bits with
    the stage-one winner's other knobs.  Stores the winner."""
    r1 = _search(frame, first, run, reps, what)
    base = r1["knobs"]
    second = [base[:4] + (nb, rb) for nb, rb in itertools.product(batches, radix)]
    r2 = _search(frame, second, run, reps, what)
    store(_shape_key(frame, what), r2["knobs"], r2["ms"])
    return {"what": what, "chosen": r2["chosen"], "candidates": r1["candidates"] + r2["candidates"]}


def _placements(cfg):
    """(sem_accumulators, sem_passes) pairs: LDS in 1..3 class ranges, and
    registers when C <= 128."""
    out = [(L.SGR_ACC_LDS, p) for p in (1, 2, 3)]
    return out + ([(L.SGR_ACC_REGISTERS, 0)] if cfg.num_classes <= 128 else [])


def tune_mapping(frame, g, grads: dict | None = None, reps: int = 5, targets=None, loss_cfg=None):
    """Chooses accumulator placement, class passes and tile order for the
    mapping pass of `frame` on Gaussians `g` (already projected and binned).
    With `targets` (as for Frame.forward_loss) the timed pass is what a
    mapping iteration runs: the fused forward + loss, then the backward of
    its gradients (one class per pixel when every target is a label map).
    Otherwise it is forward, then backward of `grads` (random if None).
    Returns a report."""
    what = "mapping" if targets is None else "mapping_loss"
    cached = load_cached(_shape_key(frame, what))
    if cached is not None:
        _set(frame.cfg, cached)
        return {"what": what, "cached": dict(zip(KNOBS, cached)), "chosen": dict(zip(KNOBS, cached))}
    out = {name: torch.empty_like(getattr(g, name)) for name in
           ("means", "scales", "quats", "opacity", "rgb", "sem_val")}
    if targets is not None:
        tl = [targets] if isinstance(targets, dict) else list(targets)
        sparse = all(t.get("label") is not None and t.get("sem") is None for t in tl)
        buf = {}

        def run():
            frame.project(g)
            frame.bin(g)
            gr, loss = frame.forward_loss(g, targets, loss_cfg, grads=buf.get("g"), sparse_sem=sparse)
            buf["g"] = gr
            frame.backward(g, dict(gr), out)
            return [loss] + list(gr.values()) + list(out.values())
    else:
        maps = frame.alloc_maps()
        if grads is None:
            gen = torch.Generator(device=frame.device).manual_seed(0)
            grads = {k: torch.randn(maps[k].shape, generator=gen, device=frame.device)
                     for k in ("rgb", "depth", "sil", "sem")}

        def run():
            frame.project(g)
            frame.bin(g)
            frame.forward(g, maps)
            frame.backward(g, dict(grads), out)
            return list(maps.values()) + list(out.values())

    sw, nb, rb = int(frame.cfg.score_workgroups), int(frame.cfg.bwd_batch), int(frame.cfg.radix_bits)
    cands = [(acc, order, sw, passes, nb, rb) for (acc, passes), order in
             itertools.product(_placements(frame.cfg), (L.SGR_TILES_XCD, L.SGR_TILES_LINEAR))]
    return _two_stage(frame, cands, run, reps, what)


def tune_score(frame, g, reps: int = 3, workgroups=(0, 512, 1024, 2048)):
    """Chooses accumulator placement, class passes, tile order and the
    persistent grid for `frame.score(g)`.  Returns a report."""
    cached = load_cached(_shape_key(frame, "score"))
    if cached is not None:
        _set(frame.cfg, cached)
        return {"what": "score", "cached": dict(zip(KNOBS, cached)), "chosen": dict(zip(KNOBS, cached))}
    ne = torch.empty(frame.V, dtype=torch.int32, device=frame.device)
    hs = torch.empty(frame.V, dtype=torch.float64, device=frame.device)

    def run():
        frame.score(g, ne, hs)
        return [ne, hs]

    nb, rb = int(frame.cfg.bwd_batch), int(frame.cfg.radix_bits)
    cands = [(acc, order, wg, passes, nb, rb) for (acc, passes), order, wg in
             itertools.product(_placements(frame.cfg), (L.SGR_TILES_XCD, L.SGR_TILES_LINEAR), workgroups)]
    # the scorer has no backward: only the digit width in stage two
    return _two_stage(frame, cands, run, reps, "score", batches=(nb,))


def clear_cache():
    _CACHE.clear()

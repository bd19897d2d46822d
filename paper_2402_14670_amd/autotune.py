"""Autotuner of the launch configuration.

Times every candidate configuration of the batched and persistent launches
on a resident batch (HIP events on the given stream), applies the fastest
with lf_set_exec and returns the whole table.  Candidates: wavefronts per
workgroup (1, 2, 4); for the persistent launch also tracks per queue claim
(1, 2, 4, 8, 16) and the grid: the occupancy limit the runtime reports, or
16, 20, 24 or 28 wavefronts per compute unit (fewer resident wavefronts can
be faster: the runtime's limit need not be what the hardware places, and
the track loop's issue rate stops growing before it).  The window capacity of the kernels (LDS staging of 32 or 64 hits
per layer) follows n_hits_window and is not a free choice.
"""
from __future__ import annotations

import itertools

from . import lf


def candidates(modes=("batched", "persistent")):
    out = []
    for mode in modes:
        for wpb in (1, 2, 4):
            if mode == "persistent":
                grids = (0,) + tuple(w // wpb for w in (16, 20, 24, 28))
                for items, bpc in itertools.product((1, 2, 4, 8, 16), grids):
                    out.append(dict(mode=mode, waves_per_block=wpb, items_per_grab=items, blocks_per_cu=bpc))
            else:
                out.append(dict(mode=mode, waves_per_block=wpb, items_per_grab=1, blocks_per_cu=0))
    return out


def time_config(ctx, batch_id, cfg, stream, steps=5, warmup=1) -> float:
    import torch
    # waves_per_block first: it resets blocks_per_cu to the occupancy limit
    lf.lf_set_exec(ctx, waves_per_block=cfg["waves_per_block"])
    lf.lf_set_exec(ctx, items_per_grab=cfg["items_per_grab"], blocks_per_cu=cfg["blocks_per_cu"])
    for _ in range(warmup):
        lf.lf_find_tracks(ctx, batch_id, cfg["mode"], stream.cuda_stream)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        lf.lf_find_tracks(ctx, batch_id, cfg["mode"], stream.cuda_stream)
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / steps


def autotune(ctx, batch_id, stream, modes=("batched", "persistent"), steps=5) -> dict:
    """Time the candidates on a resident batch; keep the fastest.

    Returns {"best": cfg with "ms", "per_mode": best cfg per mode, "table": [...]}.
    The context is left configured with the best persistent configuration's
    launch parameters when the best mode is persistent, else with the best
    batched one."""
    table = []
    cands = candidates(modes)
    # the batched mode's three candidates lie within a few percent of each
    # other: each gets more launches, timed in three interleaved rounds after
    # a warm-up of the device (the first candidate timed on a cold device
    # would lose to its order alone), and keeps its best round
    batched = [c for c in cands if c["mode"] == "batched"]
    if batched:
        time_config(ctx, batch_id, batched[0], stream, steps=max(steps, 12))
        best_ms = {}
        for _ in range(3):
            for k, cfg in enumerate(batched):
                ms = time_config(ctx, batch_id, cfg, stream, steps=max(steps, 12))
                best_ms[k] = min(best_ms.get(k, ms), ms)
        table += [dict(cfg, ms=round(best_ms[k], 4)) for k, cfg in enumerate(batched)]
    for cfg in cands:
        if cfg["mode"] == "batched":
            continue
        ms = time_config(ctx, batch_id, cfg, stream, steps=steps)
        table.append(dict(cfg, ms=round(ms, 4)))
    per_mode = {}
    for row in table:
        m = row["mode"]
        if m not in per_mode or row["ms"] < per_mode[m]["ms"]:
            per_mode[m] = row
    best = min(table, key=lambda r: r["ms"])
    lf.lf_set_exec(ctx, waves_per_block=best["waves_per_block"])
    lf.lf_set_exec(ctx, items_per_grab=best["items_per_grab"], blocks_per_cu=best["blocks_per_cu"])
    return {"best": best, "per_mode": per_mode, "table": table}

"""Helpers of the GPU parity tests: run both sides on the same batch and
compare slot by slot (indices bit-exact, parameters within 1e-5 relative)."""
from __future__ import annotations

import sys

import numpy as np

import lfgen
import oracle

W = lfgen.world()
PARAM_KEYS = ("a", "b", "c", "y0", "ty", "qop", "Q")
RTOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(ev, mode="batched", params=None, exec_cfg=None, stream=None, world=None):
    from paper_2402_14670_amd import lf
    ctx = lf.lf_create(W if world is None else world, params)
    try:
        if exec_cfg:
            lf.lf_set_exec(ctx, **exec_cfg)
        bid = lf.lf_upload_events(ctx, ev, stream)
        lf.lf_find_tracks(ctx, bid, mode, stream)
        return lf.lf_fetch_tracks(ctx, bid, ev.n_tracks, stream)
    finally:
        lf.lf_destroy(ctx)


def compare(ref: dict, got: dict, rows=None, label: str = "") -> dict:
    """Indices and flags bit-exact; parameters within RTOL relative (0 stays 0)."""
    sel = slice(None) if rows is None else rows
    for k in ("found", "n_hits", "hit_idx"):
        r, g = ref[k][sel], got[k][sel]
        if not np.array_equal(r, g):
            bad = np.nonzero((r != g).reshape(len(r), -1).any(1))[0]
            raise AssertionError(f"{label}: {k} differs on {len(bad)} tracks, first {bad[:8].tolist()}")
    exact = 0
    total = 0
    for k in PARAM_KEYS:
        r, g = ref[k][sel].astype(np.float64), got[k][sel].astype(np.float64)
        ok = np.abs(g - r) <= RTOL * np.abs(r)
        if not ok.all():
            i = int(np.nonzero(~ok)[0][0])
            raise AssertionError(f"{label}: {k} off by more than {RTOL} relative, first slot {i}: "
                                 f"gpu {g[i]!r} oracle {r[i]!r}")
        exact += int((ref[k][sel].view(np.uint32) == got[k][sel].view(np.uint32)).sum())
        total += len(r)
    return dict(bit_exact_params=exact, params=total, found=int(ref["found"][sel].sum()))


def host_threads() -> int:
    """Threads for the oracle on this host (at most 16, one GPU's share)."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def oracle_parallel(ev, params=None, world=None):
    """The oracle over a whole batch, its events split into one contiguous
    slice per host thread (the oracle's C call releases the GIL); the same
    results as one oracle.run over the batch, in the batch's track order."""
    import concurrent.futures as cf
    n = host_threads()
    bounds = [(ev.n_events * k // n, ev.n_events * (k + 1) // n) for k in range(n)]
    parts = [lfgen.select_events(ev, range(a, b)) for a, b in bounds if b > a]
    w = W if world is None else world
    with cf.ThreadPoolExecutor(max_workers=n) as pool:
        outs = list(pool.map(lambda part: oracle.run(part, w, params), parts))
    return {k: np.concatenate([o[k] for o in outs]) for k in outs[0]}


def oracle_rows(ev, events):
    """Global track rows of the given events."""
    rows = [np.arange(int(ev.trk_off[e]), int(ev.trk_off[e + 1])) for e in events]
    return np.concatenate(rows) if rows else np.zeros(0, np.int64)


def oracle_on_events(ev, events, params=None, world=None):
    """Oracle results for the listed events, placed in a full-size result."""
    sub = lfgen.select_events(ev, events)
    o = oracle.run(sub, W if world is None else world, params)
    T = ev.n_tracks
    full = dict(found=np.zeros(T, np.uint8), n_hits=np.zeros(T, np.uint8), hit_idx=np.full((T, 12), -1, np.int32))
    for k in PARAM_KEYS:
        full[k] = np.zeros(T, np.float32)
    rows = oracle_rows(ev, events)
    for k in full:
        full[k][rows] = o[k]
    return full, rows


# serving digests: the definition lives with the binding (it is part of lf.h)
def event_digests(out, trk_off):
    from paper_2402_14670_amd.lf import result_digests
    return result_digests(out, trk_off)

"""Truth matching on generated events (the paper's Benchmarking setup).

A found track is matched to a particle when more than 70% of its hits come
from that particle; it is a ghost (fake) otherwise.  A particle is
reconstructible when it has an upstream input track and leaves at least one x
hit and one u/v hit in each of the three stations.  Efficiency counts a
reconstructible particle as found when the input track it produced is found
and matched to it.

This evaluates outputs against the generator's truth; it holds none of the
track-following arithmetic.
"""
from __future__ import annotations

import numpy as np

NL = 12


def reconstructible(ev) -> np.ndarray:
    m = ev.par_mask.astype(np.int64)
    ok = ev.par_has_track.astype(bool).copy()
    for st in range(3):
        xbits = (1 << (4 * st)) | (1 << (4 * st + 3))
        uvbits = (1 << (4 * st + 1)) | (1 << (4 * st + 2))
        ok &= (m & xbits) != 0
        ok &= (m & uvbits) != 0
    return ok


def match(ev, out) -> np.ndarray:
    """Event-local particle index matched by each found track; -1 ghost, -2 not found."""
    T = ev.n_tracks
    res = np.full(T, -2, np.int64)
    found = np.nonzero(out["found"])[0]
    if found.size == 0:
        return res
    base = ev.event_hit_base().astype(np.int64)
    tev = ev.track_event().astype(np.int64)
    hi = out["hit_idx"][found].astype(np.int64)                 # (F, 12)
    present = hi >= 0
    g = np.where(present, hi + base[tev[found]][:, None], 0)
    pid = np.where(present, ev.hit_pid[g].astype(np.int64), -2)  # -2 absent, -1 noise
    # occurrences of each slot's particle among the track's hits
    same = (pid[:, :, None] == pid[:, None, :]) & present[:, None, :]
    cnt = np.where(present & (pid >= 0), same.sum(axis=2), -1)
    # the most frequent particle (ties: the first slot, as a stable mode)
    k = np.argmax(cnt, axis=1)
    best = pid[np.arange(len(found)), k]
    bc = cnt[np.arange(len(found)), k]
    n = present.sum(axis=1)
    res[found] = np.where((best >= 0) & (bc > 0.7 * n), best, -1)
    return res


def physics(ev, out, p_min: float = 0.0) -> dict:
    """Efficiency over reconstructible particles (p > p_min), ghost rate, q/p resolution."""
    m = match(ev, out)
    tev = ev.track_event().astype(np.int64)
    rec = reconstructible(ev) & (ev.par_p > p_min)
    found_par = np.zeros(len(ev.par_p), bool)
    ok = np.nonzero(m >= 0)[0]
    g = ev.par_off[tev[ok]].astype(np.int64) + m[ok]
    # credit only the particle behind this input track
    mine = ev.trk_pid[ok].astype(np.int64) == m[ok]
    found_par[g[mine]] = True
    qop_true = ev.par_q[g].astype(np.float64) / ev.par_p[g].astype(np.float64)
    rel = out["qop"][ok].astype(np.float64) / qop_true - 1.0
    n_found = int((out["found"] != 0).sum())
    return dict(
        efficiency=float(found_par[rec].mean()) if rec.any() else float("nan"),
        n_reconstructible=int(rec.sum()),
        ghost_rate=float((m == -1).sum() / n_found) if n_found else 0.0,
        n_found=n_found,
        qop_resolution=float(np.sqrt(np.mean(rel ** 2))) if len(rel) else float("nan"),
        qop_rel=rel,
    )

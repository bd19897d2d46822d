"""Truth matching on generated events (the paper's Benchmarking setup).

A found track is matched to a particle when more than 70% of its hits come
from that particle; it is a ghost (fake) otherwise.  A particle is
reconstructible when it has an upstream input track and leaves at least one x
hit and one u/v hit in each of the three stations.
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
    base = ev.event_hit_base().astype(np.int64)
    tev = ev.track_event()
    found = np.nonzero(out["found"])[0]
    for t in found:
        hi = out["hit_idx"][t]
        hi = hi[hi >= 0].astype(np.int64) + base[tev[t]]
        pids = ev.hit_pid[hi]
        vals, cnt = np.unique(pids, return_counts=True)
        k = int(np.argmax(cnt))
        res[t] = vals[k] if (vals[k] >= 0 and cnt[k] > 0.7 * len(hi)) else -1
    return res


def physics(ev, out, p_min: float = 0.0) -> dict:
    """Efficiency over reconstructible particles (p > p_min), ghost rate, q/p resolution."""
    m = match(ev, out)
    tev = ev.track_event()
    rec = reconstructible(ev) & (ev.par_p > p_min)
    found_par = np.zeros(len(ev.par_p), bool)
    rel = []
    for t in np.nonzero(m >= 0)[0]:
        g = int(ev.par_off[tev[t]]) + int(m[t])
        # credit only the particle behind this input track
        if ev.trk_pid[t] == m[t]:
            found_par[g] = True
        qop_true = float(ev.par_q[g]) / float(ev.par_p[g])
        rel.append(float(out["qop"][t]) / qop_true - 1.0)
    n_found = int((out["found"] != 0).sum())
    rel = np.asarray(rel)
    return dict(
        efficiency=float(found_par[rec].mean()) if rec.any() else float("nan"),
        n_reconstructible=int(rec.sum()),
        ghost_rate=float((m == -1).sum() / n_found) if n_found else 0.0,
        n_found=n_found,
        qop_resolution=float(np.sqrt(np.mean(rel ** 2))) if len(rel) else float("nan"),
        qop_rel=rel,
    )

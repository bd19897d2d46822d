"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each ``pin_*`` function takes an oracle library handle (``None`` = the built
oracle) and raises AssertionError when the oracle disagrees.  The same pins
are run against copies of the oracle with planted mistakes, each of which
must fail at least one pin.
"""
from __future__ import annotations

import functools
import math
import os

import numpy as np

import lfgen
import oracle
from lfgen import truth

NL = 12
X_LAYERS = (0, 3, 4, 7, 8, 11)
UV_LAYERS = (1, 2, 5, 6, 9, 10)
SEED_SETS = ((0, 4, 8), (3, 7, 11))
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_constants.txt")
W = lfgen.world()
f32 = np.float32


def golden_constants() -> dict:
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head = line.split("|")[0].split()
            out[head[0]] = float(head[1])
    return out


# ------------------------------------------------------------------ events
@functools.lru_cache(maxsize=None)
def ev_noise_free(seed: int = 11, p_min: float = 1.5, p_max: float = 50.0, n: int = 40):
    """Single-event geometry, no smearing, no noise, every layer efficient."""
    return lfgen.generate("single", seed=seed, sigma_x=0.0, qop_sigma=0.0, hit_eff=1.0, n_noise=0,
                          p_min=p_min, p_max=p_max, n_particles=n)


@functools.lru_cache(maxsize=None)
def ev_single():
    return lfgen.generate("single")


@functools.lru_cache(maxsize=None)
def ev_nominal(n: int = 2):
    return lfgen.generate("nominal", n_events=n)


@functools.lru_cache(maxsize=None)
def ev_stress():
    return lfgen.generate("stress", n_events=1)


@functools.lru_cache(maxsize=None)
def ev_tiny():
    return lfgen.generate("single", seed=7, n_events=6, n_particles=8, n_noise=20, p_min=1.5,
                          p_max=20.0)


def truth_hit(ev, t: int, layer: int) -> int:
    """Event-local index of the hit the track's particle left in ``layer`` (-1 if none)."""
    e = int(ev.track_event()[t])
    pid = int(ev.trk_pid[t])
    base = int(ev.hit_off[24 * e])
    for zone in (0, 1):
        b = 24 * e + 2 * layer + zone
        h = np.arange(int(ev.hit_off[b]), int(ev.hit_off[b + 1]))
        h = h[ev.hit_pid[h] == pid]
        if len(h):
            return int(h[0]) - base
    return -1


def particle(ev, t: int):
    e = int(ev.track_event()[t])
    g = int(ev.par_off[e]) + int(ev.trk_pid[t])
    return float(ev.par_p[g]), float(ev.par_q[g]), float(ev.par_tx[g]), float(ev.par_ty[g])


# ------------------------------------------------------------------ pins
def pin_constants(lib=None):
    """Default parameters equal the values the paper prints."""
    gold = golden_constants()
    p = oracle.make_params(None, lib)
    for k, v in gold.items():
        if k.startswith("C_"):
            got = p.C_nhits[int(k[2:]) - 9]
        elif k == "z_ref":
            got = oracle.Z_REF
        else:
            got = getattr(p, k)
        assert got == f32(v), f"{k}: oracle default {got} != paper {v}"


def pin_extrapolation_noise_free(lib=None):
    """Window centres equal the exact hit positions of noise-free tracks with
    exact q/p (x layers: x; u/v layers: x - dxdy*y), and the truth hit sits
    inside every window."""
    ev = ev_noise_free()
    o = oracle.run(ev, W, debug=True, lib=lib)
    worst = 0.0
    n = 0
    for t in range(ev.n_tracks):
        for l in range(NL):
            h = truth_hit(ev, t, l)
            if h < 0:
                continue
            base = int(ev.hit_off[24 * int(ev.track_event()[t])])
            worst = max(worst, abs(float(o["wx"][t, l, 1]) - float(ev.hit_x[base + h])))
            assert o["win"][t, l, 0] <= h < o["win"][t, l, 1], f"truth hit outside window t={t} l={l}"
            n += 1
    assert n > 300
    assert worst <= 1e-3, f"window centre off the exact hit by {worst} mm"


def pin_window_bounds(lib=None):
    """x-layer width 2*(150 + 2000/p) + 100 with the asymmetry on the bending
    side; u/v layers +-800 mm around the centre."""
    ev = ev_single()
    o = oracle.run(ev, W, debug=True, lib=lib)
    for t in range(ev.n_tracks):
        qop = float(ev.trk_qop[t])
        xtol = 150.0 + 2000.0 * abs(qop)
        for l in range(NL):
            xmin, xc, xmax = (float(v) for v in o["wx"][t, l])
            tol = 2e-3 + 1e-6 * abs(xc)
            if l in X_LAYERS:
                right = xtol + (100.0 if qop > 0 else 0.0)
                left = xtol + (100.0 if qop < 0 else 0.0)
                assert abs((xmax - xc) - right) < tol, (t, l, xmax - xc, right)
                assert abs((xc - xmin) - left) < tol, (t, l, xc - xmin, left)
            else:
                assert abs((xmax - xc) - 800.0) < tol and abs((xc - xmin) - 800.0) < tol


def _brute_window(xs, xmin, xc, xmax, N):
    """R7/R8 by brute force over the sorted bucket (bucket-relative indices)."""
    inside = [i for i in range(len(xs)) if xmin <= xs[i] <= xmax]
    if not inside:
        lo = sum(1 for v in xs if v < xmin)
        return lo, lo
    lo, hi = inside[0], inside[-1] + 1
    if hi - lo <= N:
        return lo, hi
    c = sum(1 for v in xs if v < xc)
    c = min(max(c, lo), hi)
    first = min(max(c - N // 2, lo), hi - N)
    return first, first + N


def pin_window_search(lib=None):
    """Windows (incl. the symmetric cap at n_hits_window) equal a brute-force
    scan of the bucket, on a dense event where most windows are capped."""
    for ev in (ev_stress(), ev_nominal(1)):
        o = oracle.run(ev, W, debug=True, lib=lib)
        n_capped = 0
        for t in range(ev.n_tracks):
            zone = 1 if ev.trk_ty[t] >= 0 else 0
            for l in range(NL):
                b = 2 * l + zone
                h0, h1 = int(ev.hit_off[b]), int(ev.hit_off[b + 1])
                xs = ev.hit_x[h0:h1]
                xmin, xc, xmax = o["wx"][t, l]
                f, e = _brute_window(xs, xmin, xc, xmax, 32)
                got = (int(o["win"][t, l, 0]) - h0, int(o["win"][t, l, 1]) - h0)
                assert got == (f, e), (t, l, got, (f, e))
                n_capped += (e - f) == 32
        assert n_capped > 0


def pin_window_edges_closed(lib=None):
    """Hits exactly on x_min and x_max are inside the window; the next float
    outward is not (closed interval)."""
    ev = ev_single()
    o = oracle.run(ev, W, debug=True, lib=lib)
    t, l = 0, 0
    zone = 1 if ev.trk_ty[t] >= 0 else 0
    xmin, _, xmax = (f32(v) for v in o["wx"][t, l])
    b = 2 * l + zone
    h0, h1 = int(ev.hit_off[b]), int(ev.hit_off[b + 1])
    extra = np.array([np.nextafter(xmin, f32(-np.inf)), xmin, xmax, np.nextafter(xmax, f32(np.inf))],
                     np.float32)
    xs = np.sort(np.concatenate([ev.hit_x[h0:h1], extra]), kind="stable")
    # rebuild the event with the four extra hits in bucket b
    hx = np.concatenate([ev.hit_x[:h0], xs, ev.hit_x[h1:]])
    hz = np.concatenate([ev.hit_z[:h0], np.full(len(xs), ev.hit_z[h0] if h1 > h0 else W["z"][l], np.float32),
                         ev.hit_z[h1:]])
    hd = np.concatenate([ev.hit_dxdy[:h0], np.full(len(xs), W["dxdy"][l], np.float32), ev.hit_dxdy[h1:]])
    off = ev.hit_off.astype(np.int64).copy()
    off[b + 1:] += 4
    ev2 = lfgen.Events(**{**ev.__dict__, "hit_x": hx.astype(np.float32), "hit_z": hz.astype(np.float32),
                          "hit_dxdy": hd.astype(np.float32), "hit_off": off.astype(np.uint32),
                          "hit_pid": np.zeros(len(hx), np.int32)})
    o2 = oracle.run(ev2, W, debug=True, lib=lib)
    f, e = int(o2["win"][t, l, 0]) - h0, int(o2["win"][t, l, 1]) - h0
    win = xs[f:e]
    assert (win == xmin).any() and (win == xmax).any(), "edge hits must be inside"
    assert not (win < xmin).any() and not (win > xmax).any(), "hits beyond the edges must be outside"


def closed_form_triplet_residual(Ks=(1.00177513, 1.00142634)) -> tuple[float, float]:
    """Middle-hit residual per unit dtx for each seed set, derived in float64
    from the toy field and the K factors (the paper's by default; independent
    of the oracle): x1_true - [z1*t + (x0 - t*z0)*K] for the line t through
    (z0,x0),(z2,x2)."""
    z = W["z"]
    out = []
    for (l0, l1, l2), K in zip(SEED_SETS, Ks):
        # residual is linear in dtx and independent of tx: evaluate at dtx = 1, tx = 0
        x = [(z[i] - W["z_mag"]) + W["kappa"] * (z[i] - W["z_T"]) ** 2 for i in (l0, l1, l2)]
        t = (x[2] - x[0]) / (z[l2] - z[l0])
        x1e = z[l1] * t + (x[0] - t * z[l0]) * K
        out.append(x[1] - x1e)
    return out[0], out[1]


def pin_triplet_closed_form(lib=None):
    """chi2 of every true triplet of a noise-free track equals the closed-form
    sagitta residual (C_s * dtx)^2 within 1e-3 mm."""
    ev = ev_noise_free()
    o = oracle.run(ev, W, debug=True, lib=lib, params={"n_triplets": 64})
    cf = closed_form_triplet_residual()
    checked = 0
    for t in range(ev.n_tracks):
        p, q, tx, ty = particle(ev, t)
        dtx = 1.2 * q / p
        for s, layers in enumerate(SEED_SETS):
            hs = [truth_hit(ev, t, l) for l in layers]
            if min(hs) < 0:
                continue
            rows = np.nonzero((o["trip"][t, :, 0] == s) & (o["trip"][t, :, 1] == hs[0]) &
                              (o["trip"][t, :, 3] == hs[2]))[0]
            expect = abs(cf[s] * dtx)
            if expect ** 2 >= 8.0:
                assert len(rows) == 0 or o["trip"][t, rows[0], 2] != hs[1]
                continue
            assert len(rows) == 1, f"true doublet missing t={t} set={s}"
            got = math.sqrt(float(o["trip_chi2"][t, rows[0]]))
            if o["trip"][t, rows[0], 2] == hs[1]:
                assert abs(got - expect) < 1e-3, (t, s, got, expect)
                checked += 1
            else:
                assert got <= expect + 1e-3, "a farther middle hit was preferred"
    assert checked > 40


def pin_magnet_threshold(lib=None):
    """With the magnet tolerance pinned to 6 mm, a true doublet passes exactly
    when its closed-form offset at z_mag (8.0876*dtx for the first set,
    -20.594*dtx for the last; straight line through the two hits) is below 6 mm."""
    ev = ev_noise_free()
    z = W["z"]
    offs = []
    for (l0, _, l2) in SEED_SETS:
        x0 = (z[l0] - W["z_mag"]) + W["kappa"] * (z[l0] - W["z_T"]) ** 2
        x2 = (z[l2] - W["z_mag"]) + W["kappa"] * (z[l2] - W["z_T"]) ** 2
        t = (x2 - x0) / (z[l2] - z[l0])
        offs.append(x0 + t * (W["z_mag"] - z[l0]))
    ev = ev_noise_free(seed=12, p_max=10.0, n=80)
    o = oracle.run(ev, W, debug=True, lib=lib,
                   params={"n_triplets": 64, "magtol_min": 6.0, "magtol_max": 6.0, "p_charge_cut": 0.0})
    n_in = n_out = 0
    for t in range(ev.n_tracks):
        p, q, tx, ty = particle(ev, t)
        dtx = 1.2 * q / p
        for s, layers in enumerate(SEED_SETS):
            hs = [truth_hit(ev, t, l) for l in layers]
            if min(hs) < 0:
                continue
            off = abs(offs[s] * dtx)
            if abs(off - 6.0) < 0.05:
                continue
            present = ((o["trip"][t, :, 0] == s) & (o["trip"][t, :, 1] == hs[0]) &
                       (o["trip"][t, :, 3] == hs[2])).any()
            assert present == (off < 6.0), (t, s, off, present)
            n_in += present
            n_out += not present
    assert n_in > 10 and n_out > 5


def pin_charge_filter(lib=None):
    """Below 5 GeV the doublet must bend the way the upstream charge says:
    flipping the sign of q/p removes every true low-momentum triplet."""
    ev = ev_noise_free(seed=12, p_max=10.0, n=80)
    flipped = lfgen.Events(**{**ev.__dict__, "trk_qop": (-ev.trk_qop).astype(np.float32)})
    o = oracle.run(ev, W, debug=True, lib=lib, params={"n_triplets": 64})
    of = oracle.run(flipped, W, debug=True, lib=lib, params={"n_triplets": 64})
    n_low = 0
    for t in range(ev.n_tracks):
        p, q, tx, ty = particle(ev, t)
        if p >= 4.9:
            continue
        for s, layers in enumerate(SEED_SETS):
            hs = [truth_hit(ev, t, l) for l in layers]
            if min(hs) < 0:
                continue
            key = lambda oo: ((oo["trip"][t, :, 0] == s) & (oo["trip"][t, :, 1] == hs[0]) &
                              (oo["trip"][t, :, 3] == hs[2])).any()
            assert key(o), f"true low-p triplet missing t={t}"
            assert not key(of), f"wrong-charge doublet accepted t={t}"
            n_low += 1
    assert n_low > 10


def _bruteforce_triplets(ev, t, P, NT):
    """Exhaustive O(n0*n2*n1) triplet enumeration over whole buckets, float32,
    every triplet kept, fully sorted by (chi2, set, h0, h2)."""
    e = int(ev.track_event()[t])
    base = int(ev.hit_off[24 * e])
    X, Z = ev.hit_x, ev.hit_z
    qop = f32(ev.trk_qop[t])
    x_in, tx_in, ty_in = f32(ev.trk_x[t]), f32(ev.trk_tx[t]), f32(ev.trk_ty[t])
    p = f32(1.0) / abs(qop)
    zone = 1 if ty_in >= 0 else 0
    x_mag = x_in + tx_in * (f32(W["z_mag"]) - f32(W["z_in"]))
    out = []
    for s, (l0, l1, l2) in enumerate(SEED_SETS):
        K = f32(P["K_first"] if s == 0 else P["K_last"])
        b = [24 * e + 2 * l + zone for l in (l0, l1, l2)]
        r0 = range(int(ev.hit_off[b[0]]), int(ev.hit_off[b[0] + 1]))
        r1 = range(int(ev.hit_off[b[1]]), int(ev.hit_off[b[1] + 1]))
        r2 = range(int(ev.hit_off[b[2]]), int(ev.hit_off[b[2] + 1]))
        for i0 in r0:
            for i2 in r2:
                x0, z0, x2, z2 = X[i0], Z[i0], X[i2], Z[i2]
                txd = (x2 - x0) / (z2 - z0)
                if p < f32(P["p_charge_cut"]) and not ((txd - tx_in) * qop > 0):
                    continue
                xm = x0 + txd * (f32(W["z_mag"]) - z0)
                tol = f32(P["magtol_const"]) + f32(P["magtol_pscale"]) / p + f32(P["magtol_txscale"]) * abs(txd)
                tol = min(max(tol, f32(P["magtol_min"])), f32(P["magtol_max"]))
                if not abs(xm - x_mag) < tol:
                    continue
                x1e = f32(W["z"][l1]) * txd + (x0 - txd * z0) * K
                d = [abs(X[i1] - x1e) for i1 in r1]
                if not d:
                    continue
                k = int(np.argmin(d))          # first minimum = lowest index
                if d[k] * d[k] < f32(P["T_triplet"]):
                    out.append((float(d[k] * d[k]), s, i0 - base, r1[k] - base, i2 - base))
    out.sort(key=lambda r: (r[0], r[1], r[2], r[4]))
    return out[:NT], len(out)


def pin_bruteforce_triplets(lib=None):
    """With windows spanning whole buckets, the windowed search keeps exactly
    the top-n triplets of an exhaustive enumeration (tiny events)."""
    ev = ev_tiny()
    NT = 2
    big = {"xtol_const": 1e7, "uv_halfwidth": 1e7, "n_hits_window": 100000, "n_triplets": NT,
           "T_triplet": 40.0}
    P = oracle.default_params()
    P.update(big)
    o = oracle.run(ev, W, params=big, debug=True, lib=lib)
    n_cut = 0
    for t in range(ev.n_tracks):
        ref, n_all = _bruteforce_triplets(ev, t, P, NT)
        got = [(float(o["trip_chi2"][t, r]), *map(int, o["trip"][t, r])) for r in range(NT)
               if o["trip"][t, r, 0] >= 0]
        assert len(got) == len(ref), (t, got, ref)
        for g, r in zip(got, ref):
            assert g[1:] == r[1:] and f32(g[0]) == f32(r[0]), (t, g, r)
        assert int(o["counts"][t, 2]) == n_all
        n_cut += n_all > NT
    assert n_cut > 0


def _fit_truth(p, q, tx, ty):
    dtx = W["kick"] * q / p
    T = tx + dtx
    zr = oracle.Z_REF
    a = tx * W["z_mag"] + T * (zr - W["z_mag"]) + W["kappa"] * dtx * (zr - W["z_T"]) ** 2
    b = T + 2 * W["kappa"] * dtx * (zr - W["z_T"])
    c = W["kappa"] * dtx
    return a, b, c, ty * zr, ty


def pin_fit_noise_free(lib=None):
    """Noise-free tracks: (a, b, c) = (x, dx/dz, curvature) at z_ref, (y0, ty)
    = (ty*z_ref, ty), Q ~ 0, q/p_out = q/p_true, all 12 true hits."""
    ev = ev_noise_free()
    o = oracle.run(ev, W, lib=lib)
    n = 0
    for t in np.nonzero(o["found"])[0]:
        p, q, tx, ty = particle(ev, t)
        a, b, c, y0, tyt = _fit_truth(p, q, tx, ty)
        assert abs(o["a"][t] - a) < 2e-3
        assert abs(o["b"][t] - b) < 1e-6
        assert abs(o["c"][t] - c) < 1e-3 * abs(c) + 1e-12
        assert abs(o["y0"][t] - y0) < 2e-3
        assert abs(o["ty"][t] - tyt) < 1e-5
        assert abs(o["qop"][t] * p / q - 1.0) < 1e-5
        assert o["Q"][t] < 1e-6
        for l in range(NL):
            assert o["hit_idx"][t, l] == truth_hit(ev, t, l)
        n += 1
    assert n >= 35


def lstsq_fit(ev, t, hits, P, T_uv):
    """float64 least squares over a track's hits: returns predicted x per hit,
    fitted y per u/v hit, (a,b,c,y0,ty) and Q."""
    e = int(ev.track_event()[t])
    base = int(ev.hit_off[24 * e])
    zr = oracle.Z_REF
    y_in, ty_in = float(ev.trk_y[t]), float(ev.trk_ty[t])
    rows, xs, isuv, idx = [], [], [], []
    for l in range(NL):
        h = int(hits[l])
        if h < 0:
            continue
        g = base + h
        z = float(ev.hit_z[g])
        u = z - zr
        x = float(ev.hit_x[g])
        if l in UV_LAYERS:
            x += float(ev.hit_dxdy[g]) * (y_in + ty_in * (z - W["z_in"]))
        rows.append([1.0, u, u * u * (1.0 + W.get("dRatio", 0.0) * u)])
        xs.append(x)
        isuv.append(l in UV_LAYERS)
        idx.append(g)
    A = np.array(rows)
    sol, *_ = np.linalg.lstsq(A, np.array(xs), rcond=None)
    xf = A @ sol
    r = np.array(xs) - xf
    isuv = np.array(isuv)
    Qx = float(np.sum(r[~isuv] ** 2) / P["T_x"] + np.sum(r[isuv] ** 2) / T_uv)
    # y of each u/v hit where its fibre meets the fitted x
    gi = np.array(idx)[isuv]
    ys = (xf[isuv] - ev.hit_x[gi].astype(np.float64)) / ev.hit_dxdy[gi].astype(np.float64)
    B = np.stack([np.ones(isuv.sum()), A[isuv, 1]], 1)
    ysol, *_ = np.linalg.lstsq(B, ys, rcond=None)
    ry = ys - B @ ysol
    Qy = float(np.sum(ry ** 2) / P["T_y"])
    n, nuv = len(xs), int(isuv.sum())
    Q = (Qx / (n - 3) + Qy / (nuv - 2)) * P["C_nhits"][n - 9]
    return xf, A, sol, ysol, Q


def pin_fit_lstsq(lib=None):
    """With smeared hits the oracle's float32 fits agree with float64 least
    squares over the same hits: x at every hit within 1e-3 mm, ty within 1e-5,
    Q within 1e-2 relative (the stereo-corrected x of a u/v hit is rounded to
    float32, about 1e-4 mm, on residuals of a few 0.01 mm)."""
    ev = ev_nominal(1)
    P = oracle.default_params()
    o = oracle.run(ev, W, lib=lib)
    n = 0
    for t in np.nonzero(o["found"])[0][:150]:
        T_uv = max(2.0, 50.0 * (abs(float(ev.trk_tx[t])) + abs(float(ev.trk_ty[t]))))
        xf, A, sol, ysol, Q = lstsq_fit(ev, t, o["hit_idx"][t], P, T_uv)
        mine = np.array([float(o["a"][t]), float(o["b"][t]), float(o["c"][t])])
        assert np.max(np.abs(A @ mine - xf)) < 1e-3, (t, A @ mine - xf)
        y0 = float(o["y0"][t])
        assert abs(float(o["ty"][t]) - ysol[1]) < 1e-5, (t, o["ty"][t], ysol[1])
        assert abs(y0 - ysol[0]) < 5e-3, (t, y0, ysol[0])
        assert abs(float(o["Q"][t]) - Q) <= 1e-2 * Q + 1e-7, (t, o["Q"][t], Q)
        n += 1
    assert n > 100


def pin_y_fit_recovers_slope(lib=None):
    """The y fit measures ty from the stereo hits: with the input slope off by
    +3e-4, the fitted ty returns to the true slope."""
    ev = ev_noise_free(p_min=5.0)
    d = np.float32(3e-4)
    bent = lfgen.Events(**{**ev.__dict__, "trk_ty": (ev.trk_ty + d).astype(np.float32),
                           "trk_y": (ev.trk_y + d * np.float32(W["z_in"])).astype(np.float32)})
    o = oracle.run(bent, W, lib=lib)
    n = 0
    for t in np.nonzero(o["found"])[0]:
        p, q, tx, ty = particle(ev, t)
        assert abs(float(o["ty"][t]) - ty) < 2e-5, (t, o["ty"][t], ty)
        assert abs(float(o["y0"][t]) - ty * oracle.Z_REF) < 0.1
        n += 1
    assert n >= 30


def pin_physics_single(lib=None):
    """Single-event workload (p > 5 GeV): efficiency >= 90% and q/p resolution
    below 1% (the paper's headline physics claims), ghost rate <= 10%."""
    ev = ev_single()
    o = oracle.run(ev, W, lib=lib)
    ph = truth.physics(ev, o, p_min=5.0)
    assert ph["efficiency"] >= 0.9, ph
    assert ph["qop_resolution"] < 0.01, ph
    assert ph["ghost_rate"] <= 0.1, ph


def check_invariants(ev, o, NT=12):
    tev = ev.track_event()
    for t in np.nonzero(o["found"])[0]:
        hits = o["hit_idx"][t]
        n = int((hits >= 0).sum())
        assert n == int(o["n_hits"][t]) and 9 <= n <= 12
        for st in range(3):
            assert hits[4 * st + 1] >= 0 or hits[4 * st + 2] >= 0
        zone = 1 if ev.trk_ty[t] >= 0 else 0
        base = int(ev.hit_off[24 * tev[t]])
        for l in range(NL):
            h = int(hits[l])
            if h < 0:
                continue
            b = 24 * tev[t] + 2 * l + zone
            assert ev.hit_off[b] <= base + h < ev.hit_off[b + 1], "hit outside its layer/zone bucket"
            if "win" in o:
                assert o["win"][t, l, 0] <= h < o["win"][t, l, 1], "hit outside its window"
        assert o["Q"][t] < 0.5
        assert abs(float(o["ty"][t]) - float(ev.trk_ty[t])) <= 0.02 + 1e-6
    if "trip" in o:
        assert (o["trip"].shape[1] == NT)
        for t in range(ev.n_tracks):
            ch = o["trip_chi2"][t]
            ch = ch[~np.isnan(ch)]
            assert np.all(ch < 8.0) and np.all(np.diff(ch) >= 0)
            assert len(ch) == min(NT, int(o["counts"][t, 2]))


def pin_invariants(lib=None):
    """Structural invariants of every output, on nominal and stress events."""
    for ev in (ev_nominal(1), ev_stress()):
        o = oracle.run(ev, W, debug=True, lib=lib)
        assert o["found"].sum() > 0
        check_invariants(ev, o)


def pin_batch_independence(lib=None):
    """Each event's result is the same alone, in a batch, and in another order."""
    ev = ev_nominal(2)
    o = oracle.run(ev, W, lib=lib)
    rev = lfgen.select_events(ev, [1, 0])
    orv = oracle.run(rev, W, lib=lib)
    n0 = int(ev.trk_off[1])
    n1 = ev.n_tracks - n0
    for k in ("found", "hit_idx", "a", "b", "c", "y0", "ty", "qop", "Q"):
        assert np.array_equal(o[k][:n0], orv[k][n1:]), k
        assert np.array_equal(o[k][n0:], orv[k][:n1]), k


def make_event(bucket_hits: dict, tracks: list) -> "lfgen.Events":
    """A one-event batch from hand-placed hits: {(layer, zone): [x, ...]} and
    tracks [(x, y, tx, ty, qop), ...] (hits get the layer's z and stereo)."""
    xs, zs, ds, off = [], [], [], [0]
    for b in range(24):
        l, zone = divmod(b, 2)
        v = sorted(bucket_hits.get((l, zone), []))
        xs += v
        zs += [W["z"][l]] * len(v)
        ds += [W["dxdy"][l]] * len(v)
        off.append(len(xs))
    tr = np.array(tracks, np.float32).reshape(-1, 5)
    z = np.zeros(0, np.float32)
    return lfgen.Events(
        n_events=1, hit_off=np.array(off, np.uint32), hit_x=np.array(xs, np.float32),
        hit_z=np.array(zs, np.float32), hit_dxdy=np.array(ds, np.float32),
        hit_pid=np.full(len(xs), -1, np.int32), trk_off=np.array([0, len(tr)], np.uint32),
        trk_x=tr[:, 0].copy(), trk_y=tr[:, 1].copy(), trk_tx=tr[:, 2].copy(), trk_ty=tr[:, 3].copy(),
        trk_qop=tr[:, 4].copy(), trk_pid=np.full(len(tr), -1, np.int32), par_off=np.zeros(2, np.uint32),
        par_p=z, par_q=z, par_tx=z, par_ty=z, par_mask=np.zeros(0, np.uint16),
        par_has_track=np.zeros(0, np.uint8))


def pin_tie_breaks(lib=None):
    """Equal chi2 is ordered by (set, h0, h2) and the closest-hit search keeps
    the lowest index: a straight line at x = 100 with K = 1 gives chi2 = 0 for
    every combination, with duplicated hits in layers 0, 4 and 8."""
    hits = {(l, 1): [100.0] for l in X_LAYERS}
    for l in (0, 4, 8):
        hits[(l, 1)] = [100.0, 100.0]
    ev = make_event(hits, [(100.0, 270.0, 0.0, 0.1, 1.0 / 50.0)])
    o = oracle.run(ev, W, params={"K_first": 1.0, "K_last": 1.0, "n_triplets": 8}, debug=True, lib=lib)
    off = [int(v) for v in ev.hit_off]
    L = lambda l, k=0: off[2 * l + 1] + k
    expect = [(0, L(0), L(4), L(8)), (0, L(0), L(4), L(8, 1)), (0, L(0, 1), L(4), L(8)),
              (0, L(0, 1), L(4), L(8, 1)), (1, L(3), L(7), L(11))]
    got = [tuple(int(v) for v in o["trip"][0, r]) for r in range(8) if o["trip"][0, r, 0] >= 0]
    assert got == expect, (got, expect)
    assert np.all(o["trip_chi2"][0, :5] == 0.0)


def pin_extension_rule(lib=None):
    """Each candidate adds, per missing layer, the closest window hit to the
    triplet's parabola (float64, through the three seed hits) exactly when its
    squared distance is below T_x (x layers) or T_uv (u/v layers, hit moved
    along its fibre to the input track's y)."""
    # nominal tracks, and shallow tracks (|tx| + |ty| < 0.04, where the 2 mm^2
    # floor of T_uv applies) with coarse hit resolution
    shallow = lfgen.generate("single", seed=13, tx_max=0.02, ty_max=0.02, sigma_x=0.5, p_min=5.0)
    for ev in (ev_nominal(1), shallow):
        n_add, n_rej = _extension_rule(ev, lib)
        assert n_add > 100 and n_rej > 20, (n_add, n_rej)


def _extension_rule(ev, lib):
    o = oracle.run(ev, W, debug=True, lib=lib)
    X, Z, D = (a.astype(np.float64) for a in (ev.hit_x, ev.hit_z, ev.hit_dxdy))
    n_add = n_rej = 0
    for t in range(min(ev.n_tracks, 120)):
        T_uv = max(2.0, 50.0 * (abs(float(ev.trk_tx[t])) + abs(float(ev.trk_ty[t]))))
        for r in range(o["trip"].shape[1]):
            s, h0, h1, h2 = (int(v) for v in o["trip"][t, r])
            if s < 0:
                break
            u = Z[[h0, h1, h2]] - oracle.Z_REF
            coef = np.linalg.solve(np.stack([np.ones(3), u, u * u], 1), X[[h0, h1, h2]])
            cand = o["cand_hits"][t, r]
            for l in range(NL):
                if l in SEED_SETS[s]:
                    assert cand[l] == (h0, h1, h2)[SEED_SETS[s].index(l)]
                    continue
                ul = W["z"][l] - oracle.Z_REF
                pred = coef[0] + coef[1] * ul + coef[2] * ul * ul
                f, e = int(o["win"][t, l, 0]), int(o["win"][t, l, 1])
                if l in X_LAYERS:
                    d = np.abs(X[f:e] - pred)
                    T = 2.0
                else:
                    y = float(ev.trk_y[t]) + float(ev.trk_ty[t]) * (W["z"][l] - W["z_in"])
                    d = np.abs(X[f:e] + D[f:e] * y - pred)
                    T = T_uv
                dmin = float(d.min()) if e > f else np.inf
                h = int(cand[l])
                if h >= 0:
                    assert f <= h < e
                    assert d[h - f] <= dmin + 1e-4 and d[h - f] ** 2 < T + 1e-3, (t, r, l, d[h - f], T)
                    n_add += 1
                else:
                    assert dmin ** 2 >= T - 1e-3, (t, r, l, dmin, T)
                    n_rej += 1
    return n_add, n_rej


def pin_nine_hit_tracks(lib=None):
    """A noise-free particle with exactly 9 hits (a complete seed set and a
    u/v hit per station) is found with exactly those 9 hits."""
    ev = lfgen.generate("single", seed=14, sigma_x=0.0, qop_sigma=0.0, hit_eff=0.75, n_noise=0,
                        n_particles=80, p_min=5.0)
    o = oracle.run(ev, W, lib=lib)
    n = 0
    for t in range(ev.n_tracks):
        th = [truth_hit(ev, t, l) for l in range(NL)]
        if sum(h >= 0 for h in th) != 9:
            continue
        if not all(th[4 * s + 1] >= 0 or th[4 * s + 2] >= 0 for s in range(3)):
            continue
        if not any(all(th[l] >= 0 for l in st) for st in SEED_SETS):
            continue
        assert o["found"][t], t
        # another particle's hit may join within tolerance; the 9 own hits must be there
        assert all(o["hit_idx"][t][l] == th[l] for l in range(NL) if th[l] >= 0), t
        n += int(o["n_hits"][t]) == 9
    assert n >= 3, n


# ------------------------------------------------------------------ no-UT tuning
NU = {"velo_only": 1}   # the Forward no-UT column (oracle.make_params picks its defaults)
GOLDEN_NO_UT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_constants_no_ut.txt")


@functools.lru_cache(maxsize=None)
def ev_noise_free_wide(seed: int = 21):
    """Noise-free single-event geometry over a wide momentum range (1-60 GeV)."""
    return lfgen.generate("single", seed=seed, sigma_x=0.0, qop_sigma=0.0, hit_eff=1.0, n_noise=0,
                          p_min=1.0, p_max=60.0, n_particles=120)


def _bend(p: float, q: float, z: float) -> float:
    """x displacement of the toy-field trajectory from its upstream straight line (float64)."""
    dtx = W["kick"] * q / p
    return dtx * (z - W["z_mag"]) + W["kappa"] * dtx * (z - W["z_T"]) ** 2


def _pt(p: float, tx: float, ty: float) -> float:
    t2 = tx * tx + ty * ty
    return p * math.sqrt(t2 / (1.0 + t2))


def pin_no_ut_constants(lib=None):
    """The no-UT defaults equal the values the paper prints (Tab.Tol no-UT
    column, the polynomial coefficients, the No-UT tuning text)."""
    gold = {}
    with open(GOLDEN_NO_UT) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                head = line.split("|")[0].split()
                gold[head[0]] = float(head[1])
    p = oracle.make_params(NU, lib)
    for k, v in gold.items():
        got = p.noUT_c[int(k[6:])] if k.startswith("noUT_c") else getattr(p, k)
        assert got == f32(v), f"{k}: oracle no-UT default {got} != paper {v}"


def pin_no_ut_containment(lib=None):
    """VELO-only input on noise-free tracks: above both momentum thresholds
    (p > 5.5 GeV, pt > 1.1 GeV) the true hit of every layer up to z = 9200 mm
    lies inside the window of the track's own charge side, and a hit bent by
    more than the 5 mm overlap never lies inside the other side's window."""
    ev = ev_noise_free_wide()
    o = oracle.run(ev, W, NU, debug=True, lib=lib)
    base = ev.event_hit_base()
    n_in = n_out = 0
    for t in range(ev.n_tracks):
        p, q, tx, ty = particle(ev, t)
        own = 1 if q * W["polarity"] > 0 else 0
        wx_own = o["wx1"] if own else o["wx"]
        wx_other = o["wx"] if own else o["wx1"]
        for l in range(NL):
            h = truth_hit(ev, t, l)
            if h < 0:
                continue
            x = float(ev.hit_x[base[0] + h])
            if p > 5.5 and _pt(p, tx, ty) > 1.1 and W["z"][l] < 9200.0:
                assert wx_own[t, l, 0] <= x <= wx_own[t, l, 2], (t, l, p, x, wx_own[t, l])
                n_in += 1
            if abs(_bend(p, q, W["z"][l])) > 5.0 + 1.0:
                assert not (wx_other[t, l, 0] <= x <= wx_other[t, l, 2]), (t, l, p, x, wx_other[t, l])
                n_out += 1
    assert n_in > 200 and n_out > 500, (n_in, n_out)


def pin_no_ut_low_pt_excluded(lib=None):
    """The window assumes the tighter momentum threshold: a track with p < 30
    GeV and pt < 0.55 GeV bends at the first layer (1.2 GeV x 2626 mm / p)
    beyond the widest tolerance its slopes allow (below 5,100 mm GeV x pt / p),
    so none of its true hits is in a window and it is never found."""
    ev = ev_noise_free_wide()
    o = oracle.run(ev, W, NU, lib=lib)
    m = truth.match(ev, o)
    n = 0
    for t in range(ev.n_tracks):
        p, q, tx, ty = particle(ev, t)
        if p < 30.0 and _pt(p, tx, ty) < 0.55:
            assert not (m[t] >= 0 and m[t] == int(ev.trk_pid[t])), (t, p, _pt(p, tx, ty))
            n += 1
    assert n >= 3, n


def pin_no_ut_physics(lib=None):
    """VELO-only input: noise-free tracks above the thresholds (p > 5.5 GeV,
    pt > 1.1 GeV) are found (>= 90%) with the right charge and q/p within
    1e-4 from the pt-kick of the fit; on the single-event workload the same
    tracks are found with q/p resolution below 1%."""
    for ev, tol in ((ev_noise_free_wide(), 1e-4), (ev_single(), 0.01)):
        o = oracle.run(ev, W, NU, lib=lib)
        m = truth.match(ev, o)
        sel = found = 0
        rel = []
        for t in range(ev.n_tracks):
            if int(ev.trk_pid[t]) < 0:
                continue
            p, q, tx, ty = particle(ev, t)
            if not (p > 5.5 and _pt(p, tx, ty) > 1.1):
                continue
            sel += 1
            if m[t] == int(ev.trk_pid[t]):
                found += 1
                assert np.sign(o["qop"][t]) == np.sign(q), t
                rel.append(float(o["qop"][t]) * p / q - 1.0)
        assert sel >= 10 and found >= 0.9 * sel, (sel, found)
        assert math.sqrt(np.mean(np.square(rel))) < tol, (tol, rel)


def _bruteforce_no_ut(ev, t, P, NT):
    """Exhaustive triplets for VELO input when both windows of every layer
    span the whole bucket: each side's enumeration is the same list, so the
    kept triplets come in (side 0, side 1) copies of equal chi2."""
    e = int(ev.track_event()[t])
    base = int(ev.hit_off[24 * e])
    X, Z = ev.hit_x, ev.hit_z
    x_in, tx_in, ty_in = f32(ev.trk_x[t]), f32(ev.trk_tx[t]), f32(ev.trk_ty[t])
    zone = 1 if ty_in >= 0 else 0
    x_mag = x_in + tx_in * (f32(W["z_mag"]) - f32(W["z_in"]))
    one = []
    for s, (l0, l1, l2) in enumerate(SEED_SETS):
        K = f32(P["K_first"] if s == 0 else P["K_last"])
        b = [24 * e + 2 * l + zone for l in (l0, l1, l2)]
        r0 = range(int(ev.hit_off[b[0]]), int(ev.hit_off[b[0] + 1]))
        r1 = range(int(ev.hit_off[b[1]]), int(ev.hit_off[b[1] + 1]))
        r2 = range(int(ev.hit_off[b[2]]), int(ev.hit_off[b[2] + 1]))
        for i0 in r0:
            for i2 in r2:
                x0, z0, x2, z2 = X[i0], Z[i0], X[i2], Z[i2]
                txd = (x2 - x0) / (z2 - z0)
                xm = x0 + txd * (f32(W["z_mag"]) - z0)
                if not abs(xm - x_mag) < f32(P["magtol_max"]):
                    continue
                x1e = f32(W["z"][l1]) * txd + (x0 - txd * z0) * K
                d = [abs(X[i1] - x1e) for i1 in r1]
                if not d:
                    continue
                k = int(np.argmin(d))
                if d[k] * d[k] < f32(P["T_triplet"]):
                    one.append((float(d[k] * d[k]), s, i0 - base, r1[k] - base, i2 - base))
    out = [(c, sd, s, h0, h1, h2) for sd in (0, 1) for (c, s, h0, h1, h2) in one]
    out.sort(key=lambda r: (r[0], r[1], r[2], r[3], r[5]))
    return out[:NT], len(out)


def pin_no_ut_bruteforce(lib=None):
    """VELO input with both windows of every layer spanning the whole bucket:
    the windowed, per-side search keeps exactly the top-n of an exhaustive
    enumeration ordered by (chi2, side, set, h0, h2)."""
    ev = ev_tiny()
    NT = 3
    big = dict(NU, noUT_c=[1e9] * 8, noUT_overlap=1e7, uv_halfwidth=1e7, n_hits_window=64, n_triplets=NT,
               T_triplet=40.0, magtol_const=40.0, magtol_min=40.0, magtol_max=40.0)
    P = oracle.default_params(no_ut=True)
    P.update(big)
    o = oracle.run(ev, W, params=big, debug=True, lib=lib)
    n_cut = 0
    for t in range(ev.n_tracks):
        ref, n_all = _bruteforce_no_ut(ev, t, P, NT)
        got = []
        for r in range(NT):
            tr = o["trip"][t, r]
            if tr[0] >= 0:
                got.append((float(o["trip_chi2"][t, r]), int(tr[0]) // 2, int(tr[0]) % 2, int(tr[1]), int(tr[2]),
                            int(tr[3])))
        assert len(got) == len(ref), (t, got, ref)
        for g, r in zip(got, ref):
            assert g[1:] == r[1:] and f32(g[0]) == f32(r[0]), (t, g, r)
        assert int(o["counts"][t, 2]) == n_all
        n_cut += n_all > NT
    assert n_cut > 0


def pin_no_ut_window_formula(lib=None):
    """Consistency check (a float64 re-evaluation of the no-UT window
    equations, not an independent pin): assumed momentum, polynomial
    tolerance, both windows and their centres, every layer and track."""
    ev = ev_single()
    o = oracle.run(ev, W, NU, debug=True, lib=lib)
    c = [4824.3, 426.3, 7071.1, 12080.4, 14077.8, 13909.3, 9315.3, 3209.5]
    for t in range(ev.n_tracks):
        x_in, y_in, tx, ty = (float(v[t]) for v in (ev.trk_x, ev.trk_y, ev.trk_tx, ev.trk_ty))
        t2 = tx * tx + ty * ty
        s = math.sqrt(t2 / (1 + t2))
        p = max(5.0, 1.0 / s if s > 0 else 0.0)
        ip = 1.0 / p
        xtol = ip * (c[0] + tx * (c[1] + c[2] * tx) + ty * ty * (c[3] + tx * (c[4] + c[5] * tx))
                     + ip * (c[6] * tx + c[7] * ip))
        for l in range(NL):
            xe = x_in + tx * (W["z"][l] - W["z_in"])
            ye = y_in + ty * (W["z"][l] - W["z_in"])
            x0 = xe - W["dxdy"][l] * ye if l in UV_LAYERS else xe
            tol = 1200.0 if l in UV_LAYERS else xtol
            for wx, (lo, hi) in ((o["wx"], (x0 - tol, x0 + 5.0)), (o["wx1"], (x0 - 5.0, x0 + tol))):
                for k, v in enumerate((lo, 0.5 * (lo + hi), hi)):
                    assert abs(float(wx[t, l, k]) - v) < 2e-3 + 1e-6 * abs(v), (t, l, k, wx[t, l], v)


def pin_no_ut_invariants(lib=None):
    """VELO-only outputs: every found track's hits lie in one side's windows,
    9..12 hits with a u/v hit per station, Q < T_Q and |ty - ty_in| < 0.003."""
    for ev in (ev_nominal(1), ev_single()):
        o = oracle.run(ev, W, NU, debug=True, lib=lib)
        assert o["found"].sum() > 0
        for t in np.nonzero(o["found"])[0]:
            hits = o["hit_idx"][t]
            n = int((hits >= 0).sum())
            assert n == int(o["n_hits"][t]) and 9 <= n <= 12
            for st in range(3):
                assert hits[4 * st + 1] >= 0 or hits[4 * st + 2] >= 0
            sides = [all(w[t, l, 0] <= hits[l] < w[t, l, 1] for l in range(NL) if hits[l] >= 0)
                     for w in (o["win"], o["win1"])]
            assert any(sides), t
            assert o["Q"][t] < 0.5
            assert abs(float(o["ty"][t]) - float(ev.trk_ty[t])) < 0.003 + 1e-7


NO_UT_PINS = [pin_no_ut_constants, pin_no_ut_containment, pin_no_ut_low_pt_excluded, pin_no_ut_physics,
              pin_no_ut_bruteforce, pin_no_ut_window_formula, pin_no_ut_invariants]


# ------------------------------------------------------------------ paper-form field
# Events in the "paper" field (sqrt-normalised pt-kick, an integrated field
# that depends on the entry slopes and on the bending, a falling B_y tail)
# and in the "kick" field (the same kick with a constant integral, for which
# F = 1.2 GeV is exact); the method reads the fitted F table.
W_PAPER = lfgen.world("paper")
F_CONST = [lfgen.KICK] + [0.0] * 49
W_KICK = lfgen.world("kick", F_coef=F_CONST)


@functools.lru_cache(maxsize=None)
def ev_field_noise_free(field: str, seed: int = 11, n: int = 120):
    return lfgen.generate("single", field=field, seed=seed, sigma_x=0.0, qop_sigma=0.0, hit_eff=1.0,
                          n_noise=0, p_min=1.5, p_max=50.0, n_particles=n)


def _centre_errors(ev, o):
    """(p, |window centre - exact hit x|) of every truth hit; asserts every
    truth hit lies inside its window."""
    out = []
    for t in range(ev.n_tracks):
        p = particle(ev, t)[0]
        base = int(ev.hit_off[24 * int(ev.track_event()[t])])
        for l in range(NL):
            h = truth_hit(ev, t, l)
            if h < 0:
                continue
            assert o["win"][t, l, 0] <= h < o["win"][t, l, 1], f"truth hit outside window t={t} l={l}"
            out.append((p, abs(float(o["wx"][t, l, 1]) - float(ev.hit_x[base + h]))))
    return np.array(out)


def pin_kick_extrapolation_exact(lib=None):
    """Constant integrated field: the pt-kick equation with F = 1.2 GeV is
    the world's exact kick, so with exact q/p every window centre sits on
    the exact hit position (x layers: x; u/v: x - dxdy*y), including the
    falling-tail cubic term, at every momentum."""
    ev = ev_field_noise_free("kick")
    o = oracle.run(ev, W_KICK, debug=True, lib=lib)
    e = _centre_errors(ev, o)
    assert len(e) > 1000 and (e[:, 0] < 3.0).sum() > 30
    assert e[:, 1].max() <= 2e-3, f"window centre off the exact hit by {e[:, 1].max()} mm"


def pin_kick_momentum_exact(lib=None):
    """Constant integrated field, noise-free tracks: the pt-kick equation
    returns the true q/p from the fitted slope after the magnet."""
    ev = ev_field_noise_free("kick")
    o = oracle.run(ev, W_KICK, lib=lib)
    n = 0
    for t in np.nonzero(o["found"])[0]:
        p, q, tx, ty = particle(ev, t)
        assert all(o["hit_idx"][t, l] == truth_hit(ev, t, l) for l in range(NL))
        assert abs(o["qop"][t] * p / q - 1.0) < 2e-5, (t, p, o["qop"][t] * p / q)
        n += 1
    assert n >= 90


def pin_paper_extrapolation(lib=None):
    """Paper field, exact q/p: the window centres follow the exact hits to
    within what the calibrated F and two refinements of the kick allow
    (below 3 GeV, where the slope change is largest, tens of mm against a
    half-width of 817 mm; above 5 GeV a fraction of a mm), and every truth
    hit is inside its window."""
    ev = ev_field_noise_free("paper")
    o = oracle.run(ev, W_PAPER, debug=True, lib=lib)
    e = _centre_errors(ev, o)
    for lo, hi, tol in ((1.5, 3.0, 40.0), (3.0, 5.0, 0.6), (5.0, 1e9, 0.2)):
        m = (e[:, 0] >= lo) & (e[:, 0] < hi)
        assert m.sum() > 30
        assert e[m, 1].max() <= tol, (lo, hi, e[m, 1].max())


def pin_paper_momentum(lib=None):
    """Paper field, noise-free tracks whose hits are all the particle's: the
    q/p from the pt-kick equation with the fitted F matches the truth to
    the calibration's accuracy (the table's largest relative residual over
    its acceptance sample is 1.6e-3), and typically to a few 1e-4."""
    ev = ev_field_noise_free("paper")
    o = oracle.run(ev, W_PAPER, lib=lib)
    rel = []
    for t in np.nonzero(o["found"])[0]:
        if not all(o["hit_idx"][t, l] == truth_hit(ev, t, l) for l in range(NL)):
            continue
        p, q, tx, ty = particle(ev, t)
        rel.append(float(o["qop"][t]) * p / q - 1.0)
    rel = np.abs(np.array(rel))
    assert len(rel) >= 90
    assert rel.max() <= 2e-3, rel.max()
    assert np.median(rel) <= 3e-4, np.median(rel)


def pin_paper_no_kick_solution(lib=None):
    """A kick that no slope can carry (|s_f| >= 1: a track too soft for the
    field) gives no windows and no track; a slightly harder one is searched."""
    ev = ev_field_noise_free("paper")
    import copy
    bad = copy.deepcopy(ev)
    t_s = np.arange(0, ev.n_tracks, 3)
    tx = bad.trk_tx[t_s].astype(np.float64)
    # q/p that moves s by 1.5 (F is about 1.2 GeV) in the direction of tx
    bad.trk_qop[t_s] = np.where(tx >= 0, 1.25, -1.25).astype(np.float32)
    o = oracle.run(bad, W_PAPER, debug=True, lib=lib)
    assert not o["found"][t_s].any()
    assert (o["win"][t_s] == 0).all()
    # the other tracks are unaffected
    o0 = oracle.run(ev, W_PAPER, lib=lib)
    keep = np.setdiff1d(np.arange(ev.n_tracks), t_s)
    assert np.array_equal(o["found"][keep], o0["found"][keep])
    assert np.array_equal(o["qop"][keep], o0["qop"][keep])
    # a soft track whose kick still has a solution keeps its windows
    soft = copy.deepcopy(ev)
    soft.trk_qop[t_s] = np.where(tx >= 0, -0.45, 0.45).astype(np.float32)
    o = oracle.run(soft, W_PAPER, debug=True, lib=lib)
    assert (o["win"][t_s, :, 1] > o["win"][t_s, :, 0]).any(axis=1).mean() > 0.5


def pin_paper_physics(lib=None):
    """Nominal-shape events in the paper field: efficiency >= 95%, ghost
    rate <= 2%, q/p resolution below 1% with the fitted F, and at least three
    times worse when F is replaced by its constant -- the dSlope dependence
    of the parametrisation carries the resolution."""
    ev = lfgen.generate("nominal", field="paper", n_events=2)
    o = oracle.run(ev, W_PAPER, lib=lib)
    ph = truth.physics(ev, o)
    assert ph["efficiency"] >= 0.95 and ph["ghost_rate"] <= 0.02, ph
    assert ph["qop_resolution"] < 0.01, ph
    oc = oracle.run(ev, dict(W_PAPER, F_coef=F_CONST), lib=lib)
    assert truth.physics(ev, oc)["qop_resolution"] > 3.0 * ph["qop_resolution"]


# exponents (k, m) of tx^k ty^m for the columns of F_coef: even rows use all
# ten, odd rows the first six times one more power of tx
_F_EXPONENTS = ((0, 0), (2, 0), (0, 2), (4, 0), (2, 2), (0, 4), (6, 0), (4, 2), (2, 4), (0, 6))


def pin_F_single_terms(lib=None):
    """Constant integrated field (s_f - s_i = 1.2 q/p exactly) read with a
    table of the constant 1.2 plus one extra term w * tx^k ty^m dSlope^i:
    then the method's q/p is the truth times 1.2 / (1.2 + w tx^k ty^m d^i),
    with d the true slope change -- for every term of the table in turn (the
    weight w sized for a change of at most 3% of F)."""
    ev = ev_field_noise_free("kick")
    tev = ev.track_event()
    g = ev.par_off[tev].astype(np.int64) + ev.trk_pid.astype(np.int64)
    p, q = ev.par_p[g].astype(np.float64), ev.par_q[g].astype(np.float64)
    tx, ty = ev.trk_tx.astype(np.float64), ev.trk_ty.astype(np.float64)
    d, bl, fwd = lfgen.kick(tx, ty, q / p, "kick")
    for i in range(5):
        for j in range(10 if i % 2 == 0 else 6):
            k, m = _F_EXPONENTS[j]
            k += i % 2
            term = tx ** k * ty ** m * d ** i
            if not np.any(term):
                continue
            w = 0.03 * lfgen.KICK / np.abs(term).max()
            coef = list(F_CONST)
            coef[10 * i + j] += float(np.float32(w))
            w = float(np.float32(w))
            o = oracle.run(ev, dict(W_KICK, F_coef=coef), lib=lib)
            f = np.nonzero(o["found"])[0]
            assert len(f) >= 80, (i, j, len(f))
            pure = [t for t in f if all(o["hit_idx"][t, l] == truth_hit(ev, t, l) for l in range(NL))]
            assert len(pure) >= 80, (i, j, len(pure))
            pure = np.array(pure)
            want = (q[pure] / p[pure]) * lfgen.KICK / (lfgen.KICK + w * term[pure])
            err = np.abs(o["qop"][pure].astype(np.float64) / want - 1.0)
            assert err.max() < 3e-5, (i, j, err.max())


PAPER_FIELD_PINS = [pin_kick_extrapolation_exact, pin_kick_momentum_exact, pin_paper_extrapolation,
                    pin_paper_momentum, pin_paper_no_kick_solution, pin_paper_physics, pin_F_single_terms]


# ------------------------------------------------------------------ binary16 seeding
FP16 = {"seed_fp16": 1}


def pin_h16_is_ieee_half(lib=None):
    """The oracle's binary16 rounding equals numpy's float16 conversion (IEEE
    754 round to nearest even) on normal, subnormal, tie and overflowing
    values."""
    rng = np.random.default_rng(5)
    vals = np.concatenate([
        rng.uniform(-3000, 3000, 4000), rng.uniform(-1, 1, 2000) * 10.0 ** rng.integers(-9, 5, 2000),
        (np.arange(-2048, 2048) + 0.5) * 2.0 ** rng.integers(-24, 6, 4096),     # ties at many scales
        np.array([65503.0, 65504.0, 65519.0, 65520.0, 70000.0, -65520.0, 6.1e-5, 6.0e-5, 2.0 ** -25,
                  2.0 ** -25 * 3, 0.0, -0.0])]).astype(np.float32)
    got = np.array([oracle.h16(v, lib) for v in vals], np.float32)
    with np.errstate(over="ignore"):
        want = vals.astype(np.float16).astype(np.float32)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert same.all(), (vals[~same][:5], got[~same][:5], want[~same][:5])
    assert np.array_equal(np.signbit(got), np.signbit(want))


def pin_fp16_true_triplets(lib=None):
    """binary16 seeding, noise-free tracks: every true triplet is accepted with
    a chi2 whose root matches the closed-form sagitta residual to the binary16
    accuracy of the window-relative coordinates (0.5 mm), with the paper's K
    and with K = 1.01, which makes the residuals a few mm (chi2 cut 100)."""
    ev = ev_noise_free()
    for Ks, extra in (((1.00177513, 1.00142634), {}),
                      ((1.01, 1.01), {"K_first": 1.01, "K_last": 1.01, "T_triplet": 100.0})):
        o = oracle.run(ev, W, debug=True, lib=lib, params=dict(FP16, n_triplets=64, **extra))
        cf = closed_form_triplet_residual(Ks)
        T = extra.get("T_triplet", 8.0)
        checked = 0
        for t in range(ev.n_tracks):
            p, q, tx, ty = particle(ev, t)
            dtx = 1.2 * q / p
            for s, layers in enumerate(SEED_SETS):
                hs = [truth_hit(ev, t, l) for l in layers]
                if min(hs) < 0:
                    continue
                expect = abs(cf[s] * dtx)
                if (expect + 0.5) ** 2 >= T:
                    continue
                rows = np.nonzero((o["trip"][t, :, 0] == s) & (o["trip"][t, :, 1] == hs[0]) &
                                  (o["trip"][t, :, 3] == hs[2]))[0]
                assert len(rows) == 1, f"true doublet missing t={t} set={s} K={Ks}"
                got = math.sqrt(float(o["trip_chi2"][t, rows[0]]))
                if o["trip"][t, rows[0], 2] == hs[1]:
                    assert abs(got - expect) < 0.5, (t, s, got, expect, Ks)
                    checked += 1
        assert checked > 40, checked


def pin_fp16_physics(lib=None):
    """binary16 seeding changes only tracks whose seeding decisions sit within
    the half-precision error of a cut: on nominal events at least 98% of the
    outputs equal the binary32 ones and efficiency and ghost rate move by less
    than 0.5%."""
    ev = ev_nominal(4)
    o32 = oracle.run(ev, W, lib=lib)
    o16 = oracle.run(ev, W, FP16, lib=lib)
    same = (o32["found"] == o16["found"]) & np.all(o32["hit_idx"] == o16["hit_idx"], axis=1)
    assert same.mean() >= 0.98, same.mean()
    a, b = truth.physics(ev, o32, p_min=5.0), truth.physics(ev, o16, p_min=5.0)
    assert abs(a["efficiency"] - b["efficiency"]) < 0.005 and abs(a["ghost_rate"] - b["ghost_rate"]) < 0.005
    assert b["efficiency"] > 0.95


def pin_fp16_mixed_windows_stay_binary32(lib=None):
    """A seed set whose first- or last-layer window has hits at different z is
    seeded in binary32: with every hit's z jittered the binary16 option
    changes nothing."""
    ev = ev_nominal(2)
    rng = np.random.default_rng(9)
    hz = (ev.hit_z + rng.uniform(-20.0, 20.0, ev.n_hits)).astype(np.float32)
    ev = lfgen.Events(**{**ev.__dict__, "hit_z": hz})
    o32 = oracle.run(ev, W, lib=lib)
    o16 = oracle.run(ev, W, FP16, lib=lib)
    for k in ("found", "hit_idx", "qop", "Q"):
        assert np.array_equal(o32[k], o16[k]), k


FP16_PINS = [pin_h16_is_ieee_half, pin_fp16_true_triplets, pin_fp16_physics, pin_fp16_mixed_windows_stay_binary32]

ALL_PINS = [pin_constants, pin_extrapolation_noise_free, pin_window_bounds, pin_window_search,
            pin_window_edges_closed, pin_triplet_closed_form, pin_magnet_threshold,
            pin_charge_filter, pin_bruteforce_triplets, pin_fit_noise_free, pin_fit_lstsq,
            pin_y_fit_recovers_slope, pin_physics_single, pin_invariants, pin_batch_independence,
            pin_tie_breaks, pin_extension_rule, pin_nine_hit_tracks] + NO_UT_PINS + PAPER_FIELD_PINS + FP16_PINS

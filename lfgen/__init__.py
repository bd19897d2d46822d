"""Seeded synthetic SciFi events with truth (input generator only).

Both the CPU oracle and the GPU library read the arrays produced here; this
module holds none of the track-finding arithmetic.  The five workload presets
copy the shapes of the paper's samples (about 400 hits per SciFi layer,
"Defining the search windows"; interaction-count scaling, "Performance"),
not their data, which is LHCb simulation and is not available here.

Usage::

    ev = lfgen.generate("nominal", n_events=10)
    ev.hit_x, ev.hit_off, ev.trk_qop, ...
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lfgen.c")
_LIB = os.path.join(_HERE, "liblfgen.so")

NL = 12
# SciFi layer z positions (mm): three stations of x-u-v-x.
LAYER_Z = (7826.0, 7896.0, 7966.0, 8036.0, 8508.0, 8578.0, 8648.0, 8718.0,
           9193.0, 9263.0, 9333.0, 9403.0)
STEREO_DEG = (0.0, 5.0, -5.0, 0.0) * 3
LAYER_DXDY = tuple(math.tan(math.radians(a)) for a in STEREO_DEG)
X_LAYERS = (0, 3, 4, 7, 8, 11)
UV_LAYERS = (1, 2, 5, 6, 9, 10)

# Toy field: kick at Z_MAG changing the slope by dtx; residual curvature
# KAPPA * dtx * (z - Z_T)^2 (1 + dRatio (z - Z_T)) after the magnet.
# Upstream states at Z_UP.  Two kicks (lfgen.c): the linear toy kick
# dtx = KICK * q/p with a constant B_y tail ("toy"), and the sqrt-normalised
# pt-kick with an integrated field that depends on the entry slopes and on
# the bending, and a linearly falling tail ("paper").
Z_UP = 2700.0
Z_MAG = 5200.0
Z_T = 8500.0
KICK = 1.2
KAPPA = 2e-5
# Reference plane of the x(z) model; the paper fields expand their falling
# tail about it (z_T = Z_REF), so the model of the method is exact for them.
Z_REF = 8520.0
FIELDS = {
    "toy": dict(field_form=0, dRatio=0.0, bl0=KICK, bl_tx2=0.0, bl_ty2=0.0, bl_q2=0.0),
    "paper": dict(field_form=1, dRatio=-2.0e-4, bl0=KICK, bl_tx2=-0.25, bl_ty2=-0.6, bl_q2=-0.15,
                  z_T=Z_REF),
    # the sqrt-normalised pt-kick with a constant integrated field: a paper
    # field whose momentum parametrisation is exactly F = KICK
    "kick": dict(field_form=1, dRatio=-2.0e-4, bl0=KICK, bl_tx2=0.0, bl_ty2=0.0, bl_q2=0.0, z_T=Z_REF),
}


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("first_event", ctypes.c_int32),
        ("n_events", ctypes.c_int32),
        ("n_particles", ctypes.c_int32),
        ("particles_per_int", ctypes.c_int32),
        ("mu_int", ctypes.c_double),
        ("p_min", ctypes.c_double), ("p_max", ctypes.c_double),
        ("pt_min", ctypes.c_double),
        ("tx_max", ctypes.c_double), ("ty_max", ctypes.c_double),
        ("qop_sigma", ctypes.c_double),
        ("n_true_tracks", ctypes.c_int32),
        ("n_fake_tracks", ctypes.c_int32),
        ("true_track_frac", ctypes.c_double),
        ("fake_ratio", ctypes.c_double),
        ("n_noise", ctypes.c_int32),
        ("noise_frac", ctypes.c_double),
        ("hit_eff", ctypes.c_double), ("sigma_x", ctypes.c_double),
        ("x_acc", ctypes.c_double), ("y_acc", ctypes.c_double),
        ("z_up", ctypes.c_double), ("z_mag", ctypes.c_double), ("z_T", ctypes.c_double),
        ("kick", ctypes.c_double), ("kappa", ctypes.c_double),
        ("z", ctypes.c_double * NL), ("dxdy", ctypes.c_double * NL),
        ("field_form", ctypes.c_int32), ("dRatio", ctypes.c_double),
        ("bl0", ctypes.c_double), ("bl_tx2", ctypes.c_double), ("bl_ty2", ctypes.c_double),
        ("bl_q2", ctypes.c_double),
    ]


_BASE = dict(
    seed=0, first_event=0, n_events=1, n_particles=40, particles_per_int=50, mu_int=0.0,
    p_min=5.0, p_max=50.0, pt_min=0.0, tx_max=0.3, ty_max=0.25, qop_sigma=0.15,
    n_true_tracks=-1, n_fake_tracks=0, true_track_frac=170.0 / 350.0, fake_ratio=15.0 / 85.0,
    n_noise=100, noise_frac=0.0, hit_eff=0.98, sigma_x=0.08, x_acc=3000.0, y_acc=2500.0,
)

# The five workloads.  Seeds: 0 for the single event, 2..5 for the others.
PRESETS = {
    # single event: 40 particles, p 5-50 GeV, 100 noise hits, every particle has a track
    "single": dict(seed=0, n_events=1, n_particles=40, p_min=5.0, p_max=50.0, n_noise=100,
                   n_true_tracks=-1, n_fake_tracks=0),
    # nominal: 1,000 events of 350 particles (p 2-100, pt > 0.3), 170 true + 30 fake
    # tracks, 1,500 noise hits (about 5.5k hits per event)
    "nominal": dict(seed=2, n_events=1000, n_particles=350, p_min=2.0, p_max=100.0, pt_min=0.3,
                    n_noise=1500, n_true_tracks=170, n_fake_tracks=30),
    # uneven: 20,000 events, Poisson(7.6) interactions x 50 particles, noise 25% of truth hits,
    # fakes 15% of input tracks
    "uneven": dict(seed=3, n_events=20000, mu_int=7.6, particles_per_int=50, p_min=2.0,
                   p_max=100.0, pt_min=0.3, n_noise=0, noise_frac=0.25,
                   true_track_frac=170.0 / 350.0, fake_ratio=15.0 / 85.0),
    # serving stream: nominal event shape, drawn on the fly
    "serving": dict(seed=4, n_events=200000, n_particles=350, p_min=2.0, p_max=100.0, pt_min=0.3,
                    n_noise=1500, n_true_tracks=170, n_fake_tracks=30),
    # stress: 700 low-momentum particles (1.5-10 GeV), q/p smeared 30%, noise 5x truth hits,
    # 340 true + 146 fake tracks (30% fakes)
    "stress": dict(seed=5, n_events=5000, n_particles=700, p_min=1.5, p_max=10.0, pt_min=0.3,
                   qop_sigma=0.30, n_noise=0, noise_frac=5.0, n_true_tracks=340, n_fake_tracks=146),
}


@dataclass
class Events:
    """A batch of events in the ragged SoA layout both consumers read.

    Hits are bucket-major: bucket b = 24*event + 2*layer + zone (zone 1 = y > 0),
    x non-decreasing inside a bucket; ``hit_off[b] .. hit_off[b+1]`` is bucket b.
    Track states (x, y, tx, ty, q/p) are at z = Z_UP.  ``*_pid`` are truth
    particle indices local to the event (-1 = noise hit / fake track).
    """
    n_events: int
    hit_off: np.ndarray
    hit_x: np.ndarray
    hit_z: np.ndarray
    hit_dxdy: np.ndarray
    hit_pid: np.ndarray
    trk_off: np.ndarray
    trk_x: np.ndarray
    trk_y: np.ndarray
    trk_tx: np.ndarray
    trk_ty: np.ndarray
    trk_qop: np.ndarray
    trk_pid: np.ndarray
    par_off: np.ndarray
    par_p: np.ndarray
    par_q: np.ndarray
    par_tx: np.ndarray
    par_ty: np.ndarray
    par_mask: np.ndarray
    par_has_track: np.ndarray

    @property
    def n_hits(self) -> int:
        return int(self.hit_off[-1])

    @property
    def n_tracks(self) -> int:
        return int(self.trk_off[-1])

    def event_hit_base(self) -> np.ndarray:
        """First global hit index of each event."""
        return self.hit_off[0:24 * self.n_events:24] if self.n_events else np.zeros(0, np.uint32)

    def track_event(self) -> np.ndarray:
        """Event index of every input track."""
        counts = np.diff(self.trk_off.astype(np.int64))
        return np.repeat(np.arange(self.n_events, dtype=np.int64), counts)


def build(force: bool = False) -> str:
    """Compile the generator into a shared library next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.lfgen_run.restype = ctypes.c_void_p
        lib.lfgen_run.argtypes = [ctypes.POINTER(_Cfg)]
        lib.lfgen_free.argtypes = [ctypes.c_void_p]
        lib.lfgen_sizes.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_uint64)] * 4
        lib.lfgen_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 19
        lib.lfgen_kick_many.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int64] + [ctypes.c_void_p] * 6
        _lib = lib
    return _lib


def config(preset: str = "single", **overrides) -> dict:
    """The generator settings of a preset, with overrides applied."""
    if preset not in PRESETS:
        raise KeyError(f"unknown preset {preset!r}; have {sorted(PRESETS)}")
    c = dict(_BASE)
    c.update(PRESETS[preset])
    c.update(overrides)
    return c


def _make_cfg(c: dict, field: str) -> _Cfg:
    if field not in FIELDS:
        raise KeyError(f"unknown field {field!r}; have {sorted(FIELDS)}")
    cfg = _Cfg()
    for k, v in c.items():
        if k in ("z", "dxdy"):
            continue
        setattr(cfg, k, v)
    cfg.z_up, cfg.z_mag, cfg.z_T, cfg.kick, cfg.kappa = Z_UP, Z_MAG, Z_T, KICK, KAPPA
    for k, v in FIELDS[field].items():
        setattr(cfg, k, v)
    zs = c.get("z", LAYER_Z)
    ds = c.get("dxdy", LAYER_DXDY)
    for i in range(NL):
        cfg.z[i] = zs[i]
        cfg.dxdy[i] = ds[i]
    return cfg


def generate(preset: str = "single", field: str = "toy", **overrides) -> Events:
    """Generate events of a preset (``n_events``/``first_event``/... may be
    overridden) in the field ``field`` ("toy" or "paper")."""
    c = config(preset, **overrides)
    cfg = _make_cfg(c, field)
    lib = _load()
    h = lib.lfgen_run(ctypes.byref(cfg))
    if not h:
        raise ValueError("lfgen: bad configuration or out of memory")
    try:
        E, H, T, P = (ctypes.c_uint64() for _ in range(4))
        lib.lfgen_sizes(h, ctypes.byref(E), ctypes.byref(H), ctypes.byref(T), ctypes.byref(P))
        E, H, T, P = E.value, H.value, T.value, P.value
        a = dict(
            hit_off=np.zeros(24 * E + 1, np.uint32), hit_x=np.zeros(H, np.float32),
            hit_z=np.zeros(H, np.float32), hit_dxdy=np.zeros(H, np.float32),
            hit_pid=np.zeros(H, np.int32),
            trk_off=np.zeros(E + 1, np.uint32), trk_x=np.zeros(T, np.float32),
            trk_y=np.zeros(T, np.float32), trk_tx=np.zeros(T, np.float32),
            trk_ty=np.zeros(T, np.float32), trk_qop=np.zeros(T, np.float32),
            trk_pid=np.zeros(T, np.int32),
            par_off=np.zeros(E + 1, np.uint32), par_p=np.zeros(P, np.float32),
            par_q=np.zeros(P, np.float32), par_tx=np.zeros(P, np.float32),
            par_ty=np.zeros(P, np.float32), par_mask=np.zeros(P, np.uint16),
            par_has_track=np.zeros(P, np.uint8),
        )
        order = ["hit_off", "hit_x", "hit_z", "hit_dxdy", "hit_pid", "trk_off", "trk_x", "trk_y",
                 "trk_tx", "trk_ty", "trk_qop", "trk_pid", "par_off", "par_p", "par_q", "par_tx",
                 "par_ty", "par_mask", "par_has_track"]
        lib.lfgen_copy(h, *[a[k].ctypes.data_as(ctypes.c_void_p) for k in order])
    finally:
        lib.lfgen_free(h)
    return Events(n_events=int(E), **a)


def concat(parts: list[Events]) -> Events:
    """Concatenate batches into one (offsets rebased)."""
    if not parts:
        raise ValueError("nothing to concatenate")
    out = {}
    hb = tb = pb = 0
    hit_off, trk_off, par_off = [], [], []
    for i, e in enumerate(parts):
        ho = e.hit_off.astype(np.int64) + hb
        to = e.trk_off.astype(np.int64) + tb
        po = e.par_off.astype(np.int64) + pb
        last = i == len(parts) - 1
        hit_off.append(ho if last else ho[:-1])
        trk_off.append(to if last else to[:-1])
        par_off.append(po if last else po[:-1])
        hb, tb, pb = int(ho[-1]), int(to[-1]), int(po[-1])
    out["hit_off"] = np.concatenate(hit_off).astype(np.uint32)
    out["trk_off"] = np.concatenate(trk_off).astype(np.uint32)
    out["par_off"] = np.concatenate(par_off).astype(np.uint32)
    for k in ("hit_x", "hit_z", "hit_dxdy", "hit_pid", "trk_x", "trk_y", "trk_tx", "trk_ty",
              "trk_qop", "trk_pid", "par_p", "par_q", "par_tx", "par_ty", "par_mask",
              "par_has_track"):
        out[k] = np.concatenate([getattr(e, k) for e in parts])
    return Events(n_events=sum(e.n_events for e in parts), **out)


def select_events(ev: Events, idx) -> Events:
    """A new batch holding events ``idx`` of ``ev`` (in that order)."""
    parts = []
    for e in np.asarray(idx, dtype=np.int64):
        h0, h1 = int(ev.hit_off[24 * e]), int(ev.hit_off[24 * e + 24])
        t0, t1 = int(ev.trk_off[e]), int(ev.trk_off[e + 1])
        p0, p1 = int(ev.par_off[e]), int(ev.par_off[e + 1])
        parts.append(Events(
            n_events=1,
            hit_off=(ev.hit_off[24 * e:24 * e + 25].astype(np.int64) - h0).astype(np.uint32),
            hit_x=ev.hit_x[h0:h1], hit_z=ev.hit_z[h0:h1], hit_dxdy=ev.hit_dxdy[h0:h1],
            hit_pid=ev.hit_pid[h0:h1],
            trk_off=np.array([0, t1 - t0], np.uint32),
            trk_x=ev.trk_x[t0:t1], trk_y=ev.trk_y[t0:t1], trk_tx=ev.trk_tx[t0:t1],
            trk_ty=ev.trk_ty[t0:t1], trk_qop=ev.trk_qop[t0:t1], trk_pid=ev.trk_pid[t0:t1],
            par_off=np.array([0, p1 - p0], np.uint32),
            par_p=ev.par_p[p0:p1], par_q=ev.par_q[p0:p1], par_tx=ev.par_tx[p0:p1],
            par_ty=ev.par_ty[p0:p1], par_mask=ev.par_mask[p0:p1],
            par_has_track=ev.par_has_track[p0:p1]))
    if not parts:
        z = np.zeros(0, np.float32)
        zi = np.zeros(0, np.int32)
        return Events(0, np.zeros(1, np.uint32), z, z, z, zi, np.zeros(1, np.uint32), z, z, z, z, z,
                      zi, np.zeros(1, np.uint32), z, z, z, z, np.zeros(0, np.uint16),
                      np.zeros(0, np.uint8))
    return concat(parts)


def kick(tx, ty, qop, field: str = "paper"):
    """The world's kick over arrays: (slope change d, integrated field BL, forward mask)."""
    tx, ty, qop = (np.ascontiguousarray(a, dtype=np.float64) for a in (tx, ty, qop))
    n = tx.size
    d, bl = np.zeros(n), np.zeros(n)
    ok = np.zeros(n, np.uint8)
    cfg = _make_cfg(config("single"), field)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _load().lfgen_kick_many(ctypes.byref(cfg), n, p(tx), p(ty), p(qop), p(d), p(bl), p(ok))
    return d, bl, ok.astype(bool)


# Momentum parametrisation F(tx, ty, dSlope) = sum_i c_i(tx, ty) dSlope^i,
# i = 0..4, of the paper's "Calculation of momentum and track states", as a
# table F_coef[i][j]: c_i = sum_j F_coef[i][j] m_j for even i and
# c_i = tx * sum_{j<6} F_coef[i][j] m_j for odd i, with the monomials
# m = (1, tx2, ty2, tx2^2, tx2 ty2, ty2^2, tx2^3, tx2^2 ty2, tx2 ty2^2, ty2^3),
# tx2 = tx^2, ty2 = ty^2: total degree <= 6, even in ty, and even (odd) in
# tx for even (odd) powers of dSlope -- the symmetries of a field mirror-
# symmetric in x and y.
FIT_P_MIN = 1.5
FIT_SAMPLES = 400_000
FIT_SEED = 7


@functools.lru_cache(maxsize=None)
def field_table(field: str = "paper") -> tuple:
    """F_coef (5 x 10, row-major, float32 values) fitted by least squares on
    toy tracks that populate the slope acceptance evenly with a flat q/p
    spectrum (|p| >= FIT_P_MIN) and reach the first and last SciFi layers
    inside the acceptance -- the calibration of the paper's momentum
    parametrisation, done for this synthetic field."""
    b = _BASE
    rng = np.random.default_rng(FIT_SEED)
    n = FIT_SAMPLES
    tx = rng.uniform(-b["tx_max"], b["tx_max"], n)
    ty = rng.uniform(-b["ty_max"], b["ty_max"], n)
    qop = rng.uniform(-1.0 / FIT_P_MIN, 1.0 / FIT_P_MIN, n)
    d, bl, ok = kick(tx, ty, qop, field)
    fc = FIELDS[field]
    zT = fc.get("z_T", Z_T)
    for z in (LAYER_Z[0], LAYER_Z[-1]):
        x = tx * Z_MAG + (tx + d) * (z - Z_MAG) + KAPPA * d * (z - zT) ** 2 * (1.0 + fc["dRatio"] * (z - zT))
        ok &= (np.abs(x) < b["x_acc"]) & (np.abs(ty * z) < b["y_acc"])
    tx, ty, d, bl = tx[ok], ty[ok], d[ok], bl[ok]
    x2, y2 = tx * tx, ty * ty
    m = [np.ones_like(tx), x2, y2, x2 * x2, x2 * y2, y2 * y2, x2 * x2 * x2, x2 * x2 * y2, x2 * y2 * y2,
         y2 * y2 * y2]
    cols, where = [], []
    for i in range(5):
        for j in range(10 if i % 2 == 0 else 6):
            cols.append(m[j] * d ** i * (tx if i % 2 else 1.0))
            where.append((i, j))
    coef, *_ = np.linalg.lstsq(np.stack(cols, 1), bl, rcond=None)
    table = np.zeros((5, 10), np.float32)
    for (i, j), v in zip(where, coef):
        table[i, j] = v
    return tuple(float(v) for v in table.ravel())


def world(field: str = "toy", **overrides) -> dict:
    """Detector and field description of events generated in ``field``
    (inputs of the method): geometry, the linear-kick constants, the cubic
    term and, for the paper field, the fitted momentum parametrisation."""
    if field not in FIELDS:
        raise KeyError(f"unknown field {field!r}; have {sorted(FIELDS)}")
    fc = FIELDS[field]
    w = dict(z=list(LAYER_Z), dxdy=list(LAYER_DXDY), z_in=Z_UP, z_mag=Z_MAG, z_T=fc.get("z_T", Z_T),
             kick=KICK, kappa=KAPPA, dRatio=fc["dRatio"], polarity=1, field_form=fc["field_form"])
    if fc["field_form"] == 1:
        w["F_coef"] = list(field_table(field))
    w.update(overrides)
    return w

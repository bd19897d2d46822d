"""CPU oracle for Looking Forward track following -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps the plain single-threaded C
implementation in ``lfo.c`` (built with gcc, ``-ffp-contract=off``, no
fast-math) and shares nothing with the GPU library.

``run(events, world)`` returns one result per input track; ``world`` is the
detector/field description (layer z and stereo, z of the upstream states,
bending plane, kick, residual curvature).  The track-model reference plane
z_ref = 8520 mm is the paper's ("Extending triplets to other layers").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lfo.c")
_HDR = os.path.join(_HERE, "lfo.h")
_LIB = os.path.join(_HERE, "liblfo.so")

NL = 12
MAX_TRIPLETS = 64
Z_REF = 8520.0
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
          "-shared", "-fPIC"]


class Geometry(ctypes.Structure):
    _fields_ = [("z", ctypes.c_float * NL), ("dxdy", ctypes.c_float * NL),
                ("z_in", ctypes.c_float), ("z_mag", ctypes.c_float), ("z_ref", ctypes.c_float),
                ("z_T", ctypes.c_float), ("kick", ctypes.c_float), ("kappa", ctypes.c_float),
                ("dRatio", ctypes.c_float), ("polarity", ctypes.c_int32),
                ("field_form", ctypes.c_int32), ("F_coef", (ctypes.c_float * 10) * 5)]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in (
        "T_triplet", "T_x", "T_uv_scale", "T_uv_floor", "T_ty", "T_y", "T_Q",
        "xtol_const", "xtol_pscale", "xasym", "uv_halfwidth", "K_first", "K_last",
        "magtol_const", "magtol_pscale", "magtol_txscale", "magtol_min", "magtol_max",
        "p_charge_cut")] + [("C_nhits", ctypes.c_float * 4), ("n_hits_window", ctypes.c_int32),
                            ("n_triplets", ctypes.c_int32), ("velo_only", ctypes.c_int32),
                            ("noUT_c", ctypes.c_float * 8), ("noUT_p_min", ctypes.c_float),
                            ("noUT_pt_min", ctypes.c_float), ("noUT_overlap", ctypes.c_float),
                            ("seed_fp16", ctypes.c_int32)]
_ARRAYS = ("C_nhits", "noUT_c")


class _Out(ctypes.Structure):
    _fields_ = [("found", ctypes.c_void_p), ("n_hits", ctypes.c_void_p), ("hit_idx", ctypes.c_void_p)] + \
               [(n, ctypes.c_void_p) for n in ("a", "b", "c", "y0", "ty", "qop", "Q")]


class _Dbg(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("win", "wx", "counts", "trip", "trip_chi2", "cand_Q",
                                                "cand_hits", "win1", "wx1")]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (this builds the checker; it does not run it)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _bind(lib):
    lib.lfo_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.lfo_h16.argtypes = [ctypes.c_float]
    lib.lfo_h16.restype = ctypes.c_float
    lib.lfo_default_params_no_ut.argtypes = [ctypes.POINTER(Params)]
    lib.lfo_find_tracks.restype = ctypes.c_int
    lib.lfo_find_tracks.argtypes = (
        [ctypes.POINTER(Geometry), ctypes.POINTER(Params), ctypes.c_uint32] + [ctypes.c_void_p] * 10
        + [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_Out), ctypes.POINTER(_Dbg)])
    return lib


def load_variant(path: str):
    """Load another build of lfo.c (used by tests that plant mistakes in a copy)."""
    return _bind(ctypes.CDLL(path))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def default_params(no_ut: bool = False) -> dict:
    """The oracle's own defaults: the paper's Forward tuning plus readings, or
    (no_ut) its Forward no-UT tuning for VELO-only input."""
    p = Params()
    lib = _load()
    (lib.lfo_default_params_no_ut if no_ut else lib.lfo_default_params)(ctypes.byref(p))
    d = {}
    for name, _ in Params._fields_:
        v = getattr(p, name)
        d[name] = list(v) if name in _ARRAYS else v
    return d


def make_geometry(world: dict) -> Geometry:
    g = Geometry()
    for i in range(NL):
        g.z[i] = world["z"][i]
        g.dxdy[i] = world["dxdy"][i]
    g.z_in = world["z_in"]
    g.z_mag = world["z_mag"]
    g.z_ref = world.get("z_ref", Z_REF)
    g.z_T = world["z_T"]
    g.kick = world["kick"]
    g.kappa = world["kappa"]
    g.dRatio = world.get("dRatio", 0.0)
    g.polarity = int(world.get("polarity", 1))
    g.field_form = int(world.get("field_form", 0))
    coef = world.get("F_coef", [0.0] * 50)
    for i in range(5):
        for j in range(10):
            g.F_coef[i][j] = coef[10 * i + j]
    return g


def make_params(params: dict | None, lib=None) -> Params:
    """Defaults (the no-UT column when params has velo_only set) overridden by params."""
    p = Params()
    lib = lib or _load()
    no_ut = bool((params or {}).get("velo_only", 0))
    (lib.lfo_default_params_no_ut if no_ut else lib.lfo_default_params)(ctypes.byref(p))
    for k, v in (params or {}).items():
        if k in _ARRAYS:
            arr = getattr(p, k)
            for i in range(len(arr)):
                arr[i] = v[i]
        else:
            setattr(p, k, v)
    return p


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def run(ev, world: dict, params: dict | None = None, events: tuple[int, int] | None = None,
        debug: bool = False, lib=None) -> dict:
    """Run the oracle over events [e0, e1) of ``ev`` (default: all).

    Returns arrays indexed by global input-track index; tracks outside the
    range are left "not found".  With ``debug`` also the per-layer windows,
    work counters, the kept triplets and each candidate's Q.
    """
    lib = lib or _load()
    g = make_geometry(world)
    p = make_params(params, lib)
    if not (1 <= p.n_triplets <= MAX_TRIPLETS):
        raise ValueError("n_triplets out of range")
    E = ev.n_events
    e0, e1 = events if events is not None else (0, E)
    T = ev.n_tracks
    NT = p.n_triplets
    out = dict(found=np.zeros(T, np.uint8), n_hits=np.zeros(T, np.uint8),
               hit_idx=np.full((T, NL), -1, np.int32))
    for k in ("a", "b", "c", "y0", "ty", "qop", "Q"):
        out[k] = np.zeros(T, np.float32)
    o = _Out(*[_ptr(out[k]) for k in ("found", "n_hits", "hit_idx", "a", "b", "c", "y0", "ty", "qop", "Q")])
    d = _Dbg()
    if debug:
        out["win"] = np.zeros((T, NL, 2), np.int32)
        out["wx"] = np.zeros((T, NL, 3), np.float32)
        out["counts"] = np.zeros((T, 4), np.int64)
        out["trip"] = np.full((T, NT, 4), -1, np.int32)
        out["trip_chi2"] = np.full((T, NT), np.nan, np.float32)
        out["cand_Q"] = np.full((T, NT), np.nan, np.float32)
        out["cand_hits"] = np.full((T, NT, NL), -1, np.int32)
        out["win1"] = np.zeros((T, NL, 2), np.int32)
        out["wx1"] = np.zeros((T, NL, 3), np.float32)
        d = _Dbg(*[_ptr(out[k]) for k in ("win", "wx", "counts", "trip", "trip_chi2", "cand_Q",
                                          "cand_hits", "win1", "wx1")])
    arrs = [np.ascontiguousarray(a) for a in (
        ev.hit_off.astype(np.uint32), ev.hit_x.astype(np.float32), ev.hit_z.astype(np.float32),
        ev.hit_dxdy.astype(np.float32), ev.trk_off.astype(np.uint32), ev.trk_x.astype(np.float32),
        ev.trk_y.astype(np.float32), ev.trk_tx.astype(np.float32), ev.trk_ty.astype(np.float32),
        ev.trk_qop.astype(np.float32))]
    rc = lib.lfo_find_tracks(ctypes.byref(g), ctypes.byref(p), E, *[_ptr(a) for a in arrs],
                             e0, e1, ctypes.byref(o), ctypes.byref(d))
    if rc != 0:
        raise ValueError("lfo_find_tracks rejected its arguments")
    return out


def h16(x: float, lib=None) -> float:
    """The oracle's binary16 rounding of one binary32 value."""
    return float((lib or _load()).lfo_h16(float(x)))

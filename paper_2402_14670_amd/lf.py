"""ctypes binding of the Looking Forward GPU library (include/lf.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of liblf_hip.so.  The functions carry the C names; arrays are numpy arrays
(copied to the device by lf_upload_events); ``stream`` is a hipStream_t
handle as an integer (``torch.cuda.current_stream().cuda_stream``) or None
for the context's own stream.  Importing this module fails loudly when the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

NL = 12
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblf_hip.so")

LF_OK = 0
LF_ERR_INVALID = -1
LF_ERR_TOO_LARGE = -2
LF_ERR_NOMEM = -3
LF_ERR_DEVICE = -4
LF_ERR_STATE = -5
LF_MODE_PLAIN = 0
LF_MODE_BATCHED = 1
LF_MODE_PERSISTENT = 2
MODES = {"plain": LF_MODE_PLAIN, "batched": LF_MODE_BATCHED, "persistent": LF_MODE_PERSISTENT}
WORK_COUNTERS = ("tracks", "pairs_all", "seed_items", "pairs_tested", "doublets", "triplets", "kept",
                 "fitted", "accepted", "staged_hits", "found", "cy_windows", "cy_stage", "cy_doublets", "cy_model",
                 "cy_extend", "cy_fit", "cy_select")


class LFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class lf_geometry(ctypes.Structure):
    _fields_ = [("z", ctypes.c_float * NL), ("dxdy", ctypes.c_float * NL),
                ("z_in", ctypes.c_float), ("z_mag", ctypes.c_float), ("z_ref", ctypes.c_float),
                ("z_T", ctypes.c_float), ("kick", ctypes.c_float), ("kappa", ctypes.c_float),
                ("dRatio", ctypes.c_float), ("polarity", ctypes.c_int32),
                ("field_form", ctypes.c_int32), ("F_coef", (ctypes.c_float * 10) * 5)]


_PARAM_FLOATS = ("T_triplet", "T_x", "T_uv_scale", "T_uv_floor", "T_ty", "T_y", "T_Q",
                 "xtol_const", "xtol_pscale", "xasym", "uv_halfwidth", "K_first", "K_last",
                 "magtol_const", "magtol_pscale", "magtol_txscale", "magtol_min", "magtol_max",
                 "p_charge_cut")


class lf_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in _PARAM_FLOATS] + [
        ("C_nhits", ctypes.c_float * 4), ("n_hits_window", ctypes.c_int32), ("n_triplets", ctypes.c_int32),
        ("velo_only", ctypes.c_int32), ("noUT_c", ctypes.c_float * 8), ("noUT_p_min", ctypes.c_float),
        ("noUT_pt_min", ctypes.c_float), ("noUT_overlap", ctypes.c_float), ("seed_fp16", ctypes.c_int32)]


_PARAM_ARRAYS = ("C_nhits", "noUT_c")


class lf_batch(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_uint32), ("hit_off", ctypes.c_void_p), ("hit_x", ctypes.c_void_p),
                ("hit_z", ctypes.c_void_p), ("hit_dxdy", ctypes.c_void_p), ("trk_off", ctypes.c_void_p),
                ("trk_x", ctypes.c_void_p), ("trk_y", ctypes.c_void_p), ("trk_tx", ctypes.c_void_p),
                ("trk_ty", ctypes.c_void_p), ("trk_qop", ctypes.c_void_p)]


class lf_tracks_out(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("found", "n_hits", "hit_idx", "a", "b", "c", "y0", "ty",
                                                "qop", "Q")]


class lf_serve_config(ctypes.Structure):
    _fields_ = [("max_batch_events", ctypes.c_uint32), ("min_batch_events", ctypes.c_uint32),
                ("max_wait_us", ctypes.c_uint32), ("n_slots", ctypes.c_uint32),
                ("n_pack_threads", ctypes.c_uint32), ("pool_on_device", ctypes.c_uint32),
                ("results_on_device", ctypes.c_uint32), ("verify_results", ctypes.c_uint32),
                ("device_budget_bytes", ctypes.c_size_t)]


class lf_serve_stats(ctypes.Structure):
    _fields_ = [("n_requests", ctypes.c_uint64), ("n_batches", ctypes.c_uint64), ("max_queue", ctypes.c_uint64),
                ("max_device_bytes", ctypes.c_uint64), ("wall_s", ctypes.c_double),
                ("events_per_s", ctypes.c_double), ("lat_p50_s", ctypes.c_double), ("lat_p99_s", ctypes.c_double),
                ("lat_p999_s", ctypes.c_double), ("lat_max_s", ctypes.c_double),
                ("mean_batch_events", ctypes.c_double), ("bytes_in", ctypes.c_uint64),
                ("bytes_out", ctypes.c_uint64), ("result_mismatches", ctypes.c_uint64)]


class lf_exec(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("items_per_grab", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32)]


EXPORTS = ("lf_default_params", "lf_default_params_no_ut", "lf_check_batch", "lf_create", "lf_upload_events", "lf_find_tracks",
           "lf_work_counts", "lf_fetch_tracks", "lf_copy_tracks", "lf_poison_tracks", "lf_release_batch", "lf_set_exec", "lf_batch_info",
           "lf_device_bytes_in_use", "lf_serve_run", "lf_graph_create", "lf_graph_launch", "lf_graph_destroy",
           "lf_destroy", "lf_last_error", "lf_find_tracks_noalloc")


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblf_hip.so and declare every exported signature.

    PyTorch is imported first so that the process holds a single HIP
    runtime: the library then binds to the runtime torch loaded (same
    soname), and stream handles and device memory are shared with torch.
    """
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (no CPU fallback exists)")
    import torch  # noqa: F401  (loads the process's HIP runtime)
    lib = ctypes.CDLL(path)
    P, vp, i32, u64, sz = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t
    lib.lf_default_params.argtypes = [P(lf_params)]
    lib.lf_default_params.restype = None
    lib.lf_default_params_no_ut.argtypes = [P(lf_params)]
    lib.lf_default_params_no_ut.restype = None
    lib.lf_check_batch.argtypes = [P(lf_batch)]
    lib.lf_create.argtypes = [P(lf_geometry), P(lf_params), sz, P(vp)]
    lib.lf_upload_events.argtypes = [vp, P(lf_batch), vp, P(u64)]
    lib.lf_find_tracks.argtypes = [vp, u64, i32, vp]
    lib.lf_fetch_tracks.argtypes = [vp, u64, P(lf_tracks_out), sz, vp]
    lib.lf_find_tracks_noalloc.argtypes = [vp, P(lf_batch), ctypes.c_uint32, ctypes.c_uint32, P(lf_tracks_out), i32,
                                           vp]
    lib.lf_work_counts.argtypes = [vp, u64, vp, P(ctypes.c_int64), sz]
    lib.lf_copy_tracks.argtypes = [vp, u64, P(lf_tracks_out), sz, vp]
    lib.lf_poison_tracks.argtypes = [vp, u64, vp]
    lib.lf_release_batch.argtypes = [vp, u64]
    lib.lf_set_exec.argtypes = [vp, P(lf_exec)]
    lib.lf_batch_info.argtypes = [vp, u64, P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32), P(sz)]
    lib.lf_serve_run.argtypes = [vp, P(lf_batch), ctypes.c_uint32, vp, vp, P(lf_serve_config), vp, vp,
                                 P(lf_serve_stats)]
    lib.lf_graph_create.argtypes = [vp, vp, ctypes.c_uint32, i32, P(vp)]
    lib.lf_graph_launch.argtypes = [vp, vp, vp]
    lib.lf_graph_destroy.argtypes = [vp]
    lib.lf_graph_destroy.restype = None
    lib.lf_device_bytes_in_use.argtypes = [vp]
    lib.lf_device_bytes_in_use.restype = sz
    lib.lf_destroy.argtypes = [vp]
    lib.lf_destroy.restype = None
    lib.lf_last_error.argtypes = [vp]
    lib.lf_last_error.restype = ctypes.c_char_p
    for name in ("lf_check_batch", "lf_create", "lf_upload_events", "lf_find_tracks", "lf_work_counts",
                 "lf_fetch_tracks", "lf_release_batch", "lf_set_exec", "lf_batch_info", "lf_serve_run",
                 "lf_graph_create", "lf_graph_launch", "lf_copy_tracks", "lf_poison_tracks",
                 "lf_find_tracks_noalloc"):
        getattr(lib, name).restype = i32
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc: int, ctx) -> None:
    if rc != LF_OK:
        msg = lib().lf_last_error(ctx)
        raise LFError(rc, msg.decode() if msg else "")


def _stream(s) -> ctypes.c_void_p:
    return ctypes.c_void_p(int(s) if s else 0)


def _arr(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------------ C names
def lf_default_params(no_ut: bool = False) -> dict:
    """The library's defaults: the Forward column, or (no_ut) the Forward no-UT column."""
    p = lf_params()
    (lib().lf_default_params_no_ut if no_ut else lib().lf_default_params)(ctypes.byref(p))
    d = {}
    for n, _ in lf_params._fields_:
        v = getattr(p, n)
        d[n] = list(v) if n in _PARAM_ARRAYS else v
    return d


def lf_default_params_no_ut() -> dict:
    return lf_default_params(no_ut=True)


def make_geometry(world: dict) -> lf_geometry:
    g = lf_geometry()
    for i in range(NL):
        g.z[i] = world["z"][i]
        g.dxdy[i] = world["dxdy"][i]
    g.z_in = world["z_in"]
    g.z_mag = world["z_mag"]
    g.z_ref = world.get("z_ref", 8520.0)
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


def make_params(params: dict | None = None) -> lf_params:
    """Defaults (the no-UT column when params sets velo_only) overridden by params."""
    p = lf_params()
    no_ut = bool((params or {}).get("velo_only", 0))
    (lib().lf_default_params_no_ut if no_ut else lib().lf_default_params)(ctypes.byref(p))
    for k, v in (params or {}).items():
        if k in _PARAM_ARRAYS:
            arr = getattr(p, k)
            for i in range(len(arr)):
                arr[i] = v[i]
        else:
            setattr(p, k, v)
    return p


def lf_create(world: dict, params: dict | None = None, budget_bytes: int = 0) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    g, p = make_geometry(world), make_params(params)
    rc = lib().lf_create(ctypes.byref(g), ctypes.byref(p), budget_bytes, ctypes.byref(ctx))
    if rc != LF_OK:
        raise LFError(rc, lib().lf_last_error(None).decode())
    return ctx


class _Hold:
    """Keeps the host arrays of a batch alive while the call runs."""

    def __init__(self, ev):
        self.hit_off = _arr(ev.hit_off, np.uint32)
        self.hit_x = _arr(ev.hit_x, np.float32)
        self.hit_z = _arr(ev.hit_z, np.float32)
        self.hit_dxdy = _arr(ev.hit_dxdy, np.float32)
        self.trk_off = _arr(ev.trk_off, np.uint32)
        self.trk = [_arr(getattr(ev, k), np.float32) for k in ("trk_x", "trk_y", "trk_tx", "trk_ty", "trk_qop")]
        self.n_events = int(ev.n_events)

    def struct(self) -> lf_batch:
        b = lf_batch()
        b.n_events = self.n_events
        b.hit_off = self.hit_off.ctypes.data
        b.hit_x = self.hit_x.ctypes.data
        b.hit_z = self.hit_z.ctypes.data
        b.hit_dxdy = self.hit_dxdy.ctypes.data
        b.trk_off = self.trk_off.ctypes.data
        b.trk_x, b.trk_y, b.trk_tx, b.trk_ty, b.trk_qop = (a.ctypes.data for a in self.trk)
        return b


def lf_check_batch(ev) -> None:
    """Host-side validation of a batch; raises LFError if malformed."""
    h = _Hold(ev)
    b = h.struct()
    rc = lib().lf_check_batch(ctypes.byref(b))
    if rc != LF_OK:
        raise LFError(rc, lib().lf_last_error(None).decode())


def lf_upload_events(ctx, ev, stream=None) -> int:
    """Upload a batch (any object with the lf_batch arrays as attributes)."""
    h = _Hold(ev)
    b = h.struct()
    bid = ctypes.c_uint64()
    _check(lib().lf_upload_events(ctx, ctypes.byref(b), _stream(stream), ctypes.byref(bid)), ctx)
    return bid.value


def lf_find_tracks(ctx, batch_id: int, mode=LF_MODE_BATCHED, stream=None) -> None:
    if isinstance(mode, str):
        mode = MODES[mode]
    _check(lib().lf_find_tracks(ctx, ctypes.c_uint64(batch_id), int(mode), _stream(stream)), ctx)


_IN_FIELDS = ("hit_off", "hit_x", "hit_z", "hit_dxdy", "trk_off", "trk_x", "trk_y", "trk_tx", "trk_ty", "trk_qop")
_OUT_FIELDS = ("found", "n_hits", "hit_idx", "a", "b", "c", "y0", "ty", "qop", "Q")


def lf_find_tracks_noalloc(ctx, dev_in: dict, dev_out: dict, mode=LF_MODE_BATCHED, stream=None) -> None:
    """Hot path over a batch already in device memory, into device outputs,
    with no allocation (the library's fixed scratch).  dev_in maps the
    lf_batch array names to contiguous device tensors (u32 offsets, f32
    values); dev_out maps the lf_tracks_out names to contiguous device
    tensors of at least n_tracks slots (hit_idx n_tracks x 12)."""
    if isinstance(mode, str):
        mode = MODES[mode]
    for k in _IN_FIELDS:
        if not dev_in[k].is_contiguous():
            raise ValueError(f"dev_in[{k!r}] is not contiguous")
    for k in _OUT_FIELDS:
        if not dev_out[k].is_contiguous():
            raise ValueError(f"dev_out[{k!r}] is not contiguous")
    b = lf_batch()
    b.n_events = int(dev_in["trk_off"].numel()) - 1
    for k in _IN_FIELDS:
        setattr(b, k, dev_in[k].data_ptr())
    o = lf_tracks_out(*[dev_out[k].data_ptr() for k in _OUT_FIELDS])
    _check(lib().lf_find_tracks_noalloc(ctx, ctypes.byref(b), int(dev_in["hit_x"].numel()),
                                        int(dev_in["trk_x"].numel()), ctypes.byref(o), int(mode),
                                        _stream(stream)), ctx)


def lf_work_counts(ctx, batch_id: int, stream=None) -> dict:
    """Work counters of one counting pass over a resident batch."""
    n = len(WORK_COUNTERS)
    arr = (ctypes.c_int64 * n)()
    _check(lib().lf_work_counts(ctx, ctypes.c_uint64(batch_id), _stream(stream), arr, n), ctx)
    return {k: int(arr[i]) for i, k in enumerate(WORK_COUNTERS)}


def lf_fetch_tracks(ctx, batch_id: int, n_tracks: int | None = None, stream=None, release: bool = True) -> dict:
    """Results of a batch; the batch is freed unless release is False (lf_copy_tracks)."""
    nb = lf_batch_info(ctx, batch_id)["n_tracks"]
    T = nb if n_tracks is None else int(n_tracks)
    # the call fills every slot of the batch's tracks (or fails, and the
    # arrays are dropped); slots past the batch's count keep defaults
    if T == nb:
        out = dict(found=np.empty(T, np.uint8), n_hits=np.empty(T, np.uint8), hit_idx=np.empty((T, NL), np.int32))
        for k in ("a", "b", "c", "y0", "ty", "qop", "Q"):
            out[k] = np.empty(T, np.float32)
    else:
        out = dict(found=np.zeros(T, np.uint8), n_hits=np.zeros(T, np.uint8), hit_idx=np.full((T, NL), -1, np.int32))
        for k in ("a", "b", "c", "y0", "ty", "qop", "Q"):
            out[k] = np.zeros(T, np.float32)
    o = lf_tracks_out(*[out[k].ctypes.data for k in ("found", "n_hits", "hit_idx", "a", "b", "c", "y0", "ty",
                                                      "qop", "Q")])
    fn = lib().lf_fetch_tracks if release else lib().lf_copy_tracks
    _check(fn(ctx, ctypes.c_uint64(batch_id), ctypes.byref(o), T, _stream(stream)), ctx)
    return out


def lf_copy_tracks(ctx, batch_id: int, n_tracks: int | None = None, stream=None) -> dict:
    return lf_fetch_tracks(ctx, batch_id, n_tracks, stream, release=False)


def lf_poison_tracks(ctx, batch_id: int, stream=None) -> None:
    _check(lib().lf_poison_tracks(ctx, ctypes.c_uint64(batch_id), _stream(stream)), ctx)


def lf_release_batch(ctx, batch_id: int) -> None:
    _check(lib().lf_release_batch(ctx, ctypes.c_uint64(batch_id)), ctx)


def lf_set_exec(ctx, waves_per_block: int = 0, items_per_grab: int = 0, blocks_per_cu: int = 0) -> None:
    x = lf_exec(waves_per_block, items_per_grab, blocks_per_cu)
    _check(lib().lf_set_exec(ctx, ctypes.byref(x)), ctx)


def lf_batch_info(ctx, batch_id: int) -> dict:
    e, t, h, b = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_size_t()
    _check(lib().lf_batch_info(ctx, ctypes.c_uint64(batch_id), ctypes.byref(e), ctypes.byref(t),
                               ctypes.byref(h), ctypes.byref(b)), ctx)
    return dict(n_events=e.value, n_tracks=t.value, n_hits=h.value, device_bytes=b.value)


def lf_serve_run(ctx, pool, req_event, arrival_s, config: dict | None = None):
    """Serve a request stream (see lf.h).  Returns (digests u64[n], latencies f64[n], stats dict)."""
    h = _Hold(pool)
    b = h.struct()
    req = np.ascontiguousarray(req_event, dtype=np.uint32)
    arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
    if len(req) != len(arr):
        raise ValueError("req_event and arrival_s differ in length")
    cfg = lf_serve_config()
    for k, v in (config or {}).items():
        setattr(cfg, k, int(v))
    dig = np.zeros(len(req), np.uint64)
    lat = np.zeros(len(req), np.float64)
    st = lf_serve_stats()
    _check(lib().lf_serve_run(ctx, ctypes.byref(b), len(req), req.ctypes.data, arr.ctypes.data, ctypes.byref(cfg),
                              dig.ctypes.data, lat.ctypes.data, ctypes.byref(st)), ctx)
    stats = {n: getattr(st, n) for n, _ in lf_serve_stats._fields_}
    return dig, lat, stats


def lf_graph_create(ctx, batch_ids, mode=LF_MODE_BATCHED) -> ctypes.c_void_p:
    """Capture the hot path of resident batches (in order) into a HIP graph."""
    if isinstance(mode, str):
        mode = MODES[mode]
    ids = np.ascontiguousarray(batch_ids, dtype=np.uint64)
    g = ctypes.c_void_p()
    _check(lib().lf_graph_create(ctx, ids.ctypes.data, len(ids), int(mode), ctypes.byref(g)), ctx)
    return g


def lf_graph_launch(ctx, graph, stream=None) -> None:
    _check(lib().lf_graph_launch(ctx, graph, _stream(stream)), ctx)


def lf_graph_destroy(graph) -> None:
    lib().lf_graph_destroy(graph)


def lf_device_bytes_in_use(ctx) -> int:
    return int(lib().lf_device_bytes_in_use(ctx))


def lf_destroy(ctx) -> None:
    lib().lf_destroy(ctx)


def lf_last_error(ctx=None) -> str:
    m = lib().lf_last_error(ctx)
    return m.decode() if m else ""


# ------------------------------------------------------------------ digests
_M64 = (1 << 64) - 1


def _mix64(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def result_digests(out: dict, trk_off) -> np.ndarray:
    """Per-event digest of fetched results, as lf_serve_run defines it in lf.h
    (host-side, to compare served requests with batched or single runs)."""
    T = len(out["found"])
    w = np.zeros((T, 20), np.uint64)
    w[:, 0] = out["found"].astype(np.uint64) | (out["n_hits"].astype(np.uint64) << np.uint64(8))
    w[:, 1:13] = out["hit_idx"].astype(np.int32).view(np.uint32).astype(np.uint64)
    for i, k in enumerate(("a", "b", "c", "y0", "ty", "qop", "Q")):
        w[:, 13 + i] = out[k].astype(np.float32).view(np.uint32).astype(np.uint64)
    with np.errstate(over="ignore"):
        h = np.full(T, 0xCBF29CE484222325, np.uint64)
        for k in range(20):
            h = (h ^ w[:, k]) * np.uint64(0x100000001B3)
        off = np.asarray(trk_off, np.int64)
        ev = np.repeat(np.arange(len(off) - 1), np.diff(off))
        idx = (np.arange(T, dtype=np.int64) - off[ev]).astype(np.uint64)
        m = _mix64(h ^ (idx * np.uint64(0x9E3779B97F4A7C15)))
        d = np.zeros(len(off) - 1, np.uint64)
        np.add.at(d, ev, m)
    return d


# ------------------------------------------------------------------ convenience
class Forward:
    """One context: upload, run and fetch in one call (``find``)."""

    def __init__(self, world: dict, params: dict | None = None, budget_bytes: int = 0):
        self.ctx = lf_create(world, params, budget_bytes)

    def find(self, ev, mode="batched", stream=None) -> dict:
        bid = lf_upload_events(self.ctx, ev, stream)
        try:
            lf_find_tracks(self.ctx, bid, mode, stream)
        except Exception:
            lf_release_batch(self.ctx, bid)
            raise
        return lf_fetch_tracks(self.ctx, bid, int(ev.trk_off[-1]), stream)

    def close(self) -> None:
        if self.ctx:
            lf_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""The non-allocating entry point (lf_find_tracks_noalloc): a batch already in
device memory, device outputs, the library's fixed scratch.  Two calls in a
row, the second on a smaller batch, in both modes it accepts, each compared
slot by slot with lf_upload_events + lf_find_tracks + lf_fetch_tracks on the
same batch (indices bit-exact, parameters within 1e-5 relative); the first
batch is also checked against the oracle.  Sizes beyond the fixed scratch
are rejected before anything is launched."""
import numpy as np
import pytest

import lfgen
from parity import W, compare, oracle_parallel, run_gpu, say

pytestmark = pytest.mark.gpu

IN_U32 = ("hit_off", "trk_off")
IN_F32 = ("hit_x", "hit_z", "hit_dxdy", "trk_x", "trk_y", "trk_tx", "trk_ty", "trk_qop")


def _device_batch(ev):
    import torch
    d = {}
    for k in IN_U32:
        a = np.ascontiguousarray(getattr(ev, k), dtype=np.uint32).view(np.int32)
        d[k] = torch.from_numpy(a.copy()).cuda()
    for k in IN_F32:
        d[k] = torch.from_numpy(np.ascontiguousarray(getattr(ev, k), dtype=np.float32).copy()).cuda()
    return d


def _device_out(T):
    import torch
    o = dict(found=torch.full((T,), 0xAB, dtype=torch.uint8, device="cuda"),
             n_hits=torch.full((T,), 0xAB, dtype=torch.uint8, device="cuda"),
             hit_idx=torch.full((T, 12), -7, dtype=torch.int32, device="cuda"))
    for k in ("a", "b", "c", "y0", "ty", "qop", "Q"):
        o[k] = torch.full((T,), float("nan"), dtype=torch.float32, device="cuda")
    return o


def _host(o, T):
    return {k: v[:T].cpu().numpy() for k, v in o.items()}


def test_noalloc_two_calls_match_upload_path():
    import torch
    from paper_2402_14670_amd import lf
    big = lfgen.generate("nominal", n_events=40)
    small = lfgen.generate("uneven", n_events=20)
    assert small.n_tracks < big.n_tracks and small.n_hits < big.n_hits
    stream = torch.cuda.current_stream()
    ref_big = {m: run_gpu(big, m) for m in ("batched", "persistent")}
    ref_small = {m: run_gpu(small, m) for m in ("batched", "persistent")}
    compare(oracle_parallel(big), ref_big["batched"], label="nominal[40] upload path vs oracle")
    ctx = lf.lf_create(W)
    try:
        # one output buffer sized for the larger batch, reused by both calls
        out = _device_out(big.n_tracks)
        for mode in ("batched", "persistent"):
            for name, ev, ref in (("nominal[40]", big, ref_big[mode]), ("uneven[20]", small, ref_small[mode])):
                say(f"[gpu] noalloc {name} mode={mode} tracks={ev.n_tracks} hits={ev.n_hits}")
                dev = _device_batch(ev)
                lf.lf_find_tracks_noalloc(ctx, dev, out, mode, stream.cuda_stream)
                torch.cuda.synchronize()
                got = _host(out, ev.n_tracks)
                st = compare(ref, got, label=f"noalloc {name}/{mode}")
                say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")
    finally:
        lf.lf_destroy(ctx)


def test_noalloc_rejects_sizes_beyond_the_fixed_scratch():
    import torch
    from paper_2402_14670_amd import lf
    ev = lfgen.generate("single")
    dev = _device_batch(ev)
    out = _device_out(ev.n_tracks)
    ctx = lf.lf_create(W)
    try:
        # a track count above the limit, on valid pointers: refused on the host
        b = lf.lf_batch()
        b.n_events = ev.n_events
        for k in IN_U32 + IN_F32:
            setattr(b, k, dev[k].data_ptr())
        o = lf.lf_tracks_out(*[out[k].data_ptr() for k in lf._OUT_FIELDS])
        import ctypes
        rc = lf.lib().lf_find_tracks_noalloc(ctx, ctypes.byref(b), ev.n_hits, (1 << 22) + 1, ctypes.byref(o),
                                             lf.LF_MODE_BATCHED, None)
        assert rc == lf.LF_ERR_TOO_LARGE, rc
        assert "fixed scratch" in lf.lf_last_error(ctx)
        rc = lf.lib().lf_find_tracks_noalloc(ctx, ctypes.byref(b), ev.n_hits, ev.n_tracks, ctypes.byref(o),
                                             lf.LF_MODE_PLAIN, None)
        assert rc == lf.LF_ERR_INVALID, rc
        torch.cuda.synchronize()
        # nothing was written
        assert int(out["found"].cpu()[0]) == 0xAB
    finally:
        lf.lf_destroy(ctx)

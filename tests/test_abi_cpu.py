"""The C-ABI library on the CPU: it loads, exports every symbol lf.h
declares, and validates batches on the host.  No call here touches a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import lfgen
import pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lf.h")


@pytest.fixture(scope="module")
def lf():
    from paper_2402_14670_amd import lf as binding
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lf):
    lib = ctypes.CDLL(lf.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lf.h but not exported"
    assert set(names) == set(lf.EXPORTS)


def test_default_params_match_paper(lf):
    d = lf.lf_default_params()
    gold = pins.golden_constants()
    f32 = np.float32
    for k, v in gold.items():
        if k.startswith("C_"):
            assert f32(d["C_nhits"][int(k[2:]) - 9]) == f32(v), k
        elif k == "z_ref":
            assert f32(lf.make_geometry(lfgen.world()).z_ref) == f32(v)
        else:
            assert f32(d[k]) == f32(v), k


def test_default_no_ut_params_match_paper(lf):
    d = lf.lf_default_params(no_ut=True)
    f32 = np.float32
    n = 0
    with open(pins.GOLDEN_NO_UT) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("|")[0].split()
            got = d["noUT_c"][int(k[6:])] if k.startswith("noUT_c") else d[k]
            assert f32(got) == f32(float(v)), k
            n += 1
    assert n >= 20
    # every field the no-UT column leaves alone keeps the Forward default
    fwd = lf.lf_default_params()
    for k in ("K_first", "K_last", "C_nhits", "T_uv_floor"):
        assert d[k] == fwd[k], k


def test_check_batch_accepts_generated(lf):
    lf.lf_check_batch(lfgen.generate("nominal", n_events=2))
    lf.lf_check_batch(lfgen.select_events(lfgen.generate("single"), []))


def _mutated(ev, **kw):
    d = dict(ev.__dict__)
    d.update(kw)
    return lfgen.Events(**d)


def test_check_batch_from_several_threads_at_once(lf):
    """The host worker threads are shared by every caller: batches validated
    from several threads at once (one caller's section on the workers, the
    others on their own thread) each get their own first failure."""
    import threading
    ev = lfgen.generate("nominal", n_events=120)
    H = ev.n_hits
    cases = []
    for k in range(8):
        x = ev.hit_x.copy()
        at = H // 3 + 9973 * k
        x[at] = np.nan
        cases.append((_mutated(ev, hit_x=x), f"non-finite hit {at}$"))
    cases.append((ev, None))
    errors = []

    def work(batch, expect):
        for _ in range(5):
            try:
                lf.lf_check_batch(batch)
                if expect is not None:
                    errors.append(f"accepted a batch that should fail with {expect!r}")
            except lf.LFError as e:
                if expect is None or not re.search(expect, str(e)):
                    errors.append(f"{e} (expected {expect!r})")

    threads = [threading.Thread(target=work, args=c) for c in cases]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors[:4]


@pytest.mark.parametrize("case", ["nan_hit", "inf_track", "qop_zero", "unsorted", "offset_decrease",
                                  "offset_start"])
def test_check_batch_rejects_malformed(lf, case):
    ev = lfgen.generate("single")
    if case == "nan_hit":
        x = ev.hit_x.copy(); x[5] = np.nan; bad = _mutated(ev, hit_x=x)
    elif case == "inf_track":
        t = ev.trk_tx.copy(); t[3] = np.inf; bad = _mutated(ev, trk_tx=t)
    elif case == "qop_zero":
        q = ev.trk_qop.copy(); q[0] = 0.0; bad = _mutated(ev, trk_qop=q)
    elif case == "unsorted":
        x = ev.hit_x.copy(); b0, b1 = int(ev.hit_off[3]), int(ev.hit_off[4])
        assert b1 - b0 >= 2
        x[b0], x[b0 + 1] = x[b0 + 1] + 1.0, x[b0]
        bad = _mutated(ev, hit_x=x)
    elif case == "offset_decrease":
        o = ev.hit_off.copy(); o[5] = o[6] + 1; bad = _mutated(ev, hit_off=o)
    else:
        o = ev.trk_off.copy(); o[0] = 1; bad = _mutated(ev, trk_off=o)
    with pytest.raises(lf.LFError) as e:
        lf.lf_check_batch(bad)
    assert e.value.code == lf.LF_ERR_INVALID
    assert "batch" in str(e.value)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N > 1 exits with a message before touching a GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""


def test_check_batch_reports_the_first_failure_of_a_large_batch(lf):
    """Validation of a large batch runs over slices on several host threads;
    it must still name the failure a serial scan would meet first."""
    ev = lfgen.generate("nominal", n_events=300)
    assert 12 * ev.n_hits >= 1 << 20 and 20 * ev.n_tracks >= 1 << 20   # the threaded scans
    H, T = ev.n_hits, ev.n_tracks
    x = ev.hit_x.copy(); x[H - 10] = np.nan; x[H // 7] = np.inf
    with pytest.raises(lf.LFError, match=f"non-finite hit {H // 7}$"):
        lf.lf_check_batch(_mutated(ev, hit_x=x))
    x = ev.hit_x.copy()
    buckets = []
    for k in (24 * 250 + 5, 24 * 40 + 2):
        b0, b1 = int(ev.hit_off[k]), int(ev.hit_off[k + 1])
        assert b1 - b0 >= 2
        x[b0], x[b0 + 1] = x[b0 + 1] + 1.0, x[b0]
        buckets.append(k)
    with pytest.raises(lf.LFError, match=f"bucket {min(buckets)} not sorted by x$"):
        lf.lf_check_batch(_mutated(ev, hit_x=x))
    # a bucket out of order ahead of non-finite z and dxdy further on: every
    # hit is checked for finite values before any bucket's order
    z = ev.hit_z.copy(); z[H - 5] = np.inf
    with pytest.raises(lf.LFError, match=f"non-finite hit {H - 5}$"):
        lf.lf_check_batch(_mutated(ev, hit_x=x, hit_z=z))
    d = ev.hit_dxdy.copy(); d[H // 3] = -np.inf
    with pytest.raises(lf.LFError, match=f"non-finite hit {H // 3}$"):
        lf.lf_check_batch(_mutated(ev, hit_x=x, hit_z=z, hit_dxdy=d))
    q = ev.trk_qop.copy(); q[T // 9] = 0.0
    t = ev.trk_ty.copy(); t[T - 3] = np.inf
    with pytest.raises(lf.LFError, match=f"q/p == 0 for track {T // 9}$"):
        lf.lf_check_batch(_mutated(ev, trk_qop=q, trk_ty=t))
    t = ev.trk_ty.copy(); t[T // 11] = np.nan
    with pytest.raises(lf.LFError, match=f"non-finite track state {T // 11}$"):
        lf.lf_check_batch(_mutated(ev, trk_qop=q, trk_ty=t))

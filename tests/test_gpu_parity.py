"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Indices, flags and hit counts must be bit-exact; fitted
parameters within 1e-5 relative (binary32 in the same evaluation order on
both sides, so they are expected bit-exact too)."""
import numpy as np
import pytest

import lfgen
import oracle
from parity import W, compare, oracle_on_events, run_gpu, say

pytestmark = pytest.mark.gpu
MODES = ("plain", "batched", "persistent")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _check_all_modes(ev, label, params=None, exec_cfg=None):
    ref = oracle.run(ev, W, params)
    for mode in MODES:
        say(f"[gpu] {label}: mode={mode} events={ev.n_events} tracks={ev.n_tracks} hits={ev.n_hits} "
            f"params={params} exec={exec_cfg}")
        got = run_gpu(ev, mode, params, exec_cfg)
        st = compare(ref, got, label=f"{label}/{mode}")
        say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")


def test_single_event():
    _check_all_modes(lfgen.generate("single"), "single")


def test_nominal_sample():
    _check_all_modes(lfgen.generate("nominal", n_events=20), "nominal[20]")


def test_stress_sample():
    _check_all_modes(lfgen.generate("stress", n_events=3), "stress[3]")


def test_uneven_with_empty_events():
    ev = lfgen.generate("uneven", n_events=60)
    empty = lfgen.select_events(ev, [])
    # an event with tracks but no hits, and one with hits but no tracks
    no_hits = lfgen.select_events(ev, [0])
    no_hits = lfgen.Events(**{**no_hits.__dict__, "hit_off": np.zeros(25, np.uint32),
                              "hit_x": np.zeros(0, np.float32), "hit_z": np.zeros(0, np.float32),
                              "hit_dxdy": np.zeros(0, np.float32), "hit_pid": np.zeros(0, np.int32)})
    no_trk = lfgen.select_events(ev, [1])
    z = np.zeros(0, np.float32)
    no_trk = lfgen.Events(**{**no_trk.__dict__, "trk_off": np.zeros(2, np.uint32), "trk_x": z, "trk_y": z,
                             "trk_tx": z, "trk_ty": z, "trk_qop": z, "trk_pid": np.zeros(0, np.int32)})
    parts = [lfgen.select_events(ev, range(0, 30)), no_hits, no_trk, lfgen.select_events(ev, range(30, 60))]
    mixed = lfgen.concat(parts)
    assert empty.n_events == 0
    _check_all_modes(mixed, "uneven[60]+edge")


@pytest.mark.parametrize("params", [
    {"n_hits_window": 64, "n_triplets": 32},
    {"n_hits_window": 5, "n_triplets": 1},
    {"n_hits_window": 33, "n_triplets": 7},
    {"T_uv_floor": 0.5, "T_triplet": 20.0, "T_x": 4.0},
], ids=["w64_t32", "w5_t1", "w33_t7", "loose"])
def test_parameter_variants(params):
    _check_all_modes(lfgen.generate("nominal", n_events=4), "nominal[4]", params)


def test_whole_bucket_windows_tiny_events():
    ev = lfgen.generate("single", seed=7, n_events=6, n_particles=8, n_noise=20, p_min=1.5, p_max=20.0)
    params = {"xtol_const": 1e7, "uv_halfwidth": 1e7, "n_hits_window": 64, "n_triplets": 2, "T_triplet": 40.0}
    _check_all_modes(ev, "tiny whole-bucket", params)


def test_geometry_variants():
    ev = lfgen.generate("nominal", n_events=3)
    for world in (dict(W, polarity=-1), dict(W, dRatio=-2.0e-4)):
        ref = oracle.run(ev, world)
        from paper_2402_14670_amd import lf
        ctx = lf.lf_create(world)
        try:
            for mode in MODES:
                say(f"[gpu] geometry variant polarity={world['polarity']} dRatio={world['dRatio']} mode={mode}")
                bid = lf.lf_upload_events(ctx, ev)
                lf.lf_find_tracks(ctx, bid, mode)
                got = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks)
                compare(ref, got, label=f"geometry/{mode}")
        finally:
            lf.lf_destroy(ctx)


def _jitter(ev, z_mm, slope_rel, seed):
    """Per-hit z (tilted or bowed layers) and per-hit stereo slope: the hits
    of one window no longer share a z (or a slope), so the GPU takes its
    general paths (doublets bracketed over the third window's z range,
    stereo windows scanned)."""
    rng = np.random.default_rng(seed)
    hz = ev.hit_z + rng.uniform(-z_mm, z_mm, ev.n_hits).astype(np.float32)
    hd = ev.hit_dxdy * (1.0 + rng.uniform(-slope_rel, slope_rel, ev.n_hits)).astype(np.float32)
    return lfgen.Events(**{**ev.__dict__, "hit_z": hz.astype(np.float32), "hit_dxdy": hd.astype(np.float32)})


@pytest.mark.parametrize("z_mm,slope_rel", [(1.5, 0.02), (0.0, 0.02), (3.0, 0.0)],
                         ids=["z_and_slope", "slope_only", "z_only"])
def test_per_hit_z_and_slope(z_mm, slope_rel):
    ev = _jitter(lfgen.generate("nominal", n_events=5), z_mm, slope_rel, seed=11)
    _check_all_modes(ev, f"nominal[5] z+-{z_mm} slope+-{slope_rel}")


def _jitter_layers(ev, layers, z_mm, slope_rel, seed):
    """Per-hit z and stereo slope on some layers only: mixed and common
    windows side by side in one track."""
    rng = np.random.default_rng(seed)
    sel = np.isin(ev.hit_z, np.array([lfgen.LAYER_Z[l] for l in layers], np.float32))
    hz = ev.hit_z + np.where(sel, rng.uniform(-z_mm, z_mm, ev.n_hits), 0.0).astype(np.float32)
    hd = ev.hit_dxdy * (1.0 + np.where(sel, rng.uniform(-slope_rel, slope_rel, ev.n_hits), 0.0)).astype(np.float32)
    return lfgen.Events(**{**ev.__dict__, "hit_z": hz.astype(np.float32), "hit_dxdy": hd.astype(np.float32)})


def _per_bucket(ev, e, fn):
    """Applies fn(bucket_slice_z, bucket_slice_dxdy) in place to each bucket of event e."""
    hz, hd = ev.hit_z.copy(), ev.hit_dxdy.copy()
    for k in range(24):
        f, n = int(ev.hit_off[24 * e + k]), int(ev.hit_off[24 * e + k + 1])
        if n > f:
            fn(k, hz[f:n], hd[f:n])
    return lfgen.Events(**{**ev.__dict__, "hit_z": hz, "hit_dxdy": hd})


def test_uniform_and_non_uniform_events_in_one_batch():
    """Events whose buckets each hold one z and one stereo slope stage only x
    per hit; the others read per-hit values.  One batch mixes: untouched
    events, one shifted per bucket (still uniform), ones where every hit but
    a bucket's first is moved (z, then slope), one with a single-ulp change
    on each bucket's last hit, and one fully jittered."""
    ev = lfgen.generate("nominal", n_events=6, seed=21)

    def shift(k, z, d):
        z += np.float32(0.25 * (k + 1))

    def tail_z(k, z, d):
        z[1:] += np.float32(2.0)

    def tail_slope(k, z, d):
        d[1:] *= np.float32(1.03)

    def last_ulp(k, z, d):
        z[-1] = np.nextafter(z[-1], np.float32(np.inf))

    for e, fn in ((1, shift), (2, tail_z), (3, tail_slope), (4, last_ulp)):
        ev = _per_bucket(ev, e, fn)
    jit = _jitter(lfgen.select_events(ev, [5]), 1.5, 0.02, seed=22)
    ev = lfgen.concat([lfgen.select_events(ev, range(5)), jit])
    _check_all_modes(ev, "nominal[6] uniform and non-uniform events")


def test_events_of_every_kind_in_one_batch():
    """One batch mixes nominal events, a stress event (41k hits, every window
    capped), an event with a single input track, a fully jittered event
    (per-hit z and stereo slopes), an event without tracks and a repeated
    nominal event, in both window sizes: every track's result equals the
    oracle's whatever its neighbours."""
    nom = lfgen.generate("nominal", n_events=5, seed=31)
    one = lfgen.select_events(lfgen.generate("nominal", n_events=1, seed=32), [0])
    keep = np.zeros(one.n_tracks, bool)
    keep[7] = True
    one = lfgen.Events(**{**one.__dict__, "trk_off": np.array([0, 1], np.uint32),
                          **{k: getattr(one, k)[keep] for k in ("trk_x", "trk_y", "trk_tx", "trk_ty", "trk_qop",
                                                               "trk_pid")}})
    z = np.zeros(0, np.float32)
    empty = lfgen.Events(**{**lfgen.select_events(nom, [0]).__dict__, "trk_off": np.zeros(2, np.uint32),
                            "trk_x": z, "trk_y": z, "trk_tx": z, "trk_ty": z, "trk_qop": z,
                            "trk_pid": np.zeros(0, np.int32)})
    stress = lfgen.generate("stress", n_events=1, seed=33)
    jit = _jitter(lfgen.generate("nominal", n_events=1, seed=34), 1.5, 0.02, seed=35)
    ev = lfgen.concat([nom, stress, one, jit, empty, lfgen.select_events(nom, [2])])
    for params in (None, {"n_hits_window": 64}):
        _check_all_modes(ev, "events of every kind", params)


@pytest.mark.parametrize("layers", [(8,), (11,), (0, 3, 8, 11)], ids=["layer8", "layer11", "layers0_3_8_11"])
def test_doublet_bracket_over_a_wide_z_range(layers):
    """Third-layer windows (layers 8 and 11) whose hits spread over +-60 mm in
    z: a hit's x on the track's line moves by the slope times its z offset,
    many millimetres, far beyond the doublet bracket's 0.5 mm padding, so the
    bracket must span the window's z range (corners of the slope and z
    intervals); one seed set's third window mixed and the other's common,
    and both mixed with mixed first layers."""
    ev = _jitter_layers(lfgen.generate("nominal", n_events=5, seed=41), layers, 60.0, 0.0, seed=42)
    _check_all_modes(ev, f"nominal[5] layers {layers} z+-60")


@pytest.mark.parametrize("n_hits_window", [64, 48, 32])
def test_per_hit_geometry_with_x_only_staging(n_hits_window):
    """Windows of more than 32 hits stage only x and read a mixed window's z
    and slopes from HBM: all layers mixed, and some layers mixed."""
    params = {"n_hits_window": n_hits_window}
    ev = _jitter(lfgen.generate("nominal", n_events=4), 1.5, 0.02, seed=13)
    _check_all_modes(ev, f"nominal[4] w{n_hits_window} per-hit z and slope", params)
    ev = _jitter_layers(lfgen.generate("nominal", n_events=4), (0, 5, 9, 11), 2.0, 0.03, seed=14)
    _check_all_modes(ev, f"nominal[4] w{n_hits_window} layers 0 5 9 11 mixed", params)
    _check_all_modes(ev, f"nominal[4] w{n_hits_window} layers 0 5 9 11 mixed, no-UT", dict(NO_UT, **params))


def test_inverted_windows():
    """Negative tolerances: high-momentum x windows have x_max < x_min
    (empty), the stereo windows have their centre outside the bounds."""
    ev = lfgen.generate("nominal", n_events=4)
    _check_all_modes(ev, "nominal[4] inverted", {"xtol_const": -120.0, "xasym": 300.0})
    _check_all_modes(ev, "nominal[4] inverted uv", {"uv_halfwidth": -2.0, "n_hits_window": 7})


@pytest.mark.parametrize("exec_cfg", [
    {"waves_per_block": 1}, {"waves_per_block": 4}, {"items_per_grab": 3}, {"items_per_grab": 16},
    {"blocks_per_cu": 1, "items_per_grab": 2}, {"blocks_per_cu": 40, "items_per_grab": 1},
], ids=lambda d: "-".join(f"{k}{v}" for k, v in d.items()))
def test_launch_configurations(exec_cfg):
    ev = lfgen.generate("nominal", n_events=6)
    ref = oracle.run(ev, W)
    for mode in ("batched", "persistent", "plain"):
        say(f"[gpu] exec {exec_cfg} mode={mode}")
        compare(ref, run_gpu(ev, mode, None, exec_cfg), label=f"exec/{mode}")


def test_full_nominal_batch():
    """The benchmarked workload (1,000 nominal events, batched mode), every slot."""
    ev = lfgen.generate("nominal")
    say(f"[gpu] full nominal batch events={ev.n_events} tracks={ev.n_tracks}")
    got = run_gpu(ev, "batched")
    ref = oracle.run(ev, W)
    st = compare(ref, got, label="nominal[1000]/batched")
    say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")


def test_work_counters_match_oracle():
    """The counting build's per-stage totals equal the oracle's intermediate counts."""
    from paper_2402_14670_amd import lf
    ev = lfgen.generate("nominal", n_events=10)
    o = oracle.run(ev, W, debug=True)
    n = (o["win"][:, :, 1] - o["win"][:, :, 0]).astype(np.int64)
    ctx = lf.lf_create(W)
    try:
        bid = lf.lf_upload_events(ctx, ev)
        say("[gpu] work counters, nominal[10]")
        wc = lf.lf_work_counts(ctx, bid)
        got = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks)
    finally:
        lf.lf_destroy(ctx)
    compare(oracle.run(ev, W), got, label="counting build")
    c = o["counts"]
    assert wc["tracks"] == ev.n_tracks
    assert wc["staged_hits"] == int(n.sum())
    assert wc["pairs_all"] == int((n[:, 0] * n[:, 8] + n[:, 3] * n[:, 11]).sum())
    assert wc["seed_items"] == int((n[:, 0] + n[:, 3]).sum())
    assert wc["doublets"] == int(c[:, 1].sum())
    assert wc["triplets"] == int(c[:, 2].sum())
    assert wc["kept"] == int(np.minimum(c[:, 2], 12).sum())
    assert wc["accepted"] == int(c[:, 3].sum())
    assert wc["found"] == int(o["found"].sum())
    assert wc["doublets"] <= wc["pairs_tested"] < wc["pairs_all"]
    say(f"    {wc}")


# ---- no-UT tuning: VELO-only input, two windows per layer, per-side seeding ----
NO_UT = {"velo_only": 1}


def test_no_ut_single_and_nominal():
    _check_all_modes(lfgen.generate("single"), "single no-UT", NO_UT)
    _check_all_modes(lfgen.generate("nominal", n_events=10), "nominal[10] no-UT", NO_UT)


def test_no_ut_stress_and_uneven():
    _check_all_modes(lfgen.generate("stress", n_events=2), "stress[2] no-UT", NO_UT)
    ev = lfgen.generate("uneven", n_events=40)
    parts = [lfgen.select_events(ev, range(0, 20)), lfgen.select_events(ev, []),
             lfgen.select_events(ev, range(20, 40))]
    _check_all_modes(lfgen.concat(parts), "uneven[40] no-UT", NO_UT)


@pytest.mark.parametrize("params", [
    {"n_hits_window": 32},
    {"n_hits_window": 17, "n_triplets": 5},
    {"noUT_overlap": 40.0, "n_triplets": 32, "T_triplet": 6.0},
    {"noUT_p_min": 3.0, "noUT_pt_min": 0.5, "magtol_max": 25.0, "magtol_const": 25.0, "magtol_min": 25.0},
], ids=["w32", "w17_t5", "overlap40_t32", "wide"])
def test_no_ut_parameter_variants(params):
    _check_all_modes(lfgen.generate("nominal", n_events=4), "nominal[4] no-UT", dict(NO_UT, **params))


def test_no_ut_whole_bucket_and_per_hit_geometry():
    ev = lfgen.generate("single", seed=7, n_events=6, n_particles=8, n_noise=20, p_min=1.5, p_max=20.0)
    big = dict(NO_UT, noUT_c=[1e9] * 8, noUT_overlap=1e7, uv_halfwidth=1e7, n_hits_window=64, n_triplets=7,
               T_triplet=40.0)
    _check_all_modes(ev, "tiny whole-bucket no-UT", big)
    ev = _jitter(lfgen.generate("nominal", n_events=4), 1.5, 0.02, seed=12)
    _check_all_modes(ev, "nominal[4] no-UT, per-hit z and slope", NO_UT)


def test_no_ut_work_counters_match_oracle():
    from paper_2402_14670_amd import lf
    ev = lfgen.generate("nominal", n_events=6)
    o = oracle.run(ev, W, NO_UT, debug=True)
    n0 = (o["win"][:, :, 1] - o["win"][:, :, 0]).astype(np.int64)
    n1 = (o["win1"][:, :, 1] - o["win1"][:, :, 0]).astype(np.int64)
    ctx = lf.lf_create(W, NO_UT)
    try:
        bid = lf.lf_upload_events(ctx, ev)
        say("[gpu] work counters, nominal[6] no-UT")
        wc = lf.lf_work_counts(ctx, bid)
        got = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks)
    finally:
        lf.lf_destroy(ctx)
    compare(oracle.run(ev, W, NO_UT), got, label="counting build no-UT")
    c = o["counts"]
    assert wc["staged_hits"] == int(n0.sum() + n1.sum())
    assert wc["pairs_all"] == int(sum((n[:, 0] * n[:, 8] + n[:, 3] * n[:, 11]).sum() for n in (n0, n1)))
    assert wc["seed_items"] == int(sum((n[:, 0] + n[:, 3]).sum() for n in (n0, n1)))
    assert wc["doublets"] == int(c[:, 1].sum())
    assert wc["triplets"] == int(c[:, 2].sum())
    assert wc["kept"] == int(np.minimum(c[:, 2], 20).sum())
    assert wc["accepted"] == int(c[:, 3].sum())
    assert wc["found"] == int(o["found"].sum())
    say(f"    {wc}")


def test_determinism_and_event_order():
    ev = lfgen.generate("nominal", n_events=8)
    say("[gpu] determinism: batched twice, then reversed event order")
    a = run_gpu(ev, "batched")
    b = run_gpu(ev, "batched")
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    order = list(range(ev.n_events))[::-1]
    rev = lfgen.select_events(ev, order)
    c = run_gpu(rev, "batched")
    for e_new, e_old in enumerate(order):
        r0, r1 = int(ev.trk_off[e_old]), int(ev.trk_off[e_old + 1])
        s0 = int(rev.trk_off[e_new])
        for k in a:
            assert np.array_equal(a[k][r0:r1], c[k][s0:s0 + r1 - r0]), k


def test_a_freed_batch_block_is_reused():
    """The device block of a fetched or released batch serves the next upload
    that fits it (at least its size, at most twice it): the results are those
    of a fresh block, every old content overwritten or unused.  An upload
    that does not fit gets a new block."""
    from paper_2402_14670_amd import lf
    big = lfgen.generate("nominal", n_events=20, seed=51)
    mid = lfgen.generate("nominal", n_events=14, seed=52)
    small = lfgen.generate("nominal", n_events=2, seed=53)
    ctx = lf.lf_create(W)
    try:
        say("[gpu] block reuse: nominal[20], then nominal[14] in its block, then nominal[2] in a new one")
        bid = lf.lf_upload_events(ctx, big)
        size_big = lf.lf_batch_info(ctx, bid)["device_bytes"]
        lf.lf_find_tracks(ctx, bid, "batched")
        compare(oracle.run(big, W), lf.lf_fetch_tracks(ctx, bid), label="first block")
        sizes = []
        for ev, mode in ((mid, "batched"), (small, "persistent"), (small, "plain")):
            bid = lf.lf_upload_events(ctx, ev)
            sizes.append(lf.lf_batch_info(ctx, bid)["device_bytes"])
            lf.lf_find_tracks(ctx, bid, mode)
            compare(oracle.run(ev, W), lf.lf_copy_tracks(ctx, bid), label=f"{ev.n_events} events, {mode}")
            lf.lf_release_batch(ctx, bid)
            assert lf.lf_device_bytes_in_use(ctx) == 0
        # nominal[14] in the block of nominal[20]; nominal[2] (under half of
        # it) in a new block, which the second nominal[2] reuses
        assert sizes[0] == size_big and sizes[1] < size_big // 2 and sizes[2] == sizes[1]
    finally:
        lf.lf_destroy(ctx)


def test_kept_block_within_the_device_budget():
    """Under a device budget: a kept block that does not fit the next upload
    is freed before the new allocation, two batches that fit the budget
    together stay resident, the kept block of one of them is reused, and an
    upload over the budget fails with LF_ERR_TOO_LARGE, leaving the resident
    batches as they were."""
    from paper_2402_14670_amd import lf
    big = lfgen.generate("nominal", n_events=20, seed=61)
    small = lfgen.generate("nominal", n_events=2, seed=63)
    probe = lf.lf_create(W)
    try:
        size_big = lf.lf_batch_info(probe, lf.lf_upload_events(probe, big))["device_bytes"]
        size_small = lf.lf_batch_info(probe, lf.lf_upload_events(probe, small))["device_bytes"]
    finally:
        lf.lf_destroy(probe)
    assert size_small < size_big // 2
    ref_big, ref_small = oracle.run(big, W), oracle.run(small, W)
    ctx = lf.lf_create(W, None, size_big + size_small + size_big // 20)
    try:
        say("[gpu] kept block under a budget of both batches plus 5%")
        bid = lf.lf_upload_events(ctx, big)
        lf.lf_find_tracks(ctx, bid, "batched")
        compare(ref_big, lf.lf_fetch_tracks(ctx, bid), label="budget: big")
        bs = lf.lf_upload_events(ctx, small)                  # the kept block is too large: freed
        assert lf.lf_batch_info(ctx, bs)["device_bytes"] == size_small
        bb = lf.lf_upload_events(ctx, big)                    # fits beside the small batch
        assert lf.lf_device_bytes_in_use(ctx) == size_small + size_big
        lf.lf_release_batch(ctx, bb)                          # kept
        bb = lf.lf_upload_events(ctx, big)                    # the kept block, reused
        assert lf.lf_batch_info(ctx, bb)["device_bytes"] == size_big
        with pytest.raises(lf.LFError) as e:
            lf.lf_upload_events(ctx, small)                   # over the budget
        assert e.value.code == lf.LF_ERR_TOO_LARGE
        assert lf.lf_device_bytes_in_use(ctx) == size_small + size_big
        for b_, ref, mode in ((bs, ref_small, "persistent"), (bb, ref_big, "batched")):
            lf.lf_find_tracks(ctx, b_, mode)
            compare(ref, lf.lf_fetch_tracks(ctx, b_), label=f"budget: {mode}")
        assert lf.lf_device_bytes_in_use(ctx) == 0
    finally:
        lf.lf_destroy(ctx)


def test_torch_stream():
    import torch
    ev = lfgen.generate("nominal", n_events=4)
    ref = oracle.run(ev, W)
    s = torch.cuda.Stream()
    say("[gpu] batched on a torch stream")
    got = run_gpu(ev, "batched", stream=s.cuda_stream)
    compare(ref, got, label="torch-stream")


def test_error_codes():
    from paper_2402_14670_amd import lf
    ev = lfgen.generate("nominal", n_events=2)
    say("[gpu] error codes")
    ctx = lf.lf_create(W, None, budget_bytes=1024)
    try:
        with pytest.raises(lf.LFError) as e:
            lf.lf_upload_events(ctx, ev)
        assert e.value.code == lf.LF_ERR_TOO_LARGE
        with pytest.raises(lf.LFError) as e:
            lf.lf_find_tracks(ctx, 12345, "batched")
        assert e.value.code == lf.LF_ERR_STATE
    finally:
        lf.lf_destroy(ctx)
    ctx = lf.lf_create(W)
    try:
        bid = lf.lf_upload_events(ctx, ev)
        with pytest.raises(lf.LFError) as e:
            lf.lf_find_tracks(ctx, bid, 7)
        assert e.value.code == lf.LF_ERR_INVALID
        lf.lf_find_tracks(ctx, bid, "batched")
        with pytest.raises(lf.LFError) as e:
            lf.lf_fetch_tracks(ctx, bid, ev.n_tracks - 1)
        assert e.value.code == lf.LF_ERR_INVALID
        out = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks)   # the batch is still resident
        assert out["found"].sum() > 0
        with pytest.raises(lf.LFError) as e:
            lf.lf_fetch_tracks(ctx, bid, ev.n_tracks)     # fetched batches are freed
        assert e.value.code == lf.LF_ERR_STATE
        assert lf.lf_device_bytes_in_use(ctx) == 0
    finally:
        lf.lf_destroy(ctx)
    with pytest.raises(lf.LFError) as e:
        lf.lf_create(W, {"n_triplets": 33})
    assert e.value.code == lf.LF_ERR_INVALID
    # geometry: unknown momentum form, non-finite F coefficient, zero kick in the linear form
    for bad in (dict(W, field_form=2), dict(lfgen.world("paper"), F_coef=[float("nan")] + [0.0] * 49),
                dict(W, kick=0.0)):
        with pytest.raises(lf.LFError) as e:
            lf.lf_create(bad)
        assert e.value.code == lf.LF_ERR_INVALID
    lf.lf_destroy(lf.lf_create(dict(lfgen.world("paper"), kick=0.0)))   # the paper form does not use kick


@pytest.mark.parametrize("mode", ["batched", "persistent", "plain"])
def test_graph_replays(mode):
    """A captured sequence of three batches replays identically: each replay
    follows a poison of every result slot and eager work on another batch."""
    from paper_2402_14670_amd import lf
    parts = [lfgen.generate("uneven", n_events=30, first_event=30 * i) for i in range(3)]
    other = lfgen.generate("nominal", n_events=5)
    refs = [oracle.run(p, W) for p in parts]
    ctx = lf.lf_create(W)
    try:
        ids = [lf.lf_upload_events(ctx, p) for p in parts]
        oid = lf.lf_upload_events(ctx, other)
        say(f"[gpu] graph capture mode={mode} of {len(ids)} uneven batches")
        g = lf.lf_graph_create(ctx, ids, mode)
        try:
            for rep in range(3):
                for i in ids:
                    lf.lf_poison_tracks(ctx, i)
                lf.lf_graph_launch(ctx, g)
                lf.lf_find_tracks(ctx, oid, "batched")          # eager work between replays
                for i, p, r in zip(ids, parts, refs):
                    compare(r, lf.lf_copy_tracks(ctx, i, p.n_tracks), label=f"graph/{mode}/replay{rep}")
        finally:
            lf.lf_graph_destroy(g)
    finally:
        lf.lf_destroy(ctx)


@pytest.mark.parametrize("mode", ["batched", "persistent"])
def test_graph_with_a_batch_named_twice(mode):
    """A capture list that names a batch twice is recorded in order (the two
    launches of that batch must not overlap: in persistent mode they share
    its queue words); every replay matches the oracle."""
    from paper_2402_14670_amd import lf
    parts = [lfgen.generate("uneven", n_events=20, first_event=20 * i) for i in range(2)]
    refs = [oracle.run(p, W) for p in parts]
    ctx = lf.lf_create(W)
    try:
        ids = [lf.lf_upload_events(ctx, p) for p in parts]
        say(f"[gpu] graph capture mode={mode} of batches {ids[0]}, {ids[1]}, {ids[0]}")
        g = lf.lf_graph_create(ctx, [ids[0], ids[1], ids[0]], mode)
        try:
            for rep in range(3):
                for i in ids:
                    lf.lf_poison_tracks(ctx, i)
                lf.lf_graph_launch(ctx, g)
                for i, p, r in zip(ids, parts, refs):
                    compare(r, lf.lf_copy_tracks(ctx, i, p.n_tracks), label=f"graph-twice/{mode}/replay{rep}")
        finally:
            lf.lf_graph_destroy(g)
        # the queue words were left clean: an eager persistent launch still matches
        lf.lf_poison_tracks(ctx, ids[0])
        lf.lf_find_tracks(ctx, ids[0], "persistent")
        compare(refs[0], lf.lf_copy_tracks(ctx, ids[0], parts[0].n_tracks), label=f"graph-twice/{mode}/after")
    finally:
        lf.lf_destroy(ctx)


def test_autotuner_keeps_results():
    import torch
    from paper_2402_14670_amd import autotune, lf
    ev = lfgen.generate("uneven", n_events=200)
    ref = oracle.run(ev, W, events=(0, 40))
    ctx = lf.lf_create(W)
    try:
        bid = lf.lf_upload_events(ctx, ev)
        s = torch.cuda.Stream()
        say("[gpu] autotune on uneven[200]")
        res = autotune.autotune(ctx, bid, s, steps=2)
        say(f"    best {res['best']}")
        assert len(res["table"]) == len(autotune.candidates())
        lf.lf_poison_tracks(ctx, bid)
        lf.lf_find_tracks(ctx, bid, res["best"]["mode"])
        got = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks)
    finally:
        lf.lf_destroy(ctx)
    rows = np.arange(int(ev.trk_off[40]))
    compare(ref, got, rows=rows, label="autotuned")


@pytest.mark.parametrize("variant", ["no_ut", "paper", "fp16"])
def test_variant_builds_in_graphs_and_counting(variant):
    """The no-UT, paper-form and binary16 builds replayed from a captured
    graph (persistent mode, whose queue words reset themselves) match the
    oracle on every replay, and their counting builds rewrite identical
    results with consistent totals."""
    from paper_2402_14670_amd import lf
    field = "paper" if variant == "paper" else "toy"
    world = lfgen.world(field)
    params = {"no_ut": {"velo_only": 1}, "paper": None, "fp16": {"seed_fp16": 1}}[variant]
    parts = [lfgen.generate("nominal", field=field, n_events=8, first_event=8 * i) for i in range(2)]
    refs = [oracle.run(p, world, params) for p in parts]
    ctx = lf.lf_create(world, params)
    try:
        ids = [lf.lf_upload_events(ctx, p) for p in parts]
        say(f"[gpu] {variant}: graph of {len(ids)} batches, persistent mode")
        g = lf.lf_graph_create(ctx, ids, "persistent")
        try:
            for rep in range(2):
                for i in ids:
                    lf.lf_poison_tracks(ctx, i)
                lf.lf_graph_launch(ctx, g)
                for i, p, r in zip(ids, parts, refs):
                    compare(r, lf.lf_copy_tracks(ctx, i, p.n_tracks), label=f"{variant}/graph/replay{rep}")
        finally:
            lf.lf_graph_destroy(g)
        say(f"[gpu] {variant}: counting build")
        wc = lf.lf_work_counts(ctx, ids[0])
        compare(refs[0], lf.lf_copy_tracks(ctx, ids[0], parts[0].n_tracks), label=f"{variant}/counting")
        assert wc["tracks"] == parts[0].n_tracks
        assert wc["found"] == int(refs[0]["found"].sum())
        assert wc["doublets"] <= wc["pairs_tested"] and wc["kept"] <= wc["triplets"]
        assert wc["accepted"] <= wc["fitted"] <= wc["kept"]
    finally:
        lf.lf_destroy(ctx)

"""Every output slot of the full uneven (20,000 events) and stress (5,000
events) workloads, and of the nominal batch on the general path (per-hit z
and slopes), in the launch configurations the benchmark times, against
the oracle run over the whole batch on the host's threads.  The stress batch
is the one that drives the exact top-n selection hardest (hundreds of
triplets per input track); the uneven batch is also run as four resident
sub-batches replayed from one captured HIP graph, and through the serving
loop."""
import numpy as np
import pytest

import lfgen
from parity import W, compare, event_digests, oracle_parallel, run_gpu, say

pytestmark = pytest.mark.gpu


def test_full_uneven_batch_every_slot():
    from paper_2402_14670_amd import lf
    ev = lfgen.generate("uneven")
    say(f"[gpu] uneven[{ev.n_events}] tracks={ev.n_tracks} hits={ev.n_hits}: oracle on the host")
    ref = oracle_parallel(ev)
    for mode in ("batched", "persistent"):
        say(f"[gpu] uneven[{ev.n_events}] mode={mode}")
        st = compare(ref, run_gpu(ev, mode), label=f"uneven[{ev.n_events}]/{mode}")
        say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")
    # four resident sub-batches replayed from one graph, every slot compared
    cuts = [ev.n_events * k // 4 for k in range(5)]
    parts = [lfgen.select_events(ev, range(cuts[k], cuts[k + 1])) for k in range(4)]
    rows = [np.arange(int(ev.trk_off[cuts[k]]), int(ev.trk_off[cuts[k + 1]])) for k in range(4)]
    ctx = lf.lf_create(W)
    try:
        ids = [lf.lf_upload_events(ctx, p) for p in parts]
        say(f"[gpu] uneven[{ev.n_events}] as 4 sub-batches from one graph")
        g = lf.lf_graph_create(ctx, ids, "batched")
        try:
            for rep in range(2):
                for i in ids:
                    lf.lf_poison_tracks(ctx, i)
                lf.lf_graph_launch(ctx, g)
                for k, (i, p) in enumerate(zip(ids, parts)):
                    got = lf.lf_copy_tracks(ctx, i, p.n_tracks)
                    compare({key: v[rows[k]] for key, v in ref.items()}, got, label=f"uneven graph {k}/replay{rep}")
        finally:
            lf.lf_graph_destroy(g)
    finally:
        lf.lf_destroy(ctx)


def test_full_stress_batch_every_slot():
    ev = lfgen.generate("stress")
    say(f"[gpu] stress[{ev.n_events}] tracks={ev.n_tracks} hits={ev.n_hits}: oracle on the host")
    ref = oracle_parallel(ev)
    say(f"[gpu] stress[{ev.n_events}] mode=batched")
    st = compare(ref, run_gpu(ev, "batched"), label=f"stress[{ev.n_events}]/batched")
    say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")


def test_full_nominal_general_path_every_slot():
    """The general path at the size it is timed at: the whole nominal batch
    with every hit's z jittered by +-1.5 mm and every stereo slope by +-2%
    (uniform, seed 11, the benchmark's recipe), so that no window shares one
    z or one slope; every slot against the oracle, with one wavefront per
    block as the benchmark's autotuner picks."""
    ev = lfgen.generate("nominal")
    rng = np.random.default_rng(11)
    hz = (ev.hit_z + rng.uniform(-1.5, 1.5, ev.n_hits)).astype(np.float32)
    hd = (ev.hit_dxdy * (1.0 + rng.uniform(-0.02, 0.02, ev.n_hits))).astype(np.float32)
    gev = lfgen.Events(**{**ev.__dict__, "hit_z": hz, "hit_dxdy": hd})
    say(f"[gpu] nominal[{gev.n_events}] per-hit z and slopes: oracle on the host")
    ref = oracle_parallel(gev)
    say(f"[gpu] nominal[{gev.n_events}] per-hit z and slopes, mode=batched, one wavefront per block")
    st = compare(ref, run_gpu(gev, "batched", exec_cfg={"waves_per_block": 1}), label="general path, full nominal")
    say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")


def test_stress_events_served():
    """Stress events through the serving loop (open-loop arrivals, continuous
    batching): each request's result equals the oracle's for its event alone."""
    from paper_2402_14670_amd import lf
    ev = lfgen.generate("stress", n_events=120, first_event=4000)
    ref = event_digests(oracle_parallel(ev), ev.trk_off)
    rng = np.random.default_rng(45)
    req = rng.integers(0, ev.n_events, size=1500).astype(np.uint32)
    arr = np.cumsum(rng.exponential(1.0 / 40000.0, size=len(req)))
    ctx = lf.lf_create(W)
    try:
        say(f"[gpu] serving stress pool={ev.n_events} requests={len(req)}")
        dig, lat, st = lf.lf_serve_run(ctx, ev, req, arr, {"max_batch_events": 64, "n_slots": 2})
    finally:
        lf.lf_destroy(ctx)
    say(f"    {st}")
    bad = np.nonzero(dig != ref[req])[0]
    assert len(bad) == 0, f"{len(bad)} requests differ from the oracle, first {bad[:5]}"

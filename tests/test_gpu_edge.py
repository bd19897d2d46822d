"""GPU parity on edge cases of the inputs: equal x values everywhere (ties in
every search and in the triplet keys), duplicated hits, a hand-built event
whose triplets all have chi2 = 0, and one very large event (buckets of
~12k hits: deep searches, every window capped)."""
import numpy as np
import pytest

import lfgen
import oracle
import pins
from parity import W, compare, run_gpu, say

pytestmark = pytest.mark.gpu
MODES = ("plain", "batched", "persistent")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _check(ev, label, params=None, world=None, modes=MODES):
    world = W if world is None else world
    ref = oracle.run(ev, world, params)
    for mode in modes:
        say(f"[gpu] edge {label}: mode={mode} events={ev.n_events} tracks={ev.n_tracks} hits={ev.n_hits} "
            f"params={params}")
        st = compare(ref, run_gpu(ev, mode, params, world=world), label=f"{label}/{mode}")
        say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")


def _quantised(ev, step):
    """x rounded to multiples of `step` mm: buckets stay sorted, with runs of equal x."""
    x = (np.round(ev.hit_x.astype(np.float64) / step) * step).astype(np.float32)
    return lfgen.Events(**{**ev.__dict__, "hit_x": x})


def _duplicated(ev):
    """Every hit twice, adjacent in its bucket."""
    n = ev.n_hits
    idx = np.repeat(np.arange(n), 2)
    d = {k: getattr(ev, k)[idx] for k in ("hit_x", "hit_z", "hit_dxdy", "hit_pid")}
    return lfgen.Events(**{**ev.__dict__, **d, "hit_off": (ev.hit_off.astype(np.int64) * 2).astype(np.uint32)})


@pytest.mark.parametrize("step", [1.0, 4.0])
def test_equal_x_runs(step):
    ev = _quantised(lfgen.generate("nominal", n_events=4), step)
    _check(ev, f"nominal[4] x in {step} mm steps")
    _check(ev, f"nominal[4] x in {step} mm steps, no-UT", {"velo_only": 1}, modes=("batched",))


def test_duplicated_hits():
    ev = _duplicated(lfgen.generate("nominal", n_events=3))
    _check(ev, "nominal[3] duplicated hits")
    _check(ev, "nominal[3] duplicated hits, w64", {"n_hits_window": 64}, modes=("batched",))


def test_all_triplets_tie():
    hits = {(l, 1): [100.0] for l in pins.X_LAYERS}
    for l in (0, 4, 8):
        hits[(l, 1)] = [100.0, 100.0]
    ev = pins.make_event(hits, [(100.0, 270.0, 0.0, 0.1, 1.0 / 50.0)])
    _check(ev, "chi2 = 0 everywhere", {"K_first": 1.0, "K_last": 1.0, "n_triplets": 8})


def test_one_very_large_event():
    ev = lfgen.generate("single", seed=21, n_particles=1500, n_noise=280000, n_true_tracks=60, n_fake_tracks=20,
                        p_min=1.5, p_max=50.0)
    sizes = np.diff(ev.hit_off.astype(np.int64))
    say(f"[gpu] large event: {ev.n_hits} hits, largest bucket {sizes.max()}")
    assert sizes.max() > 10000
    _check(ev, "one event of ~290k hits")
    _check(ev, "one event of ~290k hits, w64 t32", {"n_hits_window": 64, "n_triplets": 32}, modes=("batched",))

"""GPU parity of the binary16 triplet seeding (seed_fp16 = 1): the packed
half-precision doublet filters and middle-hit search against the oracle's
binary16 seeding on the same seeded inputs (a parity domain of its own:
indices and flags bit-exact, parameters within 1e-5 relative)."""
import numpy as np
import pytest

import lfgen
import oracle
from parity import W, compare, oracle_on_events, run_gpu, say

pytestmark = pytest.mark.gpu
MODES = ("plain", "batched", "persistent")
FP16 = {"seed_fp16": 1}


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _check(ev, label, params=FP16, world=None, modes=MODES):
    world = W if world is None else world
    ref = oracle.run(ev, world, params)
    for mode in modes:
        say(f"[gpu] fp16 seeding {label}: mode={mode} events={ev.n_events} tracks={ev.n_tracks} params={params}")
        st = compare(ref, run_gpu(ev, mode, params, world=world), label=f"{label}/{mode}")
        say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")


def test_fp16_single_nominal_stress():
    _check(lfgen.generate("single"), "single")
    _check(lfgen.generate("nominal", n_events=20), "nominal[20]")
    _check(lfgen.generate("stress", n_events=3), "stress[3]")


def test_fp16_full_nominal_and_sampled_uneven():
    ev = lfgen.generate("nominal")
    say("[gpu] fp16 seeding nominal[1000] batched")
    compare(oracle.run(ev, W, FP16), run_gpu(ev, "batched", FP16), label="fp16 nominal[1000]")
    ev = lfgen.generate("uneven", n_events=2000)
    events = np.sort(np.random.default_rng(4).choice(2000, size=100, replace=False))
    say("[gpu] fp16 seeding uneven[2000] batched, oracle on 100 sampled events")
    ref, rows = oracle_on_events(ev, events, FP16)
    compare(ref, run_gpu(ev, "batched", FP16), rows=rows, label="fp16 uneven[2000]")


@pytest.mark.parametrize("extra", [
    {"n_hits_window": 64, "n_triplets": 32}, {"n_hits_window": 7, "n_triplets": 3},
    {"K_first": 1.01, "K_last": 1.01, "T_triplet": 100.0}, {"p_charge_cut": 50.0},
], ids=["w64_t32", "w7_t3", "K1.01", "charge_filter_everywhere"])
def test_fp16_parameter_variants(extra):
    _check(lfgen.generate("nominal", n_events=4), "nominal[4]", dict(FP16, **extra), modes=("batched", "plain"))


def test_fp16_mixed_windows_and_paper_field():
    """Mixed-z windows fall back to binary32 per set; the paper-form kick
    feeds the window centres."""
    ev = lfgen.generate("nominal", n_events=4)
    rng = np.random.default_rng(15)
    sel = np.isin(ev.hit_z, np.array([lfgen.LAYER_Z[l] for l in (0, 11)], np.float32))
    hz = (ev.hit_z + np.where(sel, rng.uniform(-3.0, 3.0, ev.n_hits), 0.0)).astype(np.float32)
    _check(lfgen.Events(**{**ev.__dict__, "hit_z": hz}), "nominal[4] layers 0 and 11 mixed")
    _check(lfgen.generate("nominal", field="paper", n_events=6), "paper field nominal[6]", world=lfgen.world("paper"))


def test_fp16_rejected_with_velo_only():
    from paper_2402_14670_amd import lf
    with pytest.raises(lf.LFError) as e:
        lf.lf_create(W, {"seed_fp16": 1, "velo_only": 1})
    assert e.value.code == lf.LF_ERR_INVALID


@pytest.mark.parametrize("step", [0.25, 4.0])
def test_fp16_equal_x_runs_and_duplicates(step):
    """Runs of equal x (and so of equal binary16 offsets and distances) and
    duplicated hits: the middle-hit searches must return the first minimum
    of a scan, as the oracle's linear scan does."""
    ev = lfgen.generate("nominal", n_events=4)
    x = (np.round(ev.hit_x.astype(np.float64) / step) * step).astype(np.float32)
    _check(lfgen.Events(**{**ev.__dict__, "hit_x": x}), f"nominal[4] x in {step} mm steps", modes=("batched",))
    idx = np.repeat(np.arange(ev.n_hits), 2)
    d = {k: getattr(ev, k)[idx] for k in ("hit_x", "hit_z", "hit_dxdy", "hit_pid")}
    dup = lfgen.Events(**{**ev.__dict__, **d, "hit_off": (ev.hit_off.astype(np.int64) * 2).astype(np.uint32)})
    _check(dup, "nominal[4] duplicated hits", modes=("batched",))

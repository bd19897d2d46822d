"""GPU parity in the paper-form field: the sqrt-normalised pt-kick solved for
the windows and the momentum from the fourth-order parametrisation
F(tx, ty, dSlope) with the fitted coefficient table, against the CPU oracle
on the same seeded inputs (indices and flags bit-exact, parameters within
1e-5 relative)."""
import copy

import numpy as np
import pytest

import lfgen
import oracle
from parity import compare, oracle_on_events, run_gpu, say

pytestmark = pytest.mark.gpu
MODES = ("plain", "batched", "persistent")
W_PAPER = lfgen.world("paper")
F_CONST = [lfgen.KICK] + [0.0] * 49


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _check(ev, world, label, params=None, modes=MODES):
    ref = oracle.run(ev, world, params)
    for mode in modes:
        say(f"[gpu] paper field {label}: mode={mode} events={ev.n_events} tracks={ev.n_tracks} "
            f"hits={ev.n_hits} params={params}")
        st = compare(ref, run_gpu(ev, mode, params, world=world), label=f"{label}/{mode}")
        say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")


def test_paper_field_workloads():
    _check(lfgen.generate("single", field="paper"), W_PAPER, "single")
    _check(lfgen.generate("nominal", field="paper", n_events=20), W_PAPER, "nominal[20]")
    _check(lfgen.generate("stress", field="paper", n_events=3), W_PAPER, "stress[3]")


def test_paper_field_full_nominal_and_sampled_uneven():
    ev = lfgen.generate("nominal", field="paper")
    say(f"[gpu] paper field nominal[1000] batched, tracks={ev.n_tracks}")
    st = compare(oracle.run(ev, W_PAPER), run_gpu(ev, "batched", world=W_PAPER), label="paper nominal[1000]")
    say(f"    found={st['found']} bit-exact params {st['bit_exact_params']}/{st['params']}")
    ev = lfgen.generate("uneven", field="paper", n_events=2000)
    events = np.sort(np.random.default_rng(3).choice(2000, size=100, replace=False))
    say("[gpu] paper field uneven[2000] batched, oracle on 100 sampled events")
    ref, rows = oracle_on_events(ev, events, world=W_PAPER)
    compare(ref, run_gpu(ev, "batched", world=W_PAPER), rows=rows, label="paper uneven[2000]")


def test_constant_integral_and_single_term_tables():
    """The constant-integral field read with F = 1.2 and with one extra term
    of the table at a time (each power of dSlope, several monomials)."""
    ev = lfgen.generate("single", field="kick", seed=11, sigma_x=0.0, qop_sigma=0.0, hit_eff=1.0, n_noise=0,
                        p_min=1.5, p_max=50.0, n_particles=120)
    world = lfgen.world("kick", F_coef=F_CONST)
    _check(ev, world, "kick F=const")
    for i, j, w in ((0, 7, 40.0), (1, 4, 3.0), (2, 9, -200.0), (3, 0, 0.5), (4, 3, 30.0)):
        coef = list(F_CONST)
        coef[10 * i + j] += w
        _check(ev, dict(world, F_coef=coef), f"kick F_coef[{i}][{j}]+={w}", modes=("batched",))


def test_kicks_without_solution():
    """Tracks whose kick no slope can carry get no track; the rest are unaffected."""
    ev = copy.deepcopy(lfgen.generate("nominal", field="paper", n_events=4))
    t = np.arange(0, ev.n_tracks, 3)
    ev.trk_qop[t] = np.where(ev.trk_tx[t] >= 0, 1.25, -1.25).astype(np.float32)
    _check(ev, W_PAPER, "nominal[4] impossible kicks")


def test_paper_field_parameter_and_geometry_variants():
    ev = lfgen.generate("nominal", field="paper", n_events=4)
    _check(ev, W_PAPER, "nominal[4] w64_t32", {"n_hits_window": 64, "n_triplets": 32}, modes=("batched",))
    _check(ev, dict(W_PAPER, polarity=-1), "nominal[4] polarity -1", modes=("batched",))
    _check(ev, dict(W_PAPER, dRatio=0.0), "nominal[4] dRatio 0", modes=("batched",))


def test_paper_field_no_ut_momentum():
    """VELO-only input in the paper field: straight windows, q/p from F."""
    _check(lfgen.generate("nominal", field="paper", n_events=6), W_PAPER, "nominal[6] no-UT", {"velo_only": 1})

"""Synthetic input generator: layout, determinism and workload shapes."""
import numpy as np

import lfgen


def test_layout_sorted_and_zoned():
    ev = lfgen.generate("nominal", n_events=3)
    assert ev.hit_off[0] == 0 and ev.hit_off[-1] == len(ev.hit_x)
    assert np.all(np.diff(ev.hit_off.astype(np.int64)) >= 0)
    for b in range(24 * ev.n_events):
        x = ev.hit_x[ev.hit_off[b]:ev.hit_off[b + 1]]
        assert np.all(np.diff(x) >= 0)
        layer = (b % 24) // 2
        assert np.all(ev.hit_z[ev.hit_off[b]:ev.hit_off[b + 1]] == np.float32(lfgen.LAYER_Z[layer]))


def test_deterministic_and_event_independent():
    a = lfgen.generate("nominal", n_events=4)
    b = lfgen.generate("nominal", n_events=4)
    for k in ("hit_x", "hit_off", "trk_qop", "trk_x"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    # event 2 of the stream is the same whether generated alone or with others
    c = lfgen.generate("nominal", n_events=1, first_event=2)
    d = lfgen.select_events(a, [2])
    for k in ("hit_x", "hit_off", "hit_pid", "trk_qop", "trk_pid", "par_p"):
        assert np.array_equal(getattr(c, k), getattr(d, k)), k


def test_workload_shapes():
    s = lfgen.generate("single")
    assert s.n_tracks == 40 and 450 < s.n_hits < 700
    n = lfgen.generate("nominal", n_events=5)
    assert 5000 < n.n_hits / 5 < 6000 and n.n_tracks == 1000
    assert (n.trk_pid < 0).sum() == 150
    st = lfgen.generate("stress", n_events=1)
    assert 35000 < st.n_hits < 48000 and st.n_tracks == 486
    u = lfgen.generate("uneven", n_events=200)
    per = np.diff(u.hit_off[::24].astype(np.int64))
    assert per.min() < 3000 and per.max() > 9000


def test_truth_hits_match_toy_field():
    """Noise-free hits lie on the toy trajectory at every layer."""
    ev = lfgen.generate("single", sigma_x=0.0, n_noise=0, hit_eff=1.0)
    for g in range(len(ev.hit_x)):
        pid = ev.hit_pid[g]
        p, q, tx, ty = (float(a[pid]) for a in (ev.par_p, ev.par_q, ev.par_tx, ev.par_ty))
        z = float(ev.hit_z[g])
        layer = lfgen.LAYER_Z.index(z)
        dtx = lfgen.KICK * q / p
        x = tx * lfgen.Z_MAG + (tx + dtx) * (z - lfgen.Z_MAG) + lfgen.KAPPA * dtx * (z - lfgen.Z_T) ** 2
        assert abs(ev.hit_x[g] - (x - lfgen.LAYER_DXDY[layer] * ty * z)) < 1e-3

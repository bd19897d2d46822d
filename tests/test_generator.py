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


def _sine(tx, ty):
    return tx / np.sqrt(1.0 + tx * tx + ty * ty)


def test_paper_field_hits_follow_the_pt_kick():
    """Paper field: noise-free hits lie on a trajectory whose slope after the
    kick satisfies the sqrt-normalised pt-kick equation with the world's
    integrated field, and whose tail has the falling-field cubic term."""
    ev = lfgen.generate("single", field="paper", sigma_x=0.0, n_noise=0, hit_eff=1.0, p_min=1.5)
    fc = lfgen.FIELDS["paper"]
    zT = fc["z_T"]
    for g in range(len(ev.hit_x)):
        pid = ev.hit_pid[g]
        p, q, tx, ty = (float(a[pid]) for a in (ev.par_p, ev.par_q, ev.par_tx, ev.par_ty))
        bl = fc["bl0"] * (1 + fc["bl_tx2"] * tx * tx + fc["bl_ty2"] * ty * ty + fc["bl_q2"] * (fc["bl0"] * q / p) ** 2)
        sf = _sine(tx, ty) + q / p * bl
        txf = sf * np.sqrt((1 + ty * ty) / (1 - sf * sf))
        z = float(ev.hit_z[g])
        layer = lfgen.LAYER_Z.index(z)
        d = txf - tx
        x = tx * lfgen.Z_MAG + txf * (z - lfgen.Z_MAG) + lfgen.KAPPA * d * (z - zT) ** 2 * (1 + fc["dRatio"] * (z - zT))
        assert abs(ev.hit_x[g] - (x - lfgen.LAYER_DXDY[layer] * ty * z)) < 1e-3


def test_paper_field_soft_particles_curl_up():
    """A particle whose kick exceeds what any slope can carry leaves no hit."""
    tx = np.array([0.2, -0.2, 0.1])
    qop = np.array([1.0, -1.0, 0.3])
    d, bl, ok = lfgen.kick(tx, np.zeros(3), qop, "paper")
    assert list(ok) == [False, False, True]


def test_field_table_reproduces_the_integrated_field():
    """The fitted momentum parametrisation F(tx, ty, dSlope) matches the
    world's integrated field on a fresh sample over the acceptance (rms
    below 3e-4 relative, worst case below 3e-3), has the symmetry-allowed
    layout (odd rows: six terms), and is the constant kick for the
    constant-integral field."""
    t = np.array(lfgen.field_table("paper")).reshape(5, 10)
    assert not t[1, 6:].any() and not t[3, 6:].any()
    rng = np.random.default_rng(123)
    n = 50_000
    tx, ty = rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n)
    qop = rng.uniform(-1 / 1.5, 1 / 1.5, n)
    d, bl, ok = lfgen.kick(tx, ty, qop, "paper")
    zT = lfgen.FIELDS["paper"]["z_T"]
    dR = lfgen.FIELDS["paper"]["dRatio"]
    for z in (lfgen.LAYER_Z[0], lfgen.LAYER_Z[-1]):
        x = tx * lfgen.Z_MAG + (tx + d) * (z - lfgen.Z_MAG) + lfgen.KAPPA * d * (z - zT) ** 2 * (1 + dR * (z - zT))
        ok &= (np.abs(x) < 3000.0) & (np.abs(ty * z) < 2500.0)
    tx, ty, d, bl = tx[ok], ty[ok], d[ok], bl[ok]
    c = []
    for i in range(5):
        acc = np.zeros_like(tx)
        exps = ((0, 0), (2, 0), (0, 2), (4, 0), (2, 2), (0, 4), (6, 0), (4, 2), (2, 4), (0, 6))
        for j in range(10 if i % 2 == 0 else 6):
            k, m = exps[j]
            acc += t[i, j] * tx ** (k + i % 2) * ty ** m
        c.append(acc)
    F = c[0] + d * (c[1] + d * (c[2] + d * (c[3] + d * c[4])))
    rel = F / bl - 1.0
    assert np.sqrt(np.mean(rel ** 2)) < 3e-4 and np.abs(rel).max() < 3e-3
    k = np.array(lfgen.field_table("kick")).reshape(5, 10)
    assert abs(k[0, 0] - lfgen.KICK) < 1e-6 and np.abs(k.ravel()[1:]).max() < 1e-6

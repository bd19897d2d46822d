"""Planted mistakes in copies of the CPU oracle: each must fail a pin.

Every mutant is a small plausible slip (a dropped term, a wrong sign, a
swapped constant, an off-by-one) applied to a temporary copy of oracle/lfo.c,
compiled on the CPU, and run through the pins of tests/pins.py.  A mutant
that passes every pin would show a blind spot in the pins.
"""
import os
import shutil
import subprocess

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lfo.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "lfo.h")

MUTANTS = [
    ("swapped_K", "float K = s == 0 ? P->K_first : P->K_last;",
     "float K = s == 0 ? P->K_last : P->K_first;"),
    ("dropped_K", "(x0 - txd * z0) * K;", "(x0 - txd * z0);"),
    ("curvature_sign", "x_ext[l] = x_mag + T * dz + kd * dzT * dzT * (1.0f + G->dRatio * dzT);",
     "x_ext[l] = x_mag + T * dz - kd * dzT * dzT * (1.0f + G->dRatio * dzT);"),
    ("kick_dropped", "float T = tx_in + dtx;", "float T = tx_in;"),
    ("zone_flipped", "int zone = ty_in >= 0.0f ? 1 : 0;", "int zone = ty_in >= 0.0f ? 0 : 1;"),
    ("uv_centre_sign", "xc = x_ext[l] - G->dxdy[l] * y_ext[l];", "xc = x_ext[l] + G->dxdy[l] * y_ext[l];"),
    ("uv_hit_sign", "float d = fabsf(ev->x[i] + ev->dxdy[i] * y_pred - x_pred);",
     "float d = fabsf(ev->x[i] - ev->dxdy[i] * y_pred - x_pred);"),
    ("xtol_p_inverted", "float xtol = P->xtol_const + P->xtol_pscale / p;",
     "float xtol = P->xtol_const + P->xtol_pscale * p;"),
    ("asym_side", "if (q * G->polarity > 0) asymR = P->xasym; else asymL = P->xasym;",
     "if (q * G->polarity > 0) asymL = P->xasym; else asymR = P->xasym;"),
    ("window_open_right", "if (ev->x[i] <= xmax) ++hi;", "if (ev->x[i] < xmax) ++hi;"),
    ("cap_off_centre", "int first = c - N / 2;", "int first = c - N / 4;"),
    ("charge_filter_sign", "!((txd - tx_in) * qop > 0.0f)", "!((txd - tx_in) * qop < 0.0f)"),
    ("magnet_lever_arm", "float xm = x0 + txd * (G->z_mag - z0);", "float xm = x0 + txd * (G->z_mag - z2);"),
    ("magtol_no_clamp", "if (tol > P->magtol_max) tol = P->magtol_max;", ""),
    ("triplet_cut_le", "if (i1 < 0 || !(d * d < P->T_triplet)) continue;",
     "if (i1 < 0 || !(d < P->T_triplet)) continue;"),
    ("tiebreak_set", "if (a->set != b->set) return a->set < b->set ? -1 : 1;",
     "if (a->set != b->set) return a->set > b->set ? -1 : 1;"),
    ("tiebreak_h2", "if (a->h2 != b->h2) return a->h2 < b->h2 ? -1 : 1;",
     "if (a->h2 != b->h2) return a->h2 > b->h2 ? -1 : 1;"),
    ("sort_by_h0_first", "if (a->chi2 < b->chi2) return -1;\n    if (a->chi2 > b->chi2) return 1;",
     "if (a->h0 != b->h0) return a->h0 < b->h0 ? -1 : 1;\n    if (a->chi2 < b->chi2) return -1;\n    if (a->chi2 > b->chi2) return 1;"),
    ("parabola_b", "float b = s01 - c * G01;", "float b = s12 - c * G01;"),
    ("x_ext_T_x", "if (i >= 0 && d * d < P->T_x) hits[l] = i;", "if (i >= 0 && d < P->T_x) hits[l] = i;"),
    ("cramer_db_sign", "- R0 * m01 + S2 * (S1 * R2 - R1 * S2)) / det;",
     "+ R0 * m01 + S2 * (S1 * R2 - R1 * S2)) / det;"),
    ("cramer_m02", "float m02 = S1 * S12 - S11 * S2;", "float m02 = S1 * S12 - S11 * S1;"),
    ("eta_sign", "eta[l] = -res[l] / ev->dxdy[i];", "eta[l] = res[l] / ev->dxdy[i];"),
    ("uv_x_uncorrected", "xm = ev->x[i] + ev->dxdy[i] * yv;", "xm = ev->x[i];"),
    ("ndof_x", "(Qx / (float)(n - 3)", "(Qx / (float)(n - 2)"),
    ("C_index", "P->C_nhits[n - 9]", "P->C_nhits[n > 9 ? n - 10 : 0]"),
    ("Qy_tolerance", "Qy = Qy + ry * ry / P->T_y;", "Qy = Qy + ry * ry / P->T_x;"),
    ("fit_S12_term", "S12 = S12 + s * h;", "S12 = S12 + s * s;"),
    ("fit_R2_term", "R2 = R2 + h * r;", "R2 = R2 + s * r;"),
    ("fit_S0_count", "S0 = S0 + 1.0f;", "S0 = S0 + 1.0f + (l == 0 ? 1.0f : 0.0f);"),
    ("y_fit_Y1_term", "Y1 = Y1 + su[l] * eta[l];", "Y1 = Y1 + eta[l];"),
    ("Qx_uv_as_x", "Qx = Qx + res[l] * res[l] / (is_uv(l) ? T_uv : P->T_x);", "Qx = Qx + res[l] * res[l] / P->T_x;"),
    ("T_uv_floor_ignored", "if (T_uv < P->T_uv_floor) T_uv = P->T_uv_floor;", ""),
    ("ty_cut_scale", "float dslope = dty * 0.0009765625f;", "float dslope = dty;"),
    ("qop_curvature_term", "float txT = bb + 2.0f * cc * uT", "float txT = bb + cc * uT"),
    ("station_rule", "if (hits[4 * st + 1] < 0 && hits[4 * st + 2] < 0) st_ok = 0;",
     "if (hits[4 * st + 1] < 0 || hits[4 * st + 2] < 0) st_ok = 0;"),
    ("min_hits_10", "if (n < 9 || !st_ok) continue;", "if (n < 10 || !st_ok) continue;"),
    ("best_highest_Q", "if (best_rank < 0 || Q < best_Q) {", "if (best_rank < 0 || Q > best_Q) {"),
    # no-UT tuning (VELO-only input)
    ("noUT_side_swap", "if (sd == 0) { xmin = x0 - tol; xmax = x0 + P->noUT_overlap; }",
     "if (sd == 1) { xmin = x0 - tol; xmax = x0 + P->noUT_overlap; }"),
    ("noUT_pt_threshold_ignored", "p = p_pt > P->noUT_p_min ? p_pt : P->noUT_p_min;", "p = P->noUT_p_min;"),
    ("noUT_extrapolation_origin", "x_ext[l] = x_in + tx_in * (G->z[l] - G->z_in);",
     "x_ext[l] = x_in + tx_in * (G->z[l] - G->z_mag);"),
    ("noUT_overlap_sign", "else { xmin = x0 - P->noUT_overlap; xmax = x0 + tol; }",
     "else { xmin = x0 + P->noUT_overlap; xmax = x0 + tol; }"),
    ("noUT_poly_c7", "ip * (c8[6] * tx_in + c8[7] * ip)", "ip * (c8[6] * tx_in + c8[7])"),
    ("noUT_centre_edge", "xc = 0.5f * (xmin + xmax);", "xc = xmin;"),
    ("noUT_uv_tol_as_x", "float tol = is_uv(l) ? P->uv_halfwidth : xtol;", "float tol = xtol;"),
    # paper-form field (sqrt-normalised pt-kick, momentum polynomial F)
    ("pf_extrap_cubic_dropped", "kd * dzT * dzT * (1.0f + G->dRatio * dzT);", "kd * dzT * dzT;"),
    ("pf_s_without_ty", "return tx / sqrtf(1.0f + tx * tx + ty * ty);", "return tx / sqrtf(1.0f + tx * tx);"),
    ("pf_txf_without_ty", "sqrtf((1.0f + ty * ty) / (1.0f - sf * sf))", "sqrtf(1.0f / (1.0f - sf * sf))"),
    ("pf_horner_c2_dropped", "c[1] + d * (c[2] + d * (c[3] + d * c[4]))", "c[1] + d * (d * (c[3] + d * c[4]))"),
    ("pf_odd_rows_without_tx", "c[i] = (i & 1) ? tx * acc : acc;", "c[i] = acc;"),
    ("pf_monomials_swapped", "x2 * x2 * y2, x2 * y2 * y2,", "x2 * y2 * y2, x2 * x2 * y2,"),
    ("pf_no_refinement", "for (int it = 0; it < 3; ++it) {", "for (int it = 0; it < 1; ++it) {"),
    ("pf_one_refinement", "for (int it = 0; it < 3; ++it) {", "for (int it = 0; it < 2; ++it) {"),
    ("pf_momentum_F_at_zero", "field_F(G, tx_in, ty_in, txT - tx_in)", "field_F(G, tx_in, ty_in, 0.0f)"),
    ("pf_momentum_sign", "(kick_s(txT, best_par[4]) - kick_s(tx_in, ty_in))",
     "(kick_s(txT, best_par[4]) + kick_s(tx_in, ty_in))"),
    ("pf_momentum_linear", "qop_out = (kick_s(txT, best_par[4]) - kick_s(tx_in, ty_in)) /",
     "qop_out = (txT - tx_in) /"),
    # binary16 seeding
    ("fp16_C02_dropped", "float t = h16(h16(h16(X2 - X0) + C02) * RZ);", "float t = h16(h16(X2 - X0) * RZ);"),
    ("fp16_B_dropped", "float X1e = h16(h16(h16(t * A) + h16(X0 * KK)) + B);",
     "float X1e = h16(h16(t * A) + h16(X0 * KK));"),
    ("fp16_E0_sign", "float M = h16(h16(E0 + X0) + h16(t * L0));", "float M = h16(h16(X0 - E0) + h16(t * L0));"),
    ("fp16_RZ_not_inverted", "RZ = h16(1.0f / (zw2 - zw0));", "RZ = h16(zw2 - zw0);"),
    ("fp16_middle_wrong_centre", "float dd = fabsf(h16(h16(ev->x[i] - c1) - X1e));",
     "float dd = fabsf(h16(h16(ev->x[i] - c2) - X1e));"),
    ("fp16_chi2_not_squared", "float chi2 = h16(bd * bd);", "float chi2 = bd;"),
    ("fp16_twelve_bits", "q = ldexpf(1.0f, e - 11);", "q = ldexpf(1.0f, e - 12);"),
    ("fp16_subnormal_quantum", "q = 5.9604644775390625e-08f;", "q = 1.1920928955078125e-07f;"),
    ("fp16_mixed_windows_in_half",
     "common_z(ev, wfirst[sd][l0], wlast[sd][l0]) &&\n                   common_z(ev, wfirst[sd][l2], wlast[sd][l2]) &&",
     "1 &&"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old!r}"
    (tmp_path / "lfo.c").write_text(src.replace(old, new))
    shutil.copy(HDR, tmp_path / "lfo.h")
    lib_path = str(tmp_path / "liblfo_mutant.so")
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", lib_path, str(tmp_path / "lfo.c"), "-lm"], check=True)
    lib = oracle.load_variant(lib_path)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"planted mistake {name!r} passed every pin"

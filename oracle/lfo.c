/*
 * lfo.c -- CPU oracle for Looking Forward track following (arXiv 2402.14670).
 *
 * TEST INFRASTRUCTURE ONLY (see lfo.h).  Plain single-threaded C: linear
 * scans instead of binary searches, every triplet kept and fully sorted
 * instead of a bounded selection, and the steps run in the paper's order.
 * Every float expression below is binary32 and is evaluated exactly as
 * written (C left-to-right association, no contraction).
 *
 * Readings of the paper where it is silent or garbled are marked [R..] and
 * match the numbered list of readings kept with the design notes.
 */
#include "lfo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int X_LAYERS[6] = {0, 3, 4, 7, 8, 11};
static const int UV_LAYERS[6] = {1, 2, 5, 6, 9, 10};
/* Triplet seeding layer sets: first x layer of T1/T2/T3, or last x layer
 * (Triplet Seeding subsection). */
static const int SEED_SETS[2][3] = {{0, 4, 8}, {3, 7, 11}};

static int is_uv(int l) { int k = l & 3; return k == 1 || k == 2; }

void lfo_default_params(lfo_params *p) {
    memset(p, 0, sizeof(*p));
    /* Table of parameters and tolerances, "Forward" column. */
    p->T_triplet = 8.0f;
    p->T_x = 2.0f;
    p->T_uv_scale = 50.0f;       /* T_uv = 50 (tx + ty) */
    p->T_uv_floor = 2.0f;        /* [R17] */
    p->T_ty = 0.02f;
    p->T_y = 800.0f;
    p->T_Q = 0.5f;
    p->n_hits_window = 32;
    p->n_triplets = 12;
    /* Search windows: x_tol = 150 mm + 2000 GeV/p; x_asym = 100 mm; u/v +-800 mm. */
    p->xtol_const = 150.0f;
    p->xtol_pscale = 2000.0f;
    p->xasym = 100.0f;
    p->uv_halfwidth = 800.0f;
    /* Sagitta-like correction of the triplet middle hit. */
    p->K_first = 1.00177513f;
    p->K_last = 1.00142634f;
    /* Magnet x-opening tolerance, 8..40 mm as a function of p and tx [R10]. */
    p->magtol_const = 8.0f;
    p->magtol_pscale = 24.0f;
    p->magtol_txscale = 20.0f;
    p->magtol_min = 8.0f;
    p->magtol_max = 40.0f;
    p->p_charge_cut = 5.0f;
    /* C(n_hits) table. */
    p->C_nhits[0] = 5.0f;
    p->C_nhits[1] = 1.0f;
    p->C_nhits[2] = 0.8f;
    p->C_nhits[3] = 0.5f;
}

void lfo_default_params_no_ut(lfo_params *p) {
    lfo_default_params(p);
    /* Table of parameters and tolerances, "Forward no-UT" column. */
    p->T_triplet = 2.0f;
    p->T_x = 0.5f;
    p->T_uv_scale = 15.0f;       /* T_uv = 15 (tx + ty), same floor [R17] */
    p->T_ty = 0.003f;
    p->T_y = 800.0f;
    p->T_Q = 0.5f;
    p->n_hits_window = 64;
    p->n_triplets = 20;
    /* No-UT tuning section: u/v tolerance 1200 mm, magnet x tolerance fixed
     * at 10 mm, no bend-direction filter (no q/p). */
    p->uv_halfwidth = 1200.0f;
    p->magtol_const = 10.0f;
    p->magtol_pscale = 0.0f;
    p->magtol_txscale = 0.0f;
    p->magtol_min = 10.0f;
    p->magtol_max = 10.0f;
    p->p_charge_cut = 0.0f;
    p->velo_only = 1;
    /* Polynomial coefficients of the curvature tolerance (Tab.Poly). */
    const float c[8] = {4824.3f, 426.3f, 7071.1f, 12080.4f, 14077.8f, 13909.3f, 9315.3f, 3209.5f};
    for (int i = 0; i < 8; ++i) p->noUT_c[i] = c[i];
    p->noUT_p_min = 5.0f;        /* 5 GeV or pt 1 GeV, whichever is tighter [N2] */
    p->noUT_pt_min = 1.0f;
    p->noUT_overlap = 5.0f;      /* the text's 5 mm (the figure caption says 1 cm) [N4] */
}

/* ---------------------------------------------------------------- */
typedef struct {
    const float *x, *z, *dxdy;     /* event-local hit arrays */
    uint32_t begin[2 * LFO_NL];    /* event-local bucket bounds */
    uint32_t end[2 * LFO_NL];
} event_view;

typedef struct { float chi2; int side, set, h0, h1, h2; } triplet;

static int triplet_cmp(const void *pa, const void *pb) {
    const triplet *a = (const triplet *)pa, *b = (const triplet *)pb;
    /* [R13] ascending (chi2, side, set, h0, h2); side is 0 except with
     * VELO-only input [N7] */
    if (a->chi2 < b->chi2) return -1;
    if (a->chi2 > b->chi2) return 1;
    if (a->side != b->side) return a->side < b->side ? -1 : 1;
    if (a->set != b->set) return a->set < b->set ? -1 : 1;
    if (a->h0 != b->h0) return a->h0 < b->h0 ? -1 : 1;
    if (a->h2 != b->h2) return a->h2 < b->h2 ? -1 : 1;
    return 0;
}

/* The binary16 value nearest to x (IEEE 754 round to nearest, ties to even;
 * subnormals below 2^-14 with the quantum 2^-24; 65520 and above round to
 * infinity), returned as a binary32.  A binary16 operation on binary16
 * operands is the binary32 operation rounded by h16: binary32 carries more
 * than twice binary16's precision plus two bits, so the double rounding is
 * exact for +, -, * and /.  [H1] */
static float h16(float x) {
    if (x != x) return x;
    float ax = fabsf(x);
    if (ax >= 65520.0f) return copysignf(INFINITY, x);
    float q;
    if (ax < 6.103515625e-05f) {
        q = 5.9604644775390625e-08f;
    } else {
        int e;
        frexpf(ax, &e);            /* ax = m 2^e, m in [0.5, 1): 11 significant bits end at 2^(e - 11) */
        q = ldexpf(1.0f, e - 11);
    }
    return copysignf(rintf(ax / q) * q, x);
}

float lfo_h16(float x) { return h16(x); }

/* All hits of [first, last) share one z, bit for bit (an empty window does). */
static int common_z(const event_view *ev, int first, int last) {
    for (int i = first + 1; i < last; ++i)
        if (memcmp(&ev->z[i], &ev->z[first], sizeof(float)) != 0) return 0;
    return 1;
}

/* Closest hit to x_expected inside [first, last): linear scan, strict '<'
 * so the lowest index wins a tie [R12].  Returns -1 if none is finite. */
static int closest_x(const event_view *ev, int first, int last, float x_expected, float *dist) {
    int best = -1;
    float bd = INFINITY;
    for (int i = first; i < last; ++i) {
        float d = fabsf(ev->x[i] - x_expected);
        if (d < bd) { bd = d; best = i; }
    }
    *dist = bd;
    return best;
}

/* Same for a stereo layer: the hit's x at y=0 is moved to the predicted y
 * with the hit's own stereo slope before comparing [R16]. */
static int closest_uv(const event_view *ev, int first, int last, float x_pred, float y_pred,
                      float *dist) {
    int best = -1;
    float bd = INFINITY;
    for (int i = first; i < last; ++i) {
        float d = fabsf(ev->x[i] + ev->dxdy[i] * y_pred - x_pred);
        if (d < bd) { bd = d; best = i; }
    }
    *dist = bd;
    return best;
}

/* x(z) model of the Propagation section, cubic term dRatio:
 *   g(u) = u^2 (1 + dRatio u),  x(u) = a + b u + c g(u),  u = z - z_ref. */
static float g_of(float u, float dRatio) { return u * u * (1.0f + dRatio * u); }

/* Integrated field of the momentum parametrisation [M1][M2]: the 2D
 * polynomials c_i(tx, ty) over the monomials m_j summed in order of j, then
 * F = c0 + d (c1 + d (c2 + d (c3 + d c4))). */
static float field_F(const lfo_geometry *G, float tx, float ty, float d) {
    float x2 = tx * tx, y2 = ty * ty;
    float m[10] = {1.0f, x2, y2, x2 * x2, x2 * y2, y2 * y2, x2 * x2 * x2, x2 * x2 * y2, x2 * y2 * y2,
                   y2 * y2 * y2};
    float c[5];
    for (int i = 0; i < 5; ++i) {
        int nj = (i & 1) ? 6 : 10;
        float acc = G->F_coef[i][0] * m[0];
        for (int j = 1; j < nj; ++j) acc = acc + G->F_coef[i][j] * m[j];
        c[i] = (i & 1) ? tx * acc : acc;
    }
    return c[0] + d * (c[1] + d * (c[2] + d * (c[3] + d * c[4])));
}

/* Sine-like slope of the pt-kick equation, tx / sqrt(1 + tx^2 + ty^2). */
static float kick_s(float tx, float ty) { return tx / sqrtf(1.0f + tx * tx + ty * ty); }

/* x slope after the magnet from s_f and ty (ty unchanged by the kick):
 * tx_f = s_f sqrt((1 + ty^2) / (1 - s_f^2)).  Returns 0 when |s_f| >= 1:
 * no slope can carry that kick [M4]. */
static int kick_tx(float sf, float ty, float *txf) {
    if (!(sf * sf < 1.0f)) return 0;
    *txf = sf * sqrtf((1.0f + ty * ty) / (1.0f - sf * sf));
    return 1;
}

static void track_one(const lfo_geometry *G, const lfo_params *P, const event_view *ev,
                      float x_in, float y_in, float tx_in, float ty_in, float qop,
                      uint8_t *found, uint8_t *n_out, int32_t *hit_out, float *par_out,
                      int32_t *dbg_win, float *dbg_wx, int64_t *dbg_counts, int32_t *dbg_trip,
                      float *dbg_trip_chi2, float *dbg_candQ, int32_t *dbg_cand_hits,
                      int32_t *dbg_win1, float *dbg_wx1) {
    const int NT = P->n_triplets;
    *found = 0;
    *n_out = 0;
    for (int l = 0; l < LFO_NL; ++l) hit_out[l] = -1;
    for (int k = 0; k < 7; ++k) par_out[k] = 0.0f;

    /* ---- Kinematics [R2][R3]: the y-slope picks the detector half.  With
     *      VELO-only input the momentum is the assumed minimum: the tighter
     *      (larger) of noUT_p_min and the momentum at which the track's
     *      transverse momentum is noUT_pt_min [N2]. ---- */
    const int velo = P->velo_only != 0;
    float p;
    int q = 0;
    if (velo) {
        float t2 = tx_in * tx_in + ty_in * ty_in;
        float sin_t = sqrtf(t2 / (1.0f + t2));
        float p_pt = sin_t > 0.0f ? P->noUT_pt_min / sin_t : 0.0f;
        p = p_pt > P->noUT_p_min ? p_pt : P->noUT_p_min;
    } else {
        p = 1.0f / fabsf(qop);
        q = qop > 0.0f ? 1 : -1;
    }
    int zone = ty_in >= 0.0f ? 1 : 0;

    /* ---- Extrapolation to every layer.  VELO-UT input: the pt-kick model
     *      [R1], straight to the bending plane, the kick, then the post-magnet
     *      model with its cubic term [M6].  The kick is dtx = kick*q/p, or
     *      (field_form 1) the sqrt-normalised pt-kick equation solved for the
     *      slope after the magnet with F taken at dSlope = 0 and then twice at
     *      the slope change of the previous solution [M3]; a track whose kick
     *      has no solution is not found [M4].  VELO input: a straight line
     *      [N1]. ---- */
    float x_mag = x_in + tx_in * (G->z_mag - G->z_in);
    float x_ext[LFO_NL], y_ext[LFO_NL];
    if (velo) {
        for (int l = 0; l < LFO_NL; ++l) x_ext[l] = x_in + tx_in * (G->z[l] - G->z_in);
    } else {
        float dtx;
        if (G->field_form == 1) {
            float si = kick_s(tx_in, ty_in);
            float d = 0.0f, txf = 0.0f;
            for (int it = 0; it < 3; ++it) {
                if (!kick_tx(si + qop * field_F(G, tx_in, ty_in, d), ty_in, &txf)) return;
                d = txf - tx_in;
            }
            dtx = d;
        } else {
            dtx = G->kick * qop;
        }
        float T = tx_in + dtx;
        float kd = G->kappa * dtx;
        for (int l = 0; l < LFO_NL; ++l) {
            float dz = G->z[l] - G->z_mag;
            float dzT = G->z[l] - G->z_T;
            x_ext[l] = x_mag + T * dz + kd * dzT * dzT * (1.0f + G->dRatio * dzT);
        }
    }
    for (int l = 0; l < LFO_NL; ++l) y_ext[l] = y_in + ty_in * (G->z[l] - G->z_in);

    /* ---- Step 1: search windows (x_min/x_max; u/v straight line +-800 mm;
     *      at most n_hits_window hits, symmetric around the centre).  With
     *      VELO-only input every layer has two windows, side 0 for bending
     *      towards -x and side 1 towards +x: [x_ext - tol, x_ext + overlap]
     *      and [x_ext - overlap, x_ext + tol], tol the momentum polynomial on
     *      x layers and uv_halfwidth on u/v layers, centred for the cap on
     *      the middle of each window [N3]-[N6]. ---- */
    const int NS = velo ? 2 : 1;
    float xtol = P->xtol_const + P->xtol_pscale / p;          /* [R4] */
    if (velo) {                                                /* [N3] */
        const float *c8 = P->noUT_c;
        float ip = 1.0f / p;
        float ty2 = ty_in * ty_in;
        xtol = ip * (c8[0] + tx_in * (c8[1] + c8[2] * tx_in) + ty2 * (c8[3] + tx_in * (c8[4] + c8[5] * tx_in)) +
                     ip * (c8[6] * tx_in + c8[7] * ip));
    }
    float asymL = 0.0f, asymR = 0.0f;                          /* [R5] */
    if (q * G->polarity > 0) asymR = P->xasym; else asymL = P->xasym;
    int wfirst[2][LFO_NL], wlast[2][LFO_NL];
    for (int sd = 0; sd < NS; ++sd) {
        for (int l = 0; l < LFO_NL; ++l) {
            float xc, xmin, xmax;
            if (velo) {
                float x0 = is_uv(l) ? x_ext[l] - G->dxdy[l] * y_ext[l] : x_ext[l];
                float tol = is_uv(l) ? P->uv_halfwidth : xtol;
                if (sd == 0) { xmin = x0 - tol; xmax = x0 + P->noUT_overlap; }
                else { xmin = x0 - P->noUT_overlap; xmax = x0 + tol; }
                xc = 0.5f * (xmin + xmax);
            } else if (is_uv(l)) {                              /* [R6] */
                xc = x_ext[l] - G->dxdy[l] * y_ext[l];
                xmin = xc - P->uv_halfwidth;
                xmax = xc + P->uv_halfwidth;
            } else {
                xc = x_ext[l];
                xmin = xc - xtol - asymL;
                xmax = xc + xtol + asymR;
            }
            int b = 2 * l + zone;
            int begin = (int)ev->begin[b], end = (int)ev->end[b];
            /* [R7] closed interval by counting over the sorted bucket */
            int lo = begin, hi = begin, c = begin;
            for (int i = begin; i < end; ++i) {
                if (ev->x[i] < xmin) ++lo;
                if (ev->x[i] <= xmax) ++hi;
                if (ev->x[i] < xc) ++c;
            }
            if (hi < lo) hi = lo;
            if (c < lo) c = lo;
            if (c > hi) c = hi;
            int N = P->n_hits_window;
            if (hi - lo > N) {                                 /* [R8] */
                int first = c - N / 2;
                if (first < lo) first = lo;
                if (first > hi - N) first = hi - N;
                wfirst[sd][l] = first;
                wlast[sd][l] = first + N;
            } else {
                wfirst[sd][l] = lo;
                wlast[sd][l] = hi;
            }
            int32_t *dw = sd == 0 ? dbg_win : dbg_win1;
            float *dx = sd == 0 ? dbg_wx : dbg_wx1;
            if (dw) { dw[2 * l] = wfirst[sd][l]; dw[2 * l + 1] = wlast[sd][l]; }
            if (dx) { dx[3 * l] = xmin; dx[3 * l + 1] = xc; dx[3 * l + 2] = xmax; }
        }
    }

    /* ---- Step 2: triplet seeding. ---- */
    int64_t n_pairs = 0, n_doublets = 0;
    size_t cap = 64, ntrip = 0;
    triplet *trips = (triplet *)malloc(cap * sizeof(triplet));
    if (!trips) return;
    for (int sd = 0; sd < NS; ++sd)   /* VELO input: each charge assumption on its own [N7] */
    for (int s = 0; s < 2; ++s) {
        int l0 = SEED_SETS[s][0], l1 = SEED_SETS[s][1], l2 = SEED_SETS[s][2];
        float K = s == 0 ? P->K_first : P->K_last;
        /* binary16 seeding [H2]-[H5]: coordinates relative to the window
         * centres c_l = x_ext(z_l) of the three layers, the windows' common
         * z0 and z2, per-set constants rounded once from binary32 */
        int half = P->seed_fp16 && common_z(ev, wfirst[sd][l0], wlast[sd][l0]) &&
                   common_z(ev, wfirst[sd][l2], wlast[sd][l2]) &&
                   wlast[sd][l0] > wfirst[sd][l0] && wlast[sd][l2] > wfirst[sd][l2];
        float c0 = x_ext[l0], c1 = x_ext[l1], c2 = x_ext[l2];
        float RZ = 0, C02 = 0, E0 = 0, L0 = 0, A = 0, KK = 0, B = 0, TX = 0, QP = 0, TC = 0, TXS = 0, TMIN = 0,
              TMAX = 0, T3 = 0;
        if (half) {
            float zw0 = ev->z[wfirst[sd][l0]], zw2 = ev->z[wfirst[sd][l2]];
            RZ = h16(1.0f / (zw2 - zw0));
            C02 = h16(c2 - c0);
            E0 = h16(c0 - x_mag);
            L0 = h16(G->z_mag - zw0);
            A = h16(G->z[l1] - zw0 * K);
            KK = h16(K);
            B = h16(c0 * K - c1);
            TX = h16(tx_in);
            QP = h16(qop);
            TC = h16(P->magtol_const + P->magtol_pscale / p);
            TXS = h16(P->magtol_txscale);
            TMIN = h16(P->magtol_min);
            TMAX = h16(P->magtol_max);
            T3 = h16(P->T_triplet);
        }
        for (int i0 = wfirst[sd][l0]; i0 < wlast[sd][l0]; ++i0) {
            for (int i2 = wfirst[sd][l2]; i2 < wlast[sd][l2]; ++i2) {
                ++n_pairs;
                if (half) {
                    float X0 = h16(ev->x[i0] - c0), X2 = h16(ev->x[i2] - c2);
                    /* the doublet's slope, and the two filters [H3] */
                    float t = h16(h16(h16(X2 - X0) + C02) * RZ);
                    if (p < P->p_charge_cut && !(h16(h16(t - TX) * QP) > 0.0f)) continue;
                    float M = h16(h16(E0 + X0) + h16(t * L0));
                    float tol = h16(TC + h16(TXS * fabsf(t)));
                    if (tol < TMIN) tol = TMIN;
                    if (tol > TMAX) tol = TMAX;
                    if (!(fabsf(M) < tol)) continue;
                    ++n_doublets;
                    /* middle hit relative to c1, closest by linear scan [H4] */
                    float X1e = h16(h16(h16(t * A) + h16(X0 * KK)) + B);
                    int i1 = -1;
                    float bd = INFINITY;
                    for (int i = wfirst[sd][l1]; i < wlast[sd][l1]; ++i) {
                        float dd = fabsf(h16(h16(ev->x[i] - c1) - X1e));
                        if (dd < bd) { bd = dd; i1 = i; }
                    }
                    if (i1 < 0) continue;
                    float chi2 = h16(bd * bd);
                    if (!(chi2 < T3)) continue;
                    if (ntrip == cap) {
                        cap *= 2;
                        triplet *nt = (triplet *)realloc(trips, cap * sizeof(triplet));
                        if (!nt) { free(trips); return; }
                        trips = nt;
                    }
                    triplet th = {chi2, sd, s, i0, i1, i2};
                    trips[ntrip++] = th;
                    continue;
                }
                float x0 = ev->x[i0], z0 = ev->z[i0];
                float x2 = ev->x[i2], z2 = ev->z[i2];
                float txd = (x2 - x0) / (z2 - z0);
                /* doublet filter 1: below p_charge_cut the bending from the
                 * upstream track to the doublet must follow the charge [R9] */
                if (!velo && p < P->p_charge_cut && !((txd - tx_in) * qop > 0.0f)) continue;
                /* doublet filter 2: x opening at the bending plane [R10] */
                float xm = x0 + txd * (G->z_mag - z0);
                float tol = P->magtol_const + P->magtol_pscale / p + P->magtol_txscale * fabsf(txd);
                if (tol < P->magtol_min) tol = P->magtol_min;
                if (tol > P->magtol_max) tol = P->magtol_max;
                if (!(fabsf(xm - x_mag) < tol)) continue;
                ++n_doublets;
                /* middle hit: straight line corrected by K [R11] */
                float x1e = G->z[l1] * txd + (x0 - txd * z0) * K;
                float d;
                int i1 = closest_x(ev, wfirst[sd][l1], wlast[sd][l1], x1e, &d);
                if (i1 < 0 || !(d * d < P->T_triplet)) continue;
                if (ntrip == cap) {
                    cap *= 2;
                    triplet *nt = (triplet *)realloc(trips, cap * sizeof(triplet));
                    if (!nt) { free(trips); return; }
                    trips = nt;
                }
                triplet t = {d * d, sd, s, i0, i1, i2};
                trips[ntrip++] = t;
            }
        }
    }
    qsort(trips, ntrip, sizeof(triplet), triplet_cmp);        /* [R13] */
    int nkeep = (int)ntrip < NT ? (int)ntrip : NT;
    for (int r = 0; r < NT; ++r) {
        if (dbg_trip) {
            int32_t *o = dbg_trip + 4 * r;
            if (r < nkeep) {
                o[0] = trips[r].set + 2 * trips[r].side;
                o[1] = trips[r].h0; o[2] = trips[r].h1; o[3] = trips[r].h2;
            }
            else { o[0] = o[1] = o[2] = o[3] = -1; }
        }
        if (dbg_trip_chi2) dbg_trip_chi2[r] = r < nkeep ? trips[r].chi2 : NAN;
    }
    if (dbg_candQ) for (int r = 0; r < NT; ++r) dbg_candQ[r] = NAN;
    if (dbg_cand_hits) for (int r = 0; r < NT * LFO_NL; ++r) dbg_cand_hits[r] = -1;

    /* ---- Steps 3-4: extension, fit and quality for each kept triplet. ---- */
    float T_uv = P->T_uv_scale * (fabsf(tx_in) + fabsf(ty_in));   /* [R17] */
    if (T_uv < P->T_uv_floor) T_uv = P->T_uv_floor;
    int best_rank = -1, best_n = 0;
    float best_Q = 0.0f;
    int best_hits[LFO_NL];
    float best_par[5];
    int n_valid = 0;
    for (int r = 0; r < nkeep; ++r) {
        const triplet *t = &trips[r];
        int l0 = SEED_SETS[t->set][0], l1 = SEED_SETS[t->set][1], l2 = SEED_SETS[t->set][2];
        int hits[LFO_NL];
        for (int l = 0; l < LFO_NL; ++l) hits[l] = -1;
        hits[l0] = t->h0; hits[l1] = t->h1; hits[l2] = t->h2;

        /* parabola (cubic when dRatio != 0) through the three hits [R14]:
         * x - c g(u) is linear in u, so equal secant slopes give c. */
        float u0 = ev->z[t->h0] - G->z_ref, u1 = ev->z[t->h1] - G->z_ref, u2 = ev->z[t->h2] - G->z_ref;
        float X0 = ev->x[t->h0], X1 = ev->x[t->h1], X2 = ev->x[t->h2];
        float g0 = g_of(u0, G->dRatio), g1 = g_of(u1, G->dRatio), g2 = g_of(u2, G->dRatio);
        float s01 = (X1 - X0) / (u1 - u0);
        float s12 = (X2 - X1) / (u2 - u1);
        float G01 = (g1 - g0) / (u1 - u0);
        float G12 = (g2 - g1) / (u2 - u1);
        float c = (s12 - s01) / (G12 - G01);
        float b = s01 - c * G01;
        float a = X0 - b * u0 - c * g0;

        /* extension to the three missing x layers (no refit) [R15] */
        for (int k = 0; k < 6; ++k) {
            int l = X_LAYERS[k];
            if (hits[l] >= 0) continue;
            float u = G->z[l] - G->z_ref;
            float xe = a + b * u + c * g_of(u, G->dRatio);
            float d;
            int i = closest_x(ev, wfirst[t->side][l], wlast[t->side][l], xe, &d);
            if (i >= 0 && d * d < P->T_x) hits[l] = i;
        }
        /* extension to the u/v layers, slope-dependent tolerance [R16][R17] */
        for (int k = 0; k < 6; ++k) {
            int l = UV_LAYERS[k];
            float u = G->z[l] - G->z_ref;
            float xp = a + b * u + c * g_of(u, G->dRatio);
            float d;
            int i = closest_uv(ev, wfirst[t->side][l], wlast[t->side][l], xp, y_ext[l], &d);
            if (i >= 0 && d * d < T_uv) hits[l] = i;
        }
        if (dbg_cand_hits) memcpy(dbg_cand_hits + r * LFO_NL, hits, sizeof(hits));
        /* candidate rule: >= 9 hits and a u/v hit in each station [R18] */
        int n = 0, n_uv = 0, st_ok = 1;
        for (int l = 0; l < LFO_NL; ++l) if (hits[l] >= 0) { ++n; if (is_uv(l)) ++n_uv; }
        for (int st = 0; st < 3; ++st)
            if (hits[4 * st + 1] < 0 && hits[4 * st + 2] < 0) st_ok = 0;
        if (n < 9 || !st_ok) continue;

        /* ---- x least-squares fit over all hits [R19]: corrections (da, db, dc)
         * to the triplet model, basis {1, s, s^2 (1 + dRatio u)}, s = u/1024.
         * Every sum starts at +0 and adds the hits' terms in ascending layer
         * order. ---- */
        float su[LFO_NL], sh[LFO_NL], rho[LFO_NL];
        float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f, S11 = 0.0f, S12 = 0.0f, S22 = 0.0f;
        float R0 = 0.0f, R1 = 0.0f, R2 = 0.0f;
        for (int l = 0; l < LFO_NL; ++l) {
            su[l] = 0.0f; sh[l] = 0.0f; rho[l] = 0.0f;
            int i = hits[l];
            if (i < 0) continue;
            float u = ev->z[i] - G->z_ref;
            float xm;
            if (is_uv(l)) {
                float yv = y_in + ty_in * (ev->z[i] - G->z_in);
                xm = ev->x[i] + ev->dxdy[i] * yv;
            } else {
                xm = ev->x[i];
            }
            float s = u * 0.0009765625f;
            float h = s * s * (1.0f + G->dRatio * u);
            float r = xm - (a + b * u + c * g_of(u, G->dRatio));
            su[l] = s; sh[l] = h; rho[l] = r;
            S0 = S0 + 1.0f;
            S1 = S1 + s;
            S2 = S2 + h;
            S11 = S11 + s * s;
            S12 = S12 + s * h;
            S22 = S22 + h * h;
            R0 = R0 + r;
            R1 = R1 + s * r;
            R2 = R2 + h * r;
        }
        /* normal equations M (da db dc)^T = (R0 R1 R2)^T solved by Cramer's rule */
        float m00 = S11 * S22 - S12 * S12;
        float m01 = S1 * S22 - S12 * S2;
        float m02 = S1 * S12 - S11 * S2;
        float det = S0 * m00 - S1 * m01 + S2 * m02;
        if (!(fabsf(det) > 0.0f)) continue;
        float da = (R0 * m00 - S1 * (R1 * S22 - S12 * R2) + S2 * (R1 * S12 - S11 * R2)) / det;
        float db = (S0 * (R1 * S22 - S12 * R2) - R0 * m01 + S2 * (S1 * R2 - R1 * S2)) / det;
        float dc = (S0 * (S11 * R2 - R1 * S12) - S1 * (S1 * R2 - R1 * S2) + R0 * m02) / det;

        /* residuals to the fitted model; Q_x [R21] */
        float res[LFO_NL];
        float Qx = 0.0f;
        for (int l = 0; l < LFO_NL; ++l) {
            res[l] = 0.0f;
            if (hits[l] < 0) continue;
            res[l] = rho[l] - (da + db * su[l] + dc * sh[l]);
            Qx = Qx + res[l] * res[l] / (is_uv(l) ? T_uv : P->T_x);
        }

        /* ---- y least-squares line over the u/v hits [R20]: each hit's y is
         * where its fibre meets the fitted x, y = y_ext - res/dxdy, so the
         * offsets from the input line are eta = -res/dxdy. ---- */
        float eta[LFO_NL];
        float Y_S0 = 0.0f, Y_S1 = 0.0f, Y_S11 = 0.0f, Y0 = 0.0f, Y1 = 0.0f;
        for (int l = 0; l < LFO_NL; ++l) {
            eta[l] = 0.0f;
            int i = hits[l];
            if (i < 0 || !is_uv(l)) continue;
            eta[l] = -res[l] / ev->dxdy[i];
            Y_S0 = Y_S0 + 1.0f;
            Y_S1 = Y_S1 + su[l];
            Y_S11 = Y_S11 + su[l] * su[l];
            Y0 = Y0 + eta[l];
            Y1 = Y1 + su[l] * eta[l];
        }
        float D = Y_S0 * Y_S11 - Y_S1 * Y_S1;
        if (!(fabsf(D) > 0.0f)) continue;
        float dy0 = (Y0 * Y_S11 - Y_S1 * Y1) / D;
        float dty = (Y_S0 * Y1 - Y_S1 * Y0) / D;
        float dslope = dty * 0.0009765625f;
        if (!(fabsf(dslope) < P->T_ty)) continue;              /* [R22] */
        float Qy = 0.0f;
        for (int l = 0; l < LFO_NL; ++l) {
            if (hits[l] < 0 || !is_uv(l)) continue;
            float ry = eta[l] - (dy0 + dty * su[l]);
            Qy = Qy + ry * ry / P->T_y;
        }
        /* ---- quality factor [R21] ---- */
        float Q = (Qx / (float)(n - 3) + Qy / (float)(n_uv - 2)) * P->C_nhits[n - 9];
        if (dbg_candQ) dbg_candQ[r] = Q;
        if (!(Q < P->T_Q)) continue;
        ++n_valid;
        /* best candidate: lowest Q, then lowest rank [R23] */
        if (best_rank < 0 || Q < best_Q) {
            best_rank = r;
            best_Q = Q;
            memcpy(best_hits, hits, sizeof(hits));
            best_par[0] = a + da;
            best_par[1] = b + db * 0.0009765625f;
            best_par[2] = c + dc * 0.00000095367431640625f;
            best_par[3] = (y_in + ty_in * (G->z_ref - G->z_in)) + dy0;
            best_par[4] = ty_in + dslope;
            best_n = n;
        }
    }
    free(trips);
    if (dbg_counts) {
        dbg_counts[0] = n_pairs;
        dbg_counts[1] = n_doublets;
        dbg_counts[2] = (int64_t)ntrip;
        dbg_counts[3] = n_valid;
    }
    if (best_rank < 0) return;

    /* ---- momentum from the slope change at z_T [R24]; field_form 1: the
     *      pt-kick equation with the fitted slopes after the magnet and F at
     *      the measured dSlope [M5] ---- */
    float bb = best_par[1], cc = best_par[2];
    float uT = G->z_T - G->z_ref;
    float txT = bb + 2.0f * cc * uT + 3.0f * cc * G->dRatio * uT * uT;
    float qop_out;
    if (G->field_form == 1)
        qop_out = (kick_s(txT, best_par[4]) - kick_s(tx_in, ty_in)) / field_F(G, tx_in, ty_in, txT - tx_in);
    else
        qop_out = (txT - tx_in) / G->kick;

    *found = 1;
    *n_out = (uint8_t)best_n;
    for (int l = 0; l < LFO_NL; ++l) hit_out[l] = best_hits[l];
    par_out[0] = best_par[0];
    par_out[1] = best_par[1];
    par_out[2] = best_par[2];
    par_out[3] = best_par[3];
    par_out[4] = best_par[4];
    par_out[5] = qop_out;
    par_out[6] = best_Q;
}

int lfo_find_tracks(const lfo_geometry *g, const lfo_params *P, uint32_t n_events,
                    const uint32_t *hit_off, const float *hit_x, const float *hit_z,
                    const float *hit_dxdy, const uint32_t *trk_off, const float *trk_x,
                    const float *trk_y, const float *trk_tx, const float *trk_ty,
                    const float *trk_qop, uint32_t ev_begin, uint32_t ev_end,
                    lfo_out *out, lfo_debug *dbg) {
    if (!g || !P || !hit_off || !trk_off || !out || ev_end > n_events || ev_begin > ev_end)
        return -1;
    if (P->n_triplets < 1 || P->n_triplets > LFO_MAX_TRIPLETS || P->n_hits_window < 1) return -1;
    if (g->field_form != 0 && g->field_form != 1) return -1;
    if (P->seed_fp16 != 0 && P->seed_fp16 != 1) return -1;
    if (P->seed_fp16 && P->velo_only) return -1;
    const int NT = P->n_triplets;
    for (uint32_t e = ev_begin; e < ev_end; ++e) {
        uint32_t base = hit_off[24 * e];
        event_view ev;
        ev.x = hit_x + base;
        ev.z = hit_z + base;
        ev.dxdy = hit_dxdy + base;
        for (int b = 0; b < 24; ++b) {
            ev.begin[b] = hit_off[24 * e + b] - base;
            ev.end[b] = hit_off[24 * e + b + 1] - base;
        }
        for (uint32_t t = trk_off[e]; t < trk_off[e + 1]; ++t) {
            float par[7];
            track_one(g, P, &ev, trk_x[t], trk_y[t], trk_tx[t], trk_ty[t], trk_qop[t],
                      &out->found[t], &out->n_hits[t], &out->hit_idx[(size_t)t * LFO_NL], par,
                      dbg && dbg->win ? dbg->win + (size_t)t * 24 : NULL,
                      dbg && dbg->wx ? dbg->wx + (size_t)t * 36 : NULL,
                      dbg && dbg->counts ? dbg->counts + (size_t)t * 4 : NULL,
                      dbg && dbg->trip ? dbg->trip + (size_t)t * NT * 4 : NULL,
                      dbg && dbg->trip_chi2 ? dbg->trip_chi2 + (size_t)t * NT : NULL,
                      dbg && dbg->cand_Q ? dbg->cand_Q + (size_t)t * NT : NULL,
                      dbg && dbg->cand_hits ? dbg->cand_hits + (size_t)t * NT * LFO_NL : NULL,
                      dbg && dbg->win1 ? dbg->win1 + (size_t)t * 24 : NULL,
                      dbg && dbg->wx1 ? dbg->wx1 + (size_t)t * 36 : NULL);
            out->a[t] = par[0];
            out->b[t] = par[1];
            out->c[t] = par[2];
            out->y0[t] = par[3];
            out->ty[t] = par[4];
            out->qop[t] = par[5];
            out->Q[t] = par[6];
        }
    }
    return 0;
}

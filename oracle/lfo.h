/*
 * lfo.h -- CPU oracle for Looking Forward track following (arXiv 2402.14670).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or constant with the
 * GPU library: its structures below are its own.
 *
 * Arithmetic is IEEE binary32, round to nearest even, built with
 * -ffp-contract=off and without fast-math, evaluated in the order written in
 * lfo.c (the paper keeps hits in fp32; its Performance section).
 *
 * Entry point: lfo_find_tracks() runs the four steps of the paper's
 * "Algorithm logic" section (search windows, triplet seeding, extension,
 * quality filter) followed by the momentum / state computation, for every
 * input track of every event, and writes one result slot per input track.
 */
#ifndef LFO_H
#define LFO_H
#include <stdint.h>

#define LFO_NL 12
#define LFO_MAX_TRIPLETS 64

/* Detector and field description (all mm, GeV). */
typedef struct {
    float z[LFO_NL];      /* layer planes; x layers 0,3,4,7,8,11, u/v layers 1,2,5,6,9,10 */
    float dxdy[LFO_NL];   /* stereo tangent of each layer (0 for x layers) */
    float z_in;           /* z of the upstream track states */
    float z_mag;          /* bending plane of the pt-kick (z_bending) */
    float z_ref;          /* reference plane of the x(z) track model (8520 mm) */
    float z_T;            /* plane where the post-magnet slope is read for q/p */
    float kick;           /* slope kick per unit q/p: dtx = kick * q/p */
    float kappa;          /* residual curvature after the magnet, per unit dtx */
    float dRatio;         /* cubic term of the x(z) model */
    int32_t polarity;     /* +1: q > 0 bends towards +x (window asymmetry on +x) */
    /* Momentum form.  0: linear kick, slope change = kick * q/p, and
     * q/p = slope change / kick.  1: the sqrt-normalised pt-kick equation
     * with the integrated field given by the fourth-order polynomial F in
     * dSlope of "Calculation of momentum and track states":
     *   F = sum_{i=0..4} c_i dSlope^i,
     *   c_i = sum_j F_coef[i][j] m_j          (i even, j = 0..9),
     *   c_i = tx * sum_j F_coef[i][j] m_j     (i odd,  j = 0..5),
     *   m = 1, tx2, ty2, tx2^2, tx2 ty2, ty2^2, tx2^3, tx2^2 ty2, tx2 ty2^2, ty2^3,
     * with tx, ty the input (VELO) slopes; F_coef[odd][6..9] are unused. */
    int32_t field_form;
    float F_coef[5][10];
} lfo_geometry;

/* Tunable parameters (Table of tolerances, Forward column; C(n_hits) table). */
typedef struct {
    float T_triplet, T_x, T_uv_scale, T_uv_floor, T_ty, T_y, T_Q;
    float xtol_const, xtol_pscale, xasym, uv_halfwidth;
    float K_first, K_last;
    float magtol_const, magtol_pscale, magtol_txscale, magtol_min, magtol_max;
    float p_charge_cut;
    float C_nhits[4];     /* C(9), C(10), C(11), C(12) */
    int32_t n_hits_window;
    int32_t n_triplets;   /* <= LFO_MAX_TRIPLETS */
    /* No-UT tuning: VELO input tracks without q/p, extrapolated as straight
     * lines, an assumed minimum momentum, double-sided windows (one per
     * charge assumption) and seeding per side.  uv_halfwidth is then the
     * stereo-window tolerance and the Tab.Tol no-UT column applies. */
    int32_t velo_only;    /* 0: VELO-UT input (q/p used); 1: VELO input (q/p ignored) */
    float noUT_c[8];      /* x_tol polynomial coefficients c0..c7 (Tab.Poly) */
    float noUT_p_min;     /* assumed minimum momentum, GeV */
    float noUT_pt_min;    /* assumed minimum transverse momentum, GeV */
    float noUT_overlap;   /* overlap of the two windows of a layer, mm */
    /* Triplet seeding in binary16 (Performance section: the seeding needs
     * only half precision).  1: the doublet filters and the middle-hit chi2
     * of a seed set whose first- and last-layer windows each share one z
     * are evaluated in binary16 on coordinates relative to the window
     * centres, every pair of the windows tested; other sets, and every other
     * step, stay binary32.  VELO-UT input only (velo_only = 0). */
    int32_t seed_fp16;
} lfo_params;

/* One result slot per input track.  hit_idx is event-local (index into the
 * event's hits in bucket-major order), -1 where the layer has no hit. */
typedef struct {
    uint8_t *found, *n_hits;
    int32_t *hit_idx;                       /* [n_tracks * 12] */
    float *a, *b, *c, *y0, *ty, *qop, *Q;   /* x(z_ref), dx/dz(z_ref), curvature, y(z_ref), dy/dz */
} lfo_out;

/* Optional intermediate dumps (any pointer may be NULL). */
typedef struct {
    int32_t *win;          /* [n_tracks * 24]: event-local [first, last) per layer (side 0 when velo_only) */
    float *wx;             /* [n_tracks * 36]: x_min, centre, x_max per layer (side 0 when velo_only) */
    int64_t *counts;       /* [n_tracks * 4]: doublet pairs, filtered doublets, triplets, valid candidates */
    int32_t *trip;         /* [n_tracks * n_triplets * 4]: set + 2*side, h0, h1, h2 (rank order; -1 padded) */
    float *trip_chi2;      /* [n_tracks * n_triplets] */
    float *cand_Q;         /* [n_tracks * n_triplets]: Q of each candidate, NaN if rejected earlier */
    int32_t *cand_hits;    /* [n_tracks * n_triplets * 12]: hits after extension, -1 = none */
    int32_t *win1;         /* [n_tracks * 24]: side 1 windows (velo_only) */
    float *wx1;            /* [n_tracks * 36]: side 1 x_min, centre, x_max (velo_only) */
} lfo_debug;

void lfo_default_params(lfo_params *p);
/* The "Forward no-UT" tuning: VELO-only input and its tolerances. */
void lfo_default_params_no_ut(lfo_params *p);

/* Runs events [ev_begin, ev_end) of the batch.  Arrays are the whole batch:
 * hit_off[24*n_events+1] (bucket = 24*event + 2*layer + zone), hits sorted
 * by non-decreasing x inside each bucket; trk_off[n_events+1].  Output and
 * debug arrays are indexed by the global track index.  Returns 0, or -1 on
 * an argument error. */
int lfo_find_tracks(const lfo_geometry *g, const lfo_params *P, uint32_t n_events,
                    const uint32_t *hit_off, const float *hit_x, const float *hit_z,
                    const float *hit_dxdy, const uint32_t *trk_off, const float *trk_x,
                    const float *trk_y, const float *trk_tx, const float *trk_ty,
                    const float *trk_qop, uint32_t ev_begin, uint32_t ev_end,
                    lfo_out *out, lfo_debug *dbg);

/* The binary16 value nearest to x, as a binary32 (round to nearest even,
 * subnormals, overflow to infinity): the rounding of the binary16 seeding. */
float lfo_h16(float x);

#endif

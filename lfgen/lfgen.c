/*
 * lfgen.c -- seeded synthetic SciFi events with truth, for the forward
 * tracking step (Looking Forward, arXiv 2402.14670).
 *
 * This module only simulates the world: particles from the origin, a toy
 * single-kick magnet, twelve x-u-v-x SciFi layers split into y>0 / y<0
 * zones, hit smearing, noise hits and upstream (VELO-UT) track states.  It
 * holds none of the track-finding arithmetic.  Both the CPU oracle and the
 * GPU library consume its arrays; neither is linked to it.
 *
 * Detector layout follows the paper's Context section (three stations of
 * x-u-v-x layers, stereo +-5 degrees) and the "Defining the search windows"
 * subsection (about 400 hits per layer, y>0 / y<0 halves).  The field is a
 * toy: an instantaneous kick at z_mag that changes the slope from tx to
 * tx_f, then
 *   x(z) = tx*z_mag + tx_f*(z - z_mag) + kappa*d*(z - z_T)^2 (1 + dRatio (z - z_T)),
 *   y(z) = ty*z,   d = tx_f - tx,
 * which is the track model of the paper's "Propagation" section (dRatio = 0:
 * a constant B_y tail; dRatio < 0: a linearly falling one).  Two kicks:
 *   field_form 0: tx_f = tx + kick * q/p;
 *   field_form 1: the sqrt-normalised pt-kick equation of "Defining the search
 *     windows", s_f = s_i + (q/p) BL with s = tx / sqrt(1 + tx^2 + ty^2) and
 *     ty unchanged, where the integrated field BL = bl0 (1 + bl_tx2 tx^2 +
 *     bl_ty2 ty^2 + bl_q2 (bl0 q/p)^2) falls for steep and for strongly
 *     bending tracks, so that the momentum parametrisation F(tx, ty, dSlope)
 *     of "Calculation of momentum" has work to do.  A particle with
 *     |s_f| >= 1 curls up in the magnet and leaves no SciFi hit.
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, 2018) seeded per event by
 * SplitMix64 (Steele, Lea & Flood, 2014); uniforms are (next >> 11) * 2^-53;
 * normals are Box-Muller in double; Poisson counts by CDF inversion.  No
 * std:: distribution is used, so the stream is fixed by this file alone.
 * Event e of a stream with seed S depends only on (S, e).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LFG_NL 12

typedef struct {
    uint64_t seed;
    int32_t first_event;      /* events [first_event, first_event + n_events) */
    int32_t n_events;
    int32_t n_particles;      /* per event, used when mu_int <= 0 */
    int32_t particles_per_int;
    double mu_int;            /* > 0: n_particles = Poisson(mu_int) * particles_per_int */
    double p_min, p_max;      /* GeV, log-uniform */
    double pt_min;            /* redraw while pt <= pt_min (0 disables) */
    double tx_max, ty_max;    /* |tx| < tx_max, |ty| < ty_max, uniform */
    double qop_sigma;         /* relative Gaussian smear of upstream q/p */
    int32_t n_true_tracks;    /* fixed count (mu_int <= 0); -1 = every particle */
    int32_t n_fake_tracks;    /* fixed count (mu_int <= 0) */
    double true_track_frac;   /* mu_int > 0: n_true = round(n_particles * frac) */
    double fake_ratio;        /* mu_int > 0: n_fake = round(n_true * ratio) */
    int32_t n_noise;          /* absolute noise hits per event */
    double noise_frac;        /* plus round(noise_frac * truth hits) */
    double hit_eff, sigma_x;  /* per-layer efficiency, x resolution (mm) */
    double x_acc, y_acc;      /* acceptance |x| < x_acc, |y| < y_acc (mm) */
    double z_up, z_mag, z_T, kick, kappa;
    double z[LFG_NL], dxdy[LFG_NL];
    int32_t field_form;       /* 0: linear kick; 1: sqrt-normalised pt-kick */
    double dRatio;            /* cubic term of the post-magnet x(z) */
    double bl0, bl_tx2, bl_ty2, bl_q2;   /* integrated field of field_form 1 */
} lfgen_config;

typedef struct {
    /* growable host arrays, whole stream */
    uint32_t n_events;
    size_t n_hits, cap_hits;
    size_t n_trk, cap_trk;
    size_t n_par, cap_par;
    uint32_t *hit_off;   /* [24*n_events+1] */
    uint32_t *trk_off;   /* [n_events+1] */
    uint32_t *par_off;   /* [n_events+1] */
    float *hx, *hz, *hdxdy;
    int32_t *hpid;       /* event-local particle index, -1 = noise */
    float *tx_, *ty_, *ttx, *tty, *tqop;
    int32_t *tpid;       /* event-local particle index, -1 = fake */
    float *pp, *pq, *ptx, *pty;
    uint16_t *pmask;     /* bit l set: the particle left a hit in layer l */
    uint8_t *phas;       /* the particle has an upstream input track */
} lfgen_out;

/* ---------------- PRNG ---------------- */
typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t out = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return out;
}
static void rng_seed(rng_t *r, uint64_t seed, uint64_t stream) {
    uint64_t x = seed ^ (stream * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull);
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}
static double unif(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
static double unif_ab(rng_t *r, double a, double b) { return a + (b - a) * unif(r); }
static double normal(rng_t *r) {
    double u1 = unif(r), u2 = unif(r);
    if (u1 <= 0.0) u1 = 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
static int poisson(rng_t *r, double mu) {
    double u = unif(r), pk = exp(-mu), cdf = pk;
    int k = 0;
    while (u > cdf && k < 100000) { ++k; pk *= mu / k; cdf += pk; }
    return k;
}

/* ---------------- growable arrays ---------------- */
static size_t next_cap(size_t cap, size_t need) {
    size_t nc = cap ? cap : 1024;
    while (nc < need) nc *= 2;
    return nc;
}
#define RESIZE(arr, n) do {                                  \
        void *q_ = realloc((arr), (n) * sizeof(*(arr)));         \
        if (!q_) { return -1; }                                  \
        (arr) = q_;                                              \
    } while (0)

static int reserve_hits(lfgen_out *o, size_t need) {
    if (need <= o->cap_hits) return 0;
    size_t nc = next_cap(o->cap_hits, need);
    RESIZE(o->hx, nc); RESIZE(o->hz, nc); RESIZE(o->hdxdy, nc); RESIZE(o->hpid, nc);
    o->cap_hits = nc;
    return 0;
}
static int reserve_trk(lfgen_out *o, size_t need) {
    if (need <= o->cap_trk) return 0;
    size_t nc = next_cap(o->cap_trk, need);
    RESIZE(o->tx_, nc); RESIZE(o->ty_, nc); RESIZE(o->ttx, nc);
    RESIZE(o->tty, nc); RESIZE(o->tqop, nc); RESIZE(o->tpid, nc);
    o->cap_trk = nc;
    return 0;
}
static int reserve_par(lfgen_out *o, size_t need) {
    if (need <= o->cap_par) return 0;
    size_t nc = next_cap(o->cap_par, need);
    RESIZE(o->pp, nc); RESIZE(o->pq, nc); RESIZE(o->ptx, nc);
    RESIZE(o->pty, nc); RESIZE(o->pmask, nc); RESIZE(o->phas, nc);
    o->cap_par = nc;
    return 0;
}

/* ---------------- one event ---------------- */
typedef struct { uint32_t bucket; float x; uint32_t order; float dxdy, z; int32_t pid; } rawhit;

static int cmp_rawhit(const void *a, const void *b) {
    const rawhit *p = (const rawhit *)a, *q = (const rawhit *)b;
    if (p->bucket != q->bucket) return p->bucket < q->bucket ? -1 : 1;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    if (p->order != q->order) return p->order < q->order ? -1 : 1;
    return 0;
}

typedef struct { double p, q, tx, ty; } kin;

/* Slope change d = tx_f - tx of the kick for entry slopes (tx, ty), charge q
 * and momentum p; returns 0 when the particle does not leave the magnet
 * forwards (field_form 1, |s_f| >= 1).  *bl receives the integrated field
 * the particle saw (kick for form 0). */
int lfgen_kick(const lfgen_config *c, double tx, double ty, double q, double p, double *d, double *bl) {
    if (c->field_form == 0) {
        *bl = c->kick;
        *d = c->kick * q / p;
        return 1;
    }
    double qop = q / p;
    double b = c->bl0 * qop;
    double BL = c->bl0 * (1.0 + c->bl_tx2 * tx * tx + c->bl_ty2 * ty * ty + c->bl_q2 * b * b);
    double si = tx / sqrt(1.0 + tx * tx + ty * ty);
    double sf = si + qop * BL;
    *bl = BL;
    if (!(fabs(sf) < 1.0)) { *d = 0.0; return 0; }
    *d = sf * sqrt((1.0 + ty * ty) / (1.0 - sf * sf)) - tx;
    return 1;
}

static kin draw_kin(rng_t *r, const lfgen_config *c) {
    kin k;
    for (;;) {
        k.q = unif(r) < 0.5 ? -1.0 : 1.0;
        k.p = exp(log(c->p_min) + unif(r) * (log(c->p_max) - log(c->p_min)));
        k.tx = unif_ab(r, -c->tx_max, c->tx_max);
        k.ty = unif_ab(r, -c->ty_max, c->ty_max);
        double t2 = k.tx * k.tx + k.ty * k.ty;
        double pt = k.p * sqrt(t2) / sqrt(1.0 + t2);
        if (c->pt_min <= 0.0 || pt > c->pt_min) return k;
    }
}

/* lfgen_kick over arrays (q/p given; q = sign, p = 1/|q/p|); ok[i] = 0 where
 * the particle does not leave the magnet forwards or q/p is 0. */
void lfgen_kick_many(const lfgen_config *c, int64_t n, const double *tx, const double *ty,
                     const double *qop, double *d, double *bl, uint8_t *ok) {
    for (int64_t i = 0; i < n; ++i) {
        if (qop[i] == 0.0) { d[i] = 0.0; bl[i] = 0.0; ok[i] = 0; continue; }
        double q = qop[i] > 0.0 ? 1.0 : -1.0;
        ok[i] = (uint8_t)lfgen_kick(c, tx[i], ty[i], q, 1.0 / fabs(qop[i]), &d[i], &bl[i]);
    }
}

static int gen_event(const lfgen_config *c, uint32_t ev_stream, lfgen_out *o, uint32_t ev_out) {
    rng_t r;
    rng_seed(&r, c->seed, ev_stream);

    int npar;
    if (c->mu_int > 0.0) npar = poisson(&r, c->mu_int) * c->particles_per_int;
    else npar = c->n_particles;

    size_t p0 = o->n_par;
    if (reserve_par(o, p0 + (size_t)npar)) return -1;

    /* particles and their hits */
    size_t cap_raw = (size_t)npar * LFG_NL + 16;
    rawhit *raw = (rawhit *)malloc(cap_raw * sizeof(rawhit));
    if (!raw) return -1;
    size_t nraw = 0;
    uint32_t order = 0;
    for (int i = 0; i < npar; ++i) {
        kin k = draw_kin(&r, c);
        double dtx, bl;
        int forward = lfgen_kick(c, k.tx, k.ty, k.q, k.p, &dtx, &bl);
        double T = k.tx + dtx;
        uint16_t mask = 0;
        for (int l = 0; l < LFG_NL; ++l) {
            double zl = c->z[l];
            double x = k.tx * c->z_mag + T * (zl - c->z_mag) +
                       c->kappa * dtx * (zl - c->z_T) * (zl - c->z_T) * (1.0 + c->dRatio * (zl - c->z_T));
            double y = k.ty * zl;
            double ue = unif(&r);
            double nx = normal(&r);
            if (forward && fabs(x) < c->x_acc && fabs(y) < c->y_acc && ue < c->hit_eff) {
                rawhit h;
                h.bucket = (uint32_t)(l * 2 + (y >= 0.0 ? 1 : 0));
                h.x = (float)(x - c->dxdy[l] * y + c->sigma_x * nx);
                h.z = (float)zl;
                h.dxdy = (float)c->dxdy[l];
                h.pid = i;
                h.order = order++;
                raw[nraw++] = h;
                mask |= (uint16_t)(1u << l);
            }
        }
        o->pp[p0 + i] = (float)k.p;
        o->pq[p0 + i] = (float)k.q;
        o->ptx[p0 + i] = (float)k.tx;
        o->pty[p0 + i] = (float)k.ty;
        o->pmask[p0 + i] = mask;
        o->phas[p0 + i] = 0;
    }
    size_t ntruth = nraw;
    long nnoise = c->n_noise + lround(c->noise_frac * (double)ntruth);
    if (nnoise < 0) nnoise = 0;
    rawhit *raw2 = (rawhit *)realloc(raw, (nraw + (size_t)nnoise + 1) * sizeof(rawhit));
    if (!raw2) { free(raw); return -1; }
    raw = raw2;
    for (long i = 0; i < nnoise; ++i) {
        int l = (int)(unif(&r) * LFG_NL);
        if (l >= LFG_NL) l = LFG_NL - 1;
        int zone = unif(&r) < 0.5 ? 0 : 1;
        rawhit h;
        h.bucket = (uint32_t)(l * 2 + zone);
        h.x = (float)unif_ab(&r, -c->x_acc, c->x_acc);
        h.z = (float)c->z[l];
        h.dxdy = (float)c->dxdy[l];
        h.pid = -1;
        h.order = order++;
        raw[nraw++] = h;
    }
    qsort(raw, nraw, sizeof(rawhit), cmp_rawhit);

    size_t h0 = o->n_hits;
    if (reserve_hits(o, h0 + nraw)) { free(raw); return -1; }
    uint32_t *off = o->hit_off + (size_t)ev_out * 24;
    size_t j = 0;
    for (uint32_t b = 0; b < 24; ++b) {
        off[b] = (uint32_t)(h0 + j);
        while (j < nraw && raw[j].bucket == b) {
            o->hx[h0 + j] = raw[j].x;
            o->hz[h0 + j] = raw[j].z;
            o->hdxdy[h0 + j] = raw[j].dxdy;
            o->hpid[h0 + j] = raw[j].pid;
            ++j;
        }
    }
    off[24] = (uint32_t)(h0 + nraw);
    o->n_hits = h0 + nraw;
    free(raw);

    /* upstream input tracks */
    int ntrue, nfake;
    if (c->mu_int > 0.0) {
        ntrue = (int)lround((double)npar * c->true_track_frac);
        nfake = (int)lround((double)ntrue * c->fake_ratio);
    } else {
        ntrue = c->n_true_tracks < 0 ? npar : c->n_true_tracks;
        nfake = c->n_fake_tracks;
    }
    if (ntrue > npar) ntrue = npar;
    int ntrk = ntrue + nfake;
    size_t t0 = o->n_trk;
    if (reserve_trk(o, t0 + (size_t)ntrk)) return -1;

    /* choose ntrue particles uniformly without replacement (partial shuffle) */
    int *idx = (int *)malloc(((size_t)npar + 1) * sizeof(int));
    if (!idx) return -1;
    for (int i = 0; i < npar; ++i) idx[i] = i;
    for (int i = 0; i < ntrue; ++i) {
        int k = i + (int)(unif(&r) * (double)(npar - i));
        if (k >= npar) k = npar - 1;
        int t = idx[i]; idx[i] = idx[k]; idx[k] = t;
    }
    for (int i = 0; i < ntrue; ++i) {
        int pi = idx[i];
        double p = o->pp[p0 + pi], q = o->pq[p0 + pi];
        double tx = o->ptx[p0 + pi], ty = o->pty[p0 + pi];
        double f;
        do { f = 1.0 + c->qop_sigma * normal(&r); } while (f <= 0.0);
        o->tx_[t0 + i] = (float)(c->z_up * tx);
        o->ty_[t0 + i] = (float)(c->z_up * ty);
        o->ttx[t0 + i] = (float)tx;
        o->tty[t0 + i] = (float)ty;
        o->tqop[t0 + i] = (float)(q / p * f);
        o->tpid[t0 + i] = pi;
        o->phas[p0 + pi] = 1;
    }
    free(idx);
    for (int i = ntrue; i < ntrk; ++i) {
        kin k = draw_kin(&r, c);
        o->tx_[t0 + i] = (float)(c->z_up * k.tx);
        o->ty_[t0 + i] = (float)(c->z_up * k.ty);
        o->ttx[t0 + i] = (float)k.tx;
        o->tty[t0 + i] = (float)k.ty;
        o->tqop[t0 + i] = (float)(k.q / k.p);
        o->tpid[t0 + i] = -1;
    }
    /* shuffle the input tracks of this event (Fisher-Yates) */
    for (int i = ntrk - 1; i > 0; --i) {
        int k = (int)(unif(&r) * (double)(i + 1));
        if (k > i) k = i;
#define SWP(a) do { __typeof__(a[0]) t_ = a[t0 + i]; a[t0 + i] = a[t0 + k]; a[t0 + k] = t_; } while (0)
        SWP(o->tx_); SWP(o->ty_); SWP(o->ttx); SWP(o->tty); SWP(o->tqop); SWP(o->tpid);
#undef SWP
    }
    o->n_trk = t0 + (size_t)ntrk;
    o->trk_off[ev_out] = (uint32_t)t0;
    o->trk_off[ev_out + 1] = (uint32_t)o->n_trk;
    o->par_off[ev_out] = (uint32_t)p0;
    o->n_par = p0 + (size_t)npar;
    o->par_off[ev_out + 1] = (uint32_t)o->n_par;
    return 0;
}

/* ---------------- public API ---------------- */
void lfgen_free(lfgen_out *o) {
    if (!o) return;
    free(o->hit_off); free(o->trk_off); free(o->par_off);
    free(o->hx); free(o->hz); free(o->hdxdy); free(o->hpid);
    free(o->tx_); free(o->ty_); free(o->ttx); free(o->tty); free(o->tqop); free(o->tpid);
    free(o->pp); free(o->pq); free(o->ptx); free(o->pty); free(o->pmask); free(o->phas);
    free(o);
}

static lfgen_out *new_out(uint32_t n_events) {
    lfgen_out *o = (lfgen_out *)calloc(1, sizeof(lfgen_out));
    if (!o) return NULL;
    o->n_events = n_events;
    o->hit_off = (uint32_t *)calloc((size_t)n_events * 24 + 1, sizeof(uint32_t));
    o->trk_off = (uint32_t *)calloc((size_t)n_events + 1, sizeof(uint32_t));
    o->par_off = (uint32_t *)calloc((size_t)n_events + 1, sizeof(uint32_t));
    if (!o->hit_off || !o->trk_off || !o->par_off) { lfgen_free(o); return NULL; }
    return o;
}

/* Generates the events (in parallel: every event has its own random
 * stream, so the result does not depend on the thread count); returns NULL
 * on bad configuration or out of memory. */
lfgen_out *lfgen_run(const lfgen_config *c) {
    if (!c || c->n_events < 0 || c->first_event < 0 || c->p_min <= 0.0 || c->p_max < c->p_min)
        return NULL;
    const int E = c->n_events;
    lfgen_out **parts = (lfgen_out **)calloc((size_t)E + 1, sizeof(lfgen_out *));
    if (!parts) return NULL;
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : failed)
    for (int e = 0; e < E; ++e) {
        lfgen_out *p = new_out(1);
        if (!p || gen_event(c, (uint32_t)(c->first_event + e), p, 0)) failed |= 1;
        parts[e] = p;
    }
    lfgen_out *o = failed ? NULL : new_out((uint32_t)E);
    size_t H = 0, T = 0, Pn = 0;
    if (o) {
        for (int e = 0; e < E; ++e) { H += parts[e]->n_hits; T += parts[e]->n_trk; Pn += parts[e]->n_par; }
        if (H > 0xFFFFFFF0ull || reserve_hits(o, H + 1) || reserve_trk(o, T + 1) || reserve_par(o, Pn + 1)) {
            lfgen_free(o);
            o = NULL;
        }
    }
    if (o) {
        size_t h = 0, t = 0, q = 0;
        for (int e = 0; e < E; ++e) {
            const lfgen_out *p = parts[e];
            for (int b = 0; b < 24; ++b) o->hit_off[(size_t)e * 24 + b] = (uint32_t)(h + p->hit_off[b]);
            o->trk_off[e] = (uint32_t)t;
            o->par_off[e] = (uint32_t)q;
            memcpy(o->hx + h, p->hx, p->n_hits * 4); memcpy(o->hz + h, p->hz, p->n_hits * 4);
            memcpy(o->hdxdy + h, p->hdxdy, p->n_hits * 4); memcpy(o->hpid + h, p->hpid, p->n_hits * 4);
            memcpy(o->tx_ + t, p->tx_, p->n_trk * 4); memcpy(o->ty_ + t, p->ty_, p->n_trk * 4);
            memcpy(o->ttx + t, p->ttx, p->n_trk * 4); memcpy(o->tty + t, p->tty, p->n_trk * 4);
            memcpy(o->tqop + t, p->tqop, p->n_trk * 4); memcpy(o->tpid + t, p->tpid, p->n_trk * 4);
            memcpy(o->pp + q, p->pp, p->n_par * 4); memcpy(o->pq + q, p->pq, p->n_par * 4);
            memcpy(o->ptx + q, p->ptx, p->n_par * 4); memcpy(o->pty + q, p->pty, p->n_par * 4);
            memcpy(o->pmask + q, p->pmask, p->n_par * 2); memcpy(o->phas + q, p->phas, p->n_par);
            h += p->n_hits; t += p->n_trk; q += p->n_par;
        }
        o->hit_off[(size_t)E * 24] = (uint32_t)h;
        o->trk_off[E] = (uint32_t)t;
        o->par_off[E] = (uint32_t)q;
        o->n_hits = h; o->n_trk = t; o->n_par = q;
    }
    for (int e = 0; e < E; ++e) lfgen_free(parts[e]);
    free(parts);
    return o;
}

void lfgen_sizes(const lfgen_out *o, uint64_t *n_events, uint64_t *n_hits, uint64_t *n_trk, uint64_t *n_par) {
    *n_events = o->n_events; *n_hits = o->n_hits; *n_trk = o->n_trk; *n_par = o->n_par;
}

/* Copies every array into caller buffers sized from lfgen_sizes. */
void lfgen_copy(const lfgen_out *o,
                uint32_t *hit_off, float *hx, float *hz, float *hdxdy, int32_t *hpid,
                uint32_t *trk_off, float *tx, float *ty, float *ttx, float *tty, float *tqop, int32_t *tpid,
                uint32_t *par_off, float *pp, float *pq, float *ptx, float *pty, uint16_t *pmask, uint8_t *phas) {
    size_t E = o->n_events, H = o->n_hits, T = o->n_trk, P = o->n_par;
    memcpy(hit_off, o->hit_off, (E * 24 + 1) * sizeof(uint32_t));
    if (E == 0) hit_off[0] = 0;
    if (H) {
        memcpy(hx, o->hx, H * 4); memcpy(hz, o->hz, H * 4);
        memcpy(hdxdy, o->hdxdy, H * 4); memcpy(hpid, o->hpid, H * 4);
    }
    memcpy(trk_off, o->trk_off, (E + 1) * sizeof(uint32_t));
    if (T) {
        memcpy(tx, o->tx_, T * 4); memcpy(ty, o->ty_, T * 4); memcpy(ttx, o->ttx, T * 4);
        memcpy(tty, o->tty, T * 4); memcpy(tqop, o->tqop, T * 4); memcpy(tpid, o->tpid, T * 4);
    }
    memcpy(par_off, o->par_off, (E + 1) * sizeof(uint32_t));
    if (P) {
        memcpy(pp, o->pp, P * 4); memcpy(pq, o->pq, P * 4); memcpy(ptx, o->ptx, P * 4);
        memcpy(pty, o->pty, P * 4); memcpy(pmask, o->pmask, P * 2); memcpy(phas, o->phas, P);
    }
}

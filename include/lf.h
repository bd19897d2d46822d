/*
 * lf.h -- Looking Forward track following on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the GPU library.  The method is the forward tracking step of
 * "Looking Forward: A High-Throughput Track Following Algorithm for Parallel
 * Architectures" (arXiv 2402.14670): each upstream (VELO-UT) track state is
 * extended into the twelve SciFi layers (three stations of x-u-v-x layers,
 * Context section) by
 *   1. search windows in every layer from a pt-kick extrapolation
 *      ("Defining the search windows"),
 *   2. triplet seeding on x layers ("Triplet Seeding"),
 *   3. extension to the remaining x and stereo layers ("Extending triplets
 *      to other layers", track-fit model equation of the "Propagation" section),
 *   4. least-squares fits and the quality factor Q ("Quality Filter",
 *      C(n_hits) table), keeping the best candidate per input track,
 * followed by the momentum and state computation ("Calculation of momentum
 * and track states").  Every step runs in hand-written HIP kernels.
 *
 * Conventions
 *  - Every call returns LF_OK (0) or a negative LF_ERR_* code; no exception
 *    crosses the ABI and the library never exits the process.  After an
 *    error, lf_last_error(ctx) describes it.
 *  - Units are mm and GeV/c.  Arithmetic is IEEE binary32 (round to nearest
 *    even, no contraction into FMA, correctly rounded division), evaluated in
 *    a fixed order, so results do not depend on batch composition, event
 *    order or launch configuration.
 *  - A context is not thread-safe: use one per thread or serialise calls.
 *  - hip_stream arguments take a hipStream_t (for instance a PyTorch stream
 *    handle) or NULL for the context's own stream.  All streams run at the
 *    default priority.
 */
#ifndef LF_H
#define LF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LF_NLAYERS 12

/* Opaque context, owned by the library (lf_create / lf_destroy). */
typedef struct lf_ctx lf_ctx;

enum {
    LF_OK = 0,
    LF_ERR_INVALID = -1,   /* bad argument or malformed batch (NaN/inf, q/p == 0, unsorted bucket, bad offsets) */
    LF_ERR_TOO_LARGE = -2, /* the batch does not fit the context's device-memory budget */
    LF_ERR_NOMEM = -3,     /* host or device allocation failed */
    LF_ERR_DEVICE = -4,    /* a HIP runtime call failed */
    LF_ERR_STATE = -5      /* unknown batch id, or a call out of order */
};

/* Execution modes of lf_find_tracks (all write identical results). */
enum {
    LF_MODE_PLAIN = 0,      /* one kernel launch per event */
    LF_MODE_BATCHED = 1,    /* one launch over the whole batch, one wavefront per input track,
                               tracks ordered so each XCD takes a contiguous run of events */
    LF_MODE_PERSISTENT = 2  /* one launch of resident wavefronts pulling (event, track) work
                               items from per-XCD device queues */
};

/* Work counters filled by lf_work_counts, indices into its counts array. */
enum {
    LF_WC_TRACKS = 0,        /* input tracks */
    LF_WC_PAIRS_ALL = 1,     /* (h0, h2) pairs of both seed sets in the windows */
    LF_WC_SEED_ITEMS = 2,    /* first-layer hits whose h2 range was bracketed */
    LF_WC_PAIRS_TESTED = 3,  /* pairs the doublet filters were evaluated on */
    LF_WC_DOUBLETS = 4,      /* pairs passing both doublet filters */
    LF_WC_TRIPLETS = 5,      /* triplets with chi2 < T_triplet */
    LF_WC_KEPT = 6,          /* triplets kept (at most n_triplets per track) */
    LF_WC_FITTED = 7,        /* candidates passing the 9-hit / station rule (fitted) */
    LF_WC_ACCEPTED = 8,      /* candidates with Q < T_Q */
    LF_WC_STAGED_HITS = 9,   /* window hits staged */
    LF_WC_FOUND = 10,        /* tracks found */
    /* shader-clock cycles per wavefront spent in each phase, summed over tracks */
    LF_WC_CY_WINDOWS = 11, LF_WC_CY_STAGE = 12, LF_WC_CY_DOUBLETS = 13, LF_WC_CY_MODEL = 14,
    LF_WC_CY_EXTEND = 15, LF_WC_CY_FIT = 16, LF_WC_CY_SELECT = 17,
    LF_WC_N = 18
};

/* Detector and field description.  Layers 0..11 are three stations of
 * x-u-v-x planes: x layers 0,3,4,7,8,11 and stereo layers 1,2,5,6,9,10
 * (Context section).  The field enters through the pt-kick at z_mag ("Defining
 * the search windows") and the x(z) model of the "Propagation" section with
 * residual curvature kappa*dtx about z_T and cubic term dRatio:
 *   x(z) = x_mag + (tx + dtx)(z - z_mag) + kappa dtx (z - z_T)^2 (1 + dRatio (z - z_T)).
 * Two forms of the kick and of the momentum (field_form):
 *   0: dtx = kick * q/p, and q/p = (tx(z_T) - tx) / kick from the fit;
 *   1: the sqrt-normalised pt-kick equation s_f - s_i = (q/p) F with
 *      s = tx / sqrt(1 + tx^2 + ty^2) and the integrated field F the
 *      fourth-order polynomial in dSlope of "Calculation of momentum and
 *      track states", F = sum_{i=0..4} c_i dSlope^i, evaluated as
 *      c0 + d (c1 + d (c2 + d (c3 + d c4))), whose coefficients are 2D
 *      polynomials of the input slopes:
 *        c_i = sum_{j=0..9} F_coef[i][j] m_j          (i even)
 *        c_i = tx * sum_{j=0..5} F_coef[i][j] m_j     (i odd; j = 6..9 unused)
 *      m = (1, tx2, ty2, tx2^2, tx2 ty2, ty2^2, tx2^3, tx2^2 ty2, tx2 ty2^2,
 *      ty2^3), tx2 = tx^2, ty2 = ty^2, sums in order of j.  For the windows
 *      the equation is solved for the slope after the magnet with F at
 *      dSlope = 0 and then twice at the previous solution's slope change
 *      (ty unchanged); a track whose kick has no solution (|s_f| >= 1) gets
 *      no windows and is not found.  The output q/p uses the fitted slopes at
 *      z_T and F at dSlope = tx(z_T) - tx.  With velo_only the windows are
 *      straight lines in either form. */
typedef struct {
    float z[LF_NLAYERS];     /* z of each layer plane */
    float dxdy[LF_NLAYERS];  /* stereo tangent (0 for x layers, +-tan 5 deg for u/v) */
    float z_in;              /* z of the upstream track states */
    float z_mag;             /* bending plane z_bending */
    float z_ref;             /* reference plane of the track model (8520 mm) */
    float z_T;               /* plane where the post-magnet slope is read for q/p */
    float kick;              /* field_form 0: dtx = kick * q/p (non-zero) */
    float kappa;             /* residual curvature per unit dtx */
    float dRatio;            /* cubic term of x(z) */
    int32_t polarity;        /* +1: q > 0 bends towards +x; -1 the opposite */
    int32_t field_form;      /* 0: linear kick; 1: sqrt-normalised pt-kick with F (above) */
    float F_coef[5][10];     /* field_form 1: coefficients of F (finite; zero for form 0) */
} lf_geometry;

/* Tunable parameters.  Defaults (lf_default_params) are the "Forward"
 * column of the paper's table of tolerances and its C(n_hits) table, plus
 * the readings the paper leaves open (magnet tolerance form, T_uv floor). */
typedef struct {
    float T_triplet;       /* middle-hit chi2 tolerance (mm^2), 8 */
    float T_x;             /* x-layer extension chi2 tolerance (mm^2), 2 */
    float T_uv_scale;      /* T_uv = T_uv_scale * (|tx| + |ty|), 50 */
    float T_uv_floor;      /* lower bound of T_uv (mm^2), 2 */
    float T_ty;            /* |ty_fit - ty_in| tolerance, 0.02 */
    float T_y;             /* y residual normalisation (mm^2), 800 */
    float T_Q;             /* quality factor cut, 0.5 */
    float xtol_const;      /* x_tol = xtol_const + xtol_pscale / p: 150 mm */
    float xtol_pscale;     /* 2000 mm GeV */
    float xasym;           /* window asymmetry on the bending side, 100 mm */
    float uv_halfwidth;    /* stereo-layer window half width, 800 mm */
    float K_first;         /* middle-hit correction, first-layer set, 1.00177513 */
    float K_last;          /* middle-hit correction, last-layer set, 1.00142634 */
    float magtol_const;    /* magnet opening tolerance = const + pscale/p + txscale*|tx|, */
    float magtol_pscale;   /*   clamped to [magtol_min, magtol_max]: 8 + 24/p + 20|tx| in [8, 40] mm */
    float magtol_txscale;
    float magtol_min;
    float magtol_max;
    float p_charge_cut;    /* below this p (GeV) the doublet must bend with the charge, 5 */
    float C_nhits[4];      /* C(9), C(10), C(11), C(12): 5.0, 1.0, 0.8, 0.5 */
    int32_t n_hits_window; /* hits kept per window (1..64), 32 */
    int32_t n_triplets;    /* triplets kept per input track (1..32), 12 */
    /* No-UT tuning (arXiv 2402.14670, "No-UT tuning" subsection): VELO input
     * tracks without a momentum.  velo_only = 1 ignores trk_qop, extrapolates
     * each track as a straight line, assumes the momentum
     * p = max(noUT_p_min, noUT_pt_min / sin(theta)), and gives every layer
     * two windows, [x - tol, x + overlap] and [x - overlap, x + tol], one per
     * charge, with tol the polynomial below on x layers (the paper's window
     * tolerance equation, coefficients c0..c7 of its table) and uv_halfwidth
     * on u/v layers; each charge side seeds its own triplets and the n_triplets
     * best of both go on.  lf_default_params_no_ut() fills the paper's
     * "Forward no-UT" column. */
    int32_t velo_only;     /* 0: VELO-UT input (default); 1: VELO-only input */
    float noUT_c[8];       /* x_tol polynomial coefficients, mm GeV^k */
    float noUT_p_min;      /* assumed minimum momentum, GeV: 5 */
    float noUT_pt_min;     /* assumed minimum transverse momentum, GeV: 1 */
    float noUT_overlap;    /* overlap of the two windows of a layer, mm: 5 */
    /* Triplet seeding in binary16 (the paper's Performance section: seeding
     * needs only half precision and runs two combinations per half2
     * instruction).  seed_fp16 = 1: for a seed set whose first- and
     * last-layer windows each share one z, every (h0, h2) pair is tested and
     * the doublet slope, the charge and magnet filters and the middle-hit
     * search and chi2 are evaluated in binary16 on coordinates relative to
     * the window centres c_l (x - c_l rounded to binary16; per-set constants
     * rounded once from binary32), two pairs per packed instruction; other
     * sets and all other steps stay binary32.  Results are a separate parity
     * domain from seed_fp16 = 0.  VELO-UT input only (velo_only = 0), else
     * LF_ERR_INVALID. */
    int32_t seed_fp16;     /* 0 (default) or 1 */
} lf_params;

/* A batch of events in host memory, ragged structure-of-arrays.  Hits are
 * bucket-major: bucket b = 24*event + 2*layer + zone (zone 1 = y > 0 half,
 * zone 0 = y < 0 half); hits of bucket b are [hit_off[b], hit_off[b+1]) with
 * hit_off[0] == 0, and x is non-decreasing inside each bucket.  hit_x is the
 * x of the fibre at y = 0, hit_z its z, hit_dxdy its stereo tangent.  Track
 * states (x, y, tx, ty, q/p) are at z = z_in; tracks of event e are
 * [trk_off[e], trk_off[e+1]).  The library copies everything; the caller
 * keeps ownership of these buffers. */
typedef struct {
    uint32_t n_events;
    const uint32_t *hit_off;   /* [24*n_events + 1] */
    const float *hit_x, *hit_z, *hit_dxdy;
    const uint32_t *trk_off;   /* [n_events + 1] */
    const float *trk_x, *trk_y, *trk_tx, *trk_ty, *trk_qop;
} lf_batch;

/* Caller-allocated host output, one slot per input track (global track
 * order of the batch).  hit_idx[12*t + layer] is an event-local hit index
 * (index among the event's hits in bucket-major order) or -1.  a, b, c are
 * x, dx/dz and the curvature coefficient at z_ref; y0, ty the y line at
 * z_ref; qop the refined q/p; Q the quality factor.  Not-found tracks have
 * found = 0, n_hits = 0, hit_idx = -1 and zero parameters. */
typedef struct {
    uint8_t *found, *n_hits;
    int32_t *hit_idx;
    float *a, *b, *c, *y0, *ty, *qop, *Q;
} lf_tracks_out;

/* Launch configuration of the kernels (lf_set_exec).  Zero fields keep the
 * current value. */
typedef struct {
    int32_t waves_per_block;   /* 1, 2 or 4 wavefronts per workgroup */
    int32_t items_per_grab;    /* tracks a wavefront takes per queue claim (persistent mode), 1..16 */
    int32_t blocks_per_cu;     /* persistent grid = blocks_per_cu * compute units (persistent mode) */
} lf_exec;

/* Fills *p with the default parameters. */
void lf_default_params(lf_params *p);

/* Fills *p with the "Forward no-UT" parameters (velo_only = 1): T_triplet 2,
 * T_x 0.5, T_uv 15 (|tx| + |ty|) with the same floor, T_ty 0.003, T_y 800,
 * T_Q 0.5, 64 hits per window, 20 triplets, u/v tolerance 1200 mm, magnet
 * tolerance fixed at 10 mm, no bend-direction filter, the polynomial
 * coefficients 4824.3, 426.3, 7071.1, 12080.4, 14077.8, 13909.3, 9315.3,
 * 3209.5, p_min 5 GeV, pt_min 1 GeV, overlap 5 mm.  For the callers that
 * run VELO-only input, as the paper's 2022 trigger did. */
void lf_default_params_no_ut(lf_params *p);

/* Creates a context on the current HIP device (the detector of the Context
 * section; tolerances of the Table of parameters and tolerances and the
 * C(n_hits) table of the Quality Filter section).  Geometry and parameters are
 * copied.  device_budget_bytes bounds the device memory of all resident
 * batches together with the one freed block the context keeps for reuse
 * (0 = no bound).  Errors: LF_ERR_INVALID (NULL pointers, parameters out of
 * range), LF_ERR_DEVICE, LF_ERR_NOMEM. */
int lf_create(const lf_geometry *geom, const lf_params *params, size_t device_budget_bytes,
              lf_ctx **out);

/* Validates a host batch without touching the device: LF_OK, or
 * LF_ERR_INVALID with the reason in lf_last_error(NULL).  Checked: offsets
 * start at 0 and never decrease; fewer than 2^26 events, 2^30 hits and 2^26
 * tracks (device arrays stay below 4 GiB); no NULL array that has elements;
 * finite hits and track states; q/p != 0; x sorted inside every bucket.
 * lf_upload_events runs the same checks. */
int lf_check_batch(const lf_batch *batch);

/* The step's input (Algorithm logic: upstream track states and the SciFi
 * hits of each event).  Validates a host batch, copies it to device memory
 * (on hip_stream) and returns its id.  Input and output buffers of the batch stay resident until
 * lf_fetch_tracks or lf_release_batch.  The inputs pass through a pinned host
 * buffer that the context keeps (grown to the largest batch or result set
 * seen, held until lf_destroy); the call returns once they are on the
 * device.  The batch's device block is the one the context kept from the
 * last batch it freed when that fits (at least the size needed and at most
 * twice it), else a new allocation.  Errors: LF_ERR_INVALID (malformed batch; nothing is copied),
 * LF_ERR_TOO_LARGE (over budget), LF_ERR_NOMEM, LF_ERR_DEVICE. */
int lf_upload_events(lf_ctx *ctx, const lf_batch *batch, void *hip_stream, uint64_t *batch_id);

/* The whole step of Algorithm logic: search windows (Defining the search
 * windows), Triplet Seeding, Extending triplets to other layers, Quality
 * Filter and Calculation of momentum and track states.  Enqueues it for a
 * resident batch on hip_stream and returns without waiting.  mode is LF_MODE_PLAIN, LF_MODE_BATCHED or
 * LF_MODE_PERSISTENT; all modes write identical results.  May be called again on
 * the same batch (results are rewritten).  Errors: LF_ERR_STATE (unknown
 * batch), LF_ERR_INVALID (mode), LF_ERR_DEVICE. */
int lf_find_tracks(lf_ctx *ctx, uint64_t batch_id, int mode, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the hot
 * path of lf_find_tracks over a batch that already sits in device memory,
 * writing into caller-allocated device outputs, with no allocation of any
 * kind.  in holds DEVICE pointers in the lf_batch layout (in->n_events is a
 * host value; the batch must be well formed as lf_check_batch defines it:
 * it is not validated, since that would need a copy to the host);
 * n_hits = hit_off[24*n_events] and n_tracks = trk_off[n_events] are passed
 * by the caller; out holds DEVICE pointers in the lf_tracks_out layout, at
 * least n_tracks slots.  The caller owns all of these and keeps them valid
 * until the work completes.  mode is LF_MODE_BATCHED or LF_MODE_PERSISTENT
 * (the per-event mode needs host offsets).  Results equal those of
 * lf_upload_events + lf_find_tracks on the same batch.  Enqueues kernels on
 * hip_stream and returns without waiting.
 * Scratch: one fixed device array per GPU, part of the library's code
 * object (17 MiB, held until the process ends): the persistent queue words
 * (cleared by a kernel at every call), one byte per event and one word per
 * track.  Limits: at most 2^20 events and 2^22 tracks per call
 * (LF_ERR_TOO_LARGE beyond, nothing launched), fewer than 2^30 hits.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from several contexts or threads) race and must be
 * serialised by the caller.  Errors: LF_ERR_INVALID (NULL pointer, mode,
 * hit count), LF_ERR_TOO_LARGE, LF_ERR_STATE, LF_ERR_DEVICE. */
int lf_find_tracks_noalloc(lf_ctx *ctx, const lf_batch *in, uint32_t n_hits, uint32_t n_tracks,
                           const lf_tracks_out *out, int mode, void *hip_stream);

/* Runs the hot path once more over a resident batch in a counting build of
 * the kernel and writes the total work counters (LF_WC_*) to counts[0..n):
 * the units the roofline's algorithmic operation count is built from.
 * Synchronous; the results of the batch are rewritten (identically).
 * Errors: LF_ERR_STATE, LF_ERR_INVALID (NULL counts), LF_ERR_DEVICE. */
int lf_work_counts(lf_ctx *ctx, uint64_t batch_id, void *hip_stream, int64_t *counts, size_t n_counts);

/* The step's output: at most one forward track per input track, the best
 * candidate of the Quality Filter section, with its fitted x(z) and y(z)
 * parameters and the q/p of Calculation of momentum and track states.
 * Copies the results of a batch into caller buffers holding at least
 * cap_tracks >= number of input tracks slots (through the context's pinned
 * buffer, as in lf_upload_events), waits for completion and
 * frees the batch (its device block is kept for reuse, as lf_release_batch
 * describes).  Errors: LF_ERR_STATE, LF_ERR_INVALID (NULL buffer or
 * cap_tracks too small; the batch stays resident), LF_ERR_DEVICE. */
int lf_fetch_tracks(lf_ctx *ctx, uint64_t batch_id, lf_tracks_out *out, size_t cap_tracks,
                    void *hip_stream);

/* Like lf_fetch_tracks, but the batch stays resident (results can be read
 * again after further lf_find_tracks calls or graph replays). */
int lf_copy_tracks(lf_ctx *ctx, uint64_t batch_id, lf_tracks_out *out, size_t cap_tracks, void *hip_stream);

/* Overwrites a resident batch's result slots with a poison pattern (found =
 * 0xFF, hit indices -2, parameters NaN) on hip_stream, with a kernel (no
 * memset), so that a later run that failed to write a slot is visible.
 * Errors: LF_ERR_STATE, LF_ERR_DEVICE. */
int lf_poison_tracks(lf_ctx *ctx, uint64_t batch_id, void *hip_stream);

/* Frees a resident batch without fetching it, after the device has
 * finished all queued work.  As in lf_fetch_tracks, the context keeps the
 * batch's device block for a later upload (the block kept before is freed;
 * lf_destroy frees it).  Errors: LF_ERR_STATE. */
int lf_release_batch(lf_ctx *ctx, uint64_t batch_id);

/* Sets the launch configuration used by later lf_find_tracks calls.
 * Errors: LF_ERR_INVALID (value out of range). */
int lf_set_exec(lf_ctx *ctx, const lf_exec *exec);

/* Sizes of a resident batch.  Any output pointer may be NULL.
 * Errors: LF_ERR_STATE. */
int lf_batch_info(lf_ctx *ctx, uint64_t batch_id, uint32_t *n_events, uint32_t *n_tracks,
                  uint32_t *n_hits, size_t *device_bytes);

/* Device bytes held by resident batches (the kept freed block is not
 * counted). */
size_t lf_device_bytes_in_use(const lf_ctx *ctx);

/* Captured launch sequences (HIP graphs).  A graph records the hot path
 * of n resident batches in the given mode and replays it with one launch
 * call.  Distinct batches are recorded as parallel branches (their launches
 * may overlap); a list that names a batch twice is recorded in order.  The
 * batches must stay resident (not fetched or released) while the graph is
 * used.  No memset node is recorded: the persistent mode's queue words
 * reset themselves. */
typedef struct lf_graph lf_graph;

/* Errors: LF_ERR_STATE (unknown batch), LF_ERR_INVALID, LF_ERR_DEVICE. */
int lf_graph_create(lf_ctx *ctx, const uint64_t *batch_ids, uint32_t n_batches, int mode, lf_graph **out);
/* Replays the graph on hip_stream (asynchronous).  Errors: LF_ERR_INVALID, LF_ERR_DEVICE. */
int lf_graph_launch(lf_ctx *ctx, lf_graph *graph, void *hip_stream);
/* Frees a graph (NULL is ignored). */
void lf_graph_destroy(lf_graph *graph);

/* Serving loop (continuous batching).  Configuration; zero fields take the
 * defaults in brackets. */
typedef struct {
    uint32_t max_batch_events;   /* events per launch, at most [1024] */
    uint32_t min_batch_events;   /* arrived events to wait for before launching [1] ... */
    uint32_t max_wait_us;        /* ... unless the oldest has waited this long [0] */
    uint32_t n_slots;            /* batches in flight, one stream each, 1..16 [4] */
    uint32_t n_pack_threads;     /* unused (0..64): batches are assembled on the device */
    uint32_t pool_on_device;     /* 0: the pool sits in pinned host memory and every batch reads its
                                    events over the host link [0]; 1: the pool is copied to device
                                    memory before the clock starts (events left in HBM by earlier
                                    GPU stages, as in a GPU trigger) and stays resident: a batch is a
                                    list of pool events, read in place */
    uint32_t results_on_device;  /* 0: every batch's results are copied to host memory [0]; 1: the
                                    results stay in the batch's device region (for later GPU stages)
                                    and only the per-event digests come back */
    uint32_t verify_results;     /* testing (0 or 1) [0]: with results_on_device = 0, each completed
                                    batch's results in host memory are compared byte for byte with the
                                    device copy (a synchronous copy inside the loop: not for timing) */
    size_t device_budget_bytes;  /* admission budget for resident events [8 GiB] */
} lf_serve_config;

typedef struct {
    uint64_t n_requests, n_batches;
    uint64_t max_queue;          /* most arrived requests waiting for admission at once */
    uint64_t max_device_bytes;   /* most device bytes held by admitted events at once */
    double wall_s;               /* first arrival to last completion */
    double events_per_s;         /* n_requests / wall_s */
    double lat_p50_s, lat_p99_s, lat_p999_s, lat_max_s;  /* arrival to results in host memory */
    double mean_batch_events;
    uint64_t bytes_in;           /* bytes over the host link into the device: the event blobs the gather
                                    reads from the pinned pool (offsets, hits, states; none with
                                    pool_on_device) and the batch descriptors */
    uint64_t bytes_out;          /* bytes over the host link out: digests and track slots */
    uint64_t result_mismatches;  /* verify_results: bytes of host results that differ from the device's */
} lf_serve_stats;

/* Runs a stream of requests through the serving loop and returns when all
 * have completed.  The pool is a batch of distinct events (host memory,
 * lf_batch layout; copied to pinned memory before the clock starts);
 * request i is event req_event[i] of the pool arriving arrival_s[i] seconds
 * after the start (non-decreasing; open loop: arrivals do not wait for
 * service).  Arrived requests queue on the host and are admitted into a
 * device ring of device_budget_bytes in arrival order (a request that does
 * not fit waits: backpressure, nothing is dropped).  Whenever one of
 * n_slots in-flight slots is free, every admitted request (up to
 * max_batch_events) forms one batch: the host writes one descriptor per
 * event, and on the slot's stream a gather kernel reads the events straight
 * from the pinned pool into the batch's device arrays, then the hot path
 * (LF_MODE_BATCHED), a digest kernel and the download of the results run.
 * req_digest[i] (optional) receives a 64-bit digest of request i's results
 * (FNV-1a over each track slot's 20 words -- found | n_hits << 8, 12 hit
 * indices, bits of a b c y0 ty qop Q -- summed as splitmix64(h ^ index *
 * 0x9E3779B97F4A7C15) over the event's tracks); req_latency_s[i]
 * (optional) its arrival-to-results-on-host latency.
 * With pool_on_device the pool is copied to device memory once, before the
 * clock (not charged to the budget), and a batch is its list of pool
 * events: the host uploads the list and the batch's result-slot offsets, a
 * kernel maps each slot to its pool track, and the hot path reads the pool
 * in place (no gather).  With results_on_device a request completes when its
 * digest is in host memory; its results stay in device memory.
 * Errors: LF_ERR_INVALID, LF_ERR_TOO_LARGE (an event exceeds the budget),
 * LF_ERR_NOMEM, LF_ERR_DEVICE. */
int lf_serve_run(lf_ctx *ctx, const lf_batch *pool, uint32_t n_requests, const uint32_t *req_event,
                 const double *arrival_s, const lf_serve_config *config, uint64_t *req_digest,
                 double *req_latency_s, lf_serve_stats *stats);

/* Destroys the context and frees every resident batch.  NULL is ignored. */
void lf_destroy(lf_ctx *ctx);

/* Message of the last error on ctx ("" if none); valid until the next call
 * on ctx.  With ctx == NULL, the last lf_create failure of this thread. */
const char *lf_last_error(const lf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif

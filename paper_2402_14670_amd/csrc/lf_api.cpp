// lf_api.cpp -- C ABI of the Looking Forward GPU library (declared in
// include/lf.h): contexts, batch validation and residency, launches and
// result retrieval.  The numerical work is all in lf_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lf.h"
#include "lf_internal.h"

namespace {

thread_local std::string g_create_error;

struct Batch {
    void *dmem = nullptr;
    size_t bytes = 0;
    lfk::DevBatch dev{};
    uint32_t n_events = 0, n_tracks = 0, n_hits = 0;
    std::vector<uint32_t> trk_off;  // host copy, for per-event launches
    size_t out_off = 0, out_bytes = 0;   // the result arrays: one run of the allocation
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Host threads for validation and staging copies (the host share of one GPU).
unsigned host_threads(size_t work) {
    if (work < (size_t(1) << 20)) return 1;
    const unsigned hw = std::thread::hardware_concurrency();
    return std::max(1u, std::min(hw ? hw : 1u, 16u));
}

// Host worker threads shared by every context, started on first use and kept
// until the process ends (the object is never destroyed, so no thread is
// joined at exit).  One parallel section runs at a time; a caller that finds
// the workers busy runs its section alone.  The caller takes part in its own
// section, so a section completes even with no worker at all.
class Workers {
public:
    static Workers &get() {
        static Workers *w = new Workers();
        return *w;
    }
    // Runs f(k) for every k in [0, n), on the caller and the workers.
    void run(unsigned n, const std::function<void(unsigned)> &f) {
        std::unique_lock<std::mutex> use(use_, std::try_to_lock);
        if (!use.owns_lock() || n < 2) {
            for (unsigned k = 0; k < n; ++k) f(k);
            return;
        }
        start(n - 1);
        {
            std::lock_guard<std::mutex> g(m_);
            job_ = &f;
            n_ = n;
            next_.store(0);
            ++gen_;
        }
        cv_.notify_all();
        for (unsigned k; (k = next_.fetch_add(1)) < n;) f(k);
        // every index is claimed; wait for the workers still inside the
        // section, then close it (a worker that wakes later finds no job)
        std::unique_lock<std::mutex> g(m_);
        done_.wait(g, [&] { return busy_ == 0; });
        job_ = nullptr;
    }

private:
    void start(unsigned want) {
        const unsigned hw = std::thread::hardware_concurrency();
        want = std::min(want, std::min(hw > 1 ? hw - 1 : 0u, 15u));
        while (started_ < want) {
            try {
                std::thread(&Workers::loop, this).detach();
            } catch (...) {
                return;   // no more threads to be had: the sections use fewer
            }
            ++started_;
        }
    }
    void loop() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> g(m_);
        for (;;) {
            cv_.wait(g, [&] { return gen_ != seen; });
            seen = gen_;
            if (!job_) continue;   // that section has closed
            const std::function<void(unsigned)> *job = job_;
            const unsigned n = n_;
            ++busy_;
            g.unlock();
            for (unsigned k; (k = next_.fetch_add(1)) < n;) (*job)(k);
            g.lock();
            if (--busy_ == 0) done_.notify_all();
        }
    }
    std::mutex use_;   // held by the caller of the running section
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(unsigned)> *job_ = nullptr;
    unsigned n_ = 0, busy_ = 0, started_ = 0;
    uint64_t gen_ = 0;
    std::atomic<unsigned> next_{0};
};

// Runs f(k) for k in [0, n) over contiguous slices on up to host_threads(work)
// threads; f returns false at a failure.  Returns the least failing k (n if
// none), the same index a serial scan would stop at.
template <class F>
size_t first_failure(size_t n, size_t work, F f) {
    const unsigned nt = n < 2 ? 1u : std::min<unsigned>(host_threads(work), (unsigned)std::min<size_t>(n, 64));
    std::vector<size_t> first(nt, n);
    Workers::get().run(nt, [&](unsigned k) {
        for (size_t i = n * k / nt, e = n * (k + 1) / nt; i < e; ++i)
            if (!f(i)) { first[k] = i; return; }
    });
    return *std::min_element(first.begin(), first.end());
}

// memcpy of several (dst, src, n) pieces, split over host threads.
struct Piece { void *dst; const void *src; size_t n; };
void copy_pieces(const std::vector<Piece> &pcs) {
    size_t total = 0;
    for (auto &p : pcs) total += p.n;
    const size_t chunk = size_t(1) << 20;
    std::vector<Piece> jobs;
    for (auto &p : pcs)
        for (size_t o = 0; o < p.n; o += chunk)
            jobs.push_back({static_cast<char *>(p.dst) + o, static_cast<const char *>(p.src) + o, std::min(chunk, p.n - o)});
    (void)first_failure(jobs.size(), total, [&](size_t k) {
        std::memcpy(jobs[k].dst, jobs[k].src, jobs[k].n);
        return true;
    });
}

}  // namespace

struct lf_ctx {
    lf_geometry geom{};
    lf_params params{};
    lfk::KParams *d_params = nullptr;  // device copy of geometry + parameters
    size_t budget = 0;
    size_t used = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    void *fixed = nullptr;             // this device's fixed scratch (lf_find_tracks_noalloc)
    lfk::ExecCfg exec{2, 4, 0, 0};
    std::map<uint64_t, Batch> batches;
    uint64_t next_id = 1;
    std::string err;
    // pinned host staging of uploads and downloads (grown on demand, kept)
    char *pin = nullptr;
    size_t pin_cap = 0;
    // the device block of the last batch freed, kept for the next upload
    // that fits it (not counted in `used`)
    void *spare = nullptr;
    size_t spare_bytes = 0;
};

namespace {

int fail(lf_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg; else g_create_error = msg;
    return code;
}

int hip_fail(lf_ctx *c, hipError_t e, const char *what) {
    return fail(c, LF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

hipStream_t pick(lf_ctx *c, void *s) { return s ? reinterpret_cast<hipStream_t>(s) : c->stream; }

// The context's pinned staging buffer, at least `bytes` long; nullptr when
// it cannot be had (callers then copy from pageable memory directly).  Its
// previous contents are not kept.  Only used between synchronisations.
char *staging(lf_ctx *c, size_t bytes) {
    if (bytes <= c->pin_cap) return c->pin;
    if (c->pin) (void)hipHostFree(c->pin);
    c->pin = nullptr;
    c->pin_cap = 0;
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    c->pin = static_cast<char *>(p);
    c->pin_cap = bytes;
    return c->pin;
}

// A batch's device block, at least `need` bytes: the spare block when it fits
// (and is not more than twice the need), else a new allocation, the spare
// being freed first when it does not fit or when holding it would take the
// context past its budget.  *got: the block's size.
hipError_t take_block(lf_ctx *c, size_t need, void **p, size_t *got) {
    if (c->spare && c->spare_bytes >= need && c->spare_bytes / 2 <= need &&
        (!c->budget || c->used + c->spare_bytes <= c->budget)) {
        *p = c->spare;
        *got = c->spare_bytes;
        c->spare = nullptr;
        c->spare_bytes = 0;
        return hipSuccess;
    }
    if (c->spare) {
        (void)hipFree(c->spare);
        c->spare = nullptr;
        c->spare_bytes = 0;
    }
    *got = need;
    return hipMalloc(p, need);
}

// Frees a batch's block: kept as the spare (the previous spare is freed).
// The device is synchronised first, as a free would be, so that no queued
// work on any stream still uses the block when an upload reuses it.
void drop_block(lf_ctx *c, void *p, size_t bytes) {
    (void)hipDeviceSynchronize();
    if (c->spare) (void)hipFree(c->spare);
    c->spare = p;
    c->spare_bytes = bytes;
}

bool finitef(float v) { return std::isfinite(v); }

int check_params(const lf_geometry *g, const lf_params *p, std::string &why) {
    for (int l = 0; l < LF_NLAYERS; ++l)
        if (!finitef(g->z[l]) || !finitef(g->dxdy[l])) { why = "geometry: non-finite layer z or dxdy"; return 0; }
    const float gs[] = {g->z_in, g->z_mag, g->z_ref, g->z_T, g->kick, g->kappa, g->dRatio};
    for (float v : gs) if (!finitef(v)) { why = "geometry: non-finite value"; return 0; }
    if (g->field_form != 0 && g->field_form != 1) { why = "geometry: field_form must be 0 or 1"; return 0; }
    if (g->field_form == 0 && g->kick == 0.0f) { why = "geometry: kick must be non-zero"; return 0; }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 10; ++j)
            if (!finitef(g->F_coef[i][j])) { why = "geometry: non-finite F_coef entry"; return 0; }
    if (g->polarity != 1 && g->polarity != -1) { why = "geometry: polarity must be +1 or -1"; return 0; }
    if (p->n_hits_window < 1 || p->n_hits_window > lfk::MAX_WINDOW) { why = "params: n_hits_window must be 1..64"; return 0; }
    if (p->n_triplets < 1 || p->n_triplets > lfk::MAX_TRIPLETS) { why = "params: n_triplets must be 1..32"; return 0; }
    const float ps[] = {p->T_triplet, p->T_x, p->T_uv_scale, p->T_uv_floor, p->T_ty, p->T_y, p->T_Q,
                        p->xtol_const, p->xtol_pscale, p->xasym, p->uv_halfwidth, p->K_first, p->K_last,
                        p->magtol_const, p->magtol_pscale, p->magtol_txscale, p->magtol_min, p->magtol_max,
                        p->p_charge_cut, p->C_nhits[0], p->C_nhits[1], p->C_nhits[2], p->C_nhits[3]};
    for (float v : ps) if (std::isnan(v)) { why = "params: NaN value"; return 0; }
    if (p->velo_only != 0 && p->velo_only != 1) { why = "params: velo_only must be 0 or 1"; return 0; }
    for (int i = 0; i < 8; ++i)
        if (!finitef(p->noUT_c[i])) { why = "params: non-finite no-UT polynomial coefficient"; return 0; }
    if (!finitef(p->noUT_p_min) || !finitef(p->noUT_pt_min) || !finitef(p->noUT_overlap)) {
        why = "params: non-finite no-UT momentum threshold or overlap";
        return 0;
    }
    if (p->velo_only && !(p->noUT_p_min > 0.0f)) { why = "params: velo_only needs noUT_p_min > 0"; return 0; }
    if (p->seed_fp16 != 0 && p->seed_fp16 != 1) { why = "params: seed_fp16 must be 0 or 1"; return 0; }
    if (p->seed_fp16 && p->velo_only) { why = "params: seed_fp16 needs VELO-UT input (velo_only = 0)"; return 0; }
    return 1;
}

lfk::KParams to_kparams(const lf_geometry &g, const lf_params &p) {
    lfk::KParams k{};
    for (int l = 0; l < LF_NLAYERS; ++l) { k.z[l] = g.z[l]; k.dxdy[l] = g.dxdy[l]; }
    k.z_in = g.z_in; k.z_mag = g.z_mag; k.z_ref = g.z_ref; k.z_T = g.z_T;
    k.kick = g.kick; k.kappa = g.kappa; k.dRatio = g.dRatio; k.polarity = g.polarity;
    k.field_form = g.field_form;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 10; ++j) k.F_coef[i][j] = g.F_coef[i][j];
    k.T_triplet = p.T_triplet; k.T_x = p.T_x; k.T_uv_scale = p.T_uv_scale; k.T_uv_floor = p.T_uv_floor;
    k.T_ty = p.T_ty; k.T_y = p.T_y; k.T_Q = p.T_Q;
    k.xtol_const = p.xtol_const; k.xtol_pscale = p.xtol_pscale; k.xasym = p.xasym;
    k.uv_halfwidth = p.uv_halfwidth; k.K_first = p.K_first; k.K_last = p.K_last;
    k.magtol_const = p.magtol_const; k.magtol_pscale = p.magtol_pscale; k.magtol_txscale = p.magtol_txscale;
    k.magtol_min = p.magtol_min; k.magtol_max = p.magtol_max; k.p_charge_cut = p.p_charge_cut;
    for (int i = 0; i < 4; ++i) k.C_nhits[i] = p.C_nhits[i];
    k.n_hits_window = p.n_hits_window; k.n_triplets = p.n_triplets;
    k.velo_only = p.velo_only;
    k.seed_fp16 = p.seed_fp16;
    for (int i = 0; i < 8; ++i) k.noUT_c[i] = p.noUT_c[i];
    k.noUT_p_min = p.noUT_p_min; k.noUT_pt_min = p.noUT_pt_min; k.noUT_overlap = p.noUT_overlap;
    return k;
}

// Host validation of a batch (see lf_batch in lf.h).
int validate(const lf_batch *b, std::string &why) {
    const uint32_t E = b->n_events;
    if (!b->hit_off || !b->trk_off) { why = "batch: NULL offset array"; return 0; }
    if (b->hit_off[0] != 0 || b->trk_off[0] != 0) { why = "batch: offsets must start at 0"; return 0; }
    const size_t nb = (size_t)E * 24;
    for (size_t i = 0; i < nb; ++i)
        if (b->hit_off[i + 1] < b->hit_off[i]) { why = "batch: hit_off decreases at bucket " + std::to_string(i); return 0; }
    for (size_t e = 0; e < E; ++e)
        if (b->trk_off[e + 1] < b->trk_off[e]) { why = "batch: trk_off decreases at event " + std::to_string(e); return 0; }
    const uint64_t H = b->hit_off[nb], T = b->trk_off[E];
    if (E >= (1u << 26)) { why = "batch: 2^26 or more events"; return 0; }
    if (H >= (1ull << 30) || T >= (1ull << 26)) { why = "batch: 2^30 or more hits, or 2^26 or more tracks"; return 0; }
    if (H && (!b->hit_x || !b->hit_z || !b->hit_dxdy)) { why = "batch: NULL hit array"; return 0; }
    if (T && (!b->trk_x || !b->trk_y || !b->trk_tx || !b->trk_ty || !b->trk_qop)) { why = "batch: NULL track array"; return 0; }
    // the scans below run over slices on several host threads; each reports
    // the first failure a serial scan would.  Hits and buckets in one pass
    // over slices of buckets holding about equal numbers of hits: the first
    // non-finite hit of each slice (where the slice stops: that report wins),
    // and the first bucket before it not sorted by x.
    const unsigned ns = H < 2 ? 1u : std::min<unsigned>(host_threads(12 * H), 64u);
    std::vector<size_t> bad_h(ns, H), bad_b(ns, nb);
    auto bucket_at = [&](unsigned k) -> size_t {
        if (k == 0) return 0;
        if (k == ns) return nb;
        const uint64_t target = H * (uint64_t)k / ns;
        return (size_t)(std::lower_bound(b->hit_off, b->hit_off + nb + 1, (uint32_t)target) - b->hit_off);
    };
    // a bucket is first tested whole, branch-free (the loops vectorise); only
    // a failing bucket is scanned hit by hit for where it fails
    auto bits = [](const float *v, uint32_t i) { uint32_t u; std::memcpy(&u, v + i, 4); return u; };
    auto bucket_ok = [&](uint32_t i0, uint32_t i1) {
        uint32_t bad = 0;
        for (uint32_t i = i0; i < i1; ++i)
            bad |= (uint32_t)((bits(b->hit_x, i) & 0x7f800000u) == 0x7f800000u) |
                   (uint32_t)((bits(b->hit_z, i) & 0x7f800000u) == 0x7f800000u) |
                   (uint32_t)((bits(b->hit_dxdy, i) & 0x7f800000u) == 0x7f800000u);
        for (uint32_t i = i0 + 1; i < i1; ++i) bad |= (uint32_t)(b->hit_x[i] < b->hit_x[i - 1]);
        return bad == 0;
    };
    Workers::get().run(ns, [&](unsigned k) {
        for (size_t q = bucket_at(k), qe = bucket_at(k + 1); q < qe; ++q) {
            const uint32_t i0 = b->hit_off[q], i1 = b->hit_off[q + 1];
            if (bucket_ok(i0, i1)) continue;
            for (uint32_t i = i0; i < i1; ++i) {
                if (!(finitef(b->hit_x[i]) && finitef(b->hit_z[i]) && finitef(b->hit_dxdy[i]))) {
                    bad_h[k] = i;
                    return;
                }
                if (i > i0 && b->hit_x[i] < b->hit_x[i - 1] && bad_b[k] == nb) bad_b[k] = q;
            }
        }
    });
    const size_t bad_hit = *std::min_element(bad_h.begin(), bad_h.end());
    if (bad_hit < H) { why = "batch: non-finite hit " + std::to_string(bad_hit); return 0; }
    const size_t bad_bucket = *std::min_element(bad_b.begin(), bad_b.end());
    if (bad_bucket < nb) { why = "batch: bucket " + std::to_string(bad_bucket) + " not sorted by x"; return 0; }
    const size_t bad_track = first_failure(T, 20 * T, [&](size_t t) {
        return finitef(b->trk_x[t]) && finitef(b->trk_y[t]) && finitef(b->trk_tx[t]) && finitef(b->trk_ty[t]) &&
               finitef(b->trk_qop[t]) && b->trk_qop[t] != 0.0f;
    });
    if (bad_track < T) {
        const size_t t = bad_track;
        if (!finitef(b->trk_x[t]) || !finitef(b->trk_y[t]) || !finitef(b->trk_tx[t]) || !finitef(b->trk_ty[t]) ||
            !finitef(b->trk_qop[t]))
            why = "batch: non-finite track state " + std::to_string(t);
        else
            why = "batch: q/p == 0 for track " + std::to_string(t);
        return 0;
    }
    return 1;
}

// Device layout of a batch: one allocation, every array 256-byte aligned.
struct Layout {
    size_t hit_off, hx, hz, hd, trk_off, trk_ev, tx, ty, ttx, tty, tqop, uni;
    size_t found, nhits, hit_idx, a, b, c, y0, ty_o, qop, Q, counter, stats, total;
};

Layout layout(uint32_t E, uint32_t H, uint32_t T) {
    Layout L{};
    size_t o = 0;
    auto put = [&](size_t bytes) { size_t at = o; o += align256(bytes ? bytes : 1); return at; };
    L.hit_off = put(((size_t)E * 24 + 1) * 4);
    L.hx = put((size_t)H * 4); L.hz = put((size_t)H * 4); L.hd = put((size_t)H * 4);
    L.trk_off = put(((size_t)E + 1) * 4);
    L.trk_ev = put((size_t)T * 4);
    L.tx = put((size_t)T * 4); L.ty = put((size_t)T * 4); L.ttx = put((size_t)T * 4);
    L.tty = put((size_t)T * 4); L.tqop = put((size_t)T * 4);
    L.uni = put(E);
    L.found = put(T); L.nhits = put(T); L.hit_idx = put((size_t)T * 48);
    L.a = put((size_t)T * 4); L.b = put((size_t)T * 4); L.c = put((size_t)T * 4);
    L.y0 = put((size_t)T * 4); L.ty_o = put((size_t)T * 4); L.qop = put((size_t)T * 4); L.Q = put((size_t)T * 4);
    L.counter = put(4 * (size_t)lfk::QUEUE_WORDS);
    L.stats = put(32 * 8);
    L.total = o;
    return L;
}

}  // namespace

namespace lfapi {
int ctx_fail(lf_ctx *c, int code, const std::string &msg) { return fail(c, code, msg); }
const lfk::KParams *ctx_dparams(const lf_ctx *c) { return c->d_params; }
int ctx_nhits_window(const lf_ctx *c) { return c->params.n_hits_window; }
// The kernel build a context launches: 1 VELO-UT, 2 VELO-only (two windows
// per layer), 3 VELO-UT with binary16 seeding.
int ctx_sides(const lf_ctx *c) { return c->params.velo_only ? 2 : (c->params.seed_fp16 ? 3 : 1); }
const lfk::ExecCfg &ctx_exec(const lf_ctx *c) { return c->exec; }
int check_batch(const lf_batch *b, std::string &why) { return validate(b, why); }
}  // namespace lfapi

extern "C" {

void lf_default_params(lf_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    // Table of parameters and tolerances, "Forward" column.
    p->T_triplet = 8.0f;
    p->T_x = 2.0f;
    p->T_uv_scale = 50.0f;
    p->T_uv_floor = 2.0f;
    p->T_ty = 0.02f;
    p->T_y = 800.0f;
    p->T_Q = 0.5f;
    p->n_hits_window = 32;
    p->n_triplets = 12;
    // Search windows: x_tol = 150 mm + 2000 mm GeV / p, 100 mm asymmetry, +-800 mm on u/v.
    p->xtol_const = 150.0f;
    p->xtol_pscale = 2000.0f;
    p->xasym = 100.0f;
    p->uv_halfwidth = 800.0f;
    // Middle-hit corrections of the two seed sets (Triplet Seeding).
    p->K_first = 1.00177513f;
    p->K_last = 1.00142634f;
    // Magnet opening tolerance between 8 and 40 mm, function of p and the doublet slope.
    p->magtol_const = 8.0f;
    p->magtol_pscale = 24.0f;
    p->magtol_txscale = 20.0f;
    p->magtol_min = 8.0f;
    p->magtol_max = 40.0f;
    p->p_charge_cut = 5.0f;
    // C(n_hits) table.
    p->C_nhits[0] = 5.0f;
    p->C_nhits[1] = 1.0f;
    p->C_nhits[2] = 0.8f;
    p->C_nhits[3] = 0.5f;
}

void lf_default_params_no_ut(lf_params *p) {
    if (!p) return;
    lf_default_params(p);
    // Table of parameters and tolerances, "Forward no-UT" column.
    p->T_triplet = 2.0f;
    p->T_x = 0.5f;
    p->T_uv_scale = 15.0f;
    p->T_ty = 0.003f;
    p->T_y = 800.0f;
    p->T_Q = 0.5f;
    p->n_hits_window = 64;
    p->n_triplets = 20;
    // No-UT tuning: u/v tolerance 1200 mm, magnet tolerance fixed at 10 mm,
    // no q/p for the bend-direction filter.
    p->uv_halfwidth = 1200.0f;
    p->magtol_const = 10.0f;
    p->magtol_pscale = 0.0f;
    p->magtol_txscale = 0.0f;
    p->magtol_min = 10.0f;
    p->magtol_max = 10.0f;
    p->p_charge_cut = 0.0f;
    p->velo_only = 1;
    const float c[8] = {4824.3f, 426.3f, 7071.1f, 12080.4f, 14077.8f, 13909.3f, 9315.3f, 3209.5f};
    for (int i = 0; i < 8; ++i) p->noUT_c[i] = c[i];
    p->noUT_p_min = 5.0f;
    p->noUT_pt_min = 1.0f;
    p->noUT_overlap = 5.0f;
}

int lf_check_batch(const lf_batch *b) {
    if (!b) return fail(nullptr, LF_ERR_INVALID, "lf_check_batch: NULL batch");
    std::string why;
    if (!validate(b, why)) return fail(nullptr, LF_ERR_INVALID, "lf_check_batch: " + why);
    g_create_error.clear();
    return LF_OK;
}

int lf_create(const lf_geometry *geom, const lf_params *params, size_t device_budget_bytes, lf_ctx **out) {
    if (!geom || !params || !out) return fail(nullptr, LF_ERR_INVALID, "lf_create: NULL argument");
    *out = nullptr;
    std::string why;
    if (!check_params(geom, params, why)) return fail(nullptr, LF_ERR_INVALID, "lf_create: " + why);
    lf_ctx *c = new (std::nothrow) lf_ctx();
    if (!c) return fail(nullptr, LF_ERR_NOMEM, "lf_create: out of host memory");
    c->geom = *geom;
    c->params = *params;
    c->budget = device_budget_bytes;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    int ncu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess) e = lfk::fixed_scratch(&c->fixed);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&c->d_params), sizeof(lfk::KParams));
    if (e == hipSuccess) {
        const lfk::KParams k = to_kparams(*geom, *params);
        e = hipMemcpy(c->d_params, &k, sizeof(k), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        std::string msg = std::string("lf_create: ") + hipGetErrorString(e);
        lf_destroy(c);
        return fail(nullptr, LF_ERR_DEVICE, msg);
    }
    c->exec.n_cu = ncu;
    c->exec.blocks_per_cu = lfk::persistent_blocks_per_cu(params->n_hits_window, params->velo_only ? 2 : (params->seed_fp16 ? 3 : 1),
                                                          c->exec.waves_per_block);
    if (c->exec.blocks_per_cu < 1) c->exec.blocks_per_cu = 1;
    *out = c;
    return LF_OK;
}

int lf_set_exec(lf_ctx *c, const lf_exec *x) {
    if (!c || !x) return LF_ERR_INVALID;
    lfk::ExecCfg n = c->exec;
    if (x->waves_per_block) {
        if (x->waves_per_block != 1 && x->waves_per_block != 2 && x->waves_per_block != 4)
            return fail(c, LF_ERR_INVALID, "lf_set_exec: waves_per_block must be 1, 2 or 4");
        n.waves_per_block = x->waves_per_block;
        n.blocks_per_cu = lfk::persistent_blocks_per_cu(c->params.n_hits_window, lfapi::ctx_sides(c),
                                                        n.waves_per_block);
        if (n.blocks_per_cu < 1) n.blocks_per_cu = 1;
    }
    if (x->items_per_grab) {
        if (x->items_per_grab < 1 || x->items_per_grab > 16)
            return fail(c, LF_ERR_INVALID, "lf_set_exec: items_per_grab must be 1..16");
        n.items_per_grab = x->items_per_grab;
    }
    if (x->blocks_per_cu) {
        if (x->blocks_per_cu < 1 || x->blocks_per_cu > 64)
            return fail(c, LF_ERR_INVALID, "lf_set_exec: blocks_per_cu must be 1..64");
        n.blocks_per_cu = x->blocks_per_cu;
    }
    c->exec = n;
    return LF_OK;
}

int lf_upload_events(lf_ctx *c, const lf_batch *b, void *hip_stream, uint64_t *batch_id) {
    if (!c) return LF_ERR_INVALID;
    if (!b || !batch_id) return fail(c, LF_ERR_INVALID, "lf_upload_events: NULL argument");
    std::string why;
    if (!validate(b, why)) return fail(c, LF_ERR_INVALID, "lf_upload_events: " + why);
    const uint32_t E = b->n_events, H = b->hit_off[(size_t)E * 24], T = b->trk_off[E];
    const Layout L = layout(E, H, T);
    if (c->budget && c->used + L.total > c->budget)
        return fail(c, LF_ERR_TOO_LARGE, "lf_upload_events: batch needs " + std::to_string(L.total) +
                                             " device bytes, " + std::to_string(c->budget - c->used) + " left");
    Batch bt;
    bt.n_events = E; bt.n_tracks = T; bt.n_hits = H;
    bt.out_off = L.found;
    bt.out_bytes = L.counter - L.found;
    try {
        bt.trk_off.assign(b->trk_off, b->trk_off + E + 1);
    } catch (...) {
        return fail(c, LF_ERR_NOMEM, "lf_upload_events: out of host memory");
    }
    hipError_t e = take_block(c, L.total, &bt.dmem, &bt.bytes);
    if (e != hipSuccess) return fail(c, LF_ERR_NOMEM, std::string("lf_upload_events: hipMalloc: ") + hipGetErrorString(e));
    char *base = static_cast<char *>(bt.dmem);
    lfk::DevBatch &d = bt.dev;
    d.hit_off = reinterpret_cast<const uint32_t *>(base + L.hit_off);
    d.hx = reinterpret_cast<const float *>(base + L.hx);
    d.hz = reinterpret_cast<const float *>(base + L.hz);
    d.hd = reinterpret_cast<const float *>(base + L.hd);
    d.trk_off = reinterpret_cast<const uint32_t *>(base + L.trk_off);
    d.trk_ev = reinterpret_cast<const uint32_t *>(base + L.trk_ev);
    d.tx_ = reinterpret_cast<const float *>(base + L.tx);
    d.ty_ = reinterpret_cast<const float *>(base + L.ty);
    d.ttx = reinterpret_cast<const float *>(base + L.ttx);
    d.tty = reinterpret_cast<const float *>(base + L.tty);
    d.tqop = reinterpret_cast<const float *>(base + L.tqop);
    d.uni = reinterpret_cast<const uint8_t *>(base + L.uni);
    d.found = reinterpret_cast<uint8_t *>(base + L.found);
    d.nhits = reinterpret_cast<uint8_t *>(base + L.nhits);
    d.hit_idx = reinterpret_cast<int32_t *>(base + L.hit_idx);
    d.a = reinterpret_cast<float *>(base + L.a);
    d.b = reinterpret_cast<float *>(base + L.b);
    d.c = reinterpret_cast<float *>(base + L.c);
    d.y0 = reinterpret_cast<float *>(base + L.y0);
    d.ty = reinterpret_cast<float *>(base + L.ty_o);
    d.qop = reinterpret_cast<float *>(base + L.qop);
    d.Q = reinterpret_cast<float *>(base + L.Q);
    d.counter = reinterpret_cast<uint32_t *>(base + L.counter);
    d.stats = reinterpret_cast<unsigned long long *>(base + L.stats);
    d.n_events = E;
    d.n_tracks = T;
    hipStream_t s = pick(c, hip_stream);
    struct { size_t off; const void *src; size_t n; } cp[] = {
        {L.hit_off, b->hit_off, ((size_t)E * 24 + 1) * 4}, {L.hx, b->hit_x, (size_t)H * 4},
        {L.hz, b->hit_z, (size_t)H * 4}, {L.hd, b->hit_dxdy, (size_t)H * 4},
        {L.trk_off, b->trk_off, ((size_t)E + 1) * 4}, {L.tx, b->trk_x, (size_t)T * 4},
        {L.ty, b->trk_y, (size_t)T * 4}, {L.ttx, b->trk_tx, (size_t)T * 4},
        {L.tty, b->trk_ty, (size_t)T * 4}, {L.tqop, b->trk_qop, (size_t)T * 4}};
    // the inputs are one run [0, L.uni) of the allocation, staged in pinned
    // memory by several host threads in four parts (offsets and x, z, dxdy,
    // the tracks), each sent over the host link while the next is staged
    char *pin = staging(c, L.uni);
    if (pin) {
        const size_t part_end[4] = {L.hz, L.hd, L.trk_off, L.uni};
        size_t from = 0;
        for (size_t p = 0; p < 4 && e == hipSuccess; ++p) {
            std::vector<Piece> pcs;
            for (auto &x : cp)
                if (x.n && x.off >= from && x.off < part_end[p]) pcs.push_back({pin + x.off, x.src, x.n});
            copy_pieces(pcs);
            e = hipMemcpyAsync(base + from, pin + from, part_end[p] - from, hipMemcpyHostToDevice, s);
            from = part_end[p];
        }
    } else {
        for (auto &x : cp) {
            if (!x.n) continue;
            e = hipMemcpyAsync(base + x.off, x.src, x.n, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) break;
        }
    }
    if (e == hipSuccess) e = hipMemsetAsync(d.counter, 0, 4 * (size_t)lfk::QUEUE_WORDS, s);
    if (e == hipSuccess) e = lfk::launch_track_event(d, s);
    if (e == hipSuccess) e = lfk::launch_event_uniform(d, reinterpret_cast<uint8_t *>(base + L.uni), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(bt.dmem);
        return hip_fail(c, e, "lf_upload_events");
    }
    const uint64_t id = c->next_id++;
    c->used += bt.bytes;
    c->batches.emplace(id, std::move(bt));
    *batch_id = id;
    return LF_OK;
}

int lf_find_tracks(lf_ctx *c, uint64_t batch_id, int mode, void *hip_stream) {
    if (!c) return LF_ERR_INVALID;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, LF_ERR_STATE, "lf_find_tracks: unknown batch id");
    if (mode != LF_MODE_PLAIN && mode != LF_MODE_BATCHED && mode != LF_MODE_PERSISTENT)
        return fail(c, LF_ERR_INVALID, "lf_find_tracks: unknown mode");
    Batch &bt = it->second;
    const hipError_t e = lfk::launch_find(bt.dev, c->d_params, c->params.n_hits_window, lfapi::ctx_sides(c),
                                          mode, c->exec,
                                          bt.trk_off.data(), pick(c, hip_stream));
    if (e != hipSuccess) return hip_fail(c, e, "lf_find_tracks");
    return LF_OK;
}

int lf_find_tracks_noalloc(lf_ctx *c, const lf_batch *in, uint32_t n_hits, uint32_t n_tracks,
                           const lf_tracks_out *out, int mode, void *hip_stream) {
    if (!c) return LF_ERR_INVALID;
    if (!in || !out) return fail(c, LF_ERR_INVALID, "lf_find_tracks_noalloc: NULL argument");
    if (mode != LF_MODE_BATCHED && mode != LF_MODE_PERSISTENT)
        return fail(c, LF_ERR_INVALID, "lf_find_tracks_noalloc: mode must be LF_MODE_BATCHED or LF_MODE_PERSISTENT");
    const uint32_t E = in->n_events;
    if (E > lfk::FIXED_MAX_EVENTS || n_tracks > lfk::FIXED_MAX_TRACKS)
        return fail(c, LF_ERR_TOO_LARGE, "lf_find_tracks_noalloc: " + std::to_string(E) + " events and " +
                                             std::to_string(n_tracks) + " tracks exceed the fixed scratch (at most " +
                                             std::to_string(lfk::FIXED_MAX_EVENTS) + " events and " +
                                             std::to_string(lfk::FIXED_MAX_TRACKS) + " tracks)");
    if (n_hits >= (1u << 30)) return fail(c, LF_ERR_INVALID, "lf_find_tracks_noalloc: 2^30 or more hits");
    if (!in->hit_off || !in->trk_off) return fail(c, LF_ERR_INVALID, "lf_find_tracks_noalloc: NULL offset array");
    if (n_hits && (!in->hit_x || !in->hit_z || !in->hit_dxdy))
        return fail(c, LF_ERR_INVALID, "lf_find_tracks_noalloc: NULL hit array");
    if (n_tracks && (!in->trk_x || !in->trk_y || !in->trk_tx || !in->trk_ty || !in->trk_qop || !out->found ||
                     !out->n_hits || !out->hit_idx || !out->a || !out->b || !out->c || !out->y0 || !out->ty ||
                     !out->qop || !out->Q))
        return fail(c, LF_ERR_INVALID, "lf_find_tracks_noalloc: NULL track or output array");
    if (!c->fixed) return fail(c, LF_ERR_STATE, "lf_find_tracks_noalloc: no fixed scratch on this context");
    if (n_tracks == 0) return LF_OK;
    char *fx = static_cast<char *>(c->fixed);
    lfk::DevBatch d{};
    d.hit_off = in->hit_off;
    d.hx = in->hit_x; d.hz = in->hit_z; d.hd = in->hit_dxdy;
    d.trk_off = in->trk_off;
    d.trk_ev = reinterpret_cast<const uint32_t *>(fx + lfk::FIXED_TRK_EV_OFF);
    d.tx_ = in->trk_x; d.ty_ = in->trk_y; d.ttx = in->trk_tx; d.tty = in->trk_ty; d.tqop = in->trk_qop;
    d.uni = reinterpret_cast<const uint8_t *>(fx + lfk::FIXED_UNI_OFF);
    d.found = out->found; d.nhits = out->n_hits; d.hit_idx = out->hit_idx;
    d.a = out->a; d.b = out->b; d.c = out->c; d.y0 = out->y0; d.ty = out->ty; d.qop = out->qop; d.Q = out->Q;
    d.counter = reinterpret_cast<uint32_t *>(fx + lfk::FIXED_QUEUE_OFF);
    d.stats = nullptr;
    d.n_events = E;
    d.n_tracks = n_tracks;
    hipStream_t s = pick(c, hip_stream);
    hipError_t e = lfk::launch_zero_words(d.counter, lfk::QUEUE_WORDS, s);
    if (e == hipSuccess) e = lfk::launch_track_event(d, s);
    if (e == hipSuccess) e = lfk::launch_event_uniform(d, reinterpret_cast<uint8_t *>(fx + lfk::FIXED_UNI_OFF), s);
    if (e == hipSuccess)
        e = lfk::launch_find(d, c->d_params, c->params.n_hits_window, lfapi::ctx_sides(c), mode, c->exec, nullptr, s);
    if (e != hipSuccess) return hip_fail(c, e, "lf_find_tracks_noalloc");
    return LF_OK;
}

struct lf_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int lf_graph_create(lf_ctx *c, const uint64_t *ids, uint32_t n, int mode, lf_graph **out) {
    if (!c) return LF_ERR_INVALID;
    if (!ids || !out || n == 0) return fail(c, LF_ERR_INVALID, "lf_graph_create: no batches");
    if (mode != LF_MODE_PLAIN && mode != LF_MODE_BATCHED && mode != LF_MODE_PERSISTENT)
        return fail(c, LF_ERR_INVALID, "lf_graph_create: unknown mode");
    *out = nullptr;
    std::vector<Batch *> bs;
    for (uint32_t i = 0; i < n; ++i) {
        auto it = c->batches.find(ids[i]);
        if (it == c->batches.end()) return fail(c, LF_ERR_STATE, "lf_graph_create: unknown batch id");
        bs.push_back(&it->second);
    }
    // Distinct batches are independent (each writes only its own results
    // and, in persistent mode, its own queue words): captured as parallel
    // branches (a fork from the capture stream and a join back), so the
    // graph's launches may overlap and fill each other's ragged ends.  A
    // batch listed twice keeps the whole sequence in order on one stream.
    bool distinct = true;
    {
        std::vector<uint64_t> sorted(ids, ids + n);
        std::sort(sorted.begin(), sorted.end());
        distinct = std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end();
    }
    const uint32_t n_side = distinct ? n - 1 : 0;
    hipStream_t cs = nullptr;
    std::vector<hipStream_t> side(n_side, nullptr);
    std::vector<hipEvent_t> evs(n, nullptr);   // evs[0]: the fork; evs[i]: branch i's join
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (uint32_t i = 0; i < n && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&evs[i], hipEventDisableTiming);
    for (uint32_t i = 0; i < n_side && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
    auto release = [&]() {
        for (auto &x : side) if (x) (void)hipStreamDestroy(x);
        for (auto &x : evs) if (x) (void)hipEventDestroy(x);
        if (cs) (void)hipStreamDestroy(cs);
    };
    lf_graph *g = new (std::nothrow) lf_graph();
    if (!g) { release(); return fail(c, LF_ERR_NOMEM, "lf_graph_create: out of memory"); }
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = n_side ? hipEventRecord(evs[0], cs) : hipSuccess;
        for (uint32_t i = 0; i < n_side && le == hipSuccess; ++i) le = hipStreamWaitEvent(side[i], evs[0], 0);
        for (uint32_t i = 0; i < n && le == hipSuccess; ++i) {
            const bool branch = n_side && i > 0;
            hipStream_t st = branch ? side[i - 1] : cs;
            le = lfk::launch_find(bs[i]->dev, c->d_params, c->params.n_hits_window, lfapi::ctx_sides(c), mode,
                                  c->exec, bs[i]->trk_off.data(), st);
            if (le == hipSuccess && branch) le = hipEventRecord(evs[i], st);
            if (le == hipSuccess && branch) le = hipStreamWaitEvent(cs, evs[i], 0);
        }
        e = hipStreamEndCapture(cs, &g->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    release();
    if (e != hipSuccess) {
        lf_graph_destroy(g);
        return hip_fail(c, e, "lf_graph_create");
    }
    *out = g;
    return LF_OK;
}

int lf_graph_launch(lf_ctx *c, lf_graph *g, void *hip_stream) {
    if (!c) return LF_ERR_INVALID;
    if (!g || !g->exec) return fail(c, LF_ERR_INVALID, "lf_graph_launch: NULL graph");
    const hipError_t e = hipGraphLaunch(g->exec, pick(c, hip_stream));
    if (e != hipSuccess) return hip_fail(c, e, "lf_graph_launch");
    return LF_OK;
}

void lf_graph_destroy(lf_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

int lf_work_counts(lf_ctx *c, uint64_t batch_id, void *hip_stream, int64_t *counts, size_t n_counts) {
    if (!c) return LF_ERR_INVALID;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, LF_ERR_STATE, "lf_work_counts: unknown batch id");
    if (!counts) return fail(c, LF_ERR_INVALID, "lf_work_counts: NULL counts");
    Batch &bt = it->second;
    hipStream_t s = pick(c, hip_stream);
    unsigned long long host[32] = {0};
    hipError_t e = hipMemsetAsync(bt.dev.stats, 0, sizeof(host), s);
    if (e == hipSuccess)
        e = lfk::launch_count(bt.dev, c->d_params, c->params.n_hits_window, lfapi::ctx_sides(c), s);
    if (e == hipSuccess) e = hipMemcpyAsync(host, bt.dev.stats, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "lf_work_counts");
    for (size_t k = 0; k < n_counts; ++k) counts[k] = k < 32 ? (int64_t)host[k] : 0;
    return LF_OK;
}

namespace {
int copy_tracks(lf_ctx *c, uint64_t batch_id, lf_tracks_out *out, size_t cap_tracks, void *hip_stream, bool release) {
    if (!c) return LF_ERR_INVALID;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, LF_ERR_STATE, "lf_fetch_tracks: unknown batch id");
    Batch &bt = it->second;
    const size_t T = bt.n_tracks;
    if (!out || cap_tracks < T) return fail(c, LF_ERR_INVALID, "lf_fetch_tracks: output capacity below track count");
    if (T && (!out->found || !out->n_hits || !out->hit_idx || !out->a || !out->b || !out->c || !out->y0 ||
              !out->ty || !out->qop || !out->Q))
        return fail(c, LF_ERR_INVALID, "lf_fetch_tracks: NULL output array");
    hipStream_t s = pick(c, hip_stream);
    hipError_t e = hipSuccess;
    if (T) {
        const lfk::DevBatch &d = bt.dev;
        struct { void *dst; const void *src; size_t n; } cp[] = {
            {out->found, d.found, T}, {out->n_hits, d.nhits, T}, {out->hit_idx, d.hit_idx, T * 48},
            {out->a, d.a, T * 4}, {out->b, d.b, T * 4}, {out->c, d.c, T * 4}, {out->y0, d.y0, T * 4},
            {out->ty, d.ty, T * 4}, {out->qop, d.qop, T * 4}, {out->Q, d.Q, T * 4}};
        // the results are one run of the allocation: one copy over the host
        // link into pinned memory, then spread by several host threads
        const char *run = static_cast<const char *>(bt.dmem) + bt.out_off;
        char *pin = staging(c, bt.out_bytes);
        if (pin) {
            e = hipMemcpyAsync(pin, run, bt.out_bytes, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) {
                std::vector<Piece> pcs;
                for (auto &x : cp) pcs.push_back({x.dst, pin + (static_cast<const char *>(x.src) - run), x.n});
                copy_pieces(pcs);
            }
        } else {
            for (auto &x : cp) {
                e = hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyDeviceToHost, s);
                if (e != hipSuccess) break;
            }
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "lf_fetch_tracks");
    if (release) {
        drop_block(c, bt.dmem, bt.bytes);
        c->used -= bt.bytes;
        c->batches.erase(it);
    }
    return LF_OK;
}
}  // namespace

int lf_fetch_tracks(lf_ctx *c, uint64_t batch_id, lf_tracks_out *out, size_t cap_tracks, void *hip_stream) {
    return copy_tracks(c, batch_id, out, cap_tracks, hip_stream, true);
}

int lf_copy_tracks(lf_ctx *c, uint64_t batch_id, lf_tracks_out *out, size_t cap_tracks, void *hip_stream) {
    return copy_tracks(c, batch_id, out, cap_tracks, hip_stream, false);
}

int lf_poison_tracks(lf_ctx *c, uint64_t batch_id, void *hip_stream) {
    if (!c) return LF_ERR_INVALID;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, LF_ERR_STATE, "lf_poison_tracks: unknown batch id");
    const hipError_t e = lfk::launch_poison(it->second.dev, pick(c, hip_stream));
    if (e != hipSuccess) return hip_fail(c, e, "lf_poison_tracks");
    return LF_OK;
}

int lf_release_batch(lf_ctx *c, uint64_t batch_id) {
    if (!c) return LF_ERR_INVALID;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, LF_ERR_STATE, "lf_release_batch: unknown batch id");
    // work on the batch may still be queued on any stream: wait for the device
    const hipError_t e = hipDeviceSynchronize();
    drop_block(c, it->second.dmem, it->second.bytes);
    c->used -= it->second.bytes;
    c->batches.erase(it);
    if (e != hipSuccess) return hip_fail(c, e, "lf_release_batch");
    return LF_OK;
}

int lf_batch_info(lf_ctx *c, uint64_t batch_id, uint32_t *n_events, uint32_t *n_tracks, uint32_t *n_hits,
                  size_t *device_bytes) {
    if (!c) return LF_ERR_INVALID;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, LF_ERR_STATE, "lf_batch_info: unknown batch id");
    if (n_events) *n_events = it->second.n_events;
    if (n_tracks) *n_tracks = it->second.n_tracks;
    if (n_hits) *n_hits = it->second.n_hits;
    if (device_bytes) *device_bytes = it->second.bytes;
    return LF_OK;
}

size_t lf_device_bytes_in_use(const lf_ctx *c) { return c ? c->used : 0; }

void lf_destroy(lf_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->batches) (void)hipFree(kv.second.dmem);
    if (c->spare) (void)hipFree(c->spare);
    if (c->d_params) (void)hipFree(c->d_params);
    if (c->pin) (void)hipHostFree(c->pin);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *lf_last_error(const lf_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

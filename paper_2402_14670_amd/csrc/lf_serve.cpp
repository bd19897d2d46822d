// lf_serve.cpp -- trigger-style serving loop of the Looking Forward library.
//
// Requests are events that arrive over time (open loop: arrival times are
// given, independent of service).  The loop keeps a FIFO of arrived
// requests, admits them into a device-memory ring of a fixed budget, packs
// whatever has been admitted into one batch as soon as an in-flight slot is
// free (continuous batching: requests arriving while others run on the GPU
// join the next batch), and runs upload -> hot path -> digest -> download on
// that slot's stream, so copies and kernels of consecutive batches overlap.
// A request completes when its results (or, with results_on_device, their
// digests) are in host memory.  Two kinds of pool:
//  - in pinned host memory: batches are assembled on the device, the host
//    writing one 24-byte descriptor per event and a gather kernel reading the
//    events' blobs over the host link straight into the batch's arrays, so
//    no host thread copies event data on the request path;
//  - in device memory (pool_on_device, as earlier GPU stages leave events):
//    the pool stays resident as one batch, and a batch is a list of pool
//    events whose result slots a small kernel maps to pool tracks; the hot
//    path reads the pool in place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lf.h"
#include "lf_internal.h"

namespace lfk {
hipError_t launch_digest(const DevBatch &b, const uint32_t *trk_off, uint32_t n_events, unsigned long long *out,
                         hipStream_t s);
}

// Context accessors shared with lf_api.cpp.
namespace lfapi {
int ctx_fail(lf_ctx *c, int code, const std::string &msg);
const lfk::KParams *ctx_dparams(const lf_ctx *c);
int ctx_nhits_window(const lf_ctx *c);
int ctx_sides(const lf_ctx *c);
const lfk::ExecCfg &ctx_exec(const lf_ctx *c);
int check_batch(const lf_batch *b, std::string &why);
}  // namespace lfapi

namespace {

using Clock = std::chrono::steady_clock;

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Pool events as contiguous blobs in pinned host memory:
// [hit_off local u32 x 25][x H][z H][dxdy H][trk x,y,tx,ty,qop: 5 x T].
struct Pool {
    char *blob = nullptr;
    size_t bytes = 0;
    std::vector<size_t> off;       // blob offset of each event
    std::vector<uint32_t> nh, nt;  // hits, tracks per event
};

// Byte layout of one batch region in the device ring.  Host pool: the
// gathered events and the outputs.  Device pool (ref): the event list and
// slot offsets, the slot map, and the outputs.
struct BatchLayout {
    size_t desc, hit_off, hx, hz, hd, trk_off, trk_ev, tx, ty, ttx, tty, tqop, uni, in_bytes;
    size_t dig, found, nhits, hit_idx, fl, out_bytes, total;
    size_t evs, toff, map;   // device pool only
    uint32_t E, H, T;
};

BatchLayout batch_layout(uint32_t E, uint32_t H, uint32_t T) {
    BatchLayout L{};
    L.E = E; L.H = H; L.T = T;
    size_t o = 0;
    auto put = [&](size_t n) { size_t at = o; o += a256(n ? n : 1); return at; };
    L.desc = put((size_t)E * sizeof(lfk::GatherDesc));
    L.hit_off = put(((size_t)E * 24 + 1) * 4);
    L.hx = put((size_t)H * 4); L.hz = put((size_t)H * 4); L.hd = put((size_t)H * 4);
    L.trk_off = put(((size_t)E + 1) * 4); L.trk_ev = put((size_t)T * 4);
    L.tx = put((size_t)T * 4); L.ty = put((size_t)T * 4); L.ttx = put((size_t)T * 4);
    L.tty = put((size_t)T * 4); L.tqop = put((size_t)T * 4);
    L.uni = put(E);
    L.in_bytes = o;
    // outputs: one contiguous block so a single copy brings them back
    const size_t ob = o;
    L.dig = put((size_t)E * 8);
    L.found = put(T); L.nhits = put(T); L.hit_idx = put((size_t)T * 48);
    L.fl = put((size_t)T * 28);
    L.out_bytes = o - ob;
    L.total = o;
    return L;
}

BatchLayout ref_layout(uint32_t E, uint32_t T) {
    BatchLayout L{};
    L.E = E; L.T = T;
    size_t o = 0;
    auto put = [&](size_t n) { size_t at = o; o += a256(n ? n : 1); return at; };
    L.evs = put((size_t)(2 * E + 1) * 4);   // event list, then the E + 1 slot offsets
    L.toff = L.evs + (size_t)E * 4;
    L.map = put((size_t)T * 4);
    L.in_bytes = o;
    const size_t ob = o;
    L.dig = put((size_t)E * 8);
    L.found = put(T); L.nhits = put(T); L.hit_idx = put((size_t)T * 48);
    L.fl = put((size_t)T * 28);
    L.out_bytes = o - ob;
    L.total = o;
    return L;
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    lfk::GatherDesc *stage = nullptr;   // pinned, event descriptors of one batch
    char *out = nullptr;     // pinned, outputs of one batch
    size_t stage_cap = 0, out_cap = 0;
    bool busy = false;
    size_t ring_at = 0, ring_bytes = 0;
    BatchLayout lay{};
    std::vector<uint32_t> reqs;  // requests in this batch
};

// FIFO allocator over the device budget.  Batches free in submission order
// (the oldest in-flight region is released first).
struct Ring {
    size_t cap = 0, head = 0, used = 0;
    std::deque<std::pair<size_t, size_t>> live;  // (start, bytes incl. wrap waste)
    bool alloc(size_t n, size_t &at, size_t &charged) {
        if (n > cap) return false;
        size_t start = head, waste = 0;
        if (start + n > cap) { waste = cap - start; start = 0; }
        if (used + waste + n > cap) return false;
        at = start;
        charged = waste + n;
        head = start + n;
        used += charged;
        live.emplace_back(at, charged);
        return true;
    }
    void free_front() {
        used -= live.front().second;
        live.pop_front();
        if (live.empty()) { head = 0; used = 0; }
    }
};

}  // namespace

extern "C" int lf_serve_run(lf_ctx *ctx, const lf_batch *pool_b, uint32_t n_requests, const uint32_t *req_event,
                            const double *arrival_s, const lf_serve_config *cfg_in, uint64_t *req_digest,
                            double *req_latency_s, lf_serve_stats *stats) {
    if (!ctx) return LF_ERR_INVALID;
    if (!pool_b || !req_event || !arrival_s || !cfg_in)
        return lfapi::ctx_fail(ctx, LF_ERR_INVALID, "lf_serve_run: NULL argument");
    std::string why;
    if (!lfapi::check_batch(pool_b, why)) return lfapi::ctx_fail(ctx, LF_ERR_INVALID, "lf_serve_run: pool " + why);
    lf_serve_config cfg = *cfg_in;
    if (cfg.max_batch_events == 0) cfg.max_batch_events = 1024;
    if (cfg.n_slots == 0) cfg.n_slots = 4;
    if (cfg.device_budget_bytes == 0) cfg.device_budget_bytes = size_t(8) << 30;
    if (cfg.n_slots > 16 || cfg.n_pack_threads > 64 || cfg.max_batch_events > (1u << 20) || cfg.pool_on_device > 1 ||
        cfg.results_on_device > 1 || cfg.verify_results > 1)
        return lfapi::ctx_fail(ctx, LF_ERR_INVALID, "lf_serve_run: configuration out of range");
    const uint32_t PE = pool_b->n_events;
    for (uint32_t i = 0; i < n_requests; ++i) {
        if (req_event[i] >= PE) return lfapi::ctx_fail(ctx, LF_ERR_INVALID, "lf_serve_run: request event out of range");
        if (!(arrival_s[i] >= 0.0) || (i && arrival_s[i] < arrival_s[i - 1]))
            return lfapi::ctx_fail(ctx, LF_ERR_INVALID, "lf_serve_run: arrival times must be >= 0 and non-decreasing");
    }

    const bool dev_pool = cfg.pool_on_device != 0;
    // the layout of a batch region in the ring
    auto layout_of = [&](uint32_t E, uint32_t H, uint32_t T) {
        return dev_pool ? ref_layout(E, T) : batch_layout(E, H, T);
    };
    // ---- pool sizes; pinned blobs for a host pool (the events as delivered to the host) ----
    Pool pool;
    pool.off.resize(PE);
    pool.nh.resize(PE);
    pool.nt.resize(PE);
    size_t pbytes = 0;
    for (uint32_t e = 0; e < PE; ++e) {
        pool.nh[e] = pool_b->hit_off[24 * (size_t)e + 24] - pool_b->hit_off[24 * (size_t)e];
        pool.nt[e] = pool_b->trk_off[e + 1] - pool_b->trk_off[e];
        pool.off[e] = pbytes;
        if (!dev_pool) pbytes += a256(25 * 4 + (size_t)pool.nh[e] * 12 + (size_t)pool.nt[e] * 20);
    }
    size_t max_event_bytes = 0;
    for (uint32_t e = 0; e < PE; ++e) {
        const BatchLayout one = layout_of(1, pool.nh[e], pool.nt[e]);
        max_event_bytes = std::max(max_event_bytes, one.total);
    }
    if (max_event_bytes > cfg.device_budget_bytes)
        return lfapi::ctx_fail(ctx, LF_ERR_TOO_LARGE, "lf_serve_run: an event is larger than the device budget");

    std::vector<Slot> slots(cfg.n_slots);
    void *ring_mem = nullptr;
    char *pool_hbm = nullptr;   // pool_on_device: the pool, resident as one batch in device memory
    hipError_t err = hipHostMalloc(reinterpret_cast<void **>(&pool.blob), pbytes ? pbytes : 1, hipHostMallocDefault);
    if (err != hipSuccess) return lfapi::ctx_fail(ctx, LF_ERR_NOMEM, "lf_serve_run: pinned pool allocation failed");
    pool.bytes = pbytes;
    auto cleanup = [&]() {
        for (auto &s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.stage) (void)hipHostFree(s.stage);
            if (s.out) (void)hipHostFree(s.out);
        }
        if (ring_mem) (void)hipFree(ring_mem);
        if (pool_hbm) (void)hipFree(pool_hbm);
        if (pool.blob) (void)hipHostFree(pool.blob);
    };
    for (uint32_t e = 0; e < (dev_pool ? 0u : PE); ++e) {
        char *p = pool.blob + pool.off[e];
        const uint32_t h0 = pool_b->hit_off[24 * (size_t)e], t0 = pool_b->trk_off[e];
        uint32_t *ho = reinterpret_cast<uint32_t *>(p);
        for (int b = 0; b < 25; ++b) ho[b] = pool_b->hit_off[24 * (size_t)e + b] - h0;
        char *q = p + 100;
        const size_t H = pool.nh[e], T = pool.nt[e];
        std::memcpy(q, pool_b->hit_x + h0, H * 4); q += H * 4;
        std::memcpy(q, pool_b->hit_z + h0, H * 4); q += H * 4;
        std::memcpy(q, pool_b->hit_dxdy + h0, H * 4); q += H * 4;
        const float *src[5] = {pool_b->trk_x, pool_b->trk_y, pool_b->trk_tx, pool_b->trk_ty, pool_b->trk_qop};
        for (int k = 0; k < 5; ++k) { std::memcpy(q, src[k] + t0, T * 4); q += T * 4; }
    }

    // ---- device ring, slots ----
    Ring ring;
    ring.cap = cfg.device_budget_bytes;
    err = hipMalloc(&ring_mem, ring.cap);
    if (err != hipSuccess) {
        cleanup();
        return lfapi::ctx_fail(ctx, LF_ERR_NOMEM, "lf_serve_run: device budget allocation failed");
    }
    // staging sized for the largest batch the budget and the event cap allow
    uint64_t big_h = 0, big_t = 0;
    {
        std::vector<uint32_t> hs(pool.nh), ts(pool.nt);
        std::sort(hs.rbegin(), hs.rend());
        std::sort(ts.rbegin(), ts.rend());
        for (uint32_t i = 0; i < std::min<uint32_t>(cfg.max_batch_events, PE); ++i) { big_h += hs[i]; big_t += ts[i]; }
        // a batch may repeat the largest event
        if (cfg.max_batch_events > PE) {
            big_h += (uint64_t)hs[0] * (cfg.max_batch_events - PE);
            big_t += (uint64_t)ts[0] * (cfg.max_batch_events - PE);
        }
    }
    if (big_h >= (1ull << 30) || big_t >= (1ull << 26)) {
        cleanup();
        return lfapi::ctx_fail(ctx, LF_ERR_INVALID, "lf_serve_run: max_batch_events allows batches over 2^30 hits or 2^26 tracks");
    }
    const BatchLayout biggest = layout_of(cfg.max_batch_events, (uint32_t)big_h, (uint32_t)big_t);
    for (auto &s : slots) {
        err = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (err == hipSuccess)
            err = hipHostMalloc(reinterpret_cast<void **>(&s.stage), (size_t)cfg.max_batch_events * sizeof(lfk::GatherDesc),
                                hipHostMallocDefault);
        if (err == hipSuccess) err = hipHostMalloc(reinterpret_cast<void **>(&s.out), biggest.out_bytes, hipHostMallocDefault);
        if (err != hipSuccess) {
            cleanup();
            return lfapi::ctx_fail(ctx, LF_ERR_NOMEM, "lf_serve_run: slot allocation failed");
        }
        s.stage_cap = cfg.max_batch_events;
        s.out_cap = biggest.out_bytes;

    }
    // A host pool: the gather kernel reads the pinned blobs over the host
    // link.  A device pool: copied once (before the clock) as one resident
    // batch, with each track's event and each event's uniform flag.
    char *pool_dev = nullptr;
    lfk::DevBatch pool_d{};
    const uint32_t PH = pool_b->hit_off[24 * (size_t)PE], PT = pool_b->trk_off[PE];
    if (dev_pool) {
        size_t o = 0;
        auto put = [&](size_t n) { size_t at = o; o += a256(n ? n : 1); return at; };
        const size_t o_ho = put(((size_t)PE * 24 + 1) * 4), o_hx = put((size_t)PH * 4), o_hz = put((size_t)PH * 4),
                     o_hd = put((size_t)PH * 4), o_to = put(((size_t)PE + 1) * 4), o_te = put((size_t)PT * 4),
                     o_tr = put((size_t)PT * 20), o_uni = put(PE);
        err = hipMalloc(reinterpret_cast<void **>(&pool_hbm), o);
        if (err != hipSuccess) {
            cleanup();
            return lfapi::ctx_fail(ctx, LF_ERR_NOMEM, "lf_serve_run: device pool allocation failed");
        }
        char *b = pool_hbm;
        struct { size_t off; const void *src; size_t n; } cp[] = {
            {o_ho, pool_b->hit_off, ((size_t)PE * 24 + 1) * 4}, {o_hx, pool_b->hit_x, (size_t)PH * 4},
            {o_hz, pool_b->hit_z, (size_t)PH * 4}, {o_hd, pool_b->hit_dxdy, (size_t)PH * 4},
            {o_to, pool_b->trk_off, ((size_t)PE + 1) * 4}, {o_tr, pool_b->trk_x, (size_t)PT * 4},
            {o_tr + (size_t)PT * 4, pool_b->trk_y, (size_t)PT * 4}, {o_tr + (size_t)PT * 8, pool_b->trk_tx, (size_t)PT * 4},
            {o_tr + (size_t)PT * 12, pool_b->trk_ty, (size_t)PT * 4},
            {o_tr + (size_t)PT * 16, pool_b->trk_qop, (size_t)PT * 4}};
        for (auto &x : cp) {
            if (err == hipSuccess && x.n) err = hipMemcpy(b + x.off, x.src, x.n, hipMemcpyHostToDevice);
        }
        pool_d.hit_off = reinterpret_cast<const uint32_t *>(b + o_ho);
        pool_d.hx = reinterpret_cast<const float *>(b + o_hx);
        pool_d.hz = reinterpret_cast<const float *>(b + o_hz);
        pool_d.hd = reinterpret_cast<const float *>(b + o_hd);
        pool_d.trk_off = reinterpret_cast<const uint32_t *>(b + o_to);
        pool_d.trk_ev = reinterpret_cast<const uint32_t *>(b + o_te);
        pool_d.tx_ = reinterpret_cast<const float *>(b + o_tr);
        pool_d.ty_ = pool_d.tx_ + PT;
        pool_d.ttx = pool_d.tx_ + 2 * (size_t)PT;
        pool_d.tty = pool_d.tx_ + 3 * (size_t)PT;
        pool_d.tqop = pool_d.tx_ + 4 * (size_t)PT;
        pool_d.uni = reinterpret_cast<const uint8_t *>(b + o_uni);
        pool_d.n_events = PE;
        pool_d.n_tracks = PT;
        if (err == hipSuccess) err = lfk::launch_track_event(pool_d, slots[0].stream);
        if (err == hipSuccess) err = lfk::launch_event_uniform(pool_d, reinterpret_cast<uint8_t *>(b + o_uni), slots[0].stream);
        if (err == hipSuccess) err = hipStreamSynchronize(slots[0].stream);
    } else {
        err = hipHostGetDevicePointer(reinterpret_cast<void **>(&pool_dev), pool.blob, 0);
    }
    if (err != hipSuccess) {
        cleanup();
        return lfapi::ctx_fail(ctx, LF_ERR_DEVICE, std::string("lf_serve_run: ") + hipGetErrorString(err));
    }
    const lfk::KParams *P = lfapi::ctx_dparams(ctx);
    const int nhw = lfapi::ctx_nhits_window(ctx);
    const int n_sides = lfapi::ctx_sides(ctx);
    const lfk::ExecCfg exec = lfapi::ctx_exec(ctx);

    // Writes the descriptors of pool events evs[0..E) and enqueues
    // descriptors up -> gather -> hot path -> digest -> download on the
    // slot's stream into device region `at` of the ring.
    auto launch_batch = [&](Slot &s, const std::vector<uint32_t> &evs, const BatchLayout &lay,
                            size_t at) -> hipError_t {
        const uint32_t E = (uint32_t)evs.size();
        if (E > s.stage_cap) return hipErrorInvalidValue;   // descriptors must fit the slot
        const size_t down = cfg.results_on_device ? (size_t)E * 8 : lay.out_bytes;   // the digests lead the outputs
        char *dr = static_cast<char *>(ring_mem) + at;
        if (dev_pool) {
            // the event list and the slot offsets, the slot map, then the hot
            // path reading the resident pool
            uint32_t *ev_h = reinterpret_cast<uint32_t *>(s.stage), *to_h = ev_h + E;
            uint32_t T = 0;
            for (uint32_t k = 0; k < E; ++k) {
                ev_h[k] = evs[k];
                to_h[k] = T;
                T += pool.nt[evs[k]];
            }
            to_h[E] = T;
            const uint32_t *ev_d = reinterpret_cast<const uint32_t *>(dr + lay.evs);
            const uint32_t *to_d = reinterpret_cast<const uint32_t *>(dr + lay.toff);
            uint32_t *map_d = reinterpret_cast<uint32_t *>(dr + lay.map);
            lfk::DevBatch d = pool_d;
            d.trk_map = map_d;
            d.n_map = T;
            d.found = reinterpret_cast<uint8_t *>(dr + lay.found);
            d.nhits = reinterpret_cast<uint8_t *>(dr + lay.nhits);
            d.hit_idx = reinterpret_cast<int32_t *>(dr + lay.hit_idx);
            float *fl = reinterpret_cast<float *>(dr + lay.fl);
            d.a = fl; d.b = fl + T; d.c = fl + 2 * (size_t)T; d.y0 = fl + 3 * (size_t)T;
            d.ty = fl + 4 * (size_t)T; d.qop = fl + 5 * (size_t)T; d.Q = fl + 6 * (size_t)T;
            hipError_t e = hipMemcpyAsync(dr + lay.evs, s.stage, (size_t)(2 * E + 1) * 4, hipMemcpyHostToDevice,
                                          s.stream);
            if (e == hipSuccess) e = lfk::launch_track_map(ev_d, to_d, E, T, pool_d.trk_off, map_d, s.stream);
            if (e == hipSuccess && T) e = lfk::launch_find(d, P, nhw, n_sides, 1, exec, nullptr, s.stream);
            if (e == hipSuccess)
                e = lfk::launch_digest(d, to_d, E, reinterpret_cast<unsigned long long *>(dr + lay.dig), s.stream);
            if (e == hipSuccess) e = hipMemcpyAsync(s.out, dr + lay.dig, down, hipMemcpyDeviceToHost, s.stream);
            if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
            return e;
        }
        uint32_t H = 0, T = 0;
        for (uint32_t k = 0; k < E; ++k) {
            const uint32_t ev = evs[k];
            s.stage[k] = lfk::GatherDesc{reinterpret_cast<uint64_t>(pool_dev + pool.off[ev]), H, T, pool.nh[ev],
                                         pool.nt[ev]};
            H += pool.nh[ev];
            T += pool.nt[ev];
        }
        lfk::BatchIn in{};
        in.hit_off = reinterpret_cast<uint32_t *>(dr + lay.hit_off);
        in.hx = reinterpret_cast<float *>(dr + lay.hx);
        in.hz = reinterpret_cast<float *>(dr + lay.hz);
        in.hd = reinterpret_cast<float *>(dr + lay.hd);
        in.trk_off = reinterpret_cast<uint32_t *>(dr + lay.trk_off);
        in.trk_ev = reinterpret_cast<uint32_t *>(dr + lay.trk_ev);
        in.tx = reinterpret_cast<float *>(dr + lay.tx);
        in.ty = reinterpret_cast<float *>(dr + lay.ty);
        in.ttx = reinterpret_cast<float *>(dr + lay.ttx);
        in.tty = reinterpret_cast<float *>(dr + lay.tty);
        in.tqop = reinterpret_cast<float *>(dr + lay.tqop);
        lfk::DevBatch d{};
        d.hit_off = in.hit_off;
        d.hx = in.hx;
        d.hz = in.hz;
        d.hd = in.hd;
        d.trk_off = in.trk_off;
        d.trk_ev = in.trk_ev;
        d.tx_ = in.tx;
        d.ty_ = in.ty;
        d.ttx = in.ttx;
        d.tty = in.tty;
        d.tqop = in.tqop;
        d.uni = reinterpret_cast<const uint8_t *>(dr + lay.uni);
        d.found = reinterpret_cast<uint8_t *>(dr + lay.found);
        d.nhits = reinterpret_cast<uint8_t *>(dr + lay.nhits);
        d.hit_idx = reinterpret_cast<int32_t *>(dr + lay.hit_idx);
        float *fl = reinterpret_cast<float *>(dr + lay.fl);
        d.a = fl; d.b = fl + T; d.c = fl + 2 * (size_t)T; d.y0 = fl + 3 * (size_t)T;
        d.ty = fl + 4 * (size_t)T; d.qop = fl + 5 * (size_t)T; d.Q = fl + 6 * (size_t)T;
        d.counter = nullptr;
        d.stats = nullptr;
        d.n_events = E;
        d.n_tracks = T;
        const lfk::GatherDesc *ddesc = reinterpret_cast<const lfk::GatherDesc *>(dr + lay.desc);
        hipError_t e = hipMemcpyAsync(dr + lay.desc, s.stage, (size_t)E * sizeof(lfk::GatherDesc),
                                      hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess) e = lfk::launch_gather(ddesc, E, in, s.stream);
        if (e == hipSuccess) e = lfk::launch_event_uniform(d, reinterpret_cast<uint8_t *>(dr + lay.uni), s.stream);
        if (e == hipSuccess) e = lfk::launch_find(d, P, nhw, n_sides, 1, exec, nullptr, s.stream);
        if (e == hipSuccess)
            e = lfk::launch_digest(d, d.trk_off, E, reinterpret_cast<unsigned long long *>(dr + lay.dig), s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s.out, dr + lay.dig, down, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        return e;
    };

    // ---- warm-up (before the clock): one small batch through every slot ----
    {
        std::vector<uint32_t> evs;
        uint64_t H = 0, T = 0;
        for (uint32_t e = 0; e < PE && evs.size() < std::min<uint32_t>(16, cfg.max_batch_events); ++e) {
            const BatchLayout trial = layout_of((uint32_t)evs.size() + 1, (uint32_t)(H + pool.nh[e]),
                                                (uint32_t)(T + pool.nt[e]));
            if (trial.total > ring.cap || trial.out_bytes > slots[0].out_cap)
                break;
            evs.push_back(e);
            H += pool.nh[e];
            T += pool.nt[e];
        }
        if (!evs.empty()) {
            const BatchLayout lay = layout_of((uint32_t)evs.size(), (uint32_t)H, (uint32_t)T);
            for (auto &s : slots) {
                hipError_t e = launch_batch(s, evs, lay, 0);
                if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
                if (e != hipSuccess) {
                    cleanup();
                    return lfapi::ctx_fail(ctx, LF_ERR_DEVICE, std::string("lf_serve_run: ") + hipGetErrorString(e));
                }
            }
        }
    }

    // ---- the loop ----
    std::vector<double> lat(n_requests, 0.0);
    std::deque<uint32_t> queue;       // arrived, not yet in a batch
    std::deque<uint32_t> inflight;    // slot indices in submission order
    uint32_t next_arrival = 0, completed = 0;
    uint64_t n_batches = 0, batched_events = 0, max_queue = 0, bytes_in = 0, bytes_out = 0, mismatches = 0;
    std::vector<unsigned char> verify_buf;
    size_t max_dev = 0;
    int rc = LF_OK;
    const Clock::time_point t0 = Clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };
    double last_done = 0.0;
    std::vector<uint32_t> evs;

    while (completed < n_requests && rc == LF_OK) {
        bool progress = false;
        // completions, in submission order
        while (!inflight.empty()) {
            Slot &s = slots[inflight.front()];
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) { rc = lfapi::ctx_fail(ctx, LF_ERR_DEVICE, std::string("lf_serve_run: ") + hipGetErrorString(q)); break; }
            const double t = now_s();
            const unsigned long long *dig = reinterpret_cast<const unsigned long long *>(s.out);
            if (cfg.verify_results && !cfg.results_on_device) {
                // (testing) the results downloaded to host memory against the device copy
                const size_t nb = s.lay.out_bytes;
                verify_buf.resize(nb);
                const hipError_t ve = hipMemcpy(verify_buf.data(), static_cast<char *>(ring_mem) + s.ring_at + s.lay.dig,
                                                nb, hipMemcpyDeviceToHost);
                if (ve != hipSuccess) { rc = lfapi::ctx_fail(ctx, LF_ERR_DEVICE, std::string("lf_serve_run: ") + hipGetErrorString(ve)); break; }
                // the arrays only (the alignment gaps between them are never written)
                const BatchLayout &y = s.lay;
                const size_t ranges[5][2] = {{0, (size_t)y.E * 8}, {y.found - y.dig, y.T}, {y.nhits - y.dig, y.T},
                                             {y.hit_idx - y.dig, (size_t)y.T * 48}, {y.fl - y.dig, (size_t)y.T * 28}};
                for (const auto &r : ranges)
                    for (size_t k = r[0]; k < r[0] + r[1]; ++k)
                        mismatches += verify_buf[k] != static_cast<unsigned char>(s.out[k]);
            }
            for (size_t k = 0; k < s.reqs.size(); ++k) {
                const uint32_t r = s.reqs[k];
                lat[r] = t - arrival_s[r];
                if (req_digest) req_digest[r] = dig[k];
            }
            completed += (uint32_t)s.reqs.size();
            last_done = t;
            ring.free_front();
            s.busy = false;
            inflight.pop_front();
            progress = true;
        }
        if (rc != LF_OK) break;
        // arrivals
        const double t = now_s();
        while (next_arrival < n_requests && arrival_s[next_arrival] <= t) queue.push_back(next_arrival++);
        max_queue = std::max<uint64_t>(max_queue, queue.size());
        // form a batch on a free slot
        int free_slot = -1;
        for (uint32_t i = 0; i < cfg.n_slots; ++i)
            if (!slots[i].busy) { free_slot = (int)i; break; }
        if (free_slot >= 0 && !queue.empty()) {
            const bool more_coming = next_arrival < n_requests;
            const double waited = t - arrival_s[queue.front()];
            if (queue.size() >= std::max<uint32_t>(1, cfg.min_batch_events) || !more_coming ||
                waited * 1e6 >= cfg.max_wait_us) {
                Slot &s = slots[free_slot];
                // take requests while the batch fits the staging buffers and the ring
                uint64_t H = 0, T = 0;
                uint32_t E = 0;
                size_t at = 0, charged = 0;
                BatchLayout lay{};
                while (E < queue.size() && E < cfg.max_batch_events) {
                    const uint32_t ev = req_event[queue[E]];
                    const BatchLayout trial = layout_of(E + 1, (uint32_t)(H + pool.nh[ev]), (uint32_t)(T + pool.nt[ev]));
                    if (trial.out_bytes > s.out_cap) break;
                    if (ring.used + trial.total > ring.cap) break;   // admission: the budget is full
                    H += pool.nh[ev];
                    T += pool.nt[ev];
                    ++E;
                    lay = trial;
                }
                if (E > 0 && ring.alloc(lay.total, at, charged)) {
                    s.reqs.assign(queue.begin(), queue.begin() + E);
                    queue.erase(queue.begin(), queue.begin() + E);
                    s.lay = lay;
                    s.ring_at = at;
                    s.ring_bytes = charged;
                    max_dev = std::max(max_dev, ring.used);
                    evs.resize(E);
                    for (uint32_t k = 0; k < E; ++k) evs[k] = req_event[s.reqs[k]];
                    const hipError_t e = launch_batch(s, evs, lay, at);
                    if (e != hipSuccess) {
                        rc = lfapi::ctx_fail(ctx, LF_ERR_DEVICE, std::string("lf_serve_run: ") + hipGetErrorString(e));
                        break;
                    }
                    s.busy = true;
                    inflight.push_back((uint32_t)free_slot);
                    ++n_batches;
                    batched_events += E;
                    if (dev_pool) {
                        bytes_in += (uint64_t)(2 * E + 1) * 4;   // event list and slot offsets
                    } else {
                        for (uint32_t k = 0; k < E; ++k)
                            bytes_in += 25 * 4 + (uint64_t)pool.nh[evs[k]] * 12 + (uint64_t)pool.nt[evs[k]] * 20;
                        bytes_in += (uint64_t)E * sizeof(lfk::GatherDesc);
                    }
                    bytes_out += cfg.results_on_device ? (uint64_t)E * 8 : lay.out_bytes;
                    progress = true;
                }
            }
        }
        if (!progress) std::this_thread::yield();
    }
    for (auto &s : slots) (void)hipStreamSynchronize(s.stream);
    cleanup();
    if (rc != LF_OK) return rc;

    if (req_latency_s) std::memcpy(req_latency_s, lat.data(), n_requests * sizeof(double));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        std::vector<double> l(lat);
        std::sort(l.begin(), l.end());
        auto pct = [&](double p) {
            if (l.empty()) return 0.0;
            size_t k = (size_t)(p * (double)(l.size() - 1) + 0.5);
            return l[std::min(k, l.size() - 1)];
        };
        const double first = n_requests ? arrival_s[0] : 0.0;
        stats->n_requests = n_requests;
        stats->n_batches = n_batches;
        stats->wall_s = last_done - first;
        stats->events_per_s = stats->wall_s > 0 ? n_requests / stats->wall_s : 0.0;
        stats->lat_p50_s = pct(0.50);
        stats->lat_p99_s = pct(0.99);
        stats->lat_p999_s = pct(0.999);
        stats->lat_max_s = l.empty() ? 0.0 : l.back();
        stats->mean_batch_events = n_batches ? (double)batched_events / n_batches : 0.0;
        stats->max_device_bytes = max_dev;
        stats->max_queue = max_queue;
        stats->bytes_in = bytes_in;
        stats->bytes_out = bytes_out;
        stats->result_mismatches = mismatches;
    }
    return LF_OK;
}

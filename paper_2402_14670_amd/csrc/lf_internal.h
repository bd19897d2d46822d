// lf_internal.h -- structures shared by the host side (lf_api.cpp) and the
// kernels (lf_kernels.hip) of the GPU library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lfk {

constexpr int NL = 12;
constexpr int MAX_WINDOW = 64;    // n_hits_window upper bound (6-bit window-relative indices)
constexpr int MAX_TRIPLETS = 32;  // n_triplets upper bound

// Geometry and parameters, passed to every kernel by value.
struct KParams {
    float z[NL], dxdy[NL];
    float z_in, z_mag, z_ref, z_T, kick, kappa, dRatio;
    int32_t polarity;
    float T_triplet, T_x, T_uv_scale, T_uv_floor, T_ty, T_y, T_Q;
    float xtol_const, xtol_pscale, xasym, uv_halfwidth, K_first, K_last;
    float magtol_const, magtol_pscale, magtol_txscale, magtol_min, magtol_max, p_charge_cut;
    float C_nhits[4];
    int32_t n_hits_window, n_triplets;
    // No-UT tuning (VELO-only input): straight-line extrapolation, assumed
    // minimum momentum, two windows per layer
    int32_t velo_only;
    float noUT_c[8], noUT_p_min, noUT_pt_min, noUT_overlap;
    // Momentum form: 0 linear kick; 1 sqrt-normalised pt-kick with the
    // integrated field F(tx, ty, dSlope) = sum_i c_i dSlope^i, c_i from F_coef
    int32_t field_form;
    float F_coef[5][10];
    // Triplet seeding in binary16 (VELO-UT input only)
    int32_t seed_fp16;
};

// Device view of one resident batch (SoA, all in HBM).
struct DevBatch {
    const uint32_t *hit_off;   // [24*E+1]
    const float *hx, *hz, *hd; // [H]
    const uint32_t *trk_off;   // [E+1]
    const uint32_t *trk_ev;    // [T] event of each track
    const float *tx_, *ty_, *ttx, *tty, *tqop;  // [T]
    const uint8_t *uni;        // [E] 1: in every bucket of the event all hits share one z and one dxdy (bit for bit)
    uint8_t *found, *nhits;    // [T]
    int32_t *hit_idx;          // [12*T]
    float *a, *b, *c, *y0, *ty, *qop, *Q;  // [T]
    uint32_t *counter;         // [QUEUE_WORDS] persistent-mode queue heads and exited-wave count, zero between launches
    unsigned long long *stats; // [32] work counters (counting launch only)
    uint32_t n_events, n_tracks;
    // batched mode over slots of a resident pool: result slot t (< n_map)
    // follows input track trk_map[t] (nullptr: slot t is track t)
    const uint32_t *trk_map;
    uint32_t n_map;
};

// Work queues of the persistent mode: QUEUE_SUB per XCD (8 XCDs), heads
// QUEUE_STRIDE words (256 bytes) apart, then the exited-wave count.
constexpr uint32_t QUEUE_SUB = 16;
constexpr uint32_t QUEUE_N = 8 * QUEUE_SUB;
constexpr uint32_t QUEUE_STRIDE = 64;
constexpr uint32_t QUEUE_WORDS = QUEUE_STRIDE * (QUEUE_N + 1);

struct ExecCfg {
    int waves_per_block;
    int items_per_grab;
    int blocks_per_cu;
    int n_cu;
};

// One event of a serving batch: its blob in pinned host memory (device
// address) -- [bucket offsets, event-local: u32 x 25][x H][z H][dxdy H]
// [track x, y, tx, ty, q/p: 5 x T] -- and where it goes in the batch.
struct GatherDesc {
    uint64_t src;
    uint32_t hit_base, trk_base, n_hits, n_tracks;
};

// Writable view of a batch's input arrays (the serving gather fills them).
struct BatchIn {
    uint32_t *hit_off;
    float *hx, *hz, *hd;
    uint32_t *trk_off, *trk_ev;
    float *tx, *ty, *ttx, *tty, *tqop;
};

// Assembles a batch of E events on the device from their host blobs
// (zero-copy reads over the host link): offsets rebased, hits and track
// states copied, trk_ev filled.  desc is in device memory.
hipError_t launch_gather(const GatherDesc *desc, uint32_t n_events, const BatchIn &out, hipStream_t s);

// Fills trk_ev from trk_off (one thread per track).
hipError_t launch_track_event(const DevBatch &b, hipStream_t s);
// Result slots of a batch of pool events evs[0..n_events) (slots [toff[e],
// toff[e+1]) for event e, n_slots = toff[n_events], read on the device):
// map[i] = the pool track slot i follows.  All arrays in device memory.
hipError_t launch_track_map(const uint32_t *evs, const uint32_t *toff, uint32_t n_events, uint32_t n_slots,
                            const uint32_t *pool_trk_off, uint32_t *map, hipStream_t s);
// The hot path.  P points to a KParams in device memory.  mode: 0 plain
// (per-event launches), 1 batched (one wavefront per track), 2 persistent
// (resident wavefronts pulling from per-XCD work queues).
// trk_off_host is read by mode 0 only.
// n_sides: 1 for VELO-UT input, 2 for VELO-only input (two windows per
// layer), 3 for VELO-UT input with the binary16 seeding build.
hipError_t launch_find(const DevBatch &b, const KParams *P, int n_hits_window, int n_sides, int mode,
                       const ExecCfg &cfg, const uint32_t *trk_off_host, hipStream_t s);
// Writes the per-event flag of DevBatch::uni into uni[E] (one block per
// event; the batch's hits must be in place).
hipError_t launch_event_uniform(const DevBatch &b, uint8_t *uni, hipStream_t s);
// Counting launch: one wavefront per track, adds the work counters of every
// track into b.stats (which must be zeroed first).
hipError_t launch_count(const DevBatch &b, const KParams *P, int n_hits_window, int n_sides, hipStream_t s);
// Fills the result slots with a poison pattern (kernel, no memset).
hipError_t launch_poison(const DevBatch &b, hipStream_t s);
// Resident blocks per compute unit of the persistent kernel (0 on error).
int persistent_blocks_per_cu(int n_hits_window, int n_sides, int waves_per_block);

// Fixed scratch of the non-allocating entry point: one array in the code
// object's device memory per GPU, holding the persistent mode's queue words,
// the per-event uniform flags and the event of each track.
constexpr uint32_t FIXED_MAX_EVENTS = 1u << 20;
constexpr uint32_t FIXED_MAX_TRACKS = 1u << 22;
constexpr size_t FIXED_QUEUE_OFF = 0;                       // QUEUE_WORDS x u32
constexpr size_t FIXED_UNI_OFF = 4 * (size_t)QUEUE_WORDS;   // FIXED_MAX_EVENTS x u8
constexpr size_t FIXED_TRK_EV_OFF = FIXED_UNI_OFF + FIXED_MAX_EVENTS;   // FIXED_MAX_TRACKS x u32
constexpr size_t FIXED_BYTES = FIXED_TRK_EV_OFF + 4 * (size_t)FIXED_MAX_TRACKS;
// Device address of the current device's copy of the fixed scratch, looked
// up once per device (the first call on a device must run with it current).
hipError_t fixed_scratch(void **out);
// Writes zeros to n words with a kernel (no memset node under capture).
hipError_t launch_zero_words(uint32_t *p, uint32_t n, hipStream_t s);

}  // namespace lfk

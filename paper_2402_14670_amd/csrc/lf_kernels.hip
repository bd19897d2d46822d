// lf_kernels.hip -- Looking Forward track following, gfx950 kernels.
//
// One wavefront (64 lanes) carries one upstream input track through every
// step of the method (arXiv 2402.14670, "Algorithm logic"):
//
//   windows    the kick (linear, or the sqrt-normalised pt-kick with the
//              momentum parametrisation F), then 36 lanes: (layer, bound)
//              binary searches over the x-sorted bucket in HBM; 12 lanes
//              apply the symmetric cap ("Defining the search windows").
//   staging    the <= 12 x n_hits_window window hits are read coalesced from
//              HBM into this wave's LDS slice: x, z and dxdy per hit; x only
//              where LDS bounds the occupancy, and in events whose buckets
//              each hold one z and one dxdy (flagged by k_event_uniform).
//   doublets   one first-layer hit of a seed set per lane; the range of
//              third-layer hits that can pass the magnet filter is
//              bracketed by a sorted search, each pair in it tested with the
//              charge and magnet-opening filters; survivors compacted with
//              ballot + mbcnt into an LDS queue ("Triplet Seeding").
//   triplets   64 queued doublets per pass search the middle layer for the
//              closest hit; accepted triplets merge into an exact top-n list
//              keyed by (chi2, side, set, h0, h2) by rank counting.
//   extension  lanes = (candidate, missing layer): closest hit to the
//              triplet's x(z) model ("Extending triplets to other layers").
//   fit        16 lanes per candidate (lane = layer slot), four candidates
//              per pass: x and y least squares with every sum taken
//              serially in layer order by a DPP chain, Q, cuts ("Quality
//              Filter");
//              the argmin over (Q, rank) picks the track; q/p from the slope
//              change ("Calculation of momentum and track states").
//
// The arithmetic is binary32 in a fixed order (the library is built with
// -ffp-contract=off, correctly rounded division, no fast-math), so every
// decision is identical to a serial evaluation of the same expressions.
// Nothing in this file allocates; the kernels' scratch is LDS, apart from
// the fixed device array that the non-allocating entry point uses for its
// queue words and per-event and per-track indexes.
#include <cstddef>
#include <mutex>

#include "lf_internal.h"

namespace lfk {
namespace {

constexpr int WAVE = 64;
constexpr int QCAP = 128;             // doublet queue: < 64 pending + one pass of 64
constexpr int NSLOT = 9;              // extension work per candidate: 3 x layers + 6 u/v layers
constexpr float INV1024 = 0.0009765625f;            // 2^-10, exact
constexpr float INV1024SQ = 0.00000095367431640625f; // 2^-20, exact

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// The lane index, opaque to the optimiser: a kernel that loops over tracks
// hands this to each track, so that values derived from the lane are not
// hoisted out of the loop (they would stay live in registers across the
// whole loop body).
__device__ __forceinline__ int opaque_lane_id() {
    int l = (int)__lane_id();
    asm volatile("" : "+v"(l));
    return l;
}

// Element i of a device array of less than 4 GiB (the host checks the batch
// sizes): a 32-bit byte offset from a wave-uniform base, so the load takes
// the scalar-base form with one 32-bit address register.
template <class T>
__device__ __forceinline__ T ld32(const T *base, uint32_t i) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}

__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int CTRL, bool BOUND_ZERO>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, BOUND_ZERO));
}

// Serial sums over the layer slots of each 16-lane row (slot = lane % 16):
// afterwards lane 11 of a row holds ((+0 + t_0) + t_1) + ... + t_11 of that
// row's lanes 0..11, for each of the N sums; the other lanes hold partial
// sums.  Step k adds each lane's term to the partial sum moved over from the
// lane before it (row_shr:1, which reads 0 in a row's lane 0), so the partial
// sum in lane l after step k covers slots l-k..l in ascending order.  The N
// chains advance together and fill each other's DPP read hazards.
template <int N>
__device__ __forceinline__ void chain12(const float (&t)[N], float (&s)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] = 0.0f + t[i];
#pragma unroll
    for (int k = 1; k < NL; ++k) {
#pragma unroll
        for (int i = 0; i < N; ++i) s[i] = dpp<0x111, true>(s[i]) + t[i];   // row_shr:1
    }
}

// Lane 11 of each row's value, broadcast over the row (row_newbcast:11).
__device__ __forceinline__ float row_lane11(float v) { return dpp<0x15B, false>(v); }

// Lane k (0..9, a constant after unrolling) of each row's value, broadcast
// over the row (row_newbcast:k).
__device__ __forceinline__ float row_bcast_lane(float v, int k) {
    switch (k) {
        case 0: return dpp<0x150, false>(v);
        case 1: return dpp<0x151, false>(v);
        case 2: return dpp<0x152, false>(v);
        case 3: return dpp<0x153, false>(v);
        case 4: return dpp<0x154, false>(v);
        case 5: return dpp<0x155, false>(v);
        case 6: return dpp<0x156, false>(v);
        case 7: return dpp<0x157, false>(v);
        case 8: return dpp<0x158, false>(v);
        default: return dpp<0x159, false>(v);
    }
}

// The least float above x (NaN and +inf map to themselves, +-0 to the least
// positive subnormal): for every finite v, v <= x exactly when v < next_up(x).
__device__ __forceinline__ float next_up(float x) {
    const int b = __float_as_int(x);
    if (!(x < INFINITY)) return x;                 // NaN, +inf
    if ((b & 0x7fffffff) == 0) return __int_as_float(1);
    return __int_as_float(x > 0.0f ? b + 1 : b - 1);
}

// Lane i's float, broadcast (i uniform).
__device__ __forceinline__ float bcast_f(float v, int i) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}

// Lane i's 64-bit value, broadcast (i uniform).
__device__ __forceinline__ uint64_t bcast64(uint64_t v, int i) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, i);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), i);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ bool is_uv(int l) {
    const int k = l & 3;
    return k == 1 || k == 2;
}

// Packed binary16 pair: one instruction handles two seeding combinations.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ _Float16 habs(_Float16 v) { return v < (_Float16)0.0f ? -v : v; }

// x(z) model term g(u) = u^2 (1 + dRatio u), u = z - z_ref.
__device__ __forceinline__ float g_of(float u, float dR) { return u * u * (1.0f + dR * u); }

// Sine-like slope of the pt-kick equation ("Defining the search windows"),
// tx / sqrt(1 + tx^2 + ty^2).
__device__ __forceinline__ float kick_s(float tx, float ty) { return tx / sqrtf(1.0f + tx * tx + ty * ty); }

// Momentum parametrisation ("Calculation of momentum and track states"):
// F = c0 + d (c1 + d (c2 + d (c3 + d c4))) for dSlope d.
__device__ __forceinline__ float field_F(const float c[5], float d) {
    return c[0] + d * (c[1] + d * (c[2] + d * (c[3] + d * c[4])));
}

// Coefficient c_i(tx, ty) of the parametrisation for i = lane (lanes 0..4;
// other lanes return row 0): the monomials 1, tx2, ty2, tx2^2, tx2 ty2,
// ty2^2, tx2^3, tx2^2 ty2, tx2 ty2^2, ty2^3 (tx2 = tx^2, ty2 = ty^2) weighted
// by row i of the table and summed in that order, ten terms for even i, the
// first six times tx for odd i.
__device__ __forceinline__ float field_c_lane(const KParams *__restrict__ P, float tx, float ty, int lane) {
    const int i = lane < 5 ? lane : 0;
    const float *row = &P->F_coef[i][0];
    const float x2 = tx * tx, y2 = ty * ty;
    const float m[10] = {1.0f, x2, y2, x2 * x2, x2 * y2, y2 * y2, x2 * x2 * x2, x2 * x2 * y2, x2 * y2 * y2,
                         y2 * y2 * y2};
    float w[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) w[j] = row[j];
    float acc = w[0] * m[0];
#pragma unroll
    for (int j = 1; j < 6; ++j) acc = acc + w[j] * m[j];
    if (i & 1) return tx * acc;
#pragma unroll
    for (int j = 6; j < 10; ++j) acc = acc + w[j] * m[j];
    return acc;
}

// Binary searches over at most NMAX (a power of two) window entries, in a
// fixed number of steps: p advances by s = NMAX, NMAX/2, .., 1 while the
// entry before p + s still satisfies the (monotone) predicate, so p ends as
// the number of leading entries that satisfy it.  Only entries < n are read.

// Number of leading indices j < n for which pred(j) holds, for a predicate
// that holds on a prefix; two predicates searched together.
template <int NMAX, class P1, class P2>
__device__ __forceinline__ void prefix2(int n, P1 p1, P2 p2, int &c1, int &c2) {
    int p = 0, q = 0;
#pragma unroll
    for (int s = NMAX; s > 0; s >>= 1) {
        if (p + s <= n && p1(p + s - 1)) p += s;
        if (q + s <= n && p2(q + s - 1)) q += s;
    }
    c1 = p;
    c2 = q;
}

// Lower bound (v < klo) and upper bound (v <= khi) of one non-decreasing LDS
// array, searched together.
template <int NMAX>
__device__ __forceinline__ void bounds_sorted(const float *v, int n, float klo, float khi, int &lo, int &hi) {
    int p = 0, q = 0;
#pragma unroll
    for (int s = NMAX; s > 0; s >>= 1) {
        if (p + s <= n && v[p + s - 1] < klo) p += s;
        if (q + s <= n && v[q + s - 1] <= khi) q += s;
    }
    lo = p;
    hi = q;
}

// Closest hit of a window: the first index j minimising d_j = |val(j) - xe|
// (the result of a linear scan with a strict '<' update), or -1 when no d_j
// is below infinity.  val(j) must be non-decreasing in j.  Then
// RN(val(j) - xe) is non-decreasing too, so d falls up to the first j with
// val(j) >= xe and rises after it: only that index, its left neighbour and
// the plateau of equal d ending at the left neighbour can hold the answer.
// Given p = #{j < n: val(j) < xe}: the closest index as described above.
template <class Val>
__device__ __forceinline__ int closest_finish(Val val, int n, float xe, int p, float &bd) {
    int best = p;
    float d = p < n ? fabsf(val(p) - xe) : INFINITY;
    if (p > 0) {
        const float dl = fabsf(val(p - 1) - xe);
        if (!(d < dl)) {
            best = p - 1;
            d = dl;
            while (best > 0 && fabsf(val(best - 1) - xe) == dl) --best;
        }
    }
    if (!(d < INFINITY)) return -1;
    bd = d;
    return best;
}

template <int NMAX, class Val>
__device__ __forceinline__ int closest_sorted(Val val, int n, float xe, float &bd) {
    int p = 0;
#pragma unroll
    for (int s = NMAX; s > 0; s >>= 1)
        if (p + s <= n && val(p + s - 1) < xe) p += s;
    return closest_finish(val, n, xe, p, bd);
}

// Two independent sorted searches advanced step by step together, so that
// their dependent LDS reads overlap.
template <int NMAX, class ValA, class ValB>
__device__ __forceinline__ void closest_sorted2(ValA va, int na, float xa, int &ba, float &da,
                                                ValB vb, int nb, float xb, int &bb, float &db) {
    int pa = 0, pb = 0;
#pragma unroll
    for (int s = NMAX; s > 0; s >>= 1) {
        const bool ta = pa + s <= na && va(pa + s - 1) < xa;
        const bool tb = pb + s <= nb && vb(pb + s - 1) < xb;
        if (ta) pa += s;
        if (tb) pb += s;
    }
    ba = closest_finish(va, na, xa, pa, da);
    bb = closest_finish(vb, nb, xb, pb, db);
}

// The same by linear scan, for windows whose values are not sorted.
template <class Val>
__device__ __forceinline__ int closest_scan(Val val, int n, float xe, float &bd) {
    int best = -1;
    float d = INFINITY;
    for (int j = 0; j < n; ++j) {
        const float dj = fabsf(val(j) - xe);
        if (dj < d) { d = dj; best = j; }
    }
    bd = d;
    return best;
}

// Index of stereo layer l (l % 4 in {1, 2}) among the six stereo layers.
__device__ __forceinline__ int uv_index(int l) { return 2 * (l >> 2) + (l & 3) - 1; }

// NS = 1: one window per layer; NS = 2 (VELO-only input): two windows per
// layer, side 0 for bending towards -x, side 1 towards +x.
// Where LDS bounds the occupancy (two windows per layer, or 64-hit windows)
// the hits keep only x in LDS (XO): a window keeps its first hit's z (stereo
// tangent), the value of all its hits unless the window is mixed, whose
// hits are then read from HBM.
template <int NW, int NS>
struct WaveLds {
    static constexpr bool XO = NS == 2 || NW > 32;
    static constexpr int ZW = XO ? 1 : NW;
    float wx[NS][NL][NW];      // window hits: x at y = 0
    float wz[NS][NL][ZW];      //              z (XO: first hit only)
    float wd[NS][6][ZW];       //              stereo tangent (stereo layers; XO: first hit only)
    int32_t wfirst[NS][NL];    // event-local index of each window's first hit
    int32_t wlen[NS][NL];
    float gz[NL];              // z of each layer plane
    uint64_t tk[MAX_TRIPLETS];      // top-n keys, sorted
    uint8_t th1[MAX_TRIPLETS];      // middle hit of each kept triplet
    union {
        struct {               // seeding
            uint32_t qkey[QCAP];    // queued doublets: side << 17 | set << 16 | i0 << 8 | i2
        };
        struct {               // candidates (after seeding)
            float ca[MAX_TRIPLETS], cb[MAX_TRIPLETS], cc[MAX_TRIPLETS];  // triplet x(z) models
            union {
                int8_t ch[MAX_TRIPLETS][NL];    // candidate hits, window-relative, -1 = none
                uint32_t chw[MAX_TRIPLETS][NL / 4];   // the same, four layers per word
            };
        };
    };
};

// Work counters of one track (only in the counting build, CNT = true).
enum { C_TRACKS, C_PAIRS_ALL, C_ITEMS, C_PAIRS_TESTED, C_DOUBLETS, C_TRIPLETS, C_KEPT, C_FITTED,
       C_ACCEPTED, C_STAGED, C_FOUND,
       // shader-clock cycles spent per phase (counting build only)
       C_CY_WINDOWS, C_CY_STAGE, C_CY_DOUBLETS, C_CY_MODEL, C_CY_EXTEND, C_CY_FIT, C_CY_SELECT, C_N };

// H16: the binary16 seeding build (seed_fp16, one window per layer).
template <int NW, int NS, bool CNT = false, bool H16 = false>
struct Track {
    const DevBatch &B;
    const KParams *__restrict__ P;
    WaveLds<NW, NS> &L;
    int nL;    // kept triplets
    uint32_t cnt[CNT ? C_N : 1];
    uint64_t tphase;
    // bit NL * side + layer: the window's hits do not all share one z
    // (zvar) or one stereo tangent (dvar); ebase: the event's first hit
    uint32_t zvar = 0, dvar = 0, ebase = 0;
    // the event's hits share one z and one dxdy per bucket (DevBatch::uni):
    // only x is staged per hit, each window keeps its first hit's values
    bool uni = false;
    // this wave's lane index (opaque_lane_id() in kernels that loop over tracks)
    int ln = lane_id();
    // z of the middle-layer planes of the two seed sets (layers 4 and 7)
    float z4 = 0.0f, z7 = 0.0f;
    // Binary16 seeding: per seed set, whether it runs in half precision
    // (seed_fp16, both outer windows non-empty with one z each), the window
    // centres and its constants; then the ones shared by both sets.
    bool hon[2] = {false, false};
    float hc0[2] = {0.0f, 0.0f}, hc1[2] = {0.0f, 0.0f}, hc2[2] = {0.0f, 0.0f};
    _Float16 hRZ[2], hC02[2], hE0[2], hL0[2], hA[2], hKK[2], hB[2];
    _Float16 hTMAX, hT3;
    // (tx, q/p), (tx scale, constant) and (min, max) of the magnet
    // tolerance as binary16 pairs, wave-uniform (kept in scalar registers)
    uint32_t kTXQP, kTXSTC, kTMINMAX;
    // element s of a per-set pair, without indexing (a lane-dependent index
    // would put the arrays in scratch memory)
    template <class T>
    __device__ __forceinline__ static T sel(const T (&a)[2], int s) { return s ? a[1] : a[0]; }

    // z and stereo tangent of hit i of a window: from LDS, or (XO) the
    // window's one value, or from HBM for a mixed window
    static constexpr bool XO = WaveLds<NW, NS>::XO;
    __device__ __forceinline__ float zat(int sd, int l, int i) const {
        if constexpr (!XO) return L.wz[sd][l][uni ? 0 : i];
        if ((zvar >> (NL * sd + l)) & 1u) return ld32(B.hz, ebase + (uint32_t)(L.wfirst[sd][l] + i));
        return L.wz[sd][l][0];
    }
    __device__ __forceinline__ float dat(int sd, int l, int i) const {
        if constexpr (!XO) return L.wd[sd][uv_index(l)][uni ? 0 : i];
        if ((dvar >> (NL * sd + l)) & 1u) return ld32(B.hd, ebase + (uint32_t)(L.wfirst[sd][l] + i));
        return L.wd[sd][uv_index(l)][0];
    }

    // The N (<= 10) serial sums of chain12 -- ((+0 + t_0) + t_1) + ... + t_11
    // over a row's layer lanes 0..11 -- formed by a transpose through LDS
    // instead: lane (g, j) writes its terms, lane (g, k) reads the 12 terms
    // of sum k and adds them in layer order, and every lane of the row then
    // receives each sum (row_newbcast).  The same operations in the same
    // order as the chain, with 12 additions for all the sums instead of 12
    // per sum.  The scratch is the per-hit z and stereo-slope area of the
    // windows, which the fits of a uniform event do not read (they hold each
    // window's common z and slope in registers): sum slot g N + k is 12
    // floats at 48 (g N + k) bytes.  Only in builds that stage z per hit.
    template <int N>
    __device__ __forceinline__ void row_sums_lds(const float (&t)[N], float (&s)[N], int g, int j) {
        using W = WaveLds<NW, NS>;
        static_assert(!W::XO, "needs the per-hit z and slope rows");
        static_assert(N <= 10 && 4 * N * 12 <= NS * (NL + 6) * W::ZW, "4 N slots of 12 floats");
        static_assert(offsetof(W, wd) == offsetof(W, wz) + sizeof(L.wz), "wz and wd must be one run");
        // wz, then wd: one run of floats of the wave's slice
        float *base = reinterpret_cast<float *>(reinterpret_cast<char *>(&L) + offsetof(W, wz));
        wave_sync();   // the previous use of the scratch has been read
        if (j < NL) {
#pragma unroll
            for (int k = 0; k < N; ++k) base[(g * N + k) * 12 + j] = t[k];
        }
        wave_sync();
        float v = 0.0f;
        if (j < N) {
            const float4 *p = reinterpret_cast<const float4 *>(base + (g * N + j) * 12);
            const float4 q0 = p[0], q1 = p[1], q2 = p[2];
            v = 0.0f + q0.x;
            v = v + q0.y; v = v + q0.z; v = v + q0.w;
            v = v + q1.x; v = v + q1.y; v = v + q1.z; v = v + q1.w;
            v = v + q2.x; v = v + q2.y; v = v + q2.z; v = v + q2.w;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) s[k] = row_bcast_lane(v, k);
    }

    // The serial sums of chain12, the same in every lane of the row: a
    // uniform event's through LDS (row_sums_lds), otherwise the chain's
    // lane 11 broadcast over the row.
    template <int N>
    __device__ __forceinline__ void row_sums(const float (&t)[N], float (&s)[N], int g, int j) {
        if constexpr (!WaveLds<NW, NS>::XO) {
            if (uni) {
                row_sums_lds(t, s, g, j);
                return;
            }
        }
        chain12(t, s);
#pragma unroll
        for (int k = 0; k < N; ++k) s[k] = row_lane11(s[k]);
    }

    // Adds the shader-clock cycles since the previous mark to counter k.
    __device__ __forceinline__ void mark(int k) {
        if constexpr (CNT) {
            const uint64_t now = __builtin_readcyclecounter();
            cnt[k] += (uint32_t)(now - tphase);
            tphase = now;
        }
    }

    // Merge this pass's accepted triplets (one per lane) into the top-n list.
    // Every element's place in the merged order is its rank among the kept
    // list (sorted, lane i < nL holds entry i) and this pass's keys, counted
    // against broadcast keys; keys are distinct, so the ranks are too.
    __device__ void merge(bool valid, uint64_t key, int h1) {
        const int lane = ln;
        const uint64_t bal = __ballot(valid);
        const int nb = __popcll(bal);
        if (nb == 0) return;
        const int NT = P->n_triplets;
        const uint64_t mine = lane < nL ? L.tk[lane] : 0ull;
        const int mh1 = lane < nL ? L.th1[lane] : 0;
        int r_new = 0, r_old = lane;
        for (int i = 0; i < nL; ++i) r_new += L.tk[i] < key ? 1 : 0;
        for (uint64_t m = bal; m; m &= m - 1) {
            const uint64_t k = bcast64(key, __builtin_ctzll(m));
            r_new += k < key ? 1 : 0;
            r_old += k < mine ? 1 : 0;
        }
        wave_sync();   // every lane has read the old list
        if (valid && r_new < NT) {
            L.tk[r_new] = key;
            L.th1[r_new] = (uint8_t)h1;
        }
        if (lane < nL && r_old < NT) {
            L.tk[r_old] = mine;
            L.th1[r_old] = (uint8_t)mh1;
        }
        nL = nL + nb < NT ? nL + nb : NT;
        wave_sync();
    }

    // Complete the first `count` queued doublets with their closest middle hit.
    __device__ void flush(int count) {
        const int lane = ln;
        bool tri = false, valid = false;
        uint64_t key = 0;
        int best = -1;
        if (lane < count) {
            const uint32_t e = L.qkey[lane];
            const int sd = NS > 1 ? (int)((e >> 17) & 1u) : 0;
            const int s = (int)((e >> 16) & 1u), i0 = (int)((e >> 8) & 0xffu), i2 = (int)(e & 0xffu);
            const int l0 = s ? 3 : 0, l1 = s ? 7 : 4, l2 = s ? 11 : 8;
            float bd = INFINITY;
            if (H16 && sel(hon, s)) {
                // binary16: the slope as queued, the prediction relative to
                // c1, the closest hit by a scan over pairs of hits
                const _Float16 X0 = (_Float16)(L.wx[0][l0][i0] - sel(hc0, s));
                const _Float16 X2 = (_Float16)(L.wx[0][l2][i2] - sel(hc2, s));
                const _Float16 u = X2 - X0;
                const _Float16 v = u + sel(hC02, s);
                const _Float16 tt = v * sel(hRZ, s);
                const _Float16 a1 = tt * sel(hA, s);
                const _Float16 a2 = X0 * sel(hKK, s);
                const _Float16 a3 = a1 + a2;
                const _Float16 X1e = a3 + sel(hB, s);
                const float *wx1 = L.wx[0][l1];
                const int n1 = L.wlen[0][l1];
                const float c1 = sel(hc1, s);
                // The window's Y_j = h(x_j - c1) are sorted, so d_j = |h(Y_j - X1e)|
                // falls up to p = #{Y_j < X1e} and rises from p.  The first
                // minimum of a scan is p, or the first index of the plateau
                // ending at p - 1 when d_(p-1) <= d_p.
                auto Y = [&](int j) { return (_Float16)(wx1[j] - c1); };
                auto D = [&](int j) { return habs(Y(j) - X1e); };
                _Float16 hb = (_Float16)INFINITY;
                int pp = 0, qq = 0, unused = 0;
                prefix2<NW>(n1, [&](int j) { return Y(j) < X1e; }, [](int) { return false; }, pp, unused);
                if (pp < n1) { hb = D(pp); best = pp; }
                if (pp > 0) {
                    const _Float16 dl = D(pp - 1);
                    if (!(dl > hb)) {
                        prefix2<NW>(pp, [&](int j) { return D(j) > dl; }, [](int) { return false; }, qq, unused);
                        hb = dl;
                        best = qq;
                    }
                }
                if (best >= 0) {
                    const _Float16 c2h = hb * hb;
                    if (c2h < hT3) {
                        tri = true;
                        key = ((uint64_t)__float_as_uint((float)c2h) << 32) |
                              (uint64_t)(uint32_t)((sd << 13) | (s << 12) | (i0 << 6) | i2);
                        valid = nL < P->n_triplets || key < L.tk[nL - 1];
                    }
                }
                best = tri ? best : -1;
            } else {
            const float K = s ? P->K_last : P->K_first;
            const float x0 = L.wx[sd][l0][i0], z0 = zat(sd, l0, i0);
            const float txd = (L.wx[sd][l2][i2] - x0) / (zat(sd, l2, i2) - z0);   // the doublet's slope, as queued
            const float x1e = (s ? z7 : z4) * txd + (x0 - txd * z0) * K;
            const float *wx1 = L.wx[sd][l1];
            best = closest_sorted<NW>([wx1](int j) { return wx1[j]; }, L.wlen[sd][l1], x1e, bd);
            if (best >= 0) {
                const float chi2 = bd * bd;
                if (chi2 < P->T_triplet) {
                    tri = true;
                    key = ((uint64_t)__float_as_uint(chi2) << 32) |
                          (uint64_t)(uint32_t)((sd << 13) | (s << 12) | (i0 << 6) | i2);
                    // a full list only admits keys below its last one (exactly what the
                    // rank count of merge() would keep)
                    valid = nL < P->n_triplets || key < L.tk[nL - 1];
                }
            }
            }
        }
        if constexpr (CNT) cnt[C_TRIPLETS] += (uint32_t)__popcll(__ballot(tri));
        merge(valid, key, best);
    }

    // Track tin of the batch (input state), result slot t, event ev.
    __device__ void run(uint32_t t, uint32_t ev, uint32_t tin) {
        const int lane = ln;
        if constexpr (CNT) {
            for (int k = 0; k < C_N; ++k) cnt[k] = 0;
            cnt[C_TRACKS] = 1;
            tphase = __builtin_readcyclecounter();
        }
        // bucket offsets of this event (both zones), fetched with the track state
        const uint32_t ho = lane <= 2 * NL ? ld32(B.hit_off, ev * 24u + (uint32_t)lane) : 0u;
        const float x_in = B.tx_[tin], y_in = B.ty_[tin], tx_in = B.ttx[tin], ty_in = B.tty[tin];
        const float qop = B.tqop[tin];
        const float dR = P->dRatio;
        // lane l < 12: the z and stereo tangent of layer plane l (fetched by
        // the lanes that need them with a cross-lane read)
        const float gz = lane < NL ? P->z[lane] : 0.0f, gd = lane < NL ? P->dxdy[lane] : 0.0f;
        z4 = bcast_f(gz, 4);
        z7 = bcast_f(gz, 7);

        // ---- kinematics ----
        // VELO-UT input: p and q from q/p.  VELO-only input: the assumed
        // minimum momentum, the tighter (larger) of p_min and the momentum
        // at which the track's transverse momentum is pt_min.
        float p;
        int q = 0;
        if constexpr (NS == 2) {
            const float t2 = tx_in * tx_in + ty_in * ty_in;
            const float sin_t = sqrtf(t2 / (1.0f + t2));
            const float p_pt = sin_t > 0.0f ? P->noUT_pt_min / sin_t : 0.0f;
            p = p_pt > P->noUT_p_min ? p_pt : P->noUT_p_min;
        } else {
            p = 1.0f / fabsf(qop);
            q = qop > 0.0f ? 1 : -1;
        }
        const int zone = ty_in >= 0.0f ? 1 : 0;
        const float x_mag = x_in + tx_in * (P->z_mag - P->z_in);
        // The kick.  Linear: dtx = kick * q/p.  Paper form: the sqrt-normalised
        // pt-kick equation s_f = s_i + (q/p) F solved for the slope after the
        // magnet, F taken at dSlope = 0 and then twice at the slope change of
        // the previous solution; no solution (|s_f| >= 1): the track is not
        // searched.  The c_i also serve the momentum at the end.
        const bool paper = P->field_form == 1;
        float fc[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        float dtx = 0.0f;
        if (paper) {
            const float cl = field_c_lane(P, tx_in, ty_in, lane);
#pragma unroll
            for (int i = 0; i < 5; ++i) fc[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cl), i));
            if constexpr (NS == 1) {
                const float si = kick_s(tx_in, ty_in);
                float d = 0.0f;
                bool ok = true;
#pragma unroll
                for (int it = 0; it < 3; ++it) {
                    const float sf = si + qop * field_F(fc, d);
                    if (!(sf * sf < 1.0f)) { ok = false; break; }
                    d = sf * sqrtf((1.0f + ty_in * ty_in) / (1.0f - sf * sf)) - tx_in;
                }
                if (!ok) {
                    write_none(t, (size_t)t * NL);
                    return;
                }
                dtx = d;
            }
        } else {
            dtx = P->kick * qop;
        }
        const float T = tx_in + dtx;
        const float kd = P->kappa * dtx;
        ebase = (uint32_t)__builtin_amdgcn_readlane((int)ho, 0);
        uni = B.uni[ev] != 0;
        // x tolerance of the x-layer windows
        float xtol;
        if constexpr (NS == 2) {
            const float ip = 1.0f / p;
            const float ty2 = ty_in * ty_in;
            const float *c8 = P->noUT_c;
            xtol = ip * (c8[0] + tx_in * (c8[1] + c8[2] * tx_in) + ty2 * (c8[3] + tx_in * (c8[4] + c8[5] * tx_in)) +
                         ip * (c8[6] * tx_in + c8[7] * ip));
        } else {
            xtol = P->xtol_const + P->xtol_pscale / p;
        }

        // ---- search windows: lane 3*l + k searches bound k of layer l, side by side ----
        int wf[NS], wl[NS];   // lane l < 12: first hit (event-local) and length of layer l's window
        float xcl = 0.0f;     // lane 3 l + 1: the centre of layer l's window
#pragma unroll
        for (int sd = 0; sd < NS; ++sd) {
            int pos = 0;
            float zb = 0.0f, db = 0.0f;   // lane 3 l, uniform event: z and stereo tangent of the bucket
            {
                const int l = lane < 3 * NL ? lane / 3 : 0;
                const uint32_t b0 = (uint32_t)__shfl((int)ho, 2 * l + zone);
                const uint32_t b1 = (uint32_t)__shfl((int)ho, 2 * l + zone + 1);
                const float zl = __shfl(gz, l), dxl = __shfl(gd, l);
                if (lane < 3 * NL) {
                    const int k = lane - 3 * l;
                    const float ye = y_in + ty_in * (zl - P->z_in);
                    float xc, xmin, xmax;
                    if constexpr (NS == 2) {
                        // straight line; two windows per layer sharing an overlap
                        const float xe = x_in + tx_in * (zl - P->z_in);
                        const float x0 = is_uv(l) ? xe - dxl * ye : xe;
                        const float tol = is_uv(l) ? P->uv_halfwidth : xtol;
                        if (sd == 0) { xmin = x0 - tol; xmax = x0 + P->noUT_overlap; }
                        else { xmin = x0 - P->noUT_overlap; xmax = x0 + tol; }
                        xc = 0.5f * (xmin + xmax);
                    } else {
                        const float dz = zl - P->z_mag;
                        const float dzT = zl - P->z_T;
                        const float xe = x_mag + T * dz + kd * dzT * dzT * (1.0f + dR * dzT);
                        if (is_uv(l)) {
                            xc = xe - dxl * ye;
                            xmin = xc - P->uv_halfwidth;
                            xmax = xc + P->uv_halfwidth;
                        } else {
                            float asymL = 0.0f, asymR = 0.0f;
                            if (q * P->polarity > 0) asymR = P->xasym; else asymL = P->xasym;
                            xc = xe;
                            xmin = xc - xtol - asymL;
                            xmax = xc + xtol + asymR;
                        }
                    }
                    const float key = k == 0 ? xmin : (k == 1 ? xc : xmax);
                    xcl = xc;
                    if (uni && k == 0 && b1 > b0) {
                        // every hit of the bucket has these: loaded while the searches run
                        zb = ld32(B.hz, b0);
                        if (is_uv(l)) db = ld32(B.hd, b0);
                    }
                    uint32_t lo = b0;
                    uint32_t n = b1 - b0;
                    // lower bound (x < key) for x_min and the centre, upper bound
                    // (x <= key) for x_max, which for finite x is x < next_up(key)
                    const float kk = k == 2 ? next_up(key) : key;
                    while (n > 0) {
                        const uint32_t half = n >> 1;
                        const float v = ld32(B.hx, lo + half);
                        if (v < kk) { lo += half + 1; n -= half + 1; } else { n = half; }
                    }
                    pos = (int)(lo - ebase);
                }
            }
            wf[sd] = 0;
            wl[sd] = 0;
            {
                const int src = lane < NL ? 3 * lane : 0;
                const int lo = __shfl(pos, src), c0 = __shfl(pos, src + 1), hi0 = __shfl(pos, src + 2);
                float zl = 0.0f, dl = 0.0f;
                if (uni) {
                    zl = __shfl(zb, src);
                    dl = __shfl(db, src);
                }
                if (lane < NL) {
                    int hi = hi0 < lo ? lo : hi0;
                    int c = c0 < lo ? lo : (c0 > hi ? hi : c0);
                    const int N = P->n_hits_window;
                    int first = lo, len = hi - lo;
                    if (hi - lo > N) {
                        first = c - N / 2;
                        if (first < lo) first = lo;
                        if (first > hi - N) first = hi - N;
                        len = N;
                    }
                    wf[sd] = first;
                    wl[sd] = len;
                    L.wfirst[sd][lane] = first;
                    L.wlen[sd][lane] = len;
                    if (sd == 0) L.gz[lane] = gz;
                    if (uni && len > 0) {
                        // the window's (and the bucket's) one z and stereo tangent
                        L.wz[sd][lane][0] = zl;
                        if (is_uv(lane)) L.wd[sd][uv_index(lane)][0] = dl;
                    }
                }
            }
        }
        mark(C_CY_WINDOWS);

        // ---- stage window hits into LDS ----
        // Round u covers slots lane + 64 u of the 12 x NW window slots (layer
        // (lane + 64 u) / NW); every load of a side is issued before its first
        // LDS write.  The same registers tell which windows have hits that do
        // not all share one z (resp. one stereo slope), compared bit for bit:
        // bit NL * side + layer of zvar (dvar); those read z (the slope) from
        // HBM and take the general paths below.
        constexpr int SU = NL * NW / WAVE;
        constexpr int SC = SU > 6 ? 6 : SU;   // rounds per chunk of loads in flight
        // One window per layer in an event whose buckets each share one z
        // and one stereo slope: x only, each lane's window bounds taken from
        // the lane that holds them.
        if (NS == 1 && uni) {
#pragma unroll
          for (int u0 = 0; u0 < SU; u0 += SC) {
            float sx[SC];
            uint32_t smask = 0;
#pragma unroll
            for (int v = 0; v < SC; ++v) {
                const int it = lane + WAVE * (u0 + v), l = it / NW, j = it - NW * (it / NW);
                const int f = __shfl(wf[0], l), n = __shfl(wl[0], l);
                sx[v] = 0.0f;
                if (j < n) {
                    sx[v] = ld32(B.hx, ebase + (uint32_t)(f + j));
                    smask |= 1u << v;
                }
            }
#pragma unroll
            for (int v = 0; v < SC; ++v) {
                const int it = lane + WAVE * (u0 + v), l = it / NW, j = it - NW * (it / NW);
                if ((smask >> v) & 1u) L.wx[0][l][j] = sx[v];
            }
          }
        }
#pragma unroll
        for (int sd = 0; sd < ((NS == 1 && uni) ? 0 : NS); ++sd) {
#pragma unroll
          for (int u0 = 0; u0 < SU; u0 += SC) {
            float sx[SU], sz[SU], sd_[SU];
            uint32_t smask = 0;
#pragma unroll
            for (int u = u0; u < u0 + SC; ++u) {
                const int it = lane + WAVE * u, l = it / NW, j = it - NW * (it / NW);
                const int la = WAVE * u / NW, lb = (WAVE * u + WAVE - 1) / NW;
                const int fa = __builtin_amdgcn_readlane(wf[sd], la), fb = __builtin_amdgcn_readlane(wf[sd], lb);
                const int na = __builtin_amdgcn_readlane(wl[sd], la), nb = __builtin_amdgcn_readlane(wl[sd], lb);
                const int f = l == la ? fa : fb;
                const int n = l == la ? na : nb;
                sx[u] = sz[u] = sd_[u] = 0.0f;
                if (j < n) {
                    const uint32_t g = ebase + (uint32_t)(f + j);
                    sx[u] = ld32(B.hx, g);
                    if (!uni) {
                        sz[u] = ld32(B.hz, g);
                        if (is_uv(l)) sd_[u] = ld32(B.hd, g);
                    }
                    smask |= 1u << u;
                }
            }
#pragma unroll
            for (int u = u0; u < u0 + SC; ++u) {
                const int it = lane + WAVE * u, l = it / NW, j = it - NW * (it / NW);
                const int la = WAVE * u / NW, lb = (WAVE * u + WAVE - 1) / NW;
                const bool in = (smask >> u) & 1u;
                if (in) {
                    L.wx[sd][l][j] = sx[u];
                    if (!uni && (!XO || j == 0)) {
                        L.wz[sd][l][XO ? 0 : j] = sz[u];
                        if (is_uv(l)) L.wd[sd][uv_index(l)][XO ? 0 : j] = sd_[u];
                    }
                }
                // (the two-window build still runs these tests, on zeros that
                // set no bit: skipping them there trips an instruction-selection
                // error of the compiler)
                if (NS == 1 && uni) continue;
                // slot 0 of layer la sits in lane la NW - 64 u, that of lb in lane lb NW - 64 u
                const float za = bcast_f(sz[u], la * NW - WAVE * u), zb = bcast_f(sz[u], lb * NW - WAVE * u);
                const float da = bcast_f(sd_[u], la * NW - WAVE * u), db = bcast_f(sd_[u], lb * NW - WAVE * u);
                const bool zd = in && __float_as_uint(sz[u]) != __float_as_uint(l == la ? za : zb);
                const bool dd = in && __float_as_uint(sd_[u]) != __float_as_uint(l == la ? da : db);
                if (__ballot(zd && l == la)) zvar |= 1u << (NL * sd + la);
                if (__ballot(zd && l == lb)) zvar |= 1u << (NL * sd + lb);
                if (is_uv(la) && __ballot(dd && l == la)) dvar |= 1u << (NL * sd + la);
                if (is_uv(lb) && __ballot(dd && l == lb)) dvar |= 1u << (NL * sd + lb);
            }
          }
        }
        wave_sync();
        if constexpr (CNT) {
            for (int sd = 0; sd < NS; ++sd) {
                for (int l = 0; l < NL; ++l) cnt[C_STAGED] += (uint32_t)L.wlen[sd][l];
                cnt[C_PAIRS_ALL] += (uint32_t)(L.wlen[sd][0] * L.wlen[sd][8] + L.wlen[sd][3] * L.wlen[sd][11]);
            }
        }

        mark(C_CY_STAGE);
        // ---- doublets of both seed sets, filtered, queued; triplets by passes ----
        nL = 0;
        const float tolc = P->magtol_const + P->magtol_pscale / p;
        const bool low_p = NS == 1 && p < P->p_charge_cut;   // no bend-direction filter without q/p
        constexpr bool seed16 = H16;
        if constexpr (H16) {
            // binary16 seeding: coordinates relative to the window centres,
            // constants rounded once from binary32
            auto pack2 = [](float lo, float hi) {
                const half2v v = {(_Float16)lo, (_Float16)hi};
                return (uint32_t)__builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v));
            };
            kTXQP = pack2(tx_in, qop);
            kTXSTC = pack2(P->magtol_txscale, tolc);
            kTMINMAX = pack2(P->magtol_min, P->magtol_max);
            hTMAX = (_Float16)P->magtol_max;
            hT3 = (_Float16)P->T_triplet;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int l0 = s ? 3 : 0, l1 = s ? 7 : 4, l2 = s ? 11 : 8;
                const float K = s ? P->K_last : P->K_first;
                const float c0 = bcast_f(xcl, 3 * l0 + 1), c1 = bcast_f(xcl, 3 * l1 + 1), c2 = bcast_f(xcl, 3 * l2 + 1);
                hon[s] = L.wlen[0][l0] > 0 && L.wlen[0][l2] > 0 && !(((zvar >> l0) | (zvar >> l2)) & 1u);
                const float zw0 = L.wz[0][l0][0], zw2 = L.wz[0][l2][0];
                hc0[s] = c0;
                hc1[s] = c1;
                hc2[s] = c2;
                hRZ[s] = (_Float16)(1.0f / (zw2 - zw0));
                hC02[s] = (_Float16)(c2 - c0);
                hE0[s] = (_Float16)(c0 - x_mag);
                hL0[s] = (_Float16)(P->z_mag - zw0);
                hA[s] = (_Float16)(P->z[l1] - zw0 * K);
                hKK[s] = (_Float16)K;
                hB[s] = (_Float16)(c0 * K - c1);
            }
        }
        int qn = 0;
        // One item per (side, set, h0).  Each item gets the range of h2 in its third
        // window that can pass the magnet filter: a passing slope t satisfies
        // |x0 - x_mag + (z_mag - z0) t| < tol(t) <= tolb, so t lies within
        // tolb/|z_mag - z0| of t_c = (x_mag - x0) / (z_mag - z0), and
        // x2 = x0 + t (z2 - z0), with z2 the window's one z or, where its hits
        // differ in z, anywhere in their range (the extremes of x2 are then at
        // the corners of the t and z2 intervals).  The x2 interval is widened
        // by 0.5 mm + 1e-5 relative, orders of magnitude above the rounding
        // of the filter itself and of the approximate reciprocal used for the
        // bracket, and every pair in it is tested with the exact filter
        // below; pairs outside cannot pass.  A degenerate lever arm, or (in
        // builds that stage x only) a window whose hits differ in z, tests
        // every pair.
        // items in (side, set) order: group g = 2 side + set starts at c[g]
        const int c1 = L.wlen[0][0], c2 = c1 + L.wlen[0][3];
        const int c3 = NS > 1 ? c2 + L.wlen[NS - 1][0] : c2;
        const int items_total = NS > 1 ? c3 + L.wlen[NS - 1][3] : c2;
        if constexpr (CNT) cnt[C_ITEMS] = (uint32_t)items_total;
        // builds that stage z per hit (one side): the z range of each third
        // window, its one z or, where its hits differ in z, the min and max
        // over them (wave-wide); ranged: some third window of the track is
        // of the second kind (a wave-uniform choice of bracket form)
        float z2lo[2] = {0.0f, 0.0f}, z2hi[2] = {0.0f, 0.0f};
        const bool ranged = !WaveLds<NW, NS>::XO && ((zvar >> 8) & 1u || (zvar >> 11) & 1u);
        if constexpr (!WaveLds<NW, NS>::XO) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int l2 = s ? 11 : 8;
                z2lo[s] = z2hi[s] = L.wz[0][l2][0];
                if ((zvar >> l2) & 1u) {
                    const int n2 = L.wlen[0][l2];
                    const float z = lane < n2 ? L.wz[0][l2][lane < NW ? lane : 0] : 0.0f;
                    float lo = lane < n2 ? z : INFINITY, hi = lane < n2 ? z : -INFINITY;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) {
                        lo = fminf(lo, __shfl_xor(lo, off));
                        hi = fmaxf(hi, __shfl_xor(hi, off));
                    }
                    z2lo[s] = bcast_f(lo, 0);
                    z2hi[s] = bcast_f(hi, 0);
                }
            }
        }
        const float mag_z = P->z_mag, mag_txs = P->magtol_txscale, mag_min = P->magtol_min,
                    mag_max = P->magtol_max;
        for (int base = 0; base < items_total; base += WAVE) {
            const int item = base + lane;
            const int grp = item < c1 ? 0 : (item < c2 ? 1 : (item < c3 ? 2 : 3));
            const int sd = NS > 1 ? grp >> 1 : 0, s = grp & 1;
            const int i0 = item - (grp == 0 ? 0 : (grp == 1 ? c1 : (grp == 2 ? c2 : c3)));
            const int l0 = s ? 3 : 0, l2 = s ? 11 : 8;
            const int n2 = L.wlen[sd][l2];
            int jlo = 0, jhi = 0;
            float x0 = 0.0f, z0 = 0.0f;
            if (item < items_total) {
                x0 = L.wx[sd][l0][i0];
                z0 = zat(sd, l0, i0);
                jhi = n2;
                // the third window's z range: one value, or (builds that stage
                // z per hit) the range of its hits' z
                const bool mix2 = (zvar >> (NL * sd + l2)) & 1u, mix0 = (zvar >> (NL * sd + l0)) & 1u;
                if (n2 > 0 && (!WaveLds<NW, NS>::XO || !(mix0 || mix2))) {
                    const float lev = P->z_mag - z0;
                    const float dzl = (WaveLds<NW, NS>::XO ? L.wz[sd][l2][0] : sel(z2lo, s)) - z0;
                    const float dzh = (WaveLds<NW, NS>::XO ? L.wz[sd][l2][0] : sel(z2hi, s)) - z0;
                    if (fabsf(lev) > 1.0f && (dzl > 1.0f || dzh < -1.0f)) {
                        const float rl = __builtin_amdgcn_rcpf(lev);   // within 1 ulp: the bracket is padded
                        const float arl = fabsf(rl);
                        const float tc = (x_mag - x0) * rl;
                        const float dt0 = P->magtol_max * arl;
                        float tolb = tolc + (P->magtol_txscale > 0.0f ? P->magtol_txscale : 0.0f) *
                                                (fabsf(tc) + dt0);
                        if (tolb < P->magtol_min) tolb = P->magtol_min;
                        if (tolb > P->magtol_max) tolb = P->magtol_max;
                        const float dt = tolb * arl;
                        // x2 = x0 + t dz over t in [tc - dt, tc + dt] and dz in
                        // [dzl, dzh] (one value when the window shares one z)
                        float e1, e2;
                        if (ranged) {   // corners; exact also where dzl = dzh
                            const float c1 = (tc - dt) * dzl, c2 = (tc - dt) * dzh;
                            const float c3 = (tc + dt) * dzl, c4 = (tc + dt) * dzh;
                            e1 = x0 + fminf(fminf(c1, c2), fminf(c3, c4));
                            e2 = x0 + fmaxf(fmaxf(c1, c2), fmaxf(c3, c4));
                        } else {   // dzl = dzh
                            const float a1 = x0 + (tc - dt) * dzl, a2 = x0 + (tc + dt) * dzl;
                            e1 = a1 < a2 ? a1 : a2;
                            e2 = a1 < a2 ? a2 : a1;
                        }
                        const float margin = 0.5f + 1e-5f * (fabsf(e1) + fabsf(e2));
                        const float xlo = e1 - margin;
                        const float xhi = e2 + margin;
                        if (fabsf(xlo) < 1e30f && fabsf(xhi) < 1e30f) {
                            bounds_sorted<NW>(L.wx[sd][l2], n2, xlo, xhi, jlo, jhi);
                        }
                    }
                }
            }
            // binary16 sets: the pairs whose |M| is below the largest
            // tolerance.  M(h2) = (E0 + X0) + ((X2 - X0) + C02) RZ L0 is
            // monotone in x2 (every rounding step is), so they form one index
            // range of the sorted window, found by searches with the same
            // binary16 arithmetic; every passing pair lies in it.
            const bool h16 = seed16 && item < items_total && sel(hon, s);
            if (h16) {
                jlo = 0;
                jhi = n2;
                const _Float16 RZ = sel(hRZ, s), L0 = sel(hL0, s), C02 = sel(hC02, s);
                const _Float16 m1 = sel(hE0, s) + (_Float16)(x0 - sel(hc0, s));
                const _Float16 X0 = (_Float16)(x0 - sel(hc0, s));
                const float c2 = sel(hc2, s);
                const float *wx2 = L.wx[0][l2];
                const _Float16 lim = hTMAX, nlim = -hTMAX;
                auto M = [&](int j) {
                    const _Float16 X2 = (_Float16)(wx2[j] - c2);
                    const _Float16 u = X2 - X0;
                    const _Float16 v = u + C02;
                    const _Float16 t = v * RZ;
                    const _Float16 m2 = t * L0;
                    return m1 + m2;
                };
                const float rzl = (float)RZ * (float)L0;
                if (rzl > 0.0f && rzl < INFINITY) {          // M non-decreasing in x2
                    prefix2<NW>(n2, [&](int j) { return M(j) <= nlim; }, [&](int j) { return M(j) < lim; }, jlo, jhi);
                } else if (rzl < 0.0f && rzl > -INFINITY) {  // M non-increasing in x2
                    prefix2<NW>(n2, [&](int j) { return M(j) >= lim; }, [&](int j) { return M(j) > nlim; }, jlo, jhi);
                }
                if (jhi < jlo) jhi = jlo;
            }
            // the pair loop runs while any lane has pairs left (the two-window
            // build takes the wave's largest span first, which keeps its
            // register count within its occupancy bound)
            int span = jhi - jlo;
            if constexpr (NS == 2) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const int o = __shfl_xor(span, off);
                    span = o > span ? o : span;
                }
            }
            auto more = [&](int k) { return NS == 2 ? k < span : __ballot(k < span) != 0; };
            // the binary32 filter of pair (i0, i2)
            const float dzm = mag_z - z0;
            auto test32 = [&](int i2) {
                const float x2 = L.wx[sd][l2][i2], z2 = zat(sd, l2, i2);
                const float txd = (x2 - x0) / (z2 - z0);
                bool pass = !(low_p && !((txd - tx_in) * qop > 0.0f));
                const float xm = x0 + txd * dzm;
                float tol = tolc + mag_txs * fabsf(txd);
                if (tol < mag_min) tol = mag_min;
                if (tol > mag_max) tol = mag_max;
                if (!(fabsf(xm - x_mag) < tol)) pass = false;
                return pass;
            };
            // queue the passing pairs of this lane-step; a full queue is completed
            auto push = [&](bool pass, bool tested, int i2) {
                const uint64_t bal = __ballot(pass);
                if constexpr (CNT) {
                    cnt[C_PAIRS_TESTED] += (uint32_t)__popcll(__ballot(tested));
                    cnt[C_DOUBLETS] += (uint32_t)__popcll(bal);
                }
                if (pass) {
                    const int at = qn + lanes_below(bal);
                    L.qkey[at] = ((uint32_t)sd << 17) | ((uint32_t)s << 16) | ((uint32_t)i0 << 8) | (uint32_t)i2;
                }
                qn += __popcll(bal);
                if (qn >= WAVE) {
                    wave_sync();
                    flush(WAVE);
                    const int rest = qn - WAVE;
                    uint32_t k2 = 0;
                    if (lane < rest) k2 = L.qkey[WAVE + lane];
                    wave_sync();
                    if (lane < rest) L.qkey[lane] = k2;
                    qn = rest;
                    wave_sync();
                }
            };
            if constexpr (!H16) {
                for (int k = 0; more(k); ++k) {
                    const int i2 = jlo + k;
                    const bool tested = i2 < jhi;
                    // every lane evaluates the filter, without a branch (a
                    // divergent one issues the same instructions and adds the
                    // exec-mask bookkeeping); a lane without a pair reads its
                    // window's slot 0 and drops the result
                    const bool pass = test32(tested ? i2 : 0);
                    push(tested && pass, tested, i2);
                }
            } else {
                // two pairs (i2, i2 + 1) per step: one packed binary16
                // evaluation, or two binary32 ones on sets that stay binary32
                const int s_ = s;
                const _Float16 X0 = h16 ? (_Float16)(x0 - sel(hc0, s_)) : (_Float16)0.0f;
                const half2v TXQP = __builtin_bit_cast(half2v, kTXQP), TXSTC = __builtin_bit_cast(half2v, kTXSTC);
                const half2v MM = __builtin_bit_cast(half2v, kTMINMAX);
                const half2v TX = TXQP.xx, QP = TXQP.yy, TXS = TXSTC.xx, TC = TXSTC.yy;
                const _Float16 tmin = MM.x, tmax = MM.y;
                for (int k = 0; more(k); k += 2) {
                    const int ia = jlo + k, ib = ia + 1;
                    const bool ta = ia < jhi, tb = ib < jhi;
                    bool pa = false, pb = false;
                    if (h16) {
                        const float c2 = sel(hc2, s_);
                        const int ja = ta ? ia : 0, jb = tb ? ib : 0;
                        const half2v X2 = {(_Float16)(L.wx[0][l2][ja] - c2), (_Float16)(L.wx[0][l2][jb] - c2)};
                        const half2v X0v = {X0, X0};
                        const half2v C02 = {sel(hC02, s_), sel(hC02, s_)}, RZ = {sel(hRZ, s_), sel(hRZ, s_)};
                        const half2v u = X2 - X0v;
                        const half2v v = u + C02;
                        const half2v t = v * RZ;
                        bool ca = true, cb = true;
                        if (low_p) {
                            const half2v w1 = t - TX;
                            const half2v w2 = w1 * QP;
                            ca = w2.x > (_Float16)0.0f;
                            cb = w2.y > (_Float16)0.0f;
                        }
                        const half2v E0 = {sel(hE0, s_), sel(hE0, s_)}, L0 = {sel(hL0, s_), sel(hL0, s_)};
                        const half2v m1 = E0 + X0v;
                        const half2v m2 = t * L0;
                        const half2v M = m1 + m2;
                        const half2v at = {habs(t.x), habs(t.y)};
                        const half2v r1 = TXS * at;
                        const half2v tol = TC + r1;
                        _Float16 tola = tol.x, tolb = tol.y;
                        if (tola < tmin) tola = tmin;
                        if (tola > tmax) tola = tmax;
                        if (tolb < tmin) tolb = tmin;
                        if (tolb > tmax) tolb = tmax;
                        pa = ta && ca && habs(M.x) < tola;
                        pb = tb && cb && habs(M.y) < tolb;
                    } else {
                        pa = ta && test32(ia);
                        pb = tb && test32(ib);
                    }
                    push(pa, ta, ia);
                    push(pb, tb, ib);
                }
            }
        }
        if (qn > 0) {
            wave_sync();
            flush(qn);
        }

        const size_t o12 = (size_t)t * NL;
        if constexpr (CNT) cnt[C_KEPT] = (uint32_t)nL;
        if (nL == 0) {
            write_none(t, o12);
            return;
        }

        mark(C_CY_DOUBLETS);
        // ---- triplet x(z) models ----
        if (lane < nL) {
            const uint32_t lo = (uint32_t)L.tk[lane];
            const int sd = NS > 1 ? (int)((lo >> 13) & 1u) : 0;
            const int s = (int)((lo >> 12) & 1u), i0 = (int)((lo >> 6) & 63u), i2 = (int)(lo & 63u);
            const int i1 = L.th1[lane];
            const int l0 = s ? 3 : 0, l1 = s ? 7 : 4, l2 = s ? 11 : 8;
            const float u0 = zat(sd, l0, i0) - P->z_ref, u1 = zat(sd, l1, i1) - P->z_ref,
                        u2 = zat(sd, l2, i2) - P->z_ref;
            const float X0 = L.wx[sd][l0][i0], X1 = L.wx[sd][l1][i1], X2 = L.wx[sd][l2][i2];
            const float g0 = g_of(u0, dR), g1 = g_of(u1, dR), g2 = g_of(u2, dR);
            const float s01 = (X1 - X0) / (u1 - u0);
            const float s12 = (X2 - X1) / (u2 - u1);
            const float G01 = (g1 - g0) / (u1 - u0);
            const float G12 = (g2 - g1) / (u2 - u1);
            const float c = (s12 - s01) / (G12 - G01);
            const float b = s01 - c * G01;
            const float a = X0 - b * u0 - c * g0;
            L.ca[lane] = a;
            L.cb[lane] = b;
            L.cc[lane] = c;
#pragma unroll
            for (int l = 0; l < NL; ++l) L.ch[lane][l] = -1;
            L.ch[lane][l0] = (int8_t)i0;
            L.ch[lane][l1] = (int8_t)i1;
            L.ch[lane][l2] = (int8_t)i2;
        }
        wave_sync();

        mark(C_CY_MODEL);
        // ---- extension: lanes = (candidate, missing layer) ----
        const float T_uv0 = P->T_uv_scale * (fabsf(tx_in) + fabsf(ty_in));
        const float T_uv = T_uv0 < P->T_uv_floor ? P->T_uv_floor : T_uv0;
        // item it = (candidate it / 9, slot it % 9): the layer, the model's
        // prediction there and the search values
        struct Ext {
            int r, l, n, sd;
            bool uv, scan;
            float xe, yp, wd1;
            uint32_t gb;    // batch index of the window's first hit
            const float *wx, *wdv;
        };
        auto ext_item = [&](int it) {
            Ext e;
            e.r = it / NSLOT;
            const int slot = it - NSLOT * (it / NSLOT);
            const uint32_t kr = (uint32_t)L.tk[e.r];
            const int s = (int)((kr >> 12) & 1u);
            e.sd = NS > 1 ? (int)((kr >> 13) & 1u) : 0;
            if (slot < 3) e.l = s ? 4 * slot : 4 * slot + 3;
            else e.l = 4 * ((slot - 3) >> 1) + 1 + ((slot - 3) & 1);
            const float zl = L.gz[e.l];
            const float u = zl - P->z_ref;
            e.xe = L.ca[e.r] + L.cb[e.r] * u + L.cc[e.r] * g_of(u, dR);
            e.n = L.wlen[e.sd][e.l];
            e.wx = L.wx[e.sd][e.l];
            // one search for x and u/v slots alike: a u/v hit's x at y = 0 is
            // moved along its fibre to the predicted y; an x hit adds +-0, which
            // changes no distance and no comparison.  With a common stereo slope
            // in the window the values stay sorted.
            e.uv = slot >= 3;
            e.yp = e.uv ? y_in + ty_in * (zl - P->z_in) : 0.0f;
            e.scan = e.uv && ((dvar >> (NL * e.sd + e.l)) & 1u);
            e.wd1 = e.uv ? L.wd[e.sd][uv_index(e.l)][0] : 0.0f;
            e.wdv = L.wd[e.sd][e.uv ? uv_index(e.l) : 0];
            e.gb = ebase + (uint32_t)L.wfirst[e.sd][e.l];
            return e;
        };
        // sorted searches: the window's one tangent (0 for x slots, where it
        // adds +-0); scans (stereo windows whose tangents differ): per hit
        auto ext_val = [](const Ext &e) {
            const float *wx = e.wx;
            const float yp = e.yp, wd1 = e.wd1;
            return [wx, yp, wd1](int j) { return wx[j] + wd1 * yp; };
        };
        const float *hd = B.hd;
        auto ext_scan = [hd](const Ext &e) {
            const float *wx = e.wx, *wdv = e.wdv;
            const float yp = e.yp;
            const uint32_t gb = e.gb;
            return [wx, wdv, yp, gb, hd](int j) {
                return wx[j] + (XO ? ld32(hd, gb + (uint32_t)j) : wdv[j]) * yp;
            };
        };
        auto ext_keep = [&](const Ext &e, int best, float bd) {
            if (best >= 0 && bd * bd < (e.uv ? T_uv : P->T_x)) L.ch[e.r][e.l] = (int8_t)best;
        };
        const int n_items = nL * NSLOT;
        if (n_items <= WAVE) {
            if (lane < n_items) {
                const Ext e = ext_item(lane);
                float bd = INFINITY;
                const int best = e.scan ? closest_scan(ext_scan(e), e.n, e.xe, bd)
                                        : closest_sorted<NW>(ext_val(e), e.n, e.xe, bd);
                ext_keep(e, best, bd);
            }
        } else {
            // two items per lane, their searches interleaved
            for (int it = lane; it < n_items; it += 2 * WAVE) {
                const bool hb = it + WAVE < n_items;
                const Ext ea = ext_item(it);
                const Ext eb = ext_item(hb ? it + WAVE : it);
                float da = INFINITY, db = INFINITY;
                int ba, bb;
                if (!ea.scan && !eb.scan) {
                    closest_sorted2<NW>(ext_val(ea), ea.n, ea.xe, ba, da, ext_val(eb), eb.n, eb.xe, bb, db);
                } else {
                    ba = ea.scan ? closest_scan(ext_scan(ea), ea.n, ea.xe, da)
                                 : closest_sorted<NW>(ext_val(ea), ea.n, ea.xe, da);
                    bb = eb.scan ? closest_scan(ext_scan(eb), eb.n, eb.xe, db)
                                 : closest_sorted<NW>(ext_val(eb), eb.n, eb.xe, db);
                }
                ext_keep(ea, ba, da);
                if (hb) ext_keep(eb, bb, db);
            }
        }
        wave_sync();

        mark(C_CY_EXTEND);
        // ---- fits and quality: 16 lanes per candidate, 4 candidates per pass ----
        // Lane (g, j) = (lane / 16, lane % 16) holds layer j of the g-th
        // candidate of the pass.  Every fit sum is the serial sum over the
        // candidate's hits in ascending layer order (absent layers add +0,
        // which leaves a running sum that started at +0 unchanged), formed by
        // a DPP chain over the row whose result sits in lane 11; the solves
        // run in every lane, the ones of lane 11 are broadcast over the row
        // where the per-hit residuals need them, and lane 11 decides.
        uint64_t fitm = 0;   // candidates passing the candidate rule, in rank order
        {
            bool rule = false;
            if (lane < nL) {
                // a layer's byte is a hit index (sign bit clear) or -1; word st
                // holds station st, its stereo layers in bytes 1 and 2
                int n = 0;
                bool st_ok = true;
#pragma unroll
                for (int st = 0; st < 3; ++st) {
                    const uint32_t pres = ~L.chw[lane][st] & 0x80808080u;
                    n += __popc(pres);
                    st_ok = st_ok && (pres & 0x00808000u) != 0u;
                }
                rule = n >= 9 && st_ok;
            }
            fitm = __ballot(rule);
        }
        if constexpr (CNT) cnt[C_FITTED] = (uint32_t)__popcll(fitm);
        int best_r = -1, best_n = 0;
        float best_Q = 0.0f, bfa = 0.0f, bfb = 0.0f, bfc = 0.0f, bfy0 = 0.0f, bfty = 0.0f;
        const int g = lane >> 4, j = lane & 15;
        const bool uvj = j < NL && is_uv(j);
        const float Tj = uvj ? T_uv : P->T_x;
        constexpr int LR = NL - 1;   // the row lane that holds the chained sums
        // a uniform event: layer j's common z and stereo slope, read once (the
        // sums then use their LDS rows as scratch)
        float zj = 0.0f, dj = 1.0f;
        if constexpr (!WaveLds<NW, NS>::XO) {
            if (uni && j < NL) {
                zj = L.wz[0][j][0];
                if (uvj) dj = L.wd[0][uv_index(j)][0];
            }
        }
        const bool zreg = !WaveLds<NW, NS>::XO && uni;
        while (fitm) {
            int r = -1;
            int rq[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rq[k] = fitm ? (int)__builtin_ctzll(fitm) : -1;
                if (fitm) fitm &= fitm - 1;
                if (k == g) r = rq[k];
            }
            int hit = -1;
            if (r >= 0 && j < NL) hit = L.ch[r][j];
            const bool pres = hit >= 0;
            const bool pres_uv = pres && uvj;
            float a = 0.0f, b = 0.0f, c = 0.0f;
            int sd = 0;
            if (r >= 0) {
                a = L.ca[r]; b = L.cb[r]; c = L.cc[r];
                if constexpr (NS > 1) sd = (int)(((uint32_t)L.tk[r] >> 13) & 1u);
            }
            float sv = 0.0f, h = 0.0f, rr = 0.0f, dxy = 1.0f;
            if (pres) {
                const float zh = zreg ? zj : zat(sd, j, hit);
                const float u = zh - P->z_ref;
                float xm;
                if (uvj) {
                    dxy = zreg ? dj : dat(sd, j, hit);
                    const float yv = y_in + ty_in * (zh - P->z_in);
                    xm = L.wx[sd][j][hit] + dxy * yv;
                } else {
                    xm = L.wx[sd][j][hit];
                }
                sv = u * INV1024;
                h = sv * sv * (1.0f + dR * u);
                rr = xm - (a + b * u + c * g_of(u, dR));
            }
            // hit counts: integers, the same in any order
            const uint32_t row_bits = 16u * (uint32_t)g;
            const int n = __popc((uint32_t)(__ballot(pres) >> row_bits) & 0xFFFFu);
            const int n_uv = __popc((uint32_t)(__ballot(pres_uv) >> row_bits) & 0xFFFFu);
            const float S0 = (float)n, YS0 = (float)n_uv;
            // x normal equations, and the slot sums of the y line
            const float t1[10] = {sv, h, sv * sv, sv * h, h * h, rr, sv * rr, h * rr,
                                  pres_uv ? sv : 0.0f, pres_uv ? sv * sv : 0.0f};
            float s1[10];
            row_sums(t1, s1, g, j);
            const float S1 = s1[0], S2 = s1[1], S11 = s1[2], S12 = s1[3], S22 = s1[4];
            const float R0 = s1[5], R1 = s1[6], R2 = s1[7], YS1 = s1[8], YS11 = s1[9];
            const float m00 = S11 * S22 - S12 * S12;
            const float m01 = S1 * S22 - S12 * S2;
            const float m02 = S1 * S12 - S11 * S2;
            const float det = S0 * m00 - S1 * m01 + S2 * m02;
            const bool ok_x = fabsf(det) > 0.0f;
            const float det_s = ok_x ? det : 1.0f;
            // the sums are the same in every lane of the row: lanes 0, 1 and 2
            // divide the numerators of da, db and dc, and the row takes each
            const float num_x = j == 0 ? R0 * m00 - S1 * (R1 * S22 - S12 * R2) + S2 * (R1 * S12 - S11 * R2)
                              : j == 1 ? S0 * (R1 * S22 - S12 * R2) - R0 * m01 + S2 * (S1 * R2 - R1 * S2)
                                       : S0 * (S11 * R2 - R1 * S12) - S1 * (S1 * R2 - R1 * S2) + R0 * m02;
            const float q_x = num_x / det_s;
            const float da = row_bcast_lane(q_x, 0), db = row_bcast_lane(q_x, 1), dc = row_bcast_lane(q_x, 2);
            const float res = pres ? rr - (da + db * sv + dc * h) : 0.0f;
            const float eta = pres_uv ? -res / dxy : 0.0f;
            // Q_x, and the y line's residual sums
            const float t2[3] = {pres ? res * res / Tj : 0.0f, eta, pres_uv ? sv * eta : 0.0f};
            float s2[3];
            row_sums(t2, s2, g, j);
            const float Qx = s2[0], Y0 = s2[1], Y1 = s2[2];
            const float D = YS0 * YS11 - YS1 * YS1;
            const bool ok_y = fabsf(D) > 0.0f;
            const float D_s = ok_y ? D : 1.0f;
            const float q_y = (j == 0 ? Y0 * YS11 - YS1 * Y1 : YS0 * Y1 - YS1 * Y0) / D_s;   // lanes 0, 1: dy0, dty
            const float dy0 = row_bcast_lane(q_y, 0), dty = row_bcast_lane(q_y, 1);
            const float dslope = dty * INV1024;
            const float ry = pres_uv ? eta - (dy0 + dty * sv) : 0.0f;
            const float t3[1] = {pres_uv ? ry * ry / P->T_y : 0.0f};
            float s3[1];
            chain12(t3, s3);   // Q_y in lane 11
            // lane 10 divides Q_x, lane 11 Q_y; lane 11 adds the two
            const float q_q = j == LR - 1 ? Qx / (float)(n - 3) : s3[0] / (float)(n_uv - 2);
            const float Q = (dpp<0x111, true>(q_q) + q_q) * P->C_nhits[n - 9 < 0 ? 0 : (n - 9 > 3 ? 3 : n - 9)];
            const bool acc = r >= 0 && ok_x && ok_y && fabsf(dslope) < P->T_ty && Q < P->T_Q;
            // candidates of this pass in rank order: the first strict minimum wins ties
            const uint64_t accm = __ballot(acc && j == LR);
            if constexpr (CNT) cnt[C_ACCEPTED] += (uint32_t)__popcll(accm);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!((accm >> (16 * k + LR)) & 1ull)) continue;
                const int src = 16 * k + LR;
                const float qk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Q), src));
                if (best_r >= 0 && !(qk < best_Q)) continue;
                best_r = rq[k];
                best_Q = qk;
                best_n = __builtin_amdgcn_readlane(n, src);
                bfa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a + da), src));
                bfb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b + db * INV1024), src));
                bfc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c + dc * INV1024SQ), src));
                bfy0 = __int_as_float(__builtin_amdgcn_readlane(
                    __float_as_int((y_in + ty_in * (P->z_ref - P->z_in)) + dy0), src));
                bfty = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ty_in + dslope), src));
            }
        }

        mark(C_CY_FIT);
        // ---- best candidate: output ----
        if constexpr (CNT) cnt[C_FOUND] = best_r >= 0 ? 1u : 0u;
        if (best_r < 0) {
            write_none(t, o12);
            return;
        }
        if (lane == 0) {
            const float uT = P->z_T - P->z_ref;
            const float txT = bfb + 2.0f * bfc * uT + 3.0f * bfc * dR * uT * uT;
            B.found[t] = 1;
            B.nhits[t] = (uint8_t)best_n;
            B.a[t] = bfa;
            B.b[t] = bfb;
            B.c[t] = bfc;
            B.y0[t] = bfy0;
            B.ty[t] = bfty;
            B.qop[t] = paper ? (kick_s(txT, bfty) - kick_s(tx_in, ty_in)) / field_F(fc, txT - tx_in)
                             : (txT - tx_in) / P->kick;
            B.Q[t] = best_Q;
        }
        if (lane < NL) {
            const int sd = NS > 1 ? (int)(((uint32_t)L.tk[best_r] >> 13) & 1u) : 0;
            const int h = L.ch[best_r][lane];
            B.hit_idx[o12 + lane] = h >= 0 ? L.wfirst[sd][lane] + h : -1;
        }
        mark(C_CY_SELECT);
    }

    __device__ void write_none(uint32_t t, size_t o12) {
        const int lane = ln;
        if (lane < NL) B.hit_idx[o12 + lane] = -1;
        if (lane == 0) {
            B.found[t] = 0;
            B.nhits[t] = 0;
            B.a[t] = 0.0f; B.b[t] = 0.0f; B.c[t] = 0.0f; B.y0[t] = 0.0f;
            B.ty[t] = 0.0f; B.qop[t] = 0.0f; B.Q[t] = 0.0f;
        }
    }
};

template <int NW, int NS, int WPB, bool H16 = false>
__global__ __launch_bounds__(WPB * WAVE) void k_plain(DevBatch B, const KParams *__restrict__ P, uint32_t ev) {
    __shared__ WaveLds<NW, NS> lds[WPB];
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const uint32_t t = B.trk_off[ev] + blockIdx.x * WPB + w;
    if (t >= B.trk_off[ev + 1]) return;
    Track<NW, NS, false, H16> tr{B, P, lds[w], 0, {}, 0};
    tr.run(t, ev, t);
}

// Blocks are dispatched to the 8 XCDs round-robin (block b -> XCD b % 8);
// the remap gives each XCD a contiguous run of tracks, so the tracks of an
// event share one L2 and its hits are fetched from HBM once per XCD.
constexpr uint32_t NXCD = 8;

// (two-window build: at most 80 VGPRs, 6 waves per SIMD; 32-slot binary16
// build: at most 64 VGPRs, 8 waves per SIMD, a few registers spilled)
template <int NW, int NS, int WPB, bool CNT = false, bool H16 = false>
__global__ __launch_bounds__(WPB * WAVE) __attribute__((amdgpu_waves_per_eu(NS == 2 ? 6 : (H16 && NW == 32 ? 8 : 1)))) void k_grid(
    DevBatch B, const KParams *__restrict__ P) {
    __shared__ WaveLds<NW, NS> lds[WPB];
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const uint32_t per = gridDim.x / NXCD;
    const uint32_t lb = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    const uint32_t t = lb * WPB + w;
    // result slot t; its input track t, or trk_map[t] when a map is given
    uint32_t tin = t;
    if (B.trk_map) {
        if (t >= B.n_map) return;
        tin = B.trk_map[t];
    } else if (t >= B.n_tracks) {
        return;
    }
    Track<NW, NS, CNT, H16> tr{B, P, lds[w], 0, {}, 0};
    tr.run(t, B.trk_ev[tin], tin);
    if constexpr (CNT) {
        if (lane_id() == 0)
            for (int k = 0; k < C_N; ++k) atomicAdd(&B.stats[k], (unsigned long long)tr.cnt[k]);
    }
}

// Persistent: QUEUE_N work queues, QUEUE_SUB per XCD.  XCD x owns a
// contiguous eighth of the tracks, cut into chunks of `items` tracks; chunk j
// belongs to the XCD's queue j % QUEUE_SUB, whose k-th claim is chunk
// k QUEUE_SUB + j % QUEUE_SUB, so the XCD's waves move through its eighth
// together (its events stay in its L2) while their atomics spread over
// QUEUE_SUB words: device-scope atomics on one word are applied one after
// another, and one word per XCD held one-track claims to ~8 per us.  A wave
// claims its next chunk before it runs the current one, so the claim's round
// trip overlaps the track's first loads.  A wave whose queue is drained reads
// every head in one vector load (two words per lane), moves to a queue with
// chunks left -- its own XCD's first -- and exits once all are drained.
// Heads sit QUEUE_STRIDE words apart; word QUEUE_STRIDE QUEUE_N counts exited
// waves, and the last wave out puts every word back to zero, so the next
// launch on the batch starts clean without a reset kernel (or a memset node
// in a captured graph).
static_assert(QUEUE_N == 2 * WAVE, "the drained-queue scan reads two heads per lane");
static_assert(QUEUE_N == NXCD * QUEUE_SUB, "QUEUE_SUB queues per XCD");

template <int NW, int NS, int WPB, bool H16 = false>
__global__ __launch_bounds__(WPB * WAVE) void k_persistent(DevBatch B, const KParams *__restrict__ P,
                                                            uint32_t items) {
    __shared__ WaveLds<NW, NS> lds[WPB];
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    uint32_t *q = B.counter;
    const uint32_t T = B.n_tracks;
    auto xlo = [&](uint32_t x) { return (uint32_t)(((uint64_t)T * x) / NXCD); };
    // chunks of queue i
    auto n_chunks = [&](uint32_t i) -> uint32_t {
        const uint32_t x = i / QUEUE_SUB, sub = i % QUEUE_SUB;
        const uint32_t cx = (xlo(x + 1) - xlo(x) + items - 1) / items;
        return cx > sub ? (cx - sub + QUEUE_SUB - 1) / QUEUE_SUB : 0u;
    };
    auto claim = [&](uint32_t i) -> uint32_t {   // lane 0 claims; the value lives in its VGPR
        uint32_t c = 0;
        if (opaque_lane_id() == 0) c = atomicAdd(&q[QUEUE_STRIDE * i], 1u);
        return c;
    };
    // home queue: this block's XCD, waves spread over its QUEUE_SUB queues
    uint32_t qi = (blockIdx.x % NXCD) * QUEUE_SUB + ((blockIdx.x / NXCD) * WPB + w) % QUEUE_SUB;
    uint32_t k = __builtin_amdgcn_readfirstlane(claim(qi));
    for (;;) {
        if (k >= n_chunks(qi)) {
            // drained: find a queue with chunks left
            const uint32_t lane = (uint32_t)opaque_lane_id();
            const uint32_t h0 = __hip_atomic_load(&q[QUEUE_STRIDE * lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t h1 = __hip_atomic_load(&q[QUEUE_STRIDE * (lane + WAVE)], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t m0 = __ballot(h0 < n_chunks(lane)), m1 = __ballot(h1 < n_chunks(lane + WAVE));
            const uint32_t xb = (qi / QUEUE_SUB) * QUEUE_SUB;   // own XCD's first queue
            const uint64_t own = (xb < WAVE ? m0 >> xb : m1 >> (xb - WAVE)) & ((1ull << QUEUE_SUB) - 1);
            if (own) qi = xb + (uint32_t)__builtin_ctzll(own);
            else if (m0) qi = (uint32_t)__builtin_ctzll(m0);
            else if (m1) qi = WAVE + (uint32_t)__builtin_ctzll(m1);
            else break;
            k = __builtin_amdgcn_readfirstlane(claim(qi));
            continue;
        }
        const uint32_t next = claim(qi);   // in flight while this chunk runs
        const uint32_t x = qi / QUEUE_SUB, lo = xlo(x), hi = xlo(x + 1);
        const uint32_t t0 = lo + (k * QUEUE_SUB + qi % QUEUE_SUB) * items;
        const uint32_t t1 = t0 + items < hi ? t0 + items : hi;
        for (uint32_t t = t0; t < t1; ++t) {
            // keep per-track loads inside the loop: hoisting them across tracks
            // costs ~30 VGPRs of loop-carried state and two waves per SIMD
            asm volatile("" ::: "memory");
            Track<NW, NS, false, H16> tr{B, P, lds[w], 0, {}, 0};
            tr.ln = opaque_lane_id();
            tr.run(t, B.trk_ev[t], t);
        }
        k = __builtin_amdgcn_readfirstlane(next);
    }
    const uint32_t waves = gridDim.x * WPB;
    const uint32_t lane = (uint32_t)opaque_lane_id();
    uint32_t last = 0;
    if (lane == 0) {
        __threadfence();  // this wave's claims are performed before it counts itself out
        last = atomicAdd(&q[QUEUE_STRIDE * QUEUE_N], 1u) == waves - 1u ? 1u : 0u;
    }
    if (__builtin_amdgcn_readfirstlane(last)) {
        __hip_atomic_store(&q[QUEUE_STRIDE * lane], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&q[QUEUE_STRIDE * (lane + WAVE)], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane == 0) __hip_atomic_store(&q[QUEUE_STRIDE * QUEUE_N], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Serving gather: block (k, c) copies chunk c of GATHER_CHUNKS of event k's
// hits and track states from its host blob into the batch.
constexpr uint32_t GATHER_CHUNKS = 8;

__global__ __launch_bounds__(256) void k_gather(const GatherDesc *__restrict__ desc, uint32_t n_events,
                                                 BatchIn out) {
    const uint32_t k = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const GatherDesc d = desc[k];
    const char *src = reinterpret_cast<const char *>(d.src);
    const uint32_t *loc = reinterpret_cast<const uint32_t *>(src);
    if (c == 0) {
        if (tid < 24) out.hit_off[24 * k + tid] = d.hit_base + loc[tid];
        if (tid == 24) out.trk_off[k] = d.trk_base;
        if (k + 1 == n_events) {
            if (tid == 25) out.hit_off[24 * n_events] = d.hit_base + d.n_hits;
            if (tid == 26) out.trk_off[n_events] = d.trk_base + d.n_tracks;
        }
    }
    const uint32_t H = d.n_hits, T = d.n_tracks;
    const float *sx = reinterpret_cast<const float *>(src + 100);
    const float *sz = sx + H, *sd = sz + H, *st = sd + H;
    const uint32_t h0 = (uint32_t)((uint64_t)H * c / GATHER_CHUNKS), h1 = (uint32_t)((uint64_t)H * (c + 1) / GATHER_CHUNKS);
    for (uint32_t i = h0 + tid; i < h1; i += 256) {
        const uint32_t g = d.hit_base + i;
        out.hx[g] = sx[i];
        out.hz[g] = sz[i];
        out.hd[g] = sd[i];
    }
    const uint32_t t0 = (uint32_t)((uint64_t)T * c / GATHER_CHUNKS), t1 = (uint32_t)((uint64_t)T * (c + 1) / GATHER_CHUNKS);
    for (uint32_t i = t0 + tid; i < t1; i += 256) {
        const uint32_t g = d.trk_base + i;
        out.tx[g] = st[i];
        out.ty[g] = st[T + i];
        out.ttx[g] = st[2 * T + i];
        out.tty[g] = st[3 * T + i];
        out.tqop[g] = st[4 * T + i];
        out.trk_ev[g] = k;
    }
}

// Slot i of a batch of pool events (evs[0..E), result slots [toff[e],
// toff[e+1]) for event e): map[i] = the pool track it reads.
__global__ void k_track_map(const uint32_t *__restrict__ evs, const uint32_t *__restrict__ toff, uint32_t n_events,
                            const uint32_t *__restrict__ pool_trk_off, uint32_t *__restrict__ map) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= toff[n_events]) return;
    // last batch event e with toff[e] <= i
    uint32_t lo = 0, n = n_events + 1;
    while (n > 0) {
        const uint32_t half = n >> 1;
        if (toff[lo + half] <= i) { lo += half + 1; n -= half + 1; } else { n = half; }
    }
    const uint32_t e = lo - 1;
    map[i] = pool_trk_off[evs[e]] + (i - toff[e]);
}

__global__ void k_track_event(const uint32_t *__restrict__ trk_off, uint32_t n_events, uint32_t n_tracks,
                              uint32_t *__restrict__ trk_ev) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tracks) return;
    // last event e with trk_off[e] <= t
    uint32_t lo = 0, n = n_events + 1;
    while (n > 0) {
        const uint32_t half = n >> 1;
        if (trk_off[lo + half] <= t) { lo += half + 1; n -= half + 1; } else { n = half; }
    }
    trk_ev[t] = lo - 1;
}

// One block per event: uni[e] = 1 when, in each of the event's 24 buckets,
// every hit has the z and the stereo tangent of the bucket's first hit (bit
// for bit).  Such events need only x staged per hit.  The event's hits are
// streamed once, each compared with its predecessor; a difference is allowed
// only where a bucket starts.
__global__ void __launch_bounds__(1024) k_event_uniform(const uint32_t *__restrict__ hit_off,
                                                        const float *__restrict__ hz,
                                                        const float *__restrict__ hd, uint8_t *__restrict__ uni) {
    __shared__ uint32_t off[2 * NL + 1];
    const uint32_t e = blockIdx.x;
    if (threadIdx.x <= 2 * NL) off[threadIdx.x] = hit_off[2 * NL * e + threadIdx.x];
    __syncthreads();
    const uint32_t f = off[0], n = off[2 * NL];
    int odd = 0;
    for (uint32_t i = f + 1 + threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t dz = __float_as_uint(hz[i]) ^ __float_as_uint(hz[i - 1]);
        const uint32_t dd = __float_as_uint(hd[i]) ^ __float_as_uint(hd[i - 1]);
        if ((dz | dd) == 0) continue;
        bool start = false;
        for (int k = 1; k < 2 * NL; ++k) start |= off[k] == i;
        odd |= !start;
    }
    odd = __syncthreads_or(odd);
    if (threadIdx.x == 0) uni[e] = odd ? 0 : 1;
}

template <int NW, int NS, int WPB, bool H16>
hipError_t launch_nw_wpb(const DevBatch &b, const KParams *P, int mode, const ExecCfg &cfg,
                         const uint32_t *trk_off_host, hipStream_t s) {
    const dim3 block(WPB * WAVE);
    if (mode == 0) {   // plain: one launch per event
        for (uint32_t e = 0; e < b.n_events; ++e) {
            const uint32_t nt = trk_off_host[e + 1] - trk_off_host[e];
            if (nt == 0) continue;
            hipLaunchKernelGGL((k_plain<NW, NS, WPB, H16>), dim3((nt + WPB - 1) / WPB), block, 0, s, b, P, e);
        }
    } else if (mode == 2) {   // persistent: resident waves, QUEUE_SUB work queues per XCD
        uint32_t grid = (uint32_t)(cfg.blocks_per_cu * cfg.n_cu);
        const uint32_t need = (b.n_tracks + WPB - 1) / WPB;
        if (grid > need) grid = need;
        if (grid == 0) grid = 1;
        hipLaunchKernelGGL((k_persistent<NW, NS, WPB, H16>), dim3(grid), block, 0, s, b, P,
                           (uint32_t)cfg.items_per_grab);
    } else {   // batched: one launch, one wavefront per track (or per mapped slot), XCD-ordered
        const uint32_t need = ((b.trk_map ? b.n_map : b.n_tracks) + WPB - 1) / WPB;
        const uint32_t grid = (need + NXCD - 1) / NXCD * NXCD;
        if (grid) hipLaunchKernelGGL((k_grid<NW, NS, WPB, false, H16>), dim3(grid), block, 0, s, b, P);
    }
    return hipGetLastError();
}

template <int NW, int NS, bool H16 = false>
hipError_t launch_nw(const DevBatch &b, const KParams *P, int mode, const ExecCfg &cfg,
                     const uint32_t *trk_off_host, hipStream_t s) {
    switch (cfg.waves_per_block) {
        case 1: return launch_nw_wpb<NW, NS, 1, H16>(b, P, mode, cfg, trk_off_host, s);
        case 2: return launch_nw_wpb<NW, NS, 2, H16>(b, P, mode, cfg, trk_off_host, s);
        default: return launch_nw_wpb<NW, NS, 4, H16>(b, P, mode, cfg, trk_off_host, s);
    }
}

// Digest of one event's results: FNV-1a (64-bit) over the 20 words of each
// track slot -- found | n_hits << 8, the 12 hit indices, the bits of a, b,
// c, y0, ty, q/p, Q -- then the sum over the event's tracks of
// splitmix64(h ^ (index * 0x9E3779B97F4A7C15)).  One block per event.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(WAVE) void k_digest(DevBatch B, const uint32_t *__restrict__ trk_off,
                                                  unsigned long long *__restrict__ out) {
    const uint32_t e = blockIdx.x;
    const uint32_t t0 = trk_off[e], t1 = trk_off[e + 1];
    unsigned long long acc = 0;
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += WAVE) {
        uint32_t w[20];
        w[0] = (uint32_t)B.found[t] | ((uint32_t)B.nhits[t] << 8);
        for (int l = 0; l < NL; ++l) w[1 + l] = (uint32_t)B.hit_idx[(size_t)t * NL + l];
        w[13] = __float_as_uint(B.a[t]); w[14] = __float_as_uint(B.b[t]); w[15] = __float_as_uint(B.c[t]);
        w[16] = __float_as_uint(B.y0[t]); w[17] = __float_as_uint(B.ty[t]); w[18] = __float_as_uint(B.qop[t]);
        w[19] = __float_as_uint(B.Q[t]);
        unsigned long long h = 0xCBF29CE484222325ull;
        for (int k = 0; k < 20; ++k) { h ^= w[k]; h *= 0x100000001B3ull; }
        acc += mix64(h ^ ((unsigned long long)(t - t0) * 0x9E3779B97F4A7C15ull));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (threadIdx.x == 0) out[e] = acc;
}

__global__ __launch_bounds__(256) void k_poison(DevBatch B) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B.n_tracks) return;
    B.found[t] = 0xFF;
    B.nhits[t] = 0xFF;
    for (int l = 0; l < NL; ++l) B.hit_idx[(size_t)t * NL + l] = -2;
    const float nan = __uint_as_float(0x7FC00000u);
    B.a[t] = nan; B.b[t] = nan; B.c[t] = nan; B.y0[t] = nan; B.ty[t] = nan; B.qop[t] = nan; B.Q[t] = nan;
}

}  // namespace

// Fixed scratch of the non-allocating entry point (layout: FIXED_* in
// lf_internal.h).  Host code never passes this name to a kernel: it holds
// the address fixed_scratch() looked up for the current device.
static __device__ __align__(256) uint8_t scratch[FIXED_BYTES];

hipError_t fixed_scratch(void **out) {
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void *addr[MAXDEV] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

namespace {
__global__ __launch_bounds__(256) void k_zero_words(uint32_t *__restrict__ p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
}  // namespace

hipError_t launch_zero_words(uint32_t *p, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_poison(const DevBatch &b, hipStream_t s) {
    if (b.n_tracks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_poison, dim3((b.n_tracks + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_digest(const DevBatch &b, const uint32_t *trk_off, uint32_t n_events, unsigned long long *out,
                         hipStream_t s) {
    if (n_events == 0) return hipSuccess;
    hipLaunchKernelGGL(k_digest, dim3(n_events), dim3(WAVE), 0, s, b, trk_off, out);
    return hipGetLastError();
}

hipError_t launch_count(const DevBatch &b, const KParams *P, int n_hits_window, int n_sides, hipStream_t s) {
    if (b.n_tracks == 0) return hipSuccess;
    const uint32_t need = (b.n_tracks + 1) / 2;
    const uint32_t grid = (need + NXCD - 1) / NXCD * NXCD;
    const dim3 g(grid), blk(2 * WAVE);
    if (n_sides == 2) {
        if (n_hits_window <= 32) hipLaunchKernelGGL((k_grid<32, 2, 2, true>), g, blk, 0, s, b, P);
        else hipLaunchKernelGGL((k_grid<64, 2, 2, true>), g, blk, 0, s, b, P);
    } else if (n_sides == 3) {
        if (n_hits_window <= 32) hipLaunchKernelGGL((k_grid<32, 1, 2, true, true>), g, blk, 0, s, b, P);
        else hipLaunchKernelGGL((k_grid<64, 1, 2, true, true>), g, blk, 0, s, b, P);
    } else {
        if (n_hits_window <= 32) hipLaunchKernelGGL((k_grid<32, 1, 2, true>), g, blk, 0, s, b, P);
        else hipLaunchKernelGGL((k_grid<64, 1, 2, true>), g, blk, 0, s, b, P);
    }
    return hipGetLastError();
}

hipError_t launch_gather(const GatherDesc *desc, uint32_t n_events, const BatchIn &out, hipStream_t s) {
    if (n_events == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(n_events, GATHER_CHUNKS), dim3(256), 0, s, desc, n_events, out);
    return hipGetLastError();
}

hipError_t launch_track_map(const uint32_t *evs, const uint32_t *toff, uint32_t n_events, uint32_t n_slots,
                            const uint32_t *pool_trk_off, uint32_t *map, hipStream_t s) {
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_track_map, dim3((n_slots + 255) / 256), dim3(256), 0, s, evs, toff, n_events, pool_trk_off,
                       map);
    return hipGetLastError();
}

hipError_t launch_track_event(const DevBatch &b, hipStream_t s) {
    if (b.n_tracks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_track_event, dim3((b.n_tracks + 255) / 256), dim3(256), 0, s, b.trk_off, b.n_events,
                       b.n_tracks, const_cast<uint32_t *>(b.trk_ev));
    return hipGetLastError();
}

hipError_t launch_event_uniform(const DevBatch &b, uint8_t *uni, hipStream_t s) {
    if (b.n_events == 0) return hipSuccess;
    hipLaunchKernelGGL(k_event_uniform, dim3(b.n_events), dim3(1024), 0, s, b.hit_off, b.hz, b.hd, uni);
    return hipGetLastError();
}

hipError_t launch_find(const DevBatch &b, const KParams *P, int n_hits_window, int n_sides, int mode,
                       const ExecCfg &cfg, const uint32_t *trk_off_host, hipStream_t s) {
    if (b.n_tracks == 0) return hipSuccess;
    if (n_sides == 2) {
        if (n_hits_window <= 32) return launch_nw<32, 2>(b, P, mode, cfg, trk_off_host, s);
        return launch_nw<64, 2>(b, P, mode, cfg, trk_off_host, s);
    }
    if (n_sides == 3) {
        if (n_hits_window <= 32) return launch_nw<32, 1, true>(b, P, mode, cfg, trk_off_host, s);
        return launch_nw<64, 1, true>(b, P, mode, cfg, trk_off_host, s);
    }
    if (n_hits_window <= 32) return launch_nw<32, 1>(b, P, mode, cfg, trk_off_host, s);
    return launch_nw<64, 1>(b, P, mode, cfg, trk_off_host, s);
}

namespace {
template <int NW, int NS, int WPB, bool H16>
int occ() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_persistent<NW, NS, WPB, H16>),
                                                     WPB * WAVE, 0) != hipSuccess)
        return 0;
    return n;
}
}  // namespace

template <int NW, int NS, bool H16 = false>
int occ_wpb(int waves_per_block) {
    if (waves_per_block == 1) return occ<NW, NS, 1, H16>();
    if (waves_per_block == 2) return occ<NW, NS, 2, H16>();
    return occ<NW, NS, 4, H16>();
}

int persistent_blocks_per_cu(int n_hits_window, int n_sides, int waves_per_block) {
    if (n_sides == 2) return n_hits_window <= 32 ? occ_wpb<32, 2>(waves_per_block) : occ_wpb<64, 2>(waves_per_block);
    if (n_sides == 3)
        return n_hits_window <= 32 ? occ_wpb<32, 1, true>(waves_per_block) : occ_wpb<64, 1, true>(waves_per_block);
    return n_hits_window <= 32 ? occ_wpb<32, 1>(waves_per_block) : occ_wpb<64, 1>(waves_per_block);
}

}  // namespace lfk

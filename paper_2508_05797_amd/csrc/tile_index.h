// Tile index of a job's bytes and a chain walker that steps over it.
//
// The two patterns of the paper, an extreme byte search (the largest byte of
// a window, Section 4.1) and a range scan (the first byte at or above a
// threshold, Section 4.2), are answered from a summary of every 1 KiB tile
// instead of the bytes themselves: the tile's largest byte m, how many of
// its bytes equal m, whether all of them do, and the offsets of the first
// seven that do.  One streaming pass writes the summaries (16 bytes per
// KiB); a walker then keeps 64 consecutive summaries in the lanes of one
// wave (64 KiB of input per page) and answers each query with one
// lane-parallel pass over the page and a ballot:
//   * the largest byte of [lo, hi): the maxima of the tiles the range covers
//     whole, plus each partly covered end tile's maximum when one of its
//     stored positions of m falls in the range;
//   * the first byte >= T in [lo, hi): the first tile with m >= T, and in
//     it the first stored position of m in the range when m == T (every
//     byte >= T then equals m).
// Where the summary cannot decide (a partly covered end tile whose maximum
// lies outside the range and matters; m > T in a scanned tile; more than
// seven positions of m, the ones needed not stored) the walker reads that
// one tile's bytes and answers from them.  Answers are exact either way.
//
// Bytes outside the job are absent: they are not counted in m, in the
// count or the positions (a tile of a job's first or last granules holds
// bytes of other data).
#pragma once

#include "wave.h"

namespace cdc {

constexpr int kIdxPos = 7;                 // stored positions per tile
constexpr uint32_t kNoPos = 0xFFFFu;

// Successor words (one per stored position of a tile's maximum, written by
// the successor pass): a node word dt << 23 | slot << 20 | offset names the
// next node (dt tiles on, its slot among its tile's stored positions, its
// offset in that tile); or the next cut is the forced one (chunk start +
// max_chunk), or the job's end; or the summaries cannot decide.
constexpr uint32_t kSuccForced = 1u << 30;
constexpr uint32_t kSuccEnd = 2u << 30;
constexpr uint32_t kSuccUnknown = 0xFFFFFFFFu;

// entry dword 0: m | cnt << 8 (saturated at 127) | all_m << 15 | pos0 << 16;
// dwords 1..3: pos1..pos6, 16 bits each (kNoPos: none); positions ascend.
__device__ __forceinline__ uint32_t ie_max(uint32_t x) { return x & 0xFFu; }
__device__ __forceinline__ uint32_t ie_cnt(uint32_t x) { return (x >> 8) & 0x7Fu; }
__device__ __forceinline__ bool ie_all(uint32_t x) { return (x >> 15) & 1u; }

// ------------------------------------------------------------ summaries

// High bit of each byte of d set iff that byte is zero.
__device__ __forceinline__ uint32_t zero_bytes(uint32_t d) {
    const uint32_t t = (d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    return ~(t | d | 0x7F7F7F7Fu);
}

// Summary of one tile whose bytes are raw (every lane calls it alike).
// tp: job position of the tile's first byte; whole: every byte of the tile
// belongs to the job (uniform).  slots: eight 16-bit LDS words of this wave.
// guess: a likely maximum (the previous tile's); when no lane holds more
// and one holds it, the wave reduction is skipped.
template <bool INV>
__device__ __forceinline__ uint4 summarize_tile(uint4 v, int64_t tp, int64_t n,
                                                bool whole, uint16_t* slots,
                                                uint32_t guess) {
    int a = 0, b = 16;
    if (!whole) {                                  // a tile at the job's ends
        const int64_t lp = tp + 16 * (int64_t)lane_id();
        a = (int)min(max(-lp, (int64_t)0), (int64_t)16);
        b = (int)min(max(n - lp, (int64_t)0), (int64_t)16);
        v = keep_bytes(v, a, b);
    }
    const uint32_t lm = lane_max16(v);
    uint32_t m = guess;
    if (__ballot(lm > guess) || !__ballot(lm == guess)) m = uni(wave_max(lm));
    const uint32_t r = m * 0x01010101u;
    uint32_t z0 = zero_bytes(v.x ^ r), z1 = zero_bytes(v.y ^ r);
    uint32_t z2 = zero_bytes(v.z ^ r), z3 = zero_bytes(v.w ^ r);
    if (!whole) {                                  // bytes outside the job
        const uint32_t keep = 0xFFFFu >> (16 - (b - a)) << a;   // bits [a, b)
        const uint32_t k = b > a ? keep : 0u;
        auto spread = [](uint32_t nib) {           // 4 bits -> high bits of 4 bytes
            return ((nib & 1u) << 7) | ((nib & 2u) << 14) | ((nib & 4u) << 21) |
                   ((nib & 8u) << 28);
        };
        z0 &= spread(k & 15u);
        z1 &= spread((k >> 4) & 15u);
        z2 &= spread((k >> 8) & 15u);
        z3 &= spread((k >> 12) & 15u);
    }
    const uint32_t c = __builtin_popcount(z0) + __builtin_popcount(z1) +
                       __builtin_popcount(z2) + __builtin_popcount(z3);
    const int64_t lo = max(tp, (int64_t)0), hi = min(tp + kTile, n);
    const uint32_t in_tile = hi > lo ? (uint32_t)(hi - lo) : 0u;
    uint32_t total;
    uint4 p;
    const uint64_t many = __ballot(c >= 2);
    if (whole && many == ~0ull && !__ballot(c != 16)) {
        // one value throughout: its first seven positions are 0..6
        total = kTile;
        p = make_uint4(0x00010000u, 0x00030002u, 0x00050004u, 0xFFFF0006u);
    } else if (!many) {
        // at most one byte equal to m per lane: ranks by counting lanes
        const uint64_t has = __ballot(c != 0);
        total = (uint32_t)__builtin_popcountll(has);
        const uint32_t rk = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(has >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)has, 0u));
        if (lane_id() < 8) slots[lane_id()] = (uint16_t)kNoPos;
        __builtin_amdgcn_wave_barrier();
        if (c && rk < (uint32_t)kIdxPos) {
            const uint64_t lo2 = ((uint64_t)z1 << 32) | z0, hi2 = ((uint64_t)z3 << 32) | z2;
            const int i = lo2 ? (__builtin_ctzll(lo2) >> 3) : 8 + (__builtin_ctzll(hi2) >> 3);
            slots[rk] = (uint16_t)(16 * lane_id() + i);
        }
        __builtin_amdgcn_wave_barrier();
        p = *(const uint4*)slots;                  // eight halves
        __builtin_amdgcn_wave_barrier();
    } else {
        const uint32_t incl = seg_sum<kWave>(c);
        total = uni((uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1));
        const uint32_t ex = incl - c;
        if (lane_id() < 8) slots[lane_id()] = (uint16_t)kNoPos;
        __builtin_amdgcn_wave_barrier();
        if (c && ex < (uint32_t)kIdxPos) {
            // this lane's bytes equal to m, in order, into the free ranks
            uint64_t bits = ((uint64_t)z1 << 32) | z0;
            uint32_t rk = ex;
            for (int h = 0; h < 2 && rk < (uint32_t)kIdxPos; h++) {
                while (bits && rk < (uint32_t)kIdxPos) {
                    const int i = __builtin_ctzll(bits) >> 3;     // byte index
                    bits &= bits - 1;
                    slots[rk++] = (uint16_t)(16 * lane_id() + 8 * h + i);
                }
                bits = ((uint64_t)z3 << 32) | z2;
            }
        }
        __builtin_amdgcn_wave_barrier();
        p = *(const uint4*)slots;                  // eight halves
        __builtin_amdgcn_wave_barrier();
    }
    uint4 e;
    e.x = m | (min(total, 127u) << 8) | ((in_tile > 0 && total == in_tile) ? 0x8000u : 0u) |
          (p.x << 16);
    e.y = (p.x >> 16) | (p.y << 16);
    e.z = (p.y >> 16) | (p.z << 16);
    e.w = (p.z >> 16) | (p.w << 16);
    (void)INV;
    return e;
}

// ------------------------------------------------------------ walker

// A walker over a job's index from segment base `base` on.  Its positions
// are 32-bit offsets from base and its tiles are counted from the tile that
// holds base (tile k starts at offset 1024 k - ph), so that its state and
// compares stay on the scalar unit.  The page is the 64 summaries from tile
// p0 on, one per lane.
template <bool INV>
struct IdxWalker {
    const uint4* idx;     // summary of tile k at idx[k]
    const uint4* succ;    // successor words of tile k at succ[2k], succ[2k + 1]
    Source src;
    int64_t t0;           // the job's tile number of tile 0
    int32_t ph;           // offset of base inside tile 0
    int32_t n;            // job length from base (clamped)
    int32_t ntiles;       // tiles from tile 0 to the job's end (clamped)
    int32_t p0;           // first tile of the page, a multiple of 32 (far below
                          // 0 before the first load)
    uint4 e;              // this lane's summary (tile p0 + lane)
    uint4 pf;             // the summary of tile p0 + 32 + lane, loaded ahead
    uint4 sa, sb;         // this lane's successor words (slots 0-3, 4-7)
    uint4 psa, psb;       // those of tile p0 + 32 + lane, loaded ahead
    int32_t hit_t, hit_s; // node of the last fast step's cut (tile, slot), or hit_s < 0
    uint32_t reads_ebs, reads_rs;   // tiles whose bytes each pattern read

    // job_succ may be null: the walker then never stands on a node
    __device__ void init(const JobView& J, const uint4* job_idx,
                         const uint32_t* job_succ, int64_t base) {
        src.init(J.data, (uint64_t)J.n);
        t0 = (base + src.shift) >> 10;
        ph = (int32_t)((base + src.shift) & (kTile - 1));
        idx = job_idx + t0;
        succ = job_succ != nullptr ? (const uint4*)(job_succ + t0 * kSuccSlots) : nullptr;
        psa = psb = make_uint4(kSuccUnknown, kSuccUnknown, kSuccUnknown, kSuccUnknown);
        hit_s = -1;
        const int64_t nrel = J.n - base;
        n = (int32_t)min(nrel, (int64_t)0x7FFFF000);
        const int64_t nt = (int64_t)((uint64_t)(J.n + src.shift + kTile - 1) >> 10) - t0;
        ntiles = (int32_t)min(nt, (int64_t)0x7FFFFFFF);
        p0 = INT32_MIN / 2;                      // no page yet
        reads_ebs = reads_rs = 0;
    }
    __device__ __forceinline__ int32_t tile(int32_t pos) const { return (pos + ph) >> 10; }
    __device__ __forceinline__ int32_t tstart(int32_t k) const { return (k << 10) - ph; }
    // Pages start at multiples of 32 tiles.  Moving on by 32 takes the page
    // loaded ahead (a walk moves forward, so its next page is usually there
    // before it is needed); any other move loads the page where it lands.
    // (lanes past the job's last tile load that tile and are cleared when
    // the page is taken, so the load itself has no condition)
    __device__ __forceinline__ void page_load(int32_t q) {
        const int32_t t = min(q + (int32_t)lane_id(), ntiles - 1);
        pf = idx[t];
        if (succ != nullptr) {
            psa = succ[2 * t];
            psb = succ[2 * t + 1];
        }
    }
    __device__ __forceinline__ void move_to(int32_t k) {
        const int32_t q = k & ~31;
        if (q != p0 + 32) page_load(q);
        const bool in = q + (int32_t)lane_id() < ntiles;
        e = in ? pf : make_uint4(0, 0, 0, 0);
        sa = in ? psa : make_uint4(kSuccUnknown, kSuccUnknown, kSuccUnknown, kSuccUnknown);
        sb = in ? psb : make_uint4(kSuccUnknown, kSuccUnknown, kSuccUnknown, kSuccUnknown);
        p0 = q;
        // the copies above must precede the next loads: e, sa and sb are then
        // never a load's destination, and their uses wait for no load in flight
        __builtin_amdgcn_sched_barrier(0);
        page_load(q + 32);
    }
    // successor word of slot `slot` of page lane l
    __device__ __forceinline__ uint32_t succ_word(int32_t l, uint32_t slot) const {
        // a tree of bitwise selects by the slot's bits (uniform masks): seven
        // vector operations and no branch
        const uint32_t m0 = 0u - (slot & 1u), m1 = 0u - ((slot >> 1) & 1u),
                       m2 = 0u - ((slot >> 2) & 1u);
        auto sel = [](uint32_t m, uint32_t a, uint32_t b) { return (a & m) | (b & ~m); };
        const uint32_t lo = sel(m1, sel(m0, sa.w, sa.z), sel(m0, sa.y, sa.x));
        const uint32_t hi = sel(m1, sel(m0, sb.w, sb.z), sel(m0, sb.y, sb.x));
        return (uint32_t)__builtin_amdgcn_readlane((int)sel(m2, hi, lo), l);
    }
    // make tile k part of the page
    __device__ __forceinline__ void need(int32_t k) {
        if ((uint32_t)(k - p0) < (uint32_t)kWave) return;   // p0 starts far below
        move_to(k);
    }
    // make tile k part of the page with at least 31 tiles after it
    __device__ __forceinline__ void ahead(int32_t k) {
        if ((uint32_t)(k - p0) < 32u) return;
        move_to(k);
    }

    // ---- a tile's bytes (where the summary cannot decide)
    __device__ __forceinline__ uint4 tile_bytes(int32_t k, int32_t lo, int32_t hi) {
        uint4 v = src.template load<INV>(t0 + k);
        const int32_t lp = tstart(k) + 16 * (int32_t)lane_id();
        const int a = min(max(lo - lp, 0), 16), b = min(max(hi - lp, 0), 16);
        return keep_bytes(v, a, b);
    }
    __device__ uint32_t bytes_max(int32_t k, int32_t lo, int32_t hi) {
        reads_ebs++;
        return uni(wave_max(lane_max16(tile_bytes(k, lo, hi))));
    }
    // first offset in [lo, hi) within tile k with a byte >= T (1..255), or -1
    __device__ int32_t bytes_first_geq(int32_t k, int32_t lo, int32_t hi, uint32_t T) {
        reads_rs++;
        const uint4 v = tile_bytes(k, lo, hi);         // bytes outside are 0 < T
        const uint64_t ball = __ballot(lane_max16(v) >= T);
        if (!ball) return -1;
        const int f = __builtin_ctzll(ball);
        const uint32_t d[4] = {(uint32_t)__builtin_amdgcn_readlane((int)v.x, f),
                               (uint32_t)__builtin_amdgcn_readlane((int)v.y, f),
                               (uint32_t)__builtin_amdgcn_readlane((int)v.z, f),
                               (uint32_t)__builtin_amdgcn_readlane((int)v.w, f)};
        int i = 0;
#pragma unroll
        for (int j = 15; j >= 0; j--)
            if (((d[j >> 2] >> (8 * (j & 3))) & 0xFFu) >= T) i = j;
        return tstart(k) + 16 * f + i;
    }

    // ---- one tile's summary, read out to scalar registers

    // Lanes [l0, l1] of the page as a mask (0 <= l0 <= l1 <= 63).
    __device__ __forceinline__ static uint64_t lanes(int32_t l0, int32_t l1) {
        const uint64_t hi = l1 >= 63 ? ~0ull : ((2ull << l1) - 1ull);
        return hi & (~0ull << l0);
    }
    __device__ __forceinline__ uint32_t xword(int32_t l) const {
        return (uint32_t)__builtin_amdgcn_readlane((int)e.x, l);
    }
    // First stored position of the tile's maximum in offsets [a, b), from the
    // summary of lane l whose first word is x; returns kNoPos when none is
    // stored there, and sets *undecided when the tile may still hold one
    // there (more than seven positions, all stored ones before a).
    __device__ uint32_t first_pos(int32_t l, uint32_t x, uint32_t a, uint32_t b,
                                  bool& undecided) const {
        undecided = false;
        const uint32_t p0 = x >> 16;
        if (p0 >= a) return p0 < b ? p0 : kNoPos;     // the first one overall
        const uint32_t cnt = ie_cnt(x);
        if (cnt <= 1) return kNoPos;
        const uint32_t y = (uint32_t)__builtin_amdgcn_readlane((int)e.y, l);
        const uint32_t z = (uint32_t)__builtin_amdgcn_readlane((int)e.z, l);
        const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)e.w, l);
        const uint32_t ps[6] = {y & 0xFFFFu, y >> 16, z & 0xFFFFu, z >> 16,
                                w & 0xFFFFu, w >> 16};
        const uint32_t k_n = min(cnt, (uint32_t)kIdxPos) - 1;
        for (uint32_t k = 0; k < k_n; k++) {
            const uint32_t p = ps[k];
            if (p >= a) return p < b ? p : kNoPos;
        }
        undecided = cnt > (uint32_t)kIdxPos;          // all seven before a
        return kNoPos;
    }

    // End (exclusive) of the run of bytes equal to the byte at s that
    // consists of whole tiles of one value from s's tile on (or, at the job's
    // end, the job's last bytes), when that run reaches past s + w; else -1.
    __device__ int32_t const_run_end(int32_t s, int32_t w) {
        const int32_t k0 = tile(s);
        need(k0);
        const uint32_t x = xword(k0 - p0);
        if (!ie_all(x)) return -1;
        const uint32_t v = ie_max(x);
        for (int32_t k = k0;;) {
            need(k);
            const uint32_t me = e.x;
            const uint64_t brk = __ballot(!ie_all(me) || ie_max(me) != v) &
                                 (~0ull << (k - p0));
            if (brk) {
                const int32_t re = min(tstart(p0 + __builtin_ctzll(brk)), n);
                return re - 1 >= s + w ? re : -1;
            }
            k = p0 + kWave;
            if (k >= ntiles) {
                const int32_t re = n;
                return re - 1 >= s + w ? re : -1;
            }
        }
    }

    // ---- one chain step from the page's summaries alone
    //
    // Most steps need no byte and no second page: the tiles a window covers
    // whole give its largest byte (unless an end tile holds a larger one),
    // and the first byte at or above it is the first stored position of the
    // first tile whose maximum equals it.  These return -1 whenever the
    // summaries cannot decide; the exact patterns below then take the step.

    // Largest byte of a range whose end tiles are page lanes la < lb - 1,
    // from the tiles between them (m: this lane's tile maximum); -1 when an
    // end tile holds a larger byte (its part in the range then decides).
    __device__ __forceinline__ int32_t fast_max(int32_t la, int32_t lb, uint32_t m) const {
        const int32_t l = (int32_t)lane_id();
        const bool inner = l > la && l < lb;
        if (__ballot(inner && m == 255u)) return 255;
        const uint32_t T = uni(wave_max(inner ? m : 0u));
        if (__ballot((l == la || l == lb) && m > T)) return -1;
        return (int32_t)T;
    }

    // First position at or after `from` (in the tile of page lane lc) of a
    // byte >= T (1 <= T): the position, kFar when no tile of the page from lc
    // on holds one, or -1 when the summaries cannot decide.  Every lane
    // works out its own tile's answer, so the step costs two ballots and one
    // lane read, not a branch per tile.
    static constexpr int32_t kFar = 0x7FFFFFFF;
    __device__ __forceinline__ int32_t fast_first(int32_t lc, int32_t from, uint32_t T,
                                                  uint32_t m) {
        const int32_t l = (int32_t)lane_id();
        const uint32_t a = l == lc ? (uint32_t)(from - tstart(p0 + lc)) : 0u;
        // the first stored position >= a (positions ascend; unused slots
        // hold kNoPos, which is above every offset, so no count is needed)
        const uint32_t ps[7] = {e.x >> 16, e.y & 0xFFFFu, e.y >> 16, e.z & 0xFFFFu,
                                e.z >> 16, e.w & 0xFFFFu, e.w >> 16};
        uint32_t f = kNoPos, fi = 7;
#pragma unroll
        for (int i = 6; i >= 0; i--) {
            fi = ps[i] >= a ? (uint32_t)i : fi;
            f = ps[i] >= a ? ps[i] : f;
        }
        const bool all = ie_all(e.x);
        const bool ge = l >= lc && m >= T;
        // a byte >= T located: the tile is one value, or its maximum is T
        // (every byte >= T equals it) and a stored position qualifies
        const bool hit = ge && (all || (m == T && f != kNoPos));
        // a byte >= T may lie where no stored position says
        const bool lost = ge && !hit && (m != T || ie_cnt(e.x) > (uint32_t)kIdxPos);
        const uint64_t H = __ballot(hit), X = __ballot(lost);
        if (!H) return X ? -1 : kFar;
        const int32_t lh = __builtin_ctzll(H);
        if (X & ((2ull << lh) - 1ull)) return -1;   // (a lost tile at or before)
        const uint32_t pos = all ? a : f;
        // the node: a stored position (a tile of one value gives none)
        hit_t = p0 + lh;
        hit_s = (int32_t)__builtin_amdgcn_readlane((int)(all ? 7u : fi), lh);
        if (hit_s == 7) hit_s = -1;
        return tstart(p0 + lh) + __builtin_amdgcn_readlane((int)pos, lh);
    }

    // RAM's next cut from chunk start s (s + w < L = min(s + M, n)), or -1.
    __device__ __forceinline__ int32_t ram_fast(int32_t s, int32_t w, int32_t L) {
        const int32_t ka = tile(s), kb = tile(s + w - 1), kc = tile(s + w);
        ahead(ka);
        const int32_t la = ka - p0, lb = kb - p0, lc = kc - p0;
        if (lb - la < 2 || lc > kWave - 1) return -1;
        const uint32_t m = ie_max(e.x);
        if ((__ballot(ie_all(e.x)) >> la) & 1ull) return -1;   // a run of one value
        const int32_t T = fast_max(la, lb, m);
        if (T < 0) return -1;
        if (T == 0) return s + w + 1;              // every byte is >= 0
        const int32_t j = fast_first(lc, s + w, (uint32_t)T, m);
        if (j == kFar) return tile(L - 1) - p0 < kWave ? L : -1;
        if (j < 0) return -1;
        if (j < L) return j + 1;
        hit_s = -1;                                // a forced cut: no node
        return L;
    }

    // AE's next cut from chunk start s (L = min(s + M, n)), or -1: the first
    // occurrence p of the largest byte V of [s, s + w], final when nothing
    // after the window up to p + w exceeds V.
    __device__ __forceinline__ int32_t ae_fast(int32_t s, int32_t w, int32_t L) {
        const int32_t hi = min(s + w + 1, L);
        const int32_t ka = tile(s), kb = tile(hi - 1);
        ahead(ka);
        const int32_t la = ka - p0, lb = kb - p0;
        if (lb - la < 2 || lb > kWave - 1) return -1;
        const uint32_t m = ie_max(e.x);
        if ((__ballot(ie_all(e.x)) >> la) & 1ull) return -1;   // a run of one value
        const int32_t V = fast_max(la, lb, m);
        if (V <= 0) return -1;
        const int32_t p = fast_first(la, s, (uint32_t)V, m);
        if (p < 0 || p >= hi) return -1;           // (kFar included)
        if (V < 255) {
            const int32_t nhi = min(p + w + 1, L);
            if (nhi > hi) {
                const int32_t ld = tile(hi) - p0, le = tile(nhi - 1) - p0;
                if (le > kWave - 1) return -1;
                const int32_t l = (int32_t)lane_id();
                if (__ballot(l >= ld && l <= le && m > (uint32_t)V)) return -1;
            }
        }
        if (p + w < L) return p + w + 1;
        hit_s = -1;                                // a forced cut: no node
        return L;
    }

    // ---- the two patterns, exact

    // max(M, largest byte of [lo, hi) inside end tile k)
    __device__ uint32_t end_max(int32_t k, int32_t lo, int32_t hi, uint32_t M) {
        need(k);
        const int32_t l = k - p0;
        const uint32_t x = xword(l);
        const uint32_t m = ie_max(x);
        if (m <= M) return M;
        if (ie_all(x)) return m;
        const int32_t ts = tstart(k);
        bool und;
        if (first_pos(l, x, (uint32_t)(lo - ts), (uint32_t)(hi - ts), und) != kNoPos)
            return m;
        return max(M, bytes_max(k, lo, hi));          // its maximum lies outside
    }

    // Largest byte in [lo, hi) (0 <= lo < hi <= n): extreme byte search.
    __device__ uint32_t range_max(int32_t lo, int32_t hi) {
        const int32_t ka = tile(lo), kb = tile(hi - 1);
        if (ka == kb) return end_max(ka, lo, hi, 0);
        uint32_t M = 0;
        for (int32_t k = ka + 1; k < kb;) {            // tiles covered whole
            need(k);
            const int32_t last = min(kb - 1, p0 + kWave - 1);
            const uint64_t msk = lanes(k - p0, last - p0);
            const uint32_t m = ie_max(e.x);
            if (__ballot(m == 255u) & msk) return 255u;
            const int32_t l = (int32_t)lane_id();
            M = max(M, uni(wave_max(((msk >> l) & 1ull) ? m : 0u)));
            k = last + 1;
        }
        M = end_max(ka, lo, tstart(ka) + kTile, M);
        if (M < 255u) M = end_max(kb, tstart(kb), hi, M);
        return M;
    }

    // First j in [lo, hi) with byte >= T (1 <= T <= 255), or -1: range scan.
    __device__ int32_t first_geq(int32_t lo, int32_t hi, uint32_t T) {
        if (lo >= hi) return -1;
        const int32_t ka = tile(lo), kb = tile(hi - 1);
        for (int32_t k = ka; k <= kb;) {
            need(k);
            const int32_t last = min(kb, p0 + kWave - 1);
            uint64_t cand = __ballot(ie_max(e.x) >= T) & lanes(k - p0, last - p0);
            while (cand) {
                const int32_t l = __builtin_ctzll(cand);
                cand &= cand - 1;
                const int32_t kt = p0 + l;
                const uint32_t x = xword(l);
                const int32_t ts = tstart(kt);
                const int32_t a = max(lo, ts), b = min(hi, ts + kTile);
                if (ie_all(x)) return a;               // every byte is m >= T
                if (ie_max(x) == T) {                  // bytes >= T are those == m
                    bool und;
                    const uint32_t f = first_pos(l, x, (uint32_t)(a - ts),
                                                 (uint32_t)(b - ts), und);
                    if (f != kNoPos) return ts + (int32_t)f;
                    if (!und) continue;
                }
                const int32_t j = bytes_first_geq(kt, a, b, T);
                if (j >= 0) return j;
            }
            k = last + 1;
        }
        return -1;
    }
};

}  // namespace cdc

// Tile index of a job's bytes and a chain walker that steps over it.
//
// The two patterns of the paper, an extreme byte search (the largest byte of
// a window, Section 4.1) and a range scan (the first byte at or above a
// threshold, Section 4.2), are answered from a summary of every 1 KiB tile
// instead of the bytes themselves: the tile's largest byte m, how many of
// its bytes equal m, whether all of them do, and the offsets of the first
// seven that do.  One streaming pass writes the summaries (16 bytes per
// KiB); a walker then keeps 64 consecutive summaries in the lanes of one
// wave (64 KiB of input per page) and takes a chunk step with a few ballots
// and lane reads:
//   * the largest byte of [lo, hi): the maxima of the tiles the range covers
//     whole, plus each partly covered end tile's maximum when one of its
//     stored positions of m falls in the range;
//   * the first byte >= T in [lo, hi): the first tile with m >= T, and in
//     it the first stored position of m in the range when m == T (every
//     byte >= T then equals m).
// Where the summary cannot decide (a partly covered tile whose maximum lies
// outside the range and matters; m > T in the scanned tile; more than seven
// positions of m, the ones needed not stored) the walker reads that one
// tile's bytes and answers from them.  Answers are exact either way.
//
// Bytes outside the job are absent: they are not counted in m, in the
// count or the positions (a tile of a job's first or last granules holds
// bytes of other data).
#pragma once

#include "wave.h"

namespace cdc {

constexpr int kIdxPos = 7;                 // stored positions per tile

// entry dword 0: m | cnt << 8 (saturated at 127) | all_m << 15 | pos0 << 16;
// dwords 1..3: pos1..pos6, 16 bits each (0xFFFF: none)
__device__ __forceinline__ uint32_t ie_max(uint32_t x) { return x & 0xFFu; }
__device__ __forceinline__ uint32_t ie_cnt(uint32_t x) { return (x >> 8) & 0x7Fu; }
__device__ __forceinline__ bool ie_all(uint32_t x) { return (x >> 15) & 1u; }
__device__ __forceinline__ uint32_t ie_pos(const uint4& e, int k) {
    const uint32_t d = k == 0 ? e.x : k <= 2 ? e.y : k <= 4 ? e.z : e.w;
    return (k & 1) ? (d & 0xFFFFu) : (d >> 16);
}

// 16-bit mask of the lane's bytes equal to v (v <= 255).
__device__ __forceinline__ uint32_t eq_mask16(const uint4& q, uint32_t v) {
    const uint32_t r = v * 0x01010101u;
    const uint32_t d[4] = {q.x ^ r, q.y ^ r, q.z ^ r, q.w ^ r};
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        // high bit of each byte set iff that byte of d is zero
        uint32_t t = (d[i] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
        t = ~(t | d[i] | 0x7F7F7F7Fu);
        // gather the four high bits into bits 4i..4i+3
        const uint32_t g = ((t >> 7) & 1u) | ((t >> 14) & 2u) | ((t >> 21) & 4u) |
                           ((t >> 28) & 8u);
        m |= g << (4 * i);
    }
    return m;
}

// Bits [a, b) of a 16-bit mask.
__device__ __forceinline__ uint32_t bit_range16(int a, int b) {
    return b <= a ? 0u : ((0xFFFFu >> (16 - (b - a))) << a) & 0xFFFFu;
}

// Summary of tile t of the job (one wave; every lane calls it alike).
// slots: eight 16-bit LDS words of this wave.
template <bool INV>
__device__ __forceinline__ uint4 summarize_tile(const uint4& raw, int64_t tp,
                                                int64_t n, uint16_t* slots) {
    const int64_t lp = tp + 16 * (int64_t)lane_id();
    const int a = (int)min(max(-lp, (int64_t)0), (int64_t)16);
    const int b = (int)min(max(n - lp, (int64_t)0), (int64_t)16);
    const uint4 v = (a > 0 || b < 16) ? keep_bytes(raw, a, b) : raw;
    const uint32_t m = uni(wave_max(lane_max16(v)));
    const uint32_t eq = eq_mask16(v, m) & bit_range16(a, b);
    const uint32_t c = (uint32_t)__builtin_popcount(eq);
    const uint32_t incl = seg_sum<kWave>(c);
    const uint32_t total = uni((uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1));
    const uint32_t ex = incl - c;
    // bytes of the job in this tile
    const int64_t lo = max(tp, (int64_t)0), hi = min(tp + kTile, n);
    const uint32_t in_tile = hi > lo ? (uint32_t)(hi - lo) : 0u;
    if (lane_id() < 8) slots[lane_id()] = 0xFFFFu;
    __builtin_amdgcn_wave_barrier();
    uint32_t rest = eq;
    for (uint32_t r = ex; rest && r < (uint32_t)kIdxPos; r++) {
        const int bit = __builtin_ctz(rest);
        rest &= rest - 1;
        slots[r] = (uint16_t)(16 * lane_id() + bit);
    }
    __builtin_amdgcn_wave_barrier();
    const uint4 p = *(const uint4*)slots;   // 8 halves, little-endian pairs
    __builtin_amdgcn_wave_barrier();
    uint4 e;
    e.x = m | (min(total, 127u) << 8) | ((in_tile > 0 && total == in_tile) ? 0x8000u : 0u) |
          (p.x << 16);
    e.y = (p.x >> 16) | (p.y << 16);
    e.z = (p.y >> 16) | (p.z << 16);
    e.w = (p.z >> 16) | (p.w << 16);
    (void)INV;
    return e;
}

// A walker over the job's index: the page of 64 summaries from tile p0 in
// this lane's registers (and the following page loaded ahead).  Positions
// are job offsets.
template <bool INV>
struct IdxWalker {
    Source src;
    const uint4* idx;
    int64_t ntiles, n;
    int64_t p0, p1;       // first tile of the page / of the page loaded ahead
    uint4 e, e1;
    uint32_t* err;
    uint32_t fallbacks;   // tiles whose bytes were read

    __device__ void init(const JobView& J, const uint4* index, uint32_t* e_) {
        src.init(J.data, (uint64_t)J.n);
        n = J.n;
        idx = index;
        ntiles = (int64_t)((uint64_t)(J.n + src.shift + kTile - 1) >> 10);
        p0 = p1 = -1;
        err = e_;
        fallbacks = 0;
    }
    __device__ __forceinline__ uint4 load_page(int64_t t) const {
        const int64_t k = t + lane_id();
        uint4 r = make_uint4(0, 0, 0, 0);
        if (k < ntiles) r = idx[k];
        return r;
    }
    // make tile t part of the current page
    __device__ __forceinline__ void need(int64_t t) {
        if (t >= p0 && t < p0 + kWave && p0 >= 0) return;
        if (p1 >= 0 && t >= p1 && t < p1 + kWave) {
            p0 = p1;
            e = e1;
        } else {
            p0 = t;
            e = load_page(t);
        }
        p1 = p0 + kWave;
        if (p1 < ntiles)
            e1 = load_page(p1);
        else
            p1 = -1;
    }
    __device__ __forceinline__ uint4 entry(int64_t t) {
        need(t);
        const int l = (int)(t - p0);
        return make_uint4((uint32_t)__builtin_amdgcn_readlane((int)e.x, l),
                          (uint32_t)__builtin_amdgcn_readlane((int)e.y, l),
                          (uint32_t)__builtin_amdgcn_readlane((int)e.z, l),
                          (uint32_t)__builtin_amdgcn_readlane((int)e.w, l));
    }
    __device__ __forceinline__ int64_t tile_of(int64_t pos) const {
        return (pos + src.shift) >> 10;
    }
    __device__ __forceinline__ int64_t tile_start(int64_t t) const {
        return t * kTile - src.shift;
    }

    // Largest m over tiles [ta, tb) (ta < tb).
    __device__ uint32_t tiles_max(int64_t ta, int64_t tb) {
        uint32_t M = 0;
        for (int64_t t = ta; t < tb && M < 255;) {
            need(t);
            const int64_t k0 = t - p0, k1 = min(tb - p0, (int64_t)kWave);
            const int64_t l = lane_id();
            const uint32_t mv = (l >= k0 && l < k1) ? ie_max(e.x) : 0u;
            M = max(M, uni(wave_max(mv)));
            t = p0 + k1;
        }
        return M;
    }
    // First tile in [ta, tb) with m >= T, or -1.
    __device__ int64_t first_tile_geq(int64_t ta, int64_t tb, uint32_t T) {
        for (int64_t t = ta; t < tb;) {
            need(t);
            const int64_t k0 = t - p0, k1 = min(tb - p0, (int64_t)kWave);
            const int64_t l = lane_id();
            const uint64_t b = __ballot(l >= k0 && l < k1 && ie_max(e.x) >= T);
            if (b) return p0 + __builtin_ctzll(b);
            t = p0 + k1;
        }
        return -1;
    }

    // ---- the bytes of one tile (when the summary cannot decide)
    __device__ __forceinline__ uint4 tile_bytes(int64_t t, int64_t lo, int64_t hi) {
        fallbacks++;
        uint4 v = src.template load<INV>(t);
        // keep the bytes of [lo, hi) only
        const int64_t lp = tile_start(t) + 16 * (int64_t)lane_id();
        const int a = (int)min(max(lo - lp, (int64_t)0), (int64_t)16);
        const int b = (int)min(max(hi - lp, (int64_t)0), (int64_t)16);
        return keep_bytes(v, a, b);
    }
    // exact largest byte of [lo, hi) inside tile t
    __device__ uint32_t bytes_max(int64_t t, int64_t lo, int64_t hi) {
        const uint4 v = tile_bytes(t, lo, hi);
        return uni(wave_max(lane_max16(v)));
    }
    // first position in [lo, hi) inside tile t with a byte >= T (1..255), or -1
    __device__ int64_t bytes_first_geq(int64_t t, int64_t lo, int64_t hi, uint32_t T) {
        const uint4 v = tile_bytes(t, lo, hi);   // bytes outside are 0 < T
        const uint32_t lm = lane_max16(v);
        uint64_t ball = __ballot(lm >= T);
        if (!ball) return -1;
        const int f = __builtin_ctzll(ball);
        const uint32_t q0 = (uint32_t)__builtin_amdgcn_readlane((int)v.x, f);
        const uint32_t q1 = (uint32_t)__builtin_amdgcn_readlane((int)v.y, f);
        const uint32_t q2 = (uint32_t)__builtin_amdgcn_readlane((int)v.z, f);
        const uint32_t q3 = (uint32_t)__builtin_amdgcn_readlane((int)v.w, f);
        const uint32_t d[4] = {q0, q1, q2, q3};
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const uint32_t by = (d[i >> 2] >> (8 * (i & 3))) & 0xFFu;
            if (by >= T) return tile_start(t) + 16 * f + i;
        }
        return -1;   // not reached: the lane maximum was >= T
    }

    // ---- the two patterns, exact

    // Largest byte in [lo, hi) (lo < hi): extreme byte search.
    __device__ uint32_t range_max(int64_t lo, int64_t hi) {
        const int64_t ta = tile_of(lo), tb = tile_of(hi - 1);
        if (ta == tb) return part_max(ta, lo, hi, 0);
        uint32_t M = ta + 1 < tb ? tiles_max(ta + 1, tb) : 0u;
        if (M >= 255) return M;
        M = part_max(ta, lo, tile_start(ta) + kTile, M);
        if (M >= 255) return M;
        return part_max(tb, tile_start(tb), hi, M);
    }
    // max(M, largest byte of [lo, hi) inside tile t)
    __device__ uint32_t part_max(int64_t t, int64_t lo, int64_t hi, uint32_t M) {
        const uint4 q = entry(t);
        const uint32_t m = ie_max(q.x);
        if (m <= M) return M;
        const int64_t ts = tile_start(t);
        if (ie_all(q.x) || (lo <= max(ts, (int64_t)0) && hi >= min(ts + kTile, n)))
            return m;                                 // the whole tile's bytes
        const int64_t a = lo - ts, b = hi - ts;
        const uint32_t cnt = ie_cnt(q.x);
        const int k_n = (int)min(cnt, (uint32_t)kIdxPos);
        for (int k = 0; k < k_n; k++) {
            const int64_t p = ie_pos(q, k);
            if (p >= b) break;                        // sorted: none in range
            if (p >= a) return m;
        }
        return max(M, bytes_max(t, lo, hi));
    }
    // First j in [lo, hi) with byte >= T (1 <= T <= 255), or -1: range scan.
    __device__ int64_t first_geq(int64_t lo, int64_t hi, uint32_t T) {
        if (lo >= hi) return -1;
        const int64_t tl = tile_of(hi - 1);
        for (int64_t t = tile_of(lo); t <= tl;) {
            t = first_tile_geq(t, tl + 1, T);
            if (t < 0) return -1;
            const uint4 q = entry(t);
            const int64_t ts = tile_start(t);
            const int64_t a = max(lo, ts), b = min(hi, ts + kTile);
            const uint32_t m = ie_max(q.x);
            if (ie_all(q.x)) return a;                // every byte is m >= T
            if (m == T) {
                const uint32_t cnt = ie_cnt(q.x);
                const int k_n = (int)min(cnt, (uint32_t)kIdxPos);
                bool decided = false;
                for (int k = 0; k < k_n; k++) {
                    const int64_t p = ts + ie_pos(q, k);
                    if (p >= b) { decided = true; break; }   // none in [a, b)
                    if (p >= a) return p;
                }
                if (decided || cnt <= (uint32_t)kIdxPos) {
                    t++;
                    continue;
                }
            }
            const int64_t j = bytes_first_geq(t, a, b, T);
            if (j >= 0) return j;
            t++;
        }
        return -1;
    }
};

}  // namespace cdc

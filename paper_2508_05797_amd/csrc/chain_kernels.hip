// RAM and AE chunk chains on gfx950: speculate, fix up, resolve, emit.
//
// The two patterns of the paper (Section 4) as wavefront operations on
// 1 KiB tiles (64 lanes x 16 B).  A producer wave stages tiles with their
// lane maxima (SWAR v_pk_max_u16) and tile maxima (DPP) into LDS; a walker
// wave runs the chain over them:
//   * extreme byte search (Section 4.1): a window's maximum comes from the
//     maxima of the tiles it covers whole, plus the lanes of its first and
//     last tile (whole lanes by a per-lane select, reduced once by DPP where
//     the window ends; partly covered lanes read out only when they can
//     still raise the maximum);
//   * range scan (Section 4.2): tiles whose maximum is below the threshold
//     are passed by one SWAR compare of the packed tile maxima; in the tile
//     that can hold a hit, a ballot of "lane maximum >= T" names the lanes,
//     and the first one's bytes are compared with T as SWAR words.
// RAM (Section 2.1 "RAM"; Section 4.3) is one window maximum followed by a
// greater-or-equal scan; AE-Max (Section 2.1 "AE"; Section 4.3) is a chain of
// greater-than scans from the current target (inside one tile, and for
// windows of at least a tile, the chain's targets collapse to the first
// maximum of the rest of the tile); AE-Min runs as AE-Max of the
// complemented bytes.  A walker's state (chunk start, limit, position,
// threshold) is uniform and lives in scalar registers.
//
// The chain (cut k+1 depends on cut k) is split into segments.  Speculation
// runs one walker per segment from the segment start and records its cuts up
// to the first one at or past the segment end (its exit).  The fix-up pass
// runs each segment from the previous segment's speculative exit until a cut
// lands on the speculative list (the two chains coincide from there).  A
// segment whose fix-up never lands hands its successor an entry that the
// fix-up did not assume; parallel rounds re-walk exactly those successors
// (landing on either recorded list), and an ordered pass per job settles
// what is left.  RAM segments of a single byte value are resolved
// arithmetically (RAM chains there never meet).  The emit pass copies every
// segment's resolved pieces.
#include "wave.h"

namespace cdc {

constexpr int kSpan = 8;         // tiles a walker considers at once (one word of maxima)
static_assert(kSpan == 8, "a span's tile maxima are one packed 64-bit word");
constexpr int kGroup = 8;        // tiles staged per step (speculation)
constexpr int kGroupSolo = 16;   // same for the lone fix-up / re-walk walkers

// Positions inside the chain engine are 32-bit offsets from the segment
// start (segments and chunks are at most 2^28 bytes, so every position a
// walker visits fits), which keeps the walkers' compares on the scalar unit.

// ------------------------------------------------------------ lane bytes

// The 16 bytes of lane l of a tile, as uniform words.
struct Lane16 {
    uint32_t d0, d1, d2, d3;
};

__device__ __forceinline__ Lane16 lane_words(const uint4& v, int l) {
    return Lane16{(uint32_t)__builtin_amdgcn_readlane((int)v.x, l),
                  (uint32_t)__builtin_amdgcn_readlane((int)v.y, l),
                  (uint32_t)__builtin_amdgcn_readlane((int)v.z, l),
                  (uint32_t)__builtin_amdgcn_readlane((int)v.w, l)};
}

__device__ __forceinline__ uint32_t byte_of(const Lane16& q, int i) {
    const uint32_t d = i < 4 ? q.d0 : i < 8 ? q.d1 : i < 12 ? q.d2 : q.d3;
    return (d >> (8 * (i & 3))) & 0xFFu;
}

// Largest byte among bytes [a, b) of the lane (0 if the range is empty).
__device__ __forceinline__ uint32_t lane_range_max(const Lane16& q, int a,
                                                   int b) {
    const uint4 m = make_uint4(q.d0 & dword_mask(a, b, 0),
                               q.d1 & dword_mask(a, b, 1),
                               q.d2 & dword_mask(a, b, 2),
                               q.d3 & dword_mask(a, b, 3));
    return uni(lane_max16(m));
}

// High bit of every byte of x that is >= the corresponding byte of y, whose
// bytes all equal the threshold; yl = y & 0x7F7F7F7F.  Per byte: equal top
// bits compare by the low seven bits ((x | 0x80) - (y & 0x7F) keeps bit 7
// exactly when x's low part is not smaller, and never borrows from the next
// byte); different top bits compare by the top bit.
__device__ __forceinline__ uint32_t ge_bytes(uint32_t x, uint32_t y,
                                             uint32_t yl) {
    const uint32_t H = 0x80808080u;
    const uint32_t r = (x | H) - yl;
    return ((x & ~y) | (~(x ^ y) & r)) & H;
}

// Bytes [k, 8) of a 64-bit word (all for k <= 0, none for k >= 8).
__device__ __forceinline__ uint64_t bytes_from(int k) {
    return k <= 0 ? ~0ull : k >= 8 ? 0ull : (~0ull << (8 * k));
}
// Bytes [0, k) of a 64-bit word (none for k <= 0, all for k >= 8).
__device__ __forceinline__ uint64_t bytes_to(int k) {
    return k >= 8 ? ~0ull : k <= 0 ? 0ull : ((1ull << (8 * k)) - 1ull);
}

// Index of the first byte >= T among bytes [a, b) of the lane, or -1
// (0 <= T <= 255).  The lane is compared as two 64-bit SWAR words (as
// ge_bytes, eight bytes at a time).
__device__ __forceinline__ int lane_first_ge(const Lane16& q, int a, int b,
                                             uint32_t T) {
    const uint64_t H = 0x8080808080808080ull;
    const uint64_t y = (uint64_t)(T * 0x01010101u) * 0x100000001ull;
    const uint64_t yl = y & ~H;
    const uint64_t x0 = ((uint64_t)q.d1 << 32) | q.d0;
    const uint64_t x1 = ((uint64_t)q.d3 << 32) | q.d2;
    const uint64_t r0 = (x0 | H) - yl, r1 = (x1 | H) - yl;
    uint64_t g0 = ((x0 & ~y) | (~(x0 ^ y) & r0)) & H;
    uint64_t g1 = ((x1 & ~y) | (~(x1 ^ y) & r1)) & H;
    g0 &= bytes_from(a) & bytes_to(b);
    g1 &= bytes_from(a - 8) & bytes_to(b - 8);
    if (g0) return __builtin_ctzll(g0) >> 3;
    if (g1) return 8 + (__builtin_ctzll(g1) >> 3);
    return -1;
}

// Range scan: the first position j in [lo, hi) (both inside the tile at tp,
// lo < hi) whose byte is >= T, 1 <= T <= 255; -1 if there is none.  lm holds
// the lane maxima; *val receives the byte.
__device__ __forceinline__ int32_t tile_find_ge(const uint4& v, uint32_t lm,
                                                int32_t tp, int32_t lo,
                                                int32_t hi, uint32_t T,
                                                uint32_t& val) {
    const int32_t lo_t = lo - tp, hi_t = hi - tp;
    const int la = lo_t >> 4, lb = (hi_t - 1) >> 4;
    uint64_t ball = __ballot(lm >= T);
    ball &= (~0ull << la) & (lb >= 63 ? ~0ull : ((2ull << lb) - 1ull));
    while (ball) {
        const int f = __builtin_ctzll(ball);
        ball &= ball - 1;
        const Lane16 q = lane_words(v, f);
        const int i = lane_first_ge(q, lo_t - 16 * f, hi_t - 16 * f, T);
        if (i >= 0) {
            val = byte_of(q, i);
            return tp + 16 * f + i;
        }
    }
    return -1;
}

// Largest lane maximum among lanes [l0, l1) (0 if the range is empty).
__device__ __forceinline__ uint32_t lanes_max(uint32_t lm, int32_t l0,
                                              int32_t l1) {
    if (l0 >= l1) return 0;
    if (l0 == 0 && l1 == kWave) return wave_max(lm);
    const int32_t lane = (int32_t)lane_id();
    return wave_max(lane >= l0 && lane < l1 ? lm : 0u);
}

// ------------------------------------------------------------ tiles

// Per-wave LDS staging: the bytes of G tiles and their lane maxima.
template <int G>
struct Ring {
    static_assert(G % kSpan == 0, "whole spans per ring");
    static constexpr bool kCoop = false;
    uint4 t[G][kWave];
    uint8_t lm[G][kWave];
};

// A staged tile as a walker sees it: its position (relative to the segment
// start) and its largest byte, both uniform; its bytes and lane maxima stay
// in LDS and are read only where a chunk boundary falls into the tile.
struct Tile {
    const uint4* vp;
    const uint8_t* lmp;
    int32_t tp;
    uint32_t tmax;
    __device__ __forceinline__ uint4 v() const { return *vp; }
    __device__ __forceinline__ uint32_t lm() const { return *lmp; }
};

// Eight consecutive staged tiles from position gp: the walkers decide from
// the packed tile maxima which tiles they can pass without looking inside.
struct Group {
    const uint4* vp;                     // this lane's piece of tile 0
    const uint8_t* lmp;                  // this lane's maximum of tile 0
    int32_t gp;
    uint64_t tmx;                        // byte i: largest byte of tile i
    __device__ __forceinline__ uint32_t tmax(int i) const {
        return (uint32_t)(tmx >> (8 * i)) & 0xFFu;
    }
    __device__ __forceinline__ Tile tile(int i) const {
        Tile t;
        t.vp = vp + i * kWave;
        t.lmp = lmp + i * kWave;
        t.tp = gp + i * kTile;
        t.tmax = tmax(i);
        return t;
    }
};

// Index of the first tile i >= k of the group whose largest byte is >= T
// (1 <= T <= 255), kSpan if there is none; the packed maxima are compared
// as in ge_bytes.
__device__ __forceinline__ int32_t first_tile_ge(uint64_t tmx, int32_t k,
                                                 uint32_t T) {
    const uint64_t H = 0x8080808080808080ull;
    const uint64_t y = (uint64_t)(T * 0x01010101u) * 0x100000001ull;
    const uint64_t r = (tmx | H) - (y & ~H);
    const uint64_t g = ((tmx & ~y) | (~(tmx ^ y) & r)) & H & bytes_from(k);
    return g ? (int32_t)(__builtin_ctzll(g) >> 3) : kSpan;
}

// Largest byte M among positions [lo, hi) of the tile (lo < hi, both inside)
// and, in *pos, the first position holding it.  The partly covered first
// lane A is examined only when its lane maximum reaches the whole lanes'
// maximum (it comes first, so a tie makes it the answer), the partly
// covered last lane B only when its lane maximum exceeds everything before.
__device__ __forceinline__ uint32_t tile_range_argmax(const Tile& t,
                                                      const uint4& v,
                                                      uint32_t lm, int32_t lo,
                                                      int32_t hi, int32_t& pos) {
    const int32_t tp = t.tp;
    const int32_t lo_t = lo - tp, hi_t = hi - tp;
    const int32_t fl = (lo_t + 15) >> 4, fh = hi_t >> 4;   // whole lanes [fl, fh)
    int la = -1, lb = -1, aA = 0, bA = 16, bB = 16;
    if (fl > fh) {                       // inside one lane
        la = fh;
        aA = lo_t & 15;
        bA = hi_t & 15;
    } else {
        if (lo_t & 15) {
            la = fl - 1;
            aA = lo_t & 15;
        }
        if (hi_t & 15) {
            lb = fh;
            bB = hi_t & 15;
        }
    }
    const uint32_t mF = (fl == 0 && fh == kWave) ? t.tmax : lanes_max(lm, fl, fh);
    Lane16 qA{0, 0, 0, 0}, qB{0, 0, 0, 0};
    uint32_t mA = 0, mB = 0;
    bool hasA = false;
    if (la >= 0 && (uint32_t)__builtin_amdgcn_readlane((int)lm, la) >= mF) {
        qA = lane_words(v, la);
        mA = lane_range_max(qA, aA, bA);
        hasA = true;
    }
    const uint32_t M1 = max(mA, mF);
    if (lb >= 0 && (uint32_t)__builtin_amdgcn_readlane((int)lm, lb) > M1) {
        qB = lane_words(v, lb);
        mB = lane_range_max(qB, 0, bB);
    }
    const uint32_t M = max(M1, mB);
    if (hasA && mA == M) {
        pos = tp + 16 * la + lane_first_ge(qA, aA, bA, M);
    } else if (fl < fh && mF == M) {
        const int32_t lane = (int32_t)lane_id();
        const int f = __builtin_ctzll(__ballot(lane >= fl && lane < fh && lm == M));
        pos = tp + 16 * f + lane_first_ge(lane_words(v, f), 0, 16, M);
    } else {
        pos = tp + 16 * lb + lane_first_ge(qB, 0, bB, M);
    }
    return M;
}

// ------------------------------------------------------------ walkers

// Uniform state of one walker.  RAM: the window is [s, we); T holds the
// maximum so far, then the scan threshold (scan = 1).  AE: we is the target
// position and T the threshold (target byte + 1), -1 at a chunk start (the
// chunk's first byte is its first target), > 255 when nothing can exceed
// the target.
struct Walker {
    int32_t s, L, cur, we, T, scan;
};

// n: job length relative to the segment start, clamped far beyond anything
// a walker of this segment reaches.
struct Ctx {
    int32_t n, w, M;
};

constexpr int32_t kRelClamp = 0x7FFFF000;

__device__ __forceinline__ Ctx ctx_of(const JobView& J, int64_t a) {
    Ctx C;
    C.n = (int32_t)min(J.n - a, (int64_t)kRelClamp);
    C.w = (int32_t)J.w;
    C.M = (int32_t)J.M;
    return C;
}

// Start a RAM chunk at c.  When the window does not fit before the limit
// (which then is n), the chunk's end is decided without reading: returns
// true with *end = n.
__device__ __forceinline__ bool ram_start(Walker& W, const Ctx& C, int32_t c,
                                          int32_t* end) {
    W.s = c;
    W.L = min(C.n, c + C.M);
    W.cur = c;
    W.we = c + C.w;
    W.T = 0;
    W.scan = 0;
    if (W.we >= W.L) {
        *end = W.L;
        return true;
    }
    return false;
}

__device__ __forceinline__ void ae_start(Walker& W, const Ctx& C, int32_t c) {
    W.s = c;
    W.L = min(C.n, c + C.M);
    W.cur = c;
    W.we = c;
    W.T = -1;
    W.scan = 0;
}

// Window maximum under construction (RAM).  Whole tiles go into the
// walker's T by their maxima; whole lanes of the window's first and last
// tile go into acc by a select (reduced once, where the window ends).  A
// partly covered lane is looked at only if it can matter: the one in the
// window's first tile, when the window goes on past that tile, is kept in
// scalar registers (its 16 bytes, byte range and lane maximum); those in the
// tile where the window ends are read there.  At the window end nothing but
// T is looked at when T already is 255, and a partial lane is reduced
// exactly only when its lane maximum (an upper bound of its part) exceeds
// the rest of the window.
struct RamWin {
    uint32_t acc;                        // per lane
    int32_t used;
    uint32_t q0, q1, q2, q3;             // kept lane's bytes
    uint32_t kr;                         // 0, or first | end << 8 | lane max << 16 | 1 << 31

    __device__ __forceinline__ void reset() {
        acc = 0;
        used = 0;
        kr = 0;
    }
    // whole lanes among bytes [lo, hi) of the tile
    __device__ __forceinline__ void whole(uint32_t lm, int32_t lo, int32_t hi) {
        const int32_t fl = (lo + 15) >> 4, fh = hi >> 4;
        if (fl < fh) {
            const int32_t lane = (int32_t)lane_id();
            acc = lane >= fl && lane < fh ? max(acc, lm) : acc;
            used = 1;
        }
    }
    // keep lane l's bytes [a, 16)
    __device__ __forceinline__ void keep(const uint4& v, uint32_t lm, int32_t l,
                                         int32_t a) {
        q0 = (uint32_t)__builtin_amdgcn_readlane((int)v.x, l);
        q1 = (uint32_t)__builtin_amdgcn_readlane((int)v.y, l);
        q2 = (uint32_t)__builtin_amdgcn_readlane((int)v.z, l);
        q3 = (uint32_t)__builtin_amdgcn_readlane((int)v.w, l);
        const uint32_t ub = (uint32_t)__builtin_amdgcn_readlane((int)lm, l);
        kr = (uint32_t)a | (16u << 8) | (ub << 16) | 0x80000000u;
    }
    // T at the window's end, which lies in the tile (v, lm) whose window
    // bytes are [lo, hi) (offsets inside it)
    __device__ __forceinline__ uint32_t finish(uint32_t T, const uint4& v,
                                               uint32_t lm, int32_t lo,
                                               int32_t hi) const {
        if (T >= 255) return T;
        if (used) T = max(T, uni(wave_max(acc)));
        if (kr && ((kr >> 16) & 0xFFu) > T)
            T = max(T, lane_range_max(Lane16{q0, q1, q2, q3}, (int)(kr & 15u), 16));
        if (lo >= hi) return T;
        const int32_t la = lo >> 4, lb = (hi - 1) >> 4;
        if (lo & 15) {                   // partial first lane here
            const int32_t e = la == lb ? ((hi - 1) & 15) + 1 : 16;
            if ((uint32_t)__builtin_amdgcn_readlane((int)lm, la) > T)
                T = max(T, lane_range_max(lane_words(v, la), lo & 15, e));
        }
        if ((hi & 15) && (la != lb || !(lo & 15))) {   // partial last lane here
            if ((uint32_t)__builtin_amdgcn_readlane((int)lm, lb) > T)
                T = max(T, lane_range_max(lane_words(v, lb), 0, hi & 15));
        }
        return T;
    }
};

// Advance a RAM walker through the rest of a tile (from W.cur, inside it).
// emit(c) is called for every chunk end c and returns true to stop the
// walker; returns true once stopped.
template <class Emit>
__device__ __forceinline__ bool ram_tile(Walker& W, RamWin& X, const Ctx& C,
                                         const Tile& t, Emit& emit) {
    const int32_t tp = t.tp, te = tp + kTile;
    const uint4 v = t.v();
    const uint32_t lm = t.lm();
    for (;;) {
        if (!W.scan) {
            // window bytes [cur, min(we, te)) of this tile
            const int32_t lo_t = W.cur - tp, hi_t = min(W.we, te) - tp;
            if (W.we > te) {             // the window goes on
                if (lo_t == 0) {
                    W.T = max(W.T, (int32_t)t.tmax);
                } else {
                    X.whole(lm, lo_t, kTile);
                    if (lo_t & 15) X.keep(v, lm, lo_t >> 4, lo_t & 15);
                }
                W.cur = te;
                return false;
            }
            int32_t flo = lo_t, fhi = hi_t;  // parts the finish reads
            if (lo_t == 0 && hi_t == kTile) {
                W.T = max(W.T, (int32_t)t.tmax);
                flo = fhi = 0;
            } else {
                X.whole(lm, lo_t, hi_t);
            }
            W.T = (int32_t)X.finish((uint32_t)W.T, v, lm, flo, fhi);
            X.reset();
            W.scan = 1;
            W.cur = W.we;
        }
        const int32_t hi = min(W.L, te);
        int32_t j = -1;
        if (W.cur < hi) {
            if (W.T == 0) {
                j = W.cur;               // every byte is >= 0
            } else if ((int32_t)t.tmax >= W.T) {
                uint32_t val;
                j = tile_find_ge(v, lm, tp, W.cur, hi, (uint32_t)W.T, val);
            }
        }
        int32_t c;
        if (j >= 0)
            c = j + 1;
        else if (W.L <= te)
            c = W.L;
        else {
            W.cur = te;
            return false;
        }
        if (emit(c)) return true;
        int32_t end;
        if (ram_start(W, C, c, &end)) {
            emit(end);                   // end == n: every walker stops there
            return true;
        }
        if (W.cur >= te) return false;
    }
}

// Advance a RAM walker over a group.  At a tile start, the tiles that lie
// wholly inside the window only raise T by their maxima, and the tiles a
// scan crosses without a byte >= T and without reaching the limit are
// passed; the walker looks inside a tile only where a window ends or a scan
// can stop.
template <class Emit>
__device__ __forceinline__ bool ram_group(Walker& W, RamWin& X, const Ctx& C,
                                          const Group& g, Emit& emit) {
    const int32_t gp = g.gp;
    for (;;) {
        int32_t i = (W.cur - gp) >> 10;
        if (i >= kSpan) return false;
        if (W.cur == gp + i * kTile) {
            if (!W.scan) {
                const int32_t kw = min(kSpan, (W.we - 1 - gp) >> 10);
                if (W.T < 255)
                    for (int32_t k = i; k < kw; k++) W.T = max(W.T, (int32_t)g.tmax(k));
                i = max(i, kw);
            } else if (W.T > 0) {
                const int32_t k = min(first_tile_ge(g.tmx, i, (uint32_t)W.T),
                                      (W.L - 1 - gp) >> 10);
                i = max(i, k);
            }
            W.cur = gp + i * kTile;
            if (i >= kSpan) return false;
        }
        if (ram_tile(W, X, C, g.tile(i), emit)) return true;
    }
}

// Advance an AE walker through the rest of a tile (as ram_tile).
template <class Emit>
__device__ __forceinline__ bool ae_tile(Walker& W, const Ctx& C, const Tile& t,
                                        Emit& emit) {
    const int32_t tp = t.tp, te = tp + kTile;
    const uint4 v = t.v();
    const uint32_t lm = t.lm();
    for (;;) {
        if (W.T < 0 && C.w >= kTile) {
            // The chunk's first byte is its first target, and every later
            // record in this tile lies within the window of the one before
            // it, so the target ends at the first maximum of the rest of
            // the tile (up to the limit).
            const int32_t hl = min(te, W.L);
            int32_t q;
            const uint32_t M = tile_range_argmax(t, v, lm, W.cur, hl, q);
            W.we = q;
            W.T = (int32_t)M + 1;
            W.cur = hl;
            if (W.cur >= te) return false;
            continue;
        }
        if (W.T < 0) {                   // the chunk's first byte
            const int32_t o = W.cur - tp;
            const uint32_t dw = (uint32_t)__builtin_amdgcn_readlane(
                (int)pick_dword(v, (o & 15) >> 2), o >> 4);
            W.we = W.cur;
            W.T = (int32_t)((dw >> (8 * (o & 3))) & 0xFFu) + 1;
            W.cur++;
        }
        const int32_t wend = min(W.we + C.w + 1, W.L);
        const int32_t hi = min(wend, te);
        if (W.T <= (int32_t)t.tmax && W.cur < hi) {
            uint32_t val;
            const int32_t j = tile_find_ge(v, lm, tp, W.cur, hi, (uint32_t)W.T, val);
            if (j >= 0 && C.w >= kTile) {
                // Every later record in this tile lies within the window of
                // the one before it, so the target ends at the first
                // maximum of [j, min(te, L)).
                const int32_t hl = min(te, W.L);
                int32_t q;
                const uint32_t M = tile_range_argmax(t, v, lm, j, hl, q);
                W.we = q;
                W.T = (int32_t)M + 1;
                W.cur = hl;
                if (W.cur >= te) return false;
                continue;
            }
            if (j >= 0) {                // a greater byte: the new target
                W.we = j;
                W.T = (int32_t)val + 1;
                W.cur = j + 1;
                if (W.cur >= te) return false;
                continue;
            }
        }
        if (wend > te) {
            W.cur = te;
            return false;
        }
        if (emit(wend)) return true;
        ae_start(W, C, wend);
        if (W.cur >= te) return false;
    }
}

// Advance an AE walker over a group: at a tile start, tiles before the one
// where the target's window ends and without a byte above the target are
// passed.
template <class Emit>
__device__ __forceinline__ bool ae_group(Walker& W, const Ctx& C,
                                         const Group& g, Emit& emit) {
    const int32_t gp = g.gp;
    for (;;) {
        int32_t i = (W.cur - gp) >> 10;
        if (i >= kSpan) return false;
        if (W.cur == gp + i * kTile && W.T >= 0) {
            // the window can end right here (a target on the previous
            // tile's last byte with the limit at this tile's start): then
            // nothing is passed
            const int32_t kl = (min(W.we + C.w + 1, W.L) - 1 - gp) >> 10;
            const int32_t kf = W.T > 255 ? kSpan : first_tile_ge(g.tmx, i, (uint32_t)W.T);
            i = max(i, min(kf, kl));
            W.cur = gp + i * kTile;
            if (i >= kSpan) return false;
        }
        if (ae_tile(W, C, g.tile(i), emit)) return true;
    }
}

// One tile's 16-byte piece for this lane from granule pointer p; only lanes
// below `valid` read (the others get zeros).
template <bool INV>
__device__ __forceinline__ uint4 ld_tile(const uint4* p, int32_t valid) {
    uint4 r = make_uint4(0, 0, 0, 0);
    if ((int32_t)lane_id() < valid) {
        const u32x4 q = __builtin_nontemporal_load((const global_u32x4*)p);
        r = make_uint4(q.x, q.y, q.z, q.w);
    }
    if (INV) r = make_uint4(~r.x, ~r.y, ~r.z, ~r.w);
    return r;
}

__device__ __forceinline__ int32_t lanes_valid(int64_t rem) {
    return (int32_t)min(max(rem, (int64_t)0), (int64_t)kWave);
}

// Stage a loaded group: the lane maxima and tile maxima of all G tiles are
// computed together (independent chains, so the vector unit stays busy),
// then the bytes and lane maxima go to LDS; the tile maxima are packed a
// byte each into tmx.
template <int G>
__device__ __forceinline__ void stage(Ring<G>& R, const uint4 (&c)[G],
                                      uint64_t (&tmx)[(G + 7) / 8]) {
    uint32_t lm[G], tm[G];
#pragma unroll
    for (int i = 0; i < G; i++) lm[i] = lane_max16(c[i]);
#pragma unroll
    for (int i = 0; i < G; i++) tm[i] = wave_max(lm[i]);
#pragma unroll
    for (int i = 0; i < G; i++) {
        R.t[i][lane_id()] = c[i];
        R.lm[i][lane_id()] = (uint8_t)lm[i];
    }
#pragma unroll
    for (int k = 0; k < (G + 7) / 8; k++) {
        uint64_t p = 0;
#pragma unroll
        for (int i = 0; i < 8 && 8 * k + i < G; i++) p |= (uint64_t)tm[8 * k + i] << (8 * i);
        tmx[k] = p;
    }
}

// Streams tiles from the one holding position first_rel (relative to base):
// G tiles are loaded into registers while the previous G are processed from
// the LDS ring, kSpan at a time.  body(group) returns true when the wave is
// done.  A hard stop one group past the end of the job guarantees every wave
// exits.
template <bool INV, int G, class Body>
__device__ __forceinline__ void run_tiles(const Source& src, Ring<G>& R,
                                          int64_t base, int32_t first_rel,
                                          int64_t n, Body&& body,
                                          uint32_t* err) {
    const int64_t t0 = src.tile_of(base + first_rel);
    int32_t left = (int32_t)min(src.tile_of(n) + 2 - t0, (int64_t)0x7FFFFFFF);
    int32_t tp = (int32_t)(src.tile_pos(t0) - base);
    const uint4* p = src.base + t0 * kWave + lane_id();
    int64_t rem = (int64_t)src.ngran - t0 * kWave;   // granules from tile t0 on
    uint4 c[G];
    uint64_t tmx[(G + 7) / 8];
#pragma unroll
    for (int i = 0; i < G; i++) c[i] = ld_tile<INV>(p + kWave * i, lanes_valid(rem - kWave * i));
    stage(R, c, tmx);
    for (;;) {
        p += kWave * G;
        rem -= kWave * G;
#pragma unroll
        for (int i = 0; i < G; i++)
            c[i] = ld_tile<INV>(p + kWave * i, lanes_valid(rem - kWave * i));
        for (int h = 0; h < G / kSpan; h++) {
            if (left <= 0) {
                if (lane_id() == 0) atomicOr(err, kErrOverflow);
                return;
            }
            left -= kSpan;
            const Group gr{&R.t[h * kSpan][lane_id()], &R.lm[h * kSpan][lane_id()],
                           tp, tmx[h]};
            if (body(gr)) return;
            tp += kSpan * kTile;
        }
        stage(R, c, tmx);
    }
}

// Cooperative streaming: a workgroup of two waves per walker.  Wave 0 (the
// producer) loads tiles and stages them with their lane and tile maxima in
// one half of a double-buffered LDS ring, while wave 1 (the walker) runs the
// chain over the other half; the two halves swap at a workgroup barrier
// every G tiles.  The producer's vector work then no longer sits in the
// walker's instruction stream (a wave issues at most one instruction per
// issue cycle of its SIMD; the two waves sit on different SIMDs).  The
// walker decides when to stop and says so in LDS; both waves read that flag
// after each barrier, and a final barrier keeps the next walk from touching
// the ring before both have left.  The flag of group g sits in done[g & 1],
// so the walker's write for the next group can never be seen by a producer
// still reading the current one.  Each role has a loop of its own (so that
// the other role's state is not live in it); both pass the same number of
// barriers.  The walker's tile budget (a hard stop one tile past the job)
// bounds the loop.
template <int G>
struct Coop {
    static_assert(G % kSpan == 0, "whole spans per ring half");
    static constexpr bool kCoop = true;
    uint4 t[2][G][kWave];
    uint8_t lm[2][G][kWave];
    uint64_t tmx[2][(G + 7) / 8];
    int32_t done[2];
    int32_t xfer[2];                     // walker -> producer (resolution)
};

// The wave's role, as a uniform value (the compiler cannot tell on its own
// that threadIdx.x / 64 is the same across a wave).
__device__ __forceinline__ uint32_t wave_in_block() {
    return uni(threadIdx.x >> 6);
}
__device__ __forceinline__ bool walker_wave(bool coop) {
    return !coop || wave_in_block() == 1;
}

template <int G>
__device__ __forceinline__ void coop_stage(Coop<G>& L, int slot,
                                           const uint4 (&c)[G]) {
    uint32_t lm[G], tm[G];
#pragma unroll
    for (int i = 0; i < G; i++) lm[i] = lane_max16(c[i]);
#pragma unroll
    for (int i = 0; i < G; i++) tm[i] = wave_max(lm[i]);
#pragma unroll
    for (int i = 0; i < G; i++) {
        L.t[slot][i][lane_id()] = c[i];
        L.lm[slot][i][lane_id()] = (uint8_t)lm[i];
    }
#pragma unroll
    for (int k = 0; k < (G + 7) / 8; k++) {
        uint64_t p = 0;
#pragma unroll
        for (int i = 0; i < 8 && 8 * k + i < G; i++) p |= (uint64_t)tm[8 * k + i] << (8 * i);
        if (lane_id() == 0) L.tmx[slot][k] = p;
    }
}

// Constancy of the tiles staged from position tp (relative): for every tile
// that starts before `end`, st stays the common byte value (0..255) while
// each such tile holds one value throughout; -1 before the first such tile,
// -2 once one differs.
template <int G>
__device__ __forceinline__ int32_t track_constant(const uint4 (&c)[G],
                                                  int32_t tp, int32_t end,
                                                  int32_t st) {
#pragma unroll
    for (int i = 0; i < G; i++) {
        if (st == -2 || tp + i * kTile >= end) break;
        const uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane((int)c[i].x) & 0xFFu;
        const uint32_t b4 = v * 0x01010101u;
        const bool eq = c[i].x == b4 && c[i].y == b4 && c[i].z == b4 && c[i].w == b4;
        if (__ballot(eq) != ~0ull || (st >= 0 && (uint32_t)st != v))
            st = -2;
        else
            st = (int32_t)v;
    }
    return st;
}

template <bool INV, int G, class Body>
__device__ __forceinline__ int32_t run_coop(const Source& src, Coop<G>& L,
                                         int64_t base, int32_t first_rel,
                                         int64_t n, Body&& body,
                                         uint32_t* err, int32_t track_end) {
    const int64_t t0 = src.tile_of(base + first_rel);
    int32_t cst = -1;
    if (wave_in_block() == 0) {          // producer
        const uint4* p = src.base + t0 * kWave + lane_id();
        int64_t rem = (int64_t)src.ngran - t0 * kWave;
        int32_t ptp = (int32_t)(src.tile_pos(t0) - base);
        uint4 c[G];
#pragma unroll
        for (int i = 0; i < G; i++) c[i] = ld_tile<INV>(p + kWave * i, lanes_valid(rem - kWave * i));
        coop_stage(L, 0, c);
        if (track_end > 0) cst = track_constant(c, ptp, track_end, cst);
        ptp += G * kTile;
        p += kWave * G;
        rem -= kWave * G;
#pragma unroll
        for (int i = 0; i < G; i++) c[i] = ld_tile<INV>(p + kWave * i, lanes_valid(rem - kWave * i));
        __syncthreads();
        for (int g = 0;; g++) {
            coop_stage(L, (g & 1) ^ 1, c);   // group g+1
            if (track_end > 0) cst = track_constant(c, ptp, track_end, cst);
            ptp += G * kTile;
            p += kWave * G;
            rem -= kWave * G;
#pragma unroll
            for (int i = 0; i < G; i++)
                c[i] = ld_tile<INV>(p + kWave * i, lanes_valid(rem - kWave * i));
            __syncthreads();
            if (uni((uint32_t)L.done[g & 1])) break;
        }
    } else {                             // walker
        int32_t left = (int32_t)min(src.tile_of(n) + 2 - t0, (int64_t)0x7FFFFFFF);
        int32_t tp = (int32_t)(src.tile_pos(t0) - base);
        __syncthreads();
        for (int g = 0;; g++) {
            const int slot = g & 1;
            uint32_t fin = 0;
            for (int h = 0; h < G / kSpan; h++) {
                if (left <= 0) {
                    if (lane_id() == 0) atomicOr(err, kErrOverflow);
                    fin = 1;
                    break;
                }
                left -= kSpan;
                const Group gr{&L.t[slot][h * kSpan][lane_id()],
                               &L.lm[slot][h * kSpan][lane_id()], tp,
                               (uint64_t)uni64((int64_t)L.tmx[slot][h])};
                if (body(gr)) {
                    fin = 1;
                    break;
                }
                tp += kSpan * kTile;
            }
            if (lane_id() == 0) L.done[slot] = (int32_t)fin;
            __syncthreads();
            if (fin) break;
        }
    }
    __syncthreads();
    return cst;
}

// Run one walker of the job from chunk start `start` (relative to base),
// fed by one wave's own staging ring or by a cooperative producer wave (all
// waves of the workgroup call this alike; only the walker wave emits).
template <bool RAM, bool INV, class Stage, class Emit>
__device__ __forceinline__ int32_t walk(const JobView& J, const Ctx& C, Stage& S,
                                        int64_t base, int32_t start, Emit& emit,
                                        uint32_t* err, int32_t track_end = 0) {
    constexpr bool kCoop = Stage::kCoop;
    Walker W;
    RamWin X;
    X.reset();
    if (RAM) {
        int32_t end;
        if (ram_start(W, C, start, &end)) {
            if (walker_wave(kCoop)) emit(end);
            return -1;
        }
    } else {
        ae_start(W, C, start);
    }
    Source src;
    src.init(J.data, (uint64_t)J.n);
    auto body = [&](const Group& g) -> bool {
        if constexpr (RAM)
            return ram_group(W, X, C, g, emit);
        else
            return ae_group(W, C, g, emit);
    };
    if constexpr (kCoop) {
        return run_coop<INV>(src, S, base, start, J.n, body, err, track_end);
    } else {
        run_tiles<INV>(src, S, base, start, J.n, body, err);
        return -1;
    }
}

// ------------------------------------------------------------ lists

// Writer of a cut list: positions collect in the lanes of one register and
// go out 64 at a time.
struct CutList {
    uint32_t* dst;
    uint32_t cap;
    uint32_t n;
    uint32_t buf;
    uint32_t* err;

    __device__ void init(uint32_t* d, uint32_t c, uint32_t* e) {
        dst = d;
        cap = c;
        n = 0;
        buf = 0;
        err = e;
    }
    __device__ __forceinline__ void push(uint32_t c) {
        const uint32_t k = n & 63u;
        if (lane_id() == k) buf = c;
        n++;
        if (k == 63u) {
            const uint32_t i = n - 64u + lane_id();
            if (i < cap) dst[i] = buf;
        }
    }
    __device__ void finish() {
        const uint32_t k = n & 63u;
        const uint32_t i = n - k + lane_id();
        if (lane_id() < k && i < cap) dst[i] = buf;
        if (n > cap && lane_id() == 0) atomicOr(err, kErrOverflow);
    }
};

// Cursor over an increasing list in global memory, 64 entries per load, for
// lookups of increasing positions.
struct ListCursor {
    const uint32_t* src;
    uint32_t n, base, vals, last;

    __device__ void load() {
        const uint32_t i = base + lane_id();
        vals = i < n ? src[i] : kNone;
        last = (uint32_t)__builtin_amdgcn_readlane((int)vals, 63);
    }
    __device__ void init(const uint32_t* s, uint32_t cnt) {
        src = s;
        n = cnt;
        base = 0;
        load();
    }
    // Index of c in the list, or -1; successive calls pass increasing c.
    __device__ __forceinline__ int32_t find(uint32_t c) {
        while (c > last && base + 64u < n) {
            base += 64u;
            load();
        }
        const uint64_t hit = __ballot(vals == c);
        return hit ? (int32_t)(base + (uint32_t)__builtin_ctzll(hit)) : -1;
    }
};

__device__ __forceinline__ uint32_t* list_of(const JobView& J,
                                             const ChainWs& ws, uint32_t seg,
                                             uint32_t list) {
    uint32_t* b = list == kListSpec ? ws.spec : list == kListFix ? ws.fix : ws.rew;
    return b + J.slot0 + (uint64_t)seg * J.cap;
}

// ------------------------------------------------------------ speculate

// All waves of the workgroup call this alike; the walker wave records.
template <bool RAM, bool INV, class Stage>
__device__ void speculate(const JobView& J, uint32_t seg, uint32_t item,
                          const ChainWs& ws, Stage& R) {
    const bool rec = walker_wave(Stage::kCoop);
    const int64_t a = (int64_t)seg * J.seg;
    const Ctx C = ctx_of(J, a);
    const int32_t b = (int32_t)(min(J.n, a + J.seg) - a);
    CutList out;
    out.init(list_of(J, ws, seg, kListSpec), J.cap, ws.err);
    int32_t last = 0;
    auto emit = [&](int32_t c) -> bool {
        out.push((uint32_t)c);
        last = c;
        return c >= b;
    };
    // RAM: the producer also reports whether every byte of the segment is
    // one value (for the arithmetic resolution below)
    const int32_t cst = walk<RAM, INV>(J, C, R, a, 0, emit, ws.err, RAM ? b : 0);
    if (!rec) {
        if (RAM && lane_id() == 0)
            ws.meta[item].cval = cst >= 0 ? 0x100u | (uint32_t)cst : 0u;
        return;
    }
    out.finish();
    if (lane_id() == 0) {
        SegMeta& m = ws.meta[item];
        m.exit = (uint64_t)(a + last);
        m.nspec = min(out.n, J.cap);
    }
}

// ------------------------------------------------------------ resolve

// Resolve segment `seg` from entry X (absolute, >= the segment start): the
// chain from X is followed until a cut lands on the speculative list (or,
// after the fix-up round, on the fix-up list, whose continuation is known);
// the cuts before that are written to the fix-up list (fix-up round) or the
// re-walk list.  Records the resolution (entry, pieces, count, exit) and
// returns its exit.
template <bool RAM, bool INV, class Stage>
__device__ int64_t resolve_from(const JobView& J, uint32_t seg, uint32_t item,
                                int64_t X, bool fixup, const ChainWs& ws,
                                Stage& R) {
    // all waves of the workgroup decide alike; the walker wave records
    const bool rec = walker_wave(Stage::kCoop);
    const int64_t a = (int64_t)seg * J.seg;
    const Ctx C = ctx_of(J, a);
    const int32_t b = (int32_t)(min(J.n, a + J.seg) - a);
    SegMeta& m = ws.meta[item];
    const uint32_t nspec = uni(m.nspec);
    const int64_t sexit = uni64((int64_t)m.exit);
    uint32_t nfix = 0, fms = kNone;
    int64_t fexit = 0, fentry = -1;
    if (!fixup) {
        nfix = uni(m.nfix);
        fms = uni(m.fms);
        fexit = uni64((int64_t)m.fexit);
        fentry = seg == 0 ? a : uni64((int64_t)ws.meta[item - 1].exit);
    }
    const uint32_t own = fixup ? kListFix : kListRewalk;
    uint32_t np = 0, count = 0;
    int64_t rexit = X;
    auto add = [&](uint32_t list, uint32_t lo, uint32_t hi) {
        hi = min(hi, J.cap);             // a list never holds more (else flagged)
        if (hi > lo) {
            if (rec && lane_id() == 0) m.pieces[np] = Piece{list, lo, hi};
            np++;
            count += hi - lo;
        }
    };
    // the fix-up chain from its index i on
    auto follow_fix = [&](uint32_t i) {
        add(kListFix, i, nfix);
        if (fms != kNone) {
            add(kListSpec, fms, nspec);
            rexit = sexit;
        } else {
            rexit = fexit;
        }
    };
    const int32_t e = (int32_t)(X - a);
    // the fix-up chain's own record (fix-up round)
    uint32_t new_nfix = 0, new_fms = kNone;
    int64_t new_fexit = X;
    bool settled = false;
    if (e >= b) {
        settled = true;                  // the chain jumps over the segment
    } else if (e == 0) {
        add(kListSpec, 0, nspec);
        rexit = sexit;
        new_fms = 0;
        settled = true;
    } else {
        ListCursor cs;
        cs.init(list_of(J, ws, seg, kListSpec), nspec);
        const int32_t i = cs.find((uint32_t)e);
        if (i >= 0) {
            add(kListSpec, (uint32_t)i + 1, nspec);
            rexit = sexit;
            new_fms = (uint32_t)i + 1;
            settled = true;
        } else if (!fixup) {
            if (X == fentry) {
                follow_fix(0);
                settled = true;
            } else {
                ListCursor cf;
                cf.init(list_of(J, ws, seg, kListFix), nfix);
                const int32_t f = cf.find((uint32_t)e);
                if (f >= 0) {
                    follow_fix((uint32_t)f + 1);
                    settled = true;
                }
            }
        }
    }
    if (!settled) {
        CutList wl;
        wl.init(list_of(J, ws, seg, own), J.cap, ws.err);
        // RAM over a segment of one byte value (or with max_chunk = w + 1):
        // a chunk whose w + 1 bytes lie in the segment is exactly w + 1 long
        // (its last byte equals the window maximum, or the forced cut falls
        // there), so those cuts follow arithmetically; the walk resumes at
        // the last of them.
        const bool arith = RAM && (C.M == C.w + 1 || (uni(m.cval) & 0x100u));
        ListCursor cs, cf;
        cs.init(list_of(J, ws, seg, kListSpec), nspec);
        if (!fixup) cf.init(list_of(J, ws, seg, kListFix), nfix);
        auto emit = [&](int32_t c) -> bool {
            const int32_t i = cs.find((uint32_t)c);
            if (i >= 0) {                // landed on the speculative chain
                add(own, 0, wl.n);
                add(kListSpec, (uint32_t)i, nspec);
                rexit = sexit;
                new_fms = (uint32_t)i;
                return true;
            }
            if (!fixup) {
                const int32_t f = cf.find((uint32_t)c);
                if (f >= 0) {            // landed on the fix-up chain
                    add(own, 0, wl.n);
                    follow_fix((uint32_t)f);
                    return true;
                }
            }
            wl.push((uint32_t)c);
            if (c >= b) {                // left the segment on its own
                add(own, 0, wl.n);
                rexit = a + c;
                new_fexit = rexit;
                return true;
            }
            return false;
        };
        int32_t start = e;
        int32_t stopped = 0;
        if (arith) {
            if (rec) {
                for (int32_t c = start + C.w + 1; c <= b; c += C.w + 1) {
                    start = c;
                    if (emit(c)) {
                        stopped = 1;
                        break;
                    }
                }
            }
            if constexpr (Stage::kCoop) {   // the walker's outcome to the producer
                if (rec && lane_id() == 0) {
                    R.xfer[0] = start;
                    R.xfer[1] = stopped;
                }
                __syncthreads();
                start = (int32_t)uni((uint32_t)R.xfer[0]);
                stopped = (int32_t)uni((uint32_t)R.xfer[1]);
            }
        }
        if (!stopped) walk<RAM, INV>(J, C, R, a, start, emit, ws.err);
        if (!rec) return 0;
        wl.finish();
        new_nfix = min(wl.n, J.cap);
    }
    if (rec && lane_id() == 0) {
        if (fixup) {
            m.nfix = new_nfix;
            m.fms = new_fms;
            m.fexit = (uint64_t)new_fexit;
        }
        m.npieces = np;
        m.count = count;
        m.entry = (uint64_t)X;
        m.rexit = (uint64_t)rexit;
    }
    return rexit;
}

// ------------------------------------------------------------ kernels

// The per-item kernels run one workgroup of two waves (producer and walker)
// per item: with one job the grid covers its segments (one each); with a
// job table the workgroups walk the algorithm's range of the item table
// grid-stride.
constexpr int kCoopThreads = 2 * kWave;

template <bool ONE, class F>
__device__ __forceinline__ void for_items(const Plan& P, uint32_t want, F&& f) {
    if constexpr (ONE) {
        const uint32_t wid = uni(blockIdx.x);
        if (wid >= P.one_items) return;
        const JobView J = view(P.one);
        if (J.ok && J.algo == want) f(J, wid, wid);
    } else {
        uint32_t first, last;
        item_range(P, want, first, last);
        for (uint32_t wid = first + uni(blockIdx.x); wid < last; wid += gridDim.x) {
            const Item it = P.items[wid];
            const JobView J = view(P.jobs[uni(it.job)]);
            if (J.ok && J.algo == want) f(J, uni(it.seg), wid);
        }
    }
}

template <bool RAM, bool INV, bool ONE>
__global__ __launch_bounds__(kCoopThreads) void k_spec(Plan P, ChainWs ws) {
    // One job: the walkers (the pass's bound; two per SIMD beside two
    // producers) issue ahead of the producers, which have time to spare.
    // Not in batches, where the later passes of other algorithms take the
    // highest priority and the producers there have less slack.
    if (ONE && wave_in_block() == 1) __builtin_amdgcn_s_setprio(2);
    __shared__ Coop<kGroup> lds;
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    for_items<ONE>(P, want, [&](const JobView& J, uint32_t seg, uint32_t wid) {
        speculate<RAM, INV>(J, seg, wid, ws, lds);
    });
}

// Fix-up round: every segment from the previous segment's speculative exit
// (segment 0 from the job start).
template <bool RAM, bool INV, bool ONE>
__global__ __launch_bounds__(kCoopThreads) void k_fix(Plan P, ChainWs ws) {
    tail_priority();
    __shared__ Coop<kGroup> lds;
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    for_items<ONE>(P, want, [&](const JobView& J, uint32_t seg, uint32_t wid) {
        const int64_t X = seg == 0 ? 0 : uni64((int64_t)ws.meta[wid - 1].exit);
        const int64_t h = resolve_from<RAM, INV>(J, seg, wid, X, true, ws, lds);
        if (walker_wave(true) && lane_id() == 0) ws.meta[wid].xo[1] = (uint64_t)h;
    });
}

// Parallel round r >= 2: a segment whose predecessor's exit (as of round
// r-1) differs from the entry it was resolved from is resolved again.
template <bool RAM, bool INV, bool ONE>
__global__ __launch_bounds__(kCoopThreads) void k_round(Plan P, ChainWs ws, int r) {
    tail_priority();
    __shared__ Coop<kGroup> lds;
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    const int src = (r - 1) & 1, dst = r & 1;
    for_items<ONE>(P, want, [&](const JobView& J, uint32_t seg, uint32_t wid) {
        SegMeta& m = ws.meta[wid];
        int64_t h = uni64((int64_t)m.rexit);
        if (seg > 0) {
            const int64_t X = uni64((int64_t)ws.meta[wid - 1].xo[src]);
            if (X != uni64((int64_t)m.entry))
                h = resolve_from<RAM, INV>(J, seg, wid, X, false, ws, lds);
        }
        if (walker_wave(true) && lane_id() == 0) m.xo[dst] = (uint64_t)h;
    });
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024).
__device__ uint64_t block_exscan(uint64_t v, uint64_t* sh, uint64_t& total) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    sh[tid] = v;
    __syncthreads();
    for (uint32_t o = 1; o < nt; o <<= 1) {
        uint64_t add = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    total = sh[nt - 1];
    const uint64_t ex = sh[tid] - v;
    __syncthreads();
    return ex;
}

// Settle one RAM / AE job with the whole block: segments whose entry is not
// their predecessor's resolved exit are resolved again, in order, by wave 0
// (after the parallel rounds there are rarely any); then output offsets are
// assigned.
template <bool RAM, bool INV>
__device__ void settle_job(const JobView& J, const ChainWs& ws,
                           Ring<kGroupSolo>& lds0, uint64_t* sh,
                           uint32_t* flagged, uint32_t& n_flagged) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    SegMeta* M0 = ws.meta + J.item0;
    for (uint32_t base = 1; base < J.nseg; base += nt) {
        if (tid == 0) n_flagged = 0;
        __syncthreads();
        const uint32_t k = base + tid;
        if (k < J.nseg && M0[k].entry != M0[k - 1].rexit) {
            const uint32_t slot = atomicAdd(&n_flagged, 1u);
            flagged[slot] = k;
        }
        __syncthreads();
        const uint32_t cnt = n_flagged;
        if (cnt > 0) {
            if (tid == 0) {              // in segment order
                for (uint32_t i = 1; i < cnt; i++) {
                    const uint32_t v = flagged[i];
                    uint32_t j = i;
                    while (j > 0 && flagged[j - 1] > v) {
                        flagged[j] = flagged[j - 1];
                        j--;
                    }
                    flagged[j] = v;
                }
            }
            __syncthreads();
            if (tid < kWave) {
                // Walk the flagged segments in order; a segment resolved
                // again can change its successor's entry (also past this
                // block's range), which is then resolved right away.
                uint32_t li = 0;
                uint32_t k2 = uni(flagged[0]);
                int64_t prev = uni64((int64_t)M0[k2 - 1].rexit);
                for (;;) {
                    int64_t h = uni64((int64_t)M0[k2].rexit);
                    if (prev != uni64((int64_t)M0[k2].entry))
                        h = resolve_from<RAM, INV>(J, k2, J.item0 + k2, prev,
                                                   false, ws, lds0);
                    while (li < cnt && uni(flagged[li]) <= k2) li++;
                    const uint32_t nxt = k2 + 1;
                    if (nxt < J.nseg && uni64((int64_t)M0[nxt].entry) != h) {
                        k2 = nxt;
                        prev = h;
                        continue;
                    }
                    if (li == cnt) break;
                    k2 = uni(flagged[li]);
                    prev = uni64((int64_t)M0[k2 - 1].rexit);
                }
            }
            __syncthreads();
        }
    }
    // output offsets: each thread sums kRun consecutive segments, one block
    // scan per kRun x nt segments
    constexpr uint32_t kRun = 8;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < J.nseg; base += kRun * nt) {
        const uint32_t k0 = base + kRun * tid;
        uint64_t c[kRun], sum = 0;
#pragma unroll
        for (uint32_t r = 0; r < kRun; r++) {
            c[r] = k0 + r < J.nseg ? M0[k0 + r].count : 0;
            sum += c[r];
        }
        uint64_t total;
        uint64_t at = carry + block_exscan(sum, sh, total);
#pragma unroll
        for (uint32_t r = 0; r < kRun; r++) {
            if (k0 + r < J.nseg) M0[k0 + r].out = at;
            at += c[r];
        }
        carry += total;
    }
    if (tid == 0) *J.n_cuts = carry;
}

// Settle RAM / AE jobs, one block per job (grid-stride over jobs).
template <bool RAM, bool INV>
__global__ __launch_bounds__(256) void k_resolve(Plan P, uint32_t n_jobs_h,
                                                 const uint32_t* n_jobs_d,
                                                 ChainWs ws) {
    tail_priority();
    __shared__ Ring<kGroupSolo> lds[1];
    __shared__ uint64_t sh[256];
    __shared__ uint32_t flagged[256];
    __shared__ uint32_t n_flagged;
    const uint32_t n_jobs = n_jobs_d ? *n_jobs_d : n_jobs_h;
    for (uint32_t job = blockIdx.x; job < n_jobs; job += gridDim.x) {
        const JobView J = view(P.jobs ? P.jobs[job] : P.one);
        const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
        if (J.ok && J.algo == want && J.n > 0)
            settle_job<RAM, INV>(J, ws, lds[0], sh, flagged, n_flagged);
        __syncthreads();
    }
}

// Copy one segment's resolved pieces to the output.
__device__ void emit_segment(const JobView& J, uint32_t seg, uint32_t wid,
                             const ChainWs& ws) {
    const SegMeta& m = ws.meta[wid];
    const uint64_t a = (uint64_t)seg * (uint64_t)J.seg;
    const uint64_t o = (uint64_t)uni64((int64_t)m.out);
    const uint32_t count = uni(m.count);
    if (o + count > max_cuts_of(J)) {   // cannot happen for a correct chain
        if (lane_id() == 0) atomicOr(ws.err, kErrOverflow);
        return;
    }
    uint64_t* out = J.cuts + o;
    const uint32_t np = uni(m.npieces);
    for (uint32_t q = 0; q < np; q++) {
        const uint32_t list = uni(m.pieces[q].list);
        const uint32_t lo = uni(m.pieces[q].lo), hi = uni(m.pieces[q].hi);
        const uint32_t* src = list_of(J, ws, seg, list);
        for (uint32_t i = lo + lane_id(); i < hi; i += kWave)
            out[i - lo] = a + src[i];
        out += hi - lo;
    }
}

__global__ __launch_bounds__(256) void k_emit(Plan P, ChainWs ws) {
    const uint32_t count = item_count(P);
    for (uint32_t wid = wave_global_id(); wid < count; wid += wave_count()) {
        JobView J;
        uint32_t seg;
        if (!item_of(P, wid, J, seg) || !J.ok || J.algo == kMaxp) continue;
        emit_segment(J, seg, wid, ws);
    }
}

// ------------------------------------------------------------ launches

#define CDC_LAUNCH(MK, LVL, NAME, ...)                 \
    do {                                               \
        if (MK) (MK)->begin(NAME, LVL, st);            \
        hipLaunchKernelGGL(__VA_ARGS__);               \
        if (MK) (MK)->end(LVL, st);                    \
    } while (0)

template <bool RAM, bool INV, bool ONE>
static void launch_passes(const Plan& P, uint32_t items_upper,
                          const ChainWs& ws, hipStream_t st, Marks* mk,
                          const char* spec_name, int part) {
    const dim3 blk(kCoopThreads), grid(items_upper);
    if (part & kPartSpec)
        CDC_LAUNCH(mk, 1, spec_name, (k_spec<RAM, INV, ONE>), grid, blk, 0, st, P, ws);
    if (part & kPartFix)
        CDC_LAUNCH(mk, 2, "fixup", (k_fix<RAM, INV, ONE>), grid, blk, 0, st, P, ws);
    if (part & kPartRest)
        for (int r = 2; r < 2 + kRounds; r++)
            CDC_LAUNCH(mk, 2, "round", (k_round<RAM, INV, ONE>), grid, blk, 0, st, P, ws, r);
}

// With one job, items_upper is its segment count (the grid covers every
// segment); with a job table the kernels walk the items grid-stride.
template <bool RAM, bool INV>
static void launch_algo(const Plan& P, uint32_t items_upper,
                        uint32_t jobs_upper, const uint32_t* n_jobs_d,
                        const ChainWs& ws, hipStream_t st, Marks* mk,
                        const char* spec_name, int part) {
    if (P.jobs == nullptr)
        launch_passes<RAM, INV, true>(P, items_upper, ws, st, mk, spec_name, part);
    else
        launch_passes<RAM, INV, false>(P, items_upper, ws, st, mk, spec_name, part);
    if (part & kPartRest)
        CDC_LAUNCH(mk, 2, "resolve", (k_resolve<RAM, INV>),
                   dim3(min(jobs_upper, 2048u)), dim3(256), 0, st, P, jobs_upper,
                   n_jobs_d, ws);
}

hipError_t launch_chain(const Plan& P, uint32_t algo, uint32_t items_upper,
                        uint32_t jobs_upper, const uint32_t* n_jobs_d,
                        const ChainWs& ws, hipStream_t st, Marks* mk, int part) {
    const bool one = P.jobs == nullptr;
    if (algo == kRam)
        launch_algo<true, false>(P, items_upper, jobs_upper, n_jobs_d, ws, st,
                                 mk, one ? "speculate_ram" : "speculate_batch_ram", part);
    else if (algo == kAe)
        launch_algo<false, false>(P, items_upper, jobs_upper, n_jobs_d, ws, st,
                                  mk, one ? "speculate_ae" : "speculate_batch_ae", part);
    else
        launch_algo<false, true>(P, items_upper, jobs_upper, n_jobs_d, ws, st,
                                 mk, one ? "speculate_ae_min" : "speculate_batch_ae_min", part);
    return hipGetLastError();
}

hipError_t launch_emit(const Plan& P, uint32_t items_upper, const ChainWs& ws,
                       int wpb, hipStream_t st, Marks* mk) {
    const dim3 blk(kWave * wpb), grid((items_upper + wpb - 1) / wpb);
    CDC_LAUNCH(mk, 2, "emit", k_emit, grid, blk, 0, st, P, ws);
    return hipGetLastError();
}

hipError_t launch_ram_ae(const Plan& P, uint32_t items_upper,
                         uint32_t jobs_upper, const uint32_t* n_jobs_d,
                         const ChainWs& ws, int wpb, hipStream_t st,
                         Marks* mk) {
    const bool one = P.jobs == nullptr;
    for (uint32_t algo : {kRam, kAe, kAeMin}) {
        if (!one || P.one.algo == algo) {
            const hipError_t e = launch_chain(P, algo, items_upper, jobs_upper,
                                              n_jobs_d, ws, st, mk);
            if (e != hipSuccess) return e;
        }
    }
    return launch_emit(P, items_upper, ws, wpb, st, mk);
}

}  // namespace cdc

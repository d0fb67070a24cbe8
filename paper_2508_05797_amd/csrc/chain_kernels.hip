// RAM and AE chunk chains on gfx950: speculate, fix up, resolve, emit.
//
// Patterns (Section 4 of the paper) as wavefront operations on a 1 KiB tile
// (64 lanes x 16 B) staged through a per-wave LDS ring:
//   * extreme byte search (Section 4.1): every tile gets its per-lane byte
//     maxima (SWAR v_pk_max_u16) and the tile maximum (DPP reduction) once;
//     a window that covers whole tiles is then one scalar max per tile, and
//     only its two partial end tiles need a masked reduction;
//   * range scan (Section 4.2): a tile whose maximum is below the threshold
//     is skipped with one scalar compare; otherwise a ballot of the lane
//     maxima finds the first candidate lane and a scalar SWAR compare of its
//     16 bytes the exact byte.
// RAM (Section 2.1 "RAM"; Section 4.3) is one window maximum followed by a
// GEQ scan; AE-Max (Section 2.1 "AE"; Section 4.3) is a chain of GT scans
// from the current target, which visits every byte once (AE-Min runs as
// AE-Max of the complemented bytes).
//
// The chain (cut k+1 depends on cut k) is split into segments.  In each
// segment a main walker speculates the chain from the segment start, and
// kFront more walkers start at evenly spaced offsets inside the first
// chunk's length; walkers that reach the same cut coalesce (the later one
// records where and into whom).  Two walkers on the same data meet only
// when they pick the same boundary byte, and the gap between them performs
// a random walk, so a lone speculative chain can stay apart from the true
// one for a long way; with recorded walkers close on both sides, the chain
// that really enters the segment meets one of them within a few chunks.
// The fix-up pass runs each segment from the previous segment's main exit
// until it meets a recorded walker, the resolve pass walks the segments in
// order (re-running the rare ones whose true entry differs from the one the
// fix-up assumed), and the emit pass copies the resolved cuts.
#include "wave.h"

namespace cdc {

constexpr int kGroup = 8;       // tiles staged per stream step (speculation)
constexpr int kGroupSolo = 32;  // same for the lone fix-up / re-run walkers
constexpr int kFL = kFrontCap + 1;        // entries per front list
static_assert(kFL <= kWave, "a front list must fit one entry per lane");

// ------------------------------------------------------------ tile scans

// Positions inside the chain engine are 32-bit offsets from the segment
// start (segments and chunks are at most 2^28 bytes, so every position a
// walker visits fits), which keeps the walkers' compares on the scalar unit.

// Largest byte in [lo, hi) clipped to the tile at tp (uniform result).
__device__ __forceinline__ uint32_t range_max(const uint4& v, uint32_t lm,
                                              int32_t tp, int32_t lo,
                                              int32_t hi) {
    const int32_t lo_t = lo - tp, hi_t = hi - tp;        // scalar
    const int32_t lp = 16 * (int32_t)lane_id();
    const int a = min(max(lo_t - lp, 0), 16);
    const int b = min(max(hi_t - lp, 0), 16);
    uint32_t x = 0;
    if (a == 0 && b == 16)
        x = lm;
    else if (a < b)
        x = lane_max16(keep_bytes(v, a, b));
    return wave_max(x);
}

// 16-bit mask of the bytes of one lane (four dwords) that are >= T,
// 1 <= T <= 255; evaluated on uniform values it runs on the scalar unit.
__device__ __forceinline__ uint32_t geq16(uint32_t d0, uint32_t d1,
                                          uint32_t d2, uint32_t d3, int T) {
    const uint32_t k = (uint32_t)(256 - T) * 0x00010001u;
    return geq_nib(d0, k) | (geq_nib(d1, k) << 4) | (geq_nib(d2, k) << 8) |
           (geq_nib(d3, k) << 12);
}

// Range scan: the first position j in [lo, hi), clipped to the tile, whose
// byte is >= T (T <= 0: any byte, T > 255: none); -1 if there is none.
__device__ __forceinline__ int32_t find_first(const uint4& v, uint32_t lm,
                                              int32_t tp, int32_t lo,
                                              int32_t hi, int T,
                                              uint32_t& val) {
    int32_t lo_t = lo - tp, hi_t = hi - tp;
    if (lo_t < 0) lo_t = 0;
    if (hi_t > kTile) hi_t = kTile;
    if (lo_t >= hi_t || T > 255) return -1;
    if (T <= 0) {
        const uint32_t dw = __builtin_amdgcn_readlane(
            pick_dword(v, (lo_t & 15) >> 2), lo_t >> 4);
        val = (dw >> (8 * (lo_t & 3))) & 0xFFu;
        return tp + lo_t;
    }
    const int32_t lp = 16 * (int32_t)lane_id();
    const bool cand = lp + 16 > lo_t && lp < hi_t && (int)lm >= T;
    uint64_t ball = __ballot(cand);
    while (ball) {
        const int f = __builtin_ctzll(ball);
        ball &= ball - 1;
        const uint32_t d0 = __builtin_amdgcn_readlane(v.x, f);
        const uint32_t d1 = __builtin_amdgcn_readlane(v.y, f);
        const uint32_t d2 = __builtin_amdgcn_readlane(v.z, f);
        const uint32_t d3 = __builtin_amdgcn_readlane(v.w, f);
        const int32_t fp = 16 * f;
        const int a = min(max(lo_t - fp, 0), 16);
        const int b = min(max(hi_t - fp, 0), 16);
        const uint32_t bits =
            geq16(d0, d1, d2, d3, T) & ((1u << b) - 1u) & ~((1u << a) - 1u);
        if (bits) {
            const int bi = __builtin_ctz(bits);
            const uint32_t dw = bi < 4 ? d0 : bi < 8 ? d1 : bi < 12 ? d2 : d3;
            val = (dw >> (8 * (bi & 3))) & 0xFFu;
            return tp + fp + bi;
        }
    }
    return -1;
}

// ------------------------------------------------------------ walkers

// Uniform state of one walker.  RAM: phase 0 accumulates the window maximum
// in T, phase 1 scans for a byte >= T.  AE: p is the target and T the scan
// threshold (target value + 1; 0 right after a cut).
struct WState {
    int32_t s, L, cur, p;
    int32_t phase, T, pad0, pad1;
};

// n: job length relative to the segment start, clamped far beyond anything
// a walker of this segment reaches.
struct ChainCtx {
    int32_t n, w, M;
};

constexpr int32_t kRelClamp = 0x7FFFF000;

__device__ __forceinline__ ChainCtx chain_ctx(const JobView& J, int64_t a) {
    ChainCtx C;
    C.n = (int32_t)min(J.n - a, (int64_t)kRelClamp);
    C.w = (int32_t)J.w;
    C.M = (int32_t)J.M;
    return C;
}

// Start a walker at chunk start s0.  Returns true if the chunk is already
// decided without reading (RAM's last chunk when the window does not fit);
// then *c_out is its end.
template <bool RAM>
__device__ __forceinline__ bool walker_start(WState& W, const ChainCtx& C,
                                             int32_t s0, int32_t* c_out) {
    W.s = s0;
    W.L = min(C.n, s0 + C.M);
    W.cur = s0;
    W.p = s0 - 1;
    W.phase = 0;
    W.T = 0;
    if (RAM && s0 + C.w >= W.L) {
        *c_out = W.L;
        return true;
    }
    return false;
}

// Advance a walker over one tile.  emit(c) is called for every chunk end c
// and returns true to stop the walker; returns true once stopped.
template <bool RAM, class Emit>
__device__ __forceinline__ bool walker_step(WState& W, const ChainCtx& C,
                                            const uint4& v, uint32_t lm,
                                            uint32_t tmax, int32_t tp,
                                            Emit& emit) {
    const int32_t te = tp + kTile;
    if (W.cur >= te) return false;   // starts in a later tile
    for (;;) {
        int32_t c;
        if (RAM) {
            if (W.phase == 0) {
                const int32_t we = W.s + C.w;
                const int32_t hi = min(we, te);
                const uint32_t m = (W.cur <= tp && hi >= te)
                                       ? tmax
                                       : range_max(v, lm, tp, W.cur, hi);
                W.T = max(W.T, (int32_t)m);
                if (we > te) {
                    W.cur = te;
                    return false;
                }
                W.phase = 1;
                W.cur = we;
            }
            const int32_t hi = min(W.L, te);
            int32_t j = -1;
            uint32_t val = 0;
            if (!(W.cur <= tp && hi >= te && (int32_t)tmax < W.T))
                j = find_first(v, lm, tp, W.cur, hi, W.T, val);
            if (j >= 0)
                c = j + 1;
            else if (W.L <= te)
                c = W.L;
            else {
                W.cur = te;
                return false;
            }
        } else {
            const int32_t wend = min(W.p + C.w + 1, W.L);
            const int32_t hi = min(wend, te);
            int32_t j = -1;
            uint32_t val = 0;
            if (!(W.cur <= tp && hi >= te && (int32_t)tmax < W.T))
                j = find_first(v, lm, tp, W.cur, hi, W.T, val);
            if (j >= 0) {
                W.p = j;
                W.T = (int32_t)val + 1;
                W.cur = j + 1;
                continue;
            }
            if (wend > te) {
                W.cur = te;
                return false;
            }
            c = wend;
        }
        if (emit(c)) return true;
        int32_t last;
        if (walker_start<RAM>(W, C, c, &last)) {
            emit(last);          // last == n: every walker stops there
            return true;
        }
        if (W.cur >= te) return false;
    }
}

// Per-wave LDS: the staging ring and the front walkers' states.
template <int G>
struct WaveLdsT {
    uint4 ring[G][kWave];
    WState front[kFront];
};
using WaveLds = WaveLdsT<kGroup>;
using SoloLds = WaveLdsT<kGroupSolo>;

// Streams tiles from the one holding first_pos: kGroup tiles are loaded into
// registers while the previous kGroup are processed from the LDS ring.
// body(v, lm, tmax, tp) returns true when the wave is done.  A hard stop
// past the end of the job guarantees every wave exits.
template <bool INV, int G, class Body>
__device__ __forceinline__ void run_tiles(const Source& src, WaveLdsT<G>& L,
                                          int64_t base, int32_t first_rel,
                                          int64_t n, Body&& body,
                                          uint32_t* err) {
    int64_t t = src.tile_of(base + first_rel);
    const int64_t t_end = src.tile_of(n) + 1;
    uint4 c[G];
#pragma unroll
    for (int i = 0; i < G; i++) c[i] = src.load<INV>(t + i);
#pragma unroll
    for (int i = 0; i < G; i++) L.ring[i][lane_id()] = c[i];
    for (;;) {
#pragma unroll
        for (int i = 0; i < G; i++) c[i] = src.load<INV>(t + G + i);
        for (int i = 0; i < G; i++) {
            if (t + i > t_end) {
                if (lane_id() == 0) atomicOr(err, kErrOverflow);
                return;
            }
            const uint4 v = L.ring[i][lane_id()];
            const uint32_t lm = lane_max16(v);
            const uint32_t tmax = wave_max(lm);
            if (body(v, lm, tmax, (int32_t)(src.tile_pos(t + i) - base)))
                return;
        }
#pragma unroll
        for (int i = 0; i < G; i++) L.ring[i][lane_id()] = c[i];
        t += G;
    }
}

// ------------------------------------------------------------ storage

__device__ __forceinline__ uint32_t* main_list(const JobView& J,
                                               const ChainWs& ws, uint32_t seg) {
    return ws.spec + J.slot0 + (uint64_t)seg * J.cap;
}
__device__ __forceinline__ uint32_t* fix_list(const JobView& J,
                                              const ChainWs& ws, uint32_t seg) {
    return ws.fix + J.slot0 + (uint64_t)seg * J.cap;
}
__device__ __forceinline__ uint32_t* front_list(const ChainWs& ws,
                                                uint32_t item, int f) {
    return ws.front + ((uint64_t)item * kFront + f) * kFL;
}

// Offsets of the front walkers' starts: kFront + 1 evenly spaced starts
// (the main walker's included) over w + 512 bytes, the usual reach of a
// chunk; only for windows of at least one tile, where a walker ends at most
// one chunk per tile.
__device__ __forceinline__ int front_count(const JobView& J, const ChainCtx& C,
                                           int32_t b, int32_t& spacing) {
    if (C.w < kTile || !J.front) return 0;
    spacing = (C.w + 512) / (kFront + 1);
    int nf = 0;
    while (nf < kFront && (nf + 1) * spacing < b &&
           (nf + 1) * spacing + C.w < C.n)
        nf++;
    return nf;
}

// ------------------------------------------------------------ speculate

template <bool RAM, bool INV>
__device__ void speculate(const JobView& J, uint32_t seg, uint32_t item,
                          const ChainWs& ws, WaveLds& L) {
    const int64_t a = (int64_t)seg * J.seg;
    const ChainCtx C = chain_ctx(J, a);
    const int32_t b = (int32_t)(min(J.n, a + J.seg) - a);
    uint32_t* mlist = main_list(J, ws, seg);
    const uint32_t cap = J.cap;
    uint32_t ncut = 0;
    int32_t mlast = 0;
    bool main_alive = true;

    auto emit_main = [&](int32_t c) -> bool {
        if (ncut < cap) {
            if (lane_id() == 0) mlist[ncut] = (uint32_t)c;
        } else if (lane_id() == 0) {
            atomicOr(ws.err, kErrOverflow);
        }
        ncut++;
        mlast = c;
        return c >= b;
    };

    WState W0;
    int32_t c0;
    if (walker_start<RAM>(W0, C, 0, &c0)) {
        emit_main(c0);
        main_alive = false;
    }

    // front walkers: states in LDS, stored-position counts in fcnt
    int32_t spacing = 0;
    const int nf = front_count(J, C, b, spacing);
    FrontMeta* fm = ws.fmeta + (uint64_t)item * kFront;
    uint32_t alive = 0;
    uint32_t fcnt[kFront];
#pragma unroll
    for (int f = 0; f < kFront; f++) fcnt[f] = 1;
    for (int f = 0; f < nf; f++) {
        const int32_t s0 = (f + 1) * spacing;
        WState W;
        int32_t cd;
        walker_start<RAM>(W, C, s0, &cd);   // s0 + w < n: the window fits
        if (lane_id() == 0) {
            L.front[f] = W;
            front_list(ws, item, f)[0] = (uint32_t)s0;
        }
        alive |= 1u << f;
    }

    auto body = [&](const uint4& v, uint32_t lm, uint32_t tmax,
                    int32_t tp) -> bool {
        if (main_alive &&
            walker_step<RAM>(W0, C, v, lm, tmax, tp, emit_main))
            main_alive = false;
        uint32_t todo = alive;
        while (todo) {
            const int f = __builtin_ctz(todo);
            todo &= todo - 1;
            WState W = L.front[f];
            W.s = (int32_t)uni((uint32_t)W.s);
            W.L = (int32_t)uni((uint32_t)W.L);
            W.cur = (int32_t)uni((uint32_t)W.cur);
            W.p = (int32_t)uni((uint32_t)W.p);
            W.phase = (int32_t)uni((uint32_t)W.phase);
            W.T = (int32_t)uni((uint32_t)W.T);
            if (W.cur >= tp + kTile) continue;   // starts in a later tile
            uint32_t* flist = front_list(ws, item, f);
            uint32_t cnt = fcnt[0];
#pragma unroll
            for (int q = 1; q < kFront; q++)
                if (q == f) cnt = fcnt[q];
            auto emit_front = [&](int32_t c) -> bool {
                // coalescence with the main walker or a lower front walker:
                // equal cuts are reached in the same tile
                uint32_t into = 0xFFFFFFFFu;
                if (main_alive ? c == W0.s : c == mlast)
                    into = 0;
                else {
                    const uint32_t l = lane_id();
                    const bool m = l < (uint32_t)f && ((alive >> l) & 1u) &&
                                   L.front[l < kFront ? l : 0].s == c;
                    const uint64_t bb = __ballot(m);
                    if (bb) into = (uint32_t)__builtin_ctzll(bb) + 1;
                }
                if (into != 0xFFFFFFFFu) {
                    if (lane_id() == 0) fm[f] = FrontMeta{cnt, into, (uint32_t)c, 0};
                    return true;
                }
                if (lane_id() == 0) flist[cnt] = (uint32_t)c;
                cnt++;
                if (c >= b) {
                    if (lane_id() == 0) fm[f] = FrontMeta{cnt, kEndExit, (uint32_t)c, 0};
                    return true;
                }
                if (cnt == (uint32_t)kFL) {
                    if (lane_id() == 0) fm[f] = FrontMeta{cnt, kEndTrunc, (uint32_t)c, 0};
                    return true;
                }
                return false;
            };
            if (walker_step<RAM>(W, C, v, lm, tmax, tp, emit_front))
                alive &= ~(1u << f);
#pragma unroll
            for (int q = 0; q < kFront; q++)
                if (q == f) fcnt[q] = cnt;
            if (lane_id() == 0) L.front[f] = W;
        }
        return !main_alive && alive == 0;
    };
    if (main_alive || alive) {
        Source src;
        src.init(J.data, (uint64_t)J.n);
        run_tiles<INV>(src, L, a, 0, J.n, body, ws.err);
    }
    if (lane_id() == 0) {
        SegMeta& m = ws.meta[item];
        m.exit = (uint64_t)(a + mlast);
        m.nspec = min(ncut, cap);
        m.nfront = (uint32_t)nf;
    }
}

// ------------------------------------------------------------ resolve

// Membership of positions in the walkers' stored lists of one segment
// (positions relative to the segment start).
struct Lists {
    const uint32_t* main;
    uint32_t nspec;
    uint32_t fval[kFront];   // lane l: entry l of front list f (or ~0)
    uint32_t fcnt[kFront];
    uint32_t fend[kFront];
    uint32_t fdpos[kFront];
    int nf;

    // Index of r in the main list (scanning 64 entries at a time), or -1.
    __device__ int32_t find_main(uint32_t r) const {
        for (uint32_t base = 0; base < nspec; base += kWave) {
            const uint32_t i = base + lane_id();
            const uint32_t x = i < nspec ? main[i] : 0xFFFFFFFFu;
            const uint64_t hit = __ballot(x == r);
            if (hit) return (int32_t)(base + __builtin_ctzll(hit));
            const uint32_t lastv = __builtin_amdgcn_readlane(
                x, (int)min(nspec - 1 - base, 63u));
            if (lastv > r) return -1;
        }
        return -1;
    }
    __device__ int32_t find_front(int f, uint32_t r) const {
        uint32_t x = fval[0];
#pragma unroll
        for (int q = 1; q < kFront; q++)
            if (q == f) x = fval[q];
        const uint64_t hit = __ballot(x == r);
        return hit ? (int32_t)__builtin_ctzll(hit) : -1;
    }
    // Walker list holding r: 0 main, f+1 front f.
    __device__ bool find(uint32_t r, uint32_t& list, uint32_t& idx) const {
#pragma unroll
        for (int f = 0; f < kFront; f++) {
            if (f >= nf) break;
            const uint64_t hit = __ballot(fval[f] == r);
            if (hit) {
                list = f + 1;
                idx = (uint32_t)__builtin_ctzll(hit);
                return true;
            }
        }
        const int32_t m = find_main(r);
        if (m >= 0) {
            list = 0;
            idx = (uint32_t)m;
            return true;
        }
        return false;
    }
};

struct FixOutcome {
    int64_t exit;   // where the resolved chain leaves the segment (absolute)
};

// Resolve segment `seg` from the true-or-assumed entry `entry` (absolute,
// >= segment start): fix-up cuts until the chain meets a recorded walker,
// then the pieces of walker lists it follows.  Writes the segment's record.
template <bool RAM, bool INV>
__device__ FixOutcome resolve_segment(const JobView& J, uint32_t seg,
                                      uint32_t item, int64_t entry,
                                      const ChainWs& ws, SoloLds& L) {
    const int64_t a = (int64_t)seg * J.seg;
    const ChainCtx C = chain_ctx(J, a);
    const int32_t b = (int32_t)(min(J.n, a + J.seg) - a);
    const int32_t e = (int32_t)(entry - a);
    SegMeta& m = ws.meta[item];
    Lists Ls;
    Ls.main = main_list(J, ws, seg);
    Ls.nspec = uni(m.nspec);
    Ls.nf = (int)uni(m.nfront);
    const FrontMeta* fm = ws.fmeta + (uint64_t)item * kFront;
#pragma unroll
    for (int f = 0; f < kFront; f++) {
        Ls.fcnt[f] = 0;
        Ls.fend[f] = 0;
        Ls.fdpos[f] = 0;
        Ls.fval[f] = 0xFFFFFFFFu;
        if (f < Ls.nf) {
            Ls.fcnt[f] = uni(fm[f].count);
            Ls.fend[f] = uni(fm[f].end);
            Ls.fdpos[f] = uni(fm[f].dpos);
            const uint32_t* fl = front_list(ws, item, f);
            if (lane_id() < Ls.fcnt[f]) Ls.fval[f] = fl[lane_id()];
        }
    }
    const int64_t main_exit = uni64((int64_t)m.exit);
    uint32_t* fx = fix_list(J, ws, seg);
    const uint32_t cap = J.cap;
    uint32_t nfix = 0;
    Piece pc[kMaxPieces];
    uint32_t np = 0;
    int64_t exit = entry;
    uint32_t merged = 0;

    auto put_fix = [&](uint32_t c) {
        if (nfix < cap) {
            if (lane_id() == 0) fx[nfix] = c;
        } else if (lane_id() == 0) {
            atomicOr(ws.err, kErrOverflow);
        }
        nfix++;
    };

    // where the chain is: on a walker list from index lo, or walking from a
    // position
    uint32_t list = 0, lo = 0;
    bool on_list = false;
    int32_t walk_from = -1;
    uint32_t li, ix;
    if (e == 0) {
        on_list = true;
    } else if (e < b && Ls.find((uint32_t)e, li, ix)) {
        on_list = true;
        list = li;
        lo = ix + 1;
    } else if (e < b) {
        walk_from = e;
    }

    for (int round = 0; round < 64; round++) {
        if (walk_from >= 0) {
            // walk until a cut lands on a recorded walker or leaves
            bool met = false;
            auto emit_fix = [&](int32_t c) -> bool {
                uint32_t l2, i2;
                if (Ls.find((uint32_t)c, l2, i2)) {
                    met = true;
                    list = l2;
                    lo = i2;
                    return true;
                }
                put_fix((uint32_t)c);
                if (c >= b) {
                    exit = a + c;
                    return true;
                }
                return false;
            };
            WState W;
            int32_t c0;
            if (walker_start<RAM>(W, C, walk_from, &c0)) {
                emit_fix(c0);
            } else {
                Source src;
                src.init(J.data, (uint64_t)J.n);
                auto body = [&](const uint4& v, uint32_t lm, uint32_t tmax,
                                int32_t tp) -> bool {
                    return walker_step<RAM>(W, C, v, lm, tmax, tp, emit_fix);
                };
                run_tiles<INV>(src, L, a, walk_from, J.n, body, ws.err);
            }
            walk_from = -1;
            if (!met) break;      // left the segment on its own
            on_list = true;
        }
        if (!on_list) break;
        // follow walker lists from (list, lo)
        merged = 1;
        bool resume = false;
        for (int hop = 0; hop <= kFront; hop++) {
            if (list == 0) {
                pc[np++] = Piece{0, lo, Ls.nspec, 0};
                exit = main_exit;
                break;
            }
            const int f = (int)list - 1;
            uint32_t fc = Ls.fcnt[0], fe = Ls.fend[0], fd = Ls.fdpos[0];
#pragma unroll
            for (int q = 1; q < kFront; q++)
                if (q == f) {
                    fc = Ls.fcnt[q];
                    fe = Ls.fend[q];
                    fd = Ls.fdpos[q];
                }
            pc[np++] = Piece{list, lo, fc, 0};
            if (fe == kEndExit) {
                exit = a + (int64_t)fd;
                break;
            }
            if (fe == kEndTrunc) {
                // the walker was cut off: copy the pieces into the fix-up
                // list and continue walking from its last position
                for (uint32_t q = 0; q < np; q++) {
                    const uint32_t* src_list =
                        pc[q].list == 0 ? Ls.main
                                        : front_list(ws, item, (int)pc[q].list - 1);
                    for (uint32_t i = pc[q].lo; i < pc[q].hi; i++)
                        put_fix(src_list[i]);
                }
                np = 0;
                walk_from = (int32_t)fd;
                resume = true;
                break;
            }
            // coalesced into walker fe at position fd
            const int32_t idx =
                fe == 0 ? Ls.find_main(fd) : Ls.find_front((int)fe - 1, fd);
            if (idx < 0) {          // cannot happen: both lists hold fd
                if (lane_id() == 0) atomicOr(ws.err, kErrOverflow);
                exit = a + (int64_t)fd;
                break;
            }
            list = fe;
            lo = (uint32_t)idx;
        }
        if (!resume) break;
        on_list = false;
    }
    uint32_t count = min(nfix, cap);
    for (uint32_t q = 0; q < np; q++) count += pc[q].hi - pc[q].lo;
    if (lane_id() == 0) {
        m.nfix = min(nfix, cap);
        m.count = count;
        m.merged = merged;
        m.npieces = np;
        for (uint32_t q = 0; q < np; q++) m.pieces[q] = pc[q];
        m.h = (uint64_t)exit;
    }
    return FixOutcome{exit};
}

// ------------------------------------------------------------ kernels

// Per-item kernels walk the items grid-stride, one wave per item.
template <bool RAM, bool INV>
__global__ __launch_bounds__(256) void k_spec(Plan P, ChainWs ws) {
    __shared__ WaveLds lds[4];
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    const uint32_t count = item_count(P);
    for (uint32_t wid = wave_global_id(); wid < count; wid += wave_count()) {
        JobView J;
        uint32_t seg;
        if (!item_of(P, wid, J, seg) || !J.ok || J.algo != want) continue;
        speculate<RAM, INV>(J, seg, wid, ws, lds[threadIdx.x / kWave]);
    }
}

template <bool RAM, bool INV>
__global__ __launch_bounds__(64) void k_fix(Plan P, ChainWs ws) {
    __shared__ SoloLds lds[1];
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    const uint32_t count = item_count(P);
    for (uint32_t wid = wave_global_id(); wid < count; wid += wave_count()) {
        JobView J;
        uint32_t seg;
        if (!item_of(P, wid, J, seg) || !J.ok || J.algo != want) continue;
        // segment 0 starts the chain; others assume the previous main exit
        const int64_t entry =
            seg == 0 ? 0 : uni64((int64_t)ws.meta[wid - 1].exit);
        resolve_segment<RAM, INV>(J, seg, wid, entry, ws, lds[0]);
    }
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

// Resolve one RAM / AE job with the whole block: segments whose true entry
// is not the previous main exit are re-run in order by wave 0; then output
// offsets are assigned.
template <bool RAM, bool INV>
__device__ void resolve_job(const JobView& J, const ChainWs& ws, SoloLds& lds0,
                            uint64_t* sh, uint32_t* nm_list,
                            uint32_t& nm_count, int64_t& carry_x) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    SegMeta* M0 = ws.meta + J.item0;
    const bool leader = tid < kWave;

    // A segment whose resolved exit differs from its main exit hands its
    // successor an entry the fix-up did not assume.
    if (tid == 0) carry_x = -1;   // -1: the window's first entry is on track
    __syncthreads();
    for (uint32_t base = 0; base < J.nseg; base += nt) {
        if (tid == 0) nm_count = 0;
        __syncthreads();
        const uint32_t k = base + tid;
        if (k + 1 < J.nseg && M0[k].h != M0[k].exit) {
            const uint32_t slot = atomicAdd(&nm_count, 1u);
            nm_list[slot] = k;
        }
        __syncthreads();
        const uint32_t cnt = nm_count;
        if (cnt > 0 || carry_x >= 0) {
            if (tid == 0) {
                for (uint32_t i = 1; i < cnt; i++) {
                    uint32_t v = nm_list[i], j = i;
                    while (j > 0 && nm_list[j - 1] > v) {
                        nm_list[j] = nm_list[j - 1];
                        j--;
                    }
                    nm_list[j] = v;
                }
            }
            __syncthreads();
            if (leader) {
                int64_t x = uni64(carry_x);
                uint32_t k2 = base;
                uint32_t li = 0;
                const uint32_t end = min(base + nt, J.nseg);
                while (k2 < end) {
                    if (x < 0) {
                        while (li < cnt && nm_list[li] < k2) li++;
                        if (li == cnt) break;
                        const uint32_t j = uni(nm_list[li]);
                        x = uni64((int64_t)M0[j].h);
                        k2 = j + 1;
                        continue;
                    }
                    const FixOutcome o = resolve_segment<RAM, INV>(
                        J, k2, J.item0 + k2, x, ws, lds0);
                    const int64_t mexit = uni64((int64_t)M0[k2].exit);
                    x = (o.exit == mexit) ? -1 : o.exit;
                    k2++;
                }
                if (lane_id() == 0) carry_x = (k2 >= end) ? x : -1;
            }
            __syncthreads();
        }
    }

    uint64_t carry = 0;
    for (uint32_t base = 0; base < J.nseg; base += nt) {
        const uint32_t k = base + tid;
        const uint64_t c = k < J.nseg ? M0[k].count : 0;
        uint64_t total;
        const uint64_t ex = block_exscan(c, sh, total);
        if (k < J.nseg) M0[k].out = carry + ex;
        carry += total;
    }
    if (tid == 0) *J.n_cuts = carry;
}

// Resolve RAM / AE jobs, one block per job (grid-stride over jobs).
template <bool RAM, bool INV>
__global__ __launch_bounds__(256) void k_resolve(Plan P, uint32_t n_jobs_h,
                                                 const uint32_t* n_jobs_d,
                                                 ChainWs ws) {
    __shared__ SoloLds lds[1];
    __shared__ uint64_t sh[256];
    __shared__ uint32_t nm_list[256];
    __shared__ uint32_t nm_count;
    __shared__ int64_t carry_x;
    const uint32_t n_jobs = n_jobs_d ? *n_jobs_d : n_jobs_h;
    for (uint32_t job = blockIdx.x; job < n_jobs; job += gridDim.x) {
        JobView J = view(P.jobs ? P.jobs[job] : P.one);
        const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
        if (J.ok && J.algo == want && J.n > 0)
            resolve_job<RAM, INV>(J, ws, lds[0], sh, nm_list, nm_count, carry_x);
        __syncthreads();
    }
}


// Copy one segment's resolved cuts: its fix-up cuts, then its pieces.
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
    const uint32_t nfix = uni(m.nfix);
    const uint32_t* fx = fix_list(J, ws, seg);
    for (uint32_t i = lane_id(); i < nfix; i += kWave) out[i] = a + fx[i];
    out += nfix;
    const uint32_t np = uni(m.npieces);
    for (uint32_t q = 0; q < np; q++) {
        const uint32_t list = uni(m.pieces[q].list);
        const uint32_t lo = uni(m.pieces[q].lo), hi = uni(m.pieces[q].hi);
        const uint32_t* src = list == 0 ? main_list(J, ws, seg)
                                        : front_list(ws, wid, (int)list - 1);
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

template <bool RAM, bool INV>
static void launch_algo(const Plan& P, uint32_t items_upper,
                        uint32_t jobs_upper, const uint32_t* n_jobs_d,
                        const ChainWs& ws, int wpb, hipStream_t st, Marks* mk,
                        const char* spec_name) {
    const dim3 blk(kWave * wpb), grid((items_upper + wpb - 1) / wpb);
    CDC_LAUNCH(mk, 1, spec_name, (k_spec<RAM, INV>), grid, blk, 0, st, P, ws);
    CDC_LAUNCH(mk, 2, "fixup", (k_fix<RAM, INV>), dim3(items_upper),
               dim3(kWave), 0, st, P, ws);
    CDC_LAUNCH(mk, 2, "resolve", (k_resolve<RAM, INV>),
               dim3(min(jobs_upper, 2048u)), dim3(256), 0, st, P, jobs_upper,
               n_jobs_d, ws);
}

hipError_t launch_ram_ae(const Plan& P, uint32_t items_upper,
                         uint32_t jobs_upper, const uint32_t* n_jobs_d,
                         const ChainWs& ws, int wpb, hipStream_t st,
                         Marks* mk) {
    const bool one = P.jobs == nullptr;
    if (!one || P.one.algo == kRam)
        launch_algo<true, false>(P, items_upper, jobs_upper, n_jobs_d, ws, wpb,
                                 st, mk, one ? "speculate_ram" : "speculate_batch_ram");
    if (!one || P.one.algo == kAe)
        launch_algo<false, false>(P, items_upper, jobs_upper, n_jobs_d, ws, wpb,
                                  st, mk, one ? "speculate_ae" : "speculate_batch_ae");
    if (!one || P.one.algo == kAeMin)
        launch_algo<false, true>(P, items_upper, jobs_upper, n_jobs_d, ws, wpb,
                                 st, mk, one ? "speculate_ae_min" : "speculate_batch_ae_min");
    const dim3 blk(kWave * wpb), grid((items_upper + wpb - 1) / wpb);
    CDC_LAUNCH(mk, 2, "emit", k_emit, grid, blk, 0, st, P, ws);
    return hipGetLastError();
}

}  // namespace cdc

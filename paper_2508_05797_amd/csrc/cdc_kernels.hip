// HIP kernels for hashless content-defined chunking on gfx950 (MI355X).
//
// The paper reduces RAM, AE and MAXP to two patterns (Section 4): the
// extreme byte search (the maximum of a window, Section 4.1) and the range
// scan (the first byte at or above a threshold, Section 4.2).  Here both are
// wavefront operations on a 1 KiB tile held in registers (64 lanes x 16 B):
//
//   * extreme byte search: per-lane SWAR byte maxima with v_pk_max_u16
//     (two accumulators for the odd and even bytes of each dword), reduced
//     across the wave with DPP row shifts and row broadcasts;
//   * range scan: per-lane SWAR compare (a carry into bit 8 of each 16-bit
//     half marks byte >= T) giving a 16-bit hit mask per lane, a 64-lane
//     ballot, and find-first-set on the ballot and on the winning lane.
//
// The chunk chain (cut k+1 depends on cut k) is made parallel by splitting
// the input into segments.  Each wave speculates the chain of its segment as
// if a chunk started at the segment start; because a chain is determined by
// any one of its cuts, a chain entering from the previous segment joins the
// speculative one at the first cut they share.  A fix-up pass runs each
// segment from the previous segment's speculative exit until the two chains
// meet, a resolve pass walks the segments in order (re-running the rare
// segments whose entry differs from the one the fix-up assumed), and an emit
// pass writes the offsets.
//
// MAXP's boundary test (a strict local maximum over +-w) does not depend on
// where the chunk starts, so its candidates are found fully in parallel by a
// block filter (a candidate is the unique maximum of every block of at most
// w+1 bytes containing it) followed by an exact check of the +-w window; the
// chain over the candidates is then arithmetic (forced cuts every M bytes).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cdc_internal.h"

namespace cdc {

// ------------------------------------------------------------ wave basics

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t uni(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int64_t uni64(int64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Per 16-bit half maximum; the high byte of each half is the maximum of the
// high bytes.
__device__ __forceinline__ uint32_t pkmax(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(
        uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                            __builtin_bit_cast(u16x2, b)));
}

template <int CTRL, int RMASK, bool BOUND0>
__device__ __forceinline__ uint32_t dpp_max(uint32_t v) {
    return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, RMASK,
                                                        0xF, BOUND0));
}

// Maximum over the 64 lanes, returned to every lane (uniform).
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = dpp_max<0x111, 0xF, true>(v);    // row_shr:1
    v = dpp_max<0x112, 0xF, true>(v);    // row_shr:2
    v = dpp_max<0x114, 0xF, true>(v);    // row_shr:4
    v = dpp_max<0x118, 0xF, true>(v);    // row_shr:8
    v = dpp_max<0x142, 0xA, false>(v);   // row_bcast:15
    v = dpp_max<0x143, 0xC, false>(v);   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Segmented maximum / sum over aligned groups of G lanes: the last lane of
// every group receives the group's value (other lanes hold partials).
template <int G>
__device__ __forceinline__ uint32_t seg_max(uint32_t v) {
    if (G >= 2) v = dpp_max<0x111, 0xF, true>(v);
    if (G >= 4) v = dpp_max<0x112, 0xF, true>(v);
    if (G >= 8) v = dpp_max<0x114, 0xF, true>(v);
    if (G >= 16) v = dpp_max<0x118, 0xF, true>(v);
    if (G >= 32) v = dpp_max<0x142, 0xA, false>(v);
    if (G >= 64) v = dpp_max<0x143, 0xC, false>(v);
    return v;
}
template <int CTRL, int RMASK, bool BOUND0>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v) {
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, RMASK,
                                                     0xF, BOUND0);
}
template <int G>
__device__ __forceinline__ uint32_t seg_sum(uint32_t v) {
    // Prefix sums within rows with shifts 1, 2, 4, 8 (Hillis-Steele).
    if (G >= 2) v = dpp_add<0x111, 0xF, true>(v);
    if (G >= 4) v = dpp_add<0x112, 0xF, true>(v);
    if (G >= 8) v = dpp_add<0x114, 0xF, true>(v);
    if (G >= 16) v = dpp_add<0x118, 0xF, true>(v);
    if (G >= 32) v = dpp_add<0x142, 0xA, false>(v);
    if (G >= 64) v = dpp_add<0x143, 0xC, false>(v);
    return v;
}

// Largest byte of the lane's 16 bytes.
__device__ __forceinline__ uint32_t lane_max16(const uint4& v) {
    uint32_t hi = pkmax(pkmax(v.x, v.y), pkmax(v.z, v.w));
    uint32_t lo = pkmax(pkmax(v.x << 8, v.y << 8), pkmax(v.z << 8, v.w << 8));
    uint32_t m = pkmax(hi, lo);
    return max(m >> 24, (m >> 8) & 0xFFu);
}

// Bytes [a, b) of dword d of a 16-byte lane (a, b in 0..16) as a mask.
__device__ __forceinline__ uint32_t dword_mask(int a, int b, int d) {
    int lo = min(max(a - 4 * d, 0), 4);
    int hi = min(max(b - 4 * d, 0), 4);
    const uint64_t F = 0xFFFFFFFFull;
    return (uint32_t)((F << (8 * lo)) & ~(F << (8 * hi)));
}

__device__ __forceinline__ uint4 keep_bytes(const uint4& v, int a, int b) {
    return make_uint4(v.x & dword_mask(a, b, 0), v.y & dword_mask(a, b, 1),
                      v.z & dword_mask(a, b, 2), v.w & dword_mask(a, b, 3));
}

// 4-bit mask of the bytes of x that are >= T, where k = (256-T)*0x00010001
// and 1 <= T <= 255: adding 256-T to a byte carries into bit 8 of its
// 16-bit half exactly when the byte is >= T.
__device__ __forceinline__ uint32_t geq_nib(uint32_t x, uint32_t k) {
    uint32_t e = ((x & 0x00FF00FFu) + k) & 0x01000100u;
    uint32_t o = (((x >> 8) & 0x00FF00FFu) + k) & 0x01000100u;
    uint32_t m = (e >> 8) | (o >> 7);
    return (m | (m >> 14)) & 0xFu;
}

__device__ __forceinline__ uint32_t geq_mask16(const uint4& v, int T) {
    uint32_t k = (uint32_t)(256 - T) * 0x00010001u;
    return geq_nib(v.x, k) | (geq_nib(v.y, k) << 4) | (geq_nib(v.z, k) << 8) |
           (geq_nib(v.w, k) << 12);
}

__device__ __forceinline__ uint32_t pick_dword(const uint4& v, int d) {
    return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
}

// Range scan on one tile: the first position j in [lo, hi), clipped to the
// tile [tp, tp+1024), whose byte is >= T (T <= 0: any byte; T > 255: none).
// Returns j and its byte value, or -1.  Called by the whole wave with
// uniform arguments.
__device__ __forceinline__ int64_t find_geq(const uint4& v, int64_t tp,
                                            int64_t lo, int64_t hi, int T,
                                            uint32_t& val) {
    if (lo < tp) lo = tp;
    if (hi > tp + kTile) hi = tp + kTile;
    if (lo >= hi || T > 255) return -1;
    const int64_t lp = tp + 16 * (int64_t)lane_id();
    const int a = (int)min(max(lo - lp, (int64_t)0), (int64_t)16);
    const int b = (int)min(max(hi - lp, (int64_t)0), (int64_t)16);
    uint32_t hm = (T <= 0) ? 0xFFFFu : geq_mask16(v, T);
    hm &= ((1u << b) - 1u) & ~((1u << a) - 1u);
    const uint64_t ball = __ballot(hm != 0);
    if (ball == 0) return -1;
    const int f = __builtin_ctzll(ball);
    const uint32_t bits = __builtin_amdgcn_readlane(hm, f);
    const int bi = __builtin_ctz(bits);
    const uint32_t dw = __builtin_amdgcn_readlane(pick_dword(v, bi >> 2), f);
    val = (dw >> (8 * (bi & 3))) & 0xFFu;
    return tp + 16 * (int64_t)f + bi;
}

// ------------------------------------------------------------ byte source

// A job's bytes as 16-byte granules aligned in the address space.  Tile t
// is granules [64t, 64t+64); its first byte is at position 1024t - shift.
struct Source {
    const uint4* base;
    int64_t shift;
    uint64_t ngran;

    __device__ void init(const uint8_t* data, uint64_t n) {
        uintptr_t p = (uintptr_t)data;
        base = (const uint4*)(p & ~(uintptr_t)15);
        shift = (int64_t)(p & 15);
        ngran = ((uint64_t)shift + n + 15) >> 4;
    }
    // Granules that hold no byte of the job are not read (zero instead).
    template <bool INV>
    __device__ __forceinline__ uint4 load(int64_t t) const {
        uint64_t g = (uint64_t)t * 64 + lane_id();
        uint4 r = make_uint4(0, 0, 0, 0);
        if (g < ngran) {
            const u32x4 q = __builtin_nontemporal_load((const u32x4*)(base + g));
            r = make_uint4(q.x, q.y, q.z, q.w);
        }
        if (INV) r = make_uint4(~r.x, ~r.y, ~r.z, ~r.w);
        return r;
    }
    __device__ __forceinline__ int64_t tile_pos(int64_t t) const {
        return t * kTile - shift;
    }
    __device__ __forceinline__ int64_t tile_of(int64_t pos) const {
        return (pos + shift) >> 10;
    }
};

// Streams tiles from the one holding `s0` onward, four tiles in flight ahead
// of the four being processed, until step() returns true.  A hard stop past
// the end of the job guarantees every wave exits.
template <bool INV, class Step>
__device__ __forceinline__ void stream_tiles(const Source& src, int64_t s0,
                                             int64_t n, Step&& step,
                                             uint32_t* err) {
    int64_t t = src.tile_of(s0);
    const int64_t t_end = src.tile_of(n) + 1;
    uint4 b0 = src.load<INV>(t), b1 = src.load<INV>(t + 1);
    uint4 b2 = src.load<INV>(t + 2), b3 = src.load<INV>(t + 3);
    for (;;) {
        if (t > t_end) {
            if (lane_id() == 0) atomicOr(err, kErrOverflow);
            return;
        }
        uint4 c0 = src.load<INV>(t + 4), c1 = src.load<INV>(t + 5);
        uint4 c2 = src.load<INV>(t + 6), c3 = src.load<INV>(t + 7);
        if (step(b0, src.tile_pos(t))) return;
        if (step(b1, src.tile_pos(t + 1))) return;
        if (step(b2, src.tile_pos(t + 2))) return;
        if (step(b3, src.tile_pos(t + 3))) return;
        b0 = c0; b1 = c1; b2 = c2; b3 = c3;
        t += 4;
    }
}

// ------------------------------------------------------------ chain runners

// RAM: extreme byte search over [s, s+w), then a GEQ range scan from s+w.
template <class Sink>
__device__ void run_ram(const Source& src, int64_t n, int64_t w, int64_t M,
                        int64_t s0, Sink& sink, uint32_t* err) {
    int64_t s = 0, L = 0, cur = 0;
    int phase = 0, T = 0;
    uint32_t ahi = 0, alo = 0;

    // Start a chunk at c; true when the chain is finished.
    auto start = [&](int64_t c) -> bool {
        s = c;
        L = min(n, s + M);
        if (s + w >= L) {        // the window does not fit: last chunk ends at n
            sink.cut(L);
            return true;
        }
        phase = 0;
        cur = s;
        ahi = 0;
        alo = 0;
        return false;
    };
    if (start(s0)) return;

    auto step = [&](const uint4& v, int64_t tp) -> bool {
        const int64_t te = tp + kTile;
        for (;;) {
            if (phase == 0) {
                const int64_t we = s + w;
                const int64_t hi = min(we, te);
                uint4 x = v;
                if (cur > tp || hi < te) {
                    const int64_t lp = tp + 16 * (int64_t)lane_id();
                    const int a = (int)min(max(cur - lp, (int64_t)0), (int64_t)16);
                    const int b = (int)min(max(hi - lp, (int64_t)0), (int64_t)16);
                    x = keep_bytes(v, a, b);
                }
                ahi = pkmax(ahi, pkmax(pkmax(x.x, x.y), pkmax(x.z, x.w)));
                alo = pkmax(alo, pkmax(pkmax(x.x << 8, x.y << 8),
                                       pkmax(x.z << 8, x.w << 8)));
                if (we > te) {
                    cur = te;
                    return false;
                }
                const uint32_t m = pkmax(ahi, alo);
                T = (int)wave_max(max(m >> 24, (m >> 8) & 0xFFu));
                phase = 1;
                cur = we;
            }
            const int64_t hi = min(L, te);
            uint32_t val;
            const int64_t j = find_geq(v, tp, cur, hi, T, val);
            int64_t c;
            if (j >= 0)
                c = j + 1;
            else if (L <= te)
                c = L;
            else {
                cur = te;
                return false;
            }
            if (sink.cut(c)) return true;
            if (start(c)) return true;
            if (cur >= te) return false;
        }
    };
    stream_tiles<false>(src, s0, n, step, err);
}

// AE-Max: the target p is a strict record; a GT range scan over (p, p+w]
// either finds the next record or proves none exists, and then the chunk
// ends at p+w+1.  Each byte is examined once.  INV runs AE-Min as AE-Max of
// the complemented bytes.
template <bool INV, class Sink>
__device__ void run_ae(const Source& src, int64_t n, int64_t w, int64_t M,
                       int64_t s0, Sink& sink, uint32_t* err) {
    int64_t L = min(n, s0 + M), p = s0 - 1, cur = s0;
    int thr = 0;  // scan threshold: target value + 1 (0 at a chunk start)
    auto step = [&](const uint4& v, int64_t tp) -> bool {
        const int64_t te = tp + kTile;
        for (;;) {
            const int64_t wend = min(p + w + 1, L);
            uint32_t val;
            const int64_t j = find_geq(v, tp, cur, min(wend, te), thr, val);
            if (j >= 0) {
                p = j;
                thr = (int)val + 1;
                cur = j + 1;
                continue;
            }
            if (wend > te) {
                cur = te;
                return false;
            }
            if (sink.cut(wend)) return true;
            L = min(n, wend + M);
            p = wend - 1;
            thr = 0;
            cur = wend;
            if (cur >= te) return false;
        }
    };
    stream_tiles<INV>(src, s0, n, step, err);
}

// ------------------------------------------------------------ sinks

// Speculation: record every cut (relative to the segment start a) until the
// first cut at or beyond the segment end b (the exit).
struct SpecSink {
    int64_t a, b;
    uint32_t* list;
    uint32_t cap;
    uint32_t* err;
    uint32_t cnt;
    int64_t last;
    __device__ bool cut(int64_t c) {
        if (cnt < cap) {
            if (lane_id() == 0) list[cnt] = (uint32_t)(c - a);
        } else if (lane_id() == 0) {
            atomicOr(err, kErrOverflow);
        }
        cnt++;
        last = c;
        return c >= b;
    }
};

// Membership test against a sorted speculative cut list, 64 entries per
// step held one per lane.
struct SpecWindow {
    const uint32_t* spec;
    uint32_t nspec, wbase, wval, wlast;
    __device__ void load(uint32_t base) {
        wbase = base;
        const uint32_t i = base + lane_id();
        wval = i < nspec ? spec[i] : 0xFFFFFFFFu;
        const uint32_t last = min(nspec - 1 - base, 63u);
        wlast = __builtin_amdgcn_readlane(wval, last);
    }
    // Is r (relative position) in the list?  r must not decrease between
    // calls.  On success idx is its index.
    __device__ bool find(uint32_t r, uint32_t& idx) {
        for (;;) {
            const uint64_t hit = __ballot(wval == r);
            if (hit) {
                idx = wbase + (uint32_t)__builtin_ctzll(hit);
                return true;
            }
            if (r <= wlast || wbase + 64 >= nspec) return false;
            load(wbase + 64);
        }
    }
};

// Fix-up: run from an entry until a cut lands on the speculative chain
// (merge; that cut and everything after it come from the speculation) or
// reaches the segment end without meeting it.
struct FixSink {
    int64_t a, b;
    SpecWindow sw;
    uint32_t* list;
    uint32_t cap;
    uint32_t* err;
    uint32_t cnt;
    uint32_t mi;
    int merged;
    int64_t last;
    __device__ bool cut(int64_t c) {
        uint32_t idx;
        if (sw.find((uint32_t)(c - a), idx)) {
            merged = 1;
            mi = idx;
            return true;
        }
        if (cnt < cap) {
            if (lane_id() == 0) list[cnt] = (uint32_t)(c - a);
        } else if (lane_id() == 0) {
            atomicOr(err, kErrOverflow);
        }
        cnt++;
        last = c;
        if (c >= b) {
            merged = 0;
            return true;
        }
        return false;
    }
};

template <class Sink>
__device__ __forceinline__ void run_algo(uint32_t algo, const Source& src,
                                         int64_t n, int64_t w, int64_t M,
                                         int64_t s0, Sink& sink, uint32_t* err) {
    if (algo == kRam)
        run_ram(src, n, w, M, s0, sink, err);
    else if (algo == kAe)
        run_ae<false>(src, n, w, M, s0, sink, err);
    else
        run_ae<true>(src, n, w, M, s0, sink, err);
}

// ------------------------------------------------------------ job access

struct JobView {
    const uint8_t* data;
    int64_t n, w, M, seg;
    uint32_t algo, nseg, item0, cap, ok, blog;
    uint64_t slot0, blk0;
    uint64_t* cuts;
    uint64_t* n_cuts;
};

__device__ __forceinline__ JobView view(const JobDesc& J) {
    JobView v;
    v.data = (const uint8_t*)uni64((int64_t)J.data);
    v.n = uni64((int64_t)J.n);
    v.w = uni(J.w);
    v.M = uni(J.M);
    v.seg = uni64((int64_t)J.seg);
    v.algo = uni(J.algo);
    v.nseg = uni(J.nseg);
    v.item0 = uni(J.item0);
    v.cap = uni(J.cap);
    v.ok = uni((uint32_t)J.ok);
    v.blog = uni(J.blog);
    v.slot0 = (uint64_t)uni64((int64_t)J.slot0);
    v.blk0 = (uint64_t)uni64((int64_t)J.blk0);
    v.cuts = (uint64_t*)uni64((int64_t)J.cuts);
    v.n_cuts = (uint64_t*)uni64((int64_t)J.n_cuts);
    return v;
}

__device__ __forceinline__ uint32_t wave_global_id() {
    return uni(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
}

__device__ __forceinline__ bool item_of(const Plan& P, uint32_t wid,
                                        JobView& J, uint32_t& seg) {
    if (P.jobs == nullptr) {
        if (wid >= P.one_items) return false;
        J = view(P.one);
        seg = wid;
        return true;
    }
    if (wid >= uni(*P.n_items)) return false;
    const Item it = P.items[wid];
    const uint32_t job = uni(it.job);
    seg = uni(it.seg);
    J = view(P.jobs[job]);
    return true;
}

// ------------------------------------------------------------ RAM / AE

__global__ void k_spec(Plan P, SegMeta* meta, uint32_t* spec, uint32_t* err) {
    JobView J;
    uint32_t seg;
    const uint32_t wid = wave_global_id();
    if (!item_of(P, wid, J, seg) || !J.ok || J.algo == kMaxp) return;
    Source src;
    src.init(J.data, (uint64_t)J.n);
    const int64_t a = (int64_t)seg * J.seg;
    const int64_t b = min(J.n, a + J.seg);
    SpecSink sink{a, b, spec + J.slot0 + (uint64_t)seg * J.cap, J.cap, err, 0,
                  a};
    run_algo(J.algo, src, J.n, J.w, J.M, a, sink, err);
    if (lane_id() == 0) {
        SegMeta& m = meta[wid];
        m.exit = (uint64_t)sink.last;
        m.nspec = min(sink.cnt, J.cap);
    }
}

// Run segment `seg` of job J from `entry` (>= the segment start), writing
// the fix-up record.  Used by the fix-up pass (entry = speculative exit of
// the previous segment) and by the resolve pass (any other entry).
struct FixOutcome {
    uint32_t merged;
    int64_t exit;   // where the true chain leaves the segment
};

__device__ FixOutcome fix_segment(const JobView& J, uint32_t seg, uint32_t item,
                                  int64_t entry, SegMeta* meta,
                                  const uint32_t* spec, uint32_t* fix,
                                  uint32_t* err) {
    const int64_t a = (int64_t)seg * J.seg;
    const int64_t b = min(J.n, a + J.seg);
    const uint64_t slot = J.slot0 + (uint64_t)seg * J.cap;
    SegMeta& m = meta[item];
    const uint32_t nspec = uni(m.nspec);
    const int64_t spec_exit = uni64((int64_t)m.exit);
    FixSink sink;
    sink.a = a;
    sink.b = b;
    sink.sw.spec = spec + slot;
    sink.sw.nspec = nspec;
    sink.sw.load(0);
    sink.list = fix + slot;
    sink.cap = J.cap;
    sink.err = err;
    sink.cnt = 0;
    sink.mi = 0;
    sink.merged = 0;
    sink.last = entry;
    uint32_t idx;
    if (entry == a) {
        sink.merged = 1;
        sink.mi = 0;
    } else if (sink.sw.find((uint32_t)(entry - a), idx)) {
        sink.merged = 1;
        sink.mi = idx + 1;
    } else if (entry >= b) {
        sink.merged = 0;
    } else {
        Source src;
        src.init(J.data, (uint64_t)J.n);
        run_algo(J.algo, src, J.n, J.w, J.M, entry, sink, err);
    }
    const int64_t h = sink.merged ? spec_exit : sink.last;
    if (lane_id() == 0) {
        m.nfix = min(sink.cnt, J.cap);
        m.mi = sink.mi;
        m.merged = (uint32_t)sink.merged;
        m.h = (uint64_t)h;
    }
    return FixOutcome{(uint32_t)sink.merged, h};
}

__global__ void k_fix(Plan P, SegMeta* meta, const uint32_t* spec,
                      uint32_t* fix, uint32_t* err) {
    JobView J;
    uint32_t seg;
    const uint32_t wid = wave_global_id();
    if (!item_of(P, wid, J, seg) || !J.ok || J.algo == kMaxp) return;
    if (seg == 0) {
        if (lane_id() == 0) {
            SegMeta& m = meta[wid];
            m.nfix = 0;
            m.mi = 0;
            m.merged = 1;
            m.h = m.exit;
        }
        return;
    }
    const int64_t entry = uni64((int64_t)meta[wid - 1].exit);
    fix_segment(J, seg, wid, entry, meta, spec, fix, err);
}

__device__ __forceinline__ uint32_t seg_count(const SegMeta& m) {
    return m.nfix + (m.merged ? m.nspec - m.mi : 0u);
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

// Resolve one RAM / AE job (one block per job): re-run the segments whose
// true entry is not the one the fix-up assumed, then assign output offsets.
__global__ void k_resolve(Plan P, uint32_t n_jobs_h, const uint32_t* n_jobs_d,
                          SegMeta* meta, const uint32_t* spec, uint32_t* fix,
                          uint32_t* err) {
    __shared__ uint64_t sh[256];
    __shared__ uint32_t nm_list[256];
    __shared__ uint32_t nm_count;
    __shared__ int64_t carry_x;
    const uint32_t job = blockIdx.x;
    const uint32_t n_jobs = n_jobs_d ? *n_jobs_d : n_jobs_h;
    if (job >= n_jobs) return;
    JobView J = view(P.jobs ? P.jobs[job] : P.one);
    if (!J.ok || J.algo == kMaxp) return;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    SegMeta* M0 = meta + J.item0;
    const bool leader = tid < kWave;  // wave 0 re-runs diverged segments

    // Walk the segments in windows of nt: collect the non-merged segments of
    // the window (their successor's entry differs from the assumed one), and
    // let wave 0 re-run the successors in order.
    if (tid == 0) carry_x = -1;  // -1: entry of the window start is on track
    __syncthreads();
    for (uint32_t base = 0; base < J.nseg; base += nt) {
        if (tid == 0) nm_count = 0;
        __syncthreads();
        const uint32_t k = base + tid;
        if (k + 1 < J.nseg && !M0[k].merged) {
            const uint32_t slot = atomicAdd(&nm_count, 1u);
            nm_list[slot] = k;
        }
        __syncthreads();
        const uint32_t cnt = nm_count;
        if (cnt > 0 || carry_x >= 0) {
            // Sort the (few) indices so the walk goes in order.
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
                // x >= 0: the entry of segment k is x and differs from the
                // speculative exit of segment k-1, so k must be re-run.
                int64_t x = uni64(carry_x);
                uint32_t k2 = base;
                uint32_t li = 0;
                const uint32_t end = min(base + nt, J.nseg);
                while (k2 < end) {
                    if (x < 0) {
                        // on track: jump to the next non-merged segment
                        while (li < cnt && nm_list[li] < k2) li++;
                        if (li == cnt) break;
                        const uint32_t j = uni(nm_list[li]);
                        x = uni64((int64_t)M0[j].h);
                        k2 = j + 1;
                        continue;
                    }
                    // re-run segment k2 from x
                    const FixOutcome o =
                        fix_segment(J, k2, J.item0 + k2, x, meta, spec, fix, err);
                    x = o.merged ? -1 : o.exit;
                    k2++;
                }
                if (lane_id() == 0) carry_x = (k2 >= end) ? x : -1;
            }
            __syncthreads();
        }
    }

    // Output offsets: exclusive scan of the per-segment counts.
    uint64_t carry = 0;
    for (uint32_t base = 0; base < J.nseg; base += nt) {
        const uint32_t k = base + tid;
        const uint64_t c = k < J.nseg ? seg_count(M0[k]) : 0;
        uint64_t total;
        const uint64_t ex = block_exscan(c, sh, total);
        if (k < J.nseg) M0[k].out = carry + ex;
        carry += total;
    }
    if (tid == 0) *J.n_cuts = carry;
}

// Write the offsets of one segment: its fix-up cuts, then its speculative
// cuts from index mi.
__device__ __forceinline__ uint64_t max_cuts_of(const JobView& J) {
    return J.n == 0 ? 0 : (uint64_t)(J.n - 1) / (uint64_t)(J.w + 1) + 1;
}

__global__ void k_emit(Plan P, const SegMeta* meta, const uint32_t* spec,
                       const uint32_t* fix, uint32_t* err) {
    JobView J;
    uint32_t seg;
    const uint32_t wid = wave_global_id();
    if (!item_of(P, wid, J, seg) || !J.ok || J.algo == kMaxp) return;
    const SegMeta& m = meta[wid];
    const uint64_t a = (uint64_t)seg * (uint64_t)J.seg;
    const uint64_t slot = J.slot0 + (uint64_t)seg * J.cap;
    const uint32_t nfix = uni(m.nfix);
    const uint32_t mi = uni(m.mi);
    const uint32_t nsp = uni(m.merged) ? uni(m.nspec) - mi : 0u;
    const uint64_t o = (uint64_t)uni64((int64_t)m.out);
    const uint64_t room = max_cuts_of(J);
    if (o + nfix + nsp > room) {   // cannot happen for a correct chain
        if (lane_id() == 0) atomicOr(err, kErrOverflow);
        return;
    }
    uint64_t* out = J.cuts + o;
    for (uint32_t i = lane_id(); i < nfix; i += kWave)
        out[i] = a + fix[slot + i];
    out += nfix;
    for (uint32_t i = lane_id(); i < nsp; i += kWave)
        out[i] = a + spec[slot + mi + i];
}

// ------------------------------------------------------------ MAXP

// Block summaries.  Blocks are 2^blog bytes aligned in the address space
// (block beta covers positions [beta*B - shift, (beta+1)*B - shift)); bytes
// outside the job count as 0.  For each block: its maximum, and the position
// of that maximum if it occurs exactly once (else -1).  A strict local
// maximum over +-w is the unique maximum of its block whenever B <= w+1.
template <int G>
__device__ void block_summaries(const uint4& v, int64_t tp, int64_t n,
                                uint8_t* bmax, int64_t* bpos, int64_t beta0) {
    const int64_t lp = tp + 16 * (int64_t)lane_id();
    uint4 x = v;
    if (lp < 0 || lp + 16 > n) {
        const int a = (int)min(max(-lp, (int64_t)0), (int64_t)16);
        const int b = (int)min(max(n - lp, (int64_t)0), (int64_t)16);
        x = keep_bytes(v, a, b);
    }
    const uint32_t lm = lane_max16(x);
    const uint32_t gm_partial = seg_max<G>(lm);
    const uint32_t last = lane_id() | (G - 1);
    const uint32_t gm = (uint32_t)__shfl((int)gm_partial, (int)last);
    const uint32_t eq = (lm == gm) ? 1u : 0u;
    const uint32_t cnt_partial = seg_sum<G>(eq);
    const uint32_t cnt = (uint32_t)__shfl((int)cnt_partial, (int)last);
    const int64_t beta = beta0 + (int64_t)(lane_id() / G);
    if (cnt != 1) {
        if (lane_id() == last) {
            bmax[beta] = (uint8_t)gm;
            bpos[beta] = -1;
        }
    } else if (eq) {
        // the only lane holding the maximum: is it unique among its bytes?
        const uint32_t r = gm * 0x01010101u;
        uint32_t nz = 0, first = 16;
        const uint32_t d[4] = {x.x ^ r, x.y ^ r, x.z ^ r, x.w ^ r};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            // high bit of each byte set iff that byte is zero
            uint32_t t = (d[i] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
            t = ~(t | d[i] | 0x7F7F7F7Fu);
            nz += __builtin_popcount(t);
            if (t && first == 16) first = 4 * i + (__builtin_ctz(t) >> 3);
        }
        bmax[beta] = (uint8_t)gm;
        bpos[beta] = (nz == 1 && gm > 0) ? lp + first : -1;
    }
}

__global__ void k_maxp_blocks(Plan P, uint8_t* bmax, int64_t* bpos,
                              uint32_t* err) {
    JobView J;
    uint32_t seg;
    const uint32_t wid = wave_global_id();
    if (!item_of(P, wid, J, seg) || !J.ok || J.algo != kMaxp || J.blog == 0)
        return;
    Source src;
    src.init(J.data, (uint64_t)J.n);
    // Tiles owned by this segment: those whose first position lies in
    // [a, b) (tile 0 also owns the bytes before position 0).
    const int64_t a = (int64_t)seg * J.seg;
    const int64_t b = min(J.n, a + J.seg);
    int64_t t0 = (a + src.shift + kTile - 1) >> 10;
    if (seg == 0) t0 = 0;
    const int64_t t1 = (b >= J.n) ? ((J.n + src.shift + kTile - 1) >> 10)
                                  : ((b + src.shift + kTile - 1) >> 10);
    const int blog = (int)J.blog;
    const int64_t per_tile = (int64_t)kTile >> blog;   // blocks per tile
    uint8_t* bm = bmax + J.blk0;
    int64_t* bp = bpos + J.blk0;
    for (int64_t t = t0; t < t1; t++) {
        const uint4 v = src.load<false>(t);
        const int64_t tp = src.tile_pos(t);
        const int64_t beta0 = t * per_tile;
        switch (blog) {
            case 4: block_summaries<1>(v, tp, J.n, bm, bp, beta0); break;
            case 5: block_summaries<2>(v, tp, J.n, bm, bp, beta0); break;
            case 6: block_summaries<4>(v, tp, J.n, bm, bp, beta0); break;
            case 7: block_summaries<8>(v, tp, J.n, bm, bp, beta0); break;
            case 8: block_summaries<16>(v, tp, J.n, bm, bp, beta0); break;
            case 9: block_summaries<32>(v, tp, J.n, bm, bp, beta0); break;
            default: block_summaries<64>(v, tp, J.n, bm, bp, beta0); break;
        }
    }
}

__device__ __forceinline__ uint32_t byte_at(const uint8_t* d, int64_t p) {
    return d[p];
}

// Exact check that every byte in [lo, hi] is below v.
__device__ bool all_below(const uint8_t* d, int64_t lo, int64_t hi, uint32_t v) {
    for (int64_t p = lo; p <= hi; p++)
        if (byte_at(d, p) >= v) return false;
    return true;
}

// Strict local maximum test of position i (w <= i <= n-1-w) from the block
// summaries: whole blocks inside the window by their maxima, the two partial
// end blocks by their maxima or, when that is not enough, byte by byte.
__device__ bool maxp_verify(const JobView& J, const uint8_t* bm, int64_t shift,
                            int64_t i, uint32_t v) {
    const int blog = (int)J.blog;
    const int64_t lo = i - J.w, hi = i + J.w;
    const int64_t bi = (i + shift) >> blog;
    const int64_t bl = (lo + shift) >> blog, br = (hi + shift) >> blog;
    for (int64_t beta = bl + 1; beta < bi; beta++)
        if (bm[beta] >= v) return false;
    for (int64_t beta = bi + 1; beta < br; beta++)
        if (bm[beta] >= v) return false;
    if (bl < bi && bm[bl] >= v) {
        const int64_t end = ((bl + 1) << blog) - shift - 1;
        if (!all_below(J.data, lo, end, v)) return false;
    }
    if (br > bi && bm[br] >= v) {
        const int64_t start = (br << blog) - shift;
        if (!all_below(J.data, start, hi, v)) return false;
    }
    return true;
}

// Candidates of one segment, in increasing order, relative to the segment
// start a (positions in [a, b) for the direct path; for the block path, the
// unique maxima of the blocks whose summaries this segment wrote).
__global__ void k_maxp_verify(Plan P, const uint8_t* bmax, const int64_t* bpos,
                              SegMeta* meta, uint32_t* cand, uint32_t* err) {
    JobView J;
    uint32_t seg;
    const uint32_t wid = wave_global_id();
    if (!item_of(P, wid, J, seg) || !J.ok || J.algo != kMaxp) return;
    const int64_t a = (int64_t)seg * J.seg;
    const int64_t b = min(J.n, a + J.seg);
    uint32_t* out = cand + J.slot0 + (uint64_t)seg * J.cap;
    uint32_t cnt = 0;
    const int64_t lo_ok = J.w, hi_ok = J.n - 1 - J.w;   // full windows
    if (J.blog == 0) {
        // Direct test of every position (small windows).
        for (int64_t base = a; base < b; base += kWave) {
            const int64_t i = base + lane_id();
            bool c = false;
            if (i < b && i >= lo_ok && i <= hi_ok) {
                const uint32_t v = byte_at(J.data, i);
                c = all_below(J.data, i - J.w, i - 1, v) &&
                    all_below(J.data, i + 1, i + J.w, v);
            }
            const uint64_t ball = __ballot(c);
            const uint32_t rank = __builtin_popcountll(ball & ((1ull << lane_id()) - 1));
            if (c) {
                if (cnt + rank < J.cap)
                    out[cnt + rank] = (uint32_t)(i - a);
                else
                    atomicOr(err, kErrOverflow);
            }
            cnt += (uint32_t)__builtin_popcountll(ball);
        }
    } else {
        Source src;
        src.init(J.data, (uint64_t)J.n);
        const int blog = (int)J.blog;
        const int64_t per_tile = (int64_t)kTile >> blog;
        int64_t t0 = (a + src.shift + kTile - 1) >> 10;
        if (seg == 0) t0 = 0;
        const int64_t t1 = (b >= J.n) ? ((J.n + src.shift + kTile - 1) >> 10)
                                      : ((b + src.shift + kTile - 1) >> 10);
        const uint8_t* bm = bmax + J.blk0;
        const int64_t* bp = bpos + J.blk0;
        for (int64_t beta = t0 * per_tile; beta < t1 * per_tile; beta += kWave) {
            const int64_t bb = beta + lane_id();
            bool c = false;
            int64_t i = -1;
            if (bb < t1 * per_tile) {
                i = bp[bb];
                if (i >= lo_ok && i <= hi_ok)
                    c = maxp_verify(J, bm, src.shift, i, bm[bb]);
            }
            const uint64_t ball = __ballot(c);
            const uint32_t rank = __builtin_popcountll(ball & ((1ull << lane_id()) - 1));
            if (c) {
                if (cnt + rank < J.cap)
                    out[cnt + rank] = (uint32_t)(i - a);
                else
                    atomicOr(err, kErrOverflow);
            }
            cnt += (uint32_t)__builtin_popcountll(ball);
        }
    }
    if (lane_id() == 0) meta[wid].nspec = min(cnt, J.cap);
}

// The MAXP chain over the candidates (one wave per job).  From a chunk start
// s a candidate q is a boundary iff (q - s) mod M >= w: the forced cuts
// s+M, s+2M, ... in between leave it at least w bytes into its chunk.  After
// a boundary the next candidate is accepted directly unless it lies more
// than M bytes further on, so runs of accepted candidates are taken 64 at a
// time.
__device__ __forceinline__ void put_forced(uint64_t* out, uint64_t& cnt,
                                           uint64_t room, int64_t s, int64_t t,
                                           int64_t M) {
    for (int64_t i = lane_id(); i < t; i += kWave)
        if (cnt + i < room) out[cnt + i] = (uint64_t)(s + (i + 1) * M);
    cnt += (uint64_t)t;
}

__global__ void k_maxp_chain(Plan P, uint32_t n_jobs_h, const uint32_t* n_jobs_d,
                             const SegMeta* meta, const uint32_t* cand,
                             uint32_t* err) {
    const uint32_t job = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint32_t n_jobs = n_jobs_d ? *n_jobs_d : n_jobs_h;
    if (uni(job) >= n_jobs) return;
    JobView J = view(P.jobs ? P.jobs[uni(job)] : P.one);
    if (!J.ok || J.algo != kMaxp) return;
    const int64_t n = J.n, w = J.w, M = J.M;
    uint64_t* out = J.cuts;
    const uint64_t room = max_cuts_of(J);
    uint64_t cnt = 0;
    int64_t s = 0;
    for (uint32_t seg = 0; seg < J.nseg; seg++) {
        const uint32_t nc = uni(meta[J.item0 + seg].nspec);
        const uint32_t* list = cand + J.slot0 + (uint64_t)seg * J.cap;
        const int64_t a = (int64_t)seg * J.seg;
        for (uint32_t base = 0; base < nc; base += kWave) {
            const uint32_t k = base + lane_id();
            const bool valid = k < nc;
            const int64_t q = valid ? a + (int64_t)list[k] : INT64_MAX;
            int64_t qprev = __shfl_up(q, 1);
            uint32_t done = 0;  // lanes below `done` are settled
            for (;;) {
                const bool acc = valid && lane_id() >= done && q >= s &&
                                 ((q - s) % M) >= w;
                const uint64_t ball = __ballot(acc);
                if (ball == 0) break;
                const uint32_t f = (uint32_t)__builtin_ctzll(ball);
                const int64_t qf = uni64(__shfl(q, (int)f));
                // accepted run: f, then every next candidate within M+1 bytes
                const bool brk = lane_id() > f &&
                                 (!valid || (q - qprev - 1) >= M);
                const uint64_t bb = __ballot(brk);
                const uint32_t g = bb ? (uint32_t)__builtin_ctzll(bb) : 64u;
                put_forced(out, cnt, room, s, (qf - s) / M, M);
                if (lane_id() >= f && lane_id() < g &&
                    cnt + (lane_id() - f) < room)
                    out[cnt + (lane_id() - f)] = (uint64_t)(q + 1);
                cnt += g - f;
                s = uni64(__shfl(q, (int)(g - 1))) + 1;
                done = g;
                if (g >= 64) break;
            }
        }
    }
    if (n > 0) {
        put_forced(out, cnt, room, s, (n - s - 1) / M, M);
        if (lane_id() == 0 && cnt < room) out[cnt] = (uint64_t)n;
        cnt++;
    }
    if (cnt > room) {   // cannot happen for a correct chain
        if (lane_id() == 0) atomicOr(err, kErrOverflow);
        cnt = room;
    }
    if (lane_id() == 0) *J.n_cuts = cnt;
}

// ------------------------------------------------------------ launches

__global__ void k_set_u64(uint64_t* p, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_clear_u32(uint32_t* p, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_set_u64(uint64_t* p, uint64_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

hipError_t launch_clear_u32(uint32_t* p, size_t count, hipStream_t st) {
    const uint32_t grid = (uint32_t)min((count + 255) / 256, (size_t)1024);
    hipLaunchKernelGGL(k_clear_u32, dim3(grid > 0 ? grid : 1), dim3(256), 0,
                       st, p, count);
    return hipGetLastError();
}

hipError_t launch_ram_ae(const Plan& P, uint32_t items_upper,
                         uint32_t jobs_upper, const uint32_t* n_jobs_d,
                         SegMeta* meta, uint32_t* spec, uint32_t* fix,
                         uint32_t* err, int wpb, hipStream_t st) {
    const dim3 blk(kWave * wpb), grid((items_upper + wpb - 1) / wpb);
    hipLaunchKernelGGL(k_spec, grid, blk, 0, st, P, meta, spec, err);
    hipLaunchKernelGGL(k_fix, grid, blk, 0, st, P, meta, spec, fix, err);
    hipLaunchKernelGGL(k_resolve, dim3(jobs_upper), dim3(256), 0, st, P,
                       jobs_upper, n_jobs_d, meta, spec, fix, err);
    hipLaunchKernelGGL(k_emit, grid, blk, 0, st, P, meta, spec, fix, err);
    return hipGetLastError();
}

hipError_t launch_maxp(const Plan& P, uint32_t items_upper, uint32_t jobs_upper,
                       const uint32_t* n_jobs_d, SegMeta* meta, uint32_t* cand,
                       uint8_t* bmax, int64_t* bpos, uint32_t* err, int wpb,
                       bool any_blocks, hipStream_t st) {
    const dim3 blk(kWave * wpb), grid((items_upper + wpb - 1) / wpb);
    if (any_blocks)
        hipLaunchKernelGGL(k_maxp_blocks, grid, blk, 0, st, P, bmax, bpos, err);
    hipLaunchKernelGGL(k_maxp_verify, grid, blk, 0, st, P, bmax, bpos, meta,
                       cand, err);
    const uint32_t jgrid = (jobs_upper + 3) / 4;
    hipLaunchKernelGGL(k_maxp_chain, dim3(jgrid), dim3(256), 0, st, P,
                       jobs_upper, n_jobs_d, meta, cand, err);
    return hipGetLastError();
}

}  // namespace cdc

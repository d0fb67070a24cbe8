// RAM and AE chunk chains on gfx950: tile index, speculate, fix up,
// resolve, emit.
//
// RAM (Section 2.1 "RAM"; Section 4.3) is one extreme byte search over the
// first w bytes of a chunk followed by a greater-or-equal range scan from
// the first byte after them.  AE-Max (Section 2.1 "AE"; Section 4.3) moves
// its target to each greater byte until the w bytes after the target hold
// none; the walker takes it as "the first occurrence of the largest byte of
// [p, p + w]": the records between p and that occurrence are each followed
// by a greater byte within w, so the target reaches it, and the chunk ends
// w bytes after a target that is its own window's first maximum.  AE-Min
// runs as AE-Max of the complemented bytes.  Both patterns are answered
// from the tile index (tile_index.h), so a walker's step costs a few
// ballots over 64 tile summaries, not a pass over the chunk's bytes.
//
// The chain (cut k+1 depends on cut k) is split into segments.  Speculation
// runs one walker per segment from the segment start and records its cuts up
// to the first one at or past the segment end (its exit).  The fix-up pass
// runs each segment from the previous segment's speculative exit until a cut
// lands on the speculative list (the two chains coincide from there).  A
// segment whose fix-up never lands hands its successor an entry that the
// fix-up did not assume; parallel rounds re-walk exactly those successors
// (landing on either recorded list), and an ordered pass per job settles
// what is left.  The emit pass copies every segment's resolved pieces.
#include "tile_index.h"

namespace cdc {

// Positions inside the chain engine are 32-bit offsets from the segment
// start (segments and chunks are at most 2^28 bytes, so every position a
// walker of the segment reaches fits), which keeps the walkers' state and
// compares on the scalar unit.

// ------------------------------------------------------------ index pass

// Waves per item of the index pass.  A single call uses sixteen: each wave's
// share of the segment is smaller, and the waves finish together better
// than four (190 against 209 us per GiB on the mixed stream).  A batch
// keeps four: beside the other algorithms' passes, workgroups of sixteen
// waves made the three-job step slower (0.93 against 0.84 ms).
template <bool ONE>
constexpr int idx_threads() { return ONE ? 1024 : 256; }
constexpr int kIdxThreadsMax = 1024;
constexpr int kIdxAhead = 4;                     // tile loads in flight per wave

// Summaries of the tiles owned by one segment (those whose first byte lies
// in [a, b); tile 0 also owns the bytes before position 0), shared by the
// waves of the workgroup.
template <bool INV>
__device__ void index_item(const JobView& J, uint32_t seg, uint4* idx,
                           uint16_t* slots) {
    Source src;
    src.init(J.data, (uint64_t)J.n);
    const int64_t a = (int64_t)seg * J.seg;
    const int64_t b = min(J.n, a + J.seg);
    int64_t t0 = (a + src.shift + kTile - 1) >> 10;
    if (seg == 0) t0 = 0;
    const int64_t t1 = (b + src.shift + kTile - 1) >> 10;
    uint4* out = idx + J.idx0;
    const int64_t nw = blockDim.x / kWave, wv = uni(threadIdx.x / kWave);
    uint32_t guess = 255;
    for (int64_t t = t0 + wv * kIdxAhead; t < t1; t += nw * kIdxAhead) {
        uint4 v[kIdxAhead];
#pragma unroll
        for (int i = 0; i < kIdxAhead; i++)
            v[i] = t + i < t1 ? src.load<INV>(t + i) : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < kIdxAhead; i++) {
            if (t + i < t1) {
                const int64_t tp = src.tile_pos(t + i);
                const bool whole = tp >= 0 && tp + kTile <= J.n;
                const uint4 e = summarize_tile<INV>(v[i], tp, J.n, whole, slots, guess);
                guess = ie_max(e.x);
                if (lane_id() == 0) out[t + i] = e;
            }
        }
    }
}

// ------------------------------------------------------------ successor pass

// Each stored position P of a tile's maximum is a possible chain node: for
// RAM, the byte a cut lands right after (it is at or above its window's
// maximum, and where the summaries decide a step that byte is its tile's
// maximum); for AE, a final target (the cut lands w + 1 bytes after it).
// This pass works out, from the summaries alone, where the chain goes from
// every node: the node of the next cut, a forced cut (the chunk reaches
// max_chunk), the job's end, or "unknown" where the summaries cannot decide.
// A walker standing on a node then takes the step as one lookup; on
// "unknown" it takes the step itself.  Every answer recorded here is exact.
// Waves per item: eight for a single call (54 against 57 us per GiB with
// four), four in a batch (as the index pass); 64 tiles per wave at a time.
template <bool ONE>
constexpr int succ_threads() { return ONE ? 512 : 256; }
constexpr int kSuccThreadsMax = 512;
constexpr int kSuccSpan = 2 * kWave;             // tiles a wave sees: its 64 and 64 after
constexpr int kSuccScan = 8;                     // tiles a range scan may cross

// The summaries of tiles q .. q + 127 of one job, in LDS.  Positions are
// 32-bit offsets from the first byte of tile q (tile j of the page starts
// at 1024 j), and n is the job's end in the same terms (clamped far out).
struct SuccPages {
    const uint4* pg;
    int32_t n;

    __device__ static bool has(int32_t k) { return k < kSuccSpan; }
    __device__ uint4 ent(int32_t k) const { return pg[k]; }
    __device__ uint32_t word0(int32_t k) const { return pg[k].x; }
    __device__ static int32_t ts(int32_t k) { return k << 10; }
    __device__ static int32_t tile(int32_t pos) { return pos >> 10; }

    // first stored position >= a of a summary, with its slot (kNoPos if none)
    __device__ static uint32_t first_stored(const uint4& E, uint32_t a, uint32_t& slot) {
        const uint32_t ps[7] = {E.x >> 16, E.y & 0xFFFFu, E.y >> 16, E.z & 0xFFFFu,
                                E.z >> 16, E.w & 0xFFFFu, E.w >> 16};
        uint32_t f = kNoPos;
        slot = 7;
#pragma unroll
        for (int i = 6; i >= 0; i--) {
            slot = ps[i] >= a ? (uint32_t)i : slot;
            f = ps[i] >= a ? ps[i] : f;
        }
        return f;
    }
    // max(M, largest byte of [lo, hi) within tile k), or -1 if undecided
    __device__ int32_t part_max(int32_t k, int32_t lo, int32_t hi, int32_t M) const {
        const uint32_t x = word0(k);
        const int32_t m = (int32_t)ie_max(x);
        if (m <= M) return M;
        if (ie_all(x)) return m;
        uint32_t sl;
        const uint32_t f = first_stored(ent(k), (uint32_t)max(lo - ts(k), 0), sl);
        return f != kNoPos && (int32_t)f < hi - ts(k) ? m : -1;
    }
    // largest byte of [lo, hi) (lo < hi), or -1 if undecided
    __device__ int32_t range_max(int32_t lo, int32_t hi) const {
        const int32_t ka = tile(lo), kb = tile(hi - 1);
        if (!has(kb)) return -1;
        if (ka == kb) return part_max(ka, lo, hi, -1);
        int32_t I = 0;
        for (int32_t k = ka + 1; k < kb && I < 255; k++) I = max(I, (int32_t)ie_max(word0(k)));
        if (I == 255) return 255;
        I = part_max(ka, lo, hi, I);
        if (I < 0) return -1;
        return part_max(kb, lo, hi, I);
    }
    // first byte >= T (1..255) in [lo, hi): 1 and its tile, slot and offset
    // when a summary names it, 0 when there is none, -1 if undecided
    __device__ int first_geq(int32_t lo, int32_t hi, uint32_t T, int32_t& k_out,
                             uint32_t& slot, uint32_t& off) const {
        const int32_t k0 = tile(lo), k1 = tile(hi - 1);
        for (int32_t k = k0; k <= k1; k++) {
            // (a scan longer than a few tiles is left to the walker: a lane
            // that scans holds up its whole wave)
            if (!has(k) || k - k0 >= kSuccScan) return -1;
            const uint32_t x = word0(k);
            const uint32_t m = ie_max(x);
            if (m < T) continue;
            if (m > T || ie_all(x)) return -1;
            const uint32_t f = first_stored(ent(k), k == k0 ? (uint32_t)(lo - ts(k)) : 0u, slot);
            if (f != kNoPos) {
                if (ts(k) + (int32_t)f >= hi) return 0;
                k_out = k;
                off = f;
                return 1;
            }
            if (ie_cnt(x) > (uint32_t)kIdxPos) return -1;
        }
        return 0;
    }
};

// Successor word of the node at page position P in page tile u: the node
// that ends the chunk starting right after P (RAM) or w + 1 bytes after P
// (AE).
template <bool RAM>
__device__ uint32_t succ_of(const SuccPages& G, int32_t u, int32_t P, int32_t w,
                            int32_t M) {
    const int32_t n = G.n;
    int32_t k;
    uint32_t slot, off;
    if constexpr (RAM) {
        const int32_t c = P + 1, L = min(c + M, n);
        if (c + w >= L) return L == n ? kSuccEnd : kSuccUnknown;
        const int32_t T = G.range_max(c, c + w);
        if (T <= 0) return kSuccUnknown;
        const int r = G.first_geq(c + w, L, (uint32_t)T, k, slot, off);
        if (r < 0) return kSuccUnknown;
        if (r == 0) return L == n ? kSuccEnd : kSuccForced;
    } else {
        // the target: the first occurrence p of the largest byte V of
        // [c, c + w], final when no byte of (c + w, p + w] exceeds V
        const int32_t c = P + w + 1;
        if (c >= n) return kSuccUnknown;
        const int32_t L = min(c + M, n), hi = min(c + w + 1, L);
        const int32_t V = G.range_max(c, hi);
        if (V <= 0) return kSuccUnknown;
        if (G.first_geq(c, hi, (uint32_t)V, k, slot, off) != 1) return kSuccUnknown;
        const int32_t p = G.ts(k) + (int32_t)off;
        const int32_t nhi = min(p + w + 1, L);
        if (V < 255 && nhi > hi) {
            // (whole tiles, so bytes before hi, none above V, count too)
            const int32_t k1 = G.tile(nhi - 1);
            if (!G.has(k1)) return kSuccUnknown;
            for (int32_t j = G.tile(hi); j <= k1; j++)
                if ((int32_t)ie_max(G.word0(j)) > V) return kSuccUnknown;
        }
        if (p + w >= L) return L == n ? kSuccEnd : kSuccForced;
    }
    return (uint32_t)(k - u) << 23 | slot << 20 | off;
}

// Successor words of the tiles owned by one segment (as the index pass).
template <bool RAM>
__device__ void succ_item(const JobView& J, uint32_t seg, const uint4* idx,
                          uint32_t* succ, uint4* pg) {
    if (J.nseg < 2) return;                        // (walked once, without them)
    Source src;
    src.init(J.data, (uint64_t)J.n);
    const int64_t a = (int64_t)seg * J.seg;
    const int64_t b = min(J.n, a + J.seg);
    int64_t t0 = (a + src.shift + kTile - 1) >> 10;
    if (seg == 0) t0 = 0;
    const int64_t t1 = (b + src.shift + kTile - 1) >> 10;
    const int64_t ntiles = (J.n + src.shift + kTile - 1) >> 10;
    const uint4* jidx = idx + J.idx0;
    uint32_t* jsucc = succ + J.idx0 * kSuccSlots;
    const int64_t nw = blockDim.x / kWave, wv = uni(threadIdx.x / kWave);
    const int l = (int)lane_id();
    // (windows and chunks are below 2^28 bytes, so 32-bit page offsets hold
    // every position a node's step reaches)
    const int32_t w = (int32_t)J.w, M = (int32_t)J.M;
    for (int64_t q = t0 + wv * kWave; q < t1; q += nw * kWave) {
        __builtin_amdgcn_wave_barrier();
        for (int h = 0; h < kSuccSpan; h += kWave) {
            const int64_t t = q + h + l;
            pg[h + l] = t < ntiles ? jidx[t] : make_uint4(0, 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
        const int64_t base = q * kTile - src.shift;          // page offset 0
        SuccPages G{pg, (int32_t)min(J.n - base, (int64_t)0x3FFFFFFF)};
        if (q + l < t1) {
            const uint4 E = G.ent(l);
            // (a tile of one value: a walker steps over it by itself, and no
            // successor word names a position in it)
            const uint32_t cnt = ie_all(E.x) ? 0u : min(ie_cnt(E.x), (uint32_t)kIdxPos);
            uint32_t o[kSuccSlots];
#pragma unroll
            for (int i = 0; i < (int)kSuccSlots; i++) o[i] = kSuccUnknown;
            for (uint32_t i = 0; i < (uint32_t)kIdxPos; i++) {
                if (i >= cnt) break;
                const uint32_t word = i == 0 ? E.x : i <= 2 ? E.y : i <= 4 ? E.z : E.w;
                const uint32_t pos = i == 0 ? word >> 16 : (i & 1) ? word & 0xFFFFu : word >> 16;
                const uint32_t r = succ_of<RAM>(G, l, SuccPages::ts(l) + (int32_t)pos, w, M);
#pragma unroll
                for (int j = 0; j < kIdxPos; j++) o[j] = (uint32_t)j == i ? r : o[j];
            }
            uint4* dst = (uint4*)(jsucc + (q + l) * kSuccSlots);
            dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
            dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
        }
    }
}

// ------------------------------------------------------------ next()

// One chain step from chunk start s (offset from the walker's base): the
// chunk's exclusive end.
template <bool RAM, bool INV>
__device__ __forceinline__ int32_t chain_next(IdxWalker<INV>& X, int32_t s,
                                              int32_t w, int32_t M) {
    const int32_t L = s + M < X.n ? s + M : X.n;   // (no overflow: s, M < 2^29)
    if constexpr (RAM) {
        if (s + w >= L) return L;                  // the window does not fit
        const uint32_t T = X.range_max(s, s + w);
        if (T == 0) return s + w + 1;              // every byte is >= 0
        const int32_t j = X.first_geq(s + w, L, T);
        return j >= 0 ? j + 1 : L;
    } else {
        // the first occurrence q of the largest byte V of [s, s + w] is
        // where the target goes; from there only the window's new part,
        // past what was searched, can hold a greater byte
        int32_t hi = min(s + w + 1, L);
        uint32_t V = X.range_max(s, hi);
        int32_t p = V == 0 ? s : X.first_geq(s, hi, V);
        for (;;) {
            // a target of 255 cannot be exceeded: it is the last one
            if (V == 255u) break;
            const int32_t nhi = min(p + w + 1, L);
            if (nhi <= hi) break;                  // nothing new: p is final
            const uint32_t m2 = X.range_max(hi, nhi);
            if (m2 <= V) break;                    // nothing greater after p
            p = X.first_geq(hi, nhi, m2);
            V = m2;
            hi = nhi;
        }
        return p + w < L ? p + w + 1 : L;
    }
}

// Walk from chunk start `start` (relative to base); emit(c) gets each chunk
// end (relative) and returns true to stop.  The walk also stops at the
// job's end.  Inside a run of whole tiles of one value, every chunk whose
// w + 1 bytes lie in the run is exactly w + 1 long for RAM (its window's
// maximum is the value and the next byte equals it) and for AE (nothing in
// its window exceeds the first byte), so those ends follow without queries.
// Returns the tiles whose bytes the two patterns read (extreme byte search
// in the low half, range scan in the high half).
template <bool RAM, bool INV, bool SUCC, class Emit>
__device__ uint32_t walk(const JobView& J, const ChainWs& ws, int64_t base,
                         int32_t start, Emit& emit, uint32_t* steps = nullptr) {
    // chunks by how each step was decided, one count per lane 0..3 (kept
    // only when `steps` is given)
    uint32_t nk = 0;
    const uint32_t lk = lane_id();
    IdxWalker<INV> X;
    // successor words are built for jobs of several segments only (a job of
    // one segment is walked once, and the pass cost as much as it saved),
    // and for AE only where the launch asks for them (SUCC)
    const bool use_succ = SUCC && J.nseg > 1;
    X.init(J, ws.idx + J.idx0, use_succ ? ws.succ + J.idx0 * kSuccSlots : nullptr, base);
    const int32_t w = (int32_t)J.w, M = (int32_t)J.M;
    // a cut lands 1 byte (RAM) or w + 1 bytes (AE) after its node
    const int32_t delta = RAM ? 1 : w + 1;
    int32_t s = start;
    int32_t nt = 0, ns = -1;           // the node of the cut at s (ns < 0: none)
    bool stop = false;
    while (s < X.n && !stop) {
        if (SUCC && ns >= 0) {
            // on a node: successor words, one lane read per chunk, until a
            // word names no node
            uint32_t sw;
            for (;;) {
                X.ahead(nt);
                sw = X.succ_word(nt - X.p0, (uint32_t)ns);
                if (sw >= kSuccForced) break;
                nt += (int32_t)(sw >> 23);
                ns = (int32_t)((sw >> 20) & 7u);
                const int32_t c = X.tstart(nt) + (int32_t)(sw & 1023u) + delta;
                nk += lk == 0;
                if (emit(c)) {
                    stop = true;
                    break;
                }
                s = c;
            }
            if (stop) break;
            ns = -1;
            const int32_t c = sw == kSuccForced ? s + M : sw == kSuccEnd ? X.n : -1;
            if (c > s) {
                nk += lk == 0;
                if (emit(c)) break;
                s = c;
                continue;
            }
        }
        {
            const int32_t L = s + M < X.n ? s + M : X.n;
            int32_t c = -1;
            X.hit_s = -1;
            if constexpr (RAM) {
                if (s + w < L) c = X.ram_fast(s, w, L);
            } else {
                c = X.ae_fast(s, w, L);
            }
            if (c >= 0) {
                nt = X.hit_t;
                ns = use_succ ? X.hit_s : -1;
                nk += lk == 1;
                if (emit(c)) break;
                s = c;
                continue;
            }
        }
        const int32_t re = X.const_run_end(s, w);
        if (re >= 0) {
            while (s + w <= re - 1) {
                const int32_t c = s + w + 1;
                nk += lk == 2;
                if (emit(c)) {
                    stop = true;
                    break;
                }
                s = c;
            }
            continue;
        }
        const int32_t c = chain_next<RAM, INV>(X, s, w, M);
        nk += lk == 3;
        if (emit(c)) break;
        s = c;
    }
    if (steps != nullptr && lk < 4) steps[lk] = nk;
    return min(X.reads_ebs, 0xFFFFu) | (min(X.reads_rs, 0xFFFFu) << 16);
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

template <bool RAM, bool INV, bool SUCC>
__device__ void speculate(const JobView& J, uint32_t seg, uint32_t item,
                          const ChainWs& ws) {
    const int64_t a = (int64_t)seg * J.seg;
    const int32_t b = (int32_t)(min(J.n, a + J.seg) - a);
    CutList out;
    out.init(list_of(J, ws, seg, kListSpec), J.cap, ws.err);
    int32_t last = 0;
    auto emit = [&](int32_t c) -> bool {
        out.push((uint32_t)c);
        last = c;
        return c >= b;
    };
    const uint32_t reads = walk<RAM, INV, SUCC>(J, ws, a, 0, emit, ws.meta[item].steps);
    out.finish();
    if (lane_id() == 0) {
        SegMeta& m = ws.meta[item];
        m.exit = (uint64_t)(a + last);
        m.nspec = min(out.n, J.cap);
        m.reads = reads;
    }
}

// ------------------------------------------------------------ resolve

// Resolve segment `seg` from entry X (absolute, >= the segment start): the
// chain from X is followed until a cut lands on the speculative list (or,
// after the fix-up round, on the fix-up list, whose continuation is known);
// the cuts before that are written to the fix-up list (fix-up round) or the
// re-walk list.  Records the resolution (entry, pieces, count, exit) and
// returns its exit.  One wave.
template <bool RAM, bool INV, bool SUCC>
__device__ int64_t resolve_from(const JobView& J, uint32_t seg, uint32_t item,
                                int64_t X, bool fixup, const ChainWs& ws) {
    const int64_t a = (int64_t)seg * J.seg;
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
            if (lane_id() == 0) m.pieces[np] = Piece{list, lo, hi};
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
    uint32_t reads = 0;
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
        reads = walk<RAM, INV, SUCC>(J, ws, a, e, emit);
        wl.finish();
        new_nfix = min(wl.n, J.cap);
    }
    if (lane_id() == 0) {
        if (fixup) {
            m.nfix = new_nfix;
            m.fms = new_fms;
            m.fexit = (uint64_t)new_fexit;
        }
        m.npieces = np;
        m.count = count;
        m.entry = (uint64_t)X;
        m.rexit = (uint64_t)rexit;
        const uint32_t r0 = m.reads;               // two saturating halves
        m.reads = min((r0 & 0xFFFFu) + (reads & 0xFFFFu), 0xFFFFu) |
                  (min((r0 >> 16) + (reads >> 16), 0xFFFFu) << 16);
    }
    return rexit;
}

// ------------------------------------------------------------ kernels

// The per-item passes run one wave per item: with one job the grid covers
// its segments; with a job table the waves walk the algorithm's range of
// the item table grid-stride.
constexpr int kChainThreads = 256;
constexpr int kChainWaves = kChainThreads / kWave;
constexpr uint32_t kSettleList = 1024;   // flagged segments settled per pass

template <bool ONE, class F>
__device__ __forceinline__ void for_items(const Plan& P, uint32_t want, F&& f) {
    const uint32_t wv = uni(threadIdx.x / kWave);
    if constexpr (ONE) {
        const uint32_t wid = uni(blockIdx.x) * kChainWaves + wv;
        if (wid >= P.one_items) return;
        const JobView J = view(P.one);
        if (J.ok && J.algo == want) f(J, wid, wid);
    } else {
        uint32_t first, last;
        item_range(P, want, first, last);
        const uint32_t stride = gridDim.x * kChainWaves;
        for (uint32_t wid = first + uni(blockIdx.x) * kChainWaves + wv; wid < last;
             wid += stride) {
            const Item it = P.items[wid];
            const JobView J = view(P.jobs[uni(it.job)]);
            if (J.ok && J.algo == want) f(J, uni(it.seg), wid);
        }
    }
}

// Index pass: one workgroup per item (its waves share the item's tiles).
template <bool INV, bool ONE>
__global__ __launch_bounds__(idx_threads<ONE>()) void k_index(Plan P, ChainWs ws,
                                                       uint32_t want) {
    __shared__ __align__(16) uint16_t slots[kIdxThreadsMax / kWave][8];
    uint16_t* my = slots[threadIdx.x / kWave];
    if constexpr (ONE) {
        const uint32_t wid = uni(blockIdx.x);
        if (wid >= P.one_items) return;
        const JobView J = view(P.one);
        if (J.ok && J.algo == want) index_item<INV>(J, wid, ws.idx, my);
    } else {
        uint32_t first, last;
        item_range(P, want, first, last);
        for (uint32_t wid = first + uni(blockIdx.x); wid < last; wid += gridDim.x) {
            const Item it = P.items[wid];
            const JobView J = view(P.jobs[uni(it.job)]);
            if (J.ok && J.algo == want) index_item<INV>(J, uni(it.seg), ws.idx, my);
        }
    }
}

// Successor pass: one workgroup per item, as the index pass.
template <bool RAM, bool ONE>
__global__ __launch_bounds__(succ_threads<ONE>()) void k_succ(Plan P, ChainWs ws,
                                                      uint32_t want) {
    __shared__ uint4 pages[kSuccThreadsMax / kWave][kSuccSpan];
    uint4* my = pages[threadIdx.x / kWave];
    if constexpr (ONE) {
        const uint32_t wid = uni(blockIdx.x);
        if (wid >= P.one_items) return;
        const JobView J = view(P.one);
        if (J.ok && J.algo == want) succ_item<RAM>(J, wid, ws.idx, ws.succ, my);
    } else {
        uint32_t first, last;
        item_range(P, want, first, last);
        for (uint32_t wid = first + uni(blockIdx.x); wid < last; wid += gridDim.x) {
            const Item it = P.items[wid];
            const JobView J = view(P.jobs[uni(it.job)]);
            if (J.ok && J.algo == want) succ_item<RAM>(J, uni(it.seg), ws.idx, ws.succ, my);
        }
    }
}

template <bool RAM, bool INV, bool ONE, bool SUCC>
__global__ __launch_bounds__(kChainThreads) void k_spec(Plan P, ChainWs ws) {
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    for_items<ONE>(P, want, [&](const JobView& J, uint32_t seg, uint32_t wid) {
        speculate<RAM, INV, SUCC>(J, seg, wid, ws);
    });
}

// Fix-up round: every segment from the previous segment's speculative exit
// (segment 0 from the job start).
template <bool RAM, bool INV, bool ONE, bool SUCC>
__global__ __launch_bounds__(kChainThreads) void k_fix(Plan P, ChainWs ws) {
    tail_priority();
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    for_items<ONE>(P, want, [&](const JobView& J, uint32_t seg, uint32_t wid) {
        const int64_t X = seg == 0 ? 0 : uni64((int64_t)ws.meta[wid - 1].exit);
        const int64_t h = resolve_from<RAM, INV, SUCC>(J, seg, wid, X, true, ws);
        if (lane_id() == 0) ws.meta[wid].xo[1] = (uint64_t)h;
    });
}

// Parallel round r >= 2: a segment whose predecessor's exit (as of round
// r-1) differs from the entry it was resolved from is resolved again.
template <bool RAM, bool INV, bool ONE, bool SUCC>
__global__ __launch_bounds__(kChainThreads) void k_round(Plan P, ChainWs ws, int r) {
    tail_priority();
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    const int src = (r - 1) & 1, dst = r & 1;
    for_items<ONE>(P, want, [&](const JobView& J, uint32_t seg, uint32_t wid) {
        SegMeta& m = ws.meta[wid];
        int64_t h = uni64((int64_t)m.rexit);
        if (seg > 0) {
            const int64_t X = uni64((int64_t)ws.meta[wid - 1].xo[src]);
            if (X != uni64((int64_t)m.entry))
                h = resolve_from<RAM, INV, SUCC>(J, seg, wid, X, false, ws);
        }
        if (lane_id() == 0) m.xo[dst] = (uint64_t)h;
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

// ------------------------------------------------------------ gates (RAM)
//
// Runs of one byte value can hold RAM chains apart for good.  Inside a run
// every chunk is w + 1 bytes long.  Where a run of at least
// max_chunk bytes follows, a chunk that starts in the last w bytes of the
// run before it ends w + 1 bytes on when the new value is larger (its window
// holds the new value, which the byte after the window equals) and
// max_chunk bytes on when it is smaller (nothing before the limit reaches the
// window's maximum): every chain moves by the same amount, so chains that
// differ there never meet and no speculative list is landed on.  A run
// [r0, r1) of at least max_chunk bytes is a gate: a chain has exactly one
// cut in [r1 - w, r1] (chunks there are w + 1 long, and no chunk jumps the
// run), at offset phi in that window.  From a gate over the next run of L
// bytes, phi' = (phi + a) mod (w + 1), with a = -L when the new value is
// larger or phi = w (the cut is the border itself), else a = max_chunk - L.
// This pass takes a position known to be on the job's chain (the exit of the
// segment before the first one whose entry disagrees with it), follows the
// gates over the runs after it (read from the tile summaries: a tile of one
// value continues or starts a run; a tile holding the value of the run
// before and then that of the run after gives the byte where the value
// changes), and gives every segment start they pass the first cut at or
// after it as the entry the last round resolves that segment from.  Such
// entries only save work: the ordered pass still checks every segment
// against its predecessor.
constexpr int kGateThreads = 1024;
constexpr int kGatePer = 8;                            // tiles per thread and chunk (at most)
constexpr int kGateChunk = kGateThreads * kGatePer;    // tiles per chunk (at most)
constexpr uint32_t kGateList = 2048;                   // run borders kept per chunk
constexpr uint32_t kGateHeads = 64;                    // starting points per job
constexpr uint32_t kNotRun = 0x100u;                   // key of a tile of several values
constexpr uint32_t kTwoRun = 0x400u;                   // | offset: a tile of two runs
constexpr uint32_t kGateTwo = 512;                     // two-run tiles read per chunk

// LDS slot of the key of chunk tile j: one word of padding per 32, so that
// threads scanning 32 consecutive tiles each fall in different banks
__device__ __forceinline__ int xsi(int j) { return j + (j >> 5); }

// The job's constants of the gate arithmetic.
struct GateJob {
    int64_t w, M, seg, kmax;   // kmax: the last segment
    double rseg;               // 1 / seg
    uint32_t W1, Mmod;         // w + 1; max_chunk mod (w + 1)
    uint32_t smod, smod64;     // seg and 64 seg mod (w + 1)
    uint32_t h;                // the starting point's segment (entries go after it)
    bool small;                // 64 (w + 1) < 2^32
    int64_t shift;             // position of the job's first byte in tile 0
};

struct GateState {
    int64_t open;      // job position where the run not yet closed starts
    int64_t g;         // the chain's cut in the last closed run's gate (before
                       // the first run closes: the starting position)
    int64_t top;       // highest segment given an entry
    uint32_t phi;      // offset of g in its gate window
    uint32_t v, vp;    // key of the open run and of the run before it
    uint32_t first;    // the open run is the one the start lies in
    uint32_t stop;
};

// floor(x / seg) for 0 <= x < 2^52 (a double estimate, corrected)
__device__ __forceinline__ int64_t seg_of(const GateJob& G, int64_t x) {
    int64_t q = (int64_t)((double)x * G.rseg);
    if (q * G.seg > x) q--;
    else if ((q + 1) * G.seg <= x) q++;
    return q;
}

__device__ __forceinline__ uint32_t mod_w1(uint64_t d, uint32_t W1) {
    return d >> 32 ? (uint32_t)(d % W1) : (uint32_t)d % W1;
}

// Entries for segments k, k + step, ... <= k_hi, whose starts lie in a
// stretch where the chain's cuts are f, f + w + 1, ... (starts at or before
// f take f); dmod = step * seg mod (w + 1).  One lane's share; returns the
// last segment written, or -1.
__device__ int64_t gate_entries(const GateJob& G, SegMeta* M0, int slot, int64_t k,
                                int64_t k_hi, int64_t step, uint32_t dmod, int64_t f) {
    int64_t last = -1;
    const uint32_t W1 = G.W1;
    uint32_t r = 0;
    bool have = false;
    for (; k <= k_hi; k += step) {
        const int64_t S = k * G.seg;
        int64_t e = f;
        if (S > f) {
            if (!have) {
                const uint32_t dm = mod_w1((uint64_t)(S - f), W1);
                r = dm == 0 ? 0 : W1 - dm;
                have = true;
            } else {
                r = r >= dmod ? r - dmod : r + W1 - dmod;
            }
            e = S + r;
        }
        M0[k - 1].xo[slot] = (uint64_t)e;
        last = k;
    }
    return last;
}

// Wave 0: close the runs whose ends are the chunk's borders, in order, while
// each is a gate.  Border i lies bl[i] bytes after the chunk's first byte
// (at job position pos0) and opens a run of key bk[i].
__device__ void gate_close(const GateJob& G, SegMeta* M0, int slot, int64_t pos0,
                           const uint32_t* bl, const uint16_t* bk, uint32_t nb,
                           GateState& gs) {
    const uint32_t l = lane_id();
    const int64_t w = G.w, M = G.M;
    const uint32_t W1 = G.W1, wu = (uint32_t)w;
    int64_t open = gs.open, g = gs.g, top = gs.top;
    uint32_t phi = gs.phi, v = gs.v, vp = gs.vp;
    bool stop = false;
    uint32_t i = 0;
    if (gs.first && nb > 0) {
        // the run the start lies in ends at the first border: its gate by
        // steps of w + 1 from the start, and entries for the segments inside
        const int64_t r1 = pos0 + bl[0];
        const int64_t E = g, d = r1 - w - E;
        int64_t g0 = E;
        if (d > 0) {
            const uint32_t dm = mod_w1((uint64_t)d, W1);
            g0 = E + d + (dm == 0 ? 0 : W1 - dm);
        }
        const int64_t k_lo = max(seg_of(G, E) + 1, (int64_t)G.h + 1);
        const int64_t k_hi = min(seg_of(G, g0), G.kmax);
        int64_t last = -1;
        if (k_lo <= k_hi)
            last = gate_entries(G, M0, slot, k_lo + l, k_hi, kWave, G.smod64, E);
        top = max(top, (int64_t)uni(wave_max((uint32_t)max(last, (int64_t)0))));
        phi = (uint32_t)(g0 - (r1 - w));
        g = g0;
        vp = v;
        open = r1;
        v = bk[0];
        i = 1;
    }
    while (i < nb && !stop) {
        const uint32_t cnt = min(nb - i, (uint32_t)kWave);
        const bool in = l < cnt;
        const uint32_t li = in ? l : 0;        // lanes past the batch repeat lane 0
        const uint32_t bt = bl[i + li];
        const int64_t b = pos0 + bt;
        const int64_t bprev = li == 0 ? open : pos0 + bl[i + li - 1];
        const uint32_t vl = li == 0 ? v : bk[i + li - 1];
        // (every lane takes part in a shuffle: a lane left out reads as 0)
        const uint32_t vsh = (uint32_t)__shfl((int)vl, (int)(l + kWave - 1) % kWave);
        const uint32_t vpl = l == 0 ? vp : vsh;
        const int64_t L = b - bprev;
        const bool ok = in && vl != kNotRun && L >= M;
        const bool rise = vl > vpl;
        const uint32_t Lm = mod_w1((uint64_t)L, W1);
        const uint32_t ar = Lm == 0 ? 0 : W1 - Lm;             // -L mod (w+1)
        const uint32_t af = G.Mmod >= Lm ? G.Mmod - Lm : G.Mmod + W1 - Lm;
        const uint64_t okm = __ballot(ok);
        const uint32_t lim = ~okm ? min((uint32_t)__builtin_ctzll(~okm), cnt) : cnt;
        // the phases in order, as a prefix sum of the steps: a lane's step is
        // ar when its run's value rises, else af, except that a chain whose
        // cut is the border itself (phase w) steps by ar; such lanes are
        // rare, and the sum is taken again from the lane after each one
        const uint32_t A = rise ? ar : af;
        uint32_t phin = 0, from = 0, base = phi;
        for (;;) {
            const uint32_t a0 = l >= from && l < lim ? A : 0u;
            uint64_t ex_sum;                     // sum of the steps of the lanes before
            if (G.small) {                       // 64 (w + 1) < 2^32: a 32-bit DPP scan
                ex_sum = seg_sum<kWave>(a0) - a0;
            } else {
                uint64_t x = a0;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const uint64_t y = (uint64_t)__shfl_up((long long)x, (unsigned)o, kWave);
                    if ((int)l >= o) x += y;
                }
                ex_sum = x - a0;
            }
            if (l >= from) phin = mod_w1(base + ex_sum, W1);
            const uint64_t ex = __ballot(l >= from && l < lim && phin == wu && !rise);
            if (!ex) break;
            const uint32_t q = (uint32_t)__builtin_ctzll(ex);
            const uint32_t arq = (uint32_t)__builtin_amdgcn_readlane((int)ar, (int)q);
            base = wu + arq >= W1 ? wu + arq - W1 : wu + arq;
            from = q + 1;
        }
        if (lim > 0) {
            // each lane: its run's cuts f, f + w + 1, ... up to its gate
            const bool step1 = phin == wu || rise;
            uint32_t pout = phin + (step1 ? ar : af);
            if (pout >= W1) pout -= W1;
            phi = (uint32_t)__builtin_amdgcn_readlane((int)pout, (int)lim - 1);
            const int64_t gout = b - w + pout;
            const int64_t gsh = (int64_t)__shfl((long long)gout, (int)(l + kWave - 1) % kWave);
            const int64_t gin = l == 0 ? g : gsh;
            int64_t last = -1;
            if (l < lim) {
                const int64_t k_lo = max(seg_of(G, gin) + 1, (int64_t)G.h + 1);
                const int64_t k_hi = min(seg_of(G, gout), G.kmax);
                if (k_lo <= k_hi)
                    last = gate_entries(G, M0, slot, k_lo, k_hi, 1, G.smod,
                                        gin + (step1 ? (int64_t)W1 : M));
            }
            top = max(top, (int64_t)uni(wave_max((uint32_t)max(last, (int64_t)0))));
            const int q = (int)lim - 1;
            g = (int64_t)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)gout, q) |
                          ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(gout >> 32), q) << 32));
            vp = (uint32_t)__builtin_amdgcn_readlane((int)vl, q);
            const uint32_t bo = (uint32_t)__builtin_amdgcn_readlane((int)bt, q);
            open = pos0 + bo;
            v = bk[i + (uint32_t)q];
        }
        stop = lim < cnt;
        i += lim;
    }
    if (l == 0) {
        gs.open = open;
        gs.g = g;
        gs.top = top;
        gs.phi = phi;
        gs.v = v;
        gs.vp = vp;
        gs.first = gs.first && nb == 0;
        gs.stop = stop;
    }
}

// Offset p (1..1023) at which a tile (bytes v, 16 per lane) switches from
// all bytes a to all bytes b, or 0 when its bytes are not so (one wave).
__device__ uint32_t two_run_split(const uint4 v, uint32_t a, uint32_t b) {
    const uint32_t ra = a * 0x01010101u, rb = b * 0x01010101u;
    auto nib = [](uint32_t z) {            // high bit of each byte -> 4 bits
        return ((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u);
    };
    const uint32_t ea = nib(zero_bytes(v.x ^ ra)) | nib(zero_bytes(v.y ^ ra)) << 4 |
                        nib(zero_bytes(v.z ^ ra)) << 8 | nib(zero_bytes(v.w ^ ra)) << 12;
    const uint32_t eb = nib(zero_bytes(v.x ^ rb)) | nib(zero_bytes(v.y ^ rb)) << 4 |
                        nib(zero_bytes(v.z ^ rb)) << 8 | nib(zero_bytes(v.w ^ rb)) << 12;
    const bool all_a = ea == 0xFFFFu, all_b = eb == 0xFFFFu;
    // a lane that switches: a on a prefix of its bytes, b on the rest
    const bool sw = ea != 0 && !all_a && (ea & (ea + 1)) == 0 && eb == (~ea & 0xFFFFu);
    if (__ballot(!(all_a || all_b || sw))) return 0;
    const uint64_t ma = __ballot(all_a), ms = __ballot(sw), mb = __ballot(all_b);
    if (!~ma) return 0;
    const uint32_t q = (uint32_t)__builtin_ctzll(~ma);        // first lane not all a
    if (ma != (q == 0 ? 0ull : (~0ull >> (64 - q)))) return 0;
    uint32_t p = 16 * q, qb = q;
    if ((ms >> q) & 1u) {
        p += (uint32_t)__builtin_popcount((uint32_t)__builtin_amdgcn_readlane((int)ea, (int)q));
        qb = q + 1;
    }
    const uint64_t rest = qb >= 64 ? 0ull : (~0ull << qb);
    if ((mb & rest) != rest) return 0;
    return p > 0 && p < (uint32_t)kTile ? p : 0;
}

// Exclusive prefix sum of one value per thread over the block, in two
// barriers (a scan per wave, then the waves' totals).
__device__ uint32_t gate_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const uint32_t wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const uint32_t incl = seg_sum<kWave>(v);
    if (lane_id() == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (uint32_t k = 0; k < nw; k++) {
        const uint32_t s = wsum[k];
        before += k < wv ? s : 0;
        all += s;
    }
    total = all;
    __syncthreads();
    return before + incl - v;
}

// Whether the gate pass has work in a job (one wave): a starting point
// (a segment whose entry disagrees with the exit before it while its
// predecessor's agrees) whose exit lies in a tile of one value, with runs of
// one value filling about a segment after it (64 tiles sampled across the
// next segment's worth of tiles, nearly all of one value each).  Most jobs
// have none, and are passed over at this cost.
__device__ bool gate_worth(const JobView& J, const ChainWs& ws, int slot) {
    const uint32_t l = lane_id();
    const SegMeta* M0 = ws.meta + J.item0;
    const int64_t shift = (int64_t)((uintptr_t)J.data & 15);
    const int64_t NT = (J.n + shift + kTile - 1) >> 10;
    const uint32_t* kw = (const uint32_t*)(ws.idx + J.idx0);
    auto key_of = [&](int64_t t) -> uint32_t {
        const uint32_t x = kw[4 * min(t, NT - 1)];
        return t < NT && ie_all(x) ? ie_max(x) : kNotRun;
    };
    const int64_t stride = max((int64_t)1, (J.seg >> 10) / kWave);
    for (uint32_t k0 = 1; k0 < J.nseg; k0 += kWave) {
        const uint32_t k = min(k0 + l, J.nseg - 1);
        const uint64_t en = M0[k].entry, xa = M0[k - 1].xo[slot];
        const uint64_t ep = M0[k - 1].entry, xp = M0[k >= 2 ? k - 2 : 0].xo[slot];
        const int64_t E = (int64_t)xa;
        const bool head = k0 + l < J.nseg && en != xa && (k == 1 || ep == xp) &&
                          E >= 0 && E < J.n && key_of((E + shift) >> 10) != kNotRun;
        for (uint64_t hm = __ballot(head); hm; hm &= hm - 1) {
            const int q = __builtin_ctzll(hm);
            const int64_t Eq = (int64_t)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)E, q) |
                                         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(E >> 32), q) << 32));
            const int64_t tq = (Eq + shift) >> 10;
            const uint64_t mixed = __ballot(key_of(tq + 1 + (int64_t)l * stride) == kNotRun);
            if (__builtin_popcountll(mixed) <= 8) return true;
        }
    }
    return false;
}

// The gate pass over one job, by the whole block (shared arrays passed in).
__device__ void gate_job(const JobView& J, const ChainWs& ws, int slot, uint32_t* xs,
                         uint32_t* bl, uint16_t* bk, uint16_t* tr, uint32_t* wsum,
                         uint32_t* heads, uint32_t& n_heads, uint32_t& low_head,
                         uint32_t& n_tr, GateState& gs) {
    const uint32_t tid = threadIdx.x;
    SegMeta* M0 = ws.meta + J.item0;
    Source src;
    src.init(J.data, (uint64_t)J.n);
    const int64_t shift = src.shift;
    const int64_t NT = (J.n + shift + kTile - 1) >> 10;
    const uint32_t* kw = (const uint32_t*)(ws.idx + J.idx0);  // word 0 of tile t at 4t
    auto key_of = [&](int64_t t) -> uint32_t {
        const uint32_t x = kw[4 * min(t, NT - 1)];
        return t < NT && ie_all(x) ? ie_max(x) : kNotRun;
    };
    // starting points: segments whose entry disagrees with the exit before
    // them while their predecessor's agrees (that exit then ends a consistent
    // chain), and whose exit lies in a tile of one value
    if (tid == 0) {
        n_heads = 0;
        low_head = ~0u;
    }
    __syncthreads();
    constexpr uint32_t kHU = 4;              // segments per thread, loads first
    for (uint32_t k0 = 1; k0 < J.nseg; k0 += kHU * kGateThreads) {
        uint64_t en[kHU], xa[kHU], ep[kHU], xp[kHU];
#pragma unroll
        for (uint32_t u = 0; u < kHU; u++) {
            const uint32_t k = min(k0 + u * kGateThreads + tid, J.nseg - 1);
            en[u] = M0[k].entry;
            xa[u] = M0[k - 1].xo[slot];
            ep[u] = M0[k - 1].entry;
            xp[u] = M0[k >= 2 ? k - 2 : 0].xo[slot];
        }
#pragma unroll
        for (uint32_t u = 0; u < kHU; u++) {
            const uint32_t k = k0 + u * kGateThreads + tid;
            if (k < J.nseg && en[u] != xa[u] && (k == 1 || ep[u] == xp[u])) {
                const int64_t E = (int64_t)xa[u];
                if (E >= 0 && E < J.n && key_of((E + shift) >> 10) != kNotRun) {
                    atomicMin(&low_head, k);
                    const uint32_t s = atomicAdd(&n_heads, 1u);
                    if (s < kGateHeads) heads[s] = k;
                }
            }
        }
    }
    __syncthreads();
    uint32_t nh = n_heads;
    if (nh == 0) return;
    if (tid == 0) {
        if (nh > kGateHeads) {               // keep the lowest: its start is exact
            heads[0] = low_head;
        } else {
            for (uint32_t a = 1; a < nh; a++) {          // a few entries
                const uint32_t x = heads[a];
                uint32_t b = a;
                for (; b > 0 && heads[b - 1] > x; b--) heads[b] = heads[b - 1];
                heads[b] = x;
            }
        }
    }
    if (nh > kGateHeads) nh = 1;
    __syncthreads();
    // one wave per starting point, which is kept only where runs of one
    // value fill about a segment after it: 64 tiles sampled across the next
    // segment's worth of tiles must be nearly all of one value each (a
    // stretch shorter than a segment gives at most one entry, which the
    // rounds and the ordered pass find anyway)
    const int64_t stride = max((int64_t)1, (J.seg >> 10) / kWave);
    for (uint32_t hi = tid / kWave; hi < nh; hi += kGateThreads / kWave) {
        const uint32_t l = lane_id();
        const int64_t E = (int64_t)M0[heads[hi] - 1].xo[slot];
        const int64_t tE = (E + shift) >> 10;
        const uint64_t mixed = __ballot(key_of(tE + 1 + (int64_t)l * stride) == kNotRun);
        if (l == 0 && __builtin_popcountll(mixed) > 8) heads[hi] = 0;
    }
    __syncthreads();
    GateJob G;
    G.w = J.w;
    G.M = J.M;
    G.seg = J.seg;
    G.kmax = (int64_t)J.nseg - 1;
    G.rseg = 1.0 / (double)J.seg;
    G.W1 = (uint32_t)(J.w + 1);
    G.Mmod = (uint32_t)(J.M % G.W1);
    G.smod = (uint32_t)((uint64_t)J.seg % G.W1);
    G.smod64 = (uint32_t)((uint64_t)J.seg * kWave % G.W1);
    G.shift = shift;
    G.small = (uint64_t)G.W1 * kWave < (1ull << 32);
    int64_t covered = 0;
    for (uint32_t hi = 0; hi < nh; hi++) {
        const uint32_t h = heads[hi];
        if (h == 0 || (int64_t)h <= covered) continue;
        G.h = h;
        const int64_t E = (int64_t)M0[h - 1].xo[slot];
        const int64_t tE = (E + shift) >> 10;
        __syncthreads();
        if (tid == 0) {
            gs.open = E;
            gs.g = E;
            gs.top = h;
            gs.phi = 0;
            gs.v = key_of(tE);
            gs.vp = kNotRun;
            gs.first = 1;
            gs.stop = 0;
        }
        __syncthreads();
        // chunks of 1, 4, then 8 tiles per thread from E's tile on, the next
        // chunk's loads in flight while wave 0 closes this one's runs
        int64_t T = tE;
        int per = 1;
        uint32_t kv[kGatePer];
        auto fetch = [&](int64_t T0, int pr) {      // word 0 of each tile, loads first
            const uint32_t* kb = kw + 4 * T0;       // (32-bit offsets from the chunk)
            const uint32_t last = (uint32_t)min(NT - 1 - T0, (int64_t)kGateChunk);
#pragma unroll
            for (int u = 0; u < kGatePer; u++) {
                const uint32_t j = min((uint32_t)(u * kGateThreads) + tid, last);
                kv[u] = u < pr ? kb[4 * j] : 0u;
            }
        };
        fetch(T, per);
        for (bool go = true; go;) {
            const int C = per * kGateThreads;
#pragma unroll
            for (int u = 0; u < kGatePer; u++) {
                const int j = u * kGateThreads + (int)tid;
                if (u < per)
                    xs[xsi(j)] = T + j < NT && ie_all(kv[u]) ? ie_max(kv[u]) : kNotRun;
            }
            if (tid == 0) {
                xs[xsi(C)] = key_of(T + C);      // the tile after the chunk
                n_tr = 0;
            }
            const uint32_t before = gs.v;        // key of the open run (tile T - 1's end)
            __syncthreads();
            // this thread's tiles j0 .. j0 + per - 1 with a neighbour on each side
            const int j0 = (int)tid * per;
            uint32_t kk[kGatePer + 2];
#pragma unroll
            for (int u = 0; u < kGatePer + 2; u++)
                kk[u] = u <= per + 1 ? (j0 + u - 1 < 0 ? before : xs[xsi(j0 + u - 1)]) : 0u;
            // tiles holding two values between two runs of one value each
            // (a value change off the tile grid): one wave reads each
            uint32_t two = 0;
#pragma unroll
            for (int u = 0; u < kGatePer; u++) {
                if (u < per && kk[u + 1] == kNotRun && kk[u] != kNotRun &&
                    kk[u + 2] != kNotRun && kk[u] != kk[u + 2]) {
                    two |= 1u << u;
                    const uint32_t s = atomicAdd(&n_tr, 1u);
                    if (s < kGateTwo) tr[s] = (uint16_t)(j0 + u);
                }
            }
            __syncthreads();
            const uint32_t ntr = min(n_tr, kGateTwo);
            if (ntr > 0) {
                // four tiles per wave at a time, their loads first
                constexpr uint32_t kTwoAt = 4;
                const uint32_t nw = kGateThreads / kWave, wv = tid / kWave;
                for (uint32_t q0 = wv * kTwoAt; q0 < ntr; q0 += nw * kTwoAt) {
                    uint4 tb[kTwoAt];
#pragma unroll
                    for (uint32_t r = 0; r < kTwoAt; r++)
                        tb[r] = src.load<false>(T + tr[min(q0 + r, ntr - 1)]);
#pragma unroll
                    for (uint32_t r = 0; r < kTwoAt; r++) {
                        if (q0 + r < ntr) {
                            const int j = tr[q0 + r];
                            const uint32_t kp = j == 0 ? before : xs[xsi(j - 1)];
                            const uint32_t p = two_run_split(tb[r], kp, xs[xsi(j + 1)]);
                            if (lane_id() == 0 && p) xs[xsi(j)] = kTwoRun | p;
                        }
                    }
                }
                __syncthreads();
                // the checked tiles, and a neighbour before this thread's first
#pragma unroll
                for (int u = 0; u < kGatePer; u++)
                    if ((two >> u) & 1u) kk[u + 1] = xs[xsi(j0 + u)];
                if (j0 > 0 && kk[0] == kNotRun) kk[0] = xs[xsi(j0 - 1)];
            }
            // borders: a tile of one value unlike the run before it starts a
            // run at the tile; a tile of two values starts one at its switch;
            // any other tile ends the walk
            uint32_t bits = 0, pk = (kk[0] & kTwoRun) ? kk[1] : kk[0];
#pragma unroll
            for (int u = 0; u < kGatePer; u++) {
                if (u < per) {
                    const uint32_t k = kk[u + 1];
                    if (k & kTwoRun) {
                        bits |= 1u << u;
                        pk = kk[u + 2];
                    } else {
                        bits |= (uint32_t)(k == kNotRun || k != pk) << u;
                        pk = k;
                    }
                }
            }
            uint32_t total;
            uint32_t at = gate_scan((uint32_t)__builtin_popcount(bits), wsum, total);
            for (; bits; bits &= bits - 1, at++) {
                const int j = j0 + __builtin_ctz(bits);
                const uint32_t k = xs[xsi(j)];
                if (at < kGateList) {
                    bl[at] = (uint32_t)j * kTile + ((k & kTwoRun) ? (k & (kTwoRun - 1)) : 0u);
                    bk[at] = (uint16_t)((k & kTwoRun) ? xs[xsi(j + 1)] : k);
                }
            }
            __syncthreads();
            const int per2 = min(per * 4, kGatePer);
            if (T + C < NT) fetch(T + C, per2);
            if (tid < (uint32_t)kWave)
                gate_close(G, M0, slot, T * kTile - shift, bl, bk, min(total, kGateList), gs);
            __syncthreads();
            go = !gs.stop && total <= kGateList && T + C < NT;
            T += C;
            per = per2;
        }
        covered = gs.top;
    }
}

// Gate pass over the RAM jobs of kGateMinSeg or more segments, before the
// last round; `slot` is the exit slot that round reads.  Each block looks
// at kGateThreads jobs at a time, one per thread, and works on those.
__global__ __launch_bounds__(kGateThreads) void k_gates(Plan P, uint32_t n_jobs_h,
                                                        const uint32_t* n_jobs_d,
                                                        ChainWs ws, int slot) {
    __shared__ uint32_t xs[kGateChunk + 1 + (kGateChunk + 1) / 32 + 1];
    __shared__ uint32_t bl[kGateList];
    __shared__ uint16_t bk[kGateList];
    __shared__ uint16_t tr[kGateTwo];
    __shared__ uint32_t wsum[kGateThreads / kWave];
    __shared__ uint32_t heads[kGateHeads];
    __shared__ uint32_t n_heads, low_head, n_tr;
    __shared__ uint32_t cand[kGateThreads];
    __shared__ uint32_t n_cand;
    __shared__ GateState gs;
    tail_priority();
    const uint32_t tid = threadIdx.x;
    const uint32_t n_jobs = n_jobs_d ? *n_jobs_d : n_jobs_h;
    for (uint32_t base = blockIdx.x * kGateThreads; base < n_jobs;
         base += gridDim.x * kGateThreads) {
        __syncthreads();
        if (tid == 0) n_cand = 0;
        __syncthreads();
        if (base + tid < n_jobs) {
            const JobDesc& D = P.jobs ? P.jobs[base + tid] : P.one;
            if (D.ok && D.algo == kRam && D.nseg >= kGateMinSeg && D.n > 0)
                cand[atomicAdd(&n_cand, 1u)] = base + tid;
        }
        __syncthreads();
        // with several candidates, one wave per candidate first: those with
        // work stay (in place, in order); one or two go to the block at once
        const uint32_t nc = n_cand;
        if (nc > 2) {
            for (uint32_t ci = tid / kWave; ci < nc; ci += kGateThreads / kWave) {
                const JobView J = view(P.jobs ? P.jobs[cand[ci]] : P.one);
                const bool worth = gate_worth(J, ws, slot);
                if (lane_id() == 0 && !worth) cand[ci] = ~0u;
            }
            __syncthreads();
        }
        for (uint32_t ci = 0; ci < nc; ci++) {
            const uint32_t job = cand[ci];
            if (job == ~0u) continue;
            __syncthreads();
            const JobView J = view(P.jobs ? P.jobs[job] : P.one);
            gate_job(J, ws, slot, xs, bl, bk, tr, wsum, heads, n_heads, low_head,
                     n_tr, gs);
        }
    }
}

// Settle one RAM / AE job with the whole block.  A segment is flagged when
// its entry is not its predecessor's resolved exit.  Each pass takes the
// heads of the runs of flagged segments (a flagged segment whose predecessor
// is not flagged: its entry is final) side by side, one wave each; a wave
// resolves its head again and goes on into the following segments, in
// order, while the exit it found changes the next segment's entry, up to
// the next head.  Passes repeat until nothing is flagged (a head reached
// from before it changes its entry, and is flagged again); each pass
// settles every head, so a job's chain is walked once in order, by as many
// waves as it has independent stretches.  Then output offsets are
// assigned.
template <bool RAM, bool INV, bool SUCC>
__device__ void settle_job(const JobView& J, const ChainWs& ws, uint64_t* sh,
                           uint32_t* flagged, uint32_t& n_flagged) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t nwaves = nt / kWave, wv = uni(tid / kWave);
    SegMeta* M0 = ws.meta + J.item0;
    auto is_flagged = [&](uint32_t k) {
        return k >= 1 && k < J.nseg && M0[k].entry != M0[k - 1].rexit;
    };
    for (uint32_t pass = 1;; pass++) {
        if (tid == 0) {
            n_flagged = 0;
            flagged[kSettleList] = ~0u;         // the lowest head
        }
        __syncthreads();
        uint32_t any = 0;
        for (uint32_t k = 1 + tid; k < J.nseg; k += nt) {
            if (is_flagged(k)) {
                any = 1;
                if (!is_flagged(k - 1)) {        // the head of a run
                    atomicMin(&flagged[kSettleList], k);
                    const uint32_t slot = atomicAdd(&n_flagged, 1u);
                    if (slot < kSettleList) {
                        flagged[slot] = k;
                        M0[k].claim = pass;
                    }
                }
            }
        }
        any = __syncthreads_or(any);
        if (!any) break;
        if (tid == 0 && n_flagged > kSettleList) {
            // more heads than the list holds: the lowest one (its entry is
            // final) is always among those settled, so every pass progresses
            const uint32_t lo = flagged[kSettleList];
            flagged[0] = lo;
            M0[lo].claim = pass;
        }
        __syncthreads();
        const uint32_t cnt = min(n_flagged, kSettleList);
        for (uint32_t i = wv; i < cnt; i += nwaves) {
            uint32_t k2 = uni(flagged[i]);
            int64_t prev = uni64((int64_t)M0[k2 - 1].rexit);
            for (;;) {
                const int64_t h = resolve_from<RAM, INV, SUCC>(J, k2, J.item0 + k2, prev,
                                                         false, ws);
                const uint32_t nxt = k2 + 1;
                if (nxt >= J.nseg || uni(M0[nxt].claim) == pass ||
                    uni64((int64_t)M0[nxt].entry) == h)
                    break;
                k2 = nxt;
                prev = h;
            }
        }
        __syncthreads();
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
template <bool RAM, bool INV, bool SUCC>
__global__ __launch_bounds__(256) void k_resolve(Plan P, uint32_t n_jobs_h,
                                                 const uint32_t* n_jobs_d,
                                                 ChainWs ws) {
    tail_priority();
    __shared__ uint64_t sh[256];
    __shared__ uint32_t flagged[kSettleList + 1];
    __shared__ uint32_t n_flagged;
    const uint32_t n_jobs = n_jobs_d ? *n_jobs_d : n_jobs_h;
    for (uint32_t job = blockIdx.x; job < n_jobs; job += gridDim.x) {
        const JobView J = view(P.jobs ? P.jobs[job] : P.one);
        const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
        if (J.ok && J.algo == want && J.n > 0)
            settle_job<RAM, INV, SUCC>(J, ws, sh, flagged, n_flagged);
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

// AE's walkers with successor words hold about twice the registers of those
// without (some 120 against 60), so a launch of many short AE jobs keeps
// the leaner kernels and no successor pass (`succ` false); RAM always has
// them.
template <bool RAM, bool INV, bool ONE>
static void launch_passes(const Plan& P, uint32_t items_upper, uint32_t jobs_upper,
                          const uint32_t* n_jobs_d, const ChainWs& ws,
                          hipStream_t st, Marks* mk,
                          const char* spec_name, const char* idx_name, int part,
                          bool succ) {
    const dim3 blk(kChainThreads), grid((items_upper + kChainWaves - 1) / kChainWaves);
    const uint32_t want = RAM ? kRam : (INV ? kAeMin : kAe);
    const char* succ_name = RAM ? (ONE ? "successors_ram" : "successors_batch_ram")
                            : INV ? (ONE ? "successors_ae_min" : "successors_batch_ae_min")
                                  : (ONE ? "successors_ae" : "successors_batch_ae");
    if (part & kPartIndex)
        CDC_LAUNCH(mk, 1, idx_name, (k_index<INV, ONE>), dim3(items_upper),
                   dim3(idx_threads<ONE>()), 0, st, P, ws, want);
    succ = succ || RAM;
    if (part & kPartSpec) {
        if (succ)
            CDC_LAUNCH(mk, 1, succ_name, (k_succ<RAM, ONE>), dim3(items_upper),
                       dim3(succ_threads<ONE>()), 0, st, P, ws, want);
        if (succ)
            CDC_LAUNCH(mk, 1, spec_name, (k_spec<RAM, INV, ONE, true>), grid, blk, 0, st,
                       P, ws);
        else
            CDC_LAUNCH(mk, 1, spec_name, (k_spec<RAM, INV, ONE, RAM>), grid, blk, 0, st,
                       P, ws);
    }
    if (part & kPartFix) {
        if (succ)
            CDC_LAUNCH(mk, 2, "fixup", (k_fix<RAM, INV, ONE, true>), grid, blk, 0, st, P, ws);
        else
            CDC_LAUNCH(mk, 2, "fixup", (k_fix<RAM, INV, ONE, RAM>), grid, blk, 0, st, P, ws);
    }
    if (part & kPartRest)
        for (int r = 2; r < 2 + kRounds; r++) {
            if (RAM && r == 1 + kRounds && (part & kPartGates))   // entries over runs of one value
                CDC_LAUNCH(mk, 2, "gates", k_gates,
                           dim3(min((jobs_upper + kGateThreads - 1) / kGateThreads, 256u)),
                           dim3(kGateThreads), 0, st, P, jobs_upper, n_jobs_d, ws,
                           (r - 1) & 1);
            if (succ)
                CDC_LAUNCH(mk, 2, "round", (k_round<RAM, INV, ONE, true>), grid, blk, 0, st,
                           P, ws, r);
            else
                CDC_LAUNCH(mk, 2, "round", (k_round<RAM, INV, ONE, RAM>), grid, blk, 0, st,
                           P, ws, r);
        }
}

// With one job, items_upper is its segment count (the grid covers every
// segment); with a job table the kernels walk the items grid-stride.
template <bool RAM, bool INV>
static void launch_algo(const Plan& P, uint32_t items_upper,
                        uint32_t jobs_upper, const uint32_t* n_jobs_d,
                        const ChainWs& ws, hipStream_t st, Marks* mk,
                        const char* spec_name, const char* idx_name, int part,
                        bool ae_succ) {
    if (P.jobs == nullptr)
        launch_passes<RAM, INV, true>(P, items_upper, jobs_upper, n_jobs_d, ws, st, mk,
                                      spec_name, idx_name, part, true);
    else
        launch_passes<RAM, INV, false>(P, items_upper, jobs_upper, n_jobs_d, ws, st, mk,
                                       spec_name, idx_name, part, ae_succ);
    if ((part & kPartRest) && (RAM || P.jobs == nullptr || ae_succ))
        CDC_LAUNCH(mk, 2, "resolve", (k_resolve<RAM, INV, true>),
                   dim3(min(jobs_upper, 2048u)), dim3(256), 0, st, P, jobs_upper,
                   n_jobs_d, ws);
    else if (part & kPartRest)
        CDC_LAUNCH(mk, 2, "resolve", (k_resolve<RAM, INV, RAM>),
                   dim3(min(jobs_upper, 2048u)), dim3(256), 0, st, P, jobs_upper,
                   n_jobs_d, ws);
}

hipError_t launch_chain(const Plan& P, uint32_t algo, uint32_t items_upper,
                        uint32_t jobs_upper, const uint32_t* n_jobs_d,
                        const ChainWs& ws, hipStream_t st, Marks* mk, int part,
                        bool ae_succ) {
    const bool one = P.jobs == nullptr;
    if (algo == kRam)
        launch_algo<true, false>(P, items_upper, jobs_upper, n_jobs_d, ws, st, mk,
                                 one ? "speculate_ram" : "speculate_batch_ram",
                                 one ? "index_ram" : "index_batch_ram", part, true);
    else if (algo == kAe)
        launch_algo<false, false>(P, items_upper, jobs_upper, n_jobs_d, ws, st, mk,
                                  one ? "speculate_ae" : "speculate_batch_ae",
                                  one ? "index_ae" : "index_batch_ae", part, ae_succ);
    else
        launch_algo<false, true>(P, items_upper, jobs_upper, n_jobs_d, ws, st, mk,
                                 one ? "speculate_ae_min" : "speculate_batch_ae_min",
                                 one ? "index_ae_min" : "index_batch_ae_min", part,
                                 ae_succ);
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
                         Marks* mk, int part) {
    const bool one = P.jobs == nullptr;
    for (uint32_t algo : {kRam, kAe, kAeMin}) {
        if (!one || P.one.algo == algo) {
            const hipError_t e = launch_chain(P, algo, items_upper, jobs_upper,
                                              n_jobs_d, ws, st, mk, part, true);
            if (e != hipSuccess) return e;
        }
    }
    return launch_emit(P, items_upper, ws, wpb, st, mk);
}

}  // namespace cdc

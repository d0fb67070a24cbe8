// MAXP boundary finding on gfx950, and small utility kernels.
//
// MAXP (Section 2.1 "MAXP", Fig. 2b; Section 4.3) cuts right after a byte
// that is strictly greater than the w bytes before and the w bytes after
// it.  That test does not depend on where the current chunk starts, so the
// candidates are found fully in parallel: a strict local maximum over +-w is
// the unique maximum of every block of at most w+1 bytes that contains it
// (the extreme byte search of Section 4.1 over blocks), and each block's
// unique maximum is then checked against the +-w window.  Given the sorted
// candidates, the chain is arithmetic: from a chunk start s a candidate q
// ends the chunk iff (q - s) mod M >= w (the forced cuts at s+M, s+2M, ...
// leave it at least w bytes into its chunk).
#include "wave.h"

namespace cdc {

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
    const uint32_t last = lane_id() | (G - 1);
    uint32_t gm, eq, cnt;
    if constexpr (G == kWave) {
        // one block per tile: the maximum is uniform, the lanes holding it
        // are counted from a ballot
        gm = (uint32_t)__builtin_amdgcn_readlane((int)seg_max<G>(lm), kWave - 1);
        eq = (lm == gm) ? 1u : 0u;
        cnt = (uint32_t)__builtin_popcountll(__ballot(eq != 0));
    } else {
        gm = (uint32_t)__shfl((int)seg_max<G>(lm), (int)last);
        eq = (lm == gm) ? 1u : 0u;
        cnt = (uint32_t)__shfl((int)seg_sum<G>(eq), (int)last);
    }
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

// Tiles [t0, t1) of a job, kAhead loads in flight per wave.
template <int G>
__device__ void block_tiles(const Source& src, int64_t t0, int64_t t1,
                            int64_t n, uint8_t* bm, int64_t* bp) {
    constexpr int kAhead = 4;
    constexpr int64_t per_tile = kTile / (16 * G);   // blocks per tile
    for (int64_t t = t0; t < t1; t += kAhead) {
        uint4 v[kAhead];
#pragma unroll
        for (int i = 0; i < kAhead; i++)
            v[i] = t + i < t1 ? src.load<false>(t + i) : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < kAhead; i++)
            if (t + i < t1)
                block_summaries<G>(v[i], src.tile_pos(t + i), n, bm, bp,
                                   (t + i) * per_tile);
    }
}

__device__ void maxp_blocks_item(const JobView& J, uint32_t seg, uint8_t* bmax,
                                 int64_t* bpos) {
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
    uint8_t* bm = bmax + J.blk0;
    int64_t* bp = bpos + J.blk0;
    switch ((int)J.blog) {
        case 4: block_tiles<1>(src, t0, t1, J.n, bm, bp); break;
        case 5: block_tiles<2>(src, t0, t1, J.n, bm, bp); break;
        case 6: block_tiles<4>(src, t0, t1, J.n, bm, bp); break;
        case 7: block_tiles<8>(src, t0, t1, J.n, bm, bp); break;
        case 8: block_tiles<16>(src, t0, t1, J.n, bm, bp); break;
        case 9: block_tiles<32>(src, t0, t1, J.n, bm, bp); break;
        default: block_tiles<64>(src, t0, t1, J.n, bm, bp); break;
    }
}

__global__ __launch_bounds__(256) void k_maxp_blocks(Plan P, uint8_t* bmax,
                                                     int64_t* bpos,
                                                     uint32_t* err) {
    uint32_t first, last;
    item_range(P, kMaxp, first, last);
    for (uint32_t wid = first + wave_global_id(); wid < last; wid += wave_count()) {
        JobView J;
        uint32_t seg;
        if (!item_of(P, wid, J, seg) || !J.ok || J.algo != kMaxp ||
            J.blog == 0)
            continue;
        maxp_blocks_item(J, seg, bmax, bpos);
    }
}

__device__ __forceinline__ uint32_t byte_at(const uint8_t* d, int64_t p) {
    return d[p];
}

// Exact check that every byte in [lo, hi] (job positions) is below v,
// 1 <= v <= 255: 16 bytes per load, from the 16-byte granules that hold the
// range (as the tile loads do), bytes outside the range masked to zero.
__device__ bool all_below(const uint8_t* d, int64_t lo, int64_t hi, uint32_t v) {
    const uintptr_t a = (uintptr_t)(d + lo), b = (uintptr_t)(d + hi);
    for (uintptr_t g = a & ~(uintptr_t)15; g <= b; g += 16) {
        const uint4 q = *(const uint4*)g;
        const int ka = a > g ? (int)(a - g) : 0;
        const int kb = (int)min((uintptr_t)16, b - g + 1);
        if (lane_max16(keep_bytes(q, ka, kb)) >= v) return false;
    }
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
__device__ void maxp_verify_item(const JobView& J, uint32_t seg, uint32_t wid,
                                 const uint8_t* bmax, const int64_t* bpos,
                                 SegMeta* meta, uint32_t* cand,
                                 uint32_t* err) {
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

__global__ __launch_bounds__(256) void k_maxp_verify(Plan P, const uint8_t* bmax,
                                                     const int64_t* bpos,
                                                     SegMeta* meta,
                                                     uint32_t* cand,
                                                     uint32_t* err) {
    uint32_t first, last;
    item_range(P, kMaxp, first, last);
    for (uint32_t wid = first + wave_global_id(); wid < last; wid += wave_count()) {
        JobView J;
        uint32_t seg;
        if (!item_of(P, wid, J, seg) || !J.ok || J.algo != kMaxp) continue;
        maxp_verify_item(J, seg, wid, bmax, bpos, meta, cand, err);
    }
}

// The MAXP chain over the candidates (one block per job, one wave walking).  From a chunk start
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

constexpr uint32_t kChainChunk = 4096;   // segment counts staged at a time
constexpr uint32_t kChainThreads = 256;  // threads per block of the chain pass
constexpr uint32_t kForcedQ = 256;       // runs of forced cuts queued for the block

// t forced cuts s + M, s + 2M, ... at output index `at` on.  The walker only
// counts them; the whole block writes them where it meets (most of a
// stream's cuts can be forced ones: one per M bytes without a candidate).
struct ForcedRun {
    uint64_t at;
    int64_t s, t;
};

// All threads of the block write the queued runs.
__device__ void write_forced(uint64_t* out, uint64_t room, int64_t M,
                             const ForcedRun* fq, uint32_t nq) {
    for (uint32_t r = 0; r < nq; r++) {
        const ForcedRun f = fq[r];
        for (int64_t i = threadIdx.x; i < f.t; i += blockDim.x)
            if (f.at + (uint64_t)i < room) out[f.at + i] = (uint64_t)(f.s + (i + 1) * M);
    }
}

// Inclusive prefix sums of c[0 .. kChainChunk) in place, by the whole block
// (each thread sums kChainChunk / kChainThreads consecutive counts; a wave
// scan and the wave totals give each thread its start).
__device__ void chunk_prefix(uint32_t* c, uint32_t* wsum) {
    constexpr uint32_t kPer = kChainChunk / kChainThreads;
    uint32_t v[kPer];
    const uint32_t t = threadIdx.x, l = lane_id(), wv = t / kWave;
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; k++) {
        v[k] = c[t * kPer + k];
        sum += v[k];
    }
    uint32_t inc = sum;
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d);
        inc += l >= d ? o : 0u;
    }
    if (l == kWave - 1) wsum[wv] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (uint32_t j = 0; j < wv; j++) run += wsum[j];
#pragma unroll
    for (uint32_t k = 0; k < kPer; k++) {
        run += v[k];
        c[t * kPer + k] = run;
    }
    __syncthreads();
}

// All threads of the block call this; the block stages the segments'
// candidate counts in LDS (one parallel read per kChainChunk segments, zero
// past the job's last segment) and turns them into running totals; wave 0
// then takes the chunk's candidates 64 at a time in order, each lane finding
// its candidate's segment by a binary search of the totals (with a few
// candidates per segment, a step per segment would wait on one list load
// for each).
__device__ void maxp_chain_job(const JobView& J, const SegMeta* meta,
                               const uint32_t* cand, uint32_t* err,
                               uint32_t* lds_nc, uint32_t* wsum, int32_t* mk,
                               ForcedRun* fq, uint32_t& lds_nq) {
    const int64_t n = J.n, w = J.w, M = J.M;
    const bool walker = threadIdx.x < kWave;
    uint64_t* out = J.cuts;
    const uint64_t room = max_cuts_of(J);
    uint64_t cnt = 0;
    int64_t s = 0;
    uint32_t nq = 0;                     // queued forced runs (walker)
    // t forced cuts after s: queued (the wave writes the queue itself when
    // it is full)
    auto forced = [&](int64_t s0, int64_t t) {
        if (t <= 0) return;
        if (nq == kForcedQ) {
            for (uint32_t r = 0; r < nq; r++) {
                uint64_t at = fq[r].at;
                put_forced(out, at, room, fq[r].s, fq[r].t, M);
            }
            nq = 0;
        }
        if (lane_id() == 0) fq[nq] = ForcedRun{cnt, s0, t};
        nq++;
        cnt += (uint64_t)t;
    };
    // the 64 candidates (or fewer: q = INT64_MAX past the last) of one
    // batch, in order: accepted runs are taken 64 at a time
    auto take = [&](int64_t q, bool valid) {
        const int64_t qprev = __shfl_up(q, 1);
        uint32_t done = 0;  // lanes below `done` are settled
        for (;;) {
            // (the 64-bit remainder and quotient only where q lies M or
            // more past s: after a content cut the next candidate is
            // usually within M)
            const int64_t d = q - s;
            const bool acc = valid && lane_id() >= done && d >= 0 &&
                             (d < M ? d : d % M) >= w;
            const uint64_t ball = __ballot(acc);
            if (ball == 0) break;
            const uint32_t f = (uint32_t)__builtin_ctzll(ball);
            const int64_t qf = uni64(__shfl(q, (int)f));
            // accepted run: f, then every next candidate within M+1
            const bool brk = lane_id() > f &&
                             (!valid || (q - qprev - 1) >= M);
            const uint64_t bb = __ballot(brk);
            const uint32_t g = bb ? (uint32_t)__builtin_ctzll(bb) : 64u;
            forced(s, qf - s < M ? 0 : (qf - s) / M);
            if (lane_id() >= f && lane_id() < g &&
                cnt + (lane_id() - f) < room)
                out[cnt + (lane_id() - f)] = (uint64_t)(q + 1);
            cnt += g - f;
            s = uni64(__shfl(q, (int)(g - 1))) + 1;
            done = g;
            if (g >= 64) break;
        }
    };
    for (uint32_t cb = 0; cb < J.nseg; cb += kChainChunk) {
        const uint32_t m = min(kChainChunk, J.nseg - cb);
        uint32_t v[kChainChunk / kChainThreads];   // all loads in flight first
#pragma unroll
        for (uint32_t k = 0; k < kChainChunk / kChainThreads; k++) {
            const uint32_t i = threadIdx.x + k * kChainThreads;
            v[k] = i < m ? meta[J.item0 + cb + i].nspec : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kChainChunk / kChainThreads; k++)
            lds_nc[threadIdx.x + k * kChainThreads] = v[k];
        __syncthreads();
        if (m > 1) chunk_prefix(lds_nc, wsum);   // (one segment: its count)
        // lds_nc[i]: candidates of the chunk's segments 0 .. i (m - 1 holds
        // the chunk's total, the entries past it repeat it)
        const uint32_t total = lds_nc[m - 1];
        uint32_t kc = 0;     // the segment of the batch's first candidate, or before
        for (uint32_t base = 0; walker && base < total; base += kWave) {
            const uint32_t l = lane_id(), gi = base + l;
            const bool valid = gi < total;
            // segment kc + l: candidates [S, T) of the chunk
            const uint32_t kl = kc + l;
            const uint32_t T = kl < m ? lds_nc[kl] : total;
            const uint32_t S = kl == 0 ? 0u : kl - 1 < m ? lds_nc[kl - 1] : total;
            const uint32_t end = min(base + (uint32_t)kWave, total);
            uint32_t k, first;
            if (end <= (uint32_t)__builtin_amdgcn_readlane((int)T, kWave - 1)) {
                // the 64 segments from kc hold the batch: each segment that
                // starts in it marks its first lane, and a lane's segment is
                // the last mark at or before it (volatile: other lanes write
                // the slot a lane reads)
                volatile int32_t* vm = mk;
                vm[l] = -1;
                __builtin_amdgcn_wave_barrier();
                if (T > S && S < end && T > base) vm[S > base ? S - base : 0u] = (int32_t)l;
                __builtin_amdgcn_wave_barrier();
                int32_t v = vm[l];
#pragma unroll
                for (uint32_t d = 1; d < (uint32_t)kWave; d <<= 1) {
                    const int32_t o = __shfl_up(v, d);
                    v = l >= d ? max(v, o) : v;
                }
                __builtin_amdgcn_wave_barrier();   // (mk is rewritten next batch)
                v = max(v, 0);   // (lanes past the last candidate only)
                k = kc + (uint32_t)v;
                first = (uint32_t)__shfl((int)S, v);
            } else {
                // the segment k holding candidate gi: the first whose
                // running total exceeds gi (p: the last one at or below it,
                // -1 if none)
                int32_t p = -1;
#pragma unroll
                for (int32_t step = (int32_t)kChainChunk / 2; step > 0; step >>= 1)
                    if (p + step < (int32_t)m && lds_nc[p + step] <= gi) p += step;
                k = (uint32_t)(p + 1);
                first = k == 0 ? 0u : lds_nc[k - 1];
            }
            int64_t q = INT64_MAX;
            if (valid) {
                const uint32_t seg = cb + k;
                q = (int64_t)seg * J.seg +
                    (int64_t)cand[J.slot0 + (uint64_t)seg * J.cap + (gi - first)];
            }
            kc = (uint32_t)__builtin_amdgcn_readlane((int)k, kWave - 1);
            take(q, valid);
        }
        if (walker && lane_id() == 0) lds_nq = nq;
        __syncthreads();
        write_forced(out, room, M, fq, lds_nq);
        nq = 0;
        __syncthreads();                 // lds_nc and the queue are refilled next
    }
    if (walker && n > 0) {
        forced(s, (n - s - 1) / M);
        if (lane_id() == 0 && cnt < room) out[cnt] = (uint64_t)n;
        cnt++;
    }
    if (walker && lane_id() == 0) lds_nq = nq;
    __syncthreads();
    write_forced(out, room, M, fq, lds_nq);
    __syncthreads();                     // the queue is reused by the next job
    if (!walker) return;
    if (cnt > room) {   // cannot happen for a correct chain
        if (lane_id() == 0) atomicOr(err, kErrOverflow);
        cnt = room;
    }
    if (lane_id() == 0) *J.n_cuts = cnt;
}

__global__ __launch_bounds__(kChainThreads) void k_maxp_chain(Plan P, uint32_t n_jobs_h,
                                                    const uint32_t* n_jobs_d,
                                                    const SegMeta* meta,
                                                    const uint32_t* cand,
                                                    uint32_t* err) {
    tail_priority();
    __shared__ __align__(16) uint32_t nc[kChainChunk];
    __shared__ uint32_t wsum[kChainThreads / kWave];
    __shared__ int32_t mk[kWave];
    __shared__ ForcedRun fq[kForcedQ];
    __shared__ uint32_t nq;
    const uint32_t n_jobs = n_jobs_d ? *n_jobs_d : n_jobs_h;
    for (uint32_t job = blockIdx.x; job < n_jobs; job += gridDim.x) {
        const JobView J = view(P.jobs ? P.jobs[job] : P.one);
        if (!J.ok || J.algo != kMaxp || J.n == 0) continue;   // alike for the block
        maxp_chain_job(J, meta, cand, err, nc, wsum, mk, fq, nq);
    }
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

#define CDC_LAUNCH(MK, LVL, NAME, ...)                 \
    do {                                               \
        if (MK) (MK)->begin(NAME, LVL, st);            \
        hipLaunchKernelGGL(__VA_ARGS__);               \
        if (MK) (MK)->end(LVL, st);                    \
    } while (0)

hipError_t launch_maxp(const Plan& P, uint32_t items_upper, uint32_t jobs_upper,
                       const uint32_t* n_jobs_d, SegMeta* meta, uint32_t* cand,
                       uint8_t* bmax, int64_t* bpos, uint32_t* err, int wpb,
                       bool any_blocks, hipStream_t st, Marks* mk) {
    const dim3 blk(kWave * wpb), grid((items_upper + wpb - 1) / wpb);
    if (any_blocks)
        CDC_LAUNCH(mk, 1, "maxp_blocks", k_maxp_blocks, grid, blk, 0, st, P,
                   bmax, bpos, err);
    CDC_LAUNCH(mk, any_blocks ? 2 : 1, "maxp_verify", k_maxp_verify, grid, blk,
               0, st, P, bmax, bpos, meta, cand, err);
    const uint32_t jgrid = min(jobs_upper, 2048u);
    CDC_LAUNCH(mk, 2, "maxp_chain", k_maxp_chain, dim3(jgrid), dim3(kChainThreads), 0, st,
               P, jobs_upper, n_jobs_d, meta, cand, err);
    return hipGetLastError();
}

}  // namespace cdc

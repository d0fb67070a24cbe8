// Chunk fingerprints and an on-device count of distinct chunks: the step of
// the deduplication pipeline that follows chunking (Section 2: chunks are
// fingerprinted with a collision-resistant hash and compared against the
// fingerprints already stored; Section 6.2 compares the time of this step
// with chunking, using xxHash3 and SHA-256).
//
// Fingerprint: SHA-256 (FIPS 180-4) of each chunk's bytes.  The hash is
// serial within a message (each 64-byte block updates the state of the one
// before), so one lane hashes one chunk; the wave's 64 lanes hash 64
// chunks side by side.  A lane reads its chunk as aligned 16-byte granules
// (the granule that holds a chunk's first byte may start before it; bytes
// outside the chunk are never hashed) and assembles each block's sixteen
// big-endian words with byte funnel shifts, carrying the granule that
// straddles two blocks.
//
// Distinct chunks: an open-addressing table keyed by the first 64 bits of
// the digest (low bit forced to 1, so 0 marks an empty slot).  The first
// pass inserts every chunk (the lane whose compare-and-swap claims an empty
// slot stores the rest of the digest and the length there, and counts the
// chunk's bytes as unique); the second pass compares every chunk with what
// its slot holds, and counts a chunk whose 64-bit key matched a different
// digest or length as a collision (and as unique bytes).
#include "fingerprint.h"
#include "wave.h"

namespace cdc {

// Sum over the 64 lanes, returned to every lane.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint64_t)__shfl_xor((long long)v, o, kWave);
    return v;
}

// Round constants and initial state of SHA-256 (FIPS 180-4, Sections 4.2.2
// and 5.3.3): the first 32 bits of the fractional parts of the cube roots
// of the first 64 primes, and of the square roots of the first 8 primes.
__constant__ uint32_t kSha256K[64] = {
    0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u,
    0x923f82a4u, 0xab1c5ed5u, 0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u,
    0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u, 0xe49b69c1u, 0xefbe4786u,
    0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau,
    0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u,
    0x06ca6351u, 0x14292967u, 0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u,
    0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u, 0xa2bfe8a1u, 0xa81a664bu,
    0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u,
    0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au,
    0x5b9cca4fu, 0x682e6ff3u, 0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u,
    0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u};
constexpr uint32_t kSha256H0[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u,
                                   0xa54ff53au, 0x510e527fu, 0x9b05688cu,
                                   0x1f83d9abu, 0x5be0cd19u};

__device__ __forceinline__ uint32_t rotr(uint32_t x, int r) {
    return __builtin_rotateright32(x, (uint32_t)r);
}

// One compression of the 16 big-endian message words w into the state h.
__device__ __forceinline__ void sha256_block(uint32_t (&h)[8], uint32_t (&w)[16]) {
    uint32_t a = h[0], b = h[1], c = h[2], d = h[3];
    uint32_t e = h[4], f = h[5], g = h[6], k = h[7];
#pragma unroll
    for (int t = 0; t < 64; t++) {
        uint32_t wt;
        if (t < 16) {
            wt = w[t];
        } else {
            // message schedule in place: w[t mod 16] becomes W_t
            const uint32_t w15 = w[(t - 15) & 15], w2 = w[(t - 2) & 15];
            const uint32_t s0 = rotr(w15, 7) ^ rotr(w15, 18) ^ (w15 >> 3);
            const uint32_t s1 = rotr(w2, 17) ^ rotr(w2, 19) ^ (w2 >> 10);
            wt = w[t & 15] + s0 + w[(t - 7) & 15] + s1;
            w[t & 15] = wt;
        }
        const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
        const uint32_t ch = (e & f) ^ (~e & g);
        const uint32_t t1 = k + S1 + ch + kSha256K[t] + wt;
        const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
        const uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
        const uint32_t t2 = S0 + maj;
        k = g;
        g = f;
        f = e;
        e = d + t1;
        d = c;
        c = b;
        b = a;
        a = t1 + t2;
    }
    h[0] += a; h[1] += b; h[2] += c; h[3] += d;
    h[4] += e; h[5] += f; h[6] += g; h[7] += k;
}

__device__ __forceinline__ uint4 load_granule(const uint4* g) {
    const u32x4 v = __builtin_nontemporal_load((const global_u32x4*)g);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// SHA-256 of the bytes [p, p + len) into out (32 bytes, big-endian words).
__device__ void sha256_chunk(const uint8_t* p, uint64_t len, uint8_t* out) {
    uint32_t h[8];
#pragma unroll
    for (int i = 0; i < 8; i++) h[i] = kSha256H0[i];
    const uintptr_t a = (uintptr_t)p;
    const uint4* g = (const uint4*)(a & ~(uintptr_t)15);
    const int s = (int)(a & 15);
    const uint64_t full = len >> 6;
    // q holds granules 0..4 of the current block's window as 20 dwords; the
    // fifth granule (needed when s > 0) is the next block's first
    uint4 carry = len > 0 ? load_granule(g) : make_uint4(0, 0, 0, 0);
    for (uint64_t blk = 0; blk < full; blk++) {
        const uint4 g1 = load_granule(g + 1), g2 = load_granule(g + 2),
                    g3 = load_granule(g + 3);
        // the fifth granule holds bytes of this block only when s > 0
        const bool need5 = s > 0;
        const uint4 g4 = need5 ? load_granule(g + 4) : make_uint4(0, 0, 0, 0);
        const uint32_t q[20] = {carry.x, carry.y, carry.z, carry.w, g1.x, g1.y,
                                g1.z, g1.w, g2.x, g2.y, g2.z, g2.w, g3.x, g3.y,
                                g3.z, g3.w, g4.x, g4.y, g4.z, g4.w};
        uint32_t w[16];
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const int k = i + (s >> 2);
            const uint32_t lo = q[k], hi = q[k + 1 < 20 ? k + 1 : 19];
            w[i] = __builtin_bswap32(__builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(s & 3)));
        }
        sha256_block(h, w);
        g += 4;
        // the next block's (or the tail's) first granule, if it holds any
        // byte of the chunk
        const bool more = blk + 1 < full || (len & 63) != 0;
        carry = need5 ? g4 : (more ? load_granule(g) : make_uint4(0, 0, 0, 0));
    }
    // the last len mod 64 bytes, the 0x80 byte, zeros and the bit length
    const int r = (int)(len & 63);
    uint32_t tail[16];
#pragma unroll
    for (int i = 0; i < 16; i++) tail[i] = 0;
    if (r > 0) {
        // bytes [0, r) of the remaining stretch, from granules g[0..4]
        const int ng = (s + r + 15) >> 4;          // granules holding them
        uint32_t q[20];
        q[0] = carry.x; q[1] = carry.y; q[2] = carry.z; q[3] = carry.w;
#pragma unroll
        for (int j = 1; j < 5; j++) {
            const uint4 v = j < ng ? load_granule(g + j) : make_uint4(0, 0, 0, 0);
            q[4 * j] = v.x; q[4 * j + 1] = v.y; q[4 * j + 2] = v.z; q[4 * j + 3] = v.w;
        }
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const int k = i + (s >> 2);
            const uint32_t lo = q[k], hi = q[k + 1 < 20 ? k + 1 : 19];
            uint32_t v = __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(s & 3));
            // keep bytes [0, r) of the stretch
            const int keep = min(max(r - 4 * i, 0), 4);
            v &= keep >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keep)) - 1u);
            tail[i] = v;
        }
    }
    // the 0x80 byte right after the message (little-endian dword view)
    tail[r >> 2] |= 0x80u << (8 * (r & 3));
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 16; i++) w[i] = __builtin_bswap32(tail[i]);
    const uint64_t bits = len * 8;
    if (r >= 56) {                                 // the length needs a block of its own
        sha256_block(h, w);
#pragma unroll
        for (int i = 0; i < 16; i++) w[i] = 0;
    }
    w[14] = (uint32_t)(bits >> 32);
    w[15] = (uint32_t)bits;
    sha256_block(h, w);
    uint32_t* o = (uint32_t*)out;
#pragma unroll
    for (int i = 0; i < 8; i++) o[i] = __builtin_bswap32(h[i]);
}

// One lane per chunk, grid-stride over the chunks of the cut list.
__global__ __launch_bounds__(256) void k_fingerprint(const uint8_t* data,
                                                     uint64_t n,
                                                     const uint64_t* cuts,
                                                     const uint64_t* n_cuts,
                                                     uint64_t max_cuts,
                                                     uint8_t* digests) {
    const uint64_t k_cuts = min(*n_cuts, max_cuts);
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < k_cuts;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = k == 0 ? 0 : min(cuts[k - 1], n);
        const uint64_t b = min(cuts[k], n);
        sha256_chunk(data + a, b > a ? b - a : 0, digests + 32 * k);
    }
}

// ------------------------------------------------------------ distinct chunks

__device__ __forceinline__ uint64_t dedup_key(const uint64_t* d) {
    return d[0] | 1ull;
}

__device__ __forceinline__ uint64_t hash_slot(uint64_t key, uint64_t mask) {
    // the digest is already uniform; fold its bits for the index
    return (key ^ (key >> 29)) & mask;
}

__global__ __launch_bounds__(256) void k_dedup_insert(DedupDev D,
                                                      const uint8_t* digests,
                                                      const uint64_t* cuts,
                                                      const uint64_t* n_cuts,
                                                      uint64_t max_cuts) {
    const uint64_t k_cuts = min(*n_cuts, max_cuts);
    uint64_t tot = 0, uniq = 0, nuniq = 0;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < k_cuts;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t len = cuts[k] - (k == 0 ? 0 : cuts[k - 1]);
        const uint64_t* dg = (const uint64_t*)(digests + 32 * k);
        const uint64_t key = dedup_key(dg);
        uint64_t slot = hash_slot(key, D.mask);
        tot += len;
        for (uint64_t probe = 0;; probe++) {
            if (probe > D.mask) {                  // the table is full
                atomicOr((unsigned int*)&D.ctr[kDedupFlags], 1u);
                break;
            }
            const uint64_t old = atomicCAS((unsigned long long*)&D.keys[slot], 0ull,
                                           (unsigned long long)key);
            if (old == 0) {                        // this chunk claims the slot
                DedupSlot& e = D.slots[slot];
                e.d1 = dg[1];
                e.d2 = dg[2];
                e.d3 = dg[3];
                e.len = len;
                uniq += len;
                nuniq++;
                break;
            }
            if (old == key) break;                 // the key is there already
            slot = (slot + 1) & D.mask;
        }
    }
    // one atomic per wave and counter
    tot = wave_sum64(tot);
    uniq = wave_sum64(uniq);
    nuniq = wave_sum64(nuniq);
    if (lane_id() == 0 && tot)
        atomicAdd((unsigned long long*)&D.ctr[kDedupTotalBytes], (unsigned long long)tot);
    if (lane_id() == 0 && nuniq) {
        atomicAdd((unsigned long long*)&D.ctr[kDedupUniqueBytes], (unsigned long long)uniq);
        atomicAdd((unsigned long long*)&D.ctr[kDedupUniqueChunks], (unsigned long long)nuniq);
    }
}

// Every chunk against the slot its key names: a different digest or length
// there is a collision of the 64-bit keys (the chunk is distinct content).
__global__ __launch_bounds__(256) void k_dedup_verify(DedupDev D,
                                                      const uint8_t* digests,
                                                      const uint64_t* cuts,
                                                      const uint64_t* n_cuts,
                                                      uint64_t max_cuts) {
    const uint64_t k_cuts = min(*n_cuts, max_cuts);
    uint64_t coll = 0, cbytes = 0, chunks = 0;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < k_cuts;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t len = cuts[k] - (k == 0 ? 0 : cuts[k - 1]);
        const uint64_t* dg = (const uint64_t*)(digests + 32 * k);
        const uint64_t key = dedup_key(dg);
        uint64_t slot = hash_slot(key, D.mask);
        chunks++;
        for (uint64_t probe = 0; probe <= D.mask; probe++) {
            const uint64_t cur = D.keys[slot];
            if (cur == key) {
                const DedupSlot& e = D.slots[slot];
                if (e.d1 != dg[1] || e.d2 != dg[2] || e.d3 != dg[3] || e.len != len) {
                    coll++;
                    cbytes += len;
                }
                break;
            }
            if (cur == 0) break;                   // not inserted (table full)
            slot = (slot + 1) & D.mask;
        }
    }
    coll = wave_sum64(coll);
    cbytes = wave_sum64(cbytes);
    chunks = wave_sum64(chunks);
    if (lane_id() == 0 && chunks)
        atomicAdd((unsigned long long*)&D.ctr[kDedupChunks], (unsigned long long)chunks);
    if (lane_id() == 0 && coll) {
        atomicAdd((unsigned long long*)&D.ctr[kDedupCollisions], (unsigned long long)coll);
        atomicAdd((unsigned long long*)&D.ctr[kDedupUniqueBytes], (unsigned long long)cbytes);
        atomicAdd((unsigned long long*)&D.ctr[kDedupUniqueChunks], (unsigned long long)coll);
    }
}

__global__ void k_dedup_clear(DedupDev D) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= D.mask;
         i += (uint64_t)gridDim.x * blockDim.x)
        D.keys[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < kDedupCounters) D.ctr[threadIdx.x] = 0;
}

static uint32_t grid_for(uint64_t items) {
    const uint64_t g = (items + 255) / 256;
    return (uint32_t)max((uint64_t)1, min(g, (uint64_t)8192));
}

hipError_t launch_fingerprint(const uint8_t* data, uint64_t n,
                              const uint64_t* cuts, const uint64_t* n_cuts,
                              uint64_t max_cuts, uint8_t* digests,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_fingerprint, dim3(grid_for(max_cuts)), dim3(256), 0, st,
                       data, n, cuts, n_cuts, max_cuts, digests);
    return hipGetLastError();
}

hipError_t launch_dedup_add(const DedupDev& D, const uint8_t* digests,
                            const uint64_t* cuts, const uint64_t* n_cuts,
                            uint64_t max_cuts, hipStream_t st) {
    const dim3 g(grid_for(max_cuts)), b(256);
    hipLaunchKernelGGL(k_dedup_insert, g, b, 0, st, D, digests, cuts, n_cuts, max_cuts);
    hipLaunchKernelGGL(k_dedup_verify, g, b, 0, st, D, digests, cuts, n_cuts, max_cuts);
    return hipGetLastError();
}

hipError_t launch_dedup_clear(const DedupDev& D, hipStream_t st) {
    hipLaunchKernelGGL(k_dedup_clear, dim3(grid_for(D.mask + 1)), dim3(256), 0, st, D);
    return hipGetLastError();
}

}  // namespace cdc

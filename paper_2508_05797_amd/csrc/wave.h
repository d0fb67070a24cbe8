// Device-side helpers shared by the HIP kernels of libcdc: wavefront
// reductions (DPP), SWAR byte operations on a lane's 16 bytes, the byte
// source of a job, and job / work-item access.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cdc_internal.h"

namespace cdc {


// ------------------------------------------------------------ wave basics

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// The passes that follow a streaming pass (a few long walkers, one block
// per job) raise their waves' issue priority: where a batch runs them beside
// another algorithm's streaming pass on the same SIMDs, their instructions
// issue first and the streaming waves fill the gaps.
__device__ __forceinline__ void tail_priority() { __builtin_amdgcn_s_setprio(3); }

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
// Global-address-space view: global loads count only against vmcnt, while
// flat loads also hold lgkmcnt, which LDS accesses wait on.
typedef __attribute__((address_space(1))) const u32x4 global_u32x4;

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
            const u32x4 q =
                __builtin_nontemporal_load((const global_u32x4*)(base + g));
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

// ------------------------------------------------------------ job access

struct JobView {
    const uint8_t* data;
    int64_t n, w, M, seg;
    uint32_t algo, nseg, item0, cap, ok, blog;
    uint64_t slot0, blk0, idx0;
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
    v.idx0 = (uint64_t)uni64((int64_t)J.idx0);
    v.cuts = (uint64_t*)uni64((int64_t)J.cuts);
    v.n_cuts = (uint64_t*)uni64((int64_t)J.n_cuts);
    return v;
}

__device__ __forceinline__ uint32_t wave_global_id() {
    return uni(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
}

__device__ __forceinline__ uint32_t wave_count() {
    return gridDim.x * (blockDim.x / kWave);
}

// Number of work items of the plan (uniform).
__device__ __forceinline__ uint32_t item_count(const Plan& P) {
    return P.jobs == nullptr ? P.one_items : uni(*P.n_items);
}

// Items [first, last) of algorithm `algo` (with one job: all of its items if
// it runs that algorithm).
__device__ __forceinline__ void item_range(const Plan& P, uint32_t algo,
                                           uint32_t& first, uint32_t& last) {
    if (P.jobs == nullptr) {
        first = 0;
        last = P.one.algo == algo ? P.one_items : 0u;
    } else {
        first = uni(P.n_items[2 + algo]);
        last = uni(P.n_items[6 + algo]);
    }
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

__device__ __forceinline__ uint64_t max_cuts_of(const JobView& J) {
    return J.n == 0 ? 0 : (uint64_t)(J.n - 1) / (uint64_t)(J.w + 1) + 1;
}

}  // namespace cdc

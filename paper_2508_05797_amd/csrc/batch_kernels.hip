// Batch planning on the device: many independent buffers (the many-file
// case) chunked by one set of launches.
//
// k_plan reads the caller's job descriptors, validates each job, splits it
// into segments (work items), and lays out every job's slots in the shared
// workspace with exclusive scans over the jobs.  Sizes are only known on the
// device, so the launches that follow are sized by the reserved upper bound
// and walk the real item count grid-stride; the whole sequence can be
// captured into a HIP graph and replayed with new descriptor contents.
#include "cdc.h"
#include "wave.h"

namespace cdc {

static_assert(sizeof(cdc_job) == 48, "cdc_job layout");

__device__ __forceinline__ uint32_t blog_for(uint32_t w) {
    const uint64_t b = min((uint64_t)w + 1, (uint64_t)kTile);
    uint32_t lg = 0;
    while ((2ull << lg) <= b) lg++;
    return lg >= 4 ? lg : 0;
}

// Exclusive scan over the block of one value per thread (blockDim <= 1024).
__device__ uint64_t plan_exscan(uint64_t v, uint64_t* sh, uint64_t& total) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    sh[tid] = v;
    __syncthreads();
    for (uint32_t o = 1; o < nt; o <<= 1) {
        const uint64_t add = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    total = sh[nt - 1];
    const uint64_t ex = sh[tid] - v;
    __syncthreads();
    return ex;
}

__global__ __launch_bounds__(1024) void k_plan(cdc_job* jobs, uint32_t n_jobs,
                                               BatchCaps caps, JobDesc* jd,
                                               Item* items,
                                               uint32_t* n_items) {
    __shared__ uint64_t sh[1024];
    __shared__ uint32_t overflow;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    uint64_t c_items = 0, c_slots = 0, c_blocks = 0;
    for (uint32_t base = 0; base < n_jobs; base += nt) {
        const uint32_t j = base + tid;
        uint64_t nseg = 0, slots = 0, blocks = 0;
        JobDesc d{};
        if (j < n_jobs) {
            const cdc_job q = jobs[j];
            const bool ok = q.algo <= 3 && q.window >= 1 &&
                            (uint64_t)q.max_chunk >= (uint64_t)q.window + 1 &&
                            (uint64_t)q.max_chunk <= caps.max_chunk_limit &&
                            q.n_cuts != nullptr &&
                            (q.n == 0 || (q.data && q.cut_offsets));
            d.data = q.data;
            d.n = q.n;
            d.cuts = q.cut_offsets;
            d.n_cuts = q.n_cuts;
            d.status = &jobs[j].status;
            d.algo = q.algo;
            d.w = q.window;
            d.M = q.max_chunk;
            d.ok = ok ? 1 : 0;
            if (ok && q.n > 0) {
                const bool maxp = q.algo == kMaxp;
                d.seg = maxp ? caps.seg_maxp : caps.seg_chain;
                nseg = (q.n + d.seg - 1) / d.seg;
                const uint64_t span = maxp ? d.seg + kTile : d.seg + q.max_chunk;
                uint64_t cap = span / ((uint64_t)q.window + 1) + 2;
                // a job's chains never hold more cuts than the job has
                cap = min(cap, (q.n + kTile) / ((uint64_t)q.window + 1) + 2);
                d.cap = (uint32_t)cap;
                slots = nseg * cap;
                d.blog = maxp ? blog_for(q.window) : 0;
                if (maxp && d.blog) {
                    const uint64_t shift = (uintptr_t)q.data & 15;
                    blocks = (q.n + shift + kTile - 1) / kTile *
                             ((uint64_t)kTile >> d.blog);
                }
            }
            d.nseg = (uint32_t)nseg;
        }
        uint64_t t_items, t_slots, t_blocks;
        const uint64_t e_items = plan_exscan(nseg, sh, t_items);
        const uint64_t e_slots = plan_exscan(slots, sh, t_slots);
        const uint64_t e_blocks = plan_exscan(blocks, sh, t_blocks);
        if (j < n_jobs) {
            d.item0 = (uint32_t)(c_items + e_items);
            d.slot0 = c_slots + e_slots;
            d.blk0 = c_blocks + e_blocks;
            jd[j] = d;
        }
        c_items += t_items;
        c_slots += t_slots;
        c_blocks += t_blocks;
    }
    if (tid == 0)
        overflow = (c_items > caps.items || c_slots > caps.slots ||
                    c_blocks > caps.blocks)
                       ? 1u
                       : 0u;
    __syncthreads();
    const bool over = overflow != 0;
    if (tid == 0) *n_items = over ? 0u : (uint32_t)c_items;
    // statuses, zero counts for empty or rejected jobs, and the item table
    for (uint32_t j = tid; j < n_jobs; j += nt) {
        JobDesc& d = jd[j];
        const bool valid = d.ok != 0;
        if (over) d.ok = 0;
        jobs[j].status = over ? CDC_ENOMEM : (valid ? CDC_OK : CDC_EINVAL);
        if (!d.ok || d.n == 0) {
            if (d.n_cuts) *d.n_cuts = 0;
            continue;
        }
        for (uint32_t s = 0; s < d.nseg; s++) items[d.item0 + s] = Item{j, s};
    }
}

hipError_t launch_plan(cdc_job* jobs, uint32_t n_jobs, const BatchCaps& caps,
                       JobDesc* jd, Item* items, uint32_t* n_items,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, jobs, n_jobs, caps,
                       jd, items, n_items);
    return hipGetLastError();
}

}  // namespace cdc

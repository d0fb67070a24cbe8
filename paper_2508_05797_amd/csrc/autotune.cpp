// Autotuner for batched chunking: picks the segment lengths and the waves
// per workgroup that run a given batch fastest on this device, by timing the
// batch itself (coordinate descent over a small grid, HIP events on the
// caller's stream).  Tuning changes only speed, never the offsets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "cdc.h"

namespace {

using Key = std::tuple<int, uint32_t, uint64_t, uint64_t, uint64_t, uint32_t>;
std::mutex g_tune_mu;
std::map<Key, cdc_tuning> g_tuned;

// The jobs' statuses after a run: a trial whose batch did not fit the
// workspace (CDC_ENOMEM on the jobs) fails the tuning instead of being timed
// as if it had run.  Invalid jobs (CDC_EINVAL) are the caller's and do not.
int batch_status(const cdc_job* jobs, uint32_t n_jobs, hipStream_t st) {
    std::vector<cdc_job> h(n_jobs);
    if (hipMemcpyAsync(h.data(), jobs, n_jobs * sizeof(cdc_job),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return CDC_EHIP;
    for (const cdc_job& q : h)
        if (q.status != CDC_OK && q.status != CDC_EINVAL) return q.status;
    return CDC_OK;
}

// Average milliseconds of one batch under tuning t (after one untimed run).
int time_batch(const cdc_job* jobs, uint32_t n_jobs, hipStream_t st,
               const cdc_tuning& t, uint64_t T, uint32_t wmin, uint32_t mmax,
               uint32_t reps, hipEvent_t e0, hipEvent_t e1, double* ms) {
    int rc = cdc_set_tuning(&t);
    if (rc == CDC_OK) rc = cdc_reserve(st, T, n_jobs, wmin, mmax);
    if (rc == CDC_OK) rc = cdc_chunk_batch(jobs, n_jobs, st);
    if (rc != CDC_OK) return rc;
    if (hipEventRecord(e0, st) != hipSuccess) return CDC_EHIP;
    for (uint32_t r = 0; r < reps; r++) {
        rc = cdc_chunk_batch(jobs, n_jobs, st);
        if (rc != CDC_OK) return rc;
    }
    float f = 0;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&f, e0, e1) != hipSuccess)
        return CDC_EHIP;
    *ms = f / reps;
    return batch_status(jobs, n_jobs, st);
}

}  // namespace

extern "C" int cdc_autotune(const cdc_job* jobs, uint32_t n_jobs,
                            hipStream_t stream, uint32_t reps,
                            cdc_tuning* chosen) {
    if (!jobs || n_jobs == 0 || reps == 0) return CDC_EINVAL;
    std::vector<cdc_job> h(n_jobs);
    if (hipMemcpyAsync(h.data(), jobs, n_jobs * sizeof(cdc_job),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return CDC_EHIP;
    uint64_t T = 0;
    uint32_t wmin = ~0u, mmax = 2, mask = 0;
    for (const cdc_job& q : h) {
        if (q.algo > 3 || q.window == 0) continue;
        T += q.n;
        wmin = std::min(wmin, q.window);
        mmax = std::max(mmax, q.max_chunk);
        mask |= 1u << q.algo;
    }
    if (mask == 0) return CDC_EINVAL;
    // reservation bounds (jobs beyond the chunk limit are invalid anyway)
    mmax = (uint32_t)std::min<uint64_t>(
        std::max<uint64_t>(mmax, (uint64_t)wmin + 1), 1u << 28);
    int dev = 0;
    (void)hipGetDevice(&dev);
    const Key key{dev, n_jobs, T, wmin, mmax, mask};
    cdc_tuning best{};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            best = it->second;
            int rc = cdc_set_tuning(&best);
            if (rc == CDC_OK) rc = cdc_reserve(stream, T, n_jobs, wmin, mmax);
            if (rc == CDC_OK && chosen) *chosen = best;
            return rc;
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return CDC_EHIP;
    int rc = cdc_get_tuning(&best);
    double best_ms = 0;
    if (rc == CDC_OK)
        rc = time_batch(jobs, n_jobs, stream, best, T, wmin, mmax, reps, e0, e1,
                        &best_ms);
    const bool chain = (mask & ~(1u << CDC_MAXP)) != 0;
    const bool maxp = (mask & (1u << CDC_MAXP)) != 0;
    const std::vector<uint64_t> chain_segs = {256 << 10, 512 << 10, 1 << 20,
                                              2 << 20, 4 << 20};
    const std::vector<uint64_t> maxp_segs = {16 << 10, 32 << 10, 64 << 10,
                                             128 << 10, 256 << 10, 512 << 10,
                                             1 << 20};
    const std::vector<uint32_t> waves = {1, 2, 4};
    // one coordinate at a time
    for (int dim = 0; dim < 3 && rc == CDC_OK; dim++) {
        if ((dim == 0 && !chain) || (dim == 1 && !maxp)) continue;
        const size_t k = dim == 0 ? chain_segs.size()
                                  : dim == 1 ? maxp_segs.size() : waves.size();
        cdc_tuning base = best;
        for (size_t i = 0; i < k && rc == CDC_OK; i++) {
            cdc_tuning t = base;
            if (dim == 0) t.chain_segment = chain_segs[i];
            if (dim == 1) t.maxp_segment = maxp_segs[i];
            if (dim == 2) t.waves_per_block = waves[i];
            if (t.chain_segment == base.chain_segment &&
                t.maxp_segment == base.maxp_segment &&
                t.waves_per_block == base.waves_per_block)
                continue;
            double ms = 0;
            rc = time_batch(jobs, n_jobs, stream, t, T, wmin, mmax, reps, e0, e1, &ms);
            if (rc == CDC_OK && ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != CDC_OK) return rc;
    rc = cdc_set_tuning(&best);
    if (rc == CDC_OK) rc = cdc_reserve(stream, T, n_jobs, wmin, mmax);
    if (rc != CDC_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[key] = best;
    }
    if (chosen) *chosen = best;
    return CDC_OK;
}

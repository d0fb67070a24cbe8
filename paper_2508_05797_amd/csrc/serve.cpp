// The HIP executor of the request loop (include/cdc_serve.h): a pool of
// streams, one batch in flight per stream.  A launch copies the batch's
// descriptors from pinned host memory, runs cdc_chunk_batch, copies the
// descriptors (with their statuses) back and records an event; completion
// is polled with hipEventQuery.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "cdc.h"
#include "cdc_internal.h"
#include "cdc_serve.h"
#include "serve_sched.h"

namespace {

constexpr uint32_t kMaxSlots = 16;
constexpr uint32_t kMaxBatch = 65536;

uint64_t max_cuts(uint64_t n, uint32_t w) {
    return n == 0 ? 0 : (n - 1) / ((uint64_t)w + 1) + 1;
}

class HipExecutor final : public serve::Executor {
public:
    HipExecutor(const uint8_t* pool, uint64_t* cuts, uint64_t* n_cuts,
                const cdc_request* reqs, int32_t* status)
        : pool_(pool), cuts_(cuts), n_cuts_(n_cuts), reqs_(reqs),
          status_(status) {}

    ~HipExecutor() override {
        for (Slot& s : slots_) {
            if (s.stream) {
                (void)hipStreamSynchronize(s.stream);
                cdc::drop_workspace(s.stream);
            }
            if (s.ev) (void)hipEventDestroy(s.ev);
            if (s.dev) (void)hipFree(s.dev);
            if (s.host) (void)hipHostFree(s.host);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
        if (scratch_) (void)hipFree(scratch_);
    }

    int setup(uint32_t n_slots, uint32_t max_batch, uint64_t budget,
              uint32_t min_window, uint32_t max_chunk) {
        slots_.resize(n_slots);
        for (Slot& s : slots_) {
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void**)&s.host, max_batch * sizeof(cdc_job),
                              hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void**)&s.dev, max_batch * sizeof(cdc_job)) != hipSuccess)
                return CDC_EHIP;
            const int rc = cdc_reserve(s.stream, budget, max_batch, min_window,
                                       max_chunk);
            if (rc != CDC_OK) return rc;
            // touch the pinned descriptors now, not while serving
            memset(s.host, 0, max_batch * sizeof(cdc_job));
        }
        // one empty batch per slot, so that no request pays for the first
        // use of a stream and its launches
        if (hipMalloc(&scratch_, 2 * sizeof(uint64_t)) != hipSuccess) return CDC_EHIP;
        for (Slot& s : slots_) {
            cdc_job& j = s.host[0];
            j.data = pool_;
            j.n = 0;
            j.cut_offsets = (uint64_t*)scratch_;
            j.n_cuts = (uint64_t*)scratch_ + 1;
            j.algo = CDC_RAM;
            j.window = min_window;
            j.max_chunk = max_chunk;
            j.status = 0;
            if (hipMemcpyAsync(s.dev, s.host, sizeof(cdc_job), hipMemcpyHostToDevice,
                               s.stream) != hipSuccess ||
                cdc::batch_run(s.dev, 1, 0, false, s.stream) != CDC_OK)
                return CDC_EHIP;
        }
        for (Slot& s : slots_)
            if (hipStreamSynchronize(s.stream) != hipSuccess) return CDC_EHIP;
        t0_ = std::chrono::steady_clock::now();
        return CDC_OK;
    }

    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_)
            .count();
    }

    bool launch(int slot, const std::vector<uint32_t>& batch) override {
        Slot& s = slots_[slot];
        for (size_t k = 0; k < batch.size(); k++) {
            const cdc_request& q = reqs_[batch[k]];
            cdc_job& j = s.host[k];
            j.data = pool_ + q.offset;
            j.n = q.n;
            j.cut_offsets = cuts_ + q.cut_base;
            j.n_cuts = n_cuts_ + batch[k];
            j.algo = q.algo;
            j.window = q.window;
            j.max_chunk = q.max_chunk;
            j.status = 0;
        }
        uint64_t total = 0, ram_max = 0;
        uint32_t mask = 0;
        for (size_t k = 0; k < batch.size(); k++) {
            total += s.host[k].n;
            mask |= 1u << (s.host[k].algo & 3u);
            if (s.host[k].algo == CDC_RAM) ram_max = std::max<uint64_t>(ram_max, s.host[k].n);
        }
        const size_t bytes = batch.size() * sizeof(cdc_job);
        if (hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice,
                           s.stream) != hipSuccess)
            return false;
        // batches overlap across slots; within one, the algorithms run in order
        // only the passes of the algorithms the batch holds
        if (cdc::batch_run(s.dev, (uint32_t)batch.size(), total, false, s.stream,
                           mask, ram_max) != CDC_OK)
            return false;
        if (hipMemcpyAsync(s.host, s.dev, bytes, hipMemcpyDeviceToHost,
                           s.stream) != hipSuccess ||
            hipEventRecord(s.ev, s.stream) != hipSuccess)
            return false;
        s.batch = batch;
        s.running = true;
        return true;
    }

    bool done(int slot) override {
        Slot& s = slots_[slot];
        if (!s.running) return false;
        const hipError_t e = hipEventQuery(s.ev);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) error_ = true;
        for (size_t k = 0; k < s.batch.size(); k++)
            status_[s.batch[k]] = e == hipSuccess ? s.host[k].status : CDC_EHIP;
        s.running = false;
        return true;
    }

    void idle(double until) override {
        while (now() < until) {
            for (Slot& s : slots_)
                if (s.running && hipEventQuery(s.ev) != hipErrorNotReady) return;
        }
    }

    bool error() const { return error_; }

private:
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t ev = nullptr;
        cdc_job* host = nullptr;
        cdc_job* dev = nullptr;
        std::vector<uint32_t> batch;
        bool running = false;
    };
    const uint8_t* pool_;
    uint64_t* cuts_;
    uint64_t* n_cuts_;
    const cdc_request* reqs_;
    int32_t* status_;
    std::vector<Slot> slots_;
    std::chrono::steady_clock::time_point t0_;
    void* scratch_ = nullptr;            // outputs of the warm-up batches
    bool error_ = false;
};

}  // namespace

extern "C" int cdc_serve(const uint8_t* pool, uint64_t pool_bytes,
                         uint64_t* cuts, uint64_t* n_cuts,
                         const cdc_request* reqs, uint32_t n_req,
                         const cdc_serve_config* cfg, double* latency,
                         int32_t* status, cdc_serve_stats* stats) {
    if (!cfg || !reqs || !latency || !status || !n_cuts || !cuts || !pool ||
        n_req == 0 || cfg->max_batch == 0 || cfg->max_batch > kMaxBatch ||
        cfg->slots == 0 || cfg->slots > kMaxSlots || cfg->min_window == 0 ||
        (uint64_t)cfg->max_chunk < (uint64_t)cfg->min_window + 1)
        return CDC_EINVAL;
    uint64_t budget = cfg->budget_bytes;
    if (budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return CDC_EHIP;
        budget = free_b / 2;
    }
    // Requests: validity and cost.
    std::vector<serve::Request> rq(n_req);
    double last_arrival = 0;
    for (uint32_t i = 0; i < n_req; i++) {
        const cdc_request& q = reqs[i];
        if (q.arrival < last_arrival) return CDC_EINVAL;
        last_arrival = q.arrival;
        const bool ok = q.algo <= 3 && q.reserved == 0 &&
                        q.window >= cfg->min_window &&
                        q.max_chunk <= cfg->max_chunk &&
                        (uint64_t)q.max_chunk >= (uint64_t)q.window + 1 &&
                        q.offset <= pool_bytes && q.n <= pool_bytes - q.offset;
        rq[i].arrival = q.arrival;
        rq[i].valid = ok;
        rq[i].cost = q.n + 8 * max_cuts(q.n, q.window ? q.window : 1);
        latency[i] = -1.0;
        status[i] = ok ? CDC_OK : CDC_EINVAL;
    }
    HipExecutor ex(pool, cuts, n_cuts, reqs, status);
    int rc = ex.setup(cfg->slots, cfg->max_batch, budget, cfg->min_window,
                      cfg->max_chunk);
    if (rc != CDC_OK) return rc;
    const serve::Config sc{budget, cfg->max_batch, cfg->slots};
    const serve::Result R = serve::run(sc, rq, ex);
    uint64_t bytes = 0;
    for (uint32_t i = 0; i < n_req; i++) {
        latency[i] = R.latency[i];
        if (R.outcome[i] == serve::kRejectedBudget) status[i] = CDC_ENOMEM;
        if (R.outcome[i] == serve::kPending) status[i] = CDC_EHIP;
        if (R.outcome[i] == serve::kDone && status[i] == CDC_OK)
            bytes += reqs[i].n;
    }
    if (stats) {
        stats->elapsed = R.last_finish;
        stats->launches = R.launches;
        stats->rejected = R.rejected;
        stats->bytes_done = bytes;
        stats->budget_bytes = budget;
        stats->max_queue = R.max_queue;
        stats->max_inflight = R.max_inflight;
    }
    if (R.error || ex.error()) return CDC_EHIP;
    return CDC_OK;
}

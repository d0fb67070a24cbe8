// Test helper: the request scheduler of the library driven by a simulated
// device on a virtual clock.  Each batch takes base + per_byte * (its bytes)
// seconds, slots run independently.  Built by tests/test_serve_sched.py.
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "serve_sched.h"

namespace {

struct SimExecutor final : serve::Executor {
    double t = 0, base = 0, per_byte = 0;
    const uint64_t* cost = nullptr;
    std::vector<double> finish;          // per slot, < 0 when idle
    // per request: launch time, slot, batch number, finish time
    double* launch_t;
    int32_t* slot_of;
    int32_t* batch_of;
    double* done_t;
    int32_t batches = 0;
    int32_t violations = 0;              // launch on a busy slot

    double now() override { return t; }
    bool launch(int slot, const std::vector<uint32_t>& reqs) override {
        if (finish[slot] >= 0) violations++;
        uint64_t bytes = 0;
        for (uint32_t r : reqs) bytes += cost[r];
        finish[slot] = t + base + per_byte * (double)bytes;
        for (uint32_t r : reqs) {
            launch_t[r] = t;
            slot_of[r] = slot;
            batch_of[r] = batches;
            done_t[r] = finish[slot];
        }
        batches++;
        return true;
    }
    bool done(int slot) override {
        if (finish[slot] < 0 || t < finish[slot]) return false;
        finish[slot] = -1;
        return true;
    }
    void idle(double until) override {
        double next = until;
        for (double f : finish)
            if (f >= 0) next = std::min(next, f);
        t = std::max(t, next);
    }
};

}  // namespace

extern "C" int sim_run(uint32_t n, const double* arrival, const uint64_t* cost,
                       const uint8_t* valid, uint64_t budget, uint32_t max_batch,
                       uint32_t slots, double base, double per_byte,
                       double* latency, int8_t* outcome, double* launch_t,
                       int32_t* slot_of, int32_t* batch_of, double* done_t,
                       uint64_t* stats /* launches, rejected, max_queue,
                                          max_inflight, max_bytes */) {
    std::vector<serve::Request> rq(n);
    for (uint32_t i = 0; i < n; i++) {
        rq[i].arrival = arrival[i];
        rq[i].cost = cost[i];
        rq[i].valid = valid[i] != 0;
        launch_t[i] = -1;
        slot_of[i] = -1;
        batch_of[i] = -1;
        done_t[i] = -1;
    }
    SimExecutor ex;
    ex.base = base;
    ex.per_byte = per_byte;
    ex.cost = cost;
    ex.finish.assign(slots, -1.0);
    ex.launch_t = launch_t;
    ex.slot_of = slot_of;
    ex.batch_of = batch_of;
    ex.done_t = done_t;
    const serve::Config cfg{budget, max_batch, slots};
    const serve::Result R = serve::run(cfg, rq, ex);
    for (uint32_t i = 0; i < n; i++) {
        latency[i] = R.latency[i];
        outcome[i] = R.outcome[i];
    }
    stats[0] = R.launches;
    stats[1] = R.rejected;
    stats[2] = R.max_queue;
    stats[3] = R.max_inflight;
    stats[4] = R.max_bytes;
    return R.error ? -1 : ex.violations;
}

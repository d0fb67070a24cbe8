// Continuous-batching scheduler for chunking requests (host side, no HIP).
//
// Requests arrive open-loop at scheduled times.  They wait in a FIFO until
// they are admitted: a request is admitted when a batch slot (a stream) is
// free and the bytes it holds on the device fit what is left of the
// device-memory budget.  Every free slot takes the longest FIFO prefix that
// fits (at most max_batch requests) as one batched launch, so requests that
// arrive while others run join the next launch and run concurrently with
// them.  A request's latency is its completion time (the moment the poller
// sees its batch finished) minus its scheduled arrival, so queueing delay is
// included.
//
// The device side is an Executor: the library's runs HIP streams, the tests
// a simulated clock.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <vector>

namespace serve {

struct Request {
    double arrival;     // scheduled arrival (seconds from the start)
    uint64_t cost;      // device bytes held while in flight
    bool valid;         // false: rejected at arrival
};

class Executor {
public:
    virtual ~Executor() = default;
    virtual double now() = 0;                       // seconds from the start
    // Enqueue the requests (indices) as one batch on slot; false on error.
    virtual bool launch(int slot, const std::vector<uint32_t>& reqs) = 0;
    // True once the batch on slot has completed (or failed).
    virtual bool done(int slot) = 0;
    // Nothing to do before `until`: wait until then or until a running
    // batch completes, whichever is first.
    virtual void idle(double until) = 0;
};

struct Config {
    uint64_t budget;     // device bytes in flight
    uint32_t max_batch;  // requests per launch
    uint32_t slots;      // concurrent batches
};

enum Outcome : int8_t { kPending = 0, kDone = 1, kRejectedInvalid = 2,
                        kRejectedBudget = 3 };

struct Result {
    std::vector<double> latency;    // per request (-1: rejected)
    std::vector<int8_t> outcome;    // Outcome per request
    uint64_t launches = 0;
    uint64_t rejected = 0;
    uint32_t max_queue = 0;         // longest FIFO seen
    uint32_t max_inflight = 0;      // most batches running at once
    uint64_t max_bytes = 0;         // most budget bytes in flight at once
    double last_finish = 0;
    bool error = false;             // a launch failed
};

inline Result run(const Config& cfg, const std::vector<Request>& reqs,
                  Executor& ex) {
    Result R;
    const size_t n = reqs.size();
    R.latency.assign(n, -1.0);
    R.outcome.assign(n, kPending);
    std::deque<uint32_t> fifo;
    std::vector<std::vector<uint32_t>> running(cfg.slots);
    std::vector<uint64_t> slot_cost(cfg.slots, 0);
    uint64_t in_flight = 0;
    size_t next = 0, finished = 0;
    uint32_t busy = 0;
    while (finished < n) {
        const double t = ex.now();
        // arrivals
        while (next < n && reqs[next].arrival <= t) {
            if (!reqs[next].valid || reqs[next].cost > cfg.budget) {
                R.outcome[next] = reqs[next].valid ? kRejectedBudget
                                                   : kRejectedInvalid;
                R.rejected++;
                finished++;
            } else {
                fifo.push_back((uint32_t)next);
            }
            next++;
        }
        R.max_queue = std::max(R.max_queue, (uint32_t)fifo.size());
        // completions
        for (uint32_t s = 0; s < cfg.slots; s++) {
            if (running[s].empty() || !ex.done(s)) continue;
            const double tc = ex.now();
            for (uint32_t r : running[s]) {
                R.latency[r] = tc - reqs[r].arrival;
                R.outcome[r] = kDone;
            }
            R.last_finish = std::max(R.last_finish, tc);
            finished += running[s].size();
            in_flight -= slot_cost[s];
            slot_cost[s] = 0;
            running[s].clear();
            busy--;
        }
        // admission into free slots
        bool launched = false;
        for (uint32_t s = 0; s < cfg.slots && !fifo.empty(); s++) {
            if (!running[s].empty()) continue;
            std::vector<uint32_t> batch;
            uint64_t cost = 0;
            while (!fifo.empty() && batch.size() < cfg.max_batch &&
                   in_flight + cost + reqs[fifo.front()].cost <= cfg.budget) {
                cost += reqs[fifo.front()].cost;
                batch.push_back(fifo.front());
                fifo.pop_front();
            }
            if (batch.empty()) break;   // the FIFO head waits for memory
            if (!ex.launch((int)s, batch)) {
                R.error = true;
                return R;
            }
            R.launches++;
            running[s] = std::move(batch);
            slot_cost[s] = cost;
            in_flight += cost;
            busy++;
            R.max_inflight = std::max(R.max_inflight, busy);
            R.max_bytes = std::max(R.max_bytes, in_flight);
            launched = true;
        }
        if (launched || finished == n) continue;
        // wait for the next arrival or a completion
        const double until = next < n ? reqs[next].arrival : t + 1.0;
        ex.idle(until);
    }
    return R;
}

}  // namespace serve

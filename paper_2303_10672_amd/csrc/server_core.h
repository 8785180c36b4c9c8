// Scheduling core of the request server: tickets, the two request queues,
// admission of large requests by device memory, completion and latency records.
//
// The core knows nothing of HIP.  Worker threads that the server owns call
// next_large / next_small to take work and complete() to hand results back; the
// device memory figure comes from a callback, so the core can be driven on the CPU
// by a fake executor (tests build it with g++ alone).
//
// Admission of a large request: its bytes must fit the budget beside the bytes of
// the large requests running, and (unless its device state already exists) the
// free device memory reported by the callback must exceed its bytes plus a margin.
// Free memory can change without any call into the core (a client frees a handle,
// another library allocates), so a waiting worker re-reads it at least every
// recheck interval instead of relying on a notification alone.
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

namespace pvi {
namespace srv {

using clk = std::chrono::steady_clock;

enum JobState { kQueued = 0, kRunning = 1, kDone = 2 };

// One request as the core sees it.  Executors derive their own request type from it.
struct Job {
    virtual ~Job() = default;
    uint64_t ticket = 0;
    bool small = false;
    int64_t bytes = 0;        // device bytes a large request holds while it runs
    bool resident = false;    // large: its device state exists already
    int state = kQueued;
    int status = 0;           // pvi_status once done
    int worker = -1;          // worker that ran it
    std::atomic<int> launch{0};  // small: number of the slot-kernel launch serving it
    clk::time_point t_submit, t_start, t_done;
};

struct Config {
    int64_t budget = 0;          // device bytes large requests may hold together
    int64_t margin = 64 << 20;   // free memory kept beyond a request's bytes
    int recheck_us = 2000;       // longest wait between re-reads of free memory
    const char* log_path = nullptr;  // event log (one line per submit/start/done)
};

class Core {
  public:
    using FreeBytes = std::function<int64_t()>;
    explicit Core(const Config& cfg);
    ~Core();

    // ---- client side
    // Takes ownership of the jobs; writes their tickets.  False once shutting down.
    bool submit(std::vector<std::unique_ptr<Job>>& jobs, uint64_t* tickets);
    // 1: done (job returned), 0: still queued or running after timeout_us
    // (< 0: wait without limit), -1: unknown ticket.
    int wait(uint64_t ticket, int64_t timeout_us, Job** out);
    int poll(uint64_t ticket, Job** out);
    // Marks the core as stopping, completes every queued job with `cancel_status`,
    // and wakes every waiter; running jobs finish normally.
    void shutdown(int cancel_status);
    bool stopping();
    // Latency (ms, submit to done) quantiles and count over completed jobs.
    void stats(double* p50, double* p99, int64_t* completed);

    // ---- worker side
    // Blocks until the front large request is admitted (returned, state running,
    // its bytes counted), one that can never fit the budget is found (completed
    // with `busy_status`, and the wait goes on), or the core stops (nullptr).
    Job* next_large(int worker, const FreeBytes& free_bytes, int busy_status);
    // Takes up to max_jobs queued small requests (state running).  Waits for the
    // first one up to wait_us (< 0: until one arrives or the core stops).  Returns
    // the number taken; 0 with stopping() true means the core has stopped.
    int next_small(int worker, int max_jobs, int64_t wait_us, std::vector<Job*>& out);
    // Number of small requests waiting.
    size_t small_waiting();
    // Records the job's status and completion, returns its bytes to the budget and
    // wakes its waiters and the workers.
    void complete(Job* j, int status);

    int64_t bytes_in_use();
    // Calls f on the ticket's job under the core's lock (for status reports);
    // false for an unknown ticket.
    bool visit(uint64_t ticket, const std::function<void(const Job&)>& f);
    // Milliseconds from the core's creation to t.
    double ms_since_start(clk::time_point t) const;

  private:
    void log_event(const char* what, const Job* j);

    Config cfg_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Job*> small_q_, large_q_;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs_;
    std::vector<double> latency_ms_;
    uint64_t next_ticket_ = 1;
    int64_t used_ = 0;
    bool stop_ = false;
    clk::time_point t0_;
    std::FILE* log_ = nullptr;
};

}  // namespace srv
}  // namespace pvi

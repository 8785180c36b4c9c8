// CPU driver of the request server's scheduling core with a fake executor: worker
// threads that sleep instead of solving, and a free-memory figure the test changes
// behind the core's back.  Built with a host C++ compiler (no HIP) by
// tests/test_server_core.py, under ThreadSanitizer where the toolchain has it;
// prints one PASS/FAIL line per scenario.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "server_core.h"

using namespace pvi::srv;
using ms = std::chrono::milliseconds;

namespace {

constexpr int kOk = 0, kBusy = 7, kCancelled = 6;
int failures = 0;

void report(bool ok, const char* name, const std::string& detail) {
    std::printf("%s %s %s\n", ok ? "PASS" : "FAIL", name, detail.c_str());
    std::fflush(stdout);
    if (!ok) ++failures;
}

struct FakeJob : Job {
    int run_ms = 0;
};

std::unique_ptr<Job> make_job(bool small, int64_t bytes, int run_ms, bool resident = false) {
    auto j = std::make_unique<FakeJob>();
    j->small = small;
    j->bytes = bytes;
    j->run_ms = run_ms;
    j->resident = resident;
    return j;
}

uint64_t submit_one(Core& c, std::unique_ptr<Job> j) {
    std::vector<std::unique_ptr<Job>> v;
    v.push_back(std::move(j));
    uint64_t t = 0;
    if (!c.submit(v, &t)) return 0;
    return t;
}

// Large worker: runs what the core admits, tracking how many run at once.
struct LargeWorkers {
    Core& core;
    std::atomic<int64_t>& free_mem;
    std::atomic<int> running{0}, max_running{0};
    std::vector<std::thread> th;
    LargeWorkers(Core& c, std::atomic<int64_t>& f, int n) : core(c), free_mem(f) {
        for (int w = 0; w < n; ++w)
            th.emplace_back([this, w] {
                auto fb = [this] { return free_mem.load(); };
                for (;;) {
                    Job* j = core.next_large(w, fb, kBusy);
                    if (!j) return;
                    const int now = ++running;
                    int prev = max_running.load();
                    while (now > prev && !max_running.compare_exchange_weak(prev, now)) {
                    }
                    std::this_thread::sleep_for(ms(static_cast<FakeJob*>(j)->run_ms));
                    --running;
                    core.complete(j, kOk);
                }
            });
    }
    void join() {
        for (auto& t : th) t.join();
    }
};

struct SmallWorkers {
    Core& core;
    std::atomic<int> batches{0}, max_batch{0};
    std::vector<std::thread> th;
    SmallWorkers(Core& c, int n, int max_jobs) : core(c) {
        for (int w = 0; w < n; ++w)
            th.emplace_back([this, w, max_jobs] {
                std::vector<Job*> out;
                for (;;) {
                    const int k = core.next_small(100 + w, max_jobs, -1, out);
                    if (k == 0) {
                        if (core.stopping()) return;
                        continue;
                    }
                    ++batches;
                    int prev = max_batch.load();
                    while (k > prev && !max_batch.compare_exchange_weak(prev, k)) {
                    }
                    int longest = 0;
                    for (Job* j : out) longest = std::max(longest, static_cast<FakeJob*>(j)->run_ms);
                    std::this_thread::sleep_for(ms(longest));
                    for (Job* j : out) core.complete(j, kOk);
                }
            });
    }
    void join() {
        for (auto& t : th) t.join();
    }
};

// Free memory appears without any call into the core: the waiting request must
// still be admitted (the bounded re-check), well within a second.
void lost_wakeup() {
    Config cfg;
    cfg.budget = 1000;
    cfg.margin = 0;
    cfg.recheck_us = 2000;
    Core c(cfg);
    std::atomic<int64_t> free_mem{0};
    LargeWorkers lw(c, free_mem, 1);
    const uint64_t t = submit_one(c, make_job(false, 100, 1));
    std::this_thread::sleep_for(ms(50));
    const bool queued = c.poll(t, nullptr) == 0;
    const auto t0 = clk::now();
    free_mem.store(1000);  // no notification
    Job* j = nullptr;
    const int r = c.wait(t, 1000000, &j);
    const double dt = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    report(queued && r == 1 && j && j->status == kOk && dt < 500.0, "lost_wakeup",
           "queued_before=" + std::to_string(queued) + " admitted_after_ms=" + std::to_string(dt));
    c.shutdown(kCancelled);
    lw.join();
}

// The same with the re-check interval made longer than the test: free memory that
// appears without a notification leaves the request queued (the lost wakeup a
// notification-only wait would have), until another event wakes the worker.
void lost_wakeup_without_recheck() {
    Config cfg;
    cfg.budget = 1000;
    cfg.margin = 0;
    cfg.recheck_us = 600 * 1000 * 1000;
    Core c(cfg);
    std::atomic<int64_t> free_mem{0};
    LargeWorkers lw(c, free_mem, 1);
    const uint64_t t = submit_one(c, make_job(false, 100, 1));
    std::this_thread::sleep_for(ms(20));
    free_mem.store(1000);  // no notification
    const int r0 = c.wait(t, 200000, nullptr);
    submit_one(c, make_job(false, 10, 1));  // any event: the worker looks again
    const int r1 = c.wait(t, 1000000, nullptr);
    report(r0 == 0 && r1 == 1, "lost_wakeup_without_recheck",
           "unannounced=" + std::to_string(r0) + " after_event=" + std::to_string(r1));
    c.shutdown(kCancelled);
    lw.join();
}

// A request larger than the budget completes at once with the busy status, and the
// worker goes on to the next one.
void busy() {
    Config cfg;
    cfg.budget = 1000;
    Core c(cfg);
    std::atomic<int64_t> free_mem{int64_t(1) << 40};
    LargeWorkers lw(c, free_mem, 1);
    const uint64_t t1 = submit_one(c, make_job(false, 2000, 1));
    const uint64_t t2 = submit_one(c, make_job(false, 10, 1, true));
    Job *j1 = nullptr, *j2 = nullptr;
    const int r1 = c.wait(t1, 1000000, &j1), r2 = c.wait(t2, 1000000, &j2);
    report(r1 == 1 && j1->status == kBusy && r2 == 1 && j2->status == kOk, "busy",
           "status=" + std::to_string(r1 == 1 ? j1->status : -1));
    c.shutdown(kCancelled);
    lw.join();
}

// Two workers, a budget that holds one request at a time: they never overlap.
// With room for both, they do.
void budget() {
    for (int roomy = 0; roomy < 2; ++roomy) {
        Config cfg;
        cfg.budget = roomy ? 1000 : 150;
        Core c(cfg);
        std::atomic<int64_t> free_mem{int64_t(1) << 40};
        LargeWorkers lw(c, free_mem, 2);
        std::vector<uint64_t> ts;
        for (int i = 0; i < 4; ++i) ts.push_back(submit_one(c, make_job(false, 100, 40)));
        bool all = true;
        for (uint64_t t : ts) {
            Job* j = nullptr;
            all = all && c.wait(t, 2000000, &j) == 1 && j->status == kOk;
        }
        const int mx = lw.max_running.load();
        const bool ok = all && (roomy ? mx == 2 : mx == 1) && c.bytes_in_use() == 0;
        report(ok, roomy ? "budget_overlap" : "budget_serialises",
               "max_running=" + std::to_string(mx));
        c.shutdown(kCancelled);
        lw.join();
    }
}

// Small requests are taken in batches of at most max_jobs.
void small_batches() {
    Config cfg;
    cfg.budget = 1000;
    Core c(cfg);
    SmallWorkers sw(c, 1, 8);
    std::vector<std::unique_ptr<Job>> v;
    for (int i = 0; i < 50; ++i) v.push_back(make_job(true, 0, 2));
    std::vector<uint64_t> ts(50);
    c.submit(v, ts.data());
    bool all = true;
    for (uint64_t t : ts) {
        Job* j = nullptr;
        all = all && c.wait(t, 2000000, &j) == 1 && j->status == kOk;
    }
    const int nb = sw.batches.load(), mb = sw.max_batch.load();
    report(all && mb <= 8 && nb >= 7, "small_batches",
           "batches=" + std::to_string(nb) + " largest=" + std::to_string(mb));
    c.shutdown(kCancelled);
    sw.join();
}

// Shutdown completes queued requests as cancelled; later submits are refused.
void cancel() {
    Config cfg;
    cfg.budget = 1000;
    Core c(cfg);
    std::vector<std::unique_ptr<Job>> v;
    v.push_back(make_job(false, 10, 1));
    v.push_back(make_job(true, 0, 1));
    uint64_t ts[2];
    c.submit(v, ts);
    c.shutdown(kCancelled);
    Job *a = nullptr, *b = nullptr;
    const bool done = c.wait(ts[0], 0, &a) == 1 && c.wait(ts[1], 0, &b) == 1;
    std::atomic<int64_t> free_mem{1};
    Job* none = c.next_large(0, [&] { return free_mem.load(); }, kBusy);
    const uint64_t late = submit_one(c, make_job(true, 0, 1));
    report(done && a->status == kCancelled && b->status == kCancelled && none == nullptr &&
               late == 0 && c.wait(12345, 0, nullptr) == -1,
           "cancel", "");
}

// A bounded wait on a running request returns not-ready, then ready.
void wait_timeout() {
    Config cfg;
    cfg.budget = 1000;
    Core c(cfg);
    std::atomic<int64_t> free_mem{int64_t(1) << 40};
    LargeWorkers lw(c, free_mem, 1);
    const uint64_t t = submit_one(c, make_job(false, 10, 200));
    const int r0 = c.wait(t, 10000, nullptr);
    int state = -1;
    c.visit(t, [&](const Job& j) { state = j.state; });
    const int r1 = c.wait(t, 2000000, nullptr);
    report(r0 == 0 && r1 == 1 && state >= kQueued && state <= kRunning, "wait_timeout",
           "first=" + std::to_string(r0) + " second=" + std::to_string(r1));
    c.shutdown(kCancelled);
    lw.join();
}

// Many requests of both kinds from two client threads while free memory swings
// below and above what the requests need (never announced to the core): every
// request completes, the budget is returned, and the latency count matches.
void stress() {
    Config cfg;
    cfg.budget = 500;
    cfg.margin = 0;
    cfg.recheck_us = 500;
    Core c(cfg);
    std::atomic<int64_t> free_mem{1000};
    std::atomic<bool> run{true};
    std::thread swing([&] {
        std::mt19937 g(1);
        while (run.load()) {
            free_mem.store(g() % 2 ? 50 : 1000);
            std::this_thread::sleep_for(std::chrono::microseconds(300 + g() % 700));
        }
    });
    LargeWorkers lw(c, free_mem, 2);
    SmallWorkers sw(c, 2, 16);
    const int per_client = 1000;
    std::vector<uint64_t> ts(2 * per_client);
    std::vector<std::thread> clients;
    for (int k = 0; k < 2; ++k)
        clients.emplace_back([&, k] {
            std::mt19937 g(10 + k);
            for (int i = 0; i < per_client; ++i) {
                const bool small = g() % 10 < 7;
                ts[k * per_client + i] =
                    submit_one(c, make_job(small, small ? 0 : 50 + g() % 200, g() % 2));
                if (g() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
            }
        });
    for (auto& t : clients) t.join();
    bool all = true;
    for (uint64_t t : ts) {
        Job* j = nullptr;
        all = all && t != 0 && c.wait(t, 20000000, &j) == 1 && j->status == kOk;
    }
    run.store(false);
    swing.join();
    int64_t n = 0;
    c.stats(nullptr, nullptr, &n);
    report(all && n == 2 * per_client && c.bytes_in_use() == 0, "stress",
           "completed=" + std::to_string(n));
    c.shutdown(kCancelled);
    lw.join();
    sw.join();
}

}  // namespace

int main() {
    lost_wakeup();
    lost_wakeup_without_recheck();
    busy();
    budget();
    small_batches();
    cancel();
    wait_timeout();
    stress();
    return failures ? 1 : 0;
}

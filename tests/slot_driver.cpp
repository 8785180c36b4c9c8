// CPU driver of the slot feeder (continuous refill of the small-instance kernel) with
// a fake device: each launch is one thread per slot running the device side of the
// slot protocol (poll the slot's request number, the stop word and the heartbeat;
// "solve" by sleeping; write the result; publish the number as done).  Built with a
// host C++ compiler (no HIP) by tests/test_server_core.py, under ThreadSanitizer where
// the toolchain has it; prints one PASS/FAIL line per scenario.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "server_core.h"
#include "slots.h"

using namespace pvi;
using namespace pvi::srv;
using ms = std::chrono::milliseconds;

namespace {

constexpr int kOk = 0, kCancelled = 6, kDeviceError = 3;
int failures = 0;

void report(bool ok, const char* name, const std::string& detail) {
    std::printf("%s %s %s\n", ok ? "PASS" : "FAIL", name, detail.c_str());
    std::fflush(stdout);
    if (!ok) ++failures;
}

struct FakeJob : Job {
    int run_ms = 0;
    int input = 0;
    int output = -1;
    clk::time_point served_from, served_to;
};

// One slot's request as the fake device sees it (written by prepare before the slot's
// number moves, read by the device after it sees the number).
struct SlotData {
    int input = 0, run_ms = 0;
    int output = 0;
    clk::time_point from, to;
};

uint32_t ld(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
void st(uint32_t* p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }

struct FakeDevice : SlotOps {
    int nslots;
    SlotHeader hdr{};
    std::vector<SlotSync> sync;
    std::vector<SlotData> data;
    std::vector<std::thread> groups;
    std::atomic<int> alive{0};
    int idle_polls = 1000000;     // polls without a heartbeat change before a group returns
    int serve_limit = -1;         // > 0: each launch serves this many requests, then ends
    bool fail_launch = false;
    std::atomic<int> served_in_launch{0};

    explicit FakeDevice(int n) : nslots(n), sync(n), data(n) {}
    ~FakeDevice() override { wait(); }

    void prepare(int k, Job* j) override {
        auto* f = static_cast<FakeJob*>(j);
        data[k].input = f->input;
        data[k].run_ms = f->run_ms;
    }
    int collect(int k, Job* j) override {
        auto* f = static_cast<FakeJob*>(j);
        f->output = data[k].output;
        f->served_from = data[k].from;
        f->served_to = data[k].to;
        return kOk;
    }
    bool launch() override {
        if (fail_launch) return false;
        wait();
        served_in_launch = 0;
        alive = nslots;
        for (int k = 0; k < nslots; ++k) groups.emplace_back([this, k] { group(k); });
        return true;
    }
    bool finished() override { return alive.load() == 0; }
    void wait() override {
        for (auto& t : groups) t.join();
        groups.clear();
    }
    // the device side of the protocol, as slot_kernel runs it
    void group(int k) {
        uint32_t last = ld(&sync[k].done);
        for (;;) {
            uint32_t hb_seen = ld(&hdr.heartbeat), s = last;
            int still = 0;
            bool ex = false;
            for (;;) {
                // a request already in the slot is served even when the stop word is set
                s = ld(&sync[k].seq);
                if (s != last) break;
                if (ld(&hdr.stop)) {
                    ex = true;
                    break;
                }
                const uint32_t hb = ld(&hdr.heartbeat);
                if (hb != hb_seen) {
                    hb_seen = hb;
                    still = 0;
                } else if (++still > idle_polls) {
                    ex = true;
                    break;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
            if (ex) break;
            data[k].from = clk::now();
            std::this_thread::sleep_for(ms(data[k].run_ms));
            data[k].output = 2 * data[k].input + 1;
            data[k].to = clk::now();
            st(&sync[k].done, s);
            last = s;
            if (serve_limit > 0 && ++served_in_launch >= serve_limit) break;
        }
        --alive;
    }
};

std::unique_ptr<Job> job(int input, int run_ms) {
    auto j = std::make_unique<FakeJob>();
    j->small = true;
    j->input = input;
    j->run_ms = run_ms;
    return j;
}

uint64_t submit(Core& c, int input, int run_ms) {
    std::vector<std::unique_ptr<Job>> v;
    v.push_back(job(input, run_ms));
    uint64_t t = 0;
    c.submit(v, &t);
    return t;
}

struct Rig {
    Config cc;
    std::unique_ptr<Core> core;
    std::unique_ptr<FakeDevice> dev;
    std::unique_ptr<SlotFeeder> feeder;
    std::thread th;
    Rig(int nslots, int idle_ms, FakeDevice* d = nullptr) {
        cc.budget = 1 << 20;
        core = std::make_unique<Core>(cc);
        dev.reset(d ? d : new FakeDevice(nslots));
        SlotConfig sc;
        sc.nslots = nslots;
        sc.idle_ms = idle_ms;
        sc.launch_error_status = kDeviceError;
        feeder = std::make_unique<SlotFeeder>(*core, *dev, &dev->hdr, dev->sync.data(), sc);
        th = std::thread([this] { feeder->run(); });
    }
    FakeJob* get(uint64_t t, int64_t timeout_us = 5000000) {
        Job* j = nullptr;
        return core->wait(t, timeout_us, &j) == 1 ? static_cast<FakeJob*>(j) : nullptr;
    }
    void stop() {
        core->shutdown(kCancelled);
        th.join();
    }
};

// Requests arriving over time while others run are served by the same launch.
void refill() {
    Rig r(4, 500);
    std::vector<uint64_t> ts;
    for (int i = 0; i < 20; ++i) {
        ts.push_back(submit(*r.core, i, 5));
        std::this_thread::sleep_for(ms(2));
    }
    bool ok = true;
    int same = 0;
    for (int i = 0; i < 20; ++i) {
        FakeJob* j = r.get(ts[i]);
        ok = ok && j && j->status == kOk && j->output == 2 * i + 1;
        same += j && j->launch == 1;
    }
    const int n = r.feeder->launches();
    r.stop();
    report(ok && n == 1 && same == 20, "slot_refill",
           "launches=" + std::to_string(n) + " served_by_first=" + std::to_string(same));
}

// A request submitted while another runs in the same launch finishes first if shorter.
void mid_launch() {
    Rig r(4, 500);
    const uint64_t ta = submit(*r.core, 1, 120);
    std::this_thread::sleep_for(ms(20));
    const uint64_t tb = submit(*r.core, 2, 5);
    FakeJob* b = r.get(tb);
    FakeJob* a = r.get(ta);
    const bool ok = a && b && a->output == 3 && b->output == 5 && b->launch == a->launch &&
                    b->served_to < a->served_to && b->served_from > a->served_from;
    r.stop();
    report(ok, "slot_mid_launch", std::string("same_launch=") + (a && b && a->launch == b->launch ? "1" : "0"));
}

// After idle_ms without work the launch is stopped; the next request starts a new one.
void idle_relaunch() {
    Rig r(2, 30);
    FakeJob* a = r.get(submit(*r.core, 1, 2));
    std::this_thread::sleep_for(ms(150));
    const bool stopped = r.dev->finished();
    FakeJob* b = r.get(submit(*r.core, 2, 2));
    const int n = r.feeder->launches();
    r.stop();
    report(a && b && stopped && n == 2 && a->launch == 1 && b->launch == 2, "slot_idle_relaunch",
           "launches=" + std::to_string(n) + " stopped_while_idle=" + std::to_string(stopped));
}

// A launch that ends on its own (its groups return once it has served 3 requests, so
// at most 4 here) is replaced, and every
// request is still served once.
void ends_on_its_own() {
    auto* d = new FakeDevice(2);
    d->serve_limit = 3;
    Rig r(2, 500, d);
    std::vector<uint64_t> ts;
    for (int i = 0; i < 12; ++i) ts.push_back(submit(*r.core, i, 1));
    bool ok = true;
    for (int i = 0; i < 12; ++i) {
        FakeJob* j = r.get(ts[i]);
        ok = ok && j && j->status == kOk && j->output == 2 * i + 1;
    }
    const int n = r.feeder->launches();
    r.stop();
    report(ok && n >= 3, "slot_launch_ends_on_its_own", "launches=" + std::to_string(n));
}

// A launch that cannot start completes the requests in its slots with the error status.
void launch_fails() {
    auto* d = new FakeDevice(2);
    d->fail_launch = true;
    Rig r(2, 500, d);
    FakeJob* a = r.get(submit(*r.core, 1, 1));
    FakeJob* b = r.get(submit(*r.core, 2, 1));
    r.stop();
    report(a && b && a->status == kDeviceError && b->status == kDeviceError, "slot_launch_fails",
           "");
}

// Shutdown: running requests finish, queued ones are cancelled, the launch is stopped.
void shutdown_busy() {
    Rig r(2, 500);
    std::vector<uint64_t> ts;
    for (int i = 0; i < 6; ++i) ts.push_back(submit(*r.core, i, 40));
    std::this_thread::sleep_for(ms(10));
    r.stop();
    int ok_n = 0, cancelled = 0;
    for (uint64_t t : ts) {
        FakeJob* j = r.get(t, 0);
        if (j && j->status == kOk && j->output >= 1) ++ok_n;
        if (j && j->status == kCancelled) ++cancelled;
    }
    report(ok_n == 2 && cancelled == 4 && r.dev->finished(), "slot_shutdown",
           "served=" + std::to_string(ok_n) + " cancelled=" + std::to_string(cancelled));
}

// Many requests from two clients through 8 slots: every one served once, right result.
void stress() {
    Rig r(8, 200);
    const int per = 300;
    std::vector<uint64_t> ts(2 * per);
    std::vector<std::thread> cl;
    for (int c = 0; c < 2; ++c)
        cl.emplace_back([&, c] {
            for (int i = 0; i < per; ++i) {
                ts[c * per + i] = submit(*r.core, c * per + i, i % 3);
                if (i % 16 == 0) std::this_thread::sleep_for(std::chrono::microseconds(300));
            }
        });
    for (auto& t : cl) t.join();
    bool ok = true;
    for (int i = 0; i < 2 * per; ++i) {
        FakeJob* j = r.get(ts[i], 20000000);
        ok = ok && j && j->status == kOk && j->output == 2 * i + 1;
    }
    r.stop();
    report(ok, "slot_stress", "requests=" + std::to_string(2 * per));
}

}  // namespace

int main() {
    refill();
    mid_launch();
    idle_relaunch();
    ends_on_its_own();
    launch_fails();
    shutdown_busy();
    stress();
    return failures ? 1 : 0;
}

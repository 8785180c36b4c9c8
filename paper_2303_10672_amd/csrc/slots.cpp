// Slot feeder (see slots.h).  Plain C++17: no HIP.
#include "slots.h"

#include <algorithm>
#include <chrono>
#include <thread>

namespace pvi {
namespace srv {

namespace {
uint32_t load_acquire(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
void store_release(uint32_t* p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
}  // namespace

SlotFeeder::SlotFeeder(Core& core, SlotOps& ops, SlotHeader* hdr, SlotSync* sync,
                       const SlotConfig& cfg)
    : core_(core), ops_(ops), hdr_(hdr), sync_(sync), cfg_(cfg),
      busy_(cfg.nslots, nullptr), seq_(cfg.nslots, 0) {
    for (int k = 0; k < cfg_.nslots; ++k) seq_[k] = load_acquire(&sync_[k].seq);
    heartbeat_ = load_acquire(&hdr_->heartbeat);
    idle_since_ = clk::now();
}

void SlotFeeder::collect_done() {
    for (int k = 0; k < cfg_.nslots; ++k) {
        Job* j = busy_[k];
        if (!j || load_acquire(&sync_[k].done) != seq_[k]) continue;
        const int st = ops_.collect(k, j);
        busy_[k] = nullptr;
        --nbusy_;
        core_.complete(j, st);
    }
}

bool SlotFeeder::ensure_running() {
    if (running_ && !ops_.finished()) return true;
    if (running_) {
        // the launch ended on its own (its work groups saw no heartbeat for their idle
        // cap): what it finished is collected first, the rest goes to a new launch
        running_ = false;
        collect_done();
        if (nbusy_ == 0) return true;
    }
    store_release(&hdr_->stop, 0);
    if (!ops_.launch()) return false;
    running_ = true;
    const int id = ++launches_;
    for (Job* j : busy_)
        if (j) j->launch = id;
    return true;
}

void SlotFeeder::run() {
    std::vector<Job*> jobs;
    for (;;) {
        collect_done();
        const int nfree = cfg_.nslots - nbusy_;
        // with busy slots only look; with a launch idling, wait a little (the heartbeat
        // goes on meanwhile); with nothing running, wait for the next request
        const int64_t wait_us =
            nbusy_ > 0 ? 0 : running_ ? std::min<int64_t>(1000, 500 * (int64_t)cfg_.idle_ms) : -1;
        const int got = nfree > 0 ? core_.next_small(cfg_.worker, nfree, wait_us, jobs) : 0;
        if (got == 0 && nbusy_ == 0 && core_.stopping()) break;
        for (Job* j : jobs) {
            int k = 0;
            while (busy_[k]) ++k;  // a free slot exists: got <= nfree
            ops_.prepare(k, j);
            j->launch = running_ ? launches_.load() : launches_.load() + 1;
            seq_[k] += 1;
            if (seq_[k] == 0) seq_[k] = 1;  // 0 means no request yet
            store_release(&sync_[k].seq, seq_[k]);
            busy_[k] = j;
            ++nbusy_;
        }
        jobs.clear();
        if (nbusy_ > 0) {
            if (!ensure_running()) {
                // the requests in the slots cannot be served: complete them as failed
                for (int k = 0; k < cfg_.nslots; ++k)
                    if (busy_[k]) {
                        Job* j = busy_[k];
                        busy_[k] = nullptr;
                        store_release(&sync_[k].done, seq_[k]);
                        core_.complete(j, cfg_.launch_error_status);
                    }
                nbusy_ = 0;
            }
            idle_since_ = clk::now();
        }
        store_release(&hdr_->heartbeat, ++heartbeat_);
        if (nbusy_ == 0 && running_ &&
            clk::now() - idle_since_ > std::chrono::milliseconds(cfg_.idle_ms)) {
            store_release(&hdr_->stop, 1);
            ops_.wait();
            running_ = false;
        }
        if (nbusy_ > 0) std::this_thread::sleep_for(std::chrono::microseconds(cfg_.poll_us));
    }
    if (running_) {
        store_release(&hdr_->stop, 1);
        ops_.wait();
        running_ = false;
    }
}

}  // namespace srv
}  // namespace pvi

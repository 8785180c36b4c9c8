// Host side of the slot kernel: feeds small requests into the free slots of a
// running kernel launch and collects their results (continuous refill).
//
// One feeder thread owns the slot table.  Each loop it
//  1. collects the slots whose request number the device has published as done,
//     and completes their requests in the scheduling core;
//  2. takes as many queued small requests as there are free slots, writes each into
//     a free slot and then publishes the slot's new request number (release);
//  3. keeps a launch running while any slot is busy: it launches one if none runs,
//     or if the last one ended on its own (its idle cap), and writes a new heartbeat
//     word every loop, which is what keeps the work groups polling;
//  4. asks a launch that has had no busy slot for idle_ms to stop, and waits for it.
// The device side (kernels_batch.hip, slot_kernel) follows the same protocol, so a
// request that arrives while a launch runs is served by that launch.  Plain C++ (no
// HIP): the device operations come through SlotOps, and a CPU test drives the feeder
// with a fake device.
#pragma once

#include <atomic>
#include <cstdint>
#include <vector>

#include "server_core.h"
#include "slot_layout.h"

namespace pvi {
namespace srv {

// What the feeder needs from the device side.
struct SlotOps {
    virtual ~SlotOps() = default;
    // Write the request's inputs and descriptor into slot k (before its number moves).
    virtual void prepare(int k, Job* j) = 0;
    // Read the results of the request the device finished in slot k; returns its status.
    virtual int collect(int k, Job* j) = 0;
    // Start a launch serving every slot; false if it could not be started.
    virtual bool launch() = 0;
    // True once the last launch has ended.
    virtual bool finished() = 0;
    // Wait for the last launch to end.
    virtual void wait() = 0;
};

struct SlotConfig {
    int nslots = 0;
    int idle_ms = 2;     // a launch with no busy slot for this long is stopped: a
                         // resident launch holds registers and LDS that the sweep-loop
                         // kernels of large requests would otherwise use
    int poll_us = 20;    // pause between loops while slots are busy
    int worker = 0;      // worker id given to the core for the requests it takes
    int launch_error_status = 3;  // status of requests whose launch failed
};

class SlotFeeder {
  public:
    SlotFeeder(Core& core, SlotOps& ops, SlotHeader* hdr, SlotSync* sync, const SlotConfig& cfg);
    // Feeds until the core stops and no slot is busy; then stops the launch.
    void run();
    // Launches started so far.
    int launches() const { return launches_.load(); }

  private:
    void collect_done();
    bool ensure_running();

    Core& core_;
    SlotOps& ops_;
    SlotHeader* hdr_;
    SlotSync* sync_;
    SlotConfig cfg_;
    std::vector<Job*> busy_;
    std::vector<uint32_t> seq_;
    int nbusy_ = 0;
    bool running_ = false;
    uint32_t heartbeat_ = 0;
    std::atomic<int> launches_{0};
    clk::time_point idle_since_;
};

}  // namespace srv
}  // namespace pvi

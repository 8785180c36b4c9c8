// Layout of the slot table that the small-instance kernel serves.  It lives in
// coherent pinned host memory: the host writes requests and control words, the
// device writes results and completion numbers, and neither side caches the other's
// writes.  Plain C++ (no HIP), so the host-side slot logic builds without HIP.
#pragma once

#include <cstdint>

namespace pvi {

// Control words of one launch of the slot kernel.
struct alignas(64) SlotHeader {
    uint32_t stop;       // host: 1 = every work group returns at its next look
    uint32_t heartbeat;  // host: changes while the host wants the kernel to stay
    uint32_t pad[14];
};

// Completion protocol of one slot (its own 64-byte line).
struct alignas(64) SlotSync {
    uint32_t seq;   // host: number of the last request placed in the slot (0: none)
    uint32_t done;  // device: number of the last request whose results are written
    uint32_t pad[14];
};

// Polls of a slot's work group without a heartbeat change before it returns: about a
// second of waiting at the longest poll interval, so a kernel whose host stopped
// serving it always ends.
constexpr uint32_t kSlotIdlePolls = 40000;

}  // namespace pvi

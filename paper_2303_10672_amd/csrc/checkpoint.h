// Checkpoint files of a solve (layout in pvi.h, beside checkpoint_read).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

#include "mdp.h"

namespace pvi {

// FNV-1a (Fowler, Noll, Vo) over everything that defines the MDP: sizes, costs,
// discount, issuing, substitution, and the demand and life distributions.
uint64_t mdp_fingerprint(const pvi_mdp* p);

struct Checkpoint {
    int32_t rule = 0, sweeps = 0, stopped = 0;
    // the stopping threshold the writing solve tested (NaN for files of version 1,
    // which do not hold it) and its last increments max/min(V_new - V) and span
    double threshold = 0.0, dmax = 0.0, dmin = 0.0, span = 0.0;
    std::vector<std::vector<double>> tables;  // newest first
};

// What the writing solve knew when it wrote the file.
struct CheckpointStats {
    double threshold = 0.0, dmax = 0.0, dmin = 0.0, span = 0.0;
};

// Read and check a file against the handle; tables are read when want_tables.
pvi_status checkpoint_load(const pvi_mdp* p, const char* path, bool want_tables,
                           Checkpoint& out);

// Copy the device tables (newest first, n_states FP64 each) to the host on stream s
// and write them to path (via path.tmp and a rename).
pvi_status checkpoint_store(const pvi_mdp* p, const char* path, int32_t rule, int32_t sweeps,
                            int32_t stopped, const CheckpointStats& stats,
                            const double* const* tables, int n_tables, hipStream_t s);

}  // namespace pvi

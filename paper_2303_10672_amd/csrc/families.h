// Per-family dispatch of the backup kernels.
#pragma once

#include <string>

#include "mdp.h"

namespace pvi {

bool family_supported(const pvi_mdp* p);
std::string family_support_msg(const pvi_mdp* p);
int family_tiles(const pvi_mdp* p);            // number of span partial slots
size_t family_extra_bytes(const pvi_mdp* p);   // device bytes beyond the common buffers
pvi_status family_init(pvi_mdp* p);            // upload family tables
void family_free(pvi_mdp* p);
// One backup sweep vin -> vout (FP32 centred or FP64 storage), or, with
// extract = 1, the FP64 policy/gap extraction of vin.
// fixed = 1: the sweep belongs to a fixed-length run (no stopping rule).
hipError_t family_backup(pvi_mdp* p, int fp32, int kahan, int extract, int fixed,
                         const void* vin, void* vout, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);  // ev0/ev1: recorded at the backup's start
                                                     // and end (kernel time), when given
// True when the family's backup kernel reduces the span itself (its last
// workgroup applies the stopping rule), so no separate span launch follows it.
bool family_fused_span(const pvi_mdp* p);
// Initial values of a family whose paper-defined V0 is not zero (the lead-time-1
// two-product family: expected one-day revenue), written into v (FP64).
hipError_t family_initial_values(pvi_mdp* p, double* v, hipStream_t s);

}  // namespace pvi

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
hipError_t family_backup(pvi_mdp* p, int fp32, int kahan, int extract, const void* vin,
                         void* vout, hipStream_t s);

}  // namespace pvi

// Host helpers shared by the runtime sources (not part of the C-ABI).
#pragma once

#include <string>

#include "../../include/pixvod.h"
#include "gbp_device.hpp"

namespace pv {

// factor strengths of a parameter set (Lambda = sigma^-2) and the prior mean
Strengths strengths_from(const pixvod_params& P, bool has_sigma_map);
// records the message returned by pixvod_last_error(NULL)
void record_error(const std::string& msg);
// finite, positive strengths and a valid re-anchoring / damping setting
bool params_valid(const pixvod_params* p);

}  // namespace pv

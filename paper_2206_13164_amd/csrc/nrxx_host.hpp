// nrxx_host.hpp -- host-side helpers shared by the single-problem context
// (nrxx_api.cpp) and the batch (nrxx_batch_api.cpp).
#pragma once

#include <string>

#include "../../include/nrxx.h"
#include "nrxx_internal.hpp"

namespace nrxx {

// Checks a problem description; on failure stores the reason in msg.
bool validate_problem(const nrxx_problem &p, std::string &msg);
// Constants of level k (0 = finest) of problem p.
LevelArgs make_level(const nrxx_problem &p, int k);

}  // namespace nrxx

// nrxx_host.hpp -- host-side helpers shared by the single-problem context
// (nrxx_api.cpp) and the batch (nrxx_batch_api.cpp).
#pragma once

#include <stddef.h>

#include <string>

#include "../../include/nrxx.h"
#include "nrxx_internal.hpp"

namespace nrxx {

// Checks a problem description; on failure stores the reason in msg.
bool validate_problem(const nrxx_problem &p, std::string &msg);
// The same check with the reason written into a caller's buffer (no
// allocation).
bool validate_problem(const nrxx_problem &p, char *msg, size_t cap);
// Stores the text nrxx_last_error(NULL) returns (a fixed per-thread
// buffer; no allocation) and returns code.
int set_context_free_error(int code, const char *fmt, ...);
// Constants of level k (0 = finest) of problem p.
LevelArgs make_level(const nrxx_problem &p, int k);

}  // namespace nrxx

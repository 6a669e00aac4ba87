// Measured choice of the block size and tile policy (trsm_autotune): the
// process-wide table that trsm_plan consults when asked to choose n0.
#pragma once

#include <stdint.h>

namespace trsm {

// The recorded (n0, flags) for the size class of (n, k, prec); false if none.
bool tune_lookup(int64_t n, int64_t k, int prec, int64_t* n0, uint32_t* flags);

}  // namespace trsm

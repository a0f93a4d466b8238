// Host helpers shared by the solver, batch and server translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "lbrd.h"
#include "lbrd_internal.h"

namespace lbrd {

void set_error(const char *where, hipError_t e);
int validate_config(const lbrd_config *c);
lbrd_config normalise(const lbrd_config &c);
size_t scratch_bytes();
int default_vec(int storage);
int default_lanes(int nx, int vec);

}  // namespace lbrd

// Entry points of the host runtime (runtime.cpp) used by other translation units of the library (internal).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/resolvent.h"

// resolvent_apply with every workspace buffer taken from the device range [base, base + cap) instead of the
// handle's own allocations: no device memory is allocated or freed.  The range's contents on entry do not matter
// (everything that must start at zero is cleared by kernels on `stream`).  RES_EINVAL, with the byte counts, when
// the run needs more than cap bytes; no kernel has been launched then.
int res_apply_in_scratch(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                         const void* f_hat, void* u_hat, void* base, size_t cap, void* stream);
// Record an error message for resolvent_last_error and return `code`.
int res_fail(int code, const char* msg);

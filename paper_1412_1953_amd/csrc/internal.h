// Library-internal entry points shared between the host drivers (api.cpp)
// and the no-allocation variant (noalloc.hip).  Not part of the C ABI.
#pragma once
#include <stddef.h>

#include "../../include/mgcccs.h"

namespace mgc {
// mgc_cccs with its scratch in a caller-given device buffer of `bytes` bytes.
mgc_status cccs_with_scratch(mgc_grid g, void* u, const void* f, mgc_precision prec, void* scratch, size_t bytes);
// Device the handle was created on.
int handle_device(mgc_grid g);
// Record the message mgc_last_error() returns; returns s.
mgc_status set_error(mgc_status s, const char* msg);
}  // namespace mgc

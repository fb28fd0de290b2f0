// Library-internal declarations shared by the HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

// Record a HIP failure as this host thread's last error (shock_last_error).
__attribute__((visibility("hidden"))) void shock_internal_set_error(const char *what, hipError_t e);

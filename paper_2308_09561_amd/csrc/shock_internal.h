// Library-internal declarations shared by the HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

// Record a HIP failure as this host thread's last error (shock_last_error).
__attribute__((visibility("hidden"))) void shock_internal_set_error(const char *what, hipError_t e);

// Free the calling thread's cached scratch of the Rice encoder, of MPHF
// builds and of the bipartite search on the current device (called by
// shock_release_scratch).
__attribute__((visibility("hidden"))) hipError_t shock_internal_release_code_scratch(int dev);
__attribute__((visibility("hidden"))) hipError_t shock_internal_release_mphf_scratch(int dev);
__attribute__((visibility("hidden"))) hipError_t shock_internal_release_bip_scratch(int dev);

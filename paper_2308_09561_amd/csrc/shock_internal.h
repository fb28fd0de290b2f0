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

struct shock_opts;

// Search scratch bytes of one call of n_leaves leaves (per_leaf: one launch
// per leaf) and the size of its host copy of the call's counters.
__attribute__((visibility("hidden"))) size_t shock_internal_search_bytes(uint64_t n_leaves, int per_leaf);
__attribute__((visibility("hidden"))) size_t shock_internal_counter_bytes(void);

// Options with defaults filled in and checked as the search entry points
// check them (rf: rotation fitting).  SHOCK_OK or SHOCK_EINVAL.
__attribute__((visibility("hidden"))) int shock_internal_complete_opts(const shock_opts *in, uint64_t n_leaves,
                                                                       const void *keys, const void *offsets,
                                                                       const void *out_seeds,
                                                                       const void *out_orient, int rf,
                                                                       shock_opts *out);

// Enqueue a whole search of a CSR batch on `stream` without host
// synchronisation (out_rot non-null: rotation fitting).  `buf` holds
// shock_internal_search_bytes bytes; the call's counters land in host_ctr
// (pinned, shock_internal_counter_bytes) when the stream reaches the end.
// Launches are sized for leaves of n_typical keys.  Returns SHOCK_OK,
// SHOCK_EINVAL or SHOCK_EHIP.
__attribute__((visibility("hidden"))) int shock_internal_enqueue(void *buf, uint64_t n_leaves, const uint64_t *keys,
                                                                 const uint64_t *offsets, uint64_t *out_seeds,
                                                                 uint32_t *out_rot, uint64_t *out_orient,
                                                                 const shock_opts *opts, uint32_t n_typical,
                                                                 hipStream_t stream,
                                                                 unsigned long long *host_ctr);

// Status of a completed call from its counters.
__attribute__((visibility("hidden"))) int shock_internal_status(const unsigned long long *host_ctr);

// Free the current device's per-stream scratch of the asynchronous searches
// (called by shock_release_scratch after the device is idle).
__attribute__((visibility("hidden"))) hipError_t shock_internal_release_stream_scratch(int dev);

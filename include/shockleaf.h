/*
 * shockleaf -- ShockHash leaf seed search on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libshockleaf.so.  Plain pointers and sizes only.  Unless a comment
 * says otherwise, every pointer is a DEVICE pointer on the current HIP device,
 * and every buffer is owned, allocated and freed by the caller.
 *
 * The operation (ShockHash, Section 4, the equation that defines the stored
 * seed): for each leaf S of n <= 64 keys, find the smallest seed s such that
 * some choice f : S -> {0,1} makes x -> h_{f(x)}(x, s) a bijection onto
 * [0, n), and return s with one such f.  By Section 5 (equation
 * "pseudoforests-orientable") a seed qualifies exactly when the graph on [n]
 * with one edge {h0(x,s), h1(x,s)} per key is a pseudoforest.  The search
 * tries seeds in increasing order, rejects most of them with the coverage
 * bit-mask filter of Section 4, confirms the rest with a union-find test of
 * the pseudoforest property (Appendix A.1; every component must have no more
 * edges than nodes, Section 2), and stops at the first acceptance.
 *
 * Hash family (frozen; the paper assumes ideal hashing of a 64-bit master
 * code, Section 8 and Section 5's uniform-hashing footnote):
 *   fmix64 = MurmurHash3's 64-bit finaliser,
 *   a = fmix64(key), t = fmix64((s + 1) * 0x9E3779B97F4A7C15) (mod 2^64),
 *   P = (lo32(a) ^ lo32(t)) * hi32(a) + t (mod 2^64), z = lo32(P) ^ hi32(P),
 *   Q = z * n (exact 64-bit), h0 = hi32(Q), r = (lo32(Q) * (n - 1)) >> 32,
 *   h1 = r + (r >= h0) for n >= 2 (never equal to h0: no self-loops,
 *   matching the paper's implementation footnote in Section 5), h1 = 0 if n = 1.
 *
 * Orientation output: bit i of out_orient[j] is f of the i-th key of leaf j
 * (0 = the key takes h0, 1 = it takes h1); bits >= n are zero.  Among the
 * 2^c valid choices (c = number of components, Section 5, equation
 * "orientations-cycles") the numerically smallest mask is returned, so the
 * output is unique: tree keys point away from their component's cycle and
 * every cycle is directed so that its highest-index key takes h0.
 *
 * Batch layout (CSR): leaf j owns keys[offsets[j] .. offsets[j+1]); offsets
 * has n_leaves + 1 nondecreasing uint64 entries in units of keys; keys are raw
 * 64-bit patterns.  A leaf with n = 0 or n = 1 is solved by the first seed
 * tried (start_seed) with orientation 0.
 *
 * Thread safety: synchronous calls from different host threads (on
 * different streams) may run concurrently: each host thread keeps its own
 * per-device scratch cache, held until the process ends or until that thread
 * calls shock_release_scratch().
 */
#ifndef SHOCKLEAF_H
#define SHOCKLEAF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define SHOCK_OK 0
#define SHOCK_EINVAL (-1)    /* malformed batch or options; nothing launched, outputs untouched */
#define SHOCK_ENOTFOUND (-2) /* some leaf has no qualifying seed below max_seed (seed = UINT64_MAX, orient = 0) */
#define SHOCK_EDUPKEY (-3)   /* check_dups was set and some leaf holds a repeated key; outputs untouched */
#define SHOCK_ECANCELED (-4) /* the cancel flag was raised; unfinished leaves hold seed = UINT64_MAX */
#define SHOCK_EHIP (-5)      /* a HIP runtime call failed; see shock_last_error() */
#define SHOCK_ENOMEM (-6)    /* scratch allocation failed, or a request larger than a queue's budget */
#define SHOCK_EPENDING (-7)  /* the asynchronous call or request has not completed yet */

/* Launch strategies.  All produce bit-identical outputs. */
#define SHOCK_MODE_AUTO 0
#define SHOCK_MODE_PLAIN_PER_LEAF 1 /* one kernel launch per leaf, queued back to back, whole GPU on that leaf */
#define SHOCK_MODE_PERSISTENT 2     /* one launch over all leaves: persistent work-stealing workers */

#define SHOCK_DEFAULT_MAX_SEED 4294967296ULL /* 2^32, exclusive */

typedef struct shock_opts {
  uint64_t max_seed;      /* exclusive cap on seeds (at most 2^63); 0 selects SHOCK_DEFAULT_MAX_SEED */
  uint64_t start_seed;    /* first seed tried (resume point); default 0 */
  int32_t mode;           /* SHOCK_MODE_*; AUTO = PERSISTENT */
  int32_t spl;            /* seeds per lane per iteration: 1, 2 or 4; 0 = tuned default for the batch */
  int32_t block_iters;    /* units (64*spl seeds) a worker claims at once, for every leaf size; 0 = by leaf size */
  int32_t waves_per_wg;   /* waves per workgroup = leaves a workgroup works on at once (1..16); 0 = tuned */
  int32_t workers;        /* persistent waves in the grid; 0 = sized to the batch: about one wave per leaf
                             (one workgroup per leaf for heavy leaves), at least 512, at most every resident wave */
  int32_t check_dups;     /* 1 = reject leaves with repeated keys (SHOCK_EDUPKEY) */
  const volatile int32_t *cancel; /* HOST pointer (pinned or managed memory) or NULL; nonzero = stop */
  int32_t leaf_size_hint; /* typical leaf size, sizes launches where offsets are not read back (contexts); 0 = 48 */
  int32_t partial_k;      /* rotation fitting only: partial-hash period 1 or 8; 0 = 8 above 32 keys, else 1 */
  const uint16_t *block_iters_by_n; /* HOST pointer to 65 claim sizes indexed by leaf size (0 = default), or NULL;
                                       e.g. the autotuner's table; overridden by block_iters when that is set */
  int32_t team;           /* persistent mode: 1 = each wave takes its own fresh leaves; 2 = the waves of a
                             workgroup share each fresh leaf (a shorter tail: each leaf finishes sooner);
                             0 = default (2) */
  int32_t bip_pool;       /* bipartite search only: candidates kept per side and leaf, 1..7168; 0 = 7168.
                             A first pass keeps min(512, max(1, bip_pool / 2)) and lists the leaves that
                             gather more; a second searches those again keeping bip_pool.  A leaf that
                             gathers more than bip_pool on one side before its pair is reported not found */
  uint64_t n_keys;        /* keys in the keys buffer, or 0 = unchecked (the caller guarantees offsets[n_leaves]
                             is within it); a leaf reaching past n_keys makes the batch SHOCK_EINVAL before any
                             of its keys is read */
} shock_opts;

/* Defaults for every field. */
void shock_opts_init(shock_opts *opts);

/* Synchronous search on the null stream with default options.
 *   keys       device, uint64[offsets[n_leaves]]
 *   offsets    device, uint64[n_leaves + 1], nondecreasing, each leaf <= 64 keys
 *   out_seeds  device, uint64[n_leaves]: smallest qualifying seed per leaf
 *   out_orient device, uint64[n_leaves]: canonical orientation mask per leaf
 * Returns SHOCK_OK, SHOCK_EINVAL (validated on the device before the search
 * starts; outputs untouched), SHOCK_ENOTFOUND, SHOCK_EHIP or SHOCK_ENOMEM. */
int shock_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                      uint64_t *out_seeds, uint64_t *out_orient);

/* As shock_leaf_search, with options, on `hip_stream` (a hipStream_t, NULL =
 * null stream).  Synchronous: returns when the outputs are final.  opts may be
 * NULL (defaults). */
int shock_leaf_search_ex(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                         uint64_t *out_seeds, uint64_t *out_orient,
                         const shock_opts *opts, void *hip_stream);

/* As shock_leaf_search_ex, but asynchronous: the whole search is enqueued on
 * hip_stream and the call returns without waiting for the device.  The
 * return value covers only what is checked before enqueueing (arguments and
 * options: SHOCK_EINVAL, nothing enqueued) and failures to enqueue or to
 * allocate (SHOCK_EHIP, SHOCK_ENOMEM).  The batch's own status (SHOCK_OK,
 * SHOCK_EINVAL for a malformed batch found on the device, whose outputs stay
 * untouched, SHOCK_ENOTFOUND, SHOCK_EDUPKEY, SHOCK_ECANCELED) is read with
 * shock_stream_status once the stream has reached the end of the call.
 * Launch sizes come from opts->leaf_size_hint (offsets are never read back).
 * The library keeps one scratch area and one status word per (device,
 * stream); a later call on the same stream reuses them in stream order and
 * replaces the status.  Calls on one stream must not be made from several
 * host threads at once.  Keys, offsets and outputs must stay valid until the
 * stream has passed the call. */
int shock_leaf_search_async(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                            uint64_t *out_seeds, uint64_t *out_orient, const shock_opts *opts, void *hip_stream);

/* Status of the last shock_leaf_search_async / shock_rf_leaf_search_async
 * on hip_stream of the current device: SHOCK_EPENDING while the stream has
 * not yet reached its end (never blocks), then the batch's status as above.
 * SHOCK_EINVAL if no asynchronous call was made on that stream. */
int shock_stream_status(void *hip_stream);

/* ShockHash with rotation fitting (Section 4, "Rotation Fitting"; partial
 * hash calculation, Appendix A.2).  Keys are split into two fixed sets by
 * the top bit of fmix64(key ^ 0xD1B54A32D192ED03) (1 = second set).  A
 * candidate is a pair (s, r), r in [0, n): keys of the first set take their
 * slots under seed s - (s mod k), keys of the second set take their slots
 * under seed s shifted by r mod n (the cyclic rotation of their bit mask).
 * k is opts->partial_k (0 = 8 for leaves above 32 keys, else 1).
 * Candidates are tried seed first, rotation second; the smallest pair whose
 * graph is a pseudoforest is returned:
 *   out_seeds  device, uint64[n_leaves]: s (UINT64_MAX if none below max_seed)
 *   out_rot    device, uint32[n_leaves]: r
 *   out_orient device, uint64[n_leaves]: canonical orientation of that graph
 * max_seed may be at most 2^57.  Other arguments and statuses as
 * shock_leaf_search_ex; synchronous. */
int shock_rf_leaf_search_ex(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                            uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient,
                            const shock_opts *opts, void *hip_stream);

/* As shock_rf_leaf_search_ex, asynchronous in the manner of
 * shock_leaf_search_async (status from shock_stream_status). */
int shock_rf_leaf_search_async(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                               uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient,
                               const shock_opts *opts, void *hip_stream);

/* Bipartite ShockHash (the outlook of Section 9: two hash functions of range
 * [n/2], one shifted by n/2; candidates are filtered before they are paired).
 * The n cells are split into a left part [0, nl), nl = floor(n / 2), and a
 * right part [nl, n).  With z the 32-bit hash value of key x under seed s
 * (the family above):
 *   Q = z * nl (exact 64-bit), left(x, s) = hi32(Q),
 *   right(x, s) = nl + ((lo32(Q) * (n - nl)) >> 32)
 * A pair (a, b) gives key x the cells left(x, a) and right(x, b).  Per leaf:
 *   out_a, out_b device u64[n_leaves]: the first pair in the order max(a, b),
 *       then a, then b whose graph is a pseudoforest (UINT64_MAX if none with
 *       max(a, b) < max_seed); leaves of 0 or 1 keys give (0, 0);
 *   out_orient device u64[n_leaves]: the canonical orientation of its graph
 *       (edges (left, right)).
 * Options used: max_seed (at most 2^32), workers, bip_pool.  Synchronous.
 * Status as shock_leaf_search_ex; SHOCK_ENOTFOUND also when a leaf gathers
 * more than bip_pool (default 7168) candidates on one side before its pair
 * (far beyond what uniform keys need); such a leaf's outputs are those of a
 * leaf without a pair.  stats (host, may be NULL) receives seeds hashed, candidate pairs
 * formed up to each leaf's answer, the pairs among them that the peeling test
 * ran on (a pair whose graph has a key alone in both of its cells, a one-edge
 * tree, is rejected without it), the kernel time (both passes), the workers
 * of the first pass and the leaves the second pass searched again. */
typedef struct {
  uint64_t seeds_hashed;
  uint64_t pairs_tested;
  uint64_t pairs_peeled;
  double kernel_ms;
  int32_t workers;
  int32_t second_pass_leaves; /* at most INT32_MAX */
} shock_bip_stats;

int shock_bip_leaf_search_ex(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                             uint64_t *out_a, uint64_t *out_b, uint64_t *out_orient,
                             const shock_opts *opts, void *hip_stream, shock_bip_stats *stats);

/* Device-side statistics of the last completed call on this host thread. */
typedef struct shock_stats {
  uint64_t seeds_tested;     /* seeds hashed, including seeds beyond a leaf's answer */
  uint64_t filter_passes;    /* seeds that passed the coverage filter */
  uint64_t pf_checks;        /* pseudoforest tests run (union-find; with rotation fitting, peeling per rotation) */
  uint64_t blocks_claimed;   /* seed blocks handed out */
  double kernel_ms;          /* time of the search kernel(s), HIP events on the call's stream */
  int32_t workers;           /* persistent waves launched */
  int32_t spl, block_iters, waves_per_wg; /* launch parameters actually used */
} shock_stats;
int shock_last_stats(shock_stats *out);

/* Message of the last SHOCK_EHIP / SHOCK_ENOMEM on this host thread. */
const char *shock_last_error(void);
const char *shock_strerror(int status);

/* Free the calling thread's cached scratch memory of the current device: the
 * search scratch, the Rice encoder's words, the bipartite search's counters
 * and events, and the MPHF build arena with its second stream and events
 * (the arena is sized by the largest build the thread has run: about 43
 * bytes per key).  Waits for the device first.  SHOCK_EHIP if a HIP call
 * fails. */
int shock_release_scratch(void);

/* Library version of the frozen hash/orientation definition (3: h0 and r come
 * from one multiply-shift range reduction of z and the fraction it leaves;
 * version 2 reduced the two 16-bit halves of z separately; version 1
 * multiplied lo32(a ^ t) by hi32(a ^ t)). */
int shock_spec_version(void);

/* ---- A search that allocates nothing -------------------------------------
 *
 * For callers that cannot allocate device memory: code running under HIP
 * graph capture elsewhere in the process, tight serving loops, harnesses that
 * forbid hipMalloc.  The same search and outputs as shock_leaf_search_ex in
 * persistent mode (mode AUTO or PERSISTENT; PLAIN_PER_LEAF is SHOCK_EINVAL),
 * synchronous on hip_stream.  Its scratch is one fixed array of
 * SHOCK_NOALLOC_SCRATCH_BYTES per GPU, part of the library's device code and
 * held by every GPU the library runs on until the process ends; the call
 * makes no hipMalloc, hipFree, hipHostMalloc or event creation (its status
 * comes back through a plain host copy, and kernel_ms in shock_last_stats
 * stays 0).  Limits: n_leaves <= SHOCK_NOALLOC_MAX_LEAVES and opts->workers <=
 * SHOCK_NOALLOC_MAX_WORKERS, else SHOCK_EINVAL before anything is launched.
 * Every call on one GPU uses that GPU's array and leaves its contents behind;
 * each call clears what it needs.  Calls on one GPU from several host threads
 * are serialised by the library; calls from the same process must not
 * otherwise overlap (the array holds one call's state). */
#define SHOCK_NOALLOC_MAX_LEAVES 65536
#define SHOCK_NOALLOC_MAX_WORKERS 32768
#define SHOCK_NOALLOC_SCRATCH_BYTES (34u << 20)
int shock_leaf_search_noalloc(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                              uint64_t *out_seeds, uint64_t *out_orient, const shock_opts *opts, void *hip_stream);

/* ---- Contexts: asynchronous searches, several in flight, HIP graphs ------
 *
 * A context owns the scratch for batches of up to max_leaves leaves (about
 * 600 bytes per leaf plus a fixed 130 KB) and pinned status counters.
 * Searches on a context are enqueued on a stream without any host
 * synchronisation, so a caller can keep several contexts in flight on
 * different streams (continuous batching) or capture the enqueue sequence in
 * a HIP graph and replay it.  Validation (nondecreasing offsets, n <= 64,
 * repeated keys if check_dups) happens on the device: a failed batch is not
 * searched, its outputs are left untouched, and the status is reported by
 * shock_ctx_wait.  Launch sizes come from opts->leaf_size_hint (nothing is
 * read back).  One search may be pending per context; a new enqueue on a
 * pending context first waits for it.  Contexts are not thread-safe. */
typedef struct shock_ctx shock_ctx;

/* Create a context on the current device.  SHOCK_ENOMEM if its scratch does
 * not fit. */
int shock_ctx_create(uint64_t max_leaves, shock_ctx **out);
int shock_ctx_destroy(shock_ctx *ctx);

/* Enqueue a search of a CSR batch (n_leaves <= max_leaves; arguments as for
 * shock_leaf_search_ex) on hip_stream.  Returns SHOCK_EINVAL for arguments
 * checkable on the host, SHOCK_EHIP if a launch fails, else SHOCK_OK; the
 * batch's own status comes from shock_ctx_wait. */
int shock_ctx_search_async(shock_ctx *ctx, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                           uint64_t *out_seeds, uint64_t *out_orient, const shock_opts *opts, void *hip_stream);

/* As shock_ctx_search_async, with rotation fitting (see
 * shock_rf_leaf_search_ex); out_rot is a device uint32[n_leaves]. */
int shock_ctx_rf_search_async(shock_ctx *ctx, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                              uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient,
                              const shock_opts *opts, void *hip_stream);

/* 1 if the context's last search has completed (or none is pending), 0 if it
 * is still running, SHOCK_EHIP on error.  Never blocks. */
int shock_ctx_query(shock_ctx *ctx);

/* Block until the last search completes and return its status (as
 * shock_leaf_search_ex).  Fills *stats (may be NULL); kernel_ms spans the
 * search kernels, or the whole graph for graph launches. */
int shock_ctx_wait(shock_ctx *ctx, shock_stats *stats);

/* Capture the enqueue sequence of one search (same arguments as
 * shock_ctx_search_async; no cancel flag) into a HIP graph held by the context,
 * replacing any earlier one.  The graph records buffer addresses, not
 * contents: each replay searches what those buffers hold at replay time. */
int shock_ctx_graph_capture(shock_ctx *ctx, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                            uint64_t *out_seeds, uint64_t *out_orient, const shock_opts *opts, void *hip_stream);

/* Replay the captured graph on hip_stream; complete it with shock_ctx_wait. */
int shock_ctx_graph_launch(shock_ctx *ctx, void *hip_stream);

/* ---- A request queue bound to one device and an HBM budget --------------
 *
 * Build requests (CSR batches of leaves in HOST memory) are submitted with
 * shock_submit and complete asynchronously; shock_poll reports completion.
 * The queue owns one device arena of hbm_budget_bytes, `slots` HIP streams
 * (default priority) with pinned staging buffers, and a dispatcher thread.
 * The dispatcher admits queued requests in submission order: a free slot
 * takes as many requests from the head of the queue as its staging buffers
 * and the arena's free memory allow, uploads their keys and offsets, enqueues
 * one search over all of them (the persistent kernel of shock_leaf_search_ex)
 * and moves on, so batches on different slots overlap on the device.  When a
 * slot's batch completes, each request's seeds and orientations are copied
 * into its host output buffers, its arena block is freed and the next
 * requests are admitted.  The device memory a batch holds (its keys,
 * offsets, outputs and search scratch) counts against the budget.  Results
 * equal those of shock_leaf_search_ex on each request alone: leaves are
 * searched independently. */
typedef struct shock_queue shock_queue;

typedef struct shock_queue_params {
  int32_t device;            /* HIP device ordinal */
  int32_t slots;             /* batches in flight at once (1..16); 0 = 4 */
  uint64_t hbm_budget_bytes; /* device arena size; 0 = 256 MiB */
  uint64_t max_batch_leaves; /* leaves one batch may hold; 0 = 65536 */
  uint64_t max_batch_keys;   /* keys one batch may hold (pinned staging per slot: 8 bytes each); 0 = 2^22 */
  shock_opts search;         /* search options of every request: mode AUTO or PERSISTENT, no cancel flag, no
                                check_dups (a batch shares one validation); a claim table is copied at creation;
                                leaf_size_hint is ignored: launches are sized by each batch's mean leaf size */
} shock_queue_params;

void shock_queue_params_init(shock_queue_params *p);

/* Device bytes a batch of n_leaves leaves and n_keys keys holds in a queue's
 * arena (keys, offsets, outputs and search scratch; about 560 bytes per leaf,
 * 8 per key and 135 KB per batch).  A request alone above the budget is
 * rejected by shock_submit. */
uint64_t shock_queue_batch_bytes(uint64_t n_leaves, uint64_t n_keys);

/* Create a queue.  SHOCK_EINVAL for bad parameters, SHOCK_ENOMEM if the
 * arena or the staging buffers cannot be allocated, SHOCK_EHIP otherwise. */
int shock_queue_create(const shock_queue_params *params, shock_queue **out);

/* Submit a request: n_leaves leaves in HOST memory, leaf j =
 * keys[offsets[j] .. offsets[j+1]) (offsets nondecreasing, each leaf <= 64
 * keys); results go to the HOST buffers out_seeds[n_leaves] and
 * out_orient[n_leaves].  All four buffers must stay valid until shock_poll
 * reports the request done.  Returns SHOCK_OK with *ticket set, SHOCK_EINVAL
 * for a malformed request (checked here on the host), or SHOCK_ENOMEM for a
 * request that alone exceeds the budget or one batch's limits (not queued). */
int shock_submit(shock_queue *q, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                 uint64_t *out_seeds, uint64_t *out_orient, uint64_t *ticket);

/* Times of one request on the steady clock (ns) and the batch it ran in. */
typedef struct shock_ticket_info {
  int64_t submit_ns, admit_ns, done_ns;
  uint64_t batch;
  uint64_t n_leaves;
} shock_ticket_info;

/* Never blocks.  While the request is queued or running: *done = 0 and
 * SHOCK_OK.  Once it is complete: *done = 1, *info filled (may be NULL), and
 * the request's status is returned (as shock_leaf_search_ex, or
 * SHOCK_ECANCELED); the ticket is then retired.  Unknown ticket:
 * SHOCK_EINVAL. */
int shock_poll(shock_queue *q, uint64_t ticket, int *done, shock_ticket_info *info);

/* Withdraw a request that has not been admitted yet: it completes with
 * SHOCK_ECANCELED and its outputs are untouched.  SHOCK_EPENDING if it is
 * already running (it will complete normally), SHOCK_EINVAL if unknown or
 * already complete. */
int shock_cancel(shock_queue *q, uint64_t ticket);

typedef struct shock_queue_stats {
  uint64_t submitted, completed, cancelled, batches;  /* completed counts every request that ended, the
                                                         cancelled ones (also counted in cancelled) included */
  uint64_t queued, running;                    /* requests now */
  uint64_t bytes_in_flight, max_bytes_in_flight;
  int32_t batches_in_flight, max_batches_in_flight;
} shock_queue_stats;
int shock_queue_stats_get(shock_queue *q, shock_queue_stats *out);

/* Stop the dispatcher: running batches finish, queued requests complete with
 * SHOCK_ECANCELED (without polling), then everything is freed. */
int shock_queue_destroy(shock_queue *q);

#ifdef __cplusplus
}
#endif
#endif

// Asynchronous searches on a caller's stream, and a request queue bound to one
// device and an HBM budget (include/shockleaf.h).
//
// Both run the search kernels of shockleaf.hip through shock_internal_enqueue:
// the whole call (validation, premix, persistent search, counters back to a
// pinned host word) is enqueued with no host synchronisation.
//
//  * shock_leaf_search_async keeps one scratch area, one pinned status word
//    and one event per (device, stream).  Calls on a stream reuse them in
//    stream order; shock_stream_status reads the word once the event says the
//    stream has passed the call.
//  * shock_queue admits host-side build requests into slots.  Each slot is a
//    stream with pinned staging for keys, offsets and results; a batch's
//    device memory (keys, offsets, outputs, search scratch) is one block of
//    the queue's arena, a single allocation of the whole budget made at
//    creation, so admission by device memory is exact and never calls
//    hipMalloc.  A dispatcher thread admits requests in submission order,
//    enqueues batches and retires them when their event completes.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "shockleaf.h"
#include "shock_internal.h"

namespace {

#define Q_TRY(call)                              \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) {                      \
      shock_internal_set_error(#call, e_);       \
      return SHOCK_EHIP;                         \
    }                                            \
  } while (0)

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ---------------------------------------------------------------- streams --

struct StreamState {
  void *buf = nullptr;
  size_t bytes = 0;
  unsigned long long *host_ctr = nullptr;
  hipEvent_t ev = nullptr;
  bool pending = false;
  int status = SHOCK_OK;
};

std::mutex g_streams_mu;
std::map<std::pair<int, uintptr_t>, StreamState *> g_streams;

int stream_state(int dev, hipStream_t stream, StreamState **out) {
  auto key = std::make_pair(dev, (uintptr_t)stream);
  auto it = g_streams.find(key);
  if (it != g_streams.end()) {
    *out = it->second;
    return SHOCK_OK;
  }
  StreamState *st = new StreamState();
  hipError_t e = hipHostMalloc((void **)&st->host_ctr, shock_internal_counter_bytes(), hipHostMallocDefault);
  if (e != hipSuccess) {
    shock_internal_set_error("hipHostMalloc(stream status)", e);
    delete st;
    return SHOCK_ENOMEM;
  }
  memset(st->host_ctr, 0, shock_internal_counter_bytes());
  e = hipEventCreateWithFlags(&st->ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    shock_internal_set_error("hipEventCreate(stream status)", e);
    (void)hipHostFree(st->host_ctr);
    delete st;
    return SHOCK_EHIP;
  }
  g_streams[key] = st;
  *out = st;
  return SHOCK_OK;
}

int search_async(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                 uint32_t *out_rot, uint64_t *out_orient, const shock_opts *opts_in, void *hip_stream, int rf) {
  shock_opts opts;
  if (n_leaves > 0) {
    const int rc = shock_internal_complete_opts(opts_in, n_leaves, keys, offsets, out_seeds, out_orient, rf, &opts);
    if (rc != SHOCK_OK) return rc;
    if (rf && !out_rot) return SHOCK_EINVAL;
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  int dev = 0;
  Q_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_streams_mu);
  StreamState *st = nullptr;
  int rc = stream_state(dev, stream, &st);
  if (rc != SHOCK_OK) return rc;
  if (n_leaves == 0) {
    // nothing to search: the stream's status is OK once it reaches this point
    st->pending = false;
    st->status = SHOCK_OK;
    return SHOCK_OK;
  }
  const size_t need = shock_internal_search_bytes(n_leaves, opts.mode == SHOCK_MODE_PLAIN_PER_LEAF);
  if (st->bytes < need) {
    if (st->buf) {
      Q_TRY(hipStreamSynchronize(stream));  // earlier calls on this stream may still use it
      Q_TRY(hipFree(st->buf));
      st->buf = nullptr;
      st->bytes = 0;
    }
    hipError_t e = hipMalloc(&st->buf, need);
    if (e != hipSuccess) {
      shock_internal_set_error("hipMalloc(stream scratch)", e);
      return SHOCK_ENOMEM;
    }
    st->bytes = need;
  }
  const uint32_t hint = opts.leaf_size_hint ? (uint32_t)opts.leaf_size_hint : 48;
  rc = shock_internal_enqueue(st->buf, n_leaves, keys, offsets, out_seeds, out_rot, out_orient, &opts, hint, stream,
                              st->host_ctr);
  if (rc != SHOCK_OK) {
    st->pending = false;
    st->status = rc;
    return rc;
  }
  Q_TRY(hipEventRecord(st->ev, stream));
  st->pending = true;
  return SHOCK_OK;
}

// ------------------------------------------------------------ the arena --

// First-fit allocator over one device allocation: free blocks by offset,
// neighbours merged on release.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  size_t alloc(size_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }

 private:
  std::map<size_t, size_t> free_;
};

// ------------------------------------------------------------- requests --

enum { kQueued = 0, kRunning = 1, kDone = 2 };

struct QReq {
  uint64_t ticket = 0;
  const uint64_t *keys = nullptr, *offsets = nullptr;
  uint64_t *out_seeds = nullptr, *out_orient = nullptr;
  uint64_t n_leaves = 0, n_keys = 0;
  int state = kQueued, status = SHOCK_OK;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
  uint64_t batch = 0;
  uint64_t leaf_base = 0;  // first leaf within its batch
};

struct QSlot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  unsigned long long *host_ctr = nullptr;  // pinned counters of the batch
  uint64_t *h_keys = nullptr;              // pinned staging: keys, then offsets, then results
  uint64_t *h_offs = nullptr;
  uint64_t *h_out = nullptr;  // seeds [0, cap_leaves), orientations [cap_leaves, 2 cap_leaves)
  bool busy = false;
  size_t block = 0, block_bytes = 0;
  uint64_t n_leaves = 0;
  std::vector<QReq *> reqs;
};

// Device bytes of a batch: keys, offsets, seeds, orientations, search scratch.
size_t batch_bytes(uint64_t n_leaves, uint64_t n_keys) {
  return up(8 * n_keys) + up(8 * (n_leaves + 1)) + 2 * up(8 * n_leaves) + up(shock_internal_search_bytes(n_leaves, 0));
}

}  // namespace

struct shock_queue {
  shock_queue_params p{};
  void *arena_base = nullptr;
  Arena arena;
  std::vector<QSlot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<QReq *> queued;
  std::unordered_map<uint64_t, QReq *> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  uint16_t claim_table[65] = {};  // the caller's block_iters_by_n, copied
  shock_queue_stats stats{};
  int fatal = SHOCK_OK;  // a HIP failure in the dispatcher fails every later batch
};

namespace {

// Stage, upload and enqueue one batch on a slot (dispatcher thread, lock not
// held).  Returns SHOCK_OK or the status every request of the batch gets.
int launch_batch(shock_queue *q, QSlot &s) {
  char *base = (char *)q->arena_base + s.block;
  uint64_t n_keys = 0, L = 0;
  for (QReq *r : s.reqs) {
    r->leaf_base = L;
    const uint64_t k0 = r->offsets[0];
    memcpy(s.h_keys + n_keys, r->keys + k0, 8 * r->n_keys);
    for (uint64_t j = 0; j < r->n_leaves; ++j) s.h_offs[L + j] = r->offsets[j] - k0 + n_keys;
    n_keys += r->n_keys;
    L += r->n_leaves;
  }
  s.h_offs[L] = n_keys;
  s.n_leaves = L;
  uint64_t *d_keys = (uint64_t *)base;
  uint64_t *d_offs = (uint64_t *)(base + up(8 * n_keys));
  uint64_t *d_seeds = (uint64_t *)((char *)d_offs + up(8 * (L + 1)));
  uint64_t *d_orient = (uint64_t *)((char *)d_seeds + up(8 * L));
  void *scratch = (char *)d_orient + up(8 * L);
  if (n_keys) Q_TRY(hipMemcpyAsync(d_keys, s.h_keys, 8 * n_keys, hipMemcpyHostToDevice, s.stream));
  Q_TRY(hipMemcpyAsync(d_offs, s.h_offs, 8 * (L + 1), hipMemcpyHostToDevice, s.stream));
  shock_opts opts = q->p.search;
  opts.n_keys = n_keys;
  const uint32_t n_mean = (uint32_t)((n_keys + L / 2) / L);
  const int rc = shock_internal_enqueue(scratch, L, n_keys ? d_keys : d_offs, d_offs, d_seeds, nullptr, d_orient,
                                        &opts, n_mean ? n_mean : 1, s.stream, s.host_ctr);
  if (rc != SHOCK_OK) return rc;
  Q_TRY(hipMemcpyAsync(s.h_out, d_seeds, 8 * L, hipMemcpyDeviceToHost, s.stream));
  Q_TRY(hipMemcpyAsync(s.h_out + q->p.max_batch_leaves, d_orient, 8 * L, hipMemcpyDeviceToHost, s.stream));
  Q_TRY(hipEventRecord(s.ev, s.stream));
  return SHOCK_OK;
}

// Complete a slot's requests with `rc` (lock held).
void finish_batch(shock_queue *q, QSlot &s, int rc) {
  const int64_t t = now_ns();
  for (QReq *r : s.reqs) {
    if (rc == SHOCK_OK || rc == SHOCK_ENOTFOUND) {
      memcpy(r->out_seeds, s.h_out + r->leaf_base, 8 * r->n_leaves);
      memcpy(r->out_orient, s.h_out + q->p.max_batch_leaves + r->leaf_base, 8 * r->n_leaves);
    }
    // a request's own status: ENOTFOUND only if one of its leaves has no seed
    int own = rc;
    if (rc == SHOCK_ENOTFOUND) {
      own = SHOCK_OK;
      for (uint64_t j = 0; j < r->n_leaves; ++j)
        if (r->out_seeds[j] == ~0ull) own = SHOCK_ENOTFOUND;
    }
    r->status = own;
    r->state = kDone;
    r->t_done = t;
    q->stats.completed++;
    q->stats.running--;
  }
  s.reqs.clear();
  q->arena.release(s.block, s.block_bytes);
  q->stats.bytes_in_flight -= s.block_bytes;
  q->stats.batches_in_flight--;
  s.busy = false;
}

// Take requests from the head of the queue for a free slot (lock held).
// Returns false if the head request does not fit now.
bool admit(shock_queue *q, QSlot &s) {
  uint64_t L = 0, N = 0;
  size_t n = 0;
  while (n < q->queued.size()) {
    const QReq *r = q->queued[n];
    if (L + r->n_leaves > q->p.max_batch_leaves || N + r->n_keys > q->p.max_batch_keys) break;
    L += r->n_leaves;
    N += r->n_keys;
    ++n;
  }
  // shrink the batch until its block fits the arena's free memory
  while (n > 0) {
    const size_t bytes = batch_bytes(L, N);
    const size_t off = q->arena.alloc(bytes);
    if (off != SIZE_MAX) {
      s.block = off;
      s.block_bytes = bytes;
      break;
    }
    --n;
    L -= q->queued[n]->n_leaves;
    N -= q->queued[n]->n_keys;
  }
  if (n == 0) return false;
  const int64_t t = now_ns();
  const uint64_t batch = q->stats.batches++;
  for (size_t i = 0; i < n; ++i) {
    QReq *r = q->queued.front();
    q->queued.pop_front();
    r->state = kRunning;
    r->t_admit = t;
    r->batch = batch;
    s.reqs.push_back(r);
  }
  q->stats.queued -= n;
  q->stats.running += n;
  q->stats.bytes_in_flight += s.block_bytes;
  if (q->stats.bytes_in_flight > q->stats.max_bytes_in_flight) q->stats.max_bytes_in_flight = q->stats.bytes_in_flight;
  q->stats.batches_in_flight++;
  if (q->stats.batches_in_flight > q->stats.max_batches_in_flight)
    q->stats.max_batches_in_flight = q->stats.batches_in_flight;
  s.busy = true;
  return true;
}

void dispatcher(shock_queue *q) {
  (void)hipSetDevice(q->p.device);
  std::unique_lock<std::mutex> lk(q->mu);
  for (;;) {
    bool in_flight = false;
    // retire completed batches
    for (QSlot &s : q->slots) {
      if (!s.busy) continue;
      const hipError_t e = hipEventQuery(s.ev);
      if (e == hipErrorNotReady) {
        in_flight = true;
        continue;
      }
      int rc = SHOCK_EHIP;
      if (e == hipSuccess) {
        rc = shock_internal_status(s.host_ctr);
      } else {
        shock_internal_set_error("hipEventQuery(queue slot)", e);
        q->fatal = SHOCK_EHIP;
      }
      finish_batch(q, s, rc);
    }
    if (q->stop && !in_flight) break;
    // admit queued requests into free slots
    if (!q->stop) {
      for (QSlot &s : q->slots) {
        if (s.busy || q->queued.empty()) continue;
        if (!admit(q, s)) break;
        int rc = q->fatal;
        if (rc == SHOCK_OK) {
          lk.unlock();
          rc = launch_batch(q, s);
          lk.lock();
        }
        if (rc != SHOCK_OK) {
          if (rc == SHOCK_EHIP) q->fatal = rc;
          // copies already enqueued may still touch the staging and the block
          (void)hipStreamSynchronize(s.stream);
          finish_batch(q, s, rc);
        } else {
          in_flight = true;
        }
      }
    }
    if (in_flight) {
      q->cv.wait_for(lk, std::chrono::microseconds(20));
    } else if (!q->stop) {
      q->cv.wait(lk, [q] { return q->stop || !q->queued.empty(); });
    }
  }
}

void free_queue(shock_queue *q) {
  for (QSlot &s : q->slots) {
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.ev) (void)hipEventDestroy(s.ev);
    if (s.host_ctr) (void)hipHostFree(s.host_ctr);
    if (s.h_keys) (void)hipHostFree(s.h_keys);
    if (s.h_offs) (void)hipHostFree(s.h_offs);
    if (s.h_out) (void)hipHostFree(s.h_out);
  }
  if (q->arena_base) (void)hipFree(q->arena_base);
  for (auto &kv : q->reqs) delete kv.second;
  delete q;
}

}  // namespace

hipError_t shock_internal_release_stream_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_streams_mu);
  for (auto it = g_streams.begin(); it != g_streams.end();) {
    if (it->first.first != dev) {
      ++it;
      continue;
    }
    StreamState *st = it->second;
    if (st->buf) {
      hipError_t e = hipFree(st->buf);
      if (e != hipSuccess) return e;
    }
    (void)hipEventDestroy(st->ev);
    (void)hipHostFree(st->host_ctr);
    delete st;
    it = g_streams.erase(it);
  }
  return hipSuccess;
}

extern "C" {

int shock_leaf_search_async(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                            uint64_t *out_orient, const shock_opts *opts, void *hip_stream) {
  return search_async(keys, offsets, n_leaves, out_seeds, nullptr, out_orient, opts, hip_stream, 0);
}

int shock_rf_leaf_search_async(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                               uint32_t *out_rot, uint64_t *out_orient, const shock_opts *opts, void *hip_stream) {
  return search_async(keys, offsets, n_leaves, out_seeds, out_rot, out_orient, opts, hip_stream, 1);
}

int shock_stream_status(void *hip_stream) {
  int dev = 0;
  Q_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_streams_mu);
  auto it = g_streams.find(std::make_pair(dev, (uintptr_t)hip_stream));
  if (it == g_streams.end()) return SHOCK_EINVAL;
  StreamState *st = it->second;
  if (st->pending) {
    const hipError_t e = hipEventQuery(st->ev);
    if (e == hipErrorNotReady) return SHOCK_EPENDING;
    if (e != hipSuccess) {
      shock_internal_set_error("hipEventQuery(stream status)", e);
      return SHOCK_EHIP;
    }
    st->pending = false;
    st->status = shock_internal_status(st->host_ctr);
  }
  return st->status;
}

void shock_queue_params_init(shock_queue_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->slots = 4;
  p->hbm_budget_bytes = 256ull << 20;
  p->max_batch_leaves = 65536;
  p->max_batch_keys = 1ull << 22;
  shock_opts_init(&p->search);
}

uint64_t shock_queue_batch_bytes(uint64_t n_leaves, uint64_t n_keys) { return batch_bytes(n_leaves, n_keys); }

int shock_queue_create(const shock_queue_params *params, shock_queue **out) {
  if (!out) return SHOCK_EINVAL;
  *out = nullptr;
  shock_queue_params p;
  shock_queue_params_init(&p);
  if (params) p = *params;
  if (p.slots == 0) p.slots = 4;
  if (p.hbm_budget_bytes == 0) p.hbm_budget_bytes = 256ull << 20;
  if (p.max_batch_leaves == 0) p.max_batch_leaves = 65536;
  if (p.max_batch_keys == 0) p.max_batch_keys = 1ull << 22;
  if (p.search.max_seed == 0) p.search.max_seed = SHOCK_DEFAULT_MAX_SEED;
  if (p.slots < 1 || p.slots > 16 || p.max_batch_leaves > (1ull << 31) || p.max_batch_keys > (1ull << 34))
    return SHOCK_EINVAL;
  if (p.search.mode != SHOCK_MODE_AUTO && p.search.mode != SHOCK_MODE_PERSISTENT) return SHOCK_EINVAL;
  // no cancel flag is kept (a batch serves several requests), and a repeated
  // key in one request must not fail the other requests of its batch
  if (p.search.cancel != nullptr || p.search.check_dups) return SHOCK_EINVAL;
  {
    // the search options are checked as a search call checks them
    shock_opts chk;
    static const uint64_t dummy = 0;
    const int rc = shock_internal_complete_opts(&p.search, 1, &dummy, &dummy, &dummy, &dummy, 0, &chk);
    if (rc != SHOCK_OK) return rc;
  }
  int count = 0, prev = 0;
  Q_TRY(hipGetDeviceCount(&count));
  if (p.device < 0 || p.device >= count) return SHOCK_EINVAL;
  Q_TRY(hipGetDevice(&prev));
  Q_TRY(hipSetDevice(p.device));
  shock_queue *q = new shock_queue();
  q->p = p;
  if (p.search.block_iters_by_n) {  // the claim table is copied: the caller's may go away
    memcpy(q->claim_table, p.search.block_iters_by_n, sizeof(q->claim_table));
    q->p.search.block_iters_by_n = q->claim_table;
  }
  q->slots.resize(p.slots);
  auto fail = [&](const char *what, hipError_t e, int rc) {
    shock_internal_set_error(what, e);
    free_queue(q);
    (void)hipSetDevice(prev);
    return rc;
  };
  hipError_t e = hipMalloc(&q->arena_base, p.hbm_budget_bytes);
  if (e != hipSuccess) return fail("hipMalloc(queue arena)", e, SHOCK_ENOMEM);
  q->arena.reset(p.hbm_budget_bytes);
  for (QSlot &s : q->slots) {
    if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess)
      return fail("hipStreamCreate(queue slot)", e, SHOCK_EHIP);
    if ((e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming)) != hipSuccess)
      return fail("hipEventCreate(queue slot)", e, SHOCK_EHIP);
    if ((e = hipHostMalloc((void **)&s.host_ctr, shock_internal_counter_bytes(), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&s.h_keys, 8 * p.max_batch_keys, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&s.h_offs, 8 * (p.max_batch_leaves + 1), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&s.h_out, 16 * p.max_batch_leaves, hipHostMallocDefault)) != hipSuccess)
      return fail("hipHostMalloc(queue staging)", e, SHOCK_ENOMEM);
  }
  (void)hipSetDevice(prev);
  q->stats.max_batches_in_flight = 0;
  q->th = std::thread(dispatcher, q);
  *out = q;
  return SHOCK_OK;
}

int shock_submit(shock_queue *q, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                 uint64_t *out_seeds, uint64_t *out_orient, uint64_t *ticket) {
  if (!q || !ticket || !offsets) return SHOCK_EINVAL;
  if (n_leaves > 0 && (!out_seeds || !out_orient)) return SHOCK_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j)
    if (offsets[j + 1] < offsets[j] || offsets[j + 1] - offsets[j] > 64) return SHOCK_EINVAL;
  const uint64_t n_keys = offsets[n_leaves] - offsets[0];
  if (n_keys > 0 && !keys) return SHOCK_EINVAL;
  if (n_leaves > q->p.max_batch_leaves || n_keys > q->p.max_batch_keys ||
      batch_bytes(n_leaves, n_keys) > q->p.hbm_budget_bytes)
    return SHOCK_ENOMEM;
  QReq *r = new QReq();
  r->keys = keys;
  r->offsets = offsets;
  r->out_seeds = out_seeds;
  r->out_orient = out_orient;
  r->n_leaves = n_leaves;
  r->n_keys = n_keys;
  r->t_submit = now_ns();
  std::lock_guard<std::mutex> lk(q->mu);
  r->ticket = q->next_ticket++;
  q->reqs[r->ticket] = r;
  q->stats.submitted++;
  if (n_leaves == 0) {
    r->state = kDone;
    r->t_admit = r->t_done = r->t_submit;
    q->stats.completed++;
  } else {
    q->queued.push_back(r);
    q->stats.queued++;
    q->cv.notify_all();
  }
  *ticket = r->ticket;
  return SHOCK_OK;
}

int shock_poll(shock_queue *q, uint64_t ticket, int *done, shock_ticket_info *info) {
  if (!q || !done) return SHOCK_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return SHOCK_EINVAL;
  QReq *r = it->second;
  if (r->state != kDone) {
    *done = 0;
    return SHOCK_OK;
  }
  *done = 1;
  if (info) {
    info->submit_ns = r->t_submit;
    info->admit_ns = r->t_admit;
    info->done_ns = r->t_done;
    info->batch = r->batch;
    info->n_leaves = r->n_leaves;
  }
  const int rc = r->status;
  q->reqs.erase(it);
  delete r;
  return rc;
}

int shock_cancel(shock_queue *q, uint64_t ticket) {
  if (!q) return SHOCK_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end() || it->second->state == kDone) return SHOCK_EINVAL;
  QReq *r = it->second;
  if (r->state == kRunning) return SHOCK_EPENDING;
  for (auto qi = q->queued.begin(); qi != q->queued.end(); ++qi) {
    if (*qi == r) {
      q->queued.erase(qi);
      break;
    }
  }
  r->state = kDone;
  r->status = SHOCK_ECANCELED;
  r->t_done = now_ns();
  q->stats.queued--;
  q->stats.cancelled++;
  q->stats.completed++;
  return SHOCK_OK;
}

int shock_queue_stats_get(shock_queue *q, shock_queue_stats *out) {
  if (!q || !out) return SHOCK_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  *out = q->stats;
  return SHOCK_OK;
}

int shock_queue_destroy(shock_queue *q) {
  if (!q) return SHOCK_EINVAL;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->stop = true;
    for (QReq *r : q->queued) {
      r->state = kDone;
      r->status = SHOCK_ECANCELED;
    }
    q->queued.clear();
    q->cv.notify_all();
  }
  if (q->th.joinable()) q->th.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(q->p.device);
  free_queue(q);
  (void)hipSetDevice(prev);
  return SHOCK_OK;
}

}  // extern "C"

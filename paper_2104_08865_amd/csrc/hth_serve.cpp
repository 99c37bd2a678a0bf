// libhth serving loop (hth_serve_* of include/hth.h): requests of host bytes
// are admitted by device memory, gathered into batches as they arrive and
// hashed by the same planner and kernel as hth_hash_batch.  This file only
// moves bytes, schedules batches and tracks tickets; every hash value comes
// from the HIP kernels.
//
// Data path of one request:
//   submit:  bytes copied into a pinned host ring (FIFO allocation), or, for
//            hth_serve_submit_pinned, left in the caller's pinned memory;
//   slot:    admitted when the device ring (the memory budget) has room,
//            packed with the other admitted requests into a batch, copied
//            host ring -> device ring on the slot's stream, hashed (one
//            launch per output width present), results copied back to a
//            pinned buffer;
//   retire:  when the batch's event completes, results move to the ticket
//            table and latencies are recorded; ring regions are released in
//            admission order (both rings are FIFO), once every earlier batch
//            has completed too.
// Each of the `slots` slots has a stream and a thread of its own, which
// admits a new batch as soon as its previous one has retired: the host work
// of building and enqueueing batches (a dozen HIP calls each) runs on
// several threads, and the copies of one batch overlap the hashing of others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hth_host.h"

using namespace hth::host;
using Clock = std::chrono::steady_clock;

namespace {

constexpr uint64_t kAlign = 256;  // request bytes start on 256-byte boundaries in both rings
constexpr uint64_t kDefaultDevice = 1ull << 30;
constexpr uint64_t kDefaultStage = 1ull << 30;
constexpr uint64_t kDefaultRequest = 16ull << 20;
constexpr uint64_t kDefaultBatchBytes = 64ull << 20;
constexpr uint32_t kDefaultBatchRequests = 16384;
constexpr uint32_t kDefaultSlots = 3;
constexpr uint32_t kDefaultOutstanding = 1u << 20;
constexpr uint32_t kMaxSlots = 8;
constexpr uint32_t kMaxBatchRequests = 1u << 22;
constexpr uint32_t kMaxOutstanding = 1u << 24;
// The planner's workspace always fits a batch of up to this many bytes (its
// task table holds 2^19 tasks beyond one per string).
constexpr uint64_t kMaxBatchBytes = 1ull << 36;
constexpr int kWidths = 4;

uint64_t pad(uint64_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }
int widx(uint32_t w) { return (int)(w / 8) - 2; }

// FIFO allocator over a ring of `cap` bytes.  Positions grow without bound;
// an allocation never straddles the end of the ring (it moves to the next
// start instead); space is released in allocation order.  An empty ring
// starts the next allocation at the beginning of a lap, so a request of up
// to `cap` bytes always fits once the ring has drained (without that, a
// request of more than cap / 2 bytes could wait forever for a drained ring
// whose head sits mid-lap).
struct Ring {
  uint64_t cap = 0, head = 0, tail = 0;
  bool alloc(uint64_t n, uint64_t* pos) {
    if (n > cap) return false;
    if (head == tail && head % cap) head = tail = head - head % cap + cap;
    uint64_t p = head;
    const uint64_t at = p % cap;
    if (at + n > cap) p += cap - at;
    if (p + n - tail > cap) return false;
    head = p + n;
    *pos = p;
    return true;
  }
  // Space up to `end` is free again.  (A batch of empty requests ends where
  // the ring stood when it was launched, which a later lap start may have
  // passed: the tail never moves back.)
  void release(uint64_t end) {
    if (end > tail) tail = end;
  }
};

struct Request {
  uint64_t ticket;
  uint64_t host_pos, dev_pos;
  uint64_t len;
  uint32_t width;
  bool deferred;
  Clock::time_point t_submit;
  const uint8_t* src;  // caller's pinned bytes (hth_serve_submit_pinned), else null: in the host ring
};

// Bytes a request takes in the device ring: a staged request keeps its
// 256-byte padding (runs contiguous in both rings are one copy); a pinned
// one takes exactly its length, so that requests contiguous in the caller's
// memory are contiguous on the device too and go in one copy.
uint64_t dev_bytes(const Request& r) { return r.src ? r.len : pad(r.len); }

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Workspace ws;
  uint64_t* h_meta = nullptr;  // pinned: per width, offsets then lengths
  uint64_t* d_meta = nullptr;
  uint8_t* h_out = nullptr;  // pinned results, grouped by width
  uint8_t* d_out = nullptr;
  std::vector<Request> reqs;
  uint64_t out_at[kWidths] = {};  // byte offset of each width group in the results
  uint64_t seq = 0;               // admission number of the slot's batch
};

// A batch between its admission and the release of its ring regions.
struct Inflight {
  uint64_t seq;
  uint64_t host_end, dev_end;
  bool done;
};

enum : uint8_t { kFree = 0, kPending = 1, kReady = 2 };

// A ticket's slot.  Only the submitter that finds it free moves it to
// pending (the ticket numbers of outstanding requests differ modulo the table
// size), the batch's slot thread to ready (under r_mu) and the collector back
// to free (under r_mu): the state is atomic so that submitters need no lock
// of the ticket table.
struct Entry {
  std::atomic<uint64_t> ticket{0};
  std::atomic<uint8_t> state{kFree};
  uint8_t width = 0;
  uint8_t out[40];
};

// The queue's lock: its holders work for a few hundred nanoseconds (a
// submit) or microseconds (an admission), and several submitting threads
// contend for it, where a sleeping mutex queued them through the kernel on
// every conflict.  Spins briefly, then yields.
class SpinMutex {
 public:
  void lock() {
    for (int n = 0; flag_.exchange(true, std::memory_order_acquire); ++n) {
      while (flag_.load(std::memory_order_relaxed)) {
        if (++n > 64) std::this_thread::yield();
      }
    }
  }
  bool try_lock() { return !flag_.exchange(true, std::memory_order_acquire); }
  void unlock() { flag_.store(false, std::memory_order_release); }

 private:
  std::atomic<bool> flag_{false};
};

}  // namespace

struct hth_server {
  hth_serve_config cfg{};
  const hth_seed* seed = nullptr;
  int device = 0;

  uint8_t* h_ring = nullptr;
  uint8_t* d_ring = nullptr;
  std::vector<Slot> slots;

  // host ring, device ring, pending queue (queue order = host ring order)
  // and the batches in flight (admission order), all under q_mu; a
  // request's bytes are copied outside the lock, so a slot admits a request
  // only once its `copied` flag is set
  SpinMutex q_mu;
  std::condition_variable_any q_cv;
  Ring host;
  Ring dev;
  std::deque<Request> pending;
  uint64_t next_ticket = 1;
  std::unique_ptr<std::atomic<uint8_t>[]> copied;  // per ticket slot
  std::atomic<int> idle_slots{0};                 // slot threads looking for requests
  uint64_t next_seq = 0;
  std::deque<Inflight> inflight;

  // tickets
  std::mutex r_mu;
  std::condition_variable r_cv;
  std::unique_ptr<Entry[]> entries;
  uint64_t mask = 0;

  // statistics since the last reset: completions under r_mu, submissions
  // under q_mu or atomic
  std::vector<float> lat_us;
  uint64_t n_completed = 0, n_batches = 0, n_batch_reqs = 0, n_bytes = 0;
  std::atomic<uint64_t> n_submitted{0}, n_deferred{0}, n_busy{0};
  bool have_first = false;  // (under q_mu)
  Clock::time_point t_first, t_last;

  std::atomic<bool> stop{false};
  std::atomic<bool> paused{false};
  std::atomic<int> failed{0};
  std::atomic<bool> fail_claimed{false};
  std::string fail_msg;  // written once, before `failed` is set
  std::vector<std::thread> workers;  // one per slot
};

namespace {

hth_status server_error(hth_server* s) {
  return fail(HTH_E_HIP, "serving loop stopped after an error: %s", s->fail_msg.c_str());
}

void set_failed(hth_server* s, hipError_t e, const char* what) {
  if (s->fail_claimed.exchange(true)) return;  // the first error is the one reported
  s->fail_msg = std::string(what) + ": " + hipGetErrorString(e);
  s->failed.store(1);
  s->q_cv.notify_all();
  std::lock_guard<std::mutex> lk(s->r_mu);
  s->r_cv.notify_all();
}

// Admits requests from the head of the queue into slot `sl` (q_mu held):
// only requests whose bytes are copied, while the device ring has room and
// the batch limits allow.  Returns false when nothing was admitted.
bool admit_locked(hth_server* s, Slot& sl) {
  sl.reqs.clear();
  uint64_t bytes = 0;
  while (!s->pending.empty() && sl.reqs.size() < s->cfg.max_batch_requests) {
    Request& r = s->pending.front();
    if (!s->copied[r.ticket & s->mask].load()) break;  // bytes still being copied
    if (!sl.reqs.empty() && bytes + r.len > s->cfg.max_batch_bytes) break;
    uint64_t pos = 0;
    if (!s->dev.alloc(dev_bytes(r), &pos)) {
      // device budget exhausted: the request waits for a batch to retire
      if (!r.deferred) {
        r.deferred = true;
        ++s->n_deferred;
      }
      break;
    }
    r.dev_pos = pos;
    bytes += r.len;
    sl.reqs.push_back(r);
    s->pending.pop_front();
  }
  if (sl.reqs.empty()) return false;
  sl.seq = s->next_seq++;
  // host ring space up to the end of the batch's last staged request (none:
  // nothing to release)
  uint64_t host_end = 0;
  for (const Request& r : sl.reqs)
    if (!r.src) host_end = r.host_pos + pad(r.len);
  s->inflight.push_back(Inflight{sl.seq, host_end, s->dev.head, false});
  return true;
}

// Pinned requests take their device ring bytes in admission order, but
// requests from several client threads arrive interleaved, so neighbours in
// the caller's memory are rarely neighbours in the queue.  Each run of
// pinned requests that is contiguous in the device ring is laid out again in
// the order of their host addresses (the same bytes of the ring, so nothing
// else changes), which makes requests adjacent in host memory adjacent on
// the device: one copy for each run of them.
void sort_pinned_runs(hth_server* s, Slot& sl) {
  std::vector<Request>& q = sl.reqs;
  size_t i = 0;
  while (i < q.size()) {
    if (!q[i].src) {
      ++i;
      continue;
    }
    size_t j = i + 1;
    uint64_t end = q[i].dev_pos + q[i].len;
    while (j < q.size() && q[j].src && q[j].dev_pos == end && (q[i].dev_pos % s->dev.cap) + (end - q[i].dev_pos) +
                                                                     q[j].len <= s->dev.cap) {
      end += q[j].len;
      ++j;
    }
    if (j - i > 1) {
      const uint64_t d0 = q[i].dev_pos;
      std::sort(q.begin() + i, q.begin() + j, [](const Request& a, const Request& b) { return a.src < b.src; });
      uint64_t d = d0;
      for (size_t k = i; k < j; ++k) {
        q[k].dev_pos = d;
        d += q[k].len;
      }
    }
    i = j;
  }
}

// Enqueues the admitted batch of slot `sl` on its stream (no lock held).
bool launch_batch(hth_server* s, Slot& sl) {
  sort_pinned_runs(s, sl);
  // group by width, in submission order inside each group
  uint64_t n[kWidths] = {};
  for (const Request& r : sl.reqs) ++n[widx(r.width)];
  uint64_t meta_at[kWidths], out_at = 0, meta = 0;
  for (int w = 0; w < kWidths; ++w) {
    meta_at[w] = meta;
    meta += 2 * n[w];
    sl.out_at[w] = out_at;
    out_at += n[w] * (uint64_t)(16 + 8 * w);
  }
  uint64_t fillw[kWidths] = {}, waves[kWidths] = {};
  for (const Request& r : sl.reqs) {
    const int w = widx(r.width);
    waves[w] += task_bound(r.len, r.width, s->seed->block);
    sl.h_meta[meta_at[w] + fillw[w]] = r.dev_pos % s->dev.cap;
    sl.h_meta[meta_at[w] + n[w] + fillw[w]] = r.len;
    ++fillw[w];
  }

  hipError_t e = hipSuccess;
  // request bytes: runs contiguous in host memory (the ring or the caller's)
  // and in the device ring become one copy
  auto src_of = [&](const Request& r) { return r.src ? r.src : s->h_ring + r.host_pos % s->host.cap; };
  size_t i = 0;
  while (i < sl.reqs.size() && e == hipSuccess) {
    const uint8_t* h0 = src_of(sl.reqs[i]);
    const uint64_t d0 = sl.reqs[i].dev_pos;
    uint64_t len = dev_bytes(sl.reqs[i]);
    size_t j = i + 1;
    while (j < sl.reqs.size() && src_of(sl.reqs[j]) == h0 + len && sl.reqs[j].dev_pos == d0 + len &&
           (d0 % s->dev.cap) + len + dev_bytes(sl.reqs[j]) <= s->dev.cap) {
      len += dev_bytes(sl.reqs[j]);
      ++j;
    }
    if (len) e = hipMemcpyAsync(s->d_ring + d0 % s->dev.cap, h0, len, hipMemcpyHostToDevice, sl.stream);
    i = j;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(sl.d_meta, sl.h_meta, meta * 8, hipMemcpyHostToDevice, sl.stream);
  if (e != hipSuccess) {
    set_failed(s, e, "batch upload");
    return false;
  }
  for (int w = 0; w < kWidths; ++w) {
    if (!n[w]) continue;
    const uint64_t* d_off = sl.d_meta + meta_at[w];
    hth_status st = enqueue_batch(s->seed, s->d_ring, d_off, d_off + n[w], n[w], sl.d_out + sl.out_at[w],
                                  (uint32_t)(16 + 8 * w), sl.ws, sl.stream, nullptr, nullptr, waves[w]);
    if (st != HTH_OK) {
      set_failed(s, hipErrorLaunchFailure, "batch launch");
      return false;
    }
  }
  e = hipMemcpyAsync(sl.h_out, sl.d_out, out_at, hipMemcpyDeviceToHost, sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) {
    set_failed(s, e, "batch download");
    return false;
  }
  return true;
}

// Publishes the results of slot `sl`'s completed batch, then releases the
// ring regions of the completed batches at the head of the admission order.
void retire(hth_server* s, Slot& sl) {
  const Clock::time_point now = Clock::now();
  uint64_t fillw[kWidths] = {}, bytes = 0;
  {
    std::lock_guard<std::mutex> lk(s->r_mu);
    for (const Request& r : sl.reqs) {
      const int w = widx(r.width);
      Entry& en = s->entries[r.ticket & s->mask];
      std::memcpy(en.out, sl.h_out + sl.out_at[w] + fillw[w] * r.width, r.width);
      ++fillw[w];
      en.state.store(kReady, std::memory_order_release);
      s->lat_us.push_back((float)std::chrono::duration<double, std::micro>(now - r.t_submit).count());
      bytes += r.len;
    }
    s->n_completed += sl.reqs.size();
    s->n_bytes += bytes;
    ++s->n_batches;
    s->n_batch_reqs += sl.reqs.size();
    s->t_last = now;
    s->r_cv.notify_all();
  }
  {
    std::lock_guard<SpinMutex> lk(s->q_mu);
    for (Inflight& f : s->inflight)
      if (f.seq == sl.seq) f.done = true;
    while (!s->inflight.empty() && s->inflight.front().done) {
      s->host.release(s->inflight.front().host_end);
      s->dev.release(s->inflight.front().dev_end);
      s->inflight.pop_front();
    }
  }
  s->q_cv.notify_all();  // slots waiting for device ring space
  sl.reqs.clear();
}

// The thread of slot `si`: admit a batch, enqueue it, wait for it, retire
// it, until the server stops or fails.
void worker_main(hth_server* s, uint32_t si) {
  if (hipSetDevice(s->device) != hipSuccess) {
    set_failed(s, hipErrorInvalidDevice, "slot thread hipSetDevice");
    return;
  }
  Slot& sl = s->slots[si];
  for (;;) {
    bool got = false;
    {
      std::unique_lock<SpinMutex> lk(s->q_mu);
      // counted idle before looking at the queue: a submit that the look
      // misses sees the count and wakes a slot (both are sequentially
      // consistent atomics)
      s->idle_slots.fetch_add(1);
      for (;;) {
        if (s->stop.load() || s->failed.load()) break;
        if (!s->paused.load() && admit_locked(s, sl)) {
          got = true;
          break;
        }
        s->q_cv.wait_for(lk, std::chrono::milliseconds(50));
      }
      s->idle_slots.fetch_sub(1);
    }
    if (!got || !launch_batch(s, sl)) return;
    // poll the batch's event: a blocking wait adds a wake-up to every
    // request's latency
    hipError_t e;
    while ((e = hipEventQuery(sl.done)) == hipErrorNotReady) std::this_thread::yield();
    if (e != hipSuccess) {
      set_failed(s, e, "batch completion");
      return;
    }
    retire(s, sl);
  }
}

void free_server(hth_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ws.mem) (void)hipFree(sl.ws.mem);
    if (sl.h_meta) (void)hipHostFree(sl.h_meta);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.d_meta) (void)hipFree(sl.d_meta);
    if (sl.d_out) (void)hipFree(sl.d_out);
  }
  if (s->h_ring) (void)hipHostFree(s->h_ring);
  if (s->d_ring) (void)hipFree(s->d_ring);
  delete s;
}

// Writes every page of a pinned host buffer once.  The pages are resident
// from the allocation on, but the process's page table maps them on first
// touch, one fault per page: left to the submitters, those faults cost more
// than the copies themselves (a 30 KB request touches 8 pages) and
// serialise threads on the address space lock.
void prefault(uint8_t* p, uint64_t n) {
  constexpr uint64_t kPage = 4096;
  const uint32_t nt = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  const uint64_t per = (n / kPage + nt - 1) / nt * kPage;
  auto touch = [&](uint64_t lo) {
    for (uint64_t o = lo; o < std::min(n, lo + per); o += kPage) p[o] = 0;
  };
  std::vector<std::thread> pool;
  try {
    for (uint32_t t = 1; t < nt; ++t) pool.emplace_back(touch, (uint64_t)t * per);
  } catch (...) {
    for (uint32_t t = (uint32_t)pool.size() + 1; t < nt; ++t) touch((uint64_t)t * per);
  }
  touch(0);
  for (auto& th : pool) th.join();
}

hth_status take(hth_server* s, uint64_t ticket, uint8_t* out, bool block) {
  std::unique_lock<std::mutex> lk(s->r_mu);
  Entry& en = s->entries[ticket & s->mask];
  if (en.ticket.load() != ticket || en.state.load() == kFree)
    return fail(HTH_E_INVALID, "ticket %llu is unknown or already collected", (unsigned long long)ticket);
  if (en.state.load() == kPending) {
    if (!block) {
      if (s->failed.load()) return server_error(s);
      return HTH_E_BUSY;
    }
    s->r_cv.wait(lk, [&] { return en.state.load() == kReady || s->failed.load(); });
    if (en.state.load() != kReady) return server_error(s);
  }
  std::memcpy(out, en.out, en.width);
  en.state.store(kFree, std::memory_order_release);
  return HTH_OK;
}

// Accepts one request: staged (copied into the host ring) or pinned (left
// in the caller's memory until its batch's copy).
hth_status submit(hth_server* s, const void* host_bytes, uint64_t len, uint32_t out_width, uint64_t* ticket,
                  bool pinned) {
  const Clock::time_point t0 = Clock::now();
  const char* fn = pinned ? "hth_serve_submit_pinned" : "hth_serve_submit";
  if (!s || !ticket) return fail(HTH_E_INVALID, "%s: null server or ticket", fn);
  if (!width_ok(out_width)) return fail(HTH_E_INVALID, "%s: out_width %u", fn, out_width);
  if (len && !host_bytes) return fail(HTH_E_INVALID, "%s: host_bytes is null", fn);
  if (len > s->cfg.max_request_bytes)
    return fail(HTH_E_TOO_LARGE, "%s: %llu bytes above the limit %llu", fn, (unsigned long long)len,
                (unsigned long long)s->cfg.max_request_bytes);
  if (s->failed.load()) return server_error(s);
  uint64_t t = 0, pos = 0;
  {
    std::lock_guard<SpinMutex> lk(s->q_mu);
    t = s->next_ticket;
    Entry& en = s->entries[t & s->mask];
    // (a free slot was freed by its collector with a release store: its
    // previous ticket's result has been read)
    bool ok = en.state.load(std::memory_order_acquire) == kFree && (pinned || s->host.alloc(pad(len), &pos));
    if (!ok) {
      ++s->n_busy;
      return HTH_E_BUSY;
    }
    en.ticket.store(t);
    en.width = (uint8_t)out_width;
    en.state.store(kPending, std::memory_order_release);
    ++s->n_submitted;
    if (!s->have_first) {
      s->have_first = true;
      s->t_first = t0;
    }
    ++s->next_ticket;
    s->copied[t & s->mask].store(pinned ? 1 : 0);
    s->pending.push_back(
        Request{t, pos, 0, len, out_width, false, t0, pinned ? static_cast<const uint8_t*>(host_bytes) : nullptr});
    if (pinned && s->idle_slots.load()) s->q_cv.notify_one();
  }
  *ticket = t;
  if (pinned) return HTH_OK;
  if (len) std::memcpy(s->h_ring + pos % s->host.cap, host_bytes, len);
  s->copied[t & s->mask].store(1);
  if (s->idle_slots.load()) {
    // the lock orders the notify after an idle slot's look at the queue
    std::lock_guard<SpinMutex> lk(s->q_mu);
    s->q_cv.notify_one();
  }
  return HTH_OK;
}

// Load replay (hth_serve_replay, hth_serve_replay_pinned).
hth_status replay(hth_server* s, const uint8_t* base, const uint64_t* offsets, const uint64_t* lengths,
                  const uint32_t* widths, const uint64_t* arrival_ns, uint64_t n, uint32_t threads,
                  uint64_t* tickets, bool pinned) {
  if (!s || (n && (!base || !offsets || !lengths || !widths || !arrival_ns || !tickets)))
    return fail(HTH_E_INVALID, "hth_serve_replay: null pointer");
  if (threads == 0 || threads > 64) return fail(HTH_E_INVALID, "hth_serve_replay: threads %u not in 1..64", threads);
  const Clock::time_point t0 = Clock::now();
  std::atomic<int> first_err{HTH_OK};
  std::string err_msg;
  std::mutex err_mu;
  // client k submits the chunks k, k + threads, ... of kReplayChunk
  // consecutive requests, each request at its arrival time (a client's
  // requests are neighbours in memory, as a client filling its own buffer
  // would make them, so pinned ones go to the device in few copies)
  constexpr uint64_t kReplayChunk = 64;
  auto client = [&](uint32_t k) {
    for (uint64_t i = (uint64_t)k * kReplayChunk; i < n && first_err.load() == HTH_OK;
         i = (i + 1) % kReplayChunk ? i + 1 : i + 1 + (uint64_t)(threads - 1) * kReplayChunk) {
      const Clock::time_point due = t0 + std::chrono::nanoseconds(arrival_ns[i]);
      while (Clock::now() < due) {
      }
      for (;;) {
        hth_status st = submit(s, base + offsets[i], lengths[i], widths[i], tickets + i, pinned);
        if (st == HTH_OK) break;
        if (st != HTH_E_BUSY) {
          std::lock_guard<std::mutex> lk(err_mu);
          if (first_err.load() == HTH_OK) {
            err_msg = hth_last_error();
            first_err.store(st);
          }
          return;
        }
        std::this_thread::yield();  // staging full: wait for a batch to retire
      }
    }
  };
  std::vector<std::thread> pool;
  try {
    for (uint32_t k = 1; k < threads; ++k) pool.emplace_back(client, k);
  } catch (...) {
    first_err.store(HTH_E_OOM);
    err_msg = "replay thread";
  }
  client(0);
  for (auto& th : pool) th.join();
  if (first_err.load() != HTH_OK) return fail(first_err.load(), "hth_serve_replay: %s", err_msg.c_str());
  return HTH_OK;
}

}  // namespace

extern "C" {

hth_status hth_serve_create(const hth_serve_config* config, const hth_seed* seed, hth_server** out) {
  if (!out) return fail(HTH_E_INVALID, "hth_serve_create: out is null");
  *out = nullptr;
  if (!config) return fail(HTH_E_INVALID, "hth_serve_create: config is null");
  hth_serve_config c = *config;
  if (!c.max_device_bytes) c.max_device_bytes = kDefaultDevice;
  if (!c.host_stage_bytes) c.host_stage_bytes = kDefaultStage;
  if (!c.max_request_bytes) c.max_request_bytes = kDefaultRequest;
  if (!c.max_batch_bytes) c.max_batch_bytes = kDefaultBatchBytes;
  if (!c.max_batch_requests) c.max_batch_requests = kDefaultBatchRequests;
  if (!c.slots) c.slots = kDefaultSlots;
  if (!c.max_outstanding) c.max_outstanding = kDefaultOutstanding;
  if (pad(c.max_request_bytes) > c.max_device_bytes || pad(c.max_request_bytes) > c.host_stage_bytes)
    return fail(HTH_E_INVALID, "hth_serve_create: max_request_bytes %llu does not fit the device budget or staging",
                (unsigned long long)c.max_request_bytes);
  if (c.max_batch_bytes > kMaxBatchBytes)
    return fail(HTH_E_INVALID, "hth_serve_create: max_batch_bytes above %llu", (unsigned long long)kMaxBatchBytes);
  if (c.slots > kMaxSlots) return fail(HTH_E_INVALID, "hth_serve_create: slots %u above %u", c.slots, kMaxSlots);
  if (c.max_batch_requests > kMaxBatchRequests)
    return fail(HTH_E_INVALID, "hth_serve_create: max_batch_requests %u above %u", c.max_batch_requests,
                kMaxBatchRequests);
  if (c.max_outstanding > kMaxOutstanding)
    return fail(HTH_E_INVALID, "hth_serve_create: max_outstanding %u above %u", c.max_outstanding, kMaxOutstanding);
  uint32_t outstanding = 1;
  while (outstanding < c.max_outstanding) outstanding <<= 1;
  c.max_outstanding = outstanding;
  if (!seed) return fail(HTH_E_INVALID, "hth_serve_create: seed is null");

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != seed->device)
    return fail(HTH_E_INVALID, "hth_serve_create: seed lives on device %d, current is %d", seed->device, dev);

  hth_server* s = new (std::nothrow) hth_server;
  if (!s) return fail(HTH_E_OOM, "hth_serve_create: host allocation");
  s->cfg = c;
  s->seed = seed;
  s->device = dev;
  s->host.cap = c.host_stage_bytes;
  s->dev.cap = c.max_device_bytes;
  s->mask = outstanding - 1;
  try {
    s->entries.reset(new Entry[outstanding]);
    s->slots.resize(c.slots);
    s->copied.reset(new std::atomic<uint8_t>[outstanding]);
    for (uint32_t i = 0; i < outstanding; ++i) s->copied[i].store(0);
  } catch (...) {
    delete s;
    return fail(HTH_E_OOM, "hth_serve_create: host allocation");
  }
  hth_status st = HTH_OK;
  const char* what = "";
  e = hipHostMalloc((void**)&s->h_ring, c.host_stage_bytes, hipHostMallocDefault);
  what = "staging ring";
  if (e == hipSuccess) prefault(s->h_ring, c.host_stage_bytes);
  if (e == hipSuccess) {
    e = hipMalloc((void**)&s->d_ring, c.max_device_bytes);
    what = "device ring";
  }
  const uint64_t meta_bytes = (uint64_t)c.max_batch_requests * 16;
  const uint64_t out_bytes = (uint64_t)c.max_batch_requests * 40;
  for (Slot& sl : s->slots) {
    if (e != hipSuccess) break;
    what = "slot buffers";
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_meta, meta_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_out, out_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_meta, meta_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_out, out_bytes);
    if (e == hipSuccess) {
      st = ws_alloc(sl.ws, c.max_batch_requests, sl.stream);
      if (st != HTH_OK) break;
    }
  }
  if (e != hipSuccess) st = hip_fail(e, what);
  if (st != HTH_OK) {
    std::string msg = hth_last_error();
    free_server(s);
    return fail(st, "hth_serve_create: %s", msg.c_str());
  }
  try {
    for (uint32_t i = 0; i < c.slots; ++i) s->workers.emplace_back(worker_main, s, i);
  } catch (...) {
    {
      std::lock_guard<SpinMutex> lk(s->q_mu);
      s->stop.store(true);
    }
    s->q_cv.notify_all();
    for (auto& t : s->workers) t.join();
    free_server(s);
    return fail(HTH_E_OOM, "hth_serve_create: slot thread");
  }
  *out = s;
  return HTH_OK;
}

hth_status hth_serve_submit(hth_server* s, const void* host_bytes, uint64_t len, uint32_t out_width,
                            uint64_t* ticket) {
  return submit(s, host_bytes, len, out_width, ticket, false);
}

hth_status hth_serve_submit_pinned(hth_server* s, const void* pinned_bytes, uint64_t len, uint32_t out_width,
                                   uint64_t* ticket) {
  return submit(s, pinned_bytes, len, out_width, ticket, true);
}

hth_status hth_serve_poll(hth_server* s, uint64_t ticket, uint8_t* out_host) {
  if (!s || !out_host) return fail(HTH_E_INVALID, "hth_serve_poll: null server or output");
  return take(s, ticket, out_host, false);
}

hth_status hth_serve_wait(hth_server* s, uint64_t ticket, uint8_t* out_host) {
  if (!s || !out_host) return fail(HTH_E_INVALID, "hth_serve_wait: null server or output");
  return take(s, ticket, out_host, true);
}

hth_status hth_serve_wait_many(hth_server* s, const uint64_t* tickets, uint64_t n, uint8_t* out_host,
                               uint32_t out_stride) {
  if (!s || (n && (!tickets || !out_host))) return fail(HTH_E_INVALID, "hth_serve_wait_many: null pointer");
  if (out_stride < 40) return fail(HTH_E_INVALID, "hth_serve_wait_many: out_stride %u below 40", out_stride);
  for (uint64_t i = 0; i < n; ++i) {
    hth_status st = take(s, tickets[i], out_host + i * out_stride, true);
    if (st != HTH_OK) return st;
  }
  return HTH_OK;
}

hth_status hth_serve_replay(hth_server* s, const uint8_t* base, const uint64_t* offsets, const uint64_t* lengths,
                            const uint32_t* widths, const uint64_t* arrival_ns, uint64_t n, uint32_t threads,
                            uint64_t* tickets) {
  return replay(s, base, offsets, lengths, widths, arrival_ns, n, threads, tickets, false);
}

hth_status hth_serve_replay_pinned(hth_server* s, const uint8_t* base, const uint64_t* offsets,
                                   const uint64_t* lengths, const uint32_t* widths, const uint64_t* arrival_ns,
                                   uint64_t n, uint32_t threads, uint64_t* tickets) {
  return replay(s, base, offsets, lengths, widths, arrival_ns, n, threads, tickets, true);
}

hth_status hth_serve_pause(hth_server* s, int32_t paused) {
  if (!s) return fail(HTH_E_INVALID, "hth_serve_pause: null server");
  {
    std::lock_guard<SpinMutex> lk(s->q_mu);
    s->paused.store(paused != 0);
  }
  s->q_cv.notify_all();
  return HTH_OK;
}

hth_status hth_serve_stats(hth_server* s, hth_serve_report* out) {
  if (!s || !out) return fail(HTH_E_INVALID, "hth_serve_stats: null pointer");
  std::vector<float> lat;
  hth_serve_report r{};
  {
    std::lock_guard<SpinMutex> ql(s->q_mu);
    std::lock_guard<std::mutex> lk(s->r_mu);
    lat = s->lat_us;
    r.submitted = s->n_submitted;
    r.completed = s->n_completed;
    r.deferred = s->n_deferred;
    r.busy = s->n_busy;
    r.batches = s->n_batches;
    r.bytes = s->n_bytes;
    r.mean_batch_requests = s->n_batches ? (double)s->n_batch_reqs / (double)s->n_batches : 0.0;
    if (s->have_first && s->n_completed)
      r.elapsed_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
  }
  r.gbps = r.elapsed_s > 0 ? (double)r.bytes / r.elapsed_s / 1e9 : 0.0;
  if (!lat.empty()) {
    auto rank = [&](double q) {
      size_t k = (size_t)(q * (double)(lat.size() - 1) + 0.5);
      std::nth_element(lat.begin(), lat.begin() + k, lat.end());
      return (double)lat[k];
    };
    double sum = 0;
    float mx = 0;
    for (float v : lat) {
      sum += v;
      mx = std::max(mx, v);
    }
    r.latency_mean_us = sum / (double)lat.size();
    r.latency_max_us = mx;
    r.latency_p50_us = rank(0.50);
    r.latency_p99_us = rank(0.99);
  }
  *out = r;
  if (s->failed.load()) return server_error(s);
  return HTH_OK;
}

hth_status hth_serve_reset_stats(hth_server* s) {
  if (!s) return fail(HTH_E_INVALID, "hth_serve_reset_stats: null server");
  std::lock_guard<SpinMutex> ql(s->q_mu);
  std::lock_guard<std::mutex> lk(s->r_mu);
  s->lat_us.clear();
  s->n_completed = s->n_batches = s->n_batch_reqs = s->n_bytes = 0;
  s->n_submitted = s->n_deferred = s->n_busy = 0;
  s->have_first = false;
  return HTH_OK;
}

hth_status hth_serve_destroy(hth_server* s) {
  if (!s) return HTH_OK;
  {
    std::lock_guard<SpinMutex> lk(s->q_mu);
    s->stop.store(true);
  }
  s->q_cv.notify_all();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  const bool was_failed = s->failed.load() != 0;
  std::string msg = s->fail_msg;
  free_server(s);
  if (was_failed) return fail(HTH_E_HIP, "serving loop had stopped after an error: %s", msg.c_str());
  return HTH_OK;
}

}  // extern "C"

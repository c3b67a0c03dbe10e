// Continuous-batching request server over device-resident tables: per-table FIFOs, admission by
// staging bytes and batch slots, dispatch on per-table streams, retirement by completion events.
// The interface and its guarantees are stated in ct_server.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <utility>
#include <vector>

#include "ct.h"
#include "ct_segcopy.h"
#include "ct_server.h"

namespace ct_serve {

constexpr int64_t kStageAlign = 256;

int64_t round_up(int64_t x) { return (x + kStageAlign - 1) / kStageAlign * kStageAlign; }

struct Req {
  int64_t ticket;
  int32_t table, op;
  const uint64_t* keys;
  const void* vals;
  int64_t n;
  void* vals_out;
  uint8_t* flags_out;
  int64_t submit_ns;
  // device addresses of the host arrays when they are mapped pinned memory (zc): the batch then
  // moves them with copy kernels; otherwise with DMA copies
  bool zc;
  const void* dkeys;
  const void* dvals;
  void* dvout;
  void* dflags;
};

// Device address of host array `h` if it is mapped pinned memory, else null (h null: null).
inline void* mapped(const void* h) {
  if (!h) return nullptr;
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, const_cast<void*>(h), 0) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory: an expected miss, not a pending error for later calls
    return nullptr;
  }
  return d;
}

struct Done {
  int64_t ticket, submit_ns, done_ns;
  int32_t status;
};

struct Batch {
  std::vector<Req> reqs;
  int32_t table, op;
  int64_t off, bytes;
  hipEvent_t ev;
  ct_status status;
};

// First-fit allocator over [0, size) of the staging buffer; freed ranges are merged with their
// free neighbours.
class Ranges {
 public:
  void reset(int64_t size) {
    free_.clear();
    free_[0] = size;
  }
  int64_t largest() const {
    int64_t m = 0;
    for (auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  int64_t take(int64_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      int64_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return off;
    }
    return -1;
  }
  void give(int64_t off, int64_t bytes) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + bytes) {
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
  std::map<int64_t, int64_t> free_;
};

}  // namespace ct_serve

using namespace ct_serve;

struct ct_server {
  // configuration
  std::vector<ct_table*> tables;
  std::vector<int32_t> vbytes;
  std::vector<hipStream_t> streams;
  int32_t max_inflight;
  int64_t max_batch;
  uint8_t* staging;
  int64_t staging_bytes;
  int device;
  std::chrono::steady_clock::time_point t0;

  // shared with callers, under mu
  std::mutex mu;
  std::condition_variable wake, idle;
  std::deque<Req> inbox;
  std::deque<Done> done;
  int64_t submitted = 0, completed = 0, batches = 0;
  int64_t peak_bytes = 0, peak_inflight = 0;
  int64_t dispatch_ns = 0, retire_ns = 0;
  int32_t error = CT_OK;
  bool stop = false;

  // worker-private
  std::vector<std::deque<Req>> queues;
  std::set<std::pair<int64_t, int32_t>> order;  // (ticket of the queued head, table), oldest first
  std::vector<std::deque<Batch>> inflight;  // per stream, in launch (= completion) order
  int64_t n_inflight = 0;
  std::vector<hipEvent_t> spare_events;
  Ranges ranges;
  int64_t inflight_bytes = 0;
  std::thread worker;

  int64_t now_ns() const {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now() - t0)
        .count();
  }

  int64_t need(int32_t t, int32_t op, int64_t n) const {
    const int64_t vb = vbytes[t];
    int64_t b = round_up(n * 8) + round_up(n);
    if (op == CT_OP_INSERT || op == CT_OP_FIND) b += round_up(n * vb);
    return b < kStageAlign ? kStageAlign : b;
  }

  void note_error(ct_status st) {
    std::lock_guard<std::mutex> g(mu);
    if (error == CT_OK) error = st;
  }

  void dispatch(Batch& b) {
    const int32_t t = b.table;
    const int64_t vb = vbytes[t];
    hipStream_t st = streams[t % streams.size()];
    int64_t nsum = 0;
    for (auto& r : b.reqs) nsum += r.n;
    uint8_t* base = staging + b.off;
    uint64_t* dk = reinterpret_cast<uint64_t*>(base);
    int64_t p = round_up(nsum * 8);
    uint8_t* dv = nullptr;
    if ((b.op == CT_OP_INSERT || b.op == CT_OP_FIND) && vb) {
      dv = base + p;
      p += round_up(nsum * vb);
    }
    uint8_t* df = base + p;
    ct_status rc = CT_OK;
    bool zc = true;
    for (auto& r : b.reqs) zc = zc && r.zc;
    if (zc && b.op == CT_OP_FIND) {
      // a find reads each key once and writes each result once: with mapped host arrays it runs
      // directly on them, request by request, with no staging copies
      for (auto& r : b.reqs)
        if (rc == CT_OK && r.n)
          rc = ct_find_batch(tables[t], static_cast<const uint64_t*>(r.dkeys), r.n,
                             r.vals_out ? r.dvout : nullptr, static_cast<uint8_t*>(r.dflags), st);
      if (hipEventRecord(b.ev, st) != hipSuccess) {
        rc = CT_E_HIP;
        (void)hipStreamSynchronize(st);
      }
      b.status = rc;
      if (rc != CT_OK) note_error(rc);
      return;
    }
    Seg seg[kMaxSegs];
    int nseg = 0;
    auto add = [&](const void* src, void* dst, int64_t bytes) {
      if (bytes <= 0) return;
      seg[nseg++] = Seg{src, dst, bytes};
      if (nseg == kMaxSegs) {
        if (segcopy(seg, nseg, st) != hipSuccess) rc = CT_E_HIP;
        nseg = 0;
      }
    };
    auto flush = [&] {
      if (nseg && segcopy(seg, nseg, st) != hipSuccess) rc = CT_E_HIP;
      nseg = 0;
    };
    int64_t pos = 0;
    for (auto& r : b.reqs) {
      if (zc) {
        add(r.dkeys, dk + pos, r.n * 8);
        if (b.op == CT_OP_INSERT && dv) add(r.dvals, dv + pos * vb, r.n * vb);
      } else {
        if (r.n && hipMemcpyAsync(dk + pos, r.keys, r.n * 8, hipMemcpyHostToDevice, st) != hipSuccess)
          rc = CT_E_HIP;
        if (b.op == CT_OP_INSERT && dv && r.n &&
            hipMemcpyAsync(dv + pos * vb, r.vals, r.n * vb, hipMemcpyHostToDevice, st) != hipSuccess)
          rc = CT_E_HIP;
      }
      pos += r.n;
    }
    flush();
    if (rc == CT_OK) {
      ct_table* tab = tables[t];
      if (b.op == CT_OP_INSERT)
        rc = ct_insert_batch(tab, dk, dv, nsum, df, st);
      else if (b.op == CT_OP_FIND)
        rc = ct_find_batch(tab, dk, nsum, dv, df, st);
      else
        rc = ct_erase_batch(tab, dk, nsum, df, st);
    }
    pos = 0;
    for (auto& r : b.reqs) {
      if (rc == CT_OK && zc) {
        if (r.flags_out) add(df + pos, r.dflags, r.n);
        if (b.op == CT_OP_FIND && dv && r.vals_out) add(dv + pos * vb, r.dvout, r.n * vb);
      } else {
        if (rc == CT_OK && r.n && r.flags_out &&
            hipMemcpyAsync(r.flags_out, df + pos, r.n, hipMemcpyDeviceToHost, st) != hipSuccess)
          rc = CT_E_HIP;
        if (rc == CT_OK && r.n && b.op == CT_OP_FIND && dv && r.vals_out &&
            hipMemcpyAsync(r.vals_out, dv + pos * vb, r.n * vb, hipMemcpyDeviceToHost, st) !=
                hipSuccess)
          rc = CT_E_HIP;
      }
      pos += r.n;
    }
    if (rc == CT_OK) flush();
    // the event marks the end of everything enqueued for the batch, failed or not; without it
    // the stream is drained here so that the staging range is idle before it is reused
    if (hipEventRecord(b.ev, st) != hipSuccess) {
      rc = CT_E_HIP;
      (void)hipStreamSynchronize(st);
    }
    b.status = rc;
    if (rc != CT_OK) note_error(rc);
  }

  // Admit batches while the head of the oldest waiting table fits; returns the number of
  // requests admitted.
  int64_t admit() {
    int64_t any = 0;
    while (!order.empty()) {
      const int32_t t = order.begin()->second;
      std::deque<Req>& q = queues[t];
      if (n_inflight >= max_inflight) break;
      const Req& h = q.front();
      const int64_t room = ranges.largest();
      int64_t n = h.n;
      if (need(t, h.op, n) > room) break;  // back-pressure in arrival order
      size_t take = 1;
      while (take < q.size() && q[take].op == h.op && n + q[take].n <= max_batch &&
             need(t, h.op, n + q[take].n) <= room) {
        n += q[take].n;
        ++take;
      }
      Batch b;
      b.table = t;
      b.op = h.op;
      b.bytes = need(t, h.op, n);
      b.off = ranges.take(b.bytes);
      b.reqs.assign(q.begin(), q.begin() + take);
      q.erase(q.begin(), q.begin() + take);
      b.ev = spare_events.back();
      spare_events.pop_back();
      order.erase(order.begin());
      if (!q.empty()) order.insert({q.front().ticket, t});
      const int64_t d0 = now_ns();
      dispatch(b);
      const int64_t d1 = now_ns();
      inflight_bytes += b.bytes;
      any += (int64_t)take;
      inflight[t % streams.size()].push_back(std::move(b));
      ++n_inflight;
      std::lock_guard<std::mutex> g(mu);
      ++batches;
      dispatch_ns += d1 - d0;
      if (inflight_bytes > peak_bytes) peak_bytes = inflight_bytes;
      if (n_inflight > peak_inflight) peak_inflight = n_inflight;
    }
    return any;
  }

  // Retire the batches whose events have completed; returns true if any was.  A stream runs its
  // batches in launch order, so only the oldest batch of each stream needs to be queried.
  bool retire() {
    const int64_t r0 = now_ns();
    std::vector<Done> fin;
    for (auto& q : inflight) {
      while (!q.empty()) {
        Batch& b = q.front();
        const hipError_t e = hipEventQuery(b.ev);
        if (e == hipErrorNotReady) break;
        ct_status st = b.status;
        if (e != hipSuccess) {
          st = CT_E_HIP;
          note_error(st);
        }
        const int64_t now = now_ns();
        for (auto& r : b.reqs) fin.push_back(Done{r.ticket, r.submit_ns, now, (int32_t)st});
        ranges.give(b.off, b.bytes);
        inflight_bytes -= b.bytes;
        spare_events.push_back(b.ev);
        q.pop_front();
        --n_inflight;
      }
    }
    std::lock_guard<std::mutex> g(mu);
    retire_ns += now_ns() - r0;
    if (fin.empty()) return false;
    for (auto& d : fin) done.push_back(d);
    completed += (int64_t)fin.size();
    if (completed == submitted) idle.notify_all();
    return true;
  }

  void run() {
    (void)hipSetDevice(device);
    std::vector<Req> got;
    int64_t queued = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu);
        if (n_inflight == 0 && queued == 0)
          wake.wait(lk, [&] { return stop || !inbox.empty(); });
        if (stop && inbox.empty() && n_inflight == 0 && queued == 0) return;
        got.assign(inbox.begin(), inbox.end());
        inbox.clear();
      }
      for (auto& r : got) {
        if (queues[r.table].empty()) order.insert({r.ticket, r.table});
        queues[r.table].push_back(r);
      }
      queued += (int64_t)got.size();
      bool moved = retire();
      const int64_t admitted = admit();
      queued -= admitted;
      if (!moved && !admitted && got.empty()) std::this_thread::yield();
    }
  }
};

extern "C" {

ct_status ct_server_create(ct_table* const* tables, int32_t ntables, const ct_server_desc* d,
                           void* d_staging, int64_t staging_bytes, ct_server** out) {
  if (!out || !tables || ntables < 1 || !d || !d_staging) return CT_E_INVALID;
  *out = nullptr;
  if (d->streams < 1 || d->streams > 16 || d->max_inflight < 1 || d->max_inflight > 4096 ||
      d->max_batch_keys < 1 || staging_bytes < kStageAlign ||
      reinterpret_cast<uintptr_t>(d_staging) % kStageAlign)
    return CT_E_INVALID;
  for (int32_t i = 0; i < ntables; ++i)
    if (!tables[i]) return CT_E_INVALID;
  ct_server* s = new (std::nothrow) ct_server();
  if (!s) return CT_E_NOMEM;
  s->tables.assign(tables, tables + ntables);
  s->vbytes.resize(ntables);
  for (int32_t i = 0; i < ntables; ++i) ct_table_value_bytes(tables[i], &s->vbytes[i]);
  s->max_inflight = d->max_inflight;
  s->max_batch = d->max_batch_keys;
  s->staging = static_cast<uint8_t*>(d_staging);
  s->staging_bytes = staging_bytes / kStageAlign * kStageAlign;
  s->ranges.reset(s->staging_bytes);
  s->queues.resize(ntables);
  s->inflight.resize(d->streams);
  s->t0 = std::chrono::steady_clock::now();
  ct_status rc = CT_OK;
  if (hipGetDevice(&s->device) != hipSuccess) rc = CT_E_HIP;
  for (int32_t i = 0; rc == CT_OK && i < d->streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      rc = CT_E_HIP;
      break;
    }
    s->streams.push_back(st);
  }
  for (int32_t i = 0; rc == CT_OK && i < d->max_inflight; ++i) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      rc = CT_E_HIP;
      break;
    }
    s->spare_events.push_back(e);
  }
  if (rc != CT_OK) {
    for (auto e : s->spare_events) (void)hipEventDestroy(e);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return rc;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return CT_OK;
}

ct_status ct_server_submit(ct_server* s, int32_t table, int32_t op, const uint64_t* h_keys,
                           const void* h_vals, int64_t n, void* h_vals_out, uint8_t* h_flags_out,
                           int64_t* ticket) {
  if (!s || table < 0 || table >= (int32_t)s->tables.size() || n < 0) return CT_E_INVALID;
  if (op != CT_OP_INSERT && op != CT_OP_FIND && op != CT_OP_ERASE) return CT_E_INVALID;
  if (n > 0 && !h_keys) return CT_E_INVALID;
  if (n > 0 && op == CT_OP_INSERT && s->vbytes[table] && !h_vals) return CT_E_INVALID;
  if (n > (INT64_MAX / 32) || s->need(table, op, n) > s->staging_bytes) return CT_E_INVALID;
  Req r{0, table, op, h_keys, h_vals, n, h_vals_out, h_flags_out, 0,
        false, nullptr, nullptr, nullptr, nullptr};
  if (n > 0) {  // map the arrays the batch will move; any unmapped one sends it through DMA
    const int64_t vb = s->vbytes[table];
    r.dkeys = mapped(h_keys);
    r.dvals = (op == CT_OP_INSERT && vb) ? mapped(h_vals) : nullptr;
    r.dvout = (op == CT_OP_FIND && vb && h_vals_out) ? mapped(h_vals_out) : nullptr;
    r.dflags = h_flags_out ? mapped(h_flags_out) : nullptr;
    r.zc = r.dkeys && (op != CT_OP_INSERT || !vb || r.dvals) &&
           (op != CT_OP_FIND || !vb || !h_vals_out || r.dvout) && (!h_flags_out || r.dflags);
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return CT_E_INVALID;
    r.ticket = s->submitted++;
    r.submit_ns = s->now_ns();
    s->inbox.push_back(r);
  }
  s->wake.notify_one();
  if (ticket) *ticket = r.ticket;
  return CT_OK;
}

ct_status ct_server_poll(ct_server* s, int64_t* tickets, int64_t* submit_ns, int64_t* done_ns,
                         int32_t* status, int64_t max, int64_t* count) {
  if (!s || max < 0 || !count) return CT_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  int64_t k = 0;
  while (k < max && !s->done.empty()) {
    const Done& d = s->done.front();
    if (tickets) tickets[k] = d.ticket;
    if (submit_ns) submit_ns[k] = d.submit_ns;
    if (done_ns) done_ns[k] = d.done_ns;
    if (status) status[k] = d.status;
    s->done.pop_front();
    ++k;
  }
  *count = k;
  return CT_OK;
}

ct_status ct_server_wait_idle(ct_server* s) {
  if (!s) return CT_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  s->idle.wait(lk, [&] { return s->completed == s->submitted; });
  return CT_OK;
}

ct_status ct_server_get_stats(ct_server* s, ct_server_stats* out) {
  if (!s || !out) return CT_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->batches = s->batches;
  out->peak_staging_bytes = s->peak_bytes;
  out->peak_inflight = s->peak_inflight;
  out->dispatch_ns = s->dispatch_ns;
  out->retire_ns = s->retire_ns;
  out->error = s->error;
  return CT_OK;
}

ct_status ct_server_now(ct_server* s, int64_t* ns) {
  if (!s || !ns) return CT_E_INVALID;
  *ns = s->now_ns();
  return CT_OK;
}

ct_status ct_server_destroy(ct_server* s) {
  if (!s) return CT_E_INVALID;
  ct_server_wait_idle(s);
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->wake.notify_all();
  s->worker.join();
  for (auto e : s->spare_events) (void)hipEventDestroy(e);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return CT_OK;
}

}  // extern "C"

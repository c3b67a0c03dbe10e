// Scheduling test of the request server on the host: the server source is built against a
// host-only HIP stand-in and a reference table (std::unordered_map), then fed random requests from
// the caller's thread while its worker runs.  Every request's results must equal a sequential
// replay of all requests in submission order; staging bytes and batch slots stay within their
// caps; every ticket completes exactly once.  Exit status 0 on success.
#include "../../paper_1908_05936_amd/csrc/ct_server.hip"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <unordered_map>

// --- the copy kernel of the server, done on the host ---------------------------------------------
static std::atomic<int64_t> g_segcopies{0};
namespace ct_serve {
hipError_t segcopy(const Seg* segs, int n, hipStream_t) {
  if (n <= 0 || n > kMaxSegs) std::abort();
  for (int i = 0; i < n; ++i) std::memcpy(segs[i].dst, segs[i].src, (size_t)segs[i].bytes);
  ++g_segcopies;
  return hipSuccess;
}
}  // namespace ct_serve

// --- reference tables behind the ct.h batch calls ---------------------------------------------
struct ct_table {
  std::unordered_map<uint64_t, uint64_t> m;
  int64_t cap;
  int32_t vb;
};

static std::atomic<int> g_calls_in_flight{0};

extern "C" {
ct_status ct_table_value_bytes(const ct_table* t, int32_t* b) {
  *b = t->vb;
  return CT_OK;
}
static uint64_t load_val(const void* v, int32_t vb, int64_t i) {
  if (vb == 8) return static_cast<const uint64_t*>(v)[i];
  return static_cast<const uint32_t*>(v)[i];
}
static void store_val(void* v, int32_t vb, int64_t i, uint64_t x) {
  if (vb == 8) static_cast<uint64_t*>(v)[i] = x;
  else static_cast<uint32_t*>(v)[i] = (uint32_t)x;
}
ct_status ct_insert_batch(ct_table* t, const uint64_t* keys, const void* vals, int64_t n,
                          uint8_t* status, void*) {
  if (g_calls_in_flight.fetch_add(1) != 0) std::abort();  // only the worker may call in
  for (int64_t i = 0; i < n; ++i) {
    uint8_t s;
    if (t->m.count(keys[i])) s = CT_PRESENT;
    else if ((int64_t)t->m.size() >= t->cap) s = CT_FULL;
    else {
      t->m[keys[i]] = t->vb ? load_val(vals, t->vb, i) : 0;
      s = CT_INSERTED;
    }
    if (status) status[i] = s;
  }
  g_calls_in_flight.fetch_sub(1);
  return CT_OK;
}
ct_status ct_find_batch(ct_table* t, const uint64_t* keys, int64_t n, void* vals_out,
                        uint8_t* found, void*) {
  if (g_calls_in_flight.fetch_add(1) != 0) std::abort();
  for (int64_t i = 0; i < n; ++i) {
    auto it = t->m.find(keys[i]);
    if (vals_out) store_val(vals_out, t->vb, i, it == t->m.end() ? ~0ull : it->second);
    if (found) found[i] = it != t->m.end();
  }
  g_calls_in_flight.fetch_sub(1);
  return CT_OK;
}
ct_status ct_erase_batch(ct_table* t, const uint64_t* keys, int64_t n, uint8_t* erased, void*) {
  if (g_calls_in_flight.fetch_add(1) != 0) std::abort();
  for (int64_t i = 0; i < n; ++i) {
    bool e = t->m.erase(keys[i]) > 0;
    if (erased) erased[i] = e;
  }
  g_calls_in_flight.fetch_sub(1);
  return CT_OK;
}
}

struct TestReq {
  int32_t table, op;
  std::vector<uint64_t> keys, vals, vout;
  std::vector<uint32_t> vout32;
  std::vector<uint8_t> flags;
  std::vector<uint64_t> exp_vout;
  std::vector<uint8_t> exp_flags;
  int seen = 0;
};

static int fail(const char* what, long a, long b) {
  std::fprintf(stderr, "FAIL %s (%ld, %ld)\n", what, a, b);
  return 1;
}

static int run_case(uint32_t seed, int ntables, int streams, int inflight, int64_t budget,
                    int64_t max_batch, int nreq) {
  std::mt19937_64 rng(seed);
  std::vector<ct_table> tabs(ntables), model(ntables);
  std::vector<ct_table*> handles;
  for (int t = 0; t < ntables; ++t) {
    tabs[t].cap = model[t].cap = 40 + 30 * t;
    tabs[t].vb = model[t].vb = (t % 3 == 0) ? 8 : (t % 3 == 1) ? 4 : 0;
    handles.push_back(&tabs[t]);
  }
  std::vector<TestReq> reqs(nreq);
  for (auto& r : reqs) {
    r.table = (int32_t)(rng() % ntables);
    r.op = (int32_t)(1 + rng() % 3);
    const int64_t n = (int64_t)(rng() % 120);
    for (int64_t i = 0; i < n; ++i) {
      r.keys.push_back(rng() % 150);
      r.vals.push_back(rng());
    }
    r.vout.assign(n, 0x5a5a5a5a5a5a5a5aull);
    r.vout32.assign(n, 0x5a5a5a5au);
    r.flags.assign(n, 0xee);
  }
  // sequential replay in submission order
  for (auto& r : reqs) {
    ct_table& m = model[r.table];
    const int64_t n = (int64_t)r.keys.size();
    r.exp_flags.assign(n, 0);
    r.exp_vout.assign(n, 0x5a5a5a5a5a5a5a5aull);
    if (m.vb == 4)  // only the low half of each output word is written
      for (auto& v : r.exp_vout) v = 0x5a5a5a5a00000000ull;
    if (r.op == CT_OP_INSERT) {
      std::vector<uint32_t> v32(r.vals.begin(), r.vals.end());
      ct_insert_batch(&m, r.keys.data(), m.vb == 4 ? (const void*)v32.data() : r.vals.data(), n,
                      r.exp_flags.data(), nullptr);
    } else if (r.op == CT_OP_FIND) {
      std::vector<uint64_t> o(n, 0);
      if (m.vb == 4) {
        std::vector<uint32_t> o32(n);
        ct_find_batch(&m, r.keys.data(), n, o32.data(), r.exp_flags.data(), nullptr);
        for (int64_t i = 0; i < n; ++i) r.exp_vout[i] = (r.exp_vout[i] & ~0xffffffffull) | o32[i];
      } else if (m.vb == 8) {
        ct_find_batch(&m, r.keys.data(), n, r.exp_vout.data(), r.exp_flags.data(), nullptr);
      } else {
        ct_find_batch(&m, r.keys.data(), n, nullptr, r.exp_flags.data(), nullptr);
      }
    } else {
      ct_erase_batch(&m, r.keys.data(), n, r.exp_flags.data(), nullptr);
    }
  }
  // the server; 32-bit values are passed as packed u32 arrays
  std::vector<std::vector<uint32_t>> v32(nreq);
  void* staging = std::aligned_alloc(256, (size_t)budget);
  ct_server_desc d{streams, inflight, max_batch};
  ct_server* s = nullptr;
  if (ct_server_create(handles.data(), ntables, &d, staging, budget, &s) != CT_OK)
    return fail("create", 0, 0);
  std::vector<int64_t> ticket_of(nreq);
  for (int i = 0; i < nreq; ++i) {
    TestReq& r = reqs[i];
    const void* vals = r.vals.data();
    if (tabs[r.table].vb == 4) {
      v32[i].assign(r.vals.begin(), r.vals.end());
      vals = v32[i].data();
    }
    int64_t tk = -1;
    void* vout = tabs[r.table].vb == 4 ? (void*)r.vout32.data() : (void*)r.vout.data();
    ct_status rc = ct_server_submit(s, r.table, r.op, r.keys.data(), vals, (int64_t)r.keys.size(),
                                    vout, r.flags.data(), &tk);
    if (rc != CT_OK) return fail("submit", i, rc);
    if (tk != i) return fail("ticket order", i, tk);
    if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
  }
  if (ct_server_wait_idle(s) != CT_OK) return fail("wait", 0, 0);
  std::vector<int64_t> tk(nreq + 1), sub(nreq + 1), dn(nreq + 1);
  std::vector<int32_t> st(nreq + 1);
  int64_t cnt = 0;
  if (ct_server_poll(s, tk.data(), sub.data(), dn.data(), st.data(), nreq + 1, &cnt) != CT_OK)
    return fail("poll", 0, 0);
  if (cnt != nreq) return fail("completed count", cnt, nreq);
  for (int64_t j = 0; j < cnt; ++j) {
    if (tk[j] < 0 || tk[j] >= nreq) return fail("ticket range", j, tk[j]);
    if (reqs[tk[j]].seen++) return fail("ticket twice", j, tk[j]);
    if (st[j] != CT_OK) return fail("status", j, st[j]);
    if (dn[j] < sub[j]) return fail("done before submit", j, tk[j]);
  }
  ct_server_stats stats{};
  ct_server_get_stats(s, &stats);
  if (stats.peak_staging_bytes > budget) return fail("budget", stats.peak_staging_bytes, budget);
  if (stats.peak_inflight > inflight) return fail("slots", stats.peak_inflight, inflight);
  if (stats.error != CT_OK) return fail("error", stats.error, 0);
  for (int i = 0; i < nreq; ++i) {
    TestReq& r = reqs[i];
    if (r.flags != r.exp_flags) return fail("flags", i, r.op);
    if (r.op == CT_OP_FIND && tabs[r.table].vb) {
      if (tabs[r.table].vb == 8 && r.vout != r.exp_vout) return fail("values", i, 8);
      if (tabs[r.table].vb == 4)
        for (size_t k = 0; k < r.vout32.size(); ++k)
          if (r.vout32[k] != (uint32_t)r.exp_vout[k]) return fail("values", i, 4);
    }
  }
  for (int t = 0; t < ntables; ++t)
    if (tabs[t].m != model[t].m) return fail("final contents", t, 0);
  // requests that can never fit are rejected up front
  std::vector<uint64_t> big((size_t)budget, 1);
  if (ct_server_submit(s, 0, CT_OP_FIND, big.data(), nullptr, (int64_t)big.size(), nullptr,
                       nullptr, nullptr) != CT_E_INVALID)
    return fail("oversized request accepted", 0, 0);
  if (ct_server_destroy(s) != CT_OK) return fail("destroy", 0, 0);
  std::free(staging);
  if (mock_live_streams() || mock_live_events()) return fail("leak", mock_live_streams(), mock_live_events());
  std::printf("case seed=%u tables=%d streams=%d inflight=%d budget=%ld batch=%ld: %d requests, %ld batches, peak %ld B / %ld slots\n",
              seed, ntables, streams, inflight, (long)budget, (long)max_batch, nreq,
              (long)stats.batches, (long)stats.peak_staging_bytes, (long)stats.peak_inflight);
  return 0;
}

int main() {
  int bad = 0;
  bad |= run_case(1, 5, 3, 4, 1 << 14, 256, 3000);   // tight budget: back-pressure, fragmentation
  bad |= run_case(2, 7, 1, 1, 1 << 20, 1 << 20, 2000);  // one stream, one slot
  bad |= run_case(3, 3, 8, 64, 1 << 20, 64, 3000);   // many slots, small merge cap
  bad |= run_case(4, 1, 2, 16, 4096, 1 << 10, 1500); // one table, staging for a few small batches
  if (g_segcopies.load() == 0) {
    std::printf("FAIL the copy-kernel path was never taken\n");
    bad = 1;
  }
  if (!bad) std::printf("server host test passed\n");
  return bad;
}

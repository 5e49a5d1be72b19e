// CPU test of the serving scheduler with a fake executor (no GPU). Built by
// tests/test_serve_core_cpu.py with g++ under ThreadSanitizer and under
// AddressSanitizer; prints "ALL OK" and exits 0 when every check passes.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "../include/cloud.h"
#include "../paper_1609_05344_amd/csrc/serve_core.h"

using namespace cloud::serve;

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);    \
      exit(1);                                                           \
    }                                                                    \
  } while (0)

// Batches finish after `delay_polls` queries, or, with batch_ns set, like an
// in-order device: a batch runs from the later of its launch and the previous
// batch's end for base_ns + batch_ns per request. Records what it saw and
// checks the scheduler's promises: a stream is never twice in one batch nor
// in more in-flight batches than the pipeline allows, its requests reach the
// device in submission order, and memory is only handed out within the
// budget.
class FakeExecutor : public Executor {
 public:
  std::mutex mu;
  int delay_polls = 3;
  int64_t base_ns = 0, batch_ns = 0;  // > 0: timed, in-order batches
  int max_per_stream = 1;             // requests of a stream in flight
  int fail_launch_every = 0;          // every n-th launch fails (0: never)
  int fail_query_every = 0;           // every n-th batch reports a device error
  std::map<int, std::vector<Item>> slots;
  std::map<int, int> polls;
  std::map<int, int64_t> ends;
  std::map<uint64_t, int> inflight_streams;
  std::map<uint64_t, uint64_t> last_request;
  std::vector<std::vector<Item>> history;
  size_t live_bytes = 0, peak_bytes = 0;
  int launches = 0, queries_failed = 0, peak_per_stream = 0;
  int64_t device_end = 0;
  std::atomic<int> allocs{0}, releases{0};

  size_t stream_bytes(int w, int h) override { return (size_t)w * h * 32; }
  int alloc(size_t b, void** m) override {
    std::lock_guard<std::mutex> lk(mu);
    *m = malloc(b ? b : 1);
    live_bytes += b;
    peak_bytes = std::max(peak_bytes, live_bytes);
    sizes[*m] = b;
    allocs++;
    return *m ? 0 : CLOUD_E_NOMEM;
  }
  void release(void* m) override {
    std::lock_guard<std::mutex> lk(mu);
    live_bytes -= sizes[m];
    sizes.erase(m);
    free(m);
    releases++;
  }
  int launch(int slot, const std::vector<Item>& items) override {
    std::lock_guard<std::mutex> lk(mu);
    launches++;
    CHECK(slots.find(slot) == slots.end());
    std::set<uint64_t> in_batch;
    for (const Item& it : items) {
      CHECK(in_batch.insert(it.stream_id).second);               // one per stream and batch
      CHECK(++inflight_streams[it.stream_id] <= max_per_stream);
      peak_per_stream = std::max(peak_per_stream, inflight_streams[it.stream_id]);
      CHECK(it.request_id > last_request[it.stream_id]);         // in submission order
      last_request[it.stream_id] = it.request_id;
      CHECK(it.stream_mem != nullptr);
      // the output buffer and stream memory are touched like a device would
      static_cast<unsigned char*>(it.stream_mem)[0] = (unsigned char)it.frame;
    }
    history.push_back(items);
    if (fail_launch_every && launches % fail_launch_every == 0) {
      for (const Item& it : items) inflight_streams[it.stream_id]--;
      return CLOUD_E_HIP;
    }
    slots[slot] = items;
    polls[slot] = 0;
    if (batch_ns > 0) {
      device_end = std::max(device_end, now_ns()) + base_ns + batch_ns * (int64_t)items.size();
      ends[slot] = device_end;
    }
    return 0;
  }
  int query(int slot) override {
    std::lock_guard<std::mutex> lk(mu);
    auto it = slots.find(slot);
    CHECK(it != slots.end());
    if (batch_ns > 0) {
      if (now_ns() < ends[slot]) return 0;
    } else if (++polls[slot] < delay_polls) {
      return 0;
    }
    for (const Item& x : it->second) inflight_streams[x.stream_id]--;
    slots.erase(it);
    if (fail_query_every && ++queries_failed % fail_query_every == 0) return CLOUD_E_HIP;
    return 1;
  }

 private:
  std::map<void*, size_t> sizes;
};

static std::vector<Completion> drain(Scheduler& s, size_t want, int timeout_ms = 5000) {
  std::vector<Completion> got;
  auto t0 = std::chrono::steady_clock::now();
  while (got.size() < want) {
    Completion c[64];
    int n = 0;
    s.poll(c, 64, &n);
    got.insert(got.end(), c, c + n);
    if (n == 0) s.wait(2000000);
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms)) break;
  }
  return got;
}

static uint64_t submit(Scheduler& s, uint64_t sid, int w, int h, uint32_t frame, int* rc = nullptr) {
  uint64_t id = 0;
  std::string msg;
  int r = s.submit(sid, w, h, frame, nullptr, std::vector<unsigned char>(8, 1), &id, &msg);
  if (rc) *rc = r;
  else CHECK(r == 0);
  return id;
}

static uint64_t submit_out(Scheduler& s, uint64_t sid, int w, int h, uint32_t frame, void* out) {
  uint64_t id = 0;
  std::string msg;
  CHECK(s.submit(sid, w, h, frame, out, std::vector<unsigned char>(8, 1), &id, &msg) == 0);
  return id;
}

static void test_order_and_reset() {
  FakeExecutor ex;
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  {
    Scheduler s(&ex, cfg);
    std::map<uint64_t, std::vector<uint64_t>> ids;
    for (uint32_t f = 0; f < 6; ++f)
      for (uint64_t sid = 1; sid <= 4; ++sid) ids[sid].push_back(submit(s, sid, 8 + (int)sid, 8, f + 3));
    auto got = drain(s, 24);
    CHECK(got.size() == 24);
    std::map<uint64_t, std::vector<uint64_t>> seen;
    for (auto& c : got) {
      CHECK(c.status == 0);
      CHECK(c.t_submit <= c.t_admit && c.t_admit <= c.t_start && c.t_start <= c.t_done);
      seen[c.stream_id].push_back(c.request_id);
    }
    CHECK(seen == ids);   // completion order per stream == submission order
    // first request of each stream has no history -> reset; later ones do not
    std::set<uint64_t> first_seen;
    for (auto& batch : ex.history)
      for (auto& it : batch) {
        const bool first = first_seen.insert(it.stream_id).second;
        CHECK(it.reset_history == first);
      }
    // frame 0 always resets
    uint64_t r = submit(s, 2, 10, 8, 0);
    auto g2 = drain(s, 1);
    CHECK(g2.size() == 1 && g2[0].request_id == r);
    CHECK(ex.history.back().back().reset_history);
    Stats st = s.stats();
    CHECK(st.completed == 25 && st.queued == 0 && st.running == 0 && st.streams == 4);
  }
  CHECK(ex.live_bytes == 0 && ex.allocs == ex.releases);
  printf("order_and_reset ok\n");
}

static void test_budget_admission() {
  FakeExecutor ex;
  Config cfg;
  cfg.budget_bytes = 2 * 16 * 16 * 32;   // room for two 16x16 streams
  Scheduler s(&ex, cfg);
  int rc = 0;
  submit(s, 99, 64, 64, 1, &rc);
  CHECK(rc == CLOUD_E_NOMEM);             // can never fit
  for (uint64_t sid = 1; sid <= 4; ++sid) submit(s, sid, 16, 16, 1);
  auto got = drain(s, 2, 300);
  CHECK(got.size() == 2);                  // only two streams admitted
  got = drain(s, 1, 100);
  CHECK(got.empty());
  CHECK(ex.peak_bytes <= cfg.budget_bytes);
  Stats st = s.stats();
  CHECK(st.streams == 4 && st.queued == 2 && st.bytes_in_use == cfg.budget_bytes);
  // closing the admitted streams frees room for the others
  std::set<uint64_t> done;
  for (uint64_t sid = 1; sid <= 4; ++sid)
    if (s.close_stream(sid) == 0) done.insert(sid);
  (void)done;
  got = drain(s, 2, 2000);
  // two were closed before admission (cancelled) or admitted after the close
  // freed memory; either way every request completes exactly once
  CHECK(got.size() == 2);
  CHECK(ex.peak_bytes <= cfg.budget_bytes);
  printf("budget_admission ok\n");
}

static void test_queue_full_and_mismatch() {
  FakeExecutor ex;
  ex.delay_polls = 1 << 30;               // batches never finish until released
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  cfg.max_queue = 4;
  cfg.max_batch = 1;
  Scheduler* s = new Scheduler(&ex, cfg);
  int rc = 0;
  submit(*s, 1, 8, 8, 1);
  submit(*s, 1, 9, 8, 2, &rc);
  CHECK(rc == CLOUD_E_INVALID);           // resolution fixed by the first request
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  int ok = 0, busy = 0;
  for (int i = 0; i < 10; ++i) {
    submit(*s, 1, 8, 8, 2 + i, &rc);
    if (rc == 0) ok++;
    else if (rc == CLOUD_E_BUSY) busy++;
  }
  CHECK(ok == 4 && busy == 6);
  CHECK(s->stats().rejected == 6);
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    ex.delay_polls = 1;                   // let the device finish
  }
  auto got = drain(*s, 5);
  CHECK(got.size() == 5);
  delete s;
  CHECK(ex.live_bytes == 0);
  printf("queue_full_and_mismatch ok\n");
}

static void test_close_and_destroy_cancel() {
  FakeExecutor ex;
  ex.delay_polls = 1 << 30;                 // the first batch stays on the device
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  Scheduler* s = new Scheduler(&ex, cfg);
  for (int i = 0; i < 5; ++i) submit(*s, 7, 8, 8, 1 + i);
  for (int i = 0; i < 5; ++i) submit(*s, 8, 8, 8, 1 + i);
  for (int k = 0; k < 500 && s->stats().running < 2; ++k)
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  CHECK(s->stats().running == 2);           // frame 1 of both streams in flight
  CHECK(s->close_stream(7) == 0);
  CHECK(s->close_stream(12345) == CLOUD_E_NOTFOUND);
  int rc = 0;
  submit(*s, 7, 8, 8, 9, &rc);
  CHECK(rc == CLOUD_E_INVALID);             // closing while its frame is in flight
  auto got = drain(*s, 4, 1000);
  CHECK(got.size() == 4);
  for (auto& c : got) CHECK(c.status == CLOUD_E_CANCELLED && c.stream_id == 7);
  CHECK(s->stats().bytes_in_use == 2 * 8 * 8 * 32);   // freed only after the batch
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    ex.delay_polls = 1;
  }
  got = drain(*s, 2, 2000);                 // frame 1 of 7 and of 8 (and maybe more of 8)
  CHECK(got.size() >= 2);
  for (int k = 0; k < 500 && s->stats().streams != 1; ++k)
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  CHECK(s->stats().streams == 1);            // stream 7 is gone
  delete s;                                  // stream 8's queued frames are cancelled
  CHECK(ex.live_bytes == 0 && ex.allocs == ex.releases);
  printf("close_and_destroy ok\n");
}

static void test_failures() {
  FakeExecutor ex;
  ex.fail_launch_every = 3;
  ex.fail_query_every = 4;
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  cfg.max_batch = 2;
  Scheduler s(&ex, cfg);
  for (uint32_t f = 1; f <= 10; ++f)
    for (uint64_t sid = 1; sid <= 3; ++sid) submit(s, sid, 8, 8, f);
  auto got = drain(s, 30);
  CHECK(got.size() == 30);
  int failed = 0;
  for (auto& c : got)
    if (c.status == CLOUD_E_HIP) failed++;
  CHECK(failed > 0 && failed < 30);
  // after a failed batch the stream's next frame restarts its history
  std::map<uint64_t, bool> last_failed;
  std::map<uint64_t, int> status_by_id;
  for (auto& c : got) status_by_id[c.request_id] = c.status;
  for (auto& batch : ex.history)
    for (auto& it : batch) {
      if (last_failed.count(it.stream_id) && last_failed[it.stream_id]) CHECK(it.reset_history);
      last_failed[it.stream_id] = status_by_id[it.request_id] != 0;
    }
  CHECK(s.stats().failed == (uint64_t)failed);
  printf("failures ok (%d failed)\n", failed);
}

static void test_concurrent_clients() {
  FakeExecutor ex;
  ex.delay_polls = 2;
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  cfg.max_queue = 64;
  Scheduler s(&ex, cfg);
  std::atomic<int> submitted{0};
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t)
    th.emplace_back([&, t] {
      for (int i = 0; i < 200; ++i) {
        int rc = CLOUD_E_BUSY;
        while (rc == CLOUD_E_BUSY) {
          submit(s, 100 + t * 3 + i % 3, 8, 8, i, &rc);
          if (rc == CLOUD_E_BUSY) std::this_thread::yield();
        }
        CHECK(rc == 0);
        submitted++;
      }
    });
  std::vector<Completion> got;
  std::thread poller([&] {
    while (got.size() < 800) {
      Completion c[32];
      int n = 0;
      s.poll(c, 32, &n);
      got.insert(got.end(), c, c + n);
      if (!n) s.wait(1000000);
    }
  });
  for (auto& t : th) t.join();
  poller.join();
  CHECK(submitted == 800 && got.size() == 800);
  std::set<uint64_t> ids;
  for (auto& c : got) {
    CHECK(c.status == 0);
    CHECK(ids.insert(c.request_id).second);
  }
  printf("concurrent_clients ok\n");
}

// Pipelined streams on an in-order device: up to two requests of a stream in
// flight, in consecutive batches, each resolving against the history of the
// one before it (no reset after a stream's first request) and naming that
// one's output buffer.
static void test_pipeline() {
  FakeExecutor ex;
  ex.base_ns = 2000000;
  ex.batch_ns = 200000;
  ex.max_per_stream = 2;
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  cfg.pipeline = 2;
  static char bufs[4][8];
  {
    Scheduler s(&ex, cfg);
    std::map<uint64_t, std::vector<uint64_t>> ids;
    for (uint32_t f = 0; f < 8; ++f)
      for (uint64_t sid = 1; sid <= 4; ++sid)
        ids[sid].push_back(submit_out(s, sid, 8, 8, f + 1, &bufs[sid - 1][f]));
    auto got = drain(s, 32);
    CHECK(got.size() == 32);
    std::map<uint64_t, std::vector<uint64_t>> seen;
    for (auto& c : got) {
      CHECK(c.status == 0);
      seen[c.stream_id].push_back(c.request_id);
    }
    CHECK(seen == ids);
    std::map<uint64_t, void*> last_out;
    for (auto& batch : ex.history)
      for (auto& it : batch) {
        const bool first = !last_out.count(it.stream_id);
        CHECK(it.reset_history == first);
        CHECK(it.prev_out == (first ? nullptr : last_out[it.stream_id]));
        last_out[it.stream_id] = it.out;
      }
    CHECK(ex.peak_per_stream == 2);
  }
  CHECK(ex.live_bytes == 0 && ex.allocs == ex.releases);
  printf("pipeline ok\n");
}

// A failed request fails the requests of its stream already in flight behind
// it that resolve against its history; the stream's next admitted request
// starts a fresh history.
static void test_pipeline_failure() {
  FakeExecutor ex;
  ex.delay_polls = 2;
  ex.max_per_stream = 2;
  ex.fail_query_every = 3;
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  cfg.pipeline = 2;
  Scheduler s(&ex, cfg);
  for (uint32_t f = 1; f <= 12; ++f)
    for (uint64_t sid = 1; sid <= 3; ++sid) submit(s, sid, 8, 8, f);
  auto got = drain(s, 36);
  CHECK(got.size() == 36);
  std::map<uint64_t, int> status_by_id;
  int failed = 0;
  for (auto& c : got) {
    status_by_id[c.request_id] = c.status;
    if (c.status) failed++;
  }
  std::map<uint64_t, int> prev;   // status of the stream's previous request
  int reset_after_failure = 0;
  for (auto& batch : ex.history)
    for (auto& it : batch) {
      const int st = status_by_id[it.request_id];
      if (prev.count(it.stream_id) && prev[it.stream_id] != 0) {
        if (it.reset_history) reset_after_failure++;
        else CHECK(st != 0);
      }
      prev[it.stream_id] = st;
    }
  CHECK(failed > 0 && failed < 36 && reset_after_failure > 0);
  CHECK(s.stats().failed == (uint64_t)failed);
  printf("pipeline_failure ok (%d failed)\n", failed);
}

// Closed-loop streams with `window` requests each in flight on a timed
// in-order device; mean requests per batch after the first few batches.
static double closed_loop_batch(int64_t lead_ns, int window) {
  FakeExecutor ex;
  ex.base_ns = 3000000;
  ex.batch_ns = 400000;
  ex.max_per_stream = window;
  Config cfg;
  cfg.budget_bytes = 1 << 30;
  cfg.pipeline = window;
  cfg.lead_ns = lead_ns;
  const int n = 8, frames = 14;
  std::vector<Completion> got;
  {
    Scheduler s(&ex, cfg);
    std::map<uint64_t, uint32_t> sent;
    for (uint64_t sid = 0; sid < (uint64_t)n; ++sid)
      for (int w = 0; w < window; ++w) submit(s, sid, 8, 8, ++sent[sid]);
    auto t0 = std::chrono::steady_clock::now();
    while ((int)got.size() < n * frames) {
      Completion c[64];
      int k = 0;
      s.poll(c, 64, &k);
      for (int i = 0; i < k; ++i) {
        CHECK(c[i].status == 0);
        got.push_back(c[i]);
        if (sent[c[i].stream_id] < (uint32_t)frames) submit(s, c[i].stream_id, 8, 8, ++sent[c[i].stream_id]);
      }
      if (!k) s.wait(2000000);
      CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(20));
    }
  }
  std::lock_guard<std::mutex> lk(ex.mu);
  size_t items = 0, batches = 0;
  for (size_t b = 4; b + 1 < ex.history.size(); ++b, ++batches) items += ex.history[b].size();
  CHECK(batches > 0);
  return (double)items / batches;
}

static void test_start_lead() {
  // one request a stream in flight: the streams split into two groups that
  // take turns, and with the lead each batch holds a whole group
  const double eager1 = closed_loop_batch(-1, 1), lead1 = closed_loop_batch(500000, 1);
  // two in flight: with the lead every batch holds every stream
  const double eager2 = closed_loop_batch(-1, 2), lead2 = closed_loop_batch(500000, 2);
  printf("start_lead: requests a batch, at once / with the lead: window 1 %.2f / %.2f, "
         "window 2 %.2f / %.2f\n", eager1, lead1, eager2, lead2);
  // (exactly 4 and 8 when the client's resubmissions are prompt; margins
  // for a loaded machine under the sanitizers)
  CHECK(lead1 >= 3.2);
  CHECK(lead2 >= 6.5);
  printf("start_lead ok\n");
}

int main() {
  test_order_and_reset();
  test_budget_admission();
  test_queue_full_and_mismatch();
  test_close_and_destroy_cancel();
  test_failures();
  test_concurrent_clients();
  test_pipeline();
  test_pipeline_failure();
  test_start_lead();
  printf("ALL OK\n");
  return 0;
}

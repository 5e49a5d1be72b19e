// Continuous-batching scheduler (see serve_core.h).
#include "serve_core.h"

#include <time.h>

#include <algorithm>
#include <chrono>
#include <set>

#include "../../include/cloud.h"

namespace cloud {
namespace serve {

int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

// Timed waits use the system clock: libstdc++ maps steady-clock waits to
// pthread_cond_clockwait, which some thread sanitizers do not model; the
// waits are short wake-up periods, so a wall-clock step only shifts one.
static std::chrono::system_clock::time_point deadline(int64_t ns) {
  return std::chrono::system_clock::now() + std::chrono::nanoseconds(ns);
}

Scheduler::Scheduler(Executor* ex, const Config& cfg) : ex_(ex), cfg_(cfg) {
  cfg_.pipeline = std::min(std::max(cfg_.pipeline, 1), std::max(cfg_.depth, 1));
  for (int s = cfg_.depth - 1; s >= 0; --s) free_slots_.push_back(s);
  thread_ = std::thread([this] { loop(); });
}

Scheduler::~Scheduler() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    running_ = false;
    const int64_t t = now_ns();
    for (const Pending& p : pending_) {
      completions_.push_back({p.id, p.stream_id, CLOUD_E_CANCELLED, p.t_submit, 0, 0, t});
      st_.cancelled++;
    }
    st_.queued = 0;
    pending_.clear();
  }
  cv_.notify_all();
  done_cv_.notify_all();
  if (thread_.joinable()) thread_.join();
  std::lock_guard<std::mutex> lk(mu_);
  for (auto& kv : streams_)
    if (kv.second.mem) ex_->release(kv.second.mem);
  streams_.clear();
  st_.bytes_in_use = 0;
}

int Scheduler::submit(uint64_t stream_id, int width, int height, uint32_t frame, void* out,
                      std::vector<unsigned char> payload, uint64_t* request_id,
                      std::string* msg) {
  const int64_t t = now_ns();
  std::lock_guard<std::mutex> lk(mu_);
  if (!running_) {
    *msg = "server is shutting down";
    return CLOUD_E_INVALID;
  }
  if ((int)pending_.size() >= cfg_.max_queue) {
    st_.rejected++;
    *msg = "request queue is full";
    return CLOUD_E_BUSY;
  }
  const size_t need = ex_->stream_bytes(width, height);
  if (need > cfg_.budget_bytes) {
    st_.rejected++;
    *msg = "a stream of this size can never fit the memory budget";
    return CLOUD_E_NOMEM;
  }
  auto it = streams_.find(stream_id);
  if (it == streams_.end()) {
    Stream s;
    s.width = width;
    s.height = height;
    streams_.emplace(stream_id, s);
    st_.streams++;
  } else {
    if (it->second.closing) {
      *msg = "stream is being closed";
      return CLOUD_E_INVALID;
    }
    if (it->second.width != width || it->second.height != height) {
      *msg = "stream resolution differs from its first request";
      return CLOUD_E_INVALID;
    }
  }
  const uint64_t id = next_id_++;
  pending_.push_back({id, stream_id, width, height, frame, out, std::move(payload), t});
  st_.queued++;
  *request_id = id;
  cv_.notify_one();
  return CLOUD_OK;
}

void Scheduler::admit_locked(std::vector<Item>& items, std::vector<int64_t>& ts,
                             std::vector<int64_t>& ta) {
  std::set<uint64_t> taken;
  std::deque<Pending> keep;
  const int64_t t = now_ns();
  while (!pending_.empty()) {
    Pending p = std::move(pending_.front());
    pending_.pop_front();
    if ((int)items.size() >= cfg_.max_batch) {
      keep.push_back(std::move(p));
      continue;
    }
    Stream& s = streams_[p.stream_id];
    // a stream keeps its order: one request a batch, and no more in flight
    // than the pipeline depth
    if (s.inflight >= cfg_.pipeline || taken.count(p.stream_id)) {
      keep.push_back(std::move(p));
      continue;
    }
    if (!s.mem) {
      const size_t need = ex_->stream_bytes(p.width, p.height);
      if (st_.bytes_in_use + need > cfg_.budget_bytes) {
        taken.insert(p.stream_id);   // later requests of this stream wait too
        keep.push_back(std::move(p));
        continue;
      }
      void* mem = nullptr;
      if (ex_->alloc(need, &mem) != 0 || !mem) {
        completions_.push_back({p.id, p.stream_id, CLOUD_E_NOMEM, p.t_submit, t, 0, now_ns()});
        st_.failed++;
        st_.queued--;
        taken.insert(p.stream_id);
        continue;
      }
      s.mem = mem;
      s.bytes = need;
      st_.bytes_in_use += need;
    }
    Item it;
    it.request_id = p.id;
    it.stream_id = p.stream_id;
    it.width = p.width;
    it.height = p.height;
    it.frame = p.frame;
    it.seq = s.admitted++;
    // with a request of the stream in flight, this one resolves against the
    // history that request writes, unless that request is known to fail
    it.reset_history = p.frame == 0 || (s.inflight == 0 ? !s.history_valid : s.tail_doomed);
    it.out = p.out;
    it.prev_out = s.last_out;
    it.stream_mem = s.mem;
    it.payload = std::move(p.payload);
    items.push_back(std::move(it));
    ts.push_back(p.t_submit);
    ta.push_back(t);
    s.inflight++;
    s.last_out = p.out;
    s.tail_doomed = false;
    taken.insert(p.stream_id);
    st_.admitted++;
    st_.queued--;
  }
  pending_.swap(keep);
}

void Scheduler::finish_locked(Batch& b, int status) {
  const int64_t t = now_ns();
  for (size_t i = 0; i < b.items.size(); ++i) {
    const Item& it = b.items[i];
    // a request that resolved against history a failed request did not
    // write fails too
    const int st = status == 0 && b.doomed[i] ? CLOUD_E_HIP : status;
    completions_.push_back({it.request_id, it.stream_id, st, b.t_submit[i], b.t_admit[i],
                            b.t_start, t});
    if (st == 0) st_.completed++;
    else st_.failed++;
    st_.running--;
    auto sit = streams_.find(it.stream_id);
    if (st != 0) {
      // the stream's later requests in flight, in launch order; each one
      // that did not start a fresh history reads this one's
      bool tail = false;
      for (Batch& o : inflight_) {
        if (&o == &b) continue;
        for (size_t j = 0; j < o.items.size(); ++j) {
          if (o.items[j].stream_id != it.stream_id) continue;
          if (!o.items[j].reset_history) o.doomed[j] = 1;
          tail = o.doomed[j] != 0;
        }
      }
      if (sit != streams_.end() && tail) sit->second.tail_doomed = true;
    }
    if (sit == streams_.end()) continue;
    Stream& s = sit->second;
    s.inflight--;
    s.history_valid = st == 0;
    if (s.closing && s.inflight == 0) free_stream_locked(it.stream_id);
  }
  done_cv_.notify_all();
}

void Scheduler::free_stream_locked(uint64_t id) {
  auto it = streams_.find(id);
  if (it == streams_.end()) return;
  if (it->second.mem) {
    ex_->release(it->second.mem);
    st_.bytes_in_use -= it->second.bytes;
  }
  streams_.erase(it);
  st_.streams--;
}

void Scheduler::loop() {
  ex_->thread_init();
  std::unique_lock<std::mutex> lk(mu_);
  for (;;) {
    // retire every finished batch (slots may finish out of order)
    bool retired = false;
    for (auto it = inflight_.begin(); it != inflight_.end();) {
      const int q = it->launch_rc ? 1 : ex_->query(it->slot);
      if (q == 0) {
        ++it;
        continue;
      }
      const int status = it->launch_rc ? it->launch_rc : (q < 0 ? q : 0);
      const int64_t t = now_ns();
      if (status == 0 && it->cost > 0.0) {
        // device time: from the later of its launch and the previous
        // batch's end to the moment it was seen finished
        const int64_t dur = t - std::max(it->t_start, last_done_);
        if (dur > 0) {
          const double r = (double)dur / it->cost;
          ns_per_cost_ = ns_per_cost_ > 0.0 ? 0.75 * ns_per_cost_ + 0.25 * r : r;
        }
      }
      last_done_ = t;
      retired = true;
      finish_locked(*it, status);
      free_slots_.push_back(it->slot);
      it = inflight_.erase(it);
    }
    if (retired) {
      // the next batch in flight started when the last one ended (or at its
      // launch, if later), and each after it when the one before ends
      int64_t begin = last_done_;
      for (Batch& b : inflight_) {
        b.est_begin = std::max(b.t_start, begin);
        b.est_end = b.est_begin + (int64_t)(b.cost * ns_per_cost_);
        begin = b.est_end;
      }
    }
    if (!running_ && inflight_.empty()) break;
    // start a batch when a slot is free, something is admissible, and the
    // work ahead of it is about to end
    if (running_ && !free_slots_.empty() && !pending_.empty() && start_now_locked(now_ns())) {
      Batch b;
      admit_locked(b.items, b.t_submit, b.t_admit);
      if (!b.items.empty()) {
        b.slot = free_slots_.back();
        free_slots_.pop_back();
        b.t_start = now_ns();
        b.doomed.assign(b.items.size(), 0);
        b.cost = 0.0;
        for (const Item& x : b.items) b.cost += ex_->cost(x);
        b.est_begin = inflight_.empty() ? b.t_start : std::max(b.t_start, inflight_.back().est_end);
        b.est_end = b.est_begin + (int64_t)(b.cost * ns_per_cost_);
        b.launch_rc = ex_->launch(b.slot, b.items);
        st_.batches++;
        st_.running += b.items.size();
        inflight_.push_back(std::move(b));
        continue;
      }
    }
    if (inflight_.empty())
      cv_.wait(lk);
    else
      cv_.wait_until(lk, deadline(cfg_.poll_us * 1000LL));
  }
}

// With a batch in flight, the next one starts once the work ahead of it is
// expected to end within the lead, or once a full batch is queued; with
// nothing in flight, with no lead, or before any batch has been timed, at
// once.
bool Scheduler::start_now_locked(int64_t now) {
  if (inflight_.empty() || cfg_.lead_ns < 0 || !(ns_per_cost_ > 0.0)) return true;
  if ((int)pending_.size() >= cfg_.max_batch) return true;
  const int64_t ahead_end = inflight_.back().est_end;
  const int64_t lead = cfg_.lead_ns + (ahead_end - inflight_.front().est_begin) / 8;
  return now >= ahead_end - lead;
}

int Scheduler::poll(Completion* out, int max, int* n) {
  std::lock_guard<std::mutex> lk(mu_);
  const int k = std::min<int>(std::max(max, 0), (int)completions_.size());
  std::copy(completions_.begin(), completions_.begin() + k, out);
  completions_.erase(completions_.begin(), completions_.begin() + k);
  *n = k;
  return CLOUD_OK;
}

int Scheduler::wait(int64_t timeout_ns) {
  std::unique_lock<std::mutex> lk(mu_);
  done_cv_.wait_until(lk, deadline(std::max<int64_t>(timeout_ns, 0)),
                      [this] { return !completions_.empty() || !running_; });
  return completions_.empty() ? 0 : 1;
}

Stats Scheduler::stats() {
  std::lock_guard<std::mutex> lk(mu_);
  return st_;
}

int Scheduler::close_stream(uint64_t stream_id) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = streams_.find(stream_id);
  if (it == streams_.end()) return CLOUD_E_NOTFOUND;
  const int64_t t = now_ns();
  std::deque<Pending> keep;
  for (Pending& p : pending_) {
    if (p.stream_id == stream_id) {
      completions_.push_back({p.id, p.stream_id, CLOUD_E_CANCELLED, p.t_submit, 0, 0, t});
      st_.cancelled++;
      st_.queued--;
    } else {
      keep.push_back(std::move(p));
    }
  }
  pending_.swap(keep);
  it->second.closing = true;
  if (it->second.inflight == 0) free_stream_locked(stream_id);
  done_cv_.notify_all();
  cv_.notify_one();
  return CLOUD_OK;
}

}  // namespace serve
}  // namespace cloud

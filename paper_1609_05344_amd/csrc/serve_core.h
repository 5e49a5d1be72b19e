// Continuous-batching scheduler for render requests from many camera streams.
//
// Pure C++ (no HIP): the device side is behind the Executor interface, so the
// scheduling logic -- bounded queue, per-stream ordering, admission against a
// device-memory budget, batching, completion records and timestamps,
// cancellation -- is the same code in the library and in the CPU test build.
//
// Model. A request renders one frame of one stream and resolves it against
// that stream's history (the temporal accumulation of jittered frames). A
// stream's frames depend on each other through the history, so they run in
// submission order, at most one per batch; requests of different streams are
// independent and are batched together. Up to `depth` batches are in flight
// at once. When the executor runs batches in launch order, a stream may have
// up to `pipeline` requests in flight, in consecutive batches (each batch's
// resolve then finishes before the next one reads that history); otherwise
// one. A stream's state is allocated when its first request is admitted,
// counted against the budget, and freed when the stream is closed.
//
// Batch start. With nothing in flight a batch starts at once. With a batch
// in flight, the next one would only wait behind it on the device, so it
// keeps admitting arrivals until the work ahead of it is expected to end
// within the start lead (lead_ns plus an eighth of that work), or until it
// has a full batch's worth of requests queued. The expected end comes from
// the executor's cost of each request and a running average of device time
// per unit cost over finished batches.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace cloud {
namespace serve {

int64_t now_ns();   // steady clock (CLOCK_MONOTONIC), nanoseconds

struct Completion {
  uint64_t request_id, stream_id;
  int32_t status;           // 0 OK, or a negative CLOUD_E_* code
  int64_t t_submit, t_admit, t_start, t_done;
};

struct Stats {
  uint64_t queued, admitted, running, completed, rejected, cancelled, failed;
  uint64_t streams, bytes_in_use, batches;
};

// One admitted request, as handed to the executor.
struct Item {
  uint64_t request_id, stream_id;
  int width, height;
  uint32_t frame;
  uint64_t seq;             // the stream's requests admitted before this one
  bool reset_history;       // frame 0, or no valid history yet
  void* out;                // caller's output buffer
  void* prev_out;           // output buffer of the stream's previous request (or null)
  void* stream_mem;         // the stream's state allocation
  std::vector<unsigned char> payload;   // executor-specific request data
};

class Executor {
 public:
  virtual ~Executor() {}
  // Bytes of per-stream state for a width x height stream.
  virtual size_t stream_bytes(int width, int height) = 0;
  virtual int alloc(size_t bytes, void** mem) = 0;
  virtual void release(void* mem) = 0;
  // Enqueue a batch on slot (0 <= slot < depth); returns at once.
  virtual int launch(int slot, const std::vector<Item>& items) = 0;
  // 1 when the slot's batch has finished, 0 while it runs, <0 on failure.
  virtual int query(int slot) = 0;
  // Called on the scheduler thread before anything else.
  virtual void thread_init() {}
  // Relative device cost of a request (any unit, the same for all requests).
  virtual double cost(const Item& it) { return (double)it.width * it.height; }
};

struct Config {
  uint64_t budget_bytes = 0;   // device memory for stream state
  int max_batch = 64;          // requests per batch
  int max_queue = 1024;        // queued (not yet admitted) requests
  int depth = 2;               // batches in flight
  int pipeline = 1;            // requests of one stream in flight (> 1: batches run in order)
  int64_t lead_ns = -1;        // batch start lead; < 0: start as soon as a slot is free
  int poll_us = 20;            // scheduler wake-up period while batches run
};

class Scheduler {
 public:
  Scheduler(Executor* ex, const Config& cfg);
  ~Scheduler();   // cancels queued requests, waits for in-flight batches

  // Thread-safe. Returns 0 and the request id, CLOUD_E_BUSY when the queue
  // is full, CLOUD_E_NOMEM when the stream could never fit the budget,
  // CLOUD_E_INVALID for a stream whose size differs from its first request
  // or that is being closed.
  int submit(uint64_t stream_id, int width, int height, uint32_t frame, void* out,
             std::vector<unsigned char> payload, uint64_t* request_id, std::string* msg);
  int poll(Completion* out, int max, int* n);            // thread-safe, non-blocking
  int wait(int64_t timeout_ns);                          // until >= 1 completion or timeout
  Stats stats();
  int close_stream(uint64_t stream_id);

 private:
  struct Stream {
    int width = 0, height = 0;
    void* mem = nullptr;
    size_t bytes = 0;
    int inflight = 0;           // requests in flight
    uint64_t admitted = 0;      // requests admitted so far
    bool closing = false, history_valid = false;
    bool tail_doomed = false;   // the last admitted request will fail (its history is bad)
    void* last_out = nullptr;   // output buffer of the last admitted request
  };
  struct Pending {
    uint64_t id, stream_id;
    int width, height;
    uint32_t frame;
    void* out;
    std::vector<unsigned char> payload;
    int64_t t_submit;
  };
  struct Batch {
    int slot;
    std::vector<Item> items;
    std::vector<int64_t> t_submit, t_admit;
    std::vector<char> doomed;   // item reads history that a failed request did not write
    int64_t t_start;
    int launch_rc;
    double cost;
    int64_t est_begin, est_end;  // expected device start and end
  };

  void loop();
  bool start_now_locked(int64_t now);
  void admit_locked(std::vector<Item>& items, std::vector<int64_t>& ts, std::vector<int64_t>& ta);
  void finish_locked(Batch& b, int status);
  void free_stream_locked(uint64_t id);

  Executor* ex_;
  Config cfg_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<Pending> pending_;
  std::map<uint64_t, Stream> streams_;
  std::deque<Batch> inflight_;
  std::vector<Completion> completions_;
  std::vector<int> free_slots_;
  Stats st_{};
  uint64_t next_id_ = 1;
  bool running_ = true;
  double ns_per_cost_ = 0.0;     // running average of device time per unit cost (0: none yet)
  int64_t last_done_ = 0;        // when the last batch was seen finished
  std::thread thread_;
};

}  // namespace serve
}  // namespace cloud

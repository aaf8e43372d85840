// agent.h -- host side of the query-grained record transport (FlashANNS
// section 4.2): each query owns a request slot that its GPU wave writes and a
// completion word that a host agent thread writes; no query ever waits for
// another query's reads.
//
// Plain C++ (no HIP): the memory it works on is handed in by the caller, so
// the protocol can be exercised on the CPU with a thread standing in for the
// GPU.
#pragma once
#include <stdint.h>

#include <atomic>
#include <thread>
#include <vector>

namespace fa {

// One query's request slots, written by its GPU wave: with P slots in use,
// request s is the 64-bit word slot[s % P] = (node << 32) | s, stored in one
// piece, so the agent never sees a sequence number without its node.  At most
// P requests of a query are outstanding (P >= the nodes in flight of the
// schedule: 2 for strict and one-step-stale search, (delay + 1) * W in
// general) and they are consumed in order, so a wave reuses a slot only after
// consuming the request that held it.  One 64 B line per query, so that no
// two queries (and no GPU wave and agent thread pair) share a cache line.
constexpr int kMaxSlots = 8;

// Request numbers run 1, 2, ..., M, 1, 2, ... with M the largest multiple of
// the slot count below 2^30 (0 means "no request"; bit 31 of a completion word
// is the error flag; s % slots stays continuous across the wrap).  The GPU
// side steps through the same sequence.
inline uint32_t next_seq(uint32_t s, int slots) {
  const uint32_t M = (0x40000000u / (uint32_t)slots) * (uint32_t)slots;
  return s >= M ? 1u : s + 1u;
}
struct alignas(64) AgentRequest {
  uint64_t slot[kMaxSlots];
};

// Completion words of query q: cpl[kCplStride * q + (s % P)], one 64 B line
// per query.
constexpr int kCplStride = 16;

// Completion words: P per query, cpl[kCplStride q + (s % P)] = s when
// request s has been staged, s | kCplError when its read failed.  One word
// per in-flight slot keeps each request's status until its wave has
// consumed it.  A query's requests may complete out of order (reads of a
// file finish in any order); each has its own word and staging slot.
constexpr uint32_t kCplError = 0x80000000u;

// Records striped over several files (one per storage device): record v is
// record v / stripes of file v % stripes (paper section 5: several SSDs).
constexpr int kMaxStripes = 16;

// Fault injection for tests (host-forced conditions only).
struct AgentFaults {
  int32_t delay_node = -1;   // requests for this node complete after delay_us
  int32_t delay_us = 0;
  int32_t fail_node = -1;    // requests for this node complete with kCplError
  int32_t drop_node = -1;    // requests for this node never complete
};

// Counters (cumulative; relaxed atomics, read while serving).
struct AgentStats {
  std::atomic<uint64_t> requests{0};
  std::atomic<uint64_t> bytes{0};
  std::atomic<uint64_t> errors{0};
  std::atomic<int> last_errno{0};
  // where the agent threads' time goes
  std::atomic<uint64_t> passes{0};       // scans of a thread's query range
  std::atomic<uint64_t> busy_passes{0};  // scans that found or finished work
  std::atomic<uint64_t> scan_ns{0};      // reading request lines
  std::atomic<uint64_t> copy_ns{0};      // record copies into staging + completions
  std::atomic<uint64_t> io_ns{0};        // file reads: submitting and reaping
  std::atomic<uint64_t> max_batch{0};    // most requests found by one scan
  std::atomic<uint64_t> stripe_requests[kMaxStripes] = {};
};

class Agent {
 public:
  // Record source: `mem` (slot-strided records in host memory) or `nstripes`
  // files `fds` of slot-strided records (`direct` if opened with O_DIRECT;
  // record v at offset (v / nstripes) * slot of file v % nstripes).  Each
  // request copies `copy_bytes` (the useful record prefix); file reads are
  // `io_bytes` long (copy_bytes rounded up to the device block).  With
  // direct I/O, each thread keeps up to `aio_depth` reads in flight through
  // Linux asynchronous I/O; otherwise reads are synchronous.
  Agent(const uint8_t *mem, const int *fds, int nstripes, bool direct, int64_t slot,
        int32_t copy_bytes, int32_t io_bytes, int threads, int aio_depth = 64);
  ~Agent();

  // Serve the requests of `nq` queries until disarm().  `cpl` holds
  // kCplStride x nq completion words and `stage` `slots` staging slots of
  // `stage_stride` bytes per query (slot s % slots for request s, slots in
  // [1, kMaxSlots]).  The caller zeroes req/cpl.
  // `start_seq` is the request number each line has already used (0 for
  // fresh lines).
  void arm(AgentRequest *req, uint32_t *cpl, uint8_t *stage, int64_t nq, int64_t stage_stride,
           int slots, uint32_t start_seq = 0);
  // Stop serving; returns once no agent thread touches the arrays any more
  // and no read of the agent is in flight.
  void disarm();

  AgentFaults faults;  // set while disarmed
  AgentStats stats;
  int threads() const { return (int)workers_.size(); }
  bool async_io() const { return aio_depth_ > 0; }

 private:
  struct Work {
    int64_t q;
    uint32_t seq, node;
  };
  struct Io;  // one thread's asynchronous-read state
  // One thread's counts, added to `stats` once per pass: a locked add per
  // request on lines shared by all threads (and, after non-temporal stores,
  // a drain of the write-combining buffers) would cost more than the copy.
  struct Tally {
    uint64_t requests = 0, errors = 0, stripe[kMaxStripes] = {};
    uint64_t passes = 0, busy_passes = 0, scan_ns = 0, copy_ns = 0, io_ns = 0, max_batch = 0;
  };
  void run(int t);
  int scan(int64_t q0, int64_t q1, std::vector<Work> &out);
  void serve_memory(std::vector<Work> &work, Tally &tally);
  bool serve_file_sync(const Work &w, uint8_t *bounce, Tally &tally);
  void complete(const Work &w, bool ok, const uint8_t *src, Tally &tally);
  void pump_file(Io &io, std::vector<Work> &work, bool wait, Tally &tally);
  void flush(Tally &tally);

  const uint8_t *mem_;
  std::vector<int> fds_;
  bool direct_;
  int64_t slot_;
  int32_t copy_bytes_, io_bytes_;
  int aio_depth_ = 0;

  int nthreads_ = 1;
  std::vector<std::thread> workers_;
  std::atomic<bool> quit_{false};
  std::atomic<bool> armed_{false};
  std::atomic<int> busy_{0};            // workers inside a serving pass
  AgentRequest *req_ = nullptr;
  uint32_t *cpl_ = nullptr;
  uint8_t *stage_ = nullptr;
  int64_t nq_ = 0, stage_stride_ = 0;
  int slots_ = 2;
  std::vector<uint32_t> done_;          // per query: last request taken
};

}  // namespace fa

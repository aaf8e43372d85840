// agent.cpp -- host agent threads of the query-grained record transport.
//
// Query q is served by exactly one thread (static ranges), so a query's
// requests complete in order and never wait behind another query's
// (paper section 4.2: no kernel-wide barrier, a straggling read delays only
// the query that issued it).
#include "agent.h"

#include <unistd.h>

#include <cerrno>
#include <chrono>
#include <cstdlib>
#include <cstring>

namespace fa {

namespace {
inline void cpu_relax() { __builtin_ia32_pause(); }
}  // namespace

Agent::Agent(const uint8_t *mem, int fd, bool direct, int64_t slot, int32_t copy_bytes,
             int32_t io_bytes, int threads)
    : mem_(mem), fd_(fd), direct_(direct), slot_(slot), copy_bytes_(copy_bytes),
      io_bytes_(io_bytes) {
  if (threads < 1) threads = 1;
  nthreads_ = threads;
  for (int t = 0; t < threads; t++) workers_.emplace_back([this, t] { run(t); });
}

Agent::~Agent() {
  disarm();
  quit_.store(true);
  for (auto &w : workers_) w.join();
}

void Agent::arm(AgentRequest *req, uint32_t *cpl, uint8_t *stage, int64_t nq,
                int64_t stage_stride, int slots, uint32_t start_seq) {
  slots_ = slots < 1 ? 1 : (slots > kMaxSlots ? kMaxSlots : slots);
  req_ = req;
  cpl_ = cpl;
  stage_ = stage;
  nq_ = nq;
  stage_stride_ = stage_stride;
  done_.assign((size_t)nq, start_seq);
  armed_.store(true);  // seq_cst: publishes the fields above
}

void Agent::disarm() {
  armed_.store(false);
  while (busy_.load() != 0) cpu_relax();
}

// `bounce` (direct I/O only): a block-aligned private buffer; O_DIRECT reads
// cannot target the driver-mapped pinned staging memory, so they land here
// and are copied into the staging slot.
bool Agent::serve(int64_t q, uint32_t seq, uint32_t node, uint8_t *bounce) {
  if ((int32_t)node == faults.drop_node) return false;  // never completes
  if ((int32_t)node == faults.delay_node && faults.delay_us > 0)
    std::this_thread::sleep_for(std::chrono::microseconds(faults.delay_us));
  const uint32_t sl = seq % (uint32_t)slots_;
  uint8_t *dst = stage_ + (q * slots_ + sl) * stage_stride_;
  bool ok = true;
  if (mem_) {
    std::memcpy(dst, mem_ + (int64_t)node * slot_, (size_t)copy_bytes_);
  } else {
    uint8_t *buf = direct_ ? bounce : dst;
    const ssize_t r = pread(fd_, buf, (size_t)io_bytes_, (off_t)((int64_t)node * slot_));
    ok = r >= copy_bytes_;
    if (!ok) stats.last_errno.store(r < 0 ? errno : EIO, std::memory_order_relaxed);
    if (ok && direct_) std::memcpy(dst, bounce, (size_t)copy_bytes_);
  }
  if ((int32_t)node == faults.fail_node) ok = false;
  __atomic_store_n(&cpl_[q * kCplStride + sl], ok ? seq : (seq | kCplError), __ATOMIC_RELEASE);
  stats.requests.fetch_add(1, std::memory_order_relaxed);
  stats.bytes.fetch_add(mem_ ? (uint64_t)copy_bytes_ : (uint64_t)io_bytes_,
                        std::memory_order_relaxed);
  if (!ok) stats.errors.fetch_add(1, std::memory_order_relaxed);
  return true;
}

void Agent::run(int t) {
  uint8_t *bounce = nullptr;
  if (direct_ && posix_memalign((void **)&bounce, 4096, (size_t)io_bytes_ + 4096) != 0)
    bounce = nullptr;
  uint32_t idle = 0;
  while (!quit_.load(std::memory_order_relaxed)) {
    // Announce the pass before checking armed_: disarm() stores armed_ then
    // waits for busy_ to drain, so a pass either sees armed_ == false or is
    // waited for (all four accesses are sequentially consistent).
    busy_.fetch_add(1);
    if (!armed_.load()) {
      busy_.fetch_sub(1);
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      continue;
    }
    const int64_t q0 = nq_ * t / nthreads_, q1 = nq_ * (t + 1) / nthreads_;
    bool any = false;
    for (int64_t q = q0; q < q1; q++) {
      uint32_t d = done_[(size_t)q];
      for (;;) {
        const uint32_t nx = next_seq(d, slots_);
        const uint64_t w = __atomic_load_n(&req_[q].slot[nx % (uint32_t)slots_], __ATOMIC_ACQUIRE);
        if ((uint32_t)w != nx) break;
        d = nx;
        serve(q, d, (uint32_t)(w >> 32), bounce);
        any = true;
      }
      done_[(size_t)q] = d;
    }
    busy_.fetch_sub(1);
    // Idle passes spin briefly, then yield: file agents outnumber the cores,
    // and a spinning thread must not keep one with a read to issue waiting.
    if (any) {
      idle = 0;
    } else if (++idle < 64) {
      cpu_relax();
    } else {
      std::this_thread::yield();
    }
  }
  std::free(bounce);
}

}  // namespace fa

// agent.cpp -- host agent threads of the query-grained record transport.
//
// Query q is served by exactly one thread (static ranges), so no two threads
// touch one query's lines and no query waits behind another thread's queue
// (paper section 4.2: no kernel-wide barrier, a straggling read delays only
// the queries of the thread that serves it).
//
// One pass of a thread: scan its queries' request lines and collect every
// new request (the batch the paper's CPU agent gathers before issuing I/O),
// then serve the batch:
//   * records in host memory: copy each record into its staging slot with
//     non-temporal stores (the GPU reads the slot over the host link; a
//     cached copy would only be snooped back out), prefetching a few records
//     ahead so that their DRAM misses overlap, and publish completions after
//     a store fence, a small group at a time;
//   * records in files opened with O_DIRECT: submit the whole batch as Linux
//     asynchronous reads (io_submit) into per-read bounce buffers and keep
//     scanning; completed reads (io_getevents) are copied into their staging
//     slots and completed.  Up to aio_depth reads per thread are in flight.
//   * other files: synchronous pread per request.
#include "agent.h"

#include <emmintrin.h>
#include <linux/aio_abi.h>
#include <sys/syscall.h>
#include <time.h>
#include <unistd.h>

#include <cerrno>
#include <chrono>
#include <cstdlib>
#include <cstring>

namespace fa {

namespace {
inline void cpu_relax() { __builtin_ia32_pause(); }

inline uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

// Linux AIO system calls (no libaio in the image).
long sys_io_setup(unsigned nr, aio_context_t *ctx) { return syscall(__NR_io_setup, nr, ctx); }
long sys_io_destroy(aio_context_t ctx) { return syscall(__NR_io_destroy, ctx); }
long sys_io_submit(aio_context_t ctx, long nr, iocb **v) { return syscall(__NR_io_submit, ctx, nr, v); }
long sys_io_getevents(aio_context_t ctx, long min_nr, long max_nr, io_event *ev, timespec *t) {
  return syscall(__NR_io_getevents, ctx, min_nr, max_nr, ev, t);
}

// Copy n bytes (a multiple of 16, 16 B-aligned destination) with
// non-temporal stores.
inline void stream_copy(uint8_t *dst, const uint8_t *src, int32_t n) {
  for (int32_t i = 0; i < n; i += 16)
    _mm_stream_si128((__m128i *)(dst + i), _mm_loadu_si128((const __m128i *)(src + i)));
}

inline void prefetch_record(const uint8_t *p, int32_t n) {
  for (int32_t i = 0; i < n; i += 64) __builtin_prefetch(p + i, 0, 0);
}

void atomic_max(std::atomic<uint64_t> &a, uint64_t v) {
  uint64_t cur = a.load(std::memory_order_relaxed);
  while (v > cur && !a.compare_exchange_weak(cur, v, std::memory_order_relaxed)) {
  }
}

constexpr int kPrefetchAhead = 8;   // records whose DRAM misses overlap the current copy
constexpr int kCompleteGroup = 16;  // completions published per store fence
}  // namespace

// Asynchronous-read state of one thread: an AIO context, `depth` bounce
// buffers (block-aligned: O_DIRECT cannot read into the driver-mapped
// staging memory) and the work each one holds.
struct Agent::Io {
  aio_context_t ctx = 0;
  int depth = 0;
  uint8_t *bufs = nullptr;
  std::vector<iocb> cbs;
  std::vector<Work> held;      // per buffer
  std::vector<int> free_bufs;
  std::vector<iocb *> batch;
  std::vector<io_event> events;
  std::vector<Work> pending;   // taken but not yet submitted (no free buffer)
  int outstanding = 0;
};

Agent::Agent(const uint8_t *mem, const int *fds, int nstripes, bool direct, int64_t slot,
             int32_t copy_bytes, int32_t io_bytes, int threads, int aio_depth)
    : mem_(mem), direct_(direct), slot_(slot), copy_bytes_(copy_bytes), io_bytes_(io_bytes) {
  if (!mem_)
    for (int s = 0; s < nstripes && s < kMaxStripes; s++) fds_.push_back(fds[s]);
  if (fds_.empty()) fds_.push_back(-1);
  aio_depth_ = (!mem_ && direct_ && aio_depth > 0) ? aio_depth : 0;
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
  // a thread with reads in flight stays busy (it reaps them, without taking
  // new requests) until they have completed
  while (busy_.load() != 0) cpu_relax();
}

// New requests of queries [q0, q1), in query order and, per query, in
// request order.
int Agent::scan(int64_t q0, int64_t q1, std::vector<Work> &out) {
  const size_t before = out.size();
  for (int64_t q = q0; q < q1; q++) {
    uint32_t d = done_[(size_t)q];
    for (;;) {
      const uint32_t nx = next_seq(d, slots_);
      const uint64_t w = __atomic_load_n(&req_[q].slot[nx % (uint32_t)slots_], __ATOMIC_ACQUIRE);
      if ((uint32_t)w != nx) break;
      d = nx;
      out.push_back(Work{q, nx, (uint32_t)(w >> 32)});
    }
    done_[(size_t)q] = d;
  }
  return (int)(out.size() - before);
}

// Publish request w.  With `src` its record is copied into the staging slot
// first; otherwise the staged bytes are already written (and fenced, for
// non-temporal stores).
void Agent::complete(const Work &w, bool ok, const uint8_t *src, Tally &tally) {
  const uint32_t sl = w.seq % (uint32_t)slots_;
  if (src && ok) {
    stream_copy(stage_ + (w.q * slots_ + sl) * stage_stride_, src, copy_bytes_);
    _mm_sfence();
  }
  if ((int32_t)w.node == faults.fail_node) ok = false;
  __atomic_store_n(&cpl_[w.q * kCplStride + sl], ok ? w.seq : (w.seq | kCplError),
                   __ATOMIC_RELEASE);
  tally.requests++;
  tally.stripe[w.node % fds_.size()]++;
  if (!ok) tally.errors++;
}

void Agent::flush(Tally &tally) {
  const auto add = [](std::atomic<uint64_t> &a, uint64_t v) {
    if (v) a.fetch_add(v, std::memory_order_relaxed);
  };
  add(stats.requests, tally.requests);
  add(stats.bytes, tally.requests * (uint64_t)(mem_ ? copy_bytes_ : io_bytes_));
  add(stats.errors, tally.errors);
  for (size_t s = 0; s < fds_.size(); s++) add(stats.stripe_requests[s], tally.stripe[s]);
  add(stats.passes, tally.passes);
  add(stats.busy_passes, tally.busy_passes);
  add(stats.scan_ns, tally.scan_ns);
  add(stats.copy_ns, tally.copy_ns);
  add(stats.io_ns, tally.io_ns);
  if (tally.max_batch) atomic_max(stats.max_batch, tally.max_batch);
  tally = Tally{};
}

void Agent::serve_memory(std::vector<Work> &work, Tally &tally) {
  const int n = (int)work.size();
  for (int i = 0; i < n && i < kPrefetchAhead; i++)
    prefetch_record(mem_ + (int64_t)work[(size_t)i].node * slot_, copy_bytes_);
  int g0 = 0;  // first request of the group not yet completed
  for (int i = 0; i < n; i++) {
    if (i + kPrefetchAhead < n)
      prefetch_record(mem_ + (int64_t)work[(size_t)(i + kPrefetchAhead)].node * slot_, copy_bytes_);
    const Work &w = work[(size_t)i];
    if ((int32_t)w.node == faults.delay_node && faults.delay_us > 0)
      std::this_thread::sleep_for(std::chrono::microseconds(faults.delay_us));
    if ((int32_t)w.node != faults.drop_node)
      stream_copy(stage_ + (w.q * slots_ + w.seq % (uint32_t)slots_) * stage_stride_,
                  mem_ + (int64_t)w.node * slot_, copy_bytes_);
    if (i + 1 - g0 == kCompleteGroup || i + 1 == n) {
      _mm_sfence();  // the staged bytes are visible before their completions
      for (int j = g0; j <= i; j++)
        if ((int32_t)work[(size_t)j].node != faults.drop_node) complete(work[(size_t)j], true, nullptr, tally);
      g0 = i + 1;
    }
  }
}

// `bounce` (direct I/O only): a block-aligned private buffer.
bool Agent::serve_file_sync(const Work &w, uint8_t *bounce, Tally &tally) {
  if ((int32_t)w.node == faults.drop_node) return false;  // never completes
  if ((int32_t)w.node == faults.delay_node && faults.delay_us > 0)
    std::this_thread::sleep_for(std::chrono::microseconds(faults.delay_us));
  const int S = (int)fds_.size();
  const uint32_t sl = w.seq % (uint32_t)slots_;
  uint8_t *dst = stage_ + (w.q * slots_ + sl) * stage_stride_;
  uint8_t *buf = direct_ ? bounce : dst;
  const ssize_t r = pread(fds_[w.node % S], buf, (size_t)io_bytes_, (off_t)((int64_t)(w.node / S) * slot_));
  const bool ok = r >= copy_bytes_;
  if (!ok) stats.last_errno.store(r < 0 ? errno : EIO, std::memory_order_relaxed);
  complete(w, ok, direct_ && ok ? bounce : nullptr, tally);
  return true;
}

// Submit what `work` (and earlier overflow) holds while buffers are free,
// then reap completed reads; with `wait`, block briefly for at least one.
void Agent::pump_file(Io &io, std::vector<Work> &work, bool wait, Tally &tally) {
  for (const Work &w : work) io.pending.push_back(w);
  work.clear();
  const int S = (int)fds_.size();
  io.batch.clear();
  size_t taken = 0;
  while (taken < io.pending.size() && !io.free_bufs.empty()) {
    const Work w = io.pending[taken++];
    if ((int32_t)w.node == faults.drop_node) continue;  // never completes
    const int b = io.free_bufs.back();
    io.free_bufs.pop_back();
    io.held[(size_t)b] = w;
    iocb &cb = io.cbs[(size_t)b];
    std::memset(&cb, 0, sizeof(cb));
    cb.aio_data = (uint64_t)b;
    cb.aio_lio_opcode = IOCB_CMD_PREAD;
    cb.aio_fildes = (uint32_t)fds_[w.node % S];
    cb.aio_buf = (uint64_t)(uintptr_t)(io.bufs + (int64_t)b * io_bytes_);
    cb.aio_nbytes = (uint64_t)io_bytes_;
    cb.aio_offset = (int64_t)(w.node / S) * slot_;
    io.batch.push_back(&cb);
  }
  io.pending.erase(io.pending.begin(), io.pending.begin() + (long)taken);
  size_t sent = 0;
  while (sent < io.batch.size()) {
    const long r = sys_io_submit(io.ctx, (long)(io.batch.size() - sent), io.batch.data() + sent);
    if (r > 0) {
      sent += (size_t)r;
      io.outstanding += (int)r;
      continue;
    }
    if (r < 0 && errno == EAGAIN) {  // the queue is full: try again after reaping
      for (size_t i = sent; i < io.batch.size(); i++) {
        const int b = (int)io.batch[i]->aio_data;
        io.pending.insert(io.pending.begin(), io.held[(size_t)b]);
        io.free_bufs.push_back(b);
      }
      break;
    }
    // a submission error fails the requests it names
    const int b = (int)io.batch[sent]->aio_data;
    stats.last_errno.store(r < 0 ? errno : EIO, std::memory_order_relaxed);
    complete(io.held[(size_t)b], false, nullptr, tally);
    io.free_bufs.push_back(b);
    sent++;
  }
  if (io.outstanding == 0) return;
  timespec ts{0, wait ? 20000 : 0};  // 20 us
  const long got = sys_io_getevents(io.ctx, wait ? 1 : 0, (long)io.events.size(), io.events.data(), &ts);
  for (long i = 0; i < got; i++) {
    const io_event &ev = io.events[(size_t)i];
    const int b = (int)ev.data;
    const Work &w = io.held[(size_t)b];
    if ((int32_t)w.node == faults.delay_node && faults.delay_us > 0)
      std::this_thread::sleep_for(std::chrono::microseconds(faults.delay_us));
    const bool ok = ev.res >= (int64_t)copy_bytes_;
    if (!ok) stats.last_errno.store(ev.res < 0 ? (int)-ev.res : EIO, std::memory_order_relaxed);
    complete(w, ok, ok ? io.bufs + (int64_t)b * io_bytes_ : nullptr, tally);
    io.free_bufs.push_back(b);
    io.outstanding--;
  }
}

void Agent::run(int t) {
  uint8_t *bounce = nullptr;
  if (!mem_ && direct_ && posix_memalign((void **)&bounce, 4096, (size_t)io_bytes_ + 4096) != 0)
    bounce = nullptr;
  Io io;
  if (aio_depth_ > 0) {
    io.depth = aio_depth_;
    if (posix_memalign((void **)&io.bufs, 4096, (size_t)io_bytes_ * (size_t)io.depth) != 0) {
      io.bufs = nullptr;  // fall back to synchronous reads in this thread
    } else if (sys_io_setup((unsigned)io.depth, &io.ctx) != 0) {
      io.ctx = 0;  // likewise (e.g. the system's limit of AIO contexts is reached)
    } else {
      io.cbs.resize((size_t)io.depth);
      io.held.resize((size_t)io.depth);
      io.events.resize((size_t)io.depth);
      for (int b = io.depth - 1; b >= 0; b--) io.free_bufs.push_back(b);
    }
  }
  std::vector<Work> work;
  Tally tally;
  uint32_t idle = 0;
  while (!quit_.load(std::memory_order_relaxed)) {
    // Announce the pass before checking armed_: disarm() stores armed_ then
    // waits for busy_ to drain, so a pass either sees armed_ == false or is
    // waited for (all these accesses are sequentially consistent).
    busy_.fetch_add(1);
    const bool armed = armed_.load();
    const bool reads_out = io.ctx && (io.outstanding > 0 || !io.pending.empty());
    if (!armed && !reads_out) {
      if (tally.passes) flush(tally);
      busy_.fetch_sub(1);
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      continue;
    }
    bool any = false;
    work.clear();
    if (armed) {
      const int64_t q0 = nq_ * t / nthreads_, q1 = nq_ * (t + 1) / nthreads_;
      const uint64_t t0 = now_ns();
      const int found = scan(q0, q1, work);
      tally.scan_ns += now_ns() - t0;
      tally.passes++;
      if ((uint64_t)found > tally.max_batch) tally.max_batch = (uint64_t)found;
      any = found > 0;
    } else {
      // disarmed with reads in flight: their queries' requests are dropped
      // from the queue and the reads in flight are reaped
      io.pending.clear();
    }
    if (!work.empty() || reads_out) {
      const uint64_t t0 = now_ns();
      const uint64_t served = tally.requests;
      if (mem_) {
        serve_memory(work, tally);
        tally.copy_ns += now_ns() - t0;
      } else if (io.ctx) {
        pump_file(io, work, /*wait=*/!any || !armed, tally);
        any = any || tally.requests != served;
        tally.io_ns += now_ns() - t0;
      } else {
        for (const Work &w : work) serve_file_sync(w, bounce, tally);
        tally.io_ns += now_ns() - t0;
      }
    }
    if (any) tally.busy_passes++;
    // counts reach `stats` after every busy pass and every 64th idle one,
    // always before the pass ends, so a profile read after disarm() sees them
    if (any || (tally.passes & 63) == 0) flush(tally);
    busy_.fetch_sub(1);
    // Idle passes spin briefly, then yield: agent threads may outnumber the
    // cores, and a spinning thread must not keep one with work waiting.
    if (any) {
      idle = 0;
    } else if (++idle < 64) {
      cpu_relax();
    } else {
      std::this_thread::yield();
    }
  }
  if (io.ctx) sys_io_destroy(io.ctx);
  std::free(io.bufs);
  std::free(bounce);
}

}  // namespace fa

// server.cpp -- continuous-batching search service over one index.
//
// Queries arrive one by one (ann_server_submit); an admission thread moves
// them, in arrival order and while the HBM budget has room, into a ring in
// device memory (one copy per batch) and then publishes the new count with a
// stream write that is ordered after the copy.  The persistent server kernel
// keeps running: each wave takes the next published query, searches it, and
// writes its results into a host-mapped row plus a done word.  A reaper thread
// turns done words into completed results and frees the slots, so arrivals
// that come while others are on the GPU are admitted as room frees up and
// overlap on the device.
#include <hip/hip_runtime.h>

#include "agent.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/flashann.h"
#include "search_kernel.h"

// Defined in api.hip.
int ann_internal_server_args(ann_index *ix, int32_t k_max, int32_t L_max, int32_t hash_bits,
                             int32_t navigation, int32_t pq_scoring, fa::SearchArgs *base,
                             int32_t *dtype);
int ann_internal_fail(int code, const char *msg);
// Counts servers open on an index (the index refuses to replace or release
// what a running server kernel reads).
void ann_internal_server_hold(ann_index *ix, int delta);
int ann_internal_server_transport(ann_index *ix, int32_t requested, int32_t *tr,
                                  fa::Agent **agent, int64_t *stage_stride);

namespace {

double now_us() {
  return std::chrono::duration<double, std::micro>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Pending {
  std::vector<uint8_t> q;
  int32_t k, L;
  uint64_t tag;
  double submit_us;  // arrival time: admitted no earlier than this
};

struct Inflight {
  uint64_t seq = 0;
  uint64_t tag = 0;
  int32_t k = 0;
  double submit_us = 0;
  bool used = false;
};

struct Done {
  uint64_t tag;
  int32_t k;
  int32_t status;
  uint32_t steps;
  double submit_us, done_us;
  std::vector<int32_t> ids;
  std::vector<uint32_t> dists;
};

}  // namespace

struct ann_server {
  ann_index *ix = nullptr;
  bool held = false;  // counted in the index's open servers
  fa::ServerArgs args{};
  int32_t dtype = 0, delay = 1, wpb = 4, k_max = 100, L_max = 256;
  int32_t qbytes = 0, nav_stride = 0;
  int64_t queue_cap = 0, resident = 0;
  // device
  uint8_t *d_ring = nullptr;
  uint32_t *d_ctl = nullptr;  // 64 B lines: [0] next (u64), [16] published (u64), [32] stop
  // host (pinned, mapped)
  uint8_t *h_stage = nullptr;
  int32_t *h_ids = nullptr;
  uint32_t *h_dists = nullptr, *h_steps = nullptr, *h_done = nullptr;
  int32_t *h_status = nullptr;      // per slot, written by the GPU only on a failed read
  // AGENT transport: one request line per resident wave, served by agents of
  // this server's own for its whole life
  std::unique_ptr<fa::Agent> agent;
  fa::AgentRequest *h_req = nullptr;
  uint32_t *h_cpl = nullptr;
  uint8_t *h_tstage = nullptr;
  uint32_t *d_line_seq = nullptr;
  hipStream_t st_kernel = nullptr, st_copy = nullptr;
  hipEvent_t ev_kernel = nullptr;
  bool kernel_live = false;
  // host state
  std::mutex mu;
  std::condition_variable cv_admit, cv_done;
  std::deque<Pending> arrivals;
  std::vector<uint32_t> free_slots;
  std::vector<Inflight> inflight;   // per slot; only the admission thread fills a
                                    // free slot, only the reaper frees a used one
  std::vector<uint32_t> active;     // slots in use, compact (swap removal)
  std::vector<int64_t> active_pos;  // slot -> index in `active`, or -1
  std::deque<Done> done_q;
  std::vector<Done> last_poll;
  uint64_t published = 0;
  std::atomic<bool> quit{false};
  std::thread admit_thr, reap_thr;
  // stats
  std::atomic<uint64_t> submitted{0}, admitted{0}, completed{0}, relaunches{0};
  std::atomic<int64_t> max_inflight{0};
  int64_t n_inflight = 0;
  std::atomic<int> error{0};
  std::string error_msg;

  int launch_kernel() {
    hipError_t e = fa::launch_server(args, dtype, wpb, nullptr, st_kernel);
    if (e == hipSuccess) e = hipEventRecord(ev_kernel, st_kernel);
    if (e != hipSuccess) {
      error_msg = std::string("server kernel launch: ") + hipGetErrorString(e);
      error.store(ANN_EIO);
      return ANN_EIO;
    }
    kernel_live = true;
    return ANN_OK;
  }

  // Admission: arrival order, while a slot (HBM budget) is free.
  void admit_loop() {
    const int64_t eb = args.entry_bytes;
    const int64_t cap = args.ring_cap;
    std::vector<std::pair<uint32_t, Pending>> batch;
    while (!quit.load()) {
      batch.clear();
      {
        std::unique_lock<std::mutex> lk(mu);
        // an arrival is due once the clock has reached its arrival time
        // (timed submissions of an open-loop load); spin briefly for one due
        // within half a millisecond, otherwise sleep on the condition
        double wait_us = 200.0;
        if (!arrivals.empty() && !free_slots.empty()) {
          const double ahead = arrivals.front().submit_us - now_us();
          if (ahead > 0 && ahead < 500.0) {
            lk.unlock();
            while (now_us() < arrivals_front_time()) std::this_thread::yield();
            lk.lock();
          }
          wait_us = std::max(0.0, std::min(wait_us, arrivals.front().submit_us - now_us()));
        }
        cv_admit.wait_for(lk, std::chrono::microseconds((int64_t)wait_us), [&] {
          return quit.load() ||
                 (!arrivals.empty() && !free_slots.empty() && arrivals.front().submit_us <= now_us());
        });
        const double tnow = now_us();
        while (!arrivals.empty() && !free_slots.empty() && batch.size() < 4096 &&
               arrivals.front().submit_us <= tnow) {
          const uint32_t slot = free_slots.back();
          free_slots.pop_back();
          batch.emplace_back(slot, std::move(arrivals.front()));
          arrivals.pop_front();
        }
        for (size_t i = 0; i < batch.size(); i++) {
          const uint32_t slot = batch[i].first;
          Inflight &f = inflight[slot];
          f.seq = published + i;
          // the slot's 32-bit done word must not already hold this query's
          // mark, seq + 1 modulo 2^32, from an earlier use or its zero start
          __atomic_store_n(&h_done[16 * (int64_t)slot], (uint32_t)f.seq, __ATOMIC_RELAXED);
          f.tag = batch[i].second.tag;
          f.k = batch[i].second.k;
          f.submit_us = batch[i].second.submit_us;
          f.used = true;
          active_pos[slot] = (int64_t)active.size();
          active.push_back(slot);
        }
        n_inflight += (int64_t)batch.size();
        if (n_inflight > max_inflight.load()) max_inflight.store(n_inflight);
      }
      if (!batch.empty()) {
        // stage the entries, copy the (at most two) contiguous ring ranges,
        // then publish the count on the same stream
        for (size_t i = 0; i < batch.size(); i++) {
          const uint64_t seq = published + i;
          uint8_t *ent = h_stage + (int64_t)(seq % cap) * eb;
          const uint32_t ctrl[4] = {(uint32_t)(seq + 1), batch[i].first,
                                    (uint32_t)batch[i].second.k | ((uint32_t)batch[i].second.L << 16),
                                    0u};
          std::memcpy(ent, ctrl, 16);
          std::memset(ent + 16, 0, (size_t)(eb - 16));
          std::memcpy(ent + 16, batch[i].second.q.data(), (size_t)qbytes);
        }
        const uint64_t first = published, last = published + batch.size();
        hipError_t e = hipSuccess;
        uint64_t s = first;
        while (s < last && e == hipSuccess) {
          const uint64_t r0 = s % cap;
          const uint64_t run = std::min<uint64_t>(last - s, cap - r0);
          e = hipMemcpyAsync(d_ring + r0 * eb, h_stage + r0 * eb, run * eb, hipMemcpyHostToDevice,
                             st_copy);
          s += run;
        }
        if (e == hipSuccess) e = hipStreamWriteValue64(st_copy, d_ctl + 16, last, 0);
        if (e == hipSuccess) e = hipStreamSynchronize(st_copy);
        if (e != hipSuccess) {
          error_msg = std::string("admission copy: ") + hipGetErrorString(e);
          error.store(ANN_EIO);
          return;
        }
        published = last;
        admitted.fetch_add(batch.size());
      }
      // the kernel leaves after a long idle spell; start it again when work waits
      if (admitted.load() > completed.load() && (!kernel_live || hipEventQuery(ev_kernel) == hipSuccess)) {
        if (kernel_live) relaunches.fetch_add(1);
        if (launch_kernel() != ANN_OK) return;
      }
    }
  }

  // Reaper: done words -> completed results; frees slots.  It scans only the
  // slots in use; their Inflight records are not written while in use.
  void reap_loop() {
    std::vector<uint32_t> scan;
    std::vector<Done> fresh;
    std::vector<uint32_t> freed;
    while (!quit.load()) {
      {
        std::lock_guard<std::mutex> lk(mu);
        scan.assign(active.begin(), active.end());
      }
      fresh.clear();
      freed.clear();
      for (const uint32_t s : scan) {
        const Inflight &f = inflight[s];
        const uint32_t w = __atomic_load_n(&h_done[16 * (int64_t)s], __ATOMIC_ACQUIRE);
        if (w != (uint32_t)(f.seq + 1)) continue;
        Done d;
        d.tag = f.tag;
        d.k = f.k;
        d.submit_us = f.submit_us;
        d.done_us = now_us();
        d.steps = h_steps[s];
        d.status = __atomic_load_n(&h_status[s], __ATOMIC_RELAXED);
        if (d.status) __atomic_store_n(&h_status[s], 0, __ATOMIC_RELAXED);  // for the next use
        d.ids.assign(h_ids + (int64_t)s * k_max, h_ids + (int64_t)s * k_max + f.k);
        d.dists.assign(h_dists + (int64_t)s * k_max, h_dists + (int64_t)s * k_max + f.k);
        fresh.push_back(std::move(d));
        freed.push_back(s);
      }
      if (!fresh.empty()) {
        {
          std::lock_guard<std::mutex> lk(mu);
          for (uint32_t s : freed) {
            inflight[s].used = false;
            const int64_t p = active_pos[s];
            const uint32_t last = active.back();
            active[(size_t)p] = last;
            active_pos[last] = p;
            active.pop_back();
            active_pos[s] = -1;
            free_slots.push_back(s);
          }
          n_inflight -= (int64_t)freed.size();
          for (auto &d : fresh) done_q.push_back(std::move(d));
        }
        completed.fetch_add(freed.size());
        cv_admit.notify_one();
        cv_done.notify_all();
      } else {
        std::this_thread::sleep_for(std::chrono::microseconds(5));
      }
      if (error.load()) return;
    }
  }

  double arrivals_front_time() {
    std::lock_guard<std::mutex> lk(mu);
    return arrivals.empty() ? 0.0 : arrivals.front().submit_us;
  }

  int64_t n_inflight_snapshot() {
    std::lock_guard<std::mutex> lk(mu);
    return n_inflight;
  }
};

namespace {

void server_free(ann_server *s) {
  if (!s) return;
  s->agent.reset();  // joins the agents before their arrays go
  if (s->held) ann_internal_server_hold(s->ix, -1);
  s->held = false;
  if (s->h_req) (void)hipHostFree(s->h_req);
  if (s->h_cpl) (void)hipHostFree(s->h_cpl);
  if (s->h_tstage) (void)hipHostFree(s->h_tstage);
  if (s->d_line_seq) (void)hipFree(s->d_line_seq);
  if (s->h_status) (void)hipHostFree(s->h_status);
  if (s->ev_kernel) (void)hipEventDestroy(s->ev_kernel);
  if (s->st_kernel) (void)hipStreamDestroy(s->st_kernel);
  if (s->st_copy) (void)hipStreamDestroy(s->st_copy);
  if (s->d_ring) (void)hipFree(s->d_ring);
  if (s->d_ctl) (void)hipFree(s->d_ctl);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  if (s->h_ids) (void)hipHostFree(s->h_ids);
  if (s->h_dists) (void)hipHostFree(s->h_dists);
  if (s->h_steps) (void)hipHostFree(s->h_steps);
  if (s->h_done) (void)hipHostFree(s->h_done);
  delete s;
}

template <typename T>
T *mapped(T *p) {
  void *d = nullptr;
  return hipHostGetDevicePointer(&d, p, 0) == hipSuccess ? (T *)d : nullptr;
}

}  // namespace

extern "C" {

double ann_clock_us(void) { return now_us(); }

int ann_server_open(ann_index *ix, size_t hbm_budget_bytes, const ann_server_opts *opts,
                    ann_server **out) {
  if (!out) return ann_internal_fail(ANN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ix) return ann_internal_fail(ANN_EINVAL, "index is NULL");
  ann_server_opts o{};
  o.k_max = 100;
  o.L_max = 256;
  o.delay = 1;
  if (opts) o = *opts;
  if (o.k_max == 0) o.k_max = 100;
  if (o.L_max == 0) o.L_max = 256;
  const bool auto_wpb = o.waves_per_block == 0;
  if (auto_wpb) o.waves_per_block = 4;
  if (o.hash_bits == 0) o.hash_bits = 10;
  if (o.queue_cap == 0) o.queue_cap = 1 << 20;
  if (o.idle_polls == 0) o.idle_polls = 50000;
  if (o.beam_width == 0) o.beam_width = 1;
  if (o.k_max < 1 || o.k_max > 0xFFFF || o.L_max < o.k_max || o.L_max > 1024 ||
      o.delay < 0 || o.beam_width < 1 || o.waves_per_block < 1 || o.waves_per_block > 4 ||
      o.queue_cap < 1)
    return ann_internal_fail(ANN_EINVAL, "bad server options");
  if ((int64_t)(o.delay + 1) * o.beam_width > fa::kMaxPipe)
    return ann_internal_fail(ANN_ENOTSUP, "(delay+1)*beam_width exceeds the 8 nodes a query "
                                          "may hold in flight");
  ann_server *s = new (std::nothrow) ann_server();
  if (!s) return ann_internal_fail(ANN_ENOMEM, "server handle");
  s->ix = ix;
  s->k_max = o.k_max;
  s->L_max = o.L_max;
  s->delay = o.delay;
  s->queue_cap = o.queue_cap;
  s->published = o.first_ticket;  // tickets, next and published start here
  int rc = ann_internal_server_args(ix, o.k_max, o.L_max, o.hash_bits, o.navigation,
                                    o.pq_scoring, &s->args.base, &s->dtype);
  if (rc) {
    server_free(s);
    return rc;
  }
  // the default queries per workgroup shrinks to what the LDS holds
  while (auto_wpb && o.waves_per_block > 1 &&
         (int64_t)s->args.base.lds_per_wave * o.waves_per_block > 160 * 1024)
    o.waves_per_block /= 2;
  if ((int64_t)s->args.base.lds_per_wave * o.waves_per_block > 160 * 1024) {
    server_free(s);
    return ann_internal_fail(ANN_EINVAL, "LDS need per query x waves_per_block exceeds 160 KiB");
  }
  s->wpb = o.waves_per_block;
  s->args.base.delay = o.delay;
  s->args.base.beam = o.beam_width;
  s->args.base.pslots = std::max(2, (o.delay + 1) * o.beam_width);
  {
    int32_t tr = 0;
    fa::Agent *ag = nullptr;
    int64_t sstride = 0;
    rc = ann_internal_server_transport(ix, o.transport, &tr, &ag, &sstride);
    if (rc) {
      server_free(s);
      return rc;
    }
    s->agent.reset(ag);
    s->args.transport = tr;
    s->args.base.stage_stride = sstride;
  }
  s->nav_stride = s->args.base.nav_stride;
  s->qbytes = s->args.base.qbytes;
  // Per admitted query the device holds one ring entry (control + query);
  // the budget fixes how many queries may be admitted at once.  The ring
  // has room for every admitted query plus one claim per resident wave.
  const int64_t eb = 16 + s->nav_stride;
  int64_t resident = 0;
  hipError_t e = fa::launch_server(s->args, s->dtype, s->wpb, &resident, nullptr);
  if (e != hipSuccess) {
    server_free(s);
    return ann_internal_fail(ANN_EIO, "server occupancy query failed");
  }
  s->resident = resident;
  const int64_t nslots = (int64_t)(hbm_budget_bytes / (size_t)eb) - resident;
  if (nslots < 1) {
    server_free(s);
    return ann_internal_fail(ANN_ENOMEM, "HBM budget below one query plus one entry per resident wave");
  }
  const int64_t slots = std::min<int64_t>(nslots, 1 << 20);
  const int64_t ring_cap = slots + resident;
  s->args.entry_bytes = eb;
  s->args.ring_cap = (uint32_t)ring_cap;
  s->args.nslots = (uint32_t)slots;
  s->args.idle_limit = (uint32_t)o.idle_polls;
  const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
  if ((e = hipMalloc(&s->d_ring, ring_cap * eb)) != hipSuccess ||
      (e = hipMalloc(&s->d_ctl, 64 * sizeof(uint32_t))) != hipSuccess ||
      (e = hipHostMalloc((void **)&s->h_stage, ring_cap * eb, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void **)&s->h_ids, slots * o.k_max * 4, fl)) != hipSuccess ||
      (e = hipHostMalloc((void **)&s->h_dists, slots * o.k_max * 4, fl)) != hipSuccess ||
      (e = hipHostMalloc((void **)&s->h_steps, slots * 4, fl)) != hipSuccess ||
      (e = hipHostMalloc((void **)&s->h_done, slots * 64, fl)) != hipSuccess ||
      (e = hipHostMalloc((void **)&s->h_status, slots * 4, fl)) != hipSuccess ||
      (e = hipMemset(s->d_ctl, 0, 64 * sizeof(uint32_t))) != hipSuccess ||
      (e = hipMemcpy(s->d_ctl, &o.first_ticket, sizeof(uint64_t), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(s->d_ctl + 16, &o.first_ticket, sizeof(uint64_t), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipStreamCreateWithFlags(&s->st_kernel, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&s->st_copy, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&s->ev_kernel, hipEventDisableTiming)) != hipSuccess) {
    server_free(s);
    return ann_internal_fail(e == hipErrorOutOfMemory ? ANN_ENOMEM : ANN_EIO,
                             "server buffers / streams");
  }
  std::memset(s->h_done, 0, (size_t)slots * 64);
  std::memset(s->h_status, 0, (size_t)slots * 4);
  s->args.res_status = mapped(s->h_status);
  if (s->agent) {
    // one line per resident wave (the transport line of wave w is w)
    const int64_t G = resident, P = s->args.base.pslots, ss = s->args.base.stage_stride;
    if ((e = hipHostMalloc((void **)&s->h_req, sizeof(fa::AgentRequest) * G, fl)) != hipSuccess ||
        (e = hipHostMalloc((void **)&s->h_cpl, sizeof(uint32_t) * fa::kCplStride * G, fl)) !=
            hipSuccess ||
        (e = hipHostMalloc((void **)&s->h_tstage, G * P * ss, fl)) != hipSuccess ||
        (e = hipMalloc(&s->d_line_seq, sizeof(uint32_t) * G)) != hipSuccess ||
        (e = hipMemset(s->d_line_seq, 0, sizeof(uint32_t) * G)) != hipSuccess) {
      server_free(s);
      return ann_internal_fail(ANN_ENOMEM, "server transport buffers");
    }
    std::memset(s->h_req, 0, sizeof(fa::AgentRequest) * G);
    std::memset(s->h_cpl, 0, sizeof(uint32_t) * fa::kCplStride * G);
    s->args.base.req = mapped((uint64_t *)s->h_req);
    s->args.base.cpl = mapped(s->h_cpl);
    s->args.base.stage = mapped(s->h_tstage);
    s->args.base.spin_limit = o.spin_limit ? o.spin_limit : (1u << 24);
    s->args.base.poll_nap = 32u;
    s->args.base.line_seq = s->d_line_seq;
    if (!s->args.base.req || !s->args.base.cpl || !s->args.base.stage) {
      server_free(s);
      return ann_internal_fail(ANN_EIO, "server transport buffers not mapped");
    }
    s->agent->arm(s->h_req, s->h_cpl, s->h_tstage, G, ss, (int)P);
  }
  s->args.ring = s->d_ring;
  s->args.next = (uint64_t *)s->d_ctl;
  s->args.published = (const uint64_t *)(s->d_ctl + 16);
  s->args.stop = s->d_ctl + 32;
  s->args.res_ids = mapped(s->h_ids);
  s->args.res_dists = mapped(s->h_dists);
  s->args.res_steps = mapped(s->h_steps);
  s->args.done = mapped(s->h_done);
  if (!s->args.res_ids || !s->args.res_dists || !s->args.res_steps || !s->args.done ||
      !s->args.res_status) {
    server_free(s);
    return ann_internal_fail(ANN_EIO, "result rows not mapped");
  }
  s->inflight.assign((size_t)slots, Inflight{});
  s->active_pos.assign((size_t)slots, -1);
  s->active.reserve((size_t)std::min<int64_t>(slots, 1 << 16));
  s->free_slots.reserve((size_t)slots);
  for (int64_t i = slots - 1; i >= 0; i--) s->free_slots.push_back((uint32_t)i);
  if (s->launch_kernel() != ANN_OK) {
    const std::string m = s->error_msg;
    server_free(s);
    return ann_internal_fail(ANN_EIO, m.c_str());
  }
  s->admit_thr = std::thread([s] { s->admit_loop(); });
  s->reap_thr = std::thread([s] { s->reap_loop(); });
  ann_internal_server_hold(ix, +1);
  s->held = true;
  *out = s;
  return ANN_OK;
}

int ann_server_submit(ann_server *s, const void *host_query, int32_t k, int32_t L, uint64_t tag) {
  if (!s || !host_query) return ann_internal_fail(ANN_EINVAL, "NULL argument");
  if (k < 1 || k > s->k_max || L < k || L > s->L_max)
    return ann_internal_fail(ANN_EINVAL, "need 1 <= k <= k_max and k <= L <= L_max");
  if (s->error.load()) return ann_internal_fail(s->error.load(), s->error_msg.c_str());
  Pending p;
  p.q.assign((const uint8_t *)host_query, (const uint8_t *)host_query + s->qbytes);
  p.k = k;
  p.L = L;
  p.tag = tag;
  p.submit_us = now_us();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int64_t)s->arrivals.size() >= s->queue_cap)
      return ann_internal_fail(ANN_EBUSY, "arrival queue full");
    s->arrivals.push_back(std::move(p));
  }
  s->submitted.fetch_add(1);
  s->cv_admit.notify_one();
  return ANN_OK;
}

int ann_server_submit_batch(ann_server *s, const void *host_queries, int64_t n, const int32_t *ks,
                            const int32_t *Ls, const uint64_t *tags, const double *arrival_us) {
  if (!s || (n > 0 && (!host_queries || !ks || !Ls || !tags)) || n < 0)
    return ann_internal_fail(ANN_EINVAL, "NULL argument");
  if (s->error.load()) return ann_internal_fail(s->error.load(), s->error_msg.c_str());
  for (int64_t i = 0; i < n; i++) {
    if (ks[i] < 1 || ks[i] > s->k_max || Ls[i] < ks[i] || Ls[i] > s->L_max)
      return ann_internal_fail(ANN_EINVAL, "need 1 <= k <= k_max and k <= L <= L_max");
    if (arrival_us && i > 0 && arrival_us[i] < arrival_us[i - 1])
      return ann_internal_fail(ANN_EINVAL, "arrival times must not decrease");
  }
  const double t0 = now_us();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int64_t)s->arrivals.size() + n > s->queue_cap)
      return ann_internal_fail(ANN_EBUSY, "arrival queue full");
    if (arrival_us && n > 0 && !s->arrivals.empty() && arrival_us[0] < s->arrivals.back().submit_us)
      return ann_internal_fail(ANN_EINVAL, "arrival times must not go back in time");
    for (int64_t i = 0; i < n; i++) {
      Pending p;
      const uint8_t *q = (const uint8_t *)host_queries + i * (int64_t)s->qbytes;
      p.q.assign(q, q + s->qbytes);
      p.k = ks[i];
      p.L = Ls[i];
      p.tag = tags[i];
      p.submit_us = arrival_us ? arrival_us[i] : t0;
      s->arrivals.push_back(std::move(p));
    }
  }
  s->submitted.fetch_add((uint64_t)n);
  s->cv_admit.notify_one();
  return ANN_OK;
}

int ann_server_poll(ann_server *s, ann_result *out, int32_t max, int32_t *n_out,
                    int32_t timeout_us) {
  if (!s || !n_out || (max > 0 && !out)) return ann_internal_fail(ANN_EINVAL, "NULL argument");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done_q.empty() && timeout_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                        [&] { return !s->done_q.empty() || s->error.load() != 0; });
  s->last_poll.clear();
  while (!s->done_q.empty() && (int32_t)s->last_poll.size() < max) {
    s->last_poll.push_back(std::move(s->done_q.front()));
    s->done_q.pop_front();
  }
  for (size_t i = 0; i < s->last_poll.size(); i++) {
    const Done &d = s->last_poll[i];
    out[i].tag = d.tag;
    out[i].status = d.status;
    out[i].k = d.k;
    out[i].steps = d.steps;
    out[i].ids = d.ids.data();
    out[i].dists = d.dists.data();
    out[i].submit_us = d.submit_us;
    out[i].done_us = d.done_us;
  }
  *n_out = (int32_t)s->last_poll.size();
  if (*n_out == 0 && s->error.load()) return ann_internal_fail(s->error.load(), s->error_msg.c_str());
  return ANN_OK;
}

int ann_server_poll_into(ann_server *s, int32_t max, uint64_t *tags, int32_t *ks, int32_t *ids,
                         void *dists, uint32_t *steps, double *submit_us, double *done_us,
                         int32_t *status, int32_t *n_out, int32_t timeout_us) {
  if (!s || !n_out || max < 0 || (max > 0 && (!tags || !ks || !ids || !dists)))
    return ann_internal_fail(ANN_EINVAL, "NULL argument");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done_q.empty() && timeout_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                        [&] { return !s->done_q.empty() || s->error.load() != 0; });
  int32_t n = 0;
  while (!s->done_q.empty() && n < max) {
    const Done &d = s->done_q.front();
    tags[n] = d.tag;
    ks[n] = d.k;
    int32_t *row = ids + (int64_t)n * s->k_max;
    uint32_t *drow = (uint32_t *)dists + (int64_t)n * s->k_max;
    for (int32_t j = 0; j < s->k_max; j++) {
      row[j] = j < d.k ? d.ids[(size_t)j] : -1;
      drow[j] = j < d.k ? d.dists[(size_t)j] : 0xFFFFFFFFu;
    }
    if (steps) steps[n] = d.steps;
    if (submit_us) submit_us[n] = d.submit_us;
    if (done_us) done_us[n] = d.done_us;
    if (status) status[n] = d.status;
    s->done_q.pop_front();
    n++;
  }
  *n_out = n;
  if (n == 0 && s->error.load()) return ann_internal_fail(s->error.load(), s->error_msg.c_str());
  return ANN_OK;
}

int ann_server_stats_get(ann_server *s, ann_server_stats *out) {
  if (!s || !out) return ann_internal_fail(ANN_EINVAL, "NULL argument");
  out->submitted = s->submitted.load();
  out->admitted = s->admitted.load();
  out->completed = s->completed.load();
  out->relaunches = s->relaunches.load();
  out->max_inflight = s->max_inflight.load();
  out->slots = s->args.nslots;
  out->resident_waves = s->resident;
  return ANN_OK;
}

int ann_server_close(ann_server *s) {
  if (!s) return ANN_OK;
  // let admitted work finish (at most a minute), then stop the kernel
  const double give_up = now_us() + 60e6;
  while (now_us() < give_up) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->arrivals.empty() && s->n_inflight == 0) break;
    }
    if (s->error.load()) break;
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  s->quit.store(true);
  s->cv_admit.notify_all();
  if (s->admit_thr.joinable()) s->admit_thr.join();
  if (s->reap_thr.joinable()) s->reap_thr.join();
  int rc = ANN_OK;
  hipError_t e = hipStreamWriteValue32(s->st_copy, s->d_ctl + 32, 1u, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st_copy);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st_kernel);
  if (e != hipSuccess) rc = ann_internal_fail(ANN_EIO, hipGetErrorString(e));
  if (s->agent) s->agent->disarm();
  server_free(s);
  return rc;
}

}  // extern "C"

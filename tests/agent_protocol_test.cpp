// CPU exercise of the query-grained record transport: threads play the GPU
// waves (same structs, same atomics), the real agent serves them.  Built with
// ThreadSanitizer and AddressSanitizer by tests/test_agent_protocol.py.
//
// Each fake wave keeps up to `depth` requests outstanding (1: strict, 2: one
// step stale, P: a full pipeline of P slots), consumes them in order, waits on
// each completion word with acquire loads, and checks the staged bytes
// against the record store.  Faults: a slow node (straggler) and a failing
// node (error completion).
//
// Usage: agent_test NQ AGENTS [mode [dir]]; mode "mem" (records in memory,
// default), "wrap" (memory, request numbers crossing their wrap point),
// "file" (one record file in dir, O_DIRECT + asynchronous reads where the
// file system allows) or "stripes" (three striped record files in dir).
#include <fcntl.h>
#include <unistd.h>

#include <atomic>
#include <string>
#include <cstdio>
#include <deque>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "../paper_2507_10070_amd/csrc/agent.h"

using fa::AgentRequest;

static int check(bool c, const char *what) {
  if (!c) std::fprintf(stderr, "FAIL: %s\n", what);
  return c ? 0 : 1;
}

int main(int argc, char **argv) {
  const int64_t n = 5000, slot = 512, copy = 384;
  const int64_t nq = argc > 1 ? atoll(argv[1]) : 64;
  const int agents = argc > 2 ? atoi(argv[2]) : 3;
  // request numbers already used per line: "wrap" starts just below the
  // point where they wrap around, so every line crosses it
  const std::string mode = argc > 3 ? argv[3] : "mem";
  const bool wrap = mode == "wrap";
  const bool file = mode == "file" || mode == "stripes";
  const int nstripes = mode == "stripes" ? 3 : 1;
  const std::string dir = argc > 4 ? argv[4] : "/tmp";
  const int steps = 200;
  std::vector<uint8_t> records(n * slot);
  for (int64_t i = 0; i < n * slot; i++) records[i] = (uint8_t)((i * 2654435761ull) >> 13);

  // record files: record v is slot v / S of file v % S
  std::vector<int> fds;
  bool direct = true;
  for (int s = 0; file && s < nstripes; s++) {
    const std::string path = dir + "/stripe" + std::to_string(s) + ".bin";
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f) return 2;
    for (int64_t v = s; v < n; v += nstripes) std::fwrite(&records[v * slot], 1, slot, f);
    std::fclose(f);
    int fd = open(path.c_str(), O_RDONLY | O_DIRECT);
    if (fd < 0) {
      direct = false;
      fd = open(path.c_str(), O_RDONLY);
    }
    if (fd < 0) return 2;
    fds.push_back(fd);
  }
  fa::Agent agent(file ? nullptr : records.data(), fds.data(), (int)fds.size(), file && direct,
                  slot, (int32_t)copy, file && direct ? 512 : (int32_t)copy, agents, 16);
  agent.faults.delay_node = 7;
  agent.faults.delay_us = 300;
  agent.faults.fail_node = 11;

  std::vector<AgentRequest> req(nq);
  std::vector<uint32_t> cpl(fa::kCplStride * nq, 0);
  const int64_t stride = 512;
  const int P = 5;
  std::vector<uint8_t> stage(nq * P * stride, 0);
  std::memset(req.data(), 0, sizeof(AgentRequest) * nq);
  const uint32_t M = (0x40000000u / P) * P;
  const uint32_t start = wrap ? M - 37 : 0u;
  agent.arm(req.data(), cpl.data(), stage.data(), nq, stride, P, start);

  std::atomic<int> errors{0}, failures_seen{0};
  auto wave = [&](int64_t q) {
    std::mt19937 rng((unsigned)q * 7919u + 1u);
    uint32_t seq = start;
    auto issue = [&](uint32_t node) {
      seq = fa::next_seq(seq, P);
      // release: this thread's reads of the slot's previous staging data are
      // ordered before the agent may overwrite it (on the GPU the wave has
      // consumed that data into LDS before it issues the next request)
      __atomic_store_n(&req[q].slot[seq % P], ((uint64_t)node << 32) | seq, __ATOMIC_RELEASE);
      return seq;
    };
    auto consume = [&](uint32_t s, uint32_t node) {
      // wait until this slot's completion word names request s
      uint32_t c;
      while (true) {
        c = __atomic_load_n(&cpl[q * fa::kCplStride + s % P], __ATOMIC_ACQUIRE);
        if ((c & ~fa::kCplError) == s) break;
        std::this_thread::yield();
      }
      if (c & fa::kCplError) {
        if (node != 11) errors++;
        failures_seen++;
        return;
      }
      const uint8_t *got = &stage[(q * P + s % P) * stride];
      if (std::memcmp(got, &records[(int64_t)node * slot], copy) != 0) errors++;
    };
    const int depth = q % 3 == 0 ? 1 : (q % 3 == 1 ? 2 : P);
    std::deque<std::pair<uint32_t, uint32_t>> inflight;  // (seq, node), oldest first
    for (int i = 0; i < steps; i++) {
      uint32_t node = rng() % n;
      if (i % 50 == 3) node = 7;    // straggler
      if (i % 97 == 5) node = 11;   // failing read
      inflight.emplace_back(issue(node), node);
      if ((int)inflight.size() == depth) {
        consume(inflight.front().first, inflight.front().second);
        inflight.pop_front();
      }
    }
    while (!inflight.empty()) {
      consume(inflight.front().first, inflight.front().second);
      inflight.pop_front();
    }
  };
  std::vector<std::thread> waves;
  for (int64_t q = 0; q < nq; q++) waves.emplace_back(wave, q);
  for (auto &w : waves) w.join();
  agent.disarm();

  int bad = 0;
  bad += check(errors.load() == 0, "staged data or completion mismatch");
  bad += check(failures_seen.load() > 0, "injected failures observed");
  bad += check(agent.stats.requests.load() == (uint64_t)(nq * steps), "every request served");
  bad += check(agent.stats.errors.load() == (uint64_t)failures_seen.load(), "error count");
  // the agent must be reusable after disarm
  std::memset(req.data(), 0, sizeof(AgentRequest) * nq);
  std::fill(cpl.begin(), cpl.end(), 0u);
  agent.arm(req.data(), cpl.data(), stage.data(), nq, stride, 2);
  __atomic_store_n(&req[0].slot[1], (42ull << 32) | 1u, __ATOMIC_RELEASE);
  while (__atomic_load_n(&cpl[1], __ATOMIC_ACQUIRE) != 1u) std::this_thread::yield();
  bad += check(std::memcmp(&stage[1 * stride], &records[42 * slot], copy) == 0, "re-armed serve");
  agent.disarm();
  if (file) {
    uint64_t per_stripe = 0;
    for (int s = 0; s < nstripes; s++) per_stripe += agent.stats.stripe_requests[s].load();
    bad += check(per_stripe == agent.stats.requests.load(), "requests counted per stripe");
    for (int s = 0; s < nstripes; s++)
      bad += check(agent.stats.stripe_requests[s].load() > 0, "every stripe served");
    bad += check(agent.async_io() == direct, "asynchronous reads with O_DIRECT");
  }
  for (int fd : fds) close(fd);
  std::printf("%s: %lld queries x %d requests, %d agents, %d injected failures, mode %s%s\n",
              bad ? "FAIL" : "OK", (long long)nq, steps, agents, failures_seen.load(),
              mode.c_str(), file ? (direct ? " (O_DIRECT, asynchronous)" : " (buffered)") : "");
  return bad ? 1 : 0;
}

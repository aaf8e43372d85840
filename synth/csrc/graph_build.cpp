// graph_build.cpp -- deterministic proximity-graph construction for the
// synthetic workloads (index building; the paper does not describe it and
// inherits DiskANN-style graphs).  Input generation only: the greedy searches
// of the refinement step (7) build the graph and share no code with the
// search under test or with the oracle.
//
// Steps (all deterministic for a given seed, independent of thread count):
//   1. kNN pool of size K per point: exact for n <= exact_limit, otherwise
//      each point is compared with the members of its two nearest pivots'
//      partitions (pivots = a seeded sample of the points).
//   2. alpha-pruning of the pool to at most R out-edges (alpha = 1 is the
//      relative-neighbourhood rule; alpha > 1 keeps longer edges).
//   3. reverse edges, re-pruned where a list exceeds R.
//   4. long-range edges: R/8 seeded random hub edges per point, R/4 per hub,
//      and the entry (medoid) links to the hubs in farthest-point order.
//   5. every list is filled to exactly R ids with the next-closest pool
//      candidates (-1 padding only when fewer than R other points exist).
//   6. breadth-first connectivity repair from the medoid.
//   7. refinement passes in the manner of DiskANN's Vamana construction
//      (optional, `passes`): every point, in a seeded order and in batches,
//      runs a greedy best-first search for its own vector from the medoid
//      with list size Lb on the graph as it stood at the batch start; the
//      expanded nodes plus its current neighbours are alpha-pruned to its new
//      list (its long-range edges from step 4 are kept), and every new edge
//      p -> q proposes q -> p, re-pruned where a list exceeds R.  These
//      passes prune with alpha = 1: on mixtures in 96-128 dimensions all
//      distances inside a component are nearly equal, so a rule with
//      alpha = 1.2 keeps almost every candidate, the lists degenerate into
//      kNN lists, and search recall fell to about 0.3 (measured); alpha = 1
//      keeps them diverse.  Then steps 5 and 6 again.  Searches of a batch
//      read a frozen graph and updates are applied in batch order, so the
//      result does not depend on the number of threads.
// Distances are squared L2 accumulated in int32 (u8/i8) or float (f32, in
// eight partial sums) and compared as float with ties broken by id.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <thread>
#include <utility>
#include <vector>

namespace {

enum { DT_U8 = 1, DT_I8 = 2, DT_F32 = 3 };

struct Data {
  const void *base;
  int64_t n;
  int d;
  int dtype;
  float dist(int64_t i, int64_t j) const {
    if (dtype == DT_U8) {
      const uint8_t *a = (const uint8_t *)base + i * d, *b = (const uint8_t *)base + j * d;
      int32_t s = 0;
      for (int t = 0; t < d; t++) {
        int32_t x = (int32_t)a[t] - (int32_t)b[t];
        s += x * x;
      }
      return (float)s;
    }
    if (dtype == DT_I8) {
      const int8_t *a = (const int8_t *)base + i * d, *b = (const int8_t *)base + j * d;
      int32_t s = 0;
      for (int t = 0; t < d; t++) {
        int32_t x = (int32_t)a[t] - (int32_t)b[t];
        s += x * x;
      }
      return (float)s;
    }
    // eight independent partial sums (one vector register), added pairwise:
    // a single running sum is a chain of dependent adds the compiler may not
    // reorder, which made f32 builds several times slower than int8 ones
    const float *a = (const float *)base + i * d, *b = (const float *)base + j * d;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int t = 0;
    for (; t + 8 <= d; t += 8)
      for (int l = 0; l < 8; l++) {
        const float x = a[t + l] - b[t + l];
        s[l] += x * x;
      }
    float r = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    for (; t < d; t++) {
      const float x = a[t] - b[t];
      r += x * x;
    }
    return r;
  }
  // start loading row i (rows are hundreds of bytes in random order: the
  // prefetches of a whole neighbour list overlap their memory latencies)
  void prefetch(int64_t i) const {
    const int64_t bytes = (int64_t)d * (dtype == DT_F32 ? 4 : 1);
    const char *p = (const char *)base + i * bytes;
    for (int64_t o = 0; o < bytes; o += 64) __builtin_prefetch(p + o, 0, 1);
  }
};

using Cand = std::pair<float, int32_t>;  // (distance, id), lexicographic order

uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Phase reports on stderr when FLASHANN_BUILD_PROGRESS is set (long builds
// print as they go).
struct Progress {
  bool on = std::getenv("FLASHANN_BUILD_PROGRESS") != nullptr;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  void operator()(const char *what, long long a = -1, long long b = -1) const {
    if (!on) return;
    const double s =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (a >= 0) std::fprintf(stderr, "[graph %7.1fs] %s %lld/%lld\n", s, what, a, b);
    else std::fprintf(stderr, "[graph %7.1fs] %s\n", s, what);
    std::fflush(stderr);
  }
};

// Run fn(0..n-1) on `threads` threads in chunks; with a label, the thread
// that completes each tenth of the items reports it.
void parallel_for(int64_t n, int threads, const std::function<void(int64_t)> &fn,
                  const Progress *progress = nullptr, const char *label = nullptr) {
  if (threads < 1) threads = 1;
  std::atomic<int64_t> next(0), done(0);
  const int64_t chunk = 64;
  auto work = [&]() {
    for (;;) {
      int64_t s = next.fetch_add(chunk);
      if (s >= n) break;
      int64_t e = std::min(n, s + chunk);
      for (int64_t i = s; i < e; i++) fn(i);
      if (progress && label) {
        const int64_t before = done.fetch_add(e - s), after = before + (e - s);
        if (after * 10 / n != before * 10 / n) (*progress)(label, after, n);
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < threads; t++) th.emplace_back(work);
  work();
  for (auto &t : th) t.join();
}

// Keep the K smallest (distance, id) of `v` sorted ascending, in a buffer of
// exactly that size (the lists are kept per point, so the scan buffer's
// capacity must not come with them).
void keep_smallest(std::vector<Cand> &v, size_t K) {
  if (v.size() > K) {
    std::nth_element(v.begin(), v.begin() + K, v.end());
    v.resize(K);
  }
  std::sort(v.begin(), v.end());
  std::vector<Cand>(v.begin(), v.end()).swap(v);
}

// alpha-pruning: scan candidates in ascending order and keep c unless some
// kept k satisfies alpha^2 * |c - k|^2 <= |p - c|^2.
void robust_prune(const Data &D, const std::vector<Cand> &sorted_pool, int R, float alpha,
                  std::vector<int32_t> &out) {
  out.clear();
  const float a2 = alpha * alpha;
  const size_t np = sorted_pool.size();
  for (size_t i = 0; i < np && i < 4; i++) D.prefetch(sorted_pool[i].second);
  for (size_t i = 0; i < np; i++) {
    const Cand &c = sorted_pool[i];
    if ((int)out.size() >= R) break;
    if (i + 4 < np) D.prefetch(sorted_pool[i + 4].second);
    bool keep = true;
    for (int32_t k : out) {
      if (k == c.second) { keep = false; break; }
      if (a2 * D.dist(c.second, k) <= c.first) { keep = false; break; }
    }
    if (keep) out.push_back(c.second);
  }
}

// Greedy best-first search for the vector of point p on a degree-R graph
// (flat ids, -1 = empty) from `entry` with a candidate list of Lb entries;
// returns the expanded nodes with their distances to p.  `stamp` (n entries,
// per thread) marks visited nodes with the current `epoch`.
void greedy_expand(const Data &D, const int32_t *adj, int R, int64_t p, int32_t entry, int Lb,
                   std::vector<uint32_t> &stamp, uint32_t epoch, std::vector<Cand> &expanded) {
  expanded.clear();
  std::vector<std::pair<Cand, bool>> list;  // sorted by (distance, id); bool = expanded
  list.reserve((size_t)Lb + (size_t)R + 1);
  stamp[entry] = epoch;
  list.push_back({Cand(D.dist(p, entry), entry), false});
  for (;;) {
    size_t i = 0;
    while (i < list.size() && list[i].second) i++;
    if (i == list.size()) break;
    list[i].second = true;
    const int32_t u = list[i].first.second;
    expanded.push_back(list[i].first);
    const int32_t *row = adj + (int64_t)u * R;
    for (int j = 0; j < R; j++)
      if (row[j] >= 0 && stamp[row[j]] != epoch) D.prefetch(row[j]);
    for (int j = 0; j < R; j++) {
      const int32_t x = row[j];
      if (x < 0 || stamp[x] == epoch) continue;
      stamp[x] = epoch;
      const Cand c(D.dist(p, x), x);
      if ((int)list.size() >= Lb && !(c < list.back().first)) continue;
      auto pos = std::lower_bound(list.begin(), list.end(), std::make_pair(c, false),
                                  [](const std::pair<Cand, bool> &a,
                                     const std::pair<Cand, bool> &b) { return a.first < b.first; });
      list.insert(pos, {c, false});
      if ((int)list.size() > Lb) list.pop_back();
    }
  }
}

}  // namespace

extern "C" {

// Medoid: argmin_i |x_i - mean|^2 with the mean in fp64; ties -> smaller id.
int64_t synth_medoid(const void *base, int64_t n, int32_t d, int32_t dtype) {
  if (!base || n < 1 || d < 1) return -1;
  std::vector<double> mean(d, 0.0);
  auto val = [&](int64_t i, int t) -> double {
    if (dtype == DT_U8) return ((const uint8_t *)base)[i * d + t];
    if (dtype == DT_I8) return ((const int8_t *)base)[i * d + t];
    return ((const float *)base)[i * d + t];
  };
  for (int64_t i = 0; i < n; i++)
    for (int t = 0; t < d; t++) mean[t] += val(i, t);
  for (int t = 0; t < d; t++) mean[t] /= (double)n;
  int64_t best = 0;
  double bestd = INFINITY;
  for (int64_t i = 0; i < n; i++) {
    double s = 0;
    for (int t = 0; t < d; t++) {
      double x = val(i, t) - mean[t];
      s += x * x;
    }
    if (s < bestd) { bestd = s; best = i; }
  }
  return best;
}

// Random-link graph: R distinct neighbours per node, none equal to itself
// (the sample indices of the degree selector use random links).
int synth_random_graph(int64_t n, int32_t R, uint64_t seed, int32_t *adj) {
  if (n < 2 || R < 1 || !adj) return -22;
  for (int64_t i = 0; i < n; i++) {
    uint64_t s = seed ^ (0xA24BAED4963EE407ull * (uint64_t)(i + 1));
    int32_t *row = adj + i * R;
    int m = 0;
    int64_t limit = std::min<int64_t>(R, n - 1);
    while (m < limit) {
      int32_t c = (int32_t)(splitmix64(s) % (uint64_t)n);
      if (c == i) continue;
      bool dup = false;
      for (int t = 0; t < m; t++) dup |= (row[t] == c);
      if (!dup) row[m++] = c;
    }
    for (; m < R; m++) row[m] = -1;
  }
  return 0;
}

int synth_build_graph(const void *base, int64_t n, int32_t d, int32_t dtype, int32_t R,
                      uint64_t seed, int32_t threads, int32_t pool, float alpha,
                      int32_t n_hubs, int64_t exact_limit, int32_t passes, int32_t Lb,
                      int32_t *adj, int32_t *entry_out) {
  if (!base || !adj || n < 1 || d < 1 || R < 1 || pool < R ||
      (dtype != DT_U8 && dtype != DT_I8 && dtype != DT_F32))
    return -22;
  const Data D{base, n, d, dtype};
  const Progress progress;
  const int64_t medoid = synth_medoid(base, n, d, dtype);
  if (entry_out) *entry_out = (int32_t)medoid;
  if (n == 1) {
    for (int j = 0; j < R; j++) adj[j] = -1;
    return 0;
  }
  const size_t K = (size_t)std::min<int64_t>(pool, n - 1);

  // ---- hubs / pivots: a seeded sample without replacement, plus the medoid.
  int64_t H = std::max<int64_t>(1, std::min<int64_t>(n_hubs, n));
  std::vector<int32_t> hubs;
  {
    std::vector<int32_t> perm(n);
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    uint64_t s = seed;
    for (int64_t i = 0; i < H; i++) {
      int64_t j = i + (int64_t)(splitmix64(s) % (uint64_t)(n - i));
      std::swap(perm[i], perm[j]);
    }
    hubs.assign(perm.begin(), perm.begin() + H);
    if (std::find(hubs.begin(), hubs.end(), (int32_t)medoid) == hubs.end())
      hubs.push_back((int32_t)medoid);
    std::sort(hubs.begin(), hubs.end());
  }

  // ---- nearest hubs of every point (used for partitions and hub edges).
  const int64_t Hn = (int64_t)hubs.size();
  const int Rn = std::max(2, R / 8);  // random hub edges per point
  const size_t M = (size_t)std::min<int64_t>(Hn, 2);
  std::vector<std::vector<Cand>> hub_near(n);
  parallel_for(n, threads, [&](int64_t i) {
    std::vector<Cand> v;
    v.reserve(Hn);
    for (int64_t p = 0; p < Hn; p++) v.emplace_back(D.dist(i, hubs[p]), (int32_t)p);
    keep_smallest(v, M);
    hub_near[i] = std::move(v);
  }, &progress, "nearest hubs");

  progress("nearest hubs");

  // ---- 1. kNN pools.
  std::vector<std::vector<Cand>> pools(n);
  if (n <= exact_limit) {
    parallel_for(n, threads, [&](int64_t i) {
      std::vector<Cand> v;
      v.reserve(n);
      for (int64_t j = 0; j < n; j++)
        if (j != i) v.emplace_back(D.dist(i, j), (int32_t)j);
      keep_smallest(v, K);
      pools[i] = std::move(v);
    }, &progress, "kNN pools");
  } else {
    std::vector<std::vector<int32_t>> members(Hn);
    for (int64_t i = 0; i < n; i++) members[hub_near[i][0].second].push_back((int32_t)i);
    // Visit points grouped by primary partition for cache locality.
    std::vector<int32_t> order;
    order.reserve(n);
    for (int64_t p = 0; p < Hn; p++) order.insert(order.end(), members[p].begin(), members[p].end());
    parallel_for(n, threads, [&](int64_t t) {
      const int64_t i = order[t];
      std::vector<Cand> v;
      const int32_t p1 = hub_near[i][0].second;
      const int32_t p2 = hub_near[i].size() > 1 ? hub_near[i][1].second : p1;
      const int32_t parts[2] = {p1, p2};
      for (int q = 0; q < (p1 == p2 ? 1 : 2); q++)
        for (int32_t j : members[parts[q]])
          if (j != i) v.emplace_back(D.dist(i, j), j);
      keep_smallest(v, K);
      pools[i] = std::move(v);
    }, &progress, "kNN pools");
  }

  progress("kNN pools");

  // ---- 2. alpha-pruning.
  std::vector<std::vector<int32_t>> out(n);
  parallel_for(n, threads, [&](int64_t i) { robust_prune(D, pools[i], R, alpha, out[i]); },
               &progress, "pruning");

  // ---- 3. reverse edges (lists built in id order), re-pruned when too long.
  {
    std::vector<std::vector<int32_t>> rev(n);
    for (int64_t i = 0; i < n; i++)
      for (int32_t c : out[i]) rev[c].push_back((int32_t)i);
    std::vector<std::vector<int32_t>> out2(n);
    parallel_for(n, threads, [&](int64_t i) {
      std::vector<Cand> c;
      for (int32_t x : out[i]) c.emplace_back(D.dist(i, x), x);
      for (int32_t x : rev[i]) c.emplace_back(D.dist(i, x), x);
      std::sort(c.begin(), c.end());
      c.erase(std::unique(c.begin(), c.end()), c.end());
      if ((int)c.size() <= R) {
        for (auto &e : c) out2[i].push_back(e.second);
      } else {
        robust_prune(D, c, R, alpha, out2[i]);
      }
    });
    out.swap(out2);
  }

  std::vector<std::vector<int32_t>> longr(n);  // long-range edges of step 4

  // ---- 4. long-range edges.  Nearest-neighbour edges alone leave one
  // component per well-separated mixture component, and in high dimension
  // pruning rules cannot tell components apart (all points of a component
  // are nearly equidistant).  So: every point gets R/8 seeded random edges to
  // hubs, every hub R/4 random edges to other hubs (an expander over hubs),
  // and the entry's whole list is the hubs in farthest-point order, which
  // visits one hub per separated component before a second one.
  {
    const int Rh = std::max(1, R / 4);
    std::vector<uint8_t> is_hub(n, 0);
    for (int32_t h : hubs) is_hub[h] = 1;
    parallel_for(n, threads, [&](int64_t i) {
      if (i == medoid) return;
      const int want = (int)std::min<int64_t>(is_hub[i] ? Rh : Rn, Hn - (is_hub[i] ? 1 : 0));
      std::vector<int32_t> extra;
      uint64_t s = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(i + 1));
      int guard = 0;
      while ((int)extra.size() < want && guard++ < 64 * want) {
        int32_t h = hubs[splitmix64(s) % (uint64_t)Hn];
        if (h == i || std::find(extra.begin(), extra.end(), h) != extra.end()) continue;
        extra.push_back(h);
      }
      longr[i] = extra;
      std::vector<int32_t> merged;
      const int local = R - (int)extra.size();
      for (int32_t x : out[i]) {
        if ((int)merged.size() >= local) break;
        merged.push_back(x);
      }
      for (int32_t x : extra)
        if ((int)merged.size() < R && std::find(merged.begin(), merged.end(), x) == merged.end())
          merged.push_back(x);
      out[i] = merged;
    });
    // entry: farthest-point order over the hubs, starting from the entry itself
    std::vector<float> mind(Hn);
    for (int64_t a = 0; a < Hn; a++) mind[a] = D.dist(medoid, hubs[a]);
    std::vector<int32_t> eo;
    std::vector<uint8_t> taken(Hn, 0);
    while ((int)eo.size() < R && (int64_t)eo.size() < Hn) {
      int64_t best = -1;
      for (int64_t a = 0; a < Hn; a++)
        if (!taken[a] && hubs[a] != medoid && (best < 0 || mind[a] > mind[best])) best = a;
      if (best < 0) break;
      taken[best] = 1;
      eo.push_back(hubs[best]);
      for (int64_t a = 0; a < Hn; a++) mind[a] = std::min(mind[a], D.dist(hubs[best], hubs[a]));
    }
    longr[medoid] = eo;
    for (int32_t x : out[medoid]) {
      if ((int)eo.size() >= R) break;
      if (std::find(eo.begin(), eo.end(), x) == eo.end()) eo.push_back(x);
    }
    out[medoid] = eo;
  }

  // ---- 5. fill every list to exactly R from the pool (closest first).
  auto fill = [&]() {
    parallel_for(n, threads, [&](int64_t i) {
      auto &o = out[i];
      for (const Cand &c : pools[i]) {
        if ((int)o.size() >= R) break;
        if (c.second != i && std::find(o.begin(), o.end(), c.second) == o.end())
          o.push_back(c.second);
      }
    });
  };
  auto write = [&]() {
    for (int64_t i = 0; i < n; i++) {
      int32_t *row = adj + i * R;
      int m = 0;
      for (int32_t x : out[i])
        if (m < R && x != i) row[m++] = x;
      for (; m < R; m++) row[m] = -1;
    }
  };
  // ---- 6. connectivity repair from the medoid.
  auto repair = [&]() {
    std::vector<uint16_t> rep_used(n, 0);
    for (int round = 0; round < 16; round++) {
      std::vector<uint8_t> seen(n, 0);
      std::vector<int32_t> stack;
      auto bfs_from = [&](int32_t s0) {
        if (seen[s0]) return;
        seen[s0] = 1;
        stack.push_back(s0);
        while (!stack.empty()) {
          int32_t u = stack.back();
          stack.pop_back();
          for (int j = 0; j < R; j++) {
            int32_t x = adj[(int64_t)u * R + j];
            if (x >= 0 && !seen[x]) { seen[x] = 1; stack.push_back(x); }
          }
        }
      };
      bfs_from((int32_t)medoid);
      int64_t repaired = 0;
      for (int64_t x = 0; x < n; x++) {
        if (seen[x]) continue;
        // attach x to its closest reached pool neighbour, else the closest reached hub
        int32_t y = -1;
        for (const Cand &c : pools[x])
          if (seen[c.second]) { y = c.second; break; }
        if (y < 0) {
          float best = INFINITY;
          for (int32_t h : hubs)
            if (seen[h]) {
              float dd = D.dist(x, h);
              if (dd < best) { best = dd; y = h; }
            }
        }
        if (y < 0) y = (int32_t)medoid;
        int32_t *row = adj + (int64_t)y * R;
        int slot = -1;
        for (int j = 0; j < R; j++)
          if (row[j] < 0) { slot = j; break; }
        if (slot < 0) {  // overwrite the farthest slots, a different one per repair
          const int span = std::max(1, R / 2);
          slot = R - 1 - (rep_used[y] % span);
          rep_used[y]++;
        }
        row[slot] = (int32_t)x;
        repaired++;
        bfs_from((int32_t)x);
      }
      if (repaired == 0) break;
    }
  };
  fill();
  write();
  repair();
  progress("pool graph");

  // ---- 7. Vamana-style refinement passes.
  if (passes > 0 && n > 2) {
    const int L_build = std::max(Lb, R);
    std::vector<int32_t> perm(n);
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    {
      uint64_t s2 = seed ^ 0x6A09E667F3BCC909ull;
      for (int64_t i = n - 1; i > 0; i--) std::swap(perm[i], perm[splitmix64(s2) % (uint64_t)(i + 1)]);
    }
    const int64_t B = std::max<int64_t>(1024, n / 128);
    const int T = std::max(1, threads);
    std::vector<std::vector<uint32_t>> stamps(T, std::vector<uint32_t>(n, 0u));
    std::vector<uint32_t> epochs(T, 0u);
    std::vector<std::vector<int32_t>> fresh(B);
    std::vector<std::vector<int32_t>> rev(n);
    // rows as lists, excluding padding
    for (int64_t i = 0; i < n; i++) {
      out[i].clear();
      for (int j = 0; j < R; j++)
        if (adj[i * R + j] >= 0) out[i].push_back(adj[i * R + j]);
    }
    auto is_long = [&](int64_t i, int32_t x) {
      return std::find(longr[i].begin(), longr[i].end(), x) != longr[i].end();
    };
    // prune candidates of point i (sorted, unique, without i) to R edges,
    // its long-range edges kept
    auto prune_keep_long = [&](int64_t i, std::vector<Cand> &c, float a, std::vector<int32_t> &o) {
      std::vector<Cand> local;
      local.reserve(c.size());
      for (const Cand &e : c)
        if (!is_long(i, e.second)) local.push_back(e);
      const int room = R - (int)longr[i].size();
      robust_prune(D, local, std::max(room, 0), a, o);
      for (int32_t x : longr[i])
        if ((int)o.size() < R) o.push_back(x);
    };
    for (int pass = 0; pass < passes; pass++) {
      const float a = 1.0f;
      for (int64_t b0 = 0; b0 < n; b0 += B) {
        const int64_t b1 = std::min(n, b0 + B);
        // searches on the frozen graph (adj)
        std::atomic<int64_t> next(b0);
        auto work = [&](int t) {
          std::vector<Cand> ex, c;
          std::vector<int32_t> o;
          for (;;) {
            const int64_t k = next.fetch_add(1);
            if (k >= b1) break;
            const int64_t p = perm[k];
            if (p == medoid) {
              fresh[k - b0] = out[p];
              continue;
            }
            greedy_expand(D, adj, R, p, (int32_t)medoid, L_build, stamps[t], ++epochs[t], ex);
            c.clear();
            for (const Cand &e : ex)
              if (e.second != p) c.push_back(e);
            for (int32_t x : out[p])
              if (x != p) c.emplace_back(D.dist(p, x), x);
            std::sort(c.begin(), c.end());
            c.erase(std::unique(c.begin(), c.end()), c.end());
            prune_keep_long(p, c, a, o);
            fresh[k - b0] = o;
          }
        };
        {
          std::vector<std::thread> th;
          for (int t = 1; t < T; t++) th.emplace_back(work, t);
          work(0);
          for (auto &x : th) x.join();
        }
        // apply in batch order: new lists, then proposed reverse edges
        std::vector<int32_t> touched;
        for (int64_t k = b0; k < b1; k++) {
          const int64_t p = perm[k];
          out[p] = fresh[k - b0];
          for (int32_t q : out[p]) {
            if (q == medoid || is_long(p, q)) continue;
            if (rev[q].empty()) touched.push_back(q);
            rev[q].push_back((int32_t)p);
          }
        }
        std::sort(touched.begin(), touched.end());
        parallel_for((int64_t)touched.size(), threads, [&](int64_t t) {
          const int32_t q = touched[t];
          std::vector<int32_t> merged = out[q];
          for (int32_t x : rev[q])
            if (x != q && std::find(merged.begin(), merged.end(), x) == merged.end())
              merged.push_back(x);
          if ((int)merged.size() > R) {
            std::vector<Cand> c;
            for (int32_t x : merged) c.emplace_back(D.dist(q, x), x);
            std::sort(c.begin(), c.end());
            std::vector<int32_t> o;
            prune_keep_long(q, c, a, o);
            merged.swap(o);
          }
          out[q] = merged;
        });
        for (int32_t q : touched) rev[q].clear();
        for (int64_t i = b0; i < b1; i++) {
          const int64_t p = perm[i];
          int32_t *row = adj + p * R;
          int m = 0;
          for (int32_t x : out[p])
            if (m < R && x != p) row[m++] = x;
          for (; m < R; m++) row[m] = -1;
        }
        for (int32_t q : touched) {
          int32_t *row = adj + (int64_t)q * R;
          int m = 0;
          for (int32_t x : out[q])
            if (m < R && x != q) row[m++] = x;
          for (; m < R; m++) row[m] = -1;
        }
        const int64_t nb = (n + B - 1) / B, bi = b0 / B + 1;
        if (bi % 16 == 0 || bi == nb) progress("refinement batch", bi, nb);
      }
    }
    fill();
    write();
    repair();
    progress("refined graph");
  }
  return 0;
}

}  // extern "C"

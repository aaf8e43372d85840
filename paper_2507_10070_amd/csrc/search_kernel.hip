// search_kernel.hip -- batched best-first graph search on gfx950 (CDNA4),
// strict or with the dependency-relaxed fetch schedule of FlashANNS
// (arXiv 2507.10070, section 4.1).
//
// One wavefront (64 lanes) runs one query, or each half of a wave runs one
// (G = 32 lanes per query; see "lanes per query" below).  Per query, LDS holds
//   cand[Lcap]  the candidate list: u64 keys (distance << 32 | id), sorted
//               ascending; bit 31 of the id word is the "expanded" flag
//   nk[G]       new keys of the batch being merged, compacted
//   stage[G]    the record being processed (16 B per lane)
//   qbuf        the query, zero-padded to the navigation row stride
//   ids/dsc     per-batch (G neighbours) ids and their distances
//   hash[H]     visited set: exact ids in buckets of 8 slots, may forget
//   fifo[8]     generic schedule: keys of the nodes in flight, oldest first
// Forgetting is harmless: a forgotten node is either still in the list (its
// recomputed key is identical and is dropped as a duplicate) or its key is
// above the current L-th key, which never increases, so it is rejected again.
//
// A search step (section 4.1.1): select the first unexpanded candidate, fetch
// its record (full vector + R neighbour ids), score the unvisited neighbours
// with exact squared L2 against the HBM navigation copy, merge them into the
// list.  With DELAY = 1 the node selected in iteration t is processed in
// iteration t+1, so its record fetch overlaps the gathers, distances and
// merge of the previous node (section 4.1.2).  Selection always happens before
// the previous node's merge, i.e. on the list as of one step earlier.
//
// Distances: u8/i8 exactly as |q|^2 + |x|^2 - 2 q.x with 4-byte dot products
// (v_dot4), f32 as a sum of squared differences in fp32.
//
// Compressed navigation (NAV_PQ; the in-memory quantised vectors of graph
// indexes, paper section 2.2): neighbours are scored by product-quantisation
// codes (one 32 B row per node in HBM), with sub-distances taken from a
// per-query table in LDS or computed from centroids read through the cache,
// so the candidate list is ordered by PQ distance; each expanded node's
// exact distance, from the full-precision vector in its record, goes to a
// sorted result list res[k] in LDS, which is the answer.  The PQ arithmetic
// is fp32 in one fixed order (table entry: fmaf over the subspace's
// dimensions in order; PQ distance: sum over subspaces in order), so the
// list order, and with it the search path, is reproducible exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "search_kernel.h"

namespace fa {

constexpr uint32_t kFlag = 0x80000000u;
constexpr uint64_t kNoKey = 0xFFFFFFFFFFFFFFFFull;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kCplErr = 0x80000000u;   // completion word: read failed
constexpr uint32_t kTimedOut = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t kmask(uint64_t e) { return e & ~(uint64_t)kFlag; }
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Sum over each aligned group of 8 lanes; every lane of the group gets it.
__device__ __forceinline__ int group8_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  return v;
}
__device__ __forceinline__ float group8_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
  return v;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ------------------------------------------------------- lanes per query
// A query runs on a group of G lanes: the whole wave (G = 64), or one half of
// it (G = 32, two queries per wave).  The forms below are the wave-wide
// operations restricted to the caller's group.  A mask holds the group's
// lanes in bits [0, G); a broadcast reads a lane of the caller's own group.
// With G = 64 each is the plain wave operation; with G = 32 the halves may
// follow different paths (each half's control flow depends on its own query
// only), so broadcasts go through ds_bpermute, which takes a per-lane source.
template <int G>
__device__ __forceinline__ int group_lane() {
  return G == 64 ? lane_id() : (lane_id() & (G - 1));
}
template <int G>
__device__ __forceinline__ uint64_t gballot(bool p) {
  const uint64_t b = __ballot(p);
  if constexpr (G == 64) return b;
  else return (lane_id() & 32) ? (b >> 32) : (b & 0xFFFFFFFFull);
}
// Set bits of a group mask below the caller's group lane.
template <int G>
__device__ __forceinline__ uint32_t gmbcnt(uint64_t m) {
  if constexpr (G == 64) return mbcnt(m);
  else return (lane_id() & 32) ? __builtin_amdgcn_mbcnt_hi((uint32_t)m, 0u)
                               : __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u);
}
// Value of x in group lane j (j the same for every lane of the group).
template <int G>
__device__ __forceinline__ uint32_t gread(uint32_t x, int j) {
  if constexpr (G == 64) return (uint32_t)__builtin_amdgcn_readlane((int)x, j);
  else return (uint32_t)__builtin_amdgcn_ds_bpermute(((lane_id() & 32) + j) << 2, (int)x);
}
template <int G>
__device__ __forceinline__ uint64_t gread64(uint64_t x, int j) {
  if constexpr (G == 64) return readlane64(x, j);
  else return ((uint64_t)gread<G>((uint32_t)(x >> 32), j) << 32) | gread<G>((uint32_t)x, j);
}
// Value of x in the group's first lane (every lane of the group active).
template <int G>
__device__ __forceinline__ uint32_t gfirst(uint32_t x) {
  if constexpr (G == 64) return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
  else return gread<G>(x, 0);
}

// Number of entries of a[0..cnt) whose masked key is below `key`.
__device__ __forceinline__ int lower_bound(const uint64_t *a, int cnt, uint64_t key) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kmask(a[mid]) < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Visited set probe: true if x was not recorded (and is recorded now).
// The table is 2^bits slots in buckets of 8 (32 B): one bucket read answers
// the lookup, and x goes into an empty slot of its bucket by compare-and-swap
// (a slot taken meanwhile by another lane moves it to the next one).  A full
// bucket forgets one of its ids, which never changes results (see the head
// of this file); it only lets a node be scored again.
__device__ __forceinline__ bool hash_insert(uint32_t *tab, int bits, uint32_t x) {
  const uint32_t b = (x * 2654435761u) >> (32 - (bits - 3));
  uint32_t *bk = tab + 8 * b;
  const uint4 lo = *(const uint4 *)bk;
  const uint4 hi = *(const uint4 *)(bk + 4);
  if (lo.x == x || lo.y == x || lo.z == x || lo.w == x || hi.x == x || hi.y == x ||
      hi.z == x || hi.w == x)
    return false;
  const uint32_t slots[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
  for (int e = 0; e < 8; e++) {
    if (slots[e] != kEmpty) continue;
    const uint32_t cur = atomicCAS(&bk[e], kEmpty, x);
    if (cur == kEmpty) return true;
    if (cur == x) return false;
  }
  atomicExch(&bk[x & 7u], x);  // bucket full: forget one id
  return true;
}

// ---------------------------------------------------------------- dtypes

template <int DT>
struct Dist;

template <>
struct Dist<DT_U8> {
  // partial = |x|^2 - 2 q.x over this lane's chunks
  __device__ __forceinline__ static int partial(const uint4 q, const uint4 r, int acc) {
    uint32_t qx = 0, xx = 0;
    qx = __builtin_amdgcn_udot4(q.x, r.x, qx, false);
    qx = __builtin_amdgcn_udot4(q.y, r.y, qx, false);
    qx = __builtin_amdgcn_udot4(q.z, r.z, qx, false);
    qx = __builtin_amdgcn_udot4(q.w, r.w, qx, false);
    xx = __builtin_amdgcn_udot4(r.x, r.x, xx, false);
    xx = __builtin_amdgcn_udot4(r.y, r.y, xx, false);
    xx = __builtin_amdgcn_udot4(r.z, r.z, xx, false);
    xx = __builtin_amdgcn_udot4(r.w, r.w, xx, false);
    return acc + (int)xx - 2 * (int)qx;
  }
  __device__ __forceinline__ static int self(const uint4 q, int acc) {
    uint32_t s = 0;
    s = __builtin_amdgcn_udot4(q.x, q.x, s, false);
    s = __builtin_amdgcn_udot4(q.y, q.y, s, false);
    s = __builtin_amdgcn_udot4(q.z, q.z, s, false);
    s = __builtin_amdgcn_udot4(q.w, q.w, s, false);
    return acc + (int)s;
  }
  using Acc = int;
  __device__ __forceinline__ static uint32_t finish(int qq, int sum) { return (uint32_t)(qq + sum); }
};

template <>
struct Dist<DT_I8> {
  __device__ __forceinline__ static int partial(const uint4 q, const uint4 r, int acc) {
    int qx = 0, xx = 0;
    qx = __builtin_amdgcn_sdot4((int)q.x, (int)r.x, qx, false);
    qx = __builtin_amdgcn_sdot4((int)q.y, (int)r.y, qx, false);
    qx = __builtin_amdgcn_sdot4((int)q.z, (int)r.z, qx, false);
    qx = __builtin_amdgcn_sdot4((int)q.w, (int)r.w, qx, false);
    xx = __builtin_amdgcn_sdot4((int)r.x, (int)r.x, xx, false);
    xx = __builtin_amdgcn_sdot4((int)r.y, (int)r.y, xx, false);
    xx = __builtin_amdgcn_sdot4((int)r.z, (int)r.z, xx, false);
    xx = __builtin_amdgcn_sdot4((int)r.w, (int)r.w, xx, false);
    return acc + xx - 2 * qx;
  }
  __device__ __forceinline__ static int self(const uint4 q, int acc) {
    int s = 0;
    s = __builtin_amdgcn_sdot4((int)q.x, (int)q.x, s, false);
    s = __builtin_amdgcn_sdot4((int)q.y, (int)q.y, s, false);
    s = __builtin_amdgcn_sdot4((int)q.z, (int)q.z, s, false);
    s = __builtin_amdgcn_sdot4((int)q.w, (int)q.w, s, false);
    return acc + s;
  }
  using Acc = int;
  __device__ __forceinline__ static uint32_t finish(int qq, int sum) { return (uint32_t)(qq + sum); }
};

template <>
struct Dist<DT_F32> {
  __device__ __forceinline__ static float partial(const uint4 q, const uint4 r, float acc) {
    float t;
    t = __uint_as_float(q.x) - __uint_as_float(r.x); acc = fmaf(t, t, acc);
    t = __uint_as_float(q.y) - __uint_as_float(r.y); acc = fmaf(t, t, acc);
    t = __uint_as_float(q.z) - __uint_as_float(r.z); acc = fmaf(t, t, acc);
    t = __uint_as_float(q.w) - __uint_as_float(r.w); acc = fmaf(t, t, acc);
    return acc;
  }
  __device__ __forceinline__ static float self(const uint4, float acc) { return acc; }
  using Acc = float;
  __device__ __forceinline__ static uint32_t finish(float, float sum) { return __float_as_uint(sum); }
};

// ---------------------------------------------------------------- per wave

struct WaveLds {
  uint64_t *cand;
  uint64_t *nk;
  uint4 *stage;
  uint8_t *qbuf;
  uint32_t *ids;
  uint32_t *dsc;
  uint32_t *hash;
  uint64_t *fifo;
  uint64_t *res;   // NAV_PQ: exact (distance << 32 | id) keys, sorted, up to k
  float *tab;      // NAV_PQ: distance table, pq_m x 256 -- or, when centroids
                   // are read from the cache instead, the query as d floats
};

// One query's LDS region; G lanes per query (batches of G neighbours, a
// record of at most 16 G bytes).
__host__ __device__ inline LdsLayout lds_layout(int Lcap, int nav_stride, int hash_bits,
                                                int kcap, int pq_floats, int G = 64) {
  LdsLayout o;
  uint32_t off = 0;
  o.cand = off; off += 8u * (uint32_t)Lcap;
  o.nk = off; off += 8u * (uint32_t)G;
  o.stage = off; off += 16u * (uint32_t)G;
  o.qbuf = off; off += (uint32_t)nav_stride;
  o.ids = off; off += 4u * (uint32_t)G;
  o.dsc = off; off += 4u * (uint32_t)G;
  o.hash = off; off += 4u << hash_bits;
  o.fifo = off; off += 8u * (uint32_t)kMaxPipe;
  o.res = off; off += 8u * (uint32_t)kcap;
  off = (off + 15u) & ~15u;  // 16 B reads of the query floats
  o.tab = off; off += 4u * (uint32_t)pq_floats;
  o.bytes = (off + 15u) & ~15u;
  return o;
}

// Where one query's vector comes from and where its results go.
struct QueryIO {
  const uint8_t *q;   // nav_stride readable bytes when `coherent`
  bool coherent;      // q is rewritten by host copies and the result rows are
                      // read by the host: system-scope loads and stores
  int32_t *ids;       // row of `width` result ids
  uint32_t *dists;    // row of `width` distances
  uint32_t *steps;    // optional
  int L, k, width;    // list size, results, row width (entries k..width-1 padded)
  int64_t line;       // TR_AGENT: request / completion / staging line
  int32_t *status;    // TR_AGENT: where a failed read is reported (may be host memory)
};

__device__ __forceinline__ QueryIO batch_io(const SearchArgs &A, int64_t qi) {
  QueryIO io;
  io.q = A.queries + qi * (int64_t)A.qbytes;
  io.coherent = false;
  io.ids = A.out_ids + qi * A.k_stride;
  io.dists = (uint32_t *)A.out_dists + qi * A.k_stride;
  io.steps = A.out_steps ? A.out_steps + qi : nullptr;
  int L = A.L, k = A.k;
  if (A.q_L) {
    const int l = A.q_L[qi];
    L = l < 1 ? 1 : (l > A.L ? A.L : l);
  }
  if (A.q_k) {
    const int kk = A.q_k[qi];
    k = kk < 1 ? 1 : (kk > A.k ? A.k : kk);
  }
  io.L = L;
  io.k = k > L ? L : k;
  io.width = A.k_stride;
  io.line = qi;
  io.status = A.status ? A.status + qi : nullptr;
  return io;
}

// Component i of the query in LDS as a float (exact for u8 and i8).
template <int DT>
__device__ __forceinline__ float query_elem(const uint8_t *qbuf, int i) {
  if (DT == DT_U8) return (float)qbuf[i];
  if (DT == DT_I8) return (float)(int8_t)qbuf[i];
  return ((const float *)qbuf)[i];
}

template <int DT, int CPL, int TR, int NAV = NAV_FULL, int G = 64>
struct Searcher {
  using D = Dist<DT>;
  using Acc = typename D::Acc;

  const SearchArgs &A;
  WaveLds S;
  int lane, sub, grp;   // lane within the query's group; 8-lane row group
  uint4 qv[CPL];
  Acc qq;
  int nc;
  int nres;       // NAV_PQ: entries of S.res
  int L, k;       // this query's list size and result count
  QueryIO io;
  int64_t qi;
  uint32_t steps, rows, mismatches;
  uint32_t seq;   // TR_AGENT: last request number of this query
  bool failed;    // TR_AGENT: a record read failed or timed out
  uint32_t sel_id;   // hot-record cache: the last selected node and its cache
  int32_t sel_slot;  // slot, looked up at selection (kEmpty / -1: none)
  unsigned long long t_fetch, t_comp;  // summed phase ticks (strict, optional)

  __device__ __forceinline__ Searcher(const SearchArgs &args, uint8_t *base, int64_t query,
                                      const QueryIO &qio)
      : A(args), io(qio), qi(query) {
    lane = group_lane<G>();
    sub = lane & 7;
    grp = lane >> 3;
    const LdsLayout lay = lds_layout(A.Lcap, A.nav_stride, A.hash_bits,
                                     NAV == NAV_PQ ? A.k : 0, NAV == NAV_PQ ? A.pq_floats : 0, G);
    S.cand = (uint64_t *)(base + lay.cand);
    S.nk = (uint64_t *)(base + lay.nk);
    S.stage = (uint4 *)(base + lay.stage);
    S.qbuf = base + lay.qbuf;
    S.ids = (uint32_t *)(base + lay.ids);
    S.dsc = (uint32_t *)(base + lay.dsc);
    S.hash = (uint32_t *)(base + lay.hash);
    S.fifo = (uint64_t *)(base + lay.fifo);
    S.res = (uint64_t *)(base + lay.res);
    S.tab = (float *)(base + lay.tab);
    L = io.L;
    k = io.k;
    // query -> LDS, zero padded to the row stride
    const uint8_t *q = io.q;
    if (io.coherent) {
      for (int w = lane; w < A.nav_stride / 4; w += G)
        ((uint32_t *)S.qbuf)[w] = __hip_atomic_load((const uint32_t *)q + w, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
      for (int b = lane; b < A.nav_stride; b += G) S.qbuf[b] = b < A.qbytes ? q[b] : (uint8_t)0;
    }
    for (int s = lane; s < (1 << A.hash_bits); s += G) S.hash[s] = kEmpty;
    __builtin_amdgcn_wave_barrier();
    Acc a = Acc(0);
#pragma unroll
    for (int c = 0; c < CPL; c++) {
      qv[c] = *(const uint4 *)(S.qbuf + 16 * (sub + 8 * c));
      a = D::self(qv[c], a);
    }
    qq = group8_sum(a);
    nres = 0;
    if (NAV == NAV_PQ && A.pq_direct) {
      // centroids read from the cache per scored code: the query as floats
      for (int i = lane; i < A.pq_m * A.pq_dsub; i += G) S.tab[i] = query_elem<DT>(S.qbuf, i);
      __builtin_amdgcn_wave_barrier();
    } else if (NAV == NAV_PQ) {
      // distance table: entry m*256 + c is the squared distance of query
      // subspace m to centroid c (fmaf over its dimensions in order)
      const int ds = A.pq_dsub;
      for (int e = lane; e < A.pq_m * kPqKsub; e += G) {
        const int q0 = (e >> 8) * ds;
        const float *c = A.pq_cb + (int64_t)e * ds;
        float acc = 0.0f;
        for (int j = 0; j < ds; j++) {
          const float t = query_elem<DT>(S.qbuf, q0 + j) - c[j];
          acc = fmaf(t, t, acc);
        }
        S.tab[e] = acc;
      }
      __builtin_amdgcn_wave_barrier();
    }
    steps = rows = mismatches = 0;
    // request numbers continue per line when lines outlive queries
    seq = A.line_seq ? A.line_seq[io.line] : 0u;
    failed = false;
    sel_id = kEmpty;
    sel_slot = -1;
    t_fetch = t_comp = 0;
  }

  // Wall-clock stamp after every outstanding memory operation of the wave
  // has completed (phase accounting only; not used on the timed path).
  __device__ __forceinline__ unsigned long long stamp() const {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    const unsigned long long t = __builtin_amdgcn_s_memrealtime();
    __builtin_amdgcn_sched_barrier(0);
    return t;
  }

  // Distance of the query to the row at `p` (all 8 lanes of a group call).
  __device__ __forceinline__ uint32_t row_dist(const uint8_t *p) const {
    Acc a = Acc(0);
#pragma unroll
    for (int c = 0; c < CPL; c++) {
      const uint4 r = *(const uint4 *)(p + 16 * (sub + 8 * c));
      a = D::partial(qv[c], r, a);
    }
    return D::finish(qq, group8_sum(a));
  }

  // Squared distance of query subspace m (floats in S.tab) to centroid c,
  // read from the codebook: fmaf over the subspace's dimensions in order --
  // the same value as table entry m*256 + c.
  __device__ __forceinline__ float pq_sub_direct(int m, uint32_t c) const {
    const int ds = A.pq_dsub;
    const float *q = S.tab + m * ds;
    const float *cc = A.pq_cb + ((int64_t)m * kPqKsub + c) * ds;
    float acc = 0.0f;
    for (int j = 0; j < ds; j++) {
      const float t = q[j] - cc[j];
      acc = fmaf(t, t, acc);
    }
    return acc;
  }

  // PQ distance of a code row held in two 16 B registers: the sub-distances
  // of its pq_m bytes (table entries, or computed from the codebook) summed
  // in subspace order.
  // Code word I (bytes 4I..4I+3) of a code row held in two registers.
  template <int I>
  __device__ __forceinline__ static uint32_t code_word(const uint4 c0, const uint4 c1) {
    if constexpr (I == 0) return c0.x;
    else if constexpr (I == 1) return c0.y;
    else if constexpr (I == 2) return c0.z;
    else if constexpr (I == 3) return c0.w;
    else if constexpr (I == 4) return c1.x;
    else if constexpr (I == 5) return c1.y;
    else if constexpr (I == 6) return c1.z;
    else return c1.w;
  }

  // Centroid loads of subspaces [GI*SG, GI*SG + SG), d/M = DS in {4, 8},
  // SG = 32 / DS (8 x 16 B per lane); every index a compile-time constant.
  template <int DS, int GI>
  __device__ __forceinline__ void pq_load(const uint4 c0, const uint4 c1,
                                          float4 (&v)[32 / DS][DS / 4]) const {
    constexpr int SG = 32 / DS;
#pragma unroll
    for (int u = 0; u < SG; u++) {
      const int m = GI * SG + u;
      const int mm = m < A.pq_m ? m : A.pq_m - 1;  // past pq_m: a valid row, unused
      uint32_t w;
      if ((u >> 2) == 0) w = code_word<(GI * SG) / 4>(c0, c1);
      else w = code_word<(GI * SG) / 4 + ((SG - 1) >> 2)>(c0, c1);
      const uint32_t c = (w >> (8 * (m & 3))) & 0xFFu;
      const float4 *cc = (const float4 *)(A.pq_cb + ((int64_t)mm * kPqKsub + c) * DS);
#pragma unroll
      for (int h = 0; h < DS / 4; h++) v[u][h] = cc[h];
    }
  }

  // s += the sub-distances of subspaces [GI*SG, GI*SG + SG) in subspace order.
  template <int DS, int GI>
  __device__ __forceinline__ float pq_add(const float4 (&v)[32 / DS][DS / 4], float s) const {
    constexpr int SG = 32 / DS;
#pragma unroll
    for (int u = 0; u < SG; u++) {
      if (GI * SG + u < A.pq_m) {
        const float4 *q = (const float4 *)(S.tab + (GI * SG + u) * DS);
        float acc = 0.0f, t;
#pragma unroll
        for (int h = 0; h < DS / 4; h++) {
          const float4 qq = q[h];
          t = qq.x - v[u][h].x; acc = fmaf(t, t, acc);
          t = qq.y - v[u][h].y; acc = fmaf(t, t, acc);
          t = qq.z - v[u][h].z; acc = fmaf(t, t, acc);
          t = qq.w - v[u][h].w; acc = fmaf(t, t, acc);
        }
        s += acc;
      }
    }
    return s;
  }

  // Group GI is loaded (cur): issue the loads of group GI+1, then add group
  // GI, so that one group's loads are in flight during the other's FMAs.
  template <int DS, int GI>
  __device__ __forceinline__ float pq_pipe(const uint4 c0, const uint4 c1, float s,
                                           const float4 (&cur)[32 / DS][DS / 4]) const {
    constexpr int SG = 32 / DS;
    if constexpr ((GI + 1) * SG < kPqMaxM) {
      if ((GI + 1) * SG < A.pq_m) {
        float4 nxt[SG][DS / 4];
        pq_load<DS, GI + 1>(c0, c1, nxt);
        s = pq_add<DS, GI>(cur, s);
        return pq_pipe<DS, GI + 1>(c0, c1, s, nxt);
      }
    }
    return pq_add<DS, GI>(cur, s);
  }

  template <int DS>
  __device__ __forceinline__ float pq_sum_direct(const uint4 c0, const uint4 c1) const {
    float4 v[32 / DS][DS / 4];
    pq_load<DS, 0>(c0, c1, v);
    return pq_pipe<DS, 0>(c0, c1, 0.0f, v);
  }

  __device__ __forceinline__ float pq_sum(const uint4 c0, const uint4 c1) const {
    float s = 0.0f;
    if (A.pq_direct && A.pq_dsub == 4) return pq_sum_direct<4>(c0, c1);
    if (A.pq_direct && A.pq_dsub == 8) return pq_sum_direct<8>(c0, c1);
    if (A.pq_direct) {
      // other d/M: not unrolled; the word of subspace m is picked by selects
      // on the wave-uniform m (an indexed register array would live in scratch)
      for (int m = 0; m < A.pq_m; m++) {
        const int i = m >> 2;
        uint32_t w = c0.x;
        w = i == 1 ? c0.y : w;
        w = i == 2 ? c0.z : w;
        w = i == 3 ? c0.w : w;
        w = i == 4 ? c1.x : w;
        w = i == 5 ? c1.y : w;
        w = i == 6 ? c1.z : w;
        w = i == 7 ? c1.w : w;
        s += pq_sub_direct(m, (w >> (8 * (m & 3))) & 0xFFu);
      }
      return s;
    }
    const uint32_t w[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
    for (int m = 0; m < kPqMaxM; m++) {
      if (m < A.pq_m) s += S.tab[m * kPqKsub + ((w[m >> 2] >> (8 * (m & 3))) & 0xFFu)];
    }
    return s;
  }

  __device__ __forceinline__ float pq_dist(uint32_t id) const {
    const uint4 *p = (const uint4 *)(A.pq_codes + (int64_t)id * kPqStride);
    return pq_sum(p[0], p[1]);
  }

  __device__ __forceinline__ void init_entry() {
    const uint32_t e = (uint32_t)A.entry;
    uint32_t dist;
    if (NAV == NAV_PQ) dist = __float_as_uint(pq_dist(e));
    else dist = row_dist(A.nav + (int64_t)e * A.nav_stride);
    if (lane == 0) {
      S.cand[0] = ((uint64_t)dist << 32) | e;
      hash_insert(S.hash, A.hash_bits, e);
    }
    nc = 1;
    __builtin_amdgcn_wave_barrier();
  }

  // First unexpanded candidate: marks it and returns its key (kNoKey if none).
  // A correct search expands each node at most once; the cap at n expansions
  // guarantees termination regardless.
  __device__ __forceinline__ uint64_t select() {
    if ((int64_t)steps >= A.n || failed) return kNoKey;
    for (int base = 0; base < nc; base += G) {
      const int i = base + lane;
      const bool un = i < nc && !((uint32_t)S.cand[i] & kFlag);
      const uint64_t b = gballot<G>(un);
      if (b) {
        const int idx = base + __ffsll((unsigned long long)b) - 1;
        const uint64_t key = S.cand[idx];
        if (A.cache_map) {
          // the cache slot of the node whose record is fetched next, loaded
          // now so that the fetch does not wait for it behind the gathers
          sel_id = (uint32_t)key & ~kFlag;
          sel_slot = A.cache_map[sel_id];
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
          S.cand[idx] = key | kFlag;
          if (A.trace && steps < (uint32_t)A.trace_cap)
            A.trace[qi * A.trace_cap + steps] = (int32_t)((uint32_t)key & ~kFlag);
        }
        __builtin_amdgcn_wave_barrier();
        steps++;
        return key;
      }
    }
    return kNoKey;
  }

  // Record fetch: lane i loads bytes [16i, 16i+16) of the record.  Lanes past
  // the record re-read its last chunk, so the load has no branch around it
  // and the compiler can count it exactly when it places its waits.  With a
  // hot-record cache, a cached node's copy in device memory is read instead
  // (same bytes); the slot of the last selected node was looked up at
  // selection, any other node's (the generic schedule's FIFO) is looked up here.
  __device__ __forceinline__ uint4 fetch(uint32_t v) const {
    const int c = lane < A.rec_chunks ? lane : A.rec_chunks - 1;
    const uint8_t *rec = A.records + (int64_t)v * A.slot;
    if (A.cache_map) {
      const int32_t s = cache_slot(v);
      if (s >= 0) rec = A.cache + (int64_t)s * A.slot;
    }
    return *(const uint4 *)(rec + 16 * c);
  }

  // Hot-record cache slot of node v (-1: not cached); only with a cache.
  __device__ __forceinline__ int32_t cache_slot(uint32_t v) const {
    int32_t s = sel_slot;
    if (v != sel_id) s = A.cache_map[v];
    return s;
  }

  // Request slot of request number s (TR_AGENT).  At most pslots requests of
  // a query are in flight, and they are consumed in order, so request s
  // reuses the slot of request s - pslots, which was consumed already.
  __device__ __forceinline__ uint32_t pslot(uint32_t s) const {
    return s % (uint32_t)A.pslots;
  }

  // Request numbers run 1, 2, ..., M, 1, 2, ... with M the largest multiple
  // of pslots below 2^30: 0 stays "no request", bit 31 of a completion word
  // stays free for the error flag, and s % pslots stays continuous across the
  // wrap.  The host agents step through the same sequence.
  __device__ __forceinline__ uint32_t next_seq(uint32_t s) const {
    const uint32_t M = (0x40000000u / (uint32_t)A.pslots) * (uint32_t)A.pslots;
    return s >= M ? 1u : s + 1u;
  }

  // Start obtaining the record of v.  TR_DIRECT: the load itself (in flight
  // until used); `real` is ignored so that the load is unconditional.
  // TR_AGENT: post request seq+1 for v as one 64-bit system-scope store of
  // (v << 32 | seq) into the query's request slot, then continue; the
  // returned handle carries the sequence number.  The store needs no
  // release: the slot's previous request was consumed (its staged bytes
  // loaded and written to LDS) before this point, so the agent cannot
  // overwrite data the wave still reads.
  // TR_AGENT with a hot-record cache: a cached node posts no request; its
  // handle carries the cache slot + 1 in .y and consume() reads the copy.
  __device__ __forceinline__ uint4 issue(uint32_t v, bool real) {
    if (TR == TR_DIRECT) return fetch(v);
    if (!real || failed) return make_uint4(0, 0, 0, 0);
    if (A.cache_map) {
      const int32_t cs = cache_slot(v);
      if (cs >= 0) return make_uint4(0, (uint32_t)cs + 1u, 0, 0);
    }
    seq = next_seq(seq);
    if (lane == 0)
      __hip_atomic_store(A.req + 8 * io.line + pslot(seq), ((uint64_t)v << 32) | seq, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    return make_uint4(seq, 0, 0, 0);
  }

  // Finish obtaining a record.  TR_AGENT: lane 0 polls the slot's completion
  // word (system-scope acquire, bounded by spin_limit), then every lane
  // reads its 16 B of the staging slot.  A failed or timed-out read ends the
  // query with a status code.
  __device__ __forceinline__ uint4 consume(uint4 h) {
    if (TR == TR_DIRECT) return h;
    if (failed) return make_uint4(0, 0, 0, 0);
    if (h.y) {  // a cached record: read its copy in device memory
      const int ch = lane < A.rec_chunks ? lane : A.rec_chunks - 1;
      return *(const uint4 *)(A.cache + (int64_t)(h.y - 1u) * A.slot + 16 * ch);
    }
    const uint32_t s = h.x;
    if (s == 0) return make_uint4(0, 0, 0, 0);
    uint32_t c = 0;
    if (lane == 0) {
      const uint32_t *w = A.cpl + 16 * io.line + pslot(s);
      uint32_t spins = 0, nap = 1;
      for (;;) {
        c = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if ((c & ~kCplErr) == s) break;
        if (++spins > A.spin_limit) {
          c = kTimedOut;
          break;
        }
        // back off, doubling up to poll_nap x 1024 cycles (~14 us by
        // default): thousands of waiting waves must not flood the host link
        // with polls, which compete with the staged records' reads
        for (uint32_t i = 0; i < nap; i++) __builtin_amdgcn_s_sleep(16);
        nap = nap < A.poll_nap ? nap * 2 : A.poll_nap;
      }
    }
    c = gfirst<G>(c);
    if (c == kTimedOut || (c & kCplErr)) {
      failed = true;
      if (lane == 0 && io.status)
        __hip_atomic_store(io.status, c == kTimedOut ? -110 : -5, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      return make_uint4(0, 0, 0, 0);
    }
    // The staged bytes are read with system-scope loads, issued after the
    // completion word was seen; they bypass the GPU caches, so no acquire
    // fence (which would invalidate the whole L2 on every record) is needed.
    // Two 8 B loads per lane: each instruction reads the record's lines once
    // (four 4 B loads would cross the host link four times per line).
    const int ch = lane < A.rec_chunks ? lane : A.rec_chunks - 1;
    const uint64_t *src =
        (const uint64_t *)(A.stage + (io.line * A.pslots + pslot(s)) * A.stage_stride + 16 * ch);
    const uint64_t lo = __hip_atomic_load(src + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const uint64_t hi = __hip_atomic_load(src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
  }

  // Part 1 of processing node u: stage its record (false if it failed).
  __device__ __forceinline__ bool stage(uint4 h) {
    const uint4 rec = consume(h);
    if (TR == TR_AGENT && failed) return false;
    if (lane < A.rec_chunks) S.stage[lane] = rec;
    __builtin_amdgcn_wave_barrier();
    return true;
  }

  // Neighbours [b0, b0+G) of the staged record: visited filter and
  // compaction.  Returns the number of new ids (written to S.ids).
  __device__ __forceinline__ int filter(int b0) {
    const int j = b0 + lane;
    int32_t x = -1;
    if (j < A.R) x = ((const int32_t *)((const uint8_t *)S.stage + A.ids_off))[j];
    bool fresh = false;
    if (x >= 0 && (int64_t)x < A.n) fresh = hash_insert(S.hash, A.hash_bits, (uint32_t)x);
    const uint64_t m = gballot<G>(fresh);
    if (fresh) S.ids[gmbcnt<G>(m)] = (uint32_t)x;
    __builtin_amdgcn_wave_barrier();
    return __popcll((unsigned long long)m);
  }

  // Gather + distances of rows [p0, p0 + RPP*PB) of S.ids[0..m): RPP = G/8
  // rows per pass, 8 lanes per row, the loads of all PB passes issued before
  // the first reduction.  Rows past m re-read row 0 so that no load sits under a
  // branch.  WITH_FETCH issues the record fetch of `fid` into `frec` right
  // after the gathers, in straight-line code, so the compiler's wait before
  // each pass leaves that fetch in flight.
  static constexpr int PB = (8 / CPL) > 0 ? (8 / CPL) : 1;
  static constexpr int RPP = G / 8;

  template <bool WITH_FETCH>
  __device__ __forceinline__ void gather_block(int m, int p0, uint32_t fid, bool freal,
                                               uint4 &frec) {
    uint4 r[PB][CPL];
#pragma unroll
    for (int pb = 0; pb < PB; pb++) {
      const int row = p0 + RPP * pb + grp;
      const uint8_t *p = A.nav + (int64_t)S.ids[row < m ? row : 0] * A.nav_stride;
#pragma unroll
      for (int c = 0; c < CPL; c++) r[pb][c] = *(const uint4 *)(p + 16 * (sub + 8 * c));
    }
    if (WITH_FETCH) frec = issue(fid, freal);
#pragma unroll
    for (int pb = 0; pb < PB; pb++) {
      const int row = p0 + RPP * pb + grp;
      Acc a = Acc(0);
#pragma unroll
      for (int c = 0; c < CPL; c++) a = D::partial(qv[c], r[pb][c], a);
      const uint32_t dist = D::finish(qq, group8_sum(a));
      if (row < m && sub == 0) S.dsc[row] = dist;
    }
  }

  // NAV_PQ scoring of S.ids[0..m) (m <= 64): one neighbour per lane, its
  // 32 B code row in two loads, then pq_m sub-distances (pq_sum).  Lanes past m re-read
  // row 0 so that no load sits under a branch; WITH_FETCH issues the record
  // fetch after the code loads, as gather_block does.
  template <bool WITH_FETCH>
  __device__ __forceinline__ void gather_pq(int m, uint32_t fid, bool freal, uint4 &frec) {
    const uint32_t id = S.ids[lane < m ? lane : 0];
    const uint4 *p = (const uint4 *)(A.pq_codes + (int64_t)id * kPqStride);
    const uint4 c0 = p[0], c1 = p[1];
    if (WITH_FETCH) frec = issue(fid, freal);
    const float d = pq_sum(c0, c1);
    if (lane < m) S.dsc[lane] = __float_as_uint(d);
  }

  // Merge the m scored ids into the candidate list (first L of the union).
  // Keys at or above the L-th key of a full list cannot enter it: one
  // broadcast read drops them (most keys, late in a search).  The rest are
  // checked against the list (binary search: duplicate, or rank r >= L) and
  // compacted to the first lanes with their rank.  No sort is needed: a new
  // key lands at r + (new keys below it), an old entry at i + (new keys below
  // it), both counted with broadcast reads of the compacted keys.
  __device__ __forceinline__ void merge(int m) {
    uint64_t key = kNoKey;
    if (lane < m) key = ((uint64_t)S.dsc[lane] << 32) | S.ids[lane];
    if (nc >= L && key != kNoKey && key >= kmask(S.cand[L - 1])) key = kNoKey;
    int r = 0;
    if (key != kNoKey) {
      r = lower_bound(S.cand, nc, key);
      const bool dup = r < nc && kmask(S.cand[r]) == key;
      if (dup || r >= L) key = kNoKey;
    }
    uint64_t live = gballot<G>(key != kNoKey);
    if (live == 0) return;
    int cnt, below;
    for (;;) {
      // compact (key, r) into lanes [0, cnt); S.ids is free once the keys are built
      cnt = __popcll((unsigned long long)live);
      __builtin_amdgcn_wave_barrier();
      if (key != kNoKey) {
        const uint32_t p = gmbcnt<G>(live);
        S.nk[p] = key;
        S.ids[p] = (uint32_t)r;
      }
      __builtin_amdgcn_wave_barrier();
      key = lane < cnt ? S.nk[lane] : kNoKey;
      r = lane < cnt ? (int)S.ids[lane] : 0;
      // rank among the new keys; an equal key in a lower lane is a duplicate
      // (possible only when a forgotten id occurs twice in one neighbour list)
      below = 0;
      bool dupl = false;
      for (int j = 0; j < cnt; j++) {
        const uint64_t kj = S.nk[j];
        below += kj < key ? 1 : 0;
        dupl |= (kj == key) && (j < lane);
      }
      dupl = dupl && lane < cnt;
      const uint64_t drop = gballot<G>(dupl);
      if (drop == 0) break;
      if (dupl) key = kNoKey;
      live = gballot<G>(key != kNoKey);
    }
    // old entries move right by the number of smaller new keys; walk chunks
    // from the top so that no unread entry is overwritten
    const int nchunks = (nc + G - 1) / G;
    for (int t = nchunks - 1; t >= 0; t--) {
      const int i = G * t + lane;
      uint64_t e = 0;
      int pos = L;
      if (i < nc) {
        e = S.cand[i];
        const uint64_t ek = kmask(e);
        int shift = 0;
        for (int j = 0; j < cnt; j++) shift += S.nk[j] < ek ? 1 : 0;
        pos = i + shift;
      }
      __builtin_amdgcn_wave_barrier();
      if (i < nc && pos < L) S.cand[pos] = e;
      __builtin_amdgcn_wave_barrier();
    }
    if (lane < cnt && r + below < L) S.cand[r + below] = key;
    nc = nc + cnt < L ? nc + cnt : L;
    __builtin_amdgcn_wave_barrier();
  }

  // merge() for lists of at most E * G entries: the list is held in registers,
  // entry i in group lane i % G of register i / G, so every comparison is a
  // register compare and a ballot.  The new keys are visited in lane order;
  // key j is dropped if it equals a list entry or ranks at L or beyond, else
  // it survives (and later equal keys are dropped).  A survivor lands at
  // (list entries below it) + (survivors below it); a list entry moves right
  // by the survivors below it.
  template <int E>
  __device__ __forceinline__ void merge_reg(int m) {
    uint64_t cf[E], c[E];  // entries with their flags; masked keys
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int i = G * e + lane;
      cf[e] = i < nc ? S.cand[i] : kNoKey;
      c[e] = i < nc ? kmask(cf[e]) : kNoKey;
    }
    uint64_t key = kNoKey;
    if (lane < m) key = ((uint64_t)S.dsc[lane] << 32) | S.ids[lane];
    if (nc >= L) {
      uint64_t last = c[0];
#pragma unroll
      for (int e = 1; e < E; e++) last = (L - 1) / G == e ? c[e] : last;
      if (key >= gread64<G>(last, (L - 1) % G)) key = kNoKey;
    }
    uint64_t todo = gballot<G>(key != kNoKey);
    if (todo == 0) return;
    int shift[E], below = 0, r = 0;
#pragma unroll
    for (int e = 0; e < E; e++) shift[e] = 0;
    uint64_t taken = 0;
    while (todo) {
      const int j = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1;
      const uint64_t kj = gread64<G>(key, j);
      bool listed = false;
#pragma unroll
      for (int e = 0; e < E; e++) listed |= c[e] == kj;
      if (gballot<G>(listed) != 0) continue;                // already listed
      int rj = 0;
#pragma unroll
      for (int e = 0; e < E; e++) rj += __popcll((unsigned long long)gballot<G>(c[e] < kj));
      if (rj >= L) continue;                                 // beyond the first L
      todo &= ~gballot<G>(key == kj);                        // later equal keys
      taken |= 1ull << j;
      if (lane == j) r = rj;
#pragma unroll
      for (int e = 0; e < E; e++) shift[e] += kj < c[e] ? 1 : 0;
      below += kj < key ? 1 : 0;
    }
    const bool surv = (taken >> lane) & 1ull;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int i = G * e + lane;
      if (i < nc && i + shift[e] < L) S.cand[i + shift[e]] = cf[e];
    }
    if (surv && r + below < L) S.cand[r + below] = key;
    const int added = __popcll((unsigned long long)taken);
    nc = nc + added < L ? nc + added : L;
    __builtin_amdgcn_wave_barrier();
  }

  // Optional check: the record's own vector gives the same distance as the
  // node's key (the record holds the full-precision vector).
  __device__ __forceinline__ void check_record(uint64_t key) {
    Acc a = Acc(0);
    if (grp == 0) {
#pragma unroll
      for (int c = 0; c < CPL; c++) {
        const int chunk = sub + 8 * c;
        uint4 r = make_uint4(0, 0, 0, 0);
        if (16 * chunk < A.vec_pad) r = S.stage[chunk];
        a = D::partial(qv[c], r, a);
      }
    }
    const uint32_t dist = D::finish(qq, group8_sum(a));
    if (dist != (uint32_t)(key >> 32)) mismatches++;
  }

  // NAV_PQ: the staged record's vector gives the node's exact distance,
  // which enters the sorted result list (first k by (distance, id)).
  __device__ __forceinline__ void rerank(uint64_t key) {
    Acc a = Acc(0);
    if (grp == 0) {
#pragma unroll
      for (int c = 0; c < CPL; c++) {
        const int chunk = sub + 8 * c;
        uint4 r = make_uint4(0, 0, 0, 0);
        if (16 * chunk < A.vec_pad) r = S.stage[chunk];
        a = D::partial(qv[c], r, a);
      }
    }
    const uint32_t dist = gfirst<G>(D::finish(qq, group8_sum(a)));
    res_insert(((uint64_t)dist << 32) | ((uint32_t)key & ~kFlag));
  }

  // Insert a wave-uniform key into S.res[0..nres), capacity k: entries at
  // and above its rank move up one (the last drops out of a full list).
  __device__ __forceinline__ void res_insert(uint64_t key) {
    if (nres >= k && key >= S.res[k - 1]) return;
    int pos = 0;
    bool dup = false;
    for (int b = 0; b < nres; b += G) {
      const int i = b + lane;
      const uint64_t e = i < nres ? S.res[i] : kNoKey;
      pos += __popcll((unsigned long long)gballot<G>(e < key));
      dup |= gballot<G>(e == key) != 0;
    }
    if (dup) return;
    const int top = nres < k ? nres : k - 1;  // entries [pos, top) move to [pos+1, top+1)
    for (int t = (top - 1) / G; t >= 0 && G * t + G - 1 >= pos; t--) {
      const int i = G * t + lane;
      const bool mv = i >= pos && i < top;
      uint64_t e = 0;
      if (mv) e = S.res[i];
      __builtin_amdgcn_wave_barrier();
      if (mv) S.res[i + 1] = e;
      __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) S.res[pos] = key;
    nres = nres < k ? nres + 1 : k;
    __builtin_amdgcn_wave_barrier();
  }

  // Gather blocks the caller scores before finish_batch: NAV_FULL one block
  // of RPP * PB rows, NAV_PQ the whole batch.
  static constexpr int kFirst = NAV == NAV_PQ ? G : RPP * PB;

  // Score and merge the m new neighbours of one filtered batch, starting at
  // gather block p_start (earlier blocks were done by the caller).
  __device__ __forceinline__ void finish_batch(int m, int p_start) {
    uint4 unused;
    if (NAV == NAV_PQ) {
      if (p_start == 0) gather_pq<false>(m, 0u, false, unused);
    } else {
      for (int p0 = p_start; p0 < m; p0 += RPP * PB) gather_block<false>(m, p0, 0u, false, unused);
    }
    __builtin_amdgcn_wave_barrier();
    rows += (uint32_t)m;
    if (L <= G) merge_reg<1>(m);
    else if (G == 32 && L <= 64) merge_reg<2>(m);
    else merge(m);
  }

  // Process node u whose record handle is `rec`: stage, filter, gather,
  // merge.  RELAXED: exactly one record fetch (of `fid`, into `frec`) is
  // issued, right after the first block of gathers (straight-line code, so the
  // waits before the distance passes leave it in flight), or at once if the
  // first batch has no new neighbour.  `freal` is false for an empty slot.
  template <bool RELAXED>
  __device__ __forceinline__ void process(uint64_t ukey, uint4 rec, uint32_t fid, bool freal,
                                          uint4 &frec) {
    if (!stage(rec)) return;
    process_staged<RELAXED>(ukey, fid, freal, frec);
  }

  // The part of process() after the record is staged in LDS.
  template <bool RELAXED>
  __device__ __forceinline__ void process_staged(uint64_t ukey, uint32_t fid, bool freal,
                                                 uint4 &frec) {
    if (NAV == NAV_PQ) rerank(ukey);
    else if (A.stats) check_record(ukey);
    const int m = filter(0);
    if (m > 0) {
      if (NAV == NAV_PQ) gather_pq<RELAXED>(m, fid, freal, frec);
      else gather_block<RELAXED>(m, 0, fid, freal, frec);
      finish_batch(m, kFirst);
    } else if (RELAXED) {
      frec = issue(fid, freal);
    }
    for (int b0 = G; b0 < A.R; b0 += G) {
      const int mb = filter(b0);
      if (mb > 0) finish_batch(mb, 0);
    }
  }

  __device__ __forceinline__ void finish_query() {
    const uint64_t *out = NAV == NAV_PQ ? S.res : S.cand;
    const int nout = NAV == NAV_PQ ? nres : nc;
    for (int j = lane; j < io.width; j += G) {
      int32_t id = -1;
      uint32_t dist = DT == DT_F32 ? 0x7F800000u : 0xFFFFFFFFu;
      if (j < nout && j < k && !failed) {
        const uint64_t e = out[j];
        id = (int32_t)((uint32_t)e & ~kFlag);
        dist = (uint32_t)(e >> 32);
      }
      if (io.coherent) {
        // host rows read by the host once a done word follows: write-through
        // system-scope stores, so that waiting for them to complete orders
        // them before that word
        __hip_atomic_store(io.ids + j, id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(io.dists + j, dist, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      } else {
        io.ids[j] = id;
        io.dists[j] = dist;
      }
    }
    if (lane == 0) {
      if (A.line_seq) A.line_seq[io.line] = seq;
      if (io.steps) {
        if (io.coherent)
          __hip_atomic_store(io.steps, steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        else
          *io.steps = steps;
      }
      if (A.stats) {
        atomicAdd(&A.stats[0], (unsigned long long)steps);
        atomicAdd(&A.stats[1], (unsigned long long)rows);
        atomicAdd(&A.stats[2], (unsigned long long)mismatches);
      }
    }
  }
};

// Strict and relaxed drivers.  The relaxed loop is unrolled twice so the two
// in-flight record registers have static names; a slot whose id word holds
// kNoKey is an empty pipeline slot.
// One query, start to finish, in the wave's LDS region.
template <int DT, int CPL, int DELAY, int TR, int NAV = NAV_FULL, int G = 64>
__device__ __forceinline__ void run_query(const SearchArgs &A, uint8_t *lds, int64_t qi,
                                          const QueryIO &io) {
  const unsigned long long t_start = A.times ? __builtin_amdgcn_s_memrealtime() : 0ull;
  Searcher<DT, CPL, TR, NAV, G> s(A, lds, qi, io);
  s.init_entry();
  if (DELAY == SCHED_GENERIC) {
    // Any staleness delta and beam width W (section 4.1.2, with W nodes taken
    // per step): each iteration selects up to W unexpanded candidates into
    // the FIFO of in-flight nodes, then processes the oldest while more than
    // delta * W are in flight -- or the oldest min(W, in flight) when nothing
    // was selected.  TR_AGENT posts each request when its node is selected,
    // so up to (delta + 1) * W reads of one query are in flight at once.
    // TR_DIRECT loads the record of the next node in the FIFO while the
    // current one is scored (in-order memory counters allow one such load to
    // overlap the gathers that follow it).
    const int W = A.beam, lim = A.delay * A.beam;
    const uint32_t dummy = (uint32_t)A.entry;
    int head = 0, len = 0;
    uint32_t cseq = s.seq;  // TR_AGENT: request number of the last one consumed
    uint4 nxt = make_uint4(0, 0, 0, 0);
    bool have_nxt = false;
    for (;;) {
      int nsel = 0;
      while (nsel < W) {
        const uint64_t v = s.select();
        if (v == kNoKey) break;
        if (s.lane == 0) s.S.fifo[(head + len) & (kMaxPipe - 1)] = v;
        if (TR == TR_AGENT) (void)s.issue((uint32_t)v & ~kFlag, true);
        len++;
        nsel++;
      }
      __builtin_amdgcn_wave_barrier();
      if (nsel == 0 && len == 0) break;
      int todo = len > lim ? len - lim : 0;
      if (nsel == 0 && todo == 0) todo = len < W ? len : W;
      for (; todo > 0; todo--) {
        const uint64_t u = s.S.fifo[head];
        head = (head + 1) & (kMaxPipe - 1);
        len--;
        if (TR == TR_DIRECT) {
          const bool more = len > 0;
          const uint32_t fid = more ? ((uint32_t)s.S.fifo[head] & ~kFlag) : dummy;
          uint4 rec;
          if (have_nxt) rec = nxt;
          else rec = s.fetch((uint32_t)u & ~kFlag);
          s.template process<true>(u, rec, fid, more, nxt);
          have_nxt = more;
        } else {
          // the node's request was posted at selection unless it is cached
          // (the same lookup decides both times: the cache does not change
          // during a search)
          uint4 unused, h;
          const int32_t cs = s.A.cache_map ? s.A.cache_map[(uint32_t)u & ~kFlag] : -1;
          if (cs >= 0) {
            h = make_uint4(0, (uint32_t)cs + 1u, 0, 0);
          } else {
            cseq = s.next_seq(cseq);
            h = make_uint4(cseq, 0, 0, 0);
          }
          s.template process<false>(u, h, 0u, false, unused);
        }
      }
    }
  } else if (DELAY == SCHED_STRICT) {
    uint4 unused = make_uint4(0, 0, 0, 0);
    if (A.phases) {
      // the same steps with a stamp at issue, after staging and after merge:
      // fetch time (issue -> record in LDS) and compute time (filter,
      // gathers, distances, merge) per expansion, summed per query
      for (;;) {
        const uint64_t v = s.select();
        if (v == kNoKey) break;
        const unsigned long long t0 = s.stamp();
        const uint4 rec = s.issue((uint32_t)v & ~kFlag, true);
        if (!s.stage(rec)) break;
        const unsigned long long t1 = s.stamp();
        s.template process_staged<false>(v, 0u, false, unused);
        const unsigned long long t2 = s.stamp();
        s.t_fetch += t1 - t0;
        s.t_comp += t2 - t1;
      }
      if (s.lane == 0) {
        A.phases[2 * qi] = s.t_fetch;
        A.phases[2 * qi + 1] = s.t_comp;
      }
    } else {
      for (;;) {
        const uint64_t v = s.select();
        if (v == kNoKey) break;
        const uint4 rec = s.issue((uint32_t)v & ~kFlag, true);
        s.template process<false>(v, rec, 0u, false, unused);
      }
    }
  } else {
    // Two pipeline slots.  TR_DIRECT fills an empty slot (key kNoKey) with a
    // load of the entry record so that every processing issues exactly one
    // load; TR_AGENT posts no request for an empty slot.
    const uint32_t dummy = (uint32_t)A.entry;
    uint64_t k0 = kNoKey, k1 = kNoKey;
    uint4 r0 = make_uint4(0, 0, 0, 0), r1 = make_uint4(0, 0, 0, 0);
    for (;;) {
      // slot 0 receives the new selection while slot 1 (the previous
      // selection) is processed; then the roles swap
      k0 = s.select();
      if (k0 == kNoKey && k1 == kNoKey) break;
      const uint32_t f0 = k0 != kNoKey ? ((uint32_t)k0 & ~kFlag) : dummy;
      if (k1 != kNoKey) s.template process<true>(k1, r1, f0, k0 != kNoKey, r0);
      else r0 = s.issue(f0, k0 != kNoKey);
      k1 = s.select();
      if (k1 == kNoKey && k0 == kNoKey) break;
      const uint32_t f1 = k1 != kNoKey ? ((uint32_t)k1 & ~kFlag) : dummy;
      if (k0 != kNoKey) s.template process<true>(k0, r0, f1, k1 != kNoKey, r1);
      else r1 = s.issue(f1, k1 != kNoKey);
    }
  }
  s.finish_query();
  if (A.times && s.lane == 0) {
    A.times[2 * qi] = t_start;
    A.times[2 * qi + 1] = __builtin_amdgcn_s_memrealtime();
  }
}

// G lanes per query: each block of 64 * waves_per_block threads runs
// 64 / G queries per wave, query region r = threadIdx.x / G of the block's LDS.
template <int DT, int CPL, int DELAY, int TR, bool PERSIST, int NAV, int G>
__global__ void __launch_bounds__(256) search_kernel(SearchArgs A) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int region = threadIdx.x / G;
  uint8_t *lds = smem + (size_t)region * A.lds_per_wave;
  if (!PERSIST) {
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x / G) + region;
    if (qi >= A.nq) return;
    run_query<DT, CPL, DELAY, TR, NAV, G>(A, lds, qi, batch_io(A, qi));
    return;
  }
  // Persistent: take queries from the work counter until none is left; every
  // group leaves once the counter has passed nq (the two halves of a wave
  // take their queries independently).
  for (;;) {
    uint32_t t = 0;
    if (group_lane<G>() == 0) t = atomicAdd(A.work, 1u);
    t = gfirst<G>(t);
    if ((int64_t)t >= A.nq) break;
    const int64_t qi = A.order ? (int64_t)A.order[t] : (int64_t)t;
    if (qi < 0 || qi >= A.nq) continue;  // not a permutation entry: skipped
    run_query<DT, CPL, DELAY, TR, NAV, G>(A, lds, qi, batch_io(A, qi));
    __builtin_amdgcn_wave_barrier();
  }
}

template <int DT, int CPL, int DELAY, int TR, int NAV, int G>
static hipError_t launch_t(const SearchArgs &a, int waves_per_block, bool persistent,
                           hipStream_t st) {
  const int per_block = waves_per_block * (64 / G);  // queries per block
  const size_t lds = (size_t)a.lds_per_wave * per_block;
  const int threads = 64 * waves_per_block;
  if (!persistent) {
    const int64_t blocks = (a.nq + per_block - 1) / per_block;
    hipLaunchKernelGGL((search_kernel<DT, CPL, DELAY, TR, false, NAV, G>), dim3((unsigned)blocks),
                       dim3(threads), lds, st, a);
    return hipGetLastError();
  }
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, (const void *)search_kernel<DT, CPL, DELAY, TR, true, NAV, G>, threads, lds);
  if (e != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  int64_t blocks = (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
  const int64_t need = (a.nq + per_block - 1) / per_block;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL((search_kernel<DT, CPL, DELAY, TR, true, NAV, G>), dim3((unsigned)blocks),
                     dim3(threads), lds, st, a);
  return hipGetLastError();
}

// Two queries per wave (a.qlanes == 32) are built for the direct transport,
// full-precision navigation and the strict and one-step-stale schedules;
// the host validates the rest (records of at most 512 B).
template <int DT, int CPL, int TR, int NAV>
static hipError_t launch_d(const SearchArgs &a, int wpb, bool pers, hipStream_t st) {
  if (a.delay < 0 || a.beam < 1 || (a.delay + 1) * a.beam > kMaxPipe) return hipErrorInvalidValue;
  if (a.qlanes == 32) {
    if constexpr (TR == TR_DIRECT && NAV == NAV_FULL) {
      if (a.rec_chunks > 32 || a.beam != 1 || a.delay > 1) return hipErrorInvalidValue;
      if (a.delay == 0) return launch_t<DT, CPL, SCHED_STRICT, TR, NAV, 32>(a, wpb, pers, st);
      return launch_t<DT, CPL, SCHED_RELAXED, TR, NAV, 32>(a, wpb, pers, st);
    }
    return hipErrorInvalidValue;
  }
  if (a.qlanes != 0 && a.qlanes != 64) return hipErrorInvalidValue;
  if (a.beam == 1 && a.delay == 0) return launch_t<DT, CPL, SCHED_STRICT, TR, NAV, 64>(a, wpb, pers, st);
  if (a.beam == 1 && a.delay == 1) return launch_t<DT, CPL, SCHED_RELAXED, TR, NAV, 64>(a, wpb, pers, st);
  return launch_t<DT, CPL, SCHED_GENERIC, TR, NAV, 64>(a, wpb, pers, st);
}

template <int DT, int CPL, int NAV>
static hipError_t launch_tr(const SearchArgs &a, int tr, int wpb, bool pers, hipStream_t st) {
  return tr == TR_DIRECT ? launch_d<DT, CPL, TR_DIRECT, NAV>(a, wpb, pers, st)
                         : launch_d<DT, CPL, TR_AGENT, NAV>(a, wpb, pers, st);
}

template <int DT, int NAV>
static hipError_t launch_c(const SearchArgs &a, int cpl, int tr, int wpb, bool pers,
                           hipStream_t st) {
  switch (cpl) {
    case 1: return launch_tr<DT, 1, NAV>(a, tr, wpb, pers, st);
    case 2: return launch_tr<DT, 2, NAV>(a, tr, wpb, pers, st);
    case 3: return launch_tr<DT, 3, NAV>(a, tr, wpb, pers, st);
    case 4: return launch_tr<DT, 4, NAV>(a, tr, wpb, pers, st);
    default: return hipErrorInvalidValue;
  }
}

// The launchers below and the lockstep kernel are compiled in this unit
// only; the units that instantiate the batch and server kernels of one
// element type and navigation mode include this file with
// FA_SEARCH_TEMPLATES_ONLY defined.
#ifndef FA_SEARCH_TEMPLATES_ONLY

__global__ void reset_work(uint32_t *work) { *work = 0u; }

// ------------------------------------------------------- kernel-grained sync
// The alternative the paper's query-grained I/O (section 4.2) is measured
// against: synchronisation at the granularity of the whole batch.  The waves
// of a co-resident (cooperative) grid take G queries at a time and advance
// them in lockstep, one strict step per round: every live query selects its
// node and obtains the record; a grid-wide barrier waits until every record
// of the round is in; every query scores and merges; a second barrier ends
// the round.  A query never waits for its own I/O alone but for the slowest
// of the round, and no query's compute overlaps another's I/O.  Results equal
// the strict schedule.
//
// ctl (device, zeroed before launch): [0] arrivals, [1] barrier generation,
// [2], [3] live queries of even / odd rounds, [4] failure flag.

// Wait until every memory operation the wave has issued has completed, so
// that relaxed device-scope atomics issued before it are performed before
// any issued after it (vmcnt counts stores and atomics on this architecture).
__device__ __forceinline__ void drain_memory() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_sched_barrier(0);
}

// Grid barrier, two levels deep so that no counter takes more than 32
// arrivals: the waves of a block meet at the block barrier, the block's
// first thread adds the block's live queries (when `count`) to the round's
// counter, arrives at its group's counter (32 blocks per group), and the last
// block of each group arrives at the root; the last group advances the
// generation that every block leader polls.  A counter update is complete
// before the arrival that follows it, and a counter is reset before the
// arrival above it, so a block released by the new generation sees all of
// them.  Returns false (for the whole block) once any block gave up: a spin
// limit of polls bounds every wait.
constexpr int kBarrierGroup = 32;

__device__ __forceinline__ bool grid_sync(uint32_t *ctl, uint32_t nblocks, uint32_t spin_limit,
                                          bool count, bool live, uint32_t par) {
  __shared__ uint32_t s_live[4];
  __shared__ uint32_t s_ok;
  const int wave = threadIdx.x >> 6;
  if (lane_id() == 0) s_live[wave] = live ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ok = 1;
    if (count) {
      uint32_t n = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); w++) n += s_live[w];
      if (n) __hip_atomic_fetch_add(ctl + 2 + par, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    drain_memory();
    const uint32_t gen = __hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    drain_memory();  // the generation is read before this block's arrival counts
    const uint32_t grp = blockIdx.x / kBarrierGroup;
    const uint32_t gsize = min((uint32_t)kBarrierGroup, nblocks - grp * kBarrierGroup);
    const uint32_t ngroups = (nblocks + kBarrierGroup - 1) / kBarrierGroup;
    uint32_t *gc = ctl + 16 + 16 * grp;  // one 64 B line per group
    bool wait = true;
    if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == gsize) {
      __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      drain_memory();
      if (__hip_atomic_fetch_add(ctl, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u ==
          ngroups) {
        __hip_atomic_store(ctl, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        drain_memory();
        __hip_atomic_fetch_add(ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait = false;
      }
    }
    if (wait) {
      uint32_t spins = 0;
      while (__hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(ctl + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        if (++spins > spin_limit) {
          __hip_atomic_store(ctl + 4, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

template <int DT, int CPL, int TR>
__global__ void __launch_bounds__(256) lockstep_kernel(SearchArgs A, uint32_t *ctl) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6;
  uint8_t *lds = smem + (size_t)wave * A.lds_per_wave;
  const uint32_t G = gridDim.x * (blockDim.x >> 6);
  const uint32_t gw = blockIdx.x * (blockDim.x >> 6) + wave;
  const uint32_t spin = A.spin_limit;
  uint32_t round = 0;
  for (int64_t base = 0; base < A.nq; base += G) {
    const int64_t qi = base + gw;
    const bool mine = qi < A.nq;
    const int64_t qx = mine ? qi : base;  // waves without a query only keep step
    const unsigned long long t_start = A.times ? __builtin_amdgcn_s_memrealtime() : 0ull;
    Searcher<DT, CPL, TR> s(A, lds, qx, batch_io(A, qx));
    s.init_entry();
    bool live = mine;
    for (;; round++) {
      const uint32_t par = round & 1u;
      uint64_t v = kNoKey;
      if (live) {
        v = s.select();
        live = v != kNoKey;
      }
      if (live && !s.stage(s.issue((uint32_t)v & ~kFlag, true))) live = false;
      if (!grid_sync(ctl, gridDim.x, spin, false, false, par)) return;
      // every record of the round is in LDS; the other parity's live count
      // was read by every wave before its block arrived here
      if (gw == 0 && s.lane == 0)
        __hip_atomic_store(ctl + 2 + (par ^ 1u), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (live) {
        uint4 unused;
        s.template process_staged<false>(v, 0u, false, unused);
      }
      if (!grid_sync(ctl, gridDim.x, spin, true, live, par)) return;
      const uint32_t nlive =
          __hip_atomic_load(ctl + 2 + par, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (nlive == 0) {
        round++;
        break;
      }
    }
    if (mine) {
      s.finish_query();
      if (A.times && s.lane == 0) {
        A.times[2 * qi] = t_start;
        A.times[2 * qi + 1] = __builtin_amdgcn_s_memrealtime();
      }
    }
  }
}

__global__ void reset_ctl(uint32_t *ctl, uint32_t words) {
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) ctl[i] = 0u;
}

template <int DT, int CPL, int TR>
static hipError_t launch_lockstep_t(const SearchArgs &a, uint32_t *ctl, int wpb, hipStream_t st) {
  const size_t lds = (size_t)a.lds_per_wave * wpb;
  const int threads = 64 * wpb;
  const void *fn = (const void *)lockstep_kernel<DT, CPL, TR>;
  int per_cu = 0, dev = 0, cus = 0, coop = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
  if (e != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev)) != hipSuccess)
    return e;
  if (!coop || per_cu < 1) return hipErrorNotSupported;
  int64_t blocks = (int64_t)per_cu * cus;
  const int64_t need = (a.nq + wpb - 1) / wpb;
  if (blocks > need) blocks = need;
  if (blocks > (int64_t)kLockstepGroups * kBarrierGroup) blocks = (int64_t)kLockstepGroups * kBarrierGroup;
  hipLaunchKernelGGL(reset_ctl, dim3(1), dim3(256), 0, st, ctl, (uint32_t)kLockstepCtlWords);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  SearchArgs args = a;
  uint32_t *c = ctl;
  void *params[] = {(void *)&args, (void *)&c};
  // a cooperative launch fails instead of starting a grid whose waves could
  // not all be resident at once, so the barriers cannot wait for an absent wave
  return hipLaunchCooperativeKernel(fn, dim3((unsigned)blocks), dim3(threads), params,
                                    (unsigned)lds, st);
}

template <int DT>
static hipError_t launch_lockstep_c(const SearchArgs &a, uint32_t *ctl, int tr, int wpb,
                                    hipStream_t st) {
  const int cpl = a.nav_stride / 128;
#define FA_LS(C)                                                               \
  return tr == TR_DIRECT ? launch_lockstep_t<DT, C, TR_DIRECT>(a, ctl, wpb, st) \
                         : launch_lockstep_t<DT, C, TR_AGENT>(a, ctl, wpb, st)
  switch (cpl) {
    case 1: FA_LS(1);
    case 2: FA_LS(2);
    case 3: FA_LS(3);
    case 4: FA_LS(4);
    default: return hipErrorInvalidValue;
  }
#undef FA_LS
}

hipError_t launch_lockstep(const SearchArgs &a, uint32_t *ctl, int dtype, int transport,
                           int waves_per_block, hipStream_t st) {
  switch (dtype) {
    case DT_U8: return launch_lockstep_c<DT_U8>(a, ctl, transport, waves_per_block, st);
    case DT_I8: return launch_lockstep_c<DT_I8>(a, ctl, transport, waves_per_block, st);
    case DT_F32: return launch_lockstep_c<DT_F32>(a, ctl, transport, waves_per_block, st);
    default: return hipErrorInvalidValue;
  }
}

uint32_t search_lds_bytes(int Lcap, int nav_stride, int hash_bits, int kcap, int pq_floats,
                          int qlanes) {
  return lds_layout(Lcap, nav_stride, hash_bits, kcap, pq_floats, qlanes).bytes;
}

// The batch and server kernels of each element type and navigation mode are
// instantiated in units of their own (search_full_*.hip, search_pq_*.hip),
// so that they compile in parallel.
#define FA_NAV_LAUNCHERS(N, T)                                                                 \
  hipError_t launch_search_##N##_##T(const SearchArgs &a, int transport, int wpb, bool pers,   \
                                     hipStream_t st);                                          \
  hipError_t launch_server_##N##_##T(const ServerArgs &a, int wpb, int64_t *res, hipStream_t st);
FA_NAV_LAUNCHERS(full, u8)
FA_NAV_LAUNCHERS(full, i8)
FA_NAV_LAUNCHERS(full, f32)
#undef FA_NAV_LAUNCHERS

hipError_t launch_search(const SearchArgs &a, int dtype, int transport, int waves_per_block,
                         bool persistent, hipStream_t st) {
  if (a.pq_m > 0) return launch_search_pq(a, dtype, transport, waves_per_block, persistent, st);
  switch (dtype) {
    case DT_U8: return launch_search_full_u8(a, transport, waves_per_block, persistent, st);
    case DT_I8: return launch_search_full_i8(a, transport, waves_per_block, persistent, st);
    case DT_F32: return launch_search_full_f32(a, transport, waves_per_block, persistent, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reset(uint32_t *work, hipStream_t st) {
  hipLaunchKernelGGL(reset_work, dim3(1), dim3(1), 0, st, work);
  return hipGetLastError();
}

#endif  // FA_SEARCH_TEMPLATES_ONLY

// ------------------------------------------------------------------ server
// Compiled in both units like the batch kernels: full-precision navigation
// here, compressed navigation in the PQ unit.

// Continuous-batching server.  Waves take ring indices as tickets from one
// counter and serve each once the host has published it; a wave that leaves
// while idle holds no ticket (see the claim loop).  The entry is read with
// system-scope loads because ring memory is rewritten by host copies; results
// go to host-mapped rows, then the slot's done word tells the host.
template <int DT, int CPL, int DELAY, int TR, int NAV>
__global__ void __launch_bounds__(256) server_kernel(ServerArgs S) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  uint8_t *lds = smem + (size_t)wave * S.base.lds_per_wave;
  for (;;) {
    // Tickets are 64-bit on the device as on the host, so they never wrap in
    // practice and the ring entry is the ticket modulo the ring capacity on
    // both sides.
    uint64_t got = 0;
    int have = 0;
    if (lane == 0) {
      // Tickets come from one fetch-add on `next` (one L2 atomic per claim,
      // however many waves look for work at once).  A wave whose ticket is
      // not published yet keeps it while it waits, or hands it back with
      // CAS(next, t + 1 -> t), which succeeds only for the highest ticket
      // out, so returns happen in LIFO order and no ticket is ever dropped:
      // the holders of unpublished tickets always drain back to zero unless
      // new entries get published, and then they are served instead.
      uint32_t idle = 0, nap = 1;
      for (;;) {
        // relaxed system-scope polls bypass the caches without the L2
        // invalidation an acquire would cost every idle wave on every poll;
        // the entry itself is read with system-scope loads below
        uint64_t pub = __hip_atomic_load(S.published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint64_t c = __hip_atomic_load(S.next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c < pub) {
          const uint64_t t = atomicAdd((unsigned long long *)S.next, 1ull);
          uint32_t hold_nap = 1;
          for (;;) {
            if (t < pub) {
              got = t;
              have = 1;
              break;
            }
            if (atomicCAS((unsigned long long *)S.next, t + 1ull, t) == t + 1ull) break;  // handed back
            for (uint32_t i = 0; i < hold_nap; i++) __builtin_amdgcn_s_sleep(2);
            hold_nap = hold_nap < 8 ? hold_nap * 2 : 8;
            pub = __hip_atomic_load(S.published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          }
          if (have) break;
          continue;
        }
        if (__hip_atomic_load(S.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
        if (++idle > S.idle_limit) break;
        for (uint32_t i = 0; i < nap; i++) __builtin_amdgcn_s_sleep(8);
        nap = nap < 8 ? nap * 2 : 8;
      }
    }
    have = __builtin_amdgcn_readfirstlane(have);
    if (!have) return;
    got = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(got >> 32)) << 32) |
          (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
    const uint8_t *e = S.ring + (int64_t)(got % S.ring_cap) * S.entry_bytes;
    const uint32_t *ctrl = (const uint32_t *)e;
    const uint32_t slot =
        __hip_atomic_load(ctrl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const uint32_t kl = __hip_atomic_load(ctrl + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (slot >= S.nslots) continue;  // malformed entry: skipped
    int k = (int)(kl & 0xFFFFu), L = (int)(kl >> 16);
    L = L < 1 ? 1 : (L > S.base.L ? S.base.L : L);
    k = k < 1 ? 1 : (k > S.base.k ? S.base.k : k);
    if (k > L) k = L;
    QueryIO io;
    io.q = e + 16;
    io.coherent = true;
    io.ids = S.res_ids + (int64_t)slot * S.base.k;
    io.dists = S.res_dists + (int64_t)slot * S.base.k;
    io.steps = S.res_steps + slot;
    io.L = L;
    io.k = k;
    io.width = k;
    // TR_AGENT: each resident wave owns one transport line for all the
    // queries it serves (its request numbers continue in line_seq)
    io.line = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    io.status = S.res_status ? S.res_status + slot : nullptr;
    run_query<DT, CPL, DELAY, TR, NAV>(S.base, lds, (int64_t)slot, io);
    // The result rows were written with system-scope (write-through) stores:
    // once they have completed, the done word may follow.  This avoids a
    // release fence, which would write back the whole L2 for every query.
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    if (lane == 0)
      __hip_atomic_store(S.done + 16 * (int64_t)slot, (uint32_t)(got + 1u), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

template <int DT, int CPL, int DELAY, int TR, int NAV>
static hipError_t launch_server_t(const ServerArgs &a, int wpb, int64_t *resident,
                                  hipStream_t st) {
  const size_t lds = (size_t)a.base.lds_per_wave * wpb;
  const int threads = 64 * wpb;
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, (const void *)server_kernel<DT, CPL, DELAY, TR, NAV>, threads, lds);
  if (e != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  const int64_t blocks = (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
  if (resident) *resident = blocks * wpb;
  if (!st) return hipSuccess;  // size query only
  hipLaunchKernelGGL((server_kernel<DT, CPL, DELAY, TR, NAV>), dim3((unsigned)blocks), dim3(threads),
                     lds, st, a);
  return hipGetLastError();
}

template <int DT, int CPL, int TR, int NAV>
static hipError_t launch_server_s(const ServerArgs &a, int wpb, int64_t *res, hipStream_t st) {
  const int delay = a.base.delay, beam = a.base.beam;
  if (delay < 0 || beam < 1 || (delay + 1) * beam > kMaxPipe) return hipErrorInvalidValue;
  if (beam == 1 && delay == 0) return launch_server_t<DT, CPL, SCHED_STRICT, TR, NAV>(a, wpb, res, st);
  if (beam == 1 && delay == 1)
    return launch_server_t<DT, CPL, SCHED_RELAXED, TR, NAV>(a, wpb, res, st);
  return launch_server_t<DT, CPL, SCHED_GENERIC, TR, NAV>(a, wpb, res, st);
}

template <int DT, int CPL, int NAV>
static hipError_t launch_server_d(const ServerArgs &a, int wpb, int64_t *res, hipStream_t st) {
  return a.transport == TR_AGENT ? launch_server_s<DT, CPL, TR_AGENT, NAV>(a, wpb, res, st)
                                 : launch_server_s<DT, CPL, TR_DIRECT, NAV>(a, wpb, res, st);
}

template <int DT, int NAV>
static hipError_t launch_server_c(const ServerArgs &a, int wpb, int64_t *res, hipStream_t st) {
  switch (a.base.nav_stride / 128) {
    case 1: return launch_server_d<DT, 1, NAV>(a, wpb, res, st);
    case 2: return launch_server_d<DT, 2, NAV>(a, wpb, res, st);
    case 3: return launch_server_d<DT, 3, NAV>(a, wpb, res, st);
    case 4: return launch_server_d<DT, 4, NAV>(a, wpb, res, st);
    default: return hipErrorInvalidValue;
  }
}

#ifndef FA_SEARCH_TEMPLATES_ONLY

hipError_t launch_server(const ServerArgs &a, int dtype, int waves_per_block,
                         int64_t *resident_waves, hipStream_t st) {
  if (a.base.pq_m > 0) return launch_server_pq(a, dtype, waves_per_block, resident_waves, st);
  switch (dtype) {
    case DT_U8: return launch_server_full_u8(a, waves_per_block, resident_waves, st);
    case DT_I8: return launch_server_full_i8(a, waves_per_block, resident_waves, st);
    case DT_F32: return launch_server_full_f32(a, waves_per_block, resident_waves, st);
    default: return hipErrorInvalidValue;
  }
}

#endif  // FA_SEARCH_TEMPLATES_ONLY

}  // namespace fa

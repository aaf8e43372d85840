// search_kernel.h -- internal interface between the C-ABI layer and the
// gfx950 search kernels (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fa {

enum { DT_U8 = 1, DT_I8 = 2, DT_F32 = 3 };

// How a wave obtains a record: by loading it itself (HBM or host-mapped
// memory), or by posting a request that a host agent thread serves into a
// per-query staging slot (query-grained transport).
enum { TR_DIRECT = 0, TR_AGENT = 1 };

// Kernel schedules: strict (delay 0, one node per step), one-step-stale
// (delay 1, one node per step), and any delay with any beam width W, the
// in-flight nodes held in an LDS FIFO of at most (delay + 1) * W <= kMaxPipe.
enum { SCHED_STRICT = 0, SCHED_RELAXED = 1, SCHED_GENERIC = 2 };
constexpr int kMaxPipe = 8;

// Navigation: neighbours scored exactly against the full-precision HBM copy,
// or by product-quantisation codes in HBM with the expanded nodes re-ranked
// exactly from their records (compressed navigation).  PQ: M <= kPqMaxM
// subspaces of 256 centroids; code rows of kPqStride bytes (byte m = code of
// subspace m, the rest zero).
enum { NAV_FULL = 0, NAV_PQ = 1 };
constexpr int kPqStride = 32;
constexpr int kPqMaxM = 32;
constexpr int kPqKsub = 256;

// Byte offsets of one wave's LDS region.
struct LdsLayout {
  uint32_t cand, nk, stage, qbuf, ids, dsc, hash, fifo, res, tab, bytes;
};

struct SearchArgs {
  const uint8_t *nav;      // n x nav_stride bytes (HBM), rows zero-padded
  const uint8_t *records;  // n x slot bytes, device-visible (HBM or mapped host)
  const uint8_t *queries;  // nq x qbytes (device)
  int32_t *out_ids;        // nq x k
  void *out_dists;         // nq x k, u32 (u8/i8) or f32 bits
  uint32_t *out_steps;     // nq, optional
  unsigned long long *stats;  // optional: [0] steps [1] rows scored [2] record mismatches
  int32_t *trace;          // optional: nq x trace_cap selected ids, in order
  unsigned long long *times;  // optional: nq x 2 wall-clock stamps (start, end)
  unsigned long long *phases; // optional, strict schedule only: nq x 2 summed
                              // wall-clock ticks (record fetch, compute)
  // TR_AGENT only (fine-grained host memory except `status`):
  uint64_t *req;           // nq x 8 u64 (64 B per query); slot seq % pslots: (node << 32) | seq
  const uint32_t *cpl;     // nq x 16 u32 (64 B per query); word seq % pslots: seq or seq | 1<<31
  const uint8_t *stage;    // nq x pslots staging slots of stage_stride bytes
  int64_t stage_stride;
  int32_t pslots;          // request slots per query: at least the requests in flight
  uint32_t spin_limit;     // polls of a completion word before the query times out
  uint32_t poll_nap;       // longest pause between two polls, in 1024-cycle units
  int32_t *status;         // nq per-query status, device: 0, -5 (read error), -110 (timeout)
  uint32_t *line_seq;      // optional, device: last request number per transport line, kept
                           // across the queries a line serves (persistent server waves)
  int32_t trace_cap;
  int64_t nq, n, slot;
  int32_t nav_stride, qbytes, vec_pad, ids_off, rec_chunks;
  int32_t R, L, Lcap, k, entry, hash_bits;  // L, k: batch maxima when per-query arrays are set
  int32_t k_stride;        // output row stride (>= k)
  const int32_t *q_L;      // optional per-query L (clamped to [1, L])
  const int32_t *q_k;      // optional per-query k (clamped to [1, min(k, L_q)])
  const int32_t *order;    // optional processing order (persistent launches)
  uint32_t *work;          // persistent launches: device work counter, zero at launch
  int32_t delay, beam;     // SCHED_GENERIC: staleness and beam width, (delay+1)*beam <= kMaxPipe
  // NAV_PQ (pq_m > 0): codes n x kPqStride (HBM), codebooks pq_m x 256 x pq_dsub f32.
  // pq_direct: centroids read from the cache per code instead of a per-query
  // LDS table (same arithmetic); pq_floats: LDS floats of either
  const uint8_t *pq_codes;
  const float *pq_cb;
  int32_t pq_m, pq_dsub, pq_direct, pq_floats;
  // optional hot-record cache (TR_DIRECT): cache_map[v] = slot of node v's
  // record copy in `cache` (device memory, slot-strided), or -1
  const uint8_t *cache;
  const int32_t *cache_map;
  uint32_t lds_per_wave;   // LDS bytes of one query's region
  int32_t qlanes;          // lanes per query: 64 (one query per wave) or 32
                           // (two per wave: TR_DIRECT, NAV_FULL, strict or
                           // one-step-stale, records of at most 512 B)
};

// LDS bytes of one query's region; kcap (result capacity, the batch k) and
// pq_floats (SearchArgs::pq_floats) only for compressed navigation; qlanes
// the lanes per query.
uint32_t search_lds_bytes(int Lcap, int nav_stride, int hash_bits, int kcap = 0,
                          int pq_floats = 0, int qlanes = 64);
// Continuous-batching server: a persistent kernel whose waves take queries
// from a ring in device memory as the host publishes them.
//   ring entry (entry_bytes): u32 seq+1, u32 result slot, u32 k | L << 16,
//   u32 pad, then the query zero-padded to nav_stride bytes.
struct ServerArgs {
  SearchArgs base;          // index fields, Lcap / hash_bits for L_max; k = k_max
  const uint8_t *ring;      // device, ring_cap entries
  int64_t entry_bytes;
  uint32_t ring_cap, nslots;
  uint64_t *next;           // device: next ticket to claim (entry = ticket % ring_cap)
  const uint64_t *published;  // device: tickets published (written by the host's stream)
  const uint32_t *stop;     // device: non-zero = leave once idle
  int32_t *res_ids;         // host-mapped, nslots x k_max
  uint32_t *res_dists;      // host-mapped, nslots x k_max
  uint32_t *res_steps;      // host-mapped, nslots
  uint32_t *done;           // host-mapped, nslots x 16 (one 64 B line per slot)
  int32_t *res_status;      // host-mapped, nslots: written only when a record read fails
                            // (-5) or times out (-110); the host clears it per use
  int32_t transport;        // TR_DIRECT, or TR_AGENT: transport line = resident wave index
  uint32_t idle_limit;      // empty polls before a wave leaves
};
// The schedule follows a.base.delay and a.base.beam, as in launch_search;
// a.base.pq_m > 0 selects compressed navigation (launch_server_pq).
hipError_t launch_server(const ServerArgs &a, int dtype, int waves_per_block,
                         int64_t *resident_waves, hipStream_t st);
hipError_t launch_server_pq(const ServerArgs &a, int dtype, int waves_per_block,
                            int64_t *resident_waves, hipStream_t st);

// persistent: grid sized to the resident capacity of the GPU; waves take
// queries from a->work (which must be zero at launch) until all are done.
// The schedule follows a.delay and a.beam: strict or one-step-stale kernels
// for beam 1 and delay <= 1, the generic FIFO kernel otherwise.  a.pq_m > 0
// selects compressed navigation (launch_search_pq).
hipError_t launch_search(const SearchArgs &a, int dtype, int transport, int waves_per_block,
                         bool persistent, hipStream_t st);
hipError_t launch_search_pq(const SearchArgs &a, int dtype, int transport, int waves_per_block,
                            bool persistent, hipStream_t st);
// PQ codes of n rows of the navigation copy (rows of nav_stride bytes, d
// elements of dtype; M <= 32 subspaces of d / M <= 32 dimensions):
// codes[i * kPqStride + m] = nearest centroid of subspace m (fp32, fixed
// order, lowest index among equals); bytes M..31 zero.
hipError_t launch_pq_encode(const uint8_t *nav, int64_t n, int nav_stride, int dtype, int d,
                            const float *codebooks, int M, uint8_t *codes, hipStream_t st);
// Kernel-grained synchronisation (ablation): a cooperative grid advances
// groups of co-resident queries one strict step per round, with grid-wide
// barriers after the record fetches and after the compute.  `ctl` is
// kLockstepCtlWords u32 of device memory (zeroed here by a kernel); ctl[4] != 0
// afterwards means a barrier wait exceeded a.spin_limit polls and the search
// was abandoned.  The grid has at most kLockstepGroups groups of 32 blocks.
constexpr int kLockstepGroups = 256;
constexpr int kLockstepCtlWords = 16 + 16 * kLockstepGroups;
hipError_t launch_lockstep(const SearchArgs &a, uint32_t *ctl, int dtype, int transport,
                           int waves_per_block, hipStream_t st);
// Zero the persistent work counter (a kernel, so that it can be captured in a
// graph).
hipError_t launch_reset(uint32_t *work, hipStream_t st);

}  // namespace fa

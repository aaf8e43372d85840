/*
 * flashann.h -- C ABI of the MI355X (gfx950) out-of-core graph search library.
 *
 * The method is the search hot path of FlashANNS (arXiv 2507.10070): batched
 * best-first search over a fixed-degree proximity graph in which every
 * expansion fetches one node record (full-precision vector plus neighbour
 * ids) from a storage tier and scores the neighbours by squared L2 distance
 * (paper section 4.1.1), optionally with the dependency-relaxed schedule that
 * issues the next record fetch before the current distances are done
 * (section 4.1.2).  The problem statement is top-k by L2 (section 1); recall
 * is controlled by the candidate-list size L (section 5.1).
 *
 * Conventions
 *   - Every function returns ANN_OK (0) or a negative errno-style code and
 *     leaves a message for ann_last_error() on failure.
 *   - Pointers documented "device" must be device-accessible (hipMalloc or
 *     PyTorch CUDA tensors); "host" pointers are plain host memory.  The
 *     caller owns every pointer it passes; the library keeps none of them
 *     after a call returns (ann_search: after the stream work completes).
 *   - The library owns the index handle and everything inside it: the HBM
 *     navigation copy, the record store of the chosen tier, staging buffers.
 *   - Distances are squared L2 (no square root): exact uint32 for u8/i8
 *     vectors, fp32 for f32 vectors.
 *   - Vectors are row-major, d elements per row, no padding.
 */
#ifndef FLASHANN_H
#define FLASHANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ANN_OK = 0,
  ANN_EIO = -5,
  ANN_ENOMEM = -12,
  ANN_EBUSY = -16,
  ANN_ENODEV = -19,
  ANN_EINVAL = -22,
  ANN_ENOTSUP = -95,
  ANN_ETIMEDOUT = -110
};

typedef enum { ANN_U8 = 1, ANN_I8 = 2, ANN_F32 = 3 } ann_dtype;

/* Where node records live (section 4.2 places them on SSD; this build offers
 * HBM, pinned host DRAM read by the GPU over the host link, and a file). */
typedef enum { ANN_TIER_HBM = 0, ANN_TIER_HOST = 1, ANN_TIER_FILE = 2 } ann_tier;

/* How a GPU wave obtains a record.  DIRECT: the wave loads it itself (HBM, or
 * pinned host DRAM over the host link).  AGENT: the query-grained transport of
 * section 4.2 -- the wave writes a request into its own slot in host memory and
 * continues; a host agent thread reads the record (memory copy or file read)
 * into the query's staging slot and posts a per-query completion word, which
 * the wave checks when it needs the record.  AUTO: AGENT for ANN_TIER_FILE,
 * DIRECT otherwise. */
typedef enum {
  ANN_TRANSPORT_AUTO = 0,
  ANN_TRANSPORT_DIRECT = 1,
  ANN_TRANSPORT_AGENT = 2
} ann_transport;

/* How neighbours are scored (ann_search_opts.navigation). */
typedef enum {
  ANN_NAV_FULL = 0, /* exact distance against the full-precision HBM copy */
  ANN_NAV_PQ = 1    /* product-quantisation codes in HBM, expanded nodes
                       re-ranked exactly from their records (ann_index_set_pq) */
} ann_navigation;

/* How PQ distances are formed (ann_search_opts.pq_scoring); both give the
 * same fp32 values. */
typedef enum {
  ANN_PQ_AUTO = 0,  /* ANN_PQ_TABLE when the table is at most 8 KiB, else ANN_PQ_CACHE */
  ANN_PQ_TABLE = 1, /* per-query table of m x 256 floats in LDS, one read per code byte */
  ANN_PQ_CACHE = 2  /* centroids read from the codebook (cache-resident) per code byte;
                       LDS holds only the query, so more queries fit per CU */
} ann_pq_scoring;

/* ann_index_set_pq flags */
#define ANN_PQ_DROP_NAV 1 /* release the full-precision navigation copy */

typedef struct ann_index ann_index; /* opaque, owned by the library */

typedef struct {
  int64_t n;          /* base vectors */
  int32_t d;          /* dimension */
  int32_t dtype;      /* ann_dtype */
  int32_t R;          /* neighbour ids per record */
  int32_t entry;      /* entrance node of every search */
  int32_t slot_bytes; /* record slot size */
  int32_t tier;       /* ann_tier */
  int32_t nav_stride; /* bytes per row of the HBM navigation copy */
  int32_t rec_bytes;  /* bytes of each record fetched per step */
  int64_t hbm_bytes;  /* device memory held by the index */
  int32_t direct_io;  /* ANN_TIER_FILE: 1 if the file is read with O_DIRECT */
  int32_t pq_m;       /* PQ subspaces of the codes in HBM (0 = none) */
  int32_t nav_full;   /* 1 while the full-precision navigation copy is held */
  int32_t stripes;    /* ANN_TIER_FILE: record files the records are striped over */
  int32_t reserved;
  int64_t cached_records; /* records copied into the hot-record cache (0 = none) */
} ann_index_info;

/* Search options; a NULL pointer means {delay = 1, beam_width = 1, defaults}. */
typedef struct {
  int32_t delay;           /* staleness delta (section 4.1.2): a node selected in
                              one iteration is processed once delta * W newer
                              nodes are in flight; 0 = strict best-first,
                              1 = the paper's default (section 4.1.4) */
  int32_t beam_width;      /* W, nodes selected per iteration (default 1);
                              (delay + 1) * W <= 8 nodes may be in flight */
  int32_t hash_bits;       /* log2 of the per-query visited-hash slots (0 = default 10) */
  int32_t waves_per_block; /* waves per workgroup, 1..4 (0 = 4, or 2 or 1 when
                              the LDS of a workgroup cannot hold its queries);
                              one query per wave unless query_lanes = 32 */
  unsigned long long *d_stats; /* optional device counters, 3 x u64, accumulated:
                                  [0] expansions [1] neighbour distances computed
                                  [2] records whose own vector disagreed with the
                                  navigation copy (always 0 for a valid index) */
  int32_t *d_trace;        /* optional device buffer, nq x trace_cap int32: the
                              expanded node ids of each query in expansion order
                              (entries past the query's steps are left untouched) */
  int32_t trace_cap;
  unsigned long long *d_times; /* optional device buffer, nq x 2 u64: wall-clock
                                  stamps when each query's search starts and ends,
                                  in ticks of ann_device_clock_khz() kHz */
  unsigned long long *d_phases; /* optional device buffer, nq x 2 u64, strict
                                  schedule only (delay 0): per query, the summed
                                  wall-clock ticks spent obtaining records (issue
                                  to record in LDS, T_f) and computing (filter,
                                  gathers, distances, merge, T_c) -- the stage
                                  times the degree selector balances (section 4.3) */
  int32_t transport;       /* ann_transport (0 = AUTO) */
  uint32_t spin_limit;     /* AGENT: polls of a completion word before the query
                              gives up with ANN_ETIMEDOUT (0 = default 2^24) */
  /* Batches of uneven searches (one kernel for all): */
  const int32_t *d_L;      /* optional device array, nq: per-query list size,
                              clamped to [1, L]; L is then the batch maximum */
  const int32_t *d_k;      /* optional device array, nq: per-query result count,
                              clamped to [1, min(k, L_q)]; rows keep stride k and
                              are padded past k_q like missing results */
  const int32_t *d_order;  /* optional device array, nq: processing order (a
                              permutation of 0..nq-1), e.g. longest search first */
  int32_t persistent;      /* 1: one wave per resident slot of the GPU; waves take
                              the next query from a device work counter when
                              done, so long and short searches share the kernel.
                              Persistent searches on one index must be ordered
                              (one stream or synchronised). */
  int32_t sync_grain;      /* 0: query-grained (default): each query waits only
                              for its own records (section 4.2).  1: kernel-
                              grained, the comparison point of section 4.2: the
                              queries resident on the GPU advance one strict step
                              per round in lockstep, with a grid-wide barrier
                              once every record of the round is in and another
                              after the compute.  Needs delay 0, beam_width 1,
                              no persistent, d_order or d_phases; synchronous;
                              results equal the strict search.  spin_limit
                              bounds each barrier wait (0 = 2^24 polls), else
                              ANN_ETIMEDOUT. */
  int32_t navigation;      /* ann_navigation (0 = full precision).  ANN_NAV_PQ
                              (paper section 2.2: quantised vectors in memory,
                              full-precision vectors with the neighbour lists
                              in storage): the list is ordered by PQ distance,
                              each expanded node's exact distance comes from
                              the vector in its record, and ids / dists are
                              the first k expanded nodes by exact distance.
                              Needs ann_index_set_pq; sync_grain 0 only;
                              d_stats[2] stays 0. */
  int32_t pq_scoring;      /* ann_pq_scoring (0 = auto); results do not depend on it */
  int32_t poll_backoff;    /* AGENT: the longest pause between two polls of a
                              completion word, in units of 1024 GPU cycles
                              (about 0.43 us); pauses double from one unit up
                              to it.  0 = 32.  Results do not depend on it. */
  int32_t query_lanes;     /* lanes per query, the threads-per-query tile: 0 or 64
                              = one query per wave64; 32 = two queries per wave,
                              one per half (the paper runs one query per 32-lane
                              warp, section 4.2).  32 needs the direct transport,
                              full-precision navigation, sync_grain 0, delay 0 or
                              1 with beam_width 1, and records of at most 512 B,
                              else ANN_ENOTSUP.  waves_per_block stays a count of
                              waves, so a workgroup then holds 2 x that many
                              queries.  Results do not depend on it. */
} ann_search_opts;

/*
 * ann_index_create -- build a searchable index from host arrays.
 *   vectors    host, n x d elements of `dtype`
 *   adjacency  host, n x R int32 neighbour ids; ids outside [0, n) are
 *              padding and are skipped by the search
 *   entry      entrance node (e.g. the medoid), 0 <= entry < n
 *   slot_bytes record slot size; a record is the vector (padded to 16 B)
 *              followed by the R ids, so slot_bytes >= round_up(d*b,16) + 4R
 *              and a multiple of 16; the fetched part must be <= 1024 B
 *   tier       ANN_TIER_HBM or ANN_TIER_HOST (pinned host DRAM)
 * Layout follows the paper's node record: the vector then its neighbour ids
 * (section 3, challenge C3: 128 B of u8 vector + 64 x 4 B ids = 384 B).
 * Errors: ANN_EINVAL (bad sizes), ANN_ENOMEM, ANN_ENODEV (no GPU).
 */
int ann_index_create(const void *vectors, const int32_t *adjacency, int64_t n, int32_t d,
                     int32_t dtype, int32_t R, int32_t entry, int32_t slot_bytes, int32_t tier,
                     ann_index **out);

/*
 * ann_save_index -- write an index directory: meta.json (n, d, dtype, R,
 * entry, slot_bytes), vectors.bin (n x d raw elements) and records.bin (n
 * records of slot_bytes, the layout of ann_index_create).  Host pointers;
 * `dir` is created if missing.  Errors: ANN_EINVAL, ANN_EIO.
 */
int ann_save_index(const char *dir, const void *vectors, const int32_t *adjacency, int64_t n,
                   int32_t d, int32_t dtype, int32_t R, int32_t entry, int32_t slot_bytes);

/*
 * ann_build_index -- construct a degree-R proximity graph over `vectors`
 * (host, n x d; deterministic for a given seed: kNN pools, alpha = 1.2
 * pruning, reverse and long-range hub edges, connectivity repair, medoid
 * entry) and write the index directory as ann_save_index does.  The paper
 * inherits its graphs and does not describe their construction; this is
 * offline and not on the search path.  Errors: ANN_EINVAL, ANN_ENOMEM, ANN_EIO.
 */
int ann_build_index(const void *vectors, int64_t n, int32_t d, int32_t dtype, int32_t R,
                    int32_t slot_bytes, uint64_t seed, const char *out_dir);

/*
 * ann_load_records -- open an index directory on the GPU: the navigation copy
 * goes to HBM; records go to HBM or pinned host DRAM (tiers HBM, HOST), or
 * stay in the file for ANN_TIER_FILE (read per request by the agent, with
 * O_DIRECT when slot_bytes is a multiple of 512 and the file system allows).
 * `records_path` overrides <dir>/records.bin (NULL = default).
 * Errors: ANN_EINVAL, ANN_EIO, ANN_ENOMEM, ANN_ENODEV.
 */
int ann_load_records(const char *dir, int32_t tier, const char *records_path, ann_index **out);

/*
 * Records striped over several files, one per storage device (paper section
 * 5.2 and 5.6: the records of one index spread over 1 to 8 SSDs).  Record v
 * is slot v / stripes of file v % stripes, so consecutive ids alternate
 * between devices and every device serves an equal share of random reads.
 *
 * ann_save_records_striped -- write the `stripes` record files `paths[s]`
 * (host pointers; each file holds records s, s + stripes, ... in the layout
 * of ann_index_create).  Errors: ANN_EINVAL (stripes not in [1, 16], bad
 * sizes), ANN_EIO.
 *
 * ann_load_records_striped -- ann_load_records with the records in the
 * `stripes` files `paths` (meta.json and vectors.bin from `dir`).  The FILE
 * tier keeps one descriptor per stripe; the agent reads record v from file
 * v % stripes, and each agent thread keeps its asynchronous reads in flight
 * on every device at once.  HBM and HOST tiers read the stripes into memory.
 * Errors: those of ann_load_records.
 */
int ann_save_records_striped(const void *vectors, const int32_t *adjacency, int64_t n, int32_t d,
                             int32_t dtype, int32_t R, int32_t slot_bytes,
                             const char *const *paths, int32_t stripes);
int ann_load_records_striped(const char *dir, int32_t tier, const char *const *paths,
                             int32_t stripes, ann_index **out);

/*
 * ann_agent_configure -- settings of the host agent used by the AGENT
 * transport: `threads` (0 = default: hardware threads - 2, at most 32, for
 * memory copies; 8 for files read with O_DIRECT, each keeping up to 64
 * asynchronous reads in flight; 64 for buffered file reads, which block in
 * pread and set the queue depth by their number).  The other
 * arguments inject faults for tests, -1 = off: requests for `delay_node`
 * complete after `delay_us` microseconds (a straggler), requests for
 * `fail_node` complete with a read error (ANN_EIO for that query), requests
 * for `drop_node` never complete (ANN_ETIMEDOUT after spin_limit polls).
 */
int ann_agent_configure(ann_index *ix, int32_t threads, int32_t delay_node, int32_t delay_us,
                        int32_t fail_node, int32_t drop_node);

/* ann_agent_stats -- cumulative agent counters: requests served, bytes copied
 * or read, failed reads (host integers, caller-owned). */
int ann_agent_stats(const ann_index *ix, uint64_t *requests, uint64_t *bytes, uint64_t *errors);

/* ann_agent_profile_get -- where the agent threads' time went (cumulative
 * over the agent's life; zeros before its first use).  A pass is one scan of
 * a thread's query range; busy passes found or finished requests.  scan_ns:
 * reading request lines; copy_ns: copying records from host memory into
 * staging and publishing completions; io_ns: submitting and reaping file
 * reads.  max_batch: most requests one scan found.  stripe_requests[s]:
 * requests served from stripe s. */
typedef struct {
  uint64_t requests, bytes, errors, passes, busy_passes, scan_ns, copy_ns, io_ns, max_batch;
  int32_t threads;   /* agent threads */
  int32_t async_io;  /* 1 if file reads are asynchronous (O_DIRECT + Linux AIO) */
  int32_t stripes;   /* record files (1 for host memory) */
  int32_t reserved;
  uint64_t stripe_requests[16];
} ann_agent_profile;
int ann_agent_profile_get(const ann_index *ix, ann_agent_profile *out);

/*
 * ann_index_set_pq -- compressed navigation (paper section 2.2: the
 * in-memory quantised vectors of graph-indexing systems, while the
 * full-precision vectors stay in the records).  Encodes every base vector
 * on the GPU into a 32 B code row in HBM, replacing earlier codes.
 *   codebooks  host, m x 256 x (d / m) float32: subspace s covers dimensions
 *              [s * d/m, (s+1) * d/m); centroid c of subspace s at
 *              codebooks[(s * 256 + c) * (d/m)]; copied, caller keeps ownership
 *   m          subspaces, 1 <= m <= 32, d % m == 0, d / m <= 32
 *   flags      ANN_PQ_DROP_NAV: free the full-precision navigation copy
 *              afterwards (searches must then use ANN_NAV_PQ; the server and
 *              a later ann_index_set_pq need the copy)
 * Code of a vector, per subspace: the centroid of smallest fp32 squared
 * distance, accumulated with fused multiply-adds over the subspace's
 * dimensions in order; the lowest index among equals.  Synchronous: waits for
 * all device work (searches still reading the old codes) before replacing.
 * Graphs captured by ann_search_graph before this call hold the old codes
 * (or the released copy) and must not be replayed after it.
 * Errors: ANN_EINVAL (sizes, or no navigation copy to encode), ANN_EBUSY (a
 * server is open on the index), ANN_ENOMEM.
 */
int ann_index_set_pq(ann_index *ix, const float *codebooks, int32_t m, int32_t flags);

/*
 * ann_index_set_record_cache -- hot-record cache in device memory.  Not a
 * step of the paper's method (its records live in storage, section 4.2) but
 * a layout for GPUs whose memory can hold a share of the records: searches
 * read the records of the cached nodes from device memory and every other
 * record from its tier, as before.  The bytes read are the same, so results
 * do not change; only the host-link or storage traffic does.  A node's
 * cache slot is looked up (one 4 B load from a device map of n entries)
 * when the node is selected for expansion.
 *   ids    host, count distinct node ids in [0, n) whose records are copied
 *          (typically the most-visited nodes of a sample of queries); copied,
 *          caller keeps ownership
 *   count  0 releases the cache
 * Device memory: count x slot_bytes + 4 n bytes.  ANN_TIER_HOST and
 * ANN_TIER_FILE indexes (HBM-tier records are all in device memory; a file
 * tier's cached records are read from its files here).  Searches and
 * servers use it with either transport: the direct loads read a cached
 * record's copy, and the agent transport posts no request for a cached node.  Synchronous: waits for all device work before replacing
 * the cache; graphs captured before the call must not be replayed after it.
 * Errors: ANN_EINVAL (ids out of range or repeated, count > n), ANN_ENOTSUP
 * (ANN_TIER_HBM), ANN_EBUSY (a server is open on the index), ANN_EIO (a
 * record file read failed), ANN_ENOMEM.
 */
int ann_index_set_record_cache(ann_index *ix, const int32_t *ids, int64_t count);
/* ann_index_pq_codes -- copy the PQ codes to `host_codes` (caller-owned,
 * n x m bytes, row i = the m subspace codes of node i).  Synchronous.
 * Errors: ANN_EINVAL (NULL, or no codes). */
int ann_index_pq_codes(const ann_index *ix, uint8_t *host_codes);

/* ann_index_info -- sizes and layout of an index (host struct, caller-owned). */
int ann_index_info_get(const ann_index *ix, ann_index_info *out);

/*
 * ann_search -- batched top-k search on `hip_stream` (a hipStream_t; NULL =
 * default stream).  One GPU wavefront runs each query.  DIRECT transport:
 * stream-ordered, returns after the launch.  AGENT transport: returns after
 * the search has completed (the agent serves the kernel while it runs).
 *   d_queries  device, nq x d elements of the index dtype
 *   k, L       results per query and candidate-list size, 1 <= k <= L <= 1024
 *   R          neighbours used per expansion, 1 <= R <= index R (0 = index R)
 *   d_ids      device, nq x k int32, padded with -1 when fewer than k found
 *   d_dists    device, nq x k: uint32 (u8/i8, padding 0xFFFFFFFF) or float
 *              (f32, padding +inf)
 *   d_steps    device, nq uint32 expansions per query, optional (NULL)
 * Buffers must stay valid until the stream syncs.
 * Schedule: select up to W unexpanded candidates per iteration into a FIFO
 * of in-flight nodes, then process the oldest while more than delay * W are
 * in flight (the oldest min(W, in flight) when nothing was selected); stop
 * when nothing is selectable and nothing is in flight.
 * Errors: ANN_EINVAL before any device work; ANN_ENOTSUP when
 * (delay + 1) * beam_width > 8; AGENT: ANN_EIO / ANN_ETIMEDOUT when a record
 * read failed or never completed (those queries return ids -1; the others
 * are valid).
 */
int ann_search(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L, int32_t R,
               const ann_search_opts *opts, int32_t *d_ids, void *d_dists, uint32_t *d_steps,
               void *hip_stream);

/*
 * ann_search_graph -- record one persistent ann_search (DIRECT transport) in
 * a HIP graph: a kernel that zeroes the work counter, then the search.  All
 * arguments and buffers are captured as given; ann_graph_launch replays the
 * same search (the caller may rewrite the contents of the query and per-query
 * buffers between replays).  `hip_stream` must be a non-default stream.
 * Errors: as ann_search, plus ANN_EINVAL for the default stream or AGENT.
 */
typedef struct ann_graph ann_graph;
int ann_search_graph(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L,
                     int32_t R, const ann_search_opts *opts, int32_t *d_ids, void *d_dists,
                     uint32_t *d_steps, void *hip_stream, ann_graph **out);
int ann_graph_launch(ann_graph *g, void *hip_stream);
int ann_graph_free(ann_graph *g);

/*
 * ann_search_noalloc -- ann_search for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Arguments, layouts, ownership and results are those of
 * ann_search; the call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine, no memset node: scratch is cleared by kernels).
 * Its scratch -- the persistent grid's work counter and the kernel-grained
 * grid barrier state -- lives in a fixed device array of
 * ANN_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends.  Every call on a GPU shares that array, so calls that overlap
 * on one GPU race: order them (e.g. one stream).  The index's device must be
 * current.
 * Supported: the DIRECT transport (records in HBM or host DRAM), one-shot or
 * persistent grids, query- or kernel-grained synchronisation, every schedule
 * and navigation of ann_search.
 * Errors: those of ann_search; ANN_EINVAL for the AGENT transport or a FILE
 * tier (their request lines are host memory the library allocates), for
 * another device than the index's, or if the scratch need exceeded the array.
 */
#define ANN_NOALLOC_SCRATCH_BYTES 32768
int ann_search_noalloc(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L,
                       int32_t R, const ann_search_opts *opts, int32_t *d_ids, void *d_dists,
                       uint32_t *d_steps, void *hip_stream);

/* ann_device_clock_khz -- frequency of the device wall clock used by
 * ann_search_opts.d_times on the current device (host int, caller-owned). */
int ann_device_clock_khz(int32_t *khz);

/*
 * Continuous-batching service (search state stays on the device; arrivals
 * are admitted as room frees up and overlap with queries already running).
 *
 * ann_server_open -- start a persistent server kernel over `ix` (HBM or HOST
 * tier).  Each admitted query holds one entry of (16 + nav_stride) bytes of
 * device memory until its results are out; `hbm_budget_bytes` bounds the
 * number admitted at once (after one entry per resident GPU wave, which the
 * ring keeps in reserve).  Arrivals beyond that wait on the host in arrival
 * order.  The server does not hold any caller pointer.
 *   opts (NULL = defaults): k_max (100), L_max (256), delay (1),
 *   waves_per_block (4), hash_bits (10), queue_cap (2^20 waiting arrivals),
 *   idle_polls (50000: empty polls before the kernel leaves; it is started
 *   again when work arrives), beam_width (1); the schedule is that of
 *   ann_search with the same delay and beam width, and so is the
 *   navigation (full precision, or PQ codes with exact re-rank).
 *   waves_per_block 0 = 4, or fewer when the LDS cannot hold 4 queries.
 * Errors: ANN_EINVAL, ANN_ENOMEM (budget too small or allocation), ANN_EIO.
 */
typedef struct ann_server ann_server;
typedef struct {
  int32_t k_max, L_max, delay, waves_per_block, hash_bits, queue_cap, idle_polls;
  int32_t beam_width; /* W (0 = 1); (delay + 1) * W <= 8 */
  int32_t transport;  /* ann_transport: AUTO (0) = AGENT for a FILE tier, else
                         DIRECT.  With AGENT the server runs its own host
                         agents and each resident GPU wave owns one request
                         line for all the queries it serves (section 4.2) */
  uint32_t spin_limit; /* AGENT: polls of a completion word before a query
                          gives up with ANN_ETIMEDOUT (0 = 2^24) */
  int32_t navigation;  /* ann_navigation (0 = full precision); ANN_NAV_PQ as
                          in ann_search_opts (needs ann_index_set_pq) */
  int32_t pq_scoring;  /* ann_pq_scoring (0 = auto) */
  uint64_t first_ticket; /* first admission ticket (0 by default).  Tickets
                            are 64-bit on the host and the device; a start
                            near 2^32 checks that none is cut to 32 bits */
} ann_server_opts;
typedef struct {
  uint64_t tag;          /* the caller's tag */
  int32_t status;        /* ANN_OK, or ANN_EIO / ANN_ETIMEDOUT when a record read
                            failed or never completed (AGENT; ids are then -1) */
  int32_t k;             /* results in ids/dists */
  const int32_t *ids;    /* host, valid until the next ann_server_poll */
  const void *dists;     /* host, uint32 (u8/i8) or float (f32), same lifetime */
  uint32_t steps;        /* expansions */
  double submit_us;      /* ann_clock_us() at submission */
  double done_us;        /* ann_clock_us() when the host saw the result */
} ann_result;
typedef struct {
  uint64_t submitted, admitted, completed, relaunches;
  int64_t max_inflight, slots, resident_waves;
} ann_server_stats;

int ann_server_open(ann_index *ix, size_t hbm_budget_bytes, const ann_server_opts *opts,
                    ann_server **out);
/* Queue one query (host, d elements of the index dtype; copied).  1 <= k <= k_max,
 * k <= L <= L_max.  ANN_EBUSY when the arrival queue is full. */
int ann_server_submit(ann_server *s, const void *host_query, int32_t k, int32_t L, uint64_t tag);
/* Queue n queries (host, n x d) with their k, L and tags.  With `arrival_us`
 * (non-decreasing ann_clock_us() times, optional) each query is admitted no
 * earlier than its arrival time and its submit_us is that time, so an
 * open-loop load measures latency from the intended arrival. */
int ann_server_submit_batch(ann_server *s, const void *host_queries, int64_t n, const int32_t *ks,
                            const int32_t *Ls, const uint64_t *tags, const double *arrival_us);
/* Take up to `max` completed results, waiting up to timeout_us for the first. */
int ann_server_poll(ann_server *s, ann_result *out, int32_t max, int32_t *n_out,
                    int32_t timeout_us);
/* Bulk form of ann_server_poll into caller-owned host arrays of `max` rows:
 * tags, ks, ids (max x k_max, padded with -1), dists (max x k_max, padded
 * with 0xFFFFFFFF bits), and optional steps, submit_us, done_us, status. */
int ann_server_poll_into(ann_server *s, int32_t max, uint64_t *tags, int32_t *ks, int32_t *ids,
                         void *dists, uint32_t *steps, double *submit_us, double *done_us,
                         int32_t *status, int32_t *n_out, int32_t timeout_us);
int ann_server_stats_get(ann_server *s, ann_server_stats *out);
/* Finish every admitted and waiting query, stop the kernel, release all. */
int ann_server_close(ann_server *s);
/* Monotonic host clock (microseconds) of ann_result's time stamps. */
double ann_clock_us(void);

/* ann_index_free -- release everything the index holds (NULL is a no-op).
 * ANN_EBUSY, with nothing released, while a server opened on the index is
 * still open: close every server first (its kernel and agents read the
 * index's memory). */
int ann_index_free(ann_index *ix);

/* Thread-local message describing the last failure of this thread. */
const char *ann_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FLASHANN_H */

// api.hip -- C ABI of the search library: index construction (HBM navigation
// copy + record store in HBM, pinned host DRAM or a file), the on-disk index
// format, the host agent of the query-grained transport, argument validation
// and kernel dispatch.
#include <fcntl.h>
#include <hip/hip_runtime.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/flashann.h"
#include "agent.h"
#include "search_kernel.h"

extern "C" int synth_build_graph(const void *base, int64_t n, int32_t d, int32_t dtype, int32_t R,
                                 uint64_t seed, int32_t threads, int32_t pool, float alpha,
                                 int32_t n_hubs, int64_t exact_limit, int32_t passes,
                                 int32_t Lb, int32_t *adj, int32_t *entry_out);

static_assert(sizeof(fa::AgentRequest) == 64 && fa::kCplStride == 16,
              "request/completion layout shared with the kernel");

struct ann_index {
  int64_t n = 0;
  int32_t d = 0, dtype = 0, R = 0, entry = 0, slot = 0, tier = 0;
  int32_t elem = 1, vec_bytes = 0, vec_pad = 0, nav_stride = 0, rec_bytes = 0, rec_chunks = 0;
  uint8_t *nav = nullptr;       // device, n x nav_stride
  uint8_t *rec_dev = nullptr;   // device-visible record base (HBM / HOST tiers)
  uint8_t *rec_hbm = nullptr;   // hipMalloc'd records (tier HBM)
  void *rec_host = nullptr;     // hipHostMalloc'd records (tier HOST)
  int fd = -1;                  // record file of stripe 0 (tier FILE)
  std::vector<int> fds;         // tier FILE: one per stripe (fds[0] == fd)
  bool direct_io = false;
  int device = 0;
  int64_t hbm_bytes = 0;
  // query-grained transport
  int agent_threads = 0;
  fa::AgentFaults faults;
  std::unique_ptr<fa::Agent> agent;
  fa::AgentRequest *req = nullptr;  // fine-grained pinned host
  uint32_t *cpl = nullptr;          // fine-grained pinned host
  uint8_t *stage = nullptr;         // fine-grained pinned host
  int32_t *d_status = nullptr;      // device
  int64_t tcap = 0, stage_stride = 0;
  int32_t tslots = 0;               // staging slots per query
  uint32_t *d_work = nullptr;       // persistent launches: device work counter
  uint32_t *d_ctl = nullptr;        // kernel-grained launches: barrier state (16 u32)
  // compressed navigation
  uint8_t *pq_codes = nullptr;      // device, n x kPqStride
  float *pq_cb = nullptr;           // device, pq_m x 256 x (d / pq_m)
  int32_t pq_m = 0;
  // hot-record cache (direct transport, host tier)
  uint8_t *d_cache = nullptr;       // device, cache_count x slot: record copies
  int32_t *d_cache_map = nullptr;   // device, n: cache slot of each node or -1
  int64_t cache_count = 0;
  std::atomic<int> servers{0};      // servers open on this index
};

struct ann_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? ANN_ENOMEM
                   : (e == hipErrorNoDevice || e == hipErrorInvalidDevice)       ? ANN_ENODEV
                                                                                 : ANN_EIO;
  return fail(code, "%s: %s", what, hipGetErrorString(e));
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int elem_bytes(int32_t dt) { return dt == ANN_F32 ? 4 : 1; }

void free_transport(ann_index *ix) {
  ix->agent.reset();
  if (ix->req) (void)hipHostFree(ix->req);
  if (ix->cpl) (void)hipHostFree(ix->cpl);
  if (ix->stage) (void)hipHostFree(ix->stage);
  if (ix->d_status) (void)hipFree(ix->d_status);
  ix->req = nullptr;
  ix->cpl = nullptr;
  ix->stage = nullptr;
  ix->d_status = nullptr;
  ix->tcap = 0;
  ix->tslots = 0;
}

void release(ann_index *ix) {
  if (!ix) return;
  free_transport(ix);
  if (ix->d_work) (void)hipFree(ix->d_work);
  if (ix->d_ctl) (void)hipFree(ix->d_ctl);
  if (ix->nav) (void)hipFree(ix->nav);
  if (ix->pq_codes) (void)hipFree(ix->pq_codes);
  if (ix->pq_cb) (void)hipFree(ix->pq_cb);
  if (ix->d_cache) (void)hipFree(ix->d_cache);
  if (ix->d_cache_map) (void)hipFree(ix->d_cache_map);
  if (ix->rec_hbm) (void)hipFree(ix->rec_hbm);
  if (ix->rec_host) (void)hipHostFree(ix->rec_host);
  for (const int f : ix->fds)
    if (f >= 0) close(f);
  if (ix->fds.empty() && ix->fd >= 0) close(ix->fd);
  delete ix;
}

// Sizes derived from (n, d, dtype, R, slot); validates them.
int init_layout(ann_index *ix, int64_t n, int32_t d, int32_t dtype, int32_t R, int32_t entry,
                int32_t slot_bytes) {
  if (n < 1 || n > 0x7FFFFFFFll) return fail(ANN_EINVAL, "n=%lld out of range", (long long)n);
  if (d < 1) return fail(ANN_EINVAL, "d=%d", d);
  if (dtype != ANN_U8 && dtype != ANN_I8 && dtype != ANN_F32)
    return fail(ANN_EINVAL, "dtype=%d", dtype);
  if (R < 1) return fail(ANN_EINVAL, "R=%d", R);
  if (entry < 0 || entry >= n) return fail(ANN_EINVAL, "entry=%d not in [0,n)", entry);
  ix->n = n; ix->d = d; ix->dtype = dtype; ix->R = R; ix->entry = entry; ix->slot = slot_bytes;
  ix->elem = elem_bytes(dtype);
  ix->vec_bytes = d * ix->elem;
  ix->vec_pad = (int32_t)round_up(ix->vec_bytes, 16);
  ix->nav_stride = (int32_t)round_up(ix->vec_bytes, 128);
  ix->rec_bytes = (int32_t)round_up(ix->vec_pad + 4 * (int64_t)R, 16);
  ix->rec_chunks = ix->rec_bytes / 16;
  if (ix->nav_stride > 512)
    return fail(ANN_ENOTSUP, "vector of %d B exceeds the 512 B row limit", ix->vec_bytes);
  if (ix->rec_bytes > 1024)
    return fail(ANN_ENOTSUP, "record of %d B exceeds the 1024 B fetch limit", ix->rec_bytes);
  if (slot_bytes < ix->vec_pad + 4 * R || slot_bytes % 16 != 0)
    return fail(ANN_EINVAL, "slot_bytes=%d must be a multiple of 16 and >= %d", slot_bytes,
                ix->vec_pad + 4 * R);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(ANN_ENODEV, "no GPU visible");
  (void)hipGetDevice(&ix->device);
  return ANN_OK;
}

// Navigation copy in HBM: rows zero-padded to nav_stride.
int build_nav(ann_index *ix, const uint8_t *vecs) {
  const int64_t n = ix->n;
  const int64_t nav_bytes = n * (int64_t)ix->nav_stride;
  hipError_t e = hipMalloc(&ix->nav, nav_bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(navigation copy)");
  ix->hbm_bytes += nav_bytes;
  const int64_t chunk_rows = std::max<int64_t>(1, (64ll << 20) / ix->nav_stride);
  std::vector<uint8_t> buf((size_t)(std::min(n, chunk_rows) * ix->nav_stride));
  for (int64_t i0 = 0; i0 < n; i0 += chunk_rows) {
    const int64_t i1 = std::min(n, i0 + chunk_rows);
    std::memset(buf.data(), 0, buf.size());
    for (int64_t i = i0; i < i1; i++)
      std::memcpy(buf.data() + (i - i0) * ix->nav_stride, vecs + i * ix->vec_bytes, ix->vec_bytes);
    e = hipMemcpy(ix->nav + i0 * ix->nav_stride, buf.data(), (i1 - i0) * ix->nav_stride,
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(navigation copy)");
  }
  return ANN_OK;
}

// Record layout: vector, zero pad to 16 B, R int32 ids, zero pad to the slot
// (paper section 3, C3: the node is its full vector plus its neighbour ids).
void pack_records(int64_t i0, int64_t i1, int32_t vec_bytes, int32_t vec_pad, int32_t R,
                  int32_t slot, const uint8_t *vecs, const int32_t *adj, uint8_t *dst) {
  for (int64_t i = i0; i < i1; i++) {
    uint8_t *r = dst + (i - i0) * slot;
    std::memcpy(r, vecs + i * vec_bytes, vec_bytes);
    std::memset(r + vec_bytes, 0, slot - vec_bytes);
    std::memcpy(r + vec_pad, adj + i * R, 4 * (size_t)R);
  }
}

// Record source for the HBM / HOST tiers: either packed from arrays or read
// from a records file (fd, already in the layout above).
struct RecordSource {
  const uint8_t *vecs = nullptr;
  const int32_t *adj = nullptr;
  int fd = -1;
  const int *stripes = nullptr;  // striped files (record v: file v % S, slot v / S)
  int nstripes = 0;
  int fill(const ann_index *ix, int64_t i0, int64_t i1, uint8_t *dst) const {
    if (nstripes > 1) {
      for (int64_t i = i0; i < i1; i++) {
        const int64_t off = (i / nstripes) * ix->slot;
        if (pread(stripes[i % nstripes], dst + (i - i0) * ix->slot, (size_t)ix->slot, (off_t)off) !=
            (ssize_t)ix->slot)
          return fail(ANN_EIO, "stripe %lld read failed at %lld", (long long)(i % nstripes),
                      (long long)off);
      }
      return ANN_OK;
    }
    if (fd < 0) {
      pack_records(i0, i1, ix->vec_bytes, ix->vec_pad, ix->R, ix->slot, vecs, adj, dst);
      return ANN_OK;
    }
    const int64_t want = (i1 - i0) * ix->slot;
    int64_t got = 0;
    while (got < want) {
      const ssize_t r = pread(fd, dst + got, (size_t)(want - got), (off_t)(i0 * ix->slot + got));
      if (r <= 0)
        return fail(ANN_EIO, "records file read failed at %lld", (long long)(i0 * ix->slot + got));
      got += r;
    }
    return ANN_OK;
  }
};

int build_records(ann_index *ix, const RecordSource &src) {
  const int64_t n = ix->n, slot = ix->slot, total = n * slot;
  hipError_t e;
  if (ix->tier == ANN_TIER_HBM) {
    if ((e = hipMalloc(&ix->rec_hbm, total)) != hipSuccess) return hip_fail(e, "hipMalloc(records)");
    ix->hbm_bytes += total;
    const int64_t chunk_rows = std::max<int64_t>(1, (64ll << 20) / slot);
    std::vector<uint8_t> buf((size_t)(std::min(n, chunk_rows) * slot));
    for (int64_t i0 = 0; i0 < n; i0 += chunk_rows) {
      const int64_t i1 = std::min(n, i0 + chunk_rows);
      int rc = src.fill(ix, i0, i1, buf.data());
      if (rc) return rc;
      if ((e = hipMemcpy(ix->rec_hbm + i0 * slot, buf.data(), (i1 - i0) * slot,
                         hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(records)");
    }
    ix->rec_dev = ix->rec_hbm;
    return ANN_OK;
  }
  // Pinned host DRAM mapped into the GPU address space, non-coherent
  // (coarse-grained): records are immutable while kernels run.
  if ((e = hipHostMalloc(&ix->rec_host, total, hipHostMallocNonCoherent)) != hipSuccess)
    return hip_fail(e, "hipHostMalloc(records)");
  int rc = src.fill(ix, 0, n, (uint8_t *)ix->rec_host);
  if (rc) return rc;
  void *dp = nullptr;
  if ((e = hipHostGetDevicePointer(&dp, ix->rec_host, 0)) != hipSuccess)
    return hip_fail(e, "hipHostGetDevicePointer(records)");
  ix->rec_dev = (uint8_t *)dp;
  return ANN_OK;
}

// Memory copies are CPU-bound: one thread per spare hardware thread.  Direct
// file reads are asynchronous (kAioDepth in flight per thread), so a few
// threads keep the storage queues full; buffered reads block in pread, so
// there more threads keep more reads in flight.
constexpr int kAioDepth = 64;
int default_agent_threads(bool file, bool direct) {
  const int hw = (int)std::thread::hardware_concurrency();
  if (file) return direct ? 8 : 64;
  return std::max(1, std::min(32, hw - 2));
}

fa::Agent *new_agent(ann_index *ix, int threads) {
  const bool file = ix->tier == ANN_TIER_FILE;
  const int32_t io = file && ix->direct_io ? (int32_t)round_up(ix->rec_bytes, 512) : ix->rec_bytes;
  const int t = threads > 0 ? threads : default_agent_threads(file, ix->direct_io);
  return new (std::nothrow) fa::Agent(file ? nullptr : (const uint8_t *)ix->rec_host,
                                      ix->fds.data(), (int)ix->fds.size(), ix->direct_io,
                                      ix->slot, ix->rec_bytes, io, t, kAioDepth);
}

// Transport buffers for nq queries and the agent itself.
int ensure_transport(ann_index *ix, int64_t nq, int32_t pslots) {
  const bool file = ix->tier == ANN_TIER_FILE;
  const int32_t io = file && ix->direct_io ? (int32_t)round_up(ix->rec_bytes, 512) : ix->rec_bytes;
  if (!ix->agent) {
    ix->agent.reset(new_agent(ix, ix->agent_threads));
    if (!ix->agent) return fail(ANN_ENOMEM, "agent");
  }
  if (nq <= ix->tcap && pslots <= ix->tslots) return ANN_OK;
  const int64_t cap = std::max<int64_t>({nq, ix->tcap, 1024});
  const int32_t slots = std::max(pslots, ix->tslots);
  fa::Agent *keep = ix->agent.release();
  free_transport(ix);
  ix->agent.reset(keep);
  ix->stage_stride = round_up(io, 512);
  hipError_t e;
  const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
  if ((e = hipHostMalloc((void **)&ix->req, sizeof(fa::AgentRequest) * cap, fl)) != hipSuccess ||
      (e = hipHostMalloc((void **)&ix->cpl, sizeof(uint32_t) * fa::kCplStride * cap, fl)) !=
          hipSuccess ||
      (e = hipHostMalloc((void **)&ix->stage, ix->stage_stride * slots * cap, fl)) != hipSuccess ||
      (e = hipMalloc(&ix->d_status, sizeof(int32_t) * cap)) != hipSuccess) {
    free_transport(ix);
    return hip_fail(e, "transport buffers");
  }
  ix->tcap = cap;
  ix->tslots = slots;
  return ANN_OK;
}

template <typename T>
T *dev_ptr(T *host) {
  void *dp = nullptr;
  return hipHostGetDevicePointer(&dp, host, 0) == hipSuccess ? (T *)dp : nullptr;
}

const char *dtype_name(int32_t dt) { return dt == ANN_U8 ? "u8" : dt == ANN_I8 ? "i8" : "f32"; }

// Minimal reader of the flat meta.json written by ann_save_index.
bool meta_int(const std::string &s, const char *key, int64_t *out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k);
  if (p == std::string::npos) return false;
  p = s.find(':', p + k.size());
  if (p == std::string::npos) return false;
  char *end = nullptr;
  const long long v = std::strtoll(s.c_str() + p + 1, &end, 10);
  if (end == s.c_str() + p + 1) return false;
  *out = v;
  return true;
}

bool meta_dtype(const std::string &s, int32_t *out) {
  size_t p = s.find("\"dtype\"");
  if (p == std::string::npos) return false;
  p = s.find('"', s.find(':', p) + 1);
  if (p == std::string::npos) return false;
  const std::string v = s.substr(p + 1, s.find('"', p + 1) - p - 1);
  *out = v == "u8" ? ANN_U8 : v == "i8" ? ANN_I8 : v == "f32" ? ANN_F32 : 0;
  return *out != 0;
}

// Flush a written file to the device before closing it: an index file is
// then durable, and reads of it never compete with its own write-back.
bool sync_close(FILE *f) {
  bool ok = std::fflush(f) == 0;
  ok = fsync(fileno(f)) == 0 && ok;
  return std::fclose(f) == 0 && ok;
}

int write_all(const std::string &path, const void *p, int64_t bytes) {
  FILE *f = std::fopen(path.c_str(), "wb");
  if (!f) return fail(ANN_EIO, "cannot create %s: %s", path.c_str(), std::strerror(errno));
  const bool ok = bytes == 0 || std::fwrite(p, 1, (size_t)bytes, f) == (size_t)bytes;
  if (!sync_close(f) || !ok) return fail(ANN_EIO, "write of %s failed", path.c_str());
  return ANN_OK;
}

}  // namespace

extern "C" {

const char *ann_last_error(void) { return g_err.c_str(); }

int ann_index_create(const void *vectors, const int32_t *adjacency, int64_t n, int32_t d,
                     int32_t dtype, int32_t R, int32_t entry, int32_t slot_bytes, int32_t tier,
                     ann_index **out) {
  if (!out) return fail(ANN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!vectors || !adjacency) return fail(ANN_EINVAL, "vectors/adjacency is NULL");
  if (tier != ANN_TIER_HBM && tier != ANN_TIER_HOST)
    return fail(ANN_EINVAL, "tier=%d: ann_index_create takes HBM or HOST (files: ann_load_records)",
                tier);
  ann_index *ix = new (std::nothrow) ann_index();
  if (!ix) return fail(ANN_ENOMEM, "handle");
  ix->tier = tier;
  int rc = init_layout(ix, n, d, dtype, R, entry, slot_bytes);
  if (!rc) rc = build_nav(ix, (const uint8_t *)vectors);
  if (!rc) {
    RecordSource src;
    src.vecs = (const uint8_t *)vectors;
    src.adj = adjacency;
    rc = build_records(ix, src);
  }
  if (rc) {
    release(ix);
    return rc;
  }
  *out = ix;
  return ANN_OK;
}

int ann_save_index(const char *dir, const void *vectors, const int32_t *adjacency, int64_t n,
                   int32_t d, int32_t dtype, int32_t R, int32_t entry, int32_t slot_bytes) {
  if (!dir || !vectors || !adjacency) return fail(ANN_EINVAL, "NULL argument");
  if (n < 1 || d < 1 || R < 1 || entry < 0 || entry >= n ||
      (dtype != ANN_U8 && dtype != ANN_I8 && dtype != ANN_F32))
    return fail(ANN_EINVAL, "bad sizes");
  const int32_t vb = d * elem_bytes(dtype), vp = (int32_t)round_up(vb, 16);
  if (slot_bytes < vp + 4 * R || slot_bytes % 16 != 0)
    return fail(ANN_EINVAL, "slot_bytes=%d must be a multiple of 16 and >= %d", slot_bytes, vp + 4 * R);
  if (mkdir(dir, 0755) != 0 && errno != EEXIST)
    return fail(ANN_EIO, "cannot create %s: %s", dir, std::strerror(errno));
  const std::string base(dir);
  char meta[512];
  snprintf(meta, sizeof meta,
           "{\"format\": \"flashann-1\", \"n\": %lld, \"d\": %d, \"dtype\": \"%s\", \"R\": %d, "
           "\"entry\": %d, \"slot_bytes\": %d}\n",
           (long long)n, d, dtype_name(dtype), R, entry, slot_bytes);
  int rc = write_all(base + "/meta.json", meta, (int64_t)strlen(meta));
  if (!rc) rc = write_all(base + "/vectors.bin", vectors, n * vb);
  if (rc) return rc;
  FILE *f = std::fopen((base + "/records.bin").c_str(), "wb");
  if (!f) return fail(ANN_EIO, "cannot create records.bin: %s", std::strerror(errno));
  const int64_t chunk = std::max<int64_t>(1, (32ll << 20) / slot_bytes);
  std::vector<uint8_t> buf((size_t)(std::min(n, chunk) * slot_bytes));
  bool ok = true;
  for (int64_t i0 = 0; i0 < n && ok; i0 += chunk) {
    const int64_t i1 = std::min(n, i0 + chunk);
    pack_records(i0, i1, vb, vp, R, slot_bytes, (const uint8_t *)vectors, adjacency, buf.data());
    const size_t bytes = (size_t)((i1 - i0) * slot_bytes);
    ok = std::fwrite(buf.data(), 1, bytes, f) == bytes;
  }
  if (!sync_close(f) || !ok) return fail(ANN_EIO, "write of records.bin failed");
  return ANN_OK;
}

int ann_save_records_striped(const void *vectors, const int32_t *adjacency, int64_t n, int32_t d,
                             int32_t dtype, int32_t R, int32_t slot_bytes,
                             const char *const *paths, int32_t stripes) {
  if (!vectors || !adjacency || !paths) return fail(ANN_EINVAL, "NULL argument");
  if (stripes < 1 || stripes > fa::kMaxStripes)
    return fail(ANN_EINVAL, "stripes=%d not in [1, %d]", stripes, fa::kMaxStripes);
  if (n < 1 || d < 1 || R < 1 || (dtype != ANN_U8 && dtype != ANN_I8 && dtype != ANN_F32))
    return fail(ANN_EINVAL, "bad sizes");
  const int32_t vb = d * elem_bytes(dtype), vp = (int32_t)round_up(vb, 16);
  if (slot_bytes < vp + 4 * R || slot_bytes % 16 != 0)
    return fail(ANN_EINVAL, "slot_bytes=%d must be a multiple of 16 and >= %d", slot_bytes, vp + 4 * R);
  std::vector<uint8_t> rec((size_t)slot_bytes);
  for (int32_t s = 0; s < stripes; s++) {
    if (!paths[s]) return fail(ANN_EINVAL, "stripe path %d is NULL", s);
    FILE *f = std::fopen(paths[s], "wb");
    if (!f) return fail(ANN_EIO, "cannot create %s: %s", paths[s], std::strerror(errno));
    bool ok = true;
    // stripe s holds records s, s + S, s + 2S, ... back to back
    const int64_t chunk = std::max<int64_t>(1, (32ll << 20) / slot_bytes);
    std::vector<uint8_t> buf((size_t)(chunk * slot_bytes));
    int64_t inbuf = 0;
    for (int64_t i = s; i < n && ok; i += stripes) {
      pack_records(i, i + 1, vb, vp, R, slot_bytes, (const uint8_t *)vectors, adjacency,
                   buf.data() + inbuf * slot_bytes);
      inbuf++;
      if (inbuf == chunk) {
        ok = std::fwrite(buf.data(), 1, (size_t)(inbuf * slot_bytes), f) == (size_t)(inbuf * slot_bytes);
        inbuf = 0;
      }
    }
    if (ok && inbuf)
      ok = std::fwrite(buf.data(), 1, (size_t)(inbuf * slot_bytes), f) == (size_t)(inbuf * slot_bytes);
    if (!sync_close(f) || !ok) return fail(ANN_EIO, "write of %s failed", paths[s]);
  }
  return ANN_OK;
}

int ann_build_index(const void *vectors, int64_t n, int32_t d, int32_t dtype, int32_t R,
                    int32_t slot_bytes, uint64_t seed, const char *out_dir) {
  if (!vectors || !out_dir) return fail(ANN_EINVAL, "NULL argument");
  if (n < 1 || n > 0x7FFFFFFFll || d < 1 || R < 1 ||
      (dtype != ANN_U8 && dtype != ANN_I8 && dtype != ANN_F32))
    return fail(ANN_EINVAL, "bad sizes");
  std::vector<int32_t> adj;
  try {
    adj.resize((size_t)(n * R));
  } catch (...) {
    return fail(ANN_ENOMEM, "adjacency of %lld x %d", (long long)n, R);
  }
  int32_t entry = -1;
  const int threads = std::max(1, std::min(64, (int)std::thread::hardware_concurrency()));
  const int64_t hubs = std::min<int64_t>(std::max<int64_t>(64, n / 1000), 4096);
  const int rc = synth_build_graph(vectors, n, d, dtype, R, seed, threads, std::max(2 * R, 64),
                                   1.2f, (int32_t)hubs, 20000, 1, std::max(64, 3 * R / 2),
                                   adj.data(), &entry);
  if (rc) return fail(ANN_EINVAL, "graph construction failed (%d)", rc);
  return ann_save_index(out_dir, vectors, adj.data(), n, d, dtype, R, entry, slot_bytes);
}

int ann_load_records(const char *dir, int32_t tier, const char *records_path, ann_index **out) {
  if (!dir) return fail(ANN_EINVAL, "NULL argument");
  const std::string def = std::string(dir) + "/records.bin";
  const char *path = records_path ? records_path : def.c_str();
  return ann_load_records_striped(dir, tier, &path, 1, out);
}

int ann_load_records_striped(const char *dir, int32_t tier, const char *const *paths,
                             int32_t stripes, ann_index **out) {
  if (!out || !dir || !paths) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  if (stripes < 1 || stripes > fa::kMaxStripes)
    return fail(ANN_EINVAL, "stripes=%d not in [1, %d]", stripes, fa::kMaxStripes);
  for (int32_t s = 0; s < stripes; s++)
    if (!paths[s]) return fail(ANN_EINVAL, "stripe path %d is NULL", s);
  if (tier != ANN_TIER_HBM && tier != ANN_TIER_HOST && tier != ANN_TIER_FILE)
    return fail(ANN_EINVAL, "tier=%d", tier);
  const std::string base(dir);
  std::string meta;
  {
    FILE *f = std::fopen((base + "/meta.json").c_str(), "rb");
    if (!f) return fail(ANN_EIO, "cannot open %s/meta.json", dir);
    char buf[1024];
    const size_t r = std::fread(buf, 1, sizeof buf - 1, f);
    std::fclose(f);
    meta.assign(buf, r);
  }
  int64_t n, d, R, entry, slot;
  int32_t dtype;
  if (!meta_int(meta, "n", &n) || !meta_int(meta, "d", &d) || !meta_int(meta, "R", &R) ||
      !meta_int(meta, "entry", &entry) || !meta_int(meta, "slot_bytes", &slot) ||
      !meta_dtype(meta, &dtype))
    return fail(ANN_EINVAL, "malformed %s/meta.json", dir);
  ann_index *ix = new (std::nothrow) ann_index();
  if (!ix) return fail(ANN_ENOMEM, "handle");
  ix->tier = tier;
  int rc = init_layout(ix, n, (int32_t)d, dtype, (int32_t)R, (int32_t)entry, (int32_t)slot);
  std::vector<uint8_t> vecs;
  if (!rc) {
    FILE *f = std::fopen((base + "/vectors.bin").c_str(), "rb");
    if (!f) {
      rc = fail(ANN_EIO, "cannot open %s/vectors.bin", dir);
    } else {
      try {
        vecs.resize((size_t)(n * ix->vec_bytes));
      } catch (...) {
        rc = fail(ANN_ENOMEM, "vectors");
      }
      if (!rc && std::fread(vecs.data(), 1, vecs.size(), f) != vecs.size())
        rc = fail(ANN_EIO, "short read of vectors.bin");
      std::fclose(f);
    }
  }
  if (!rc) rc = build_nav(ix, vecs.data());
  vecs.clear();
  vecs.shrink_to_fit();
  // stripe s holds records s, s + S, ...: ceil((n - s) / S) slots
  for (int32_t s = 0; s < stripes && !rc; s++) {
    struct stat st;
    const int64_t need = (n - s + stripes - 1) / stripes * slot;
    if (stat(paths[s], &st) != 0 || st.st_size < need)
      rc = fail(ANN_EIO, "%s missing or shorter than its %lld records", paths[s],
                (long long)(need / slot));
  }
  if (!rc && tier == ANN_TIER_FILE) {
    // O_DIRECT when the slot is a multiple of the 512 B sector and the file
    // system accepts it for every stripe; buffered reads otherwise.
    bool direct = slot % 512 == 0;
    for (int32_t s = 0; s < stripes && !rc; s++) {
      int f = direct ? open(paths[s], O_RDONLY | O_DIRECT) : -1;
      if (f < 0 && direct) {  // fall back for every stripe
        direct = false;
        for (const int g : ix->fds) close(g);
        ix->fds.clear();
        s = -1;
        continue;
      }
      if (f < 0) f = open(paths[s], O_RDONLY);
      if (f < 0) {
        rc = fail(ANN_EIO, "cannot open %s: %s", paths[s], std::strerror(errno));
        break;
      }
      ix->fds.push_back(f);
    }
    ix->direct_io = direct;
    if (!ix->fds.empty()) ix->fd = ix->fds[0];
  } else if (!rc) {
    std::vector<int> fds;
    for (int32_t s = 0; s < stripes && !rc; s++) {
      const int f = open(paths[s], O_RDONLY);
      if (f < 0)
        rc = fail(ANN_EIO, "cannot open %s", paths[s]);
      else
        fds.push_back(f);
    }
    if (!rc) {
      RecordSource src;
      src.fd = fds[0];
      src.stripes = fds.data();
      src.nstripes = stripes;
      rc = build_records(ix, src);
    }
    for (const int f : fds) close(f);
  }
  if (rc) {
    release(ix);
    return rc;
  }
  *out = ix;
  return ANN_OK;
}

int ann_index_info_get(const ann_index *ix, ann_index_info *out) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
  out->n = ix->n; out->d = ix->d; out->dtype = ix->dtype; out->R = ix->R;
  out->entry = ix->entry; out->slot_bytes = ix->slot; out->tier = ix->tier;
  out->nav_stride = ix->nav_stride; out->rec_bytes = ix->rec_bytes; out->hbm_bytes = ix->hbm_bytes;
  out->direct_io = ix->direct_io ? 1 : 0;
  out->stripes = ix->tier == ANN_TIER_FILE ? (int32_t)ix->fds.size() : 0;
  out->pq_m = ix->pq_m;
  out->nav_full = ix->nav ? 1 : 0;
  out->reserved = 0;
  out->cached_records = ix->cache_count;
  return ANN_OK;
}

int ann_index_set_pq(ann_index *ix, const float *codebooks, int32_t m, int32_t flags) {
  if (!ix || !codebooks) return fail(ANN_EINVAL, "NULL argument");
  if (m < 1 || m > fa::kPqMaxM || ix->d % m != 0 || ix->d / m > 32)
    return fail(ANN_EINVAL, "m=%d: need 1 <= m <= %d, d %% m == 0 and d / m <= 32 (d=%d)", m,
                fa::kPqMaxM, ix->d);
  if (flags & ~ANN_PQ_DROP_NAV) return fail(ANN_EINVAL, "flags=%d", flags);
  if (!ix->nav) return fail(ANN_EINVAL, "the navigation copy was released; nothing to encode");
  if (ix->servers.load() > 0)
    return fail(ANN_EBUSY, "a server is open on this index; close it first");
  const size_t cb_bytes = sizeof(float) * (size_t)m * fa::kPqKsub * (size_t)(ix->d / m);
  const size_t code_bytes = (size_t)ix->n * fa::kPqStride;
  uint8_t *codes = nullptr;
  float *cb = nullptr;
  hipError_t e = hipMalloc(&codes, code_bytes);
  if (e == hipSuccess) e = hipMalloc(&cb, cb_bytes);
  if (e == hipSuccess) e = hipMemcpy(cb, codebooks, cb_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = fa::launch_pq_encode(ix->nav, ix->n, ix->nav_stride, ix->dtype, ix->d, cb, m, codes,
                             nullptr);
  // also waits for searches still reading the codes or the copy replaced below
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (codes) (void)hipFree(codes);
    if (cb) (void)hipFree(cb);
    return hip_fail(e, "PQ encoding");
  }
  if (ix->pq_codes) {
    (void)hipFree(ix->pq_codes);
    ix->hbm_bytes -= (int64_t)ix->n * fa::kPqStride;
  }
  if (ix->pq_cb) {
    (void)hipFree(ix->pq_cb);
    ix->hbm_bytes -= (int64_t)sizeof(float) * ix->pq_m * fa::kPqKsub * (ix->d / ix->pq_m);
  }
  ix->pq_codes = codes;
  ix->pq_cb = cb;
  ix->pq_m = m;
  ix->hbm_bytes += (int64_t)(code_bytes + cb_bytes);
  if (flags & ANN_PQ_DROP_NAV) {
    (void)hipFree(ix->nav);
    ix->nav = nullptr;
    ix->hbm_bytes -= ix->n * (int64_t)ix->nav_stride;
  }
  return ANN_OK;
}

int ann_index_pq_codes(const ann_index *ix, uint8_t *host_codes) {
  if (!ix || !host_codes) return fail(ANN_EINVAL, "NULL argument");
  if (!ix->pq_codes) return fail(ANN_EINVAL, "the index has no PQ codes");
  hipError_t e = hipMemcpy2D(host_codes, (size_t)ix->pq_m, ix->pq_codes, fa::kPqStride,
                             (size_t)ix->pq_m, (size_t)ix->n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "PQ code copy");
  return ANN_OK;
}

int ann_agent_configure(ann_index *ix, int32_t threads, int32_t delay_node, int32_t delay_us,
                        int32_t fail_node, int32_t drop_node) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (threads < 0 || threads > 256 || delay_us < 0) return fail(ANN_EINVAL, "bad agent settings");
  if (threads != ix->agent_threads) ix->agent.reset();  // recreated on next use
  ix->agent_threads = threads;
  ix->faults.delay_node = delay_node;
  ix->faults.delay_us = delay_us;
  ix->faults.fail_node = fail_node;
  ix->faults.drop_node = drop_node;
  return ANN_OK;
}

int ann_agent_profile_get(const ann_index *ix, ann_agent_profile *out) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = ann_agent_profile{};
  const fa::Agent *a = ix->agent.get();
  if (!a) return ANN_OK;
  const fa::AgentStats &s = a->stats;
  out->requests = s.requests.load();
  out->bytes = s.bytes.load();
  out->errors = s.errors.load();
  out->passes = s.passes.load();
  out->busy_passes = s.busy_passes.load();
  out->scan_ns = s.scan_ns.load();
  out->copy_ns = s.copy_ns.load();
  out->io_ns = s.io_ns.load();
  out->max_batch = s.max_batch.load();
  out->threads = a->threads();
  out->async_io = a->async_io() ? 1 : 0;
  out->stripes = ix->tier == ANN_TIER_FILE ? (int32_t)ix->fds.size() : 1;
  for (int i = 0; i < fa::kMaxStripes; i++) out->stripe_requests[i] = s.stripe_requests[i].load();
  return ANN_OK;
}

int ann_agent_stats(const ann_index *ix, uint64_t *requests, uint64_t *bytes, uint64_t *errors) {
  if (!ix || !requests || !bytes || !errors) return fail(ANN_EINVAL, "NULL argument");
  *requests = ix->agent ? ix->agent->stats.requests.load() : 0;
  *bytes = ix->agent ? ix->agent->stats.bytes.load() : 0;
  *errors = ix->agent ? ix->agent->stats.errors.load() : 0;
  return ANN_OK;
}

}  // extern "C"

namespace {

// Waits for a kernel-grained search and reports an abandoned barrier wait.
int check_lockstep(const uint32_t *ctl, hipStream_t st) {
  uint32_t flag = 0;
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(&flag, ctl + 4, sizeof(flag), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "kernel-grained search");
  if (flag) return fail(ANN_ETIMEDOUT, "a grid barrier wait exceeded spin_limit; results invalid");
  return ANN_OK;
}

// Compressed-navigation kernel arguments (codes and codebooks of the index).
void set_pq_args(const ann_index *ix, int32_t pq_scoring, fa::SearchArgs *a) {
  a->pq_codes = ix->pq_codes;
  a->pq_cb = ix->pq_cb;
  a->pq_m = ix->pq_m;
  a->pq_dsub = ix->d / ix->pq_m;
  // default: centroids from the cache unless the table is small
  a->pq_direct = pq_scoring == ANN_PQ_CACHE ||
                 (pq_scoring == ANN_PQ_AUTO && ix->pq_m * fa::kPqKsub * 4 > 8192);
  a->pq_floats = a->pq_direct ? (int32_t)round_up(ix->d, 4) : ix->pq_m * fa::kPqKsub;
}

// Validates a search and fills the kernel arguments.  Returns ANN_OK with
// *empty set when there is nothing to launch (nq == 0).
int prepare_search(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L,
                   int32_t R, const ann_search_opts *opts, int32_t *d_ids, void *d_dists,
                   uint32_t *d_steps, ann_search_opts *o_out, int *transport_out,
                   fa::SearchArgs *args, bool *empty, bool may_allocate = true) {
  *empty = false;
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (nq < 0) return fail(ANN_EINVAL, "nq=%lld", (long long)nq);
  if (k < 1) return fail(ANN_EINVAL, "k=%d must be >= 1", k);
  if (L < k || L > 1024) return fail(ANN_EINVAL, "L=%d must satisfy k <= L <= 1024", L);
  if (R == 0) R = ix->R;
  if (R < 1 || R > ix->R) return fail(ANN_EINVAL, "R=%d must be in [1, %d]", R, ix->R);
  ann_search_opts o{};
  o.delay = 1;
  o.beam_width = 1;
  if (opts) o = *opts;
  if (o.hash_bits == 0) o.hash_bits = 10;
  const bool auto_wpb = o.waves_per_block == 0;
  if (auto_wpb) o.waves_per_block = 4;
  if (o.delay < 0) return fail(ANN_EINVAL, "delay=%d must be >= 0", o.delay);
  if (o.beam_width < 1) return fail(ANN_EINVAL, "beam_width=%d must be >= 1", o.beam_width);
  if ((int64_t)(o.delay + 1) * o.beam_width > fa::kMaxPipe)
    return fail(ANN_ENOTSUP, "(delay+1)*beam_width = %lld nodes in flight exceeds %d",
                (long long)(o.delay + 1) * o.beam_width, fa::kMaxPipe);
  if (o.hash_bits < 6 || o.hash_bits > 14) return fail(ANN_EINVAL, "hash_bits=%d not in [6,14]", o.hash_bits);
  if (o.waves_per_block < 1 || o.waves_per_block > 4)
    return fail(ANN_EINVAL, "waves_per_block=%d not in [1,4]", o.waves_per_block);
  if (o.d_trace && o.trace_cap < 1) return fail(ANN_EINVAL, "trace_cap=%d with a trace buffer", o.trace_cap);
  if (o.d_phases && o.delay != 0)
    return fail(ANN_EINVAL, "phase times are measured on the strict schedule (delay 0) only");
  int transport = o.transport;
  if (transport == ANN_TRANSPORT_AUTO)
    transport = ix->tier == ANN_TIER_FILE ? ANN_TRANSPORT_AGENT : ANN_TRANSPORT_DIRECT;
  if (transport != ANN_TRANSPORT_DIRECT && transport != ANN_TRANSPORT_AGENT)
    return fail(ANN_EINVAL, "transport=%d", o.transport);
  if (transport == ANN_TRANSPORT_DIRECT && ix->tier == ANN_TIER_FILE)
    return fail(ANN_EINVAL, "a file tier is read through the agent transport only");
  if (transport == ANN_TRANSPORT_AGENT && ix->tier == ANN_TIER_HBM)
    return fail(ANN_EINVAL, "HBM records are read directly by the kernel");
  if (o.persistent != 0 && o.persistent != 1) return fail(ANN_EINVAL, "persistent=%d", o.persistent);
  if (o.sync_grain != 0 && o.sync_grain != 1) return fail(ANN_EINVAL, "sync_grain=%d", o.sync_grain);
  if (o.sync_grain == 1 && (o.delay != 0 || o.beam_width != 1 || o.persistent || o.d_order ||
                            o.d_phases))
    return fail(ANN_EINVAL, "kernel-grained search runs the strict schedule (delay 0, beam 1) "
                            "without persistent waves, order or phase times");
  if (o.navigation != ANN_NAV_FULL && o.navigation != ANN_NAV_PQ)
    return fail(ANN_EINVAL, "navigation=%d", o.navigation);
  if (o.navigation == ANN_NAV_PQ && !ix->pq_codes)
    return fail(ANN_EINVAL, "PQ navigation needs codes (ann_index_set_pq)");
  if (o.navigation == ANN_NAV_FULL && !ix->nav)
    return fail(ANN_EINVAL, "the full-precision navigation copy was released; use ANN_NAV_PQ");
  if (o.pq_scoring < 0 || o.pq_scoring > ANN_PQ_CACHE)
    return fail(ANN_EINVAL, "pq_scoring=%d", o.pq_scoring);
  if (o.poll_backoff < 0 || o.poll_backoff > 1024)
    return fail(ANN_EINVAL, "poll_backoff=%d not in [0, 1024]", o.poll_backoff);
  if (o.navigation == ANN_NAV_PQ && o.sync_grain)
    return fail(ANN_ENOTSUP, "kernel-grained search scores with the full-precision copy only");
  if (o.query_lanes == 0) o.query_lanes = 64;
  if (o.query_lanes != 64 && o.query_lanes != 32)
    return fail(ANN_EINVAL, "query_lanes=%d must be 32 or 64", o.query_lanes);
  if (o.query_lanes == 32 &&
      (transport != ANN_TRANSPORT_DIRECT || o.navigation != ANN_NAV_FULL || o.sync_grain ||
       o.delay > 1 || o.beam_width != 1 || ix->rec_chunks > 32))
    return fail(ANN_ENOTSUP, "two queries per wave (query_lanes 32) run the direct transport, "
                             "full-precision navigation, delay 0 or 1 with beam 1 and records "
                             "of at most 512 B (these are %d B)", 16 * ix->rec_chunks);
  if (nq > 0x7FFFFFFFll) return fail(ANN_EINVAL, "nq=%lld too large", (long long)nq);
  *o_out = o;
  *transport_out = transport;
  if (nq == 0) {
    *empty = true;
    return ANN_OK;
  }
  if (!d_queries || !d_ids || !d_dists) return fail(ANN_EINVAL, "NULL query/output pointer");
  if (o.persistent && !ix->d_work && may_allocate) {
    hipError_t e = hipMalloc(&ix->d_work, sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(work counter)");
  }
  if (o.sync_grain && !ix->d_ctl && may_allocate) {
    hipError_t e = hipMalloc(&ix->d_ctl, fa::kLockstepCtlWords * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(barrier state)");
  }

  fa::SearchArgs &a = *args;
  a = fa::SearchArgs{};
  a.nav = ix->nav;
  a.records = ix->rec_dev;
  a.queries = (const uint8_t *)d_queries;
  a.out_ids = d_ids;
  a.out_dists = d_dists;
  a.out_steps = d_steps;
  a.stats = o.d_stats;
  a.trace = o.d_trace;
  a.trace_cap = o.d_trace ? o.trace_cap : 0;
  a.times = o.d_times;
  a.phases = o.d_phases;
  a.nq = nq; a.n = ix->n; a.slot = ix->slot;
  a.nav_stride = ix->nav_stride; a.qbytes = ix->vec_bytes; a.vec_pad = ix->vec_pad;
  a.ids_off = ix->vec_pad; a.rec_chunks = ix->rec_chunks;
  a.R = R; a.L = L; a.Lcap = (int32_t)round_up(L, 64); a.k = k; a.entry = ix->entry;
  a.k_stride = k;
  a.q_L = o.d_L;
  a.q_k = o.d_k;
  a.order = o.d_order;
  a.work = ix->d_work;
  a.hash_bits = o.hash_bits;
  a.delay = o.delay;
  a.beam = o.beam_width;
  a.pslots = std::max(2, (o.delay + 1) * o.beam_width);
  if (o.navigation == ANN_NAV_PQ) set_pq_args(ix, o.pq_scoring, &a);
  if (ix->cache_count > 0) {
    a.cache = ix->d_cache;
    a.cache_map = ix->d_cache_map;
  }
  a.qlanes = o.query_lanes;
  a.lds_per_wave = fa::search_lds_bytes(a.Lcap, a.nav_stride, a.hash_bits,
                                        a.pq_m ? a.k : 0, a.pq_floats, a.qlanes);
  // the default waves per workgroup shrinks to what the LDS holds
  const int per_wave = 64 / a.qlanes;
  while (auto_wpb && o.waves_per_block > 1 &&
         (int64_t)a.lds_per_wave * o.waves_per_block * per_wave > 160 * 1024)
    o.waves_per_block /= 2;
  *o_out = o;
  if ((int64_t)a.lds_per_wave * o.waves_per_block * per_wave > 160 * 1024)
    return fail(ANN_EINVAL, "LDS need %u B per query x %d exceeds 160 KiB", a.lds_per_wave,
                o.waves_per_block * per_wave);
  return ANN_OK;
}

}  // namespace

extern "C" {

int ann_search(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L, int32_t R,
               const ann_search_opts *opts, int32_t *d_ids, void *d_dists, uint32_t *d_steps,
               void *hip_stream) {
  ann_search_opts o;
  int transport = 0;
  fa::SearchArgs a;
  bool empty = false;
  int rc = prepare_search(ix, d_queries, nq, k, L, R, opts, d_ids, d_dists, d_steps, &o,
                          &transport, &a, &empty);
  if (rc || empty) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (o.sync_grain) a.spin_limit = o.spin_limit ? o.spin_limit : (1u << 24);
  if (transport == ANN_TRANSPORT_DIRECT && o.sync_grain) {
    hipError_t e = fa::launch_lockstep(a, ix->d_ctl, ix->dtype, fa::TR_DIRECT, o.waves_per_block, st);
    if (e != hipSuccess) return hip_fail(e, "kernel-grained search launch");
    return check_lockstep(ix->d_ctl, st);
  }
  if (transport == ANN_TRANSPORT_DIRECT) {
    hipError_t e = hipSuccess;
    if (o.persistent) e = fa::launch_reset(ix->d_work, st);
    if (e == hipSuccess)
      e = fa::launch_search(a, ix->dtype, fa::TR_DIRECT, o.waves_per_block,
                            o.persistent != 0, st);
    if (e != hipSuccess) return hip_fail(e, "search launch");
    return ANN_OK;
  }

  // Query-grained transport: arm the agent, run, wait, disarm.  Synchronous
  // with respect to the host so that the request, completion and staging
  // arrays are never reused while a kernel may still touch them.
  rc = ensure_transport(ix, nq, a.pslots);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(st);  // earlier work on the stream
  if (e != hipSuccess) return hip_fail(e, "stream sync");
  std::memset(ix->req, 0, sizeof(fa::AgentRequest) * nq);
  std::memset(ix->cpl, 0, sizeof(uint32_t) * fa::kCplStride * nq);
  if ((e = hipMemsetAsync(ix->d_status, 0, sizeof(int32_t) * nq, st)) != hipSuccess)
    return hip_fail(e, "status reset");
  a.req = dev_ptr((uint64_t *)ix->req);
  a.cpl = dev_ptr(ix->cpl);
  a.stage = dev_ptr(ix->stage);
  a.stage_stride = ix->stage_stride;
  a.spin_limit = o.spin_limit ? o.spin_limit : (1u << 24);
  a.poll_nap = o.poll_backoff > 0 ? (uint32_t)o.poll_backoff : 32u;
  a.status = ix->d_status;
  if (!a.req || !a.cpl || !a.stage) return fail(ANN_EIO, "transport buffers not mapped");
  ix->agent->faults = ix->faults;
  ix->agent->arm(ix->req, ix->cpl, ix->stage, nq, ix->stage_stride, a.pslots);
  if (o.persistent) e = fa::launch_reset(ix->d_work, st);
  if (e == hipSuccess)
    e = o.sync_grain ? fa::launch_lockstep(a, ix->d_ctl, ix->dtype, fa::TR_AGENT,
                                           o.waves_per_block, st)
                     : fa::launch_search(a, ix->dtype, fa::TR_AGENT, o.waves_per_block,
                                         o.persistent != 0, st);
  const hipError_t es = e == hipSuccess ? hipStreamSynchronize(st) : e;
  ix->agent->disarm();
  if (e != hipSuccess) return hip_fail(e, "search launch");
  if (es != hipSuccess) return hip_fail(es, "search");
  if (o.sync_grain && (rc = check_lockstep(ix->d_ctl, st)) != ANN_OK) return rc;
  std::vector<int32_t> status((size_t)nq);
  if ((e = hipMemcpy(status.data(), ix->d_status, sizeof(int32_t) * nq, hipMemcpyDeviceToHost)) !=
      hipSuccess)
    return hip_fail(e, "status copy");
  int64_t bad = 0, first = -1;
  int code = ANN_OK;
  for (int64_t i = 0; i < nq; i++)
    if (status[(size_t)i]) {
      if (first < 0) {
        first = i;
        code = status[(size_t)i];
      }
      bad++;
    }
  if (bad) {
    const int en = ix->agent->stats.last_errno.load();
    return fail(code, "%lld queries failed (first: query %lld, %s%s%s); their ids are -1",
                (long long)bad, (long long)first, code == ANN_ETIMEDOUT ? "timed out" : "read error",
                en ? ": " : "", en ? std::strerror(en) : "");
  }
  return ANN_OK;
}

int ann_search_graph(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L,
                     int32_t R, const ann_search_opts *opts, int32_t *d_ids, void *d_dists,
                     uint32_t *d_steps, void *hip_stream, ann_graph **out) {
  if (!out) return fail(ANN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!hip_stream) return fail(ANN_EINVAL, "graph capture needs a non-default stream");
  ann_search_opts o0{};
  o0.delay = 1;
  o0.beam_width = 1;
  if (opts) o0 = *opts;
  o0.persistent = 1;
  ann_search_opts o;
  int transport = 0;
  fa::SearchArgs a;
  bool empty = false;
  int rc = prepare_search(ix, d_queries, nq, k, L, R, &o0, d_ids, d_dists, d_steps, &o,
                          &transport, &a, &empty);
  if (rc) return rc;
  if (empty) return fail(ANN_EINVAL, "nothing to capture (nq == 0)");
  if (transport != ANN_TRANSPORT_DIRECT)
    return fail(ANN_EINVAL, "graphs capture the DIRECT transport only");
  if (o.sync_grain) return fail(ANN_EINVAL, "graphs capture query-grained searches only");
  hipStream_t st = (hipStream_t)hip_stream;
  ann_graph *g = new (std::nothrow) ann_graph();
  if (!g) return fail(ANN_ENOMEM, "graph handle");
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e1 = fa::launch_reset(ix->d_work, st);
    if (e1 == hipSuccess)
      e1 = fa::launch_search(a, ix->dtype, fa::TR_DIRECT, o.waves_per_block, true, st);
    e = hipStreamEndCapture(st, &g->graph);
    if (e == hipSuccess) e = e1;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    ann_graph_free(g);
    return hip_fail(e, "graph capture");
  }
  *out = g;
  return ANN_OK;
}

int ann_graph_launch(ann_graph *g, void *hip_stream) {
  if (!g || !g->exec) return fail(ANN_EINVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return ANN_OK;
}

int ann_graph_free(ann_graph *g) {
  if (!g) return ANN_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return ANN_OK;
}

}  // extern "C"

// ------------------------------------------------ search without allocation
// ann_search_noalloc keeps its scratch -- the persistent grid's work counter
// (byte 0) and the kernel-grained grid barrier state (from byte 256) -- in
// one fixed device array.  Each GPU the library runs on holds its own copy
// until the process ends; every call on that GPU shares it, so calls that
// overlap on one GPU race (the caller orders them, e.g. on one stream).  In
// host code `scratch` is only a host-side stand-in: its device address on
// the current GPU comes from hipGetSymbolAddress, once per device.
namespace {

constexpr size_t kScratchCtlOffset = 256;
static_assert(kScratchCtlOffset + fa::kLockstepCtlWords * sizeof(uint32_t) <= ANN_NOALLOC_SCRATCH_BYTES,
              "the barrier state must fit the scratch array");
static __device__ __align__(256) uint32_t scratch[ANN_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on GPU `dev` (which is current).
int scratch_on(int dev, uint32_t **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ANN_ENODEV, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(ANN_EIO, "scratch array has no device address");
    g_scratch_dev[dev] = (uint32_t *)p;
  }
  *out = g_scratch_dev[dev];
  return ANN_OK;
}

}  // namespace

extern "C" {

int ann_search_noalloc(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L,
                       int32_t R, const ann_search_opts *opts, int32_t *d_ids, void *d_dists,
                       uint32_t *d_steps, void *hip_stream) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != ix->device)
    return fail(ANN_EINVAL, "the index lives on device %d; make it current (device %d is)",
                ix->device, dev);
  ann_search_opts o;
  int transport = 0;
  fa::SearchArgs a;
  bool empty = false;
  int rc = prepare_search(ix, d_queries, nq, k, L, R, opts, d_ids, d_dists, d_steps, &o,
                          &transport, &a, &empty, /*may_allocate=*/false);
  if (rc || empty) return rc;
  if (transport != ANN_TRANSPORT_DIRECT)
    return fail(ANN_EINVAL, "the allocation-free search reads records directly (HBM or host "
                            "tier); the agent transport needs host request lines");
  // the scratch need is fixed: one work counter and one barrier state
  const size_t need = kScratchCtlOffset + (o.sync_grain ? fa::kLockstepCtlWords * sizeof(uint32_t) : 0);
  if (need > ANN_NOALLOC_SCRATCH_BYTES)
    return fail(ANN_EINVAL, "scratch need %zu B exceeds the %d B array", need,
                ANN_NOALLOC_SCRATCH_BYTES);
  uint32_t *base = nullptr;
  if ((rc = scratch_on(dev, &base)) != ANN_OK) return rc;
  uint32_t *work = base;
  uint32_t *ctl = base + kScratchCtlOffset / sizeof(uint32_t);
  hipStream_t st = (hipStream_t)hip_stream;
  if (o.sync_grain) {
    a.spin_limit = o.spin_limit ? o.spin_limit : (1u << 24);
    // the launcher clears the barrier state with a kernel before the search
    e = fa::launch_lockstep(a, ctl, ix->dtype, fa::TR_DIRECT, o.waves_per_block, st);
    if (e != hipSuccess) return hip_fail(e, "kernel-grained search launch");
    return check_lockstep(ctl, st);
  }
  a.work = work;
  e = hipSuccess;
  if (o.persistent) e = fa::launch_reset(work, st);  // a kernel, not a memset
  if (e == hipSuccess)
    e = fa::launch_search(a, ix->dtype, fa::TR_DIRECT, o.waves_per_block, o.persistent != 0, st);
  if (e != hipSuccess) return hip_fail(e, "search launch");
  return ANN_OK;
}

}  // extern "C"

// Shared with server.cpp: error reporting and the index fields of a search.
int ann_internal_fail(int code, const char *msg) { return fail(code, "%s", msg); }

// Transport of a server over this index (AUTO: AGENT for a FILE tier, else
// DIRECT) and, for AGENT, an agent of its own reading the index's records;
// *stage_stride is the staging slot size it needs.
int ann_internal_server_transport(ann_index *ix, int32_t requested, int32_t *tr,
                                  fa::Agent **agent, int64_t *stage_stride) {
  int t = requested;
  if (t == ANN_TRANSPORT_AUTO)
    t = ix->tier == ANN_TIER_FILE ? ANN_TRANSPORT_AGENT : ANN_TRANSPORT_DIRECT;
  if (t != ANN_TRANSPORT_DIRECT && t != ANN_TRANSPORT_AGENT)
    return fail(ANN_EINVAL, "transport=%d", requested);
  if (t == ANN_TRANSPORT_DIRECT && ix->tier == ANN_TIER_FILE)
    return fail(ANN_EINVAL, "a file tier is served through the agent transport only");
  if (t == ANN_TRANSPORT_AGENT && ix->tier == ANN_TIER_HBM)
    return fail(ANN_EINVAL, "HBM records are read directly by the kernel");
  *tr = t == ANN_TRANSPORT_AGENT ? fa::TR_AGENT : fa::TR_DIRECT;
  *agent = nullptr;
  *stage_stride = 0;
  if (t == ANN_TRANSPORT_AGENT) {
    const bool file = ix->tier == ANN_TIER_FILE;
    const int32_t io = file && ix->direct_io ? (int32_t)round_up(ix->rec_bytes, 512) : ix->rec_bytes;
    *agent = new_agent(ix, ix->agent_threads);
    if (!*agent) return fail(ANN_ENOMEM, "server agent");
    (*agent)->faults = ix->faults;
    *stage_stride = round_up(io, 512);
  }
  return ANN_OK;
}

int ann_internal_server_args(ann_index *ix, int32_t k_max, int32_t L_max, int32_t hash_bits,
                             int32_t navigation, int32_t pq_scoring, fa::SearchArgs *base,
                             int32_t *dtype) {
  if (hash_bits < 6 || hash_bits > 14) return fail(ANN_EINVAL, "hash_bits=%d", hash_bits);
  if (navigation != ANN_NAV_FULL && navigation != ANN_NAV_PQ)
    return fail(ANN_EINVAL, "navigation=%d", navigation);
  if (pq_scoring < 0 || pq_scoring > ANN_PQ_CACHE) return fail(ANN_EINVAL, "pq_scoring=%d", pq_scoring);
  if (navigation == ANN_NAV_FULL && !ix->nav)
    return fail(ANN_EINVAL, "the full-precision navigation copy was released; use ANN_NAV_PQ");
  if (navigation == ANN_NAV_PQ && !ix->pq_codes)
    return fail(ANN_EINVAL, "PQ navigation needs codes (ann_index_set_pq)");
  fa::SearchArgs &a = *base;
  a = fa::SearchArgs{};
  a.nav = ix->nav;
  a.records = ix->rec_dev;
  a.n = ix->n;
  a.slot = ix->slot;
  a.nav_stride = ix->nav_stride;
  a.qbytes = ix->vec_bytes;
  a.vec_pad = ix->vec_pad;
  a.ids_off = ix->vec_pad;
  a.rec_chunks = ix->rec_chunks;
  a.R = ix->R;
  a.L = L_max;
  a.Lcap = (int32_t)round_up(L_max, 64);
  a.k = k_max;
  a.k_stride = k_max;
  a.entry = ix->entry;
  a.hash_bits = hash_bits;
  if (navigation == ANN_NAV_PQ) set_pq_args(ix, pq_scoring, &a);
  if (ix->cache_count > 0) {
    a.cache = ix->d_cache;
    a.cache_map = ix->d_cache_map;
  }
  a.lds_per_wave = fa::search_lds_bytes(a.Lcap, a.nav_stride, a.hash_bits, a.pq_m ? a.k : 0,
                                        a.pq_floats);
  *dtype = ix->dtype;
  return ANN_OK;
}

extern "C" {

int ann_device_clock_khz(int32_t *khz) {
  if (!khz) return fail(ANN_EINVAL, "khz is NULL");
  int dev = 0, v = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return hip_fail(e, "wall clock rate");
  *khz = v;
  return ANN_OK;
}

int ann_index_set_record_cache(ann_index *ix, const int32_t *ids, int64_t count) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (count < 0 || count > ix->n)
    return fail(ANN_EINVAL, "count=%lld not in [0, n=%lld]", (long long)count, (long long)ix->n);
  if (count > 0 && !ids) return fail(ANN_EINVAL, "ids is NULL");
  if (count > 0 && ix->tier == ANN_TIER_HBM)
    return fail(ANN_ENOTSUP, "HBM-tier records are all in device memory already");
  if (ix->servers.load() > 0)
    return fail(ANN_EBUSY, "a server is open on this index; close it first");
  std::vector<int32_t> map;
  if (count > 0) {
    map.assign((size_t)ix->n, -1);
    for (int64_t i = 0; i < count; i++) {
      const int32_t v = ids[i];
      if (v < 0 || v >= ix->n) return fail(ANN_EINVAL, "ids[%lld]=%d not in [0, n)", (long long)i, v);
      if (map[(size_t)v] >= 0) return fail(ANN_EINVAL, "ids[%lld]=%d listed twice", (long long)i, v);
      map[(size_t)v] = (int32_t)i;
    }
  }
  // searches still reading the cache being replaced finish first
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "record cache");
  if (ix->d_cache) (void)hipFree(ix->d_cache);
  if (ix->d_cache_map) (void)hipFree(ix->d_cache_map);
  ix->hbm_bytes -= ix->cache_count * ix->slot + (ix->cache_count ? ix->n * 4 : 0);
  ix->d_cache = nullptr;
  ix->d_cache_map = nullptr;
  ix->cache_count = 0;
  if (count == 0) return ANN_OK;
  const size_t cbytes = (size_t)count * (size_t)ix->slot;
  e = hipMalloc(&ix->d_cache, cbytes);
  if (e == hipSuccess) e = hipMalloc(&ix->d_cache_map, sizeof(int32_t) * (size_t)ix->n);
  if (e == hipSuccess)
    e = hipMemcpy(ix->d_cache_map, map.data(), sizeof(int32_t) * (size_t)ix->n,
                  hipMemcpyHostToDevice);
  // the copies are gathered in host chunks of up to 64 MiB: from host memory,
  // or read from the record files (record v: file v % S at (v / S) * slot;
  // reads of whole 512 B sectors into an aligned buffer when O_DIRECT)
  const int64_t per = std::max<int64_t>(1, (64ll << 20) / ix->slot);
  std::vector<uint8_t> buf;
  const bool file = ix->tier == ANN_TIER_FILE;
  const size_t io = file && ix->direct_io ? (size_t)round_up(ix->rec_bytes, 512) : (size_t)ix->rec_bytes;
  void *bounce = nullptr;
  if (file && posix_memalign(&bounce, 4096, (size_t)round_up((int64_t)io, 4096)) != 0) {
    bounce = nullptr;
    e = hipErrorOutOfMemory;
  }
  int rd_err = 0;
  for (int64_t b = 0; e == hipSuccess && !rd_err && b < count; b += per) {
    const int64_t m = std::min<int64_t>(per, count - b);
    buf.assign((size_t)m * (size_t)ix->slot, 0);
    for (int64_t i = 0; i < m && !rd_err; i++) {
      const int64_t v = ids[b + i];
      uint8_t *dst = buf.data() + (size_t)i * ix->slot;
      if (!file) {
        std::memcpy(dst, (const uint8_t *)ix->rec_host + (size_t)v * (size_t)ix->slot,
                    (size_t)ix->slot);
        continue;
      }
      const int S = (int)ix->fds.size();
      const ssize_t r = pread(ix->fds[(size_t)(v % S)], bounce, io, (off_t)((v / S) * ix->slot));
      if (r < (ssize_t)ix->rec_bytes) rd_err = r < 0 ? errno : EIO;
      else std::memcpy(dst, bounce, (size_t)ix->rec_bytes);
    }
    if (!rd_err)
      e = hipMemcpy(ix->d_cache + (size_t)b * ix->slot, buf.data(), (size_t)m * ix->slot,
                    hipMemcpyHostToDevice);
  }
  free(bounce);
  if (e != hipSuccess || rd_err) {
    if (ix->d_cache) (void)hipFree(ix->d_cache);
    if (ix->d_cache_map) (void)hipFree(ix->d_cache_map);
    ix->d_cache = nullptr;
    ix->d_cache_map = nullptr;
    if (rd_err) return fail(ANN_EIO, "record cache: reading a record failed: %s", std::strerror(rd_err));
    return hip_fail(e, "record cache");
  }
  ix->cache_count = count;
  ix->hbm_bytes += count * ix->slot + ix->n * 4;
  return ANN_OK;
}

int ann_index_free(ann_index *ix) {
  // an open server's kernel and agents read the index's memory
  if (ix && ix->servers.load() > 0)
    return fail(ANN_EBUSY, "a server is open on this index: close it first");
  release(ix);
  return ANN_OK;
}

}  // extern "C"

void ann_internal_server_hold(ann_index *ix, int delta) {
  if (ix) ix->servers.fetch_add(delta);
}

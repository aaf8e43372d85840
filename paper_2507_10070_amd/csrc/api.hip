// api.hip -- C ABI of the search library: index construction in device and
// pinned host memory, argument validation and kernel dispatch.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/flashann.h"
#include "search_kernel.h"

struct ann_index {
  int64_t n = 0;
  int32_t d = 0, dtype = 0, R = 0, entry = 0, slot = 0, tier = 0;
  int32_t elem = 1, vec_bytes = 0, vec_pad = 0, nav_stride = 0, rec_bytes = 0, rec_chunks = 0;
  uint8_t *nav = nullptr;       // device, n x nav_stride
  uint8_t *rec_dev = nullptr;   // device-visible record base
  uint8_t *rec_hbm = nullptr;   // hipMalloc'd records (tier HBM)
  void *rec_host = nullptr;     // hipHostMalloc'd records (tier HOST)
  int device = 0;
  int64_t hbm_bytes = 0;
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

void release(ann_index *ix) {
  if (!ix) return;
  if (ix->nav) (void)hipFree(ix->nav);
  if (ix->rec_hbm) (void)hipFree(ix->rec_hbm);
  if (ix->rec_host) (void)hipHostFree(ix->rec_host);
  delete ix;
}

// Pack records [i0, i1) into `dst` (slot bytes each): vector, zero pad to
// 16 B, R int32 ids, zero pad to the slot.
void pack_records(const ann_index *ix, const uint8_t *vecs, const int32_t *adj, int64_t i0,
                  int64_t i1, uint8_t *dst) {
  for (int64_t i = i0; i < i1; i++) {
    uint8_t *r = dst + (i - i0) * ix->slot;
    std::memcpy(r, vecs + i * ix->vec_bytes, ix->vec_bytes);
    std::memset(r + ix->vec_bytes, 0, ix->slot - ix->vec_bytes);
    std::memcpy(r + ix->vec_pad, adj + i * ix->R, 4 * (size_t)ix->R);
  }
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
  if (n < 1 || n > 0x7FFFFFFFll) return fail(ANN_EINVAL, "n=%lld out of range", (long long)n);
  if (d < 1) return fail(ANN_EINVAL, "d=%d", d);
  if (dtype != ANN_U8 && dtype != ANN_I8 && dtype != ANN_F32)
    return fail(ANN_EINVAL, "dtype=%d", dtype);
  if (R < 1) return fail(ANN_EINVAL, "R=%d", R);
  if (entry < 0 || entry >= n) return fail(ANN_EINVAL, "entry=%d not in [0,n)", entry);
  if (tier != ANN_TIER_HBM && tier != ANN_TIER_HOST)
    return fail(ANN_EINVAL, "tier=%d not supported by ann_index_create", tier);

  ann_index *ix = new (std::nothrow) ann_index();
  if (!ix) return fail(ANN_ENOMEM, "handle");
  ix->n = n; ix->d = d; ix->dtype = dtype; ix->R = R; ix->entry = entry;
  ix->slot = slot_bytes; ix->tier = tier;
  ix->elem = elem_bytes(dtype);
  ix->vec_bytes = d * ix->elem;
  ix->vec_pad = (int32_t)round_up(ix->vec_bytes, 16);
  ix->nav_stride = (int32_t)round_up(ix->vec_bytes, 128);
  ix->rec_bytes = (int32_t)round_up(ix->vec_pad + 4 * (int64_t)R, 16);
  ix->rec_chunks = ix->rec_bytes / 16;
  if (ix->nav_stride > 512) {
    release(ix);
    return fail(ANN_ENOTSUP, "vector of %d B exceeds the 512 B row limit", d * elem_bytes(dtype));
  }
  if (ix->rec_bytes > 1024) {
    release(ix);
    return fail(ANN_ENOTSUP, "record of %d B exceeds the 1024 B fetch limit", ix->rec_bytes);
  }
  if (slot_bytes < ix->vec_pad + 4 * R || slot_bytes % 16 != 0) {
    release(ix);
    return fail(ANN_EINVAL, "slot_bytes=%d must be a multiple of 16 and >= %d", slot_bytes,
                ix->vec_pad + 4 * R);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    release(ix);
    return fail(ANN_ENODEV, "no GPU visible");
  }
  (void)hipGetDevice(&ix->device);

  hipError_t e;
  // navigation copy: rows zero-padded to nav_stride
  const int64_t nav_bytes = n * (int64_t)ix->nav_stride;
  if ((e = hipMalloc(&ix->nav, nav_bytes)) != hipSuccess) {
    release(ix);
    return hip_fail(e, "hipMalloc(navigation copy)");
  }
  ix->hbm_bytes += nav_bytes;
  const uint8_t *vecs = (const uint8_t *)vectors;
  {
    const int64_t chunk_rows = std::max<int64_t>(1, (64ll << 20) / ix->nav_stride);
    std::vector<uint8_t> buf((size_t)(std::min(n, chunk_rows) * ix->nav_stride));
    for (int64_t i0 = 0; i0 < n; i0 += chunk_rows) {
      const int64_t i1 = std::min(n, i0 + chunk_rows);
      std::memset(buf.data(), 0, buf.size());
      for (int64_t i = i0; i < i1; i++)
        std::memcpy(buf.data() + (i - i0) * ix->nav_stride, vecs + i * ix->vec_bytes,
                    ix->vec_bytes);
      e = hipMemcpy(ix->nav + i0 * ix->nav_stride, buf.data(), (i1 - i0) * ix->nav_stride,
                    hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        release(ix);
        return hip_fail(e, "hipMemcpy(navigation copy)");
      }
    }
  }
  // records
  const int64_t rec_total = n * (int64_t)slot_bytes;
  if (tier == ANN_TIER_HBM) {
    if ((e = hipMalloc(&ix->rec_hbm, rec_total)) != hipSuccess) {
      release(ix);
      return hip_fail(e, "hipMalloc(records)");
    }
    ix->hbm_bytes += rec_total;
    const int64_t chunk_rows = std::max<int64_t>(1, (64ll << 20) / slot_bytes);
    std::vector<uint8_t> buf((size_t)(std::min(n, chunk_rows) * slot_bytes));
    for (int64_t i0 = 0; i0 < n; i0 += chunk_rows) {
      const int64_t i1 = std::min(n, i0 + chunk_rows);
      pack_records(ix, vecs, adjacency, i0, i1, buf.data());
      e = hipMemcpy(ix->rec_hbm + i0 * slot_bytes, buf.data(), (i1 - i0) * slot_bytes,
                    hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        release(ix);
        return hip_fail(e, "hipMemcpy(records)");
      }
    }
    ix->rec_dev = ix->rec_hbm;
  } else {
    // Pinned host DRAM, mapped into the GPU address space.  Non-coherent
    // (coarse-grained): records are immutable while kernels run, so the GPU
    // may cache them.
    if ((e = hipHostMalloc(&ix->rec_host, rec_total, hipHostMallocNonCoherent)) != hipSuccess) {
      release(ix);
      return hip_fail(e, "hipHostMalloc(records)");
    }
    pack_records(ix, vecs, adjacency, 0, n, (uint8_t *)ix->rec_host);
    void *dp = nullptr;
    if ((e = hipHostGetDevicePointer(&dp, ix->rec_host, 0)) != hipSuccess) {
      release(ix);
      return hip_fail(e, "hipHostGetDevicePointer(records)");
    }
    ix->rec_dev = (uint8_t *)dp;
  }
  *out = ix;
  return ANN_OK;
}

int ann_index_info_get(const ann_index *ix, ann_index_info *out) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
  out->n = ix->n; out->d = ix->d; out->dtype = ix->dtype; out->R = ix->R;
  out->entry = ix->entry; out->slot_bytes = ix->slot; out->tier = ix->tier;
  out->nav_stride = ix->nav_stride; out->rec_bytes = ix->rec_bytes; out->hbm_bytes = ix->hbm_bytes;
  return ANN_OK;
}

int ann_search(ann_index *ix, const void *d_queries, int64_t nq, int32_t k, int32_t L, int32_t R,
               const ann_search_opts *opts, int32_t *d_ids, void *d_dists, uint32_t *d_steps,
               void *hip_stream) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (nq < 0) return fail(ANN_EINVAL, "nq=%lld", (long long)nq);
  if (k < 1) return fail(ANN_EINVAL, "k=%d must be >= 1", k);
  if (L < k || L > 1024) return fail(ANN_EINVAL, "L=%d must satisfy k <= L <= 1024", L);
  if (R == 0) R = ix->R;
  if (R < 1 || R > ix->R) return fail(ANN_EINVAL, "R=%d must be in [1, %d]", R, ix->R);
  ann_search_opts o = {1, 1, 10, 4, nullptr, nullptr, 0, nullptr};
  if (opts) {
    o = *opts;
    if (o.hash_bits == 0) o.hash_bits = 10;
    if (o.waves_per_block == 0) o.waves_per_block = 4;
  }
  if (o.delay < 0) return fail(ANN_EINVAL, "delay=%d must be >= 0", o.delay);
  if (o.beam_width < 1) return fail(ANN_EINVAL, "beam_width=%d must be >= 1", o.beam_width);
  if (o.delay > 1) return fail(ANN_ENOTSUP, "delay=%d: the GPU kernels implement 0 and 1", o.delay);
  if (o.beam_width != 1) return fail(ANN_ENOTSUP, "beam_width=%d: only 1 is implemented", o.beam_width);
  if (o.hash_bits < 6 || o.hash_bits > 14) return fail(ANN_EINVAL, "hash_bits=%d not in [6,14]", o.hash_bits);
  if (o.waves_per_block < 1 || o.waves_per_block > 4)
    return fail(ANN_EINVAL, "waves_per_block=%d not in [1,4]", o.waves_per_block);
  if (o.d_trace && o.trace_cap < 1) return fail(ANN_EINVAL, "trace_cap=%d with a trace buffer", o.trace_cap);
  if (nq == 0) return ANN_OK;
  if (!d_queries || !d_ids || !d_dists) return fail(ANN_EINVAL, "NULL query/output pointer");

  fa::SearchArgs a{};
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
  a.nq = nq; a.n = ix->n; a.slot = ix->slot;
  a.nav_stride = ix->nav_stride; a.qbytes = ix->vec_bytes; a.vec_pad = ix->vec_pad;
  a.ids_off = ix->vec_pad; a.rec_chunks = ix->rec_chunks;
  a.R = R; a.L = L; a.Lcap = (int32_t)round_up(L, 64); a.k = k; a.entry = ix->entry;
  a.hash_bits = o.hash_bits;
  a.lds_per_wave = fa::search_lds_bytes(a.Lcap, a.nav_stride, a.hash_bits);
  if ((int64_t)a.lds_per_wave * o.waves_per_block > 160 * 1024)
    return fail(ANN_EINVAL, "LDS need %u B per query x %d exceeds 160 KiB", a.lds_per_wave,
                o.waves_per_block);
  hipError_t e = fa::launch_search(a, ix->dtype, o.delay, o.waves_per_block, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "search launch");
  return ANN_OK;
}

int ann_device_clock_khz(int32_t *khz) {
  if (!khz) return fail(ANN_EINVAL, "khz is NULL");
  int dev = 0, v = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return hip_fail(e, "wall clock rate");
  *khz = v;
  return ANN_OK;
}

int ann_index_free(ann_index *ix) {
  release(ix);
  return ANN_OK;
}

}  // extern "C"

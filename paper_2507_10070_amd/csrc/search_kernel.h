// search_kernel.h -- internal interface between the C-ABI layer and the
// gfx950 search kernels (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fa {

enum { DT_U8 = 1, DT_I8 = 2, DT_F32 = 3 };

// Byte offsets of one wave's LDS region.
struct LdsLayout {
  uint32_t cand, nk, stage, qbuf, ids, dsc, hash, bytes;
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
  int32_t trace_cap;
  int64_t nq, n, slot;
  int32_t nav_stride, qbytes, vec_pad, ids_off, rec_chunks;
  int32_t R, L, Lcap, k, entry, hash_bits;
  uint32_t lds_per_wave;
};

uint32_t search_lds_bytes(int Lcap, int nav_stride, int hash_bits);
hipError_t launch_search(const SearchArgs &a, int dtype, int delay, int waves_per_block,
                         hipStream_t st);

}  // namespace fa
